// Photon trace kernels for gfx950 (MI355X).
//
// One photon per lane.  Photon state lives in registers (FP64 position, direction, wavelength,
// time); the optical prescription is read with uniform (scalar) loads; screens are gathered from
// global memory through L2 / Infinity Cache; image bins are 32-bit atomics, aggregated across the
// wavefront when several lanes hit the same pixel; per-(status, surface) counters are kept in LDS
// and flushed once per workgroup.
//
// Random numbers: Philox4x32-10 keyed by (seed, source) with counter (photon index lo, hi, block,
// stream), so each photon is reproducible alone.  Block/word map of stream 0:
//   block 0: pupil radius, pupil angle, time, wavelength
//   block 1: wavelength blur within an SED bin, Sersic angle, conversion length, unused
//   blocks 2-5: coating roulette of surfaces 4(b-2) .. 4(b-2)+3
//   block 6: diffusion normal pair
// Stream 1, block t: trial t of the Gamma sampler used by Sersic sources.
#include <hip/hip_runtime.h>

#include "phx_internal.h"

namespace phx {
namespace {

constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr double kHcEvM = 1.2398419843320026e-6;  // h c / e in eV m
constexpr double kNewtonTol = 1e-12;             // m
constexpr int kNewtonMax = 16;
constexpr int kBlock = 256;

// ---------------------------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11).
__device__ __forceinline__ uint4 philox(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
        const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// (w + 1/2) 2^-32, exact in double.
__device__ __forceinline__ double u01(uint32_t w) {
    return fma((double)w, 2.3283064365386963e-10, 1.1641532182693481e-10);
}

struct Rng {
    uint32_t k0, k1, lo, hi;
    __device__ uint4 block(uint32_t b, uint32_t stream = 0) const {
        return philox(make_uint4(lo, hi, b, stream), k0, k1);
    }
};

__device__ __forceinline__ double sellmeier(const DevParams& P, double lam) {
    const double l2 = (lam * 1e6) * (lam * 1e6);
    double s = 1.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) s += P.sell_b[i] * l2 / (l2 - P.sell_c[i]);
    return sqrt(s);
}

__device__ __forceinline__ double n_silicon(double lam) {
    const double e = kHcEvM / lam;
    return 3.36 + 0.211 * e + 2.79 * exp((e - 3.30) / 0.398);
}

// Rajkanan absorption coefficient in m^-1 (constants at the device temperature precomputed).
__device__ __forceinline__ double absorption(const DevParams& P, double lam) {
    const double e = kHcEvM / lam;
    const double C[2] = {5.5, 4.0};
    const double A[2] = {3.231e2, 7.237e3};
    const double ep[2] = {1.827e-2, 5.773e-2};
    double alpha = 0.0;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const double a = e - P.eg[j] + ep[i];
            const double b = e - P.eg[j] - ep[i];
            double term = 0.0;
            if (a > 0.0) term += a * a / P.absorb[i];
            if (b > 0.0) term += b * b / P.emit[i];
            alpha += C[i] * A[j] * term;
        }
    }
    if (e > P.egd) alpha += 1.052e6 * sqrt(e - P.egd);
    return alpha * 100.0;
}

// ---------------------------------------------------------------------------------------------
// Surfaces.

// Noll Z4..Z15 on the unit disk and their gradients; z[] are the amplitudes.
__device__ void zernike_sum(const double* z, double u, double v, double& s, double& du,
                            double& dv) {
    const double r2 = u * u + v * v;
    const double s3 = 1.7320508075688772, s6 = 2.449489742783178, s8 = 2.8284271247461903;
    const double s5 = 2.23606797749979, s10 = 3.1622776601683795;
    const double uu = u * u, vv = v * v;
    s = 0.0; du = 0.0; dv = 0.0;
    // Z4
    s += z[0] * s3 * (2.0 * r2 - 1.0);  du += z[0] * s3 * 4.0 * u;  dv += z[0] * s3 * 4.0 * v;
    // Z5, Z6
    s += z[1] * s6 * 2.0 * u * v;       du += z[1] * s6 * 2.0 * v;  dv += z[1] * s6 * 2.0 * u;
    s += z[2] * s6 * (uu - vv);         du += z[2] * s6 * 2.0 * u;  dv -= z[2] * s6 * 2.0 * v;
    // Z7, Z8
    s += z[3] * s8 * (3.0 * r2 - 2.0) * v;
    du += z[3] * s8 * 6.0 * u * v;      dv += z[3] * s8 * (3.0 * uu + 9.0 * vv - 2.0);
    s += z[4] * s8 * (3.0 * r2 - 2.0) * u;
    du += z[4] * s8 * (9.0 * uu + 3.0 * vv - 2.0);  dv += z[4] * s8 * 6.0 * u * v;
    // Z9, Z10
    s += z[5] * s8 * (3.0 * uu * v - vv * v);
    du += z[5] * s8 * 6.0 * u * v;      dv += z[5] * s8 * (3.0 * uu - 3.0 * vv);
    s += z[6] * s8 * (uu * u - 3.0 * u * vv);
    du += z[6] * s8 * (3.0 * uu - 3.0 * vv);  dv -= z[6] * s8 * 6.0 * u * v;
    // Z11
    s += z[7] * s5 * (6.0 * r2 * r2 - 6.0 * r2 + 1.0);
    du += z[7] * s5 * (24.0 * r2 - 12.0) * u;  dv += z[7] * s5 * (24.0 * r2 - 12.0) * v;
    // Z12, Z13
    const double w = 4.0 * r2 - 3.0;
    s += z[8] * s10 * w * (uu - vv);
    du += z[8] * s10 * (8.0 * u * (uu - vv) + 2.0 * w * u);
    dv += z[8] * s10 * (8.0 * v * (uu - vv) - 2.0 * w * v);
    s += z[9] * s10 * w * 2.0 * u * v;
    du += z[9] * s10 * (16.0 * uu * v + 2.0 * w * v);
    dv += z[9] * s10 * (16.0 * u * vv + 2.0 * w * u);
    // Z14, Z15
    s += z[10] * s10 * (uu * uu - 6.0 * uu * vv + vv * vv);
    du += z[10] * s10 * (4.0 * uu * u - 12.0 * u * vv);
    dv += z[10] * s10 * (4.0 * vv * v - 12.0 * uu * v);
    s += z[11] * s10 * (4.0 * uu * u * v - 4.0 * u * vv * v);
    du += z[11] * s10 * (12.0 * uu * v - 4.0 * vv * v);
    dv += z[11] * s10 * (4.0 * uu * u - 12.0 * u * vv);
}

// Sag S(x, y) and g with (dS/dx, dS/dy) = (x g, y g) + zernike gradient.  Returns false outside
// the conic's domain.
__device__ __forceinline__ bool sag(const DevParams& P, const DevSurface& s, double x, double y,
                                    double& S, double& gx, double& gy) {
    const double r2 = x * x + y * y;
    const double arg = 1.0 - s.kappa1 * s.c * s.c * r2;
    if (arg < 0.0) return false;
    const double root = sqrt(arg);
    S = s.c * r2 / (1.0 + root);
    double g = s.c / root;
    if (s.asphere) {
        const double r = sqrt(r2);
        // sum alpha_i r^i and sum i alpha_i r^(i-2), i = 3..10
        double pw = r;          // r^(i-2) for i = 3
        double acc_s = 0.0, acc_g = 0.0;
#pragma unroll
        for (int i = 3; i <= 10; ++i) {
            const double a = s.alpha[i - 3];
            acc_g += (double)i * a * pw;
            acc_s += a * pw * r2;
            pw *= r;
        }
        S += acc_s;
        g += acc_g;
    }
    gx = x * g;
    gy = y * g;
    if (s.zernike) {
        double zs, zu, zv;
        zernike_sum(P.zern, x * P.zern_inv_r, y * P.zern_inv_r, zs, zu, zv);
        S += zs;
        gx += zu * P.zern_inv_r;
        gy += zv * P.zern_inv_r;
    }
    return true;
}

// Intersection of the ray q + l d with the surface: exact conic root, then Newton on
// f(l) = q_z + l d_z - S(q_x + l d_x, q_y + l d_y).  Returns 0 or a status; gx, gy receive the
// sag gradient at the last evaluation.
__device__ int intersect(const DevParams& P, const DevSurface& s, const double q[3],
                         const double d[3], double& l, double& gx, double& gy, int& iters) {
    const double A = s.c * (d[0] * d[0] + d[1] * d[1] + s.kappa1 * d[2] * d[2]);
    const double B = s.c * (q[0] * d[0] + q[1] * d[1] + s.kappa1 * q[2] * d[2]) - d[2];
    const double C = s.c * (q[0] * q[0] + q[1] * q[1] + s.kappa1 * q[2] * q[2]) - 2.0 * q[2];
    const double disc = B * B - A * C;
    if (disc < 0.0) return PHX_MISSED;
    const double sq = sqrt(disc);
    const double den = B >= 0.0 ? B + sq : B - sq;
    if (den == 0.0) return PHX_MISSED;
    l = -C / den;
    for (int it = 1; it <= kNewtonMax; ++it) {
        const double x = q[0] + l * d[0], y = q[1] + l * d[1], z = q[2] + l * d[2];
        double S;
        if (!sag(P, s, x, y, S, gx, gy)) return PHX_MISSED;
        const double fp = d[2] - (gx * d[0] + gy * d[1]);
        if (fp == 0.0) return PHX_NONCONV;
        const double dl = (z - S) / fp;
        l -= dl;
        iters += 1;
        if (fabs(dl) <= kNewtonTol) return 0;
    }
    return PHX_NONCONV;
}

__device__ __forceinline__ double coating(const DevParams& P, int c, double s, double lam) {
    const float* t = P.coat + (size_t)c * P.n_s * P.n_lam;
    double fs = s / P.s_step;
    double fl = (lam - P.lam0) / P.dlam;
    fs = fmin(fmax(fs, 0.0), (double)(P.n_s - 1));
    fl = fmin(fmax(fl, 0.0), (double)(P.n_lam - 1));
    int is = min((int)floor(fs), P.n_s - 2);
    int il = min((int)floor(fl), P.n_lam - 2);
    const double a = fs - is, b = fl - il;
    const float* r0 = t + (size_t)is * P.n_lam + il;
    const float* r1 = r0 + P.n_lam;
    return (1.0 - a) * ((1.0 - b) * (double)r0[0] + b * (double)r0[1]) +
           a * ((1.0 - b) * (double)r1[0] + b * (double)r1[1]);
}

// Upper bound of a coating's transmission over all angles at wavelength lam (pre-roll).
__device__ __forceinline__ double coating_max(const DevParams& P, int c, double lam) {
    double fl = (lam - P.lam0) / P.dlam;
    fl = fmin(fmax(fl, 0.0), (double)(P.n_lam - 1));
    const int il = min((int)floor(fl), P.n_lam - 2);
    const float* m = P.coat_max + (size_t)c * P.n_lam + il;
    return fmax((double)m[0], (double)m[1]);
}

__device__ __forceinline__ void screen_tap(const float2* g, int64_t N, double xs, double ys,
                                           double& ax, double& ay) {
    const double fx = floor(xs), fy = floor(ys);
    const double a = xs - fx, b = ys - fy;
    const int64_t m = N - 1;
    const int64_t i0 = (int64_t)fx & m, j0 = (int64_t)fy & m;
    const int64_t i1 = (i0 + 1) & m, j1 = (j0 + 1) & m;
    const float2 v00 = g[j0 * N + i0], v10 = g[j0 * N + i1];
    const float2 v01 = g[j1 * N + i0], v11 = g[j1 * N + i1];
    ax = (1.0 - b) * ((1.0 - a) * (double)v00.x + a * (double)v10.x) +
         b * ((1.0 - a) * (double)v01.x + a * (double)v11.x);
    ay = (1.0 - b) * ((1.0 - a) * (double)v00.y + a * (double)v10.y) +
         b * ((1.0 - a) * (double)v01.y + a * (double)v11.y);
}

__device__ __forceinline__ void normalise(double n[3]) {
    const double inv = 1.0 / sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    n[0] *= inv; n[1] *= inv; n[2] *= inv;
}

// Gamma(shape) by Marsaglia & Tsang, trial t on stream 1 block t.
__device__ double gamma_sample(const Rng& rng, double shape) {
    const double a = shape < 1.0 ? shape + 1.0 : shape;
    const double dd = a - 1.0 / 3.0, cc = 1.0 / sqrt(9.0 * dd);
    for (uint32_t t = 0; t < 64; ++t) {
        const uint4 w = rng.block(t, 1);
        const double u0 = u01(w.x), u1 = u01(w.y), u2 = u01(w.z);
        const double x = sqrt(-2.0 * log(u0)) * cos(kTwoPi * u1);
        double v = 1.0 + cc * x;
        if (v <= 0.0) continue;
        v = v * v * v;
        const double x2 = x * x;
        bool accept = u2 < 1.0 - 0.0331 * x2 * x2;
        if (!accept) accept = log(u2) < 0.5 * x2 + dd * (1.0 - v + log(v));
        if (accept) {
            double g = dd * v;
            if (shape < 1.0) g *= pow(u01(w.w), 1.0 / shape);
            return g;
        }
    }
    return shape;
}

struct Outcome {
    int status, surface, newton;
    int pix_i, pix_j;
    double x, y, z, xe, ye, lam;
};

// The whole per-photon path.  `culled` photons return PHX_CULLED without being traced.
__device__ Outcome trace_photon(const DevParams& P, const Launch& L, int si, uint64_t idx) {
    const DevSource& src = P.src[si];
    Outcome o;
    o.status = PHX_MISSED; o.surface = -1; o.newton = 0; o.pix_i = -1; o.pix_j = -1;
    o.x = o.y = o.z = o.xe = o.ye = 0.0;
    const Rng rng{L.seed, (uint32_t)si, (uint32_t)idx, (uint32_t)(idx >> 32)};
    const uint4 w0 = rng.block(0);
    const uint4 w1 = rng.block(1);

    // wavelength (section 2.2): flat photon spectrum or tabulated SED CDF + blur in the bin
    double lam;
    if (src.sed < 0) {
        lam = src.lambda_lo + u01(w0.w) * src.lambda_span;
    } else {
        const double* cdf = P.sed_cdf + (size_t)src.sed * (P.sed_k + 1);
        const double u = u01(w0.w);
        int lo = 0, hi = P.sed_k - 1;   // smallest k in [0, K-1] with cdf[k+1] > u
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (cdf[mid + 1] > u) hi = mid; else lo = mid + 1;
        }
        lam = P.sed_edges[lo] + u01(w1.x) * (P.sed_edges[lo + 1] - P.sed_edges[lo]);
    }
    lam = lam * src.redshift1;
    o.lam = lam;

    // pre-roll (section 3.2): a photon whose roulette draw exceeds the worst-case transmission of
    // a coated surface cannot be detected
    if ((L.flags & PHX_F_CULL) && (L.flags & PHX_F_COATINGS)) {
        for (int b = 0; b * 4 < P.n_surf; ++b) {
            bool any = false;
            for (int k = 4 * b; k < min(4 * b + 4, P.n_surf); ++k) any |= P.surf[k].coating >= 0;
            if (!any) continue;
            const uint4 w = rng.block(2 + b);
            const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
            for (int k = 4 * b; k < min(4 * b + 4, P.n_surf); ++k) {
                const int c = P.surf[k].coating;
                if (c < 0) continue;
                if (u01(ws[k & 3]) > coating_max(P, c, lam) + 1e-12) {
                    o.status = PHX_CULLED;
                    o.surface = -1;
                    return o;
                }
            }
        }
    }

    // direction (section 2.2) and extended-source perturbation (section 2.2.1)
    double n[3] = {src.xi, src.eta, src.nz};
    if (src.kind == 1) {
        const double g = gamma_sample(rng, 2.0 * src.sersic_n);
        const double rr = pow(g / src.sersic_bn, src.sersic_n);
        double sp, cp;
        sincos(kTwoPi * u01(w1.y), &sp, &cp);
        const double dmaj = src.sersic_a * rr * cp, dmin = src.sersic_b * rr * sp;
        n[0] += dmaj * src.cos_pa - dmin * src.sin_pa;
        n[1] += dmaj * src.sin_pa + dmin * src.cos_pa;
        normalise(n);
    }
    const double t = L.exposure * u01(w0.z);

    // pupil sample on the first surface (section 2.2)
    double p[3];
    {
        const double ro = P.pupil_r_out + L.pupil_margin;
        const double ri = fmax(P.pupil_r_in - L.pupil_margin, 0.0);
        const double r = sqrt(u01(w0.x) * (ro * ro - ri * ri) + ri * ri);
        double sphi, cphi;
        sincos(kTwoPi * u01(w0.y), &sphi, &cphi);
        p[0] = r * cphi;
        p[1] = r * sphi;
        const DevSurface& s0 = P.surf[0];
        const double r2 = p[0] * p[0] + p[1] * p[1];
        const double arg = 1.0 - s0.kappa1 * s0.c * s0.c * r2;
        double z = s0.t[2] + (arg >= 0.0 ? s0.c * r2 / (1.0 + sqrt(arg)) : 0.0);
        if (s0.asphere) {
            double pw = r * r2;
            for (int i = 3; i <= 10; ++i) {
                z += s0.alpha[i - 3] * pw;
                pw *= r;
            }
        }
        p[2] = z;
    }

    // atmosphere (sections 2.3.1-2.3.2): move up to the highest layer, then down layer by layer,
    // deflecting by the wind-shifted screen gradients scaled by (lambda/lambda_ref)^(-1/5)
    if ((L.flags & PHX_F_ATMOSPHERE) && P.n_layers > 0) {
        const double kick = pow(lam / P.lambda_ref, -0.2);
        const int64_t N = P.screen_n;
        for (int i = P.n_layers - 1; i >= 0; --i) {
            const double h = P.height[i];
            const double l = (h - p[2]) / n[2];
            p[0] += n[0] * l;
            p[1] += n[1] * l;
            p[2] = h;
            const double sx = p[0] - P.wind[i][0] * t;
            const double sy = p[1] - P.wind[i][1] * t;
            double gx = 0.0, gy = 0.0;
            for (int s = 0; s < P.n_scales; ++s) {
                const float2* g = P.grad + ((size_t)(i * P.n_scales + s)) * N * N;
                double ax, ay;
                screen_tap(g, N, sx * P.inv_pix[s], sy * P.inv_pix[s], ax, ay);
                gx += ax;
                gy += ay;
            }
            n[0] += kick * gx;
            n[1] += kick * gy;
            normalise(n);
        }
    }
    {
        const double l = (P.z_start - p[2]) / n[2];
        p[0] += n[0] * l;
        p[1] += n[1] * l;
        p[2] = P.z_start;
    }
    if (P.obsc_r > 0.0) {
        const double l = (P.obsc_z - p[2]) / n[2];
        const double x = p[0] + n[0] * l, y = p[1] + n[1] * l;
        if (sqrt(x * x + y * y) < P.obsc_r) {
            o.status = PHX_OBSCURED;
            o.surface = -1;
            o.x = x; o.y = y; o.z = P.obsc_z;
            return o;
        }
    }

    const double n_glass = P.has_glass ? sellmeier(P, lam) : 1.0;
    double n_cur = 1.0;
    uint4 wc = make_uint4(0, 0, 0, 0);
    int wc_block = -1;
    for (int k = 0; k < P.n_surf; ++k) {
        const DevSurface& s = P.surf[k];
        double q[3], d[3];
        if (s.moved) {
            const double r0 = p[0] - s.t[0], r1 = p[1] - s.t[1], r2 = p[2] - s.t[2];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                q[i] = s.R[i] * r0 + s.R[3 + i] * r1 + s.R[6 + i] * r2;
                d[i] = s.R[i] * n[0] + s.R[3 + i] * n[1] + s.R[6 + i] * n[2];
            }
        } else {
            q[0] = p[0]; q[1] = p[1]; q[2] = p[2] - s.t[2];
            d[0] = n[0]; d[1] = n[1]; d[2] = n[2];
        }
        double l, gx = 0.0, gy = 0.0;
        int st = intersect(P, s, q, d, l, gx, gy, o.newton);
        if (st == 0 && !(l > 0.0)) st = PHX_MISSED;
        if (st != 0) {
            o.status = st; o.surface = k; o.x = q[0]; o.y = q[1]; o.z = q[2];
            return o;
        }
        q[0] += d[0] * l; q[1] += d[1] * l; q[2] += d[2] * l;
        const double rq = sqrt(q[0] * q[0] + q[1] * q[1]);
        if (rq < s.r_in || rq > s.r_out) {
            o.status = PHX_VIGNETTED; o.surface = k; o.x = q[0]; o.y = q[1]; o.z = q[2];
            return o;
        }
        double N[3] = {-gx, -gy, 1.0};
        normalise(N);
        double dn = d[0] * N[0] + d[1] * N[1] + d[2] * N[2];
        if (dn > 0.0) { N[0] = -N[0]; N[1] = -N[1]; N[2] = -N[2]; dn = -dn; }
        const double cosi = -dn;
        if ((L.flags & PHX_F_COATINGS) && s.coating >= 0) {
            const int blk = 2 + (k >> 2);
            if (blk != wc_block) { wc = rng.block(blk); wc_block = blk; }
            const uint32_t ws[4] = {wc.x, wc.y, wc.z, wc.w};
            const double T = coating(P, s.coating, 1.0 - cosi * cosi, lam);
            if (!(u01(ws[k & 3]) < T)) {
                o.status = PHX_ABSORBED; o.surface = k; o.x = q[0]; o.y = q[1]; o.z = q[2];
                return o;
            }
        }
        const bool det = s.kind == PHX_DETECTOR;
        if (s.kind == PHX_MIRROR) {
            d[0] -= 2.0 * dn * N[0]; d[1] -= 2.0 * dn * N[1]; d[2] -= 2.0 * dn * N[2];
        } else if (!det || (L.flags & PHX_F_SILICON)) {
            const double n2 = s.medium == PHX_GLASS ? n_glass
                            : (s.medium == PHX_SILICON ? n_silicon(lam) : 1.0);
            const double mu = n_cur / n2;
            const double kk = 1.0 - mu * mu * (1.0 - cosi * cosi);
            if (kk < 0.0) {
                o.status = PHX_TIR; o.surface = k; o.x = q[0]; o.y = q[1]; o.z = q[2];
                return o;
            }
            const double f = mu * cosi - sqrt(kk);
            d[0] = mu * d[0] + f * N[0]; d[1] = mu * d[1] + f * N[1]; d[2] = mu * d[2] + f * N[2];
            n_cur = n2;
        }
        if (det) {
            o.x = q[0]; o.y = q[1]; o.z = q[2]; o.surface = k;
            double xc = q[0], yc = q[1];
            if (L.flags & PHX_F_SILICON) {
                // conversion length = mean free path x Exp(1) (section 2.4.2)
                const double alpha = absorption(P, lam);
                const double L_conv = alpha > 0.0 ? -log(u01(w1.z)) / alpha : INFINITY;
                const double depth = L_conv * fabs(d[2]);
                if (!(depth <= P.t_si)) {
                    o.status = PHX_ESCAPED;
                    return o;
                }
                xc += d[0] * L_conv;
                yc += d[1] * L_conv;
                if (L.flags & PHX_F_DIFFUSION) {
                    const uint4 wd = rng.block(6);
                    const double sigma = P.sigma_max * (P.t_si - depth) / P.t_si;
                    const double rad = sqrt(-2.0 * log(u01(wd.x)));
                    double sa, ca;
                    sincos(kTwoPi * u01(wd.y), &sa, &ca);
                    xc += sigma * rad * ca;
                    yc += sigma * rad * sa;
                }
            }
            o.xe = xc; o.ye = yc;
            const double fx = (xc - P.chip_x0) / P.pixel, fy = (yc - P.chip_y0) / P.pixel;
            const double ix = floor(fx), iy = floor(fy);
            o.status = PHX_OFF_CHIP;
            if (ix >= 0.0 && ix < (double)P.nx && iy >= 0.0 && iy < (double)P.ny) {
                o.status = PHX_DETECTED;
                o.pix_i = (int)ix;
                o.pix_j = (int)iy;
            }
            return o;
        }
        if (s.moved) {
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                p[i] = s.R[3 * i] * q[0] + s.R[3 * i + 1] * q[1] + s.R[3 * i + 2] * q[2] + s.t[i];
                n[i] = s.R[3 * i] * d[0] + s.R[3 * i + 1] * d[1] + s.R[3 * i + 2] * d[2];
            }
        } else {
            p[0] = q[0]; p[1] = q[1]; p[2] = q[2] + s.t[2];
            n[0] = d[0]; n[1] = d[1]; n[2] = d[2];
        }
    }
    o.status = PHX_MISSED;
    o.surface = P.n_surf;
    return o;
}

// Wavefront-aggregated increment: lanes with the same pixel elect one leader that adds the
// group's count.
__device__ __forceinline__ void bin_photon(uint32_t* image, int pix, bool active) {
    uint64_t pending = __ballot(active);
    const int lane = __lane_id();
    while (pending) {
        const int leader = __ffsll((unsigned long long)pending) - 1;
        const int key = __shfl(pix, leader);
        const uint64_t same = __ballot(active && pix == key);
        if (lane == leader) atomicAdd(&image[key], (uint32_t)__popcll(same));
        pending &= ~same;
    }
}

__global__ __launch_bounds__(kBlock) void trace_kernel(const DevParams* __restrict__ Pg,
                                                       const Launch L) {
    __shared__ uint32_t s_stats[PHX_STATS_LEN];
    for (int i = threadIdx.x; i < PHX_STATS_LEN; i += blockDim.x) s_stats[i] = 0;
    __syncthreads();
    const DevParams& P = *Pg;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    // every lane of a wavefront runs the same number of iterations (bin_photon uses ballots)
    const uint64_t n_iter = (L.total + stride - 1) / stride;
    uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t newton = 0, traced = 0;
    for (uint64_t it = 0; it < n_iter; ++it, g += stride) {
        const bool valid = g < L.total;
        int pix = -1;
        if (valid) {
            int s;
            uint64_t local;
            if (L.uniform_count) {
                s = (int)(g / L.uniform_count);
                local = g - (uint64_t)s * L.uniform_count;
            } else {
                int lo = 0, hi = L.n_src - 1;   // largest s with prefix[s] <= g
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (L.prefix[mid] <= g) lo = mid; else hi = mid - 1;
                }
                s = lo;
                local = g - L.prefix[s];
            }
            const int si = L.src_begin + s;
            const uint64_t idx = L.photon_begin + local;
            const Outcome o = trace_photon(P, L, si, idx);
            atomicAdd(&s_stats[o.status * PHX_STAT_COLS + min(o.surface + 1, PHX_STAT_COLS - 1)], 1u);
            newton += o.newton;
            traced += o.status != PHX_CULLED;
            if (o.status == PHX_DETECTED) pix = o.pix_j * P.nx + o.pix_i;
            if ((L.flags & PHX_F_MOMENTS) && o.status <= PHX_OFF_CHIP) {
                double* m = L.moments + (size_t)si * PHX_MOMENT_LEN;
                atomicAdd(m + 0, 1.0);
                atomicAdd(m + 1, o.xe);
                atomicAdd(m + 2, o.ye);
                atomicAdd(m + 3, o.xe * o.xe);
                atomicAdd(m + 4, o.ye * o.ye);
                atomicAdd(m + 5, o.xe * o.ye);
            }
            if ((L.flags & PHX_F_EVENTS) && (g % L.event_stride) == 0) {
                phx_event& e = L.events[g / L.event_stride];
                e.photon = idx; e.source = si; e.status = o.status; e.surface = o.surface;
                e.pix_i = o.pix_i; e.pix_j = o.pix_j; e.newton = o.newton;
                e.x = o.x; e.y = o.y; e.z = o.z; e.xe = o.xe; e.ye = o.ye; e.lambda = o.lam;
            }
        }
        bin_photon(L.image, pix, pix >= 0);
    }
    atomicAdd(&s_stats[PHX_STAT_NEWTON], newton);
    atomicAdd(&s_stats[PHX_STAT_TRACED], traced);
    __syncthreads();
    if (L.stats) {
        for (int i = threadIdx.x; i < PHX_STATS_LEN; i += blockDim.x)
            if (s_stats[i]) atomicAdd(&L.stats[i], (unsigned long long)s_stats[i]);
    }
}

// Centred-difference gradients of periodic OPD screens (the refractive kick of section 2.3.2 is
// the phase gradient), single precision: g_x = (W[j][i+1] - W[j][i-1]) * (1/(2p)).
__global__ void gradient_kernel(const float* __restrict__ opd, float2* __restrict__ grad, int n,
                                int n_scales, const float* inv2p, int64_t total) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= total) return;
    const int64_t nn = (int64_t)n * n;
    const int64_t plane = id / nn;
    const int64_t r = id - plane * nn;
    const int j = (int)(r / n), i = (int)(r - (int64_t)j * n);
    const float* w = opd + plane * nn;
    const float f = inv2p[plane % n_scales];
    const int ip = i + 1 == n ? 0 : i + 1, im = i == 0 ? n - 1 : i - 1;
    const int jp = j + 1 == n ? 0 : j + 1, jm = j == 0 ? n - 1 : j - 1;
    const float dx = w[(int64_t)j * n + ip] - w[(int64_t)j * n + im];
    const float dy = w[(int64_t)jp * n + i] - w[(int64_t)jm * n + i];
    grad[id] = make_float2(dx * f, dy * f);
}

}  // namespace

hipError_t launch_trace(const DevParams* dparams, const Launch& L, int n_cu, hipStream_t stream) {
    if (L.total == 0) return hipSuccess;
    const uint64_t want = (L.total + kBlock - 1) / kBlock;
    const uint64_t cap = (uint64_t)n_cu * 8;
    const int grid = (int)(want < cap ? want : cap);
    hipLaunchKernelGGL(trace_kernel, dim3(grid), dim3(kBlock), 0, stream, dparams, L);
    return hipGetLastError();
}

hipError_t launch_gradients(const float* opd, float2* grad, int n_layers, int n_scales, int n,
                            const double* pixel, hipStream_t stream) {
    // inverse 2p per scale, rounded to float once (the same value for every texel)
    float h_inv2p[PHX_MAX_SCALES];
    for (int s = 0; s < n_scales; ++s) h_inv2p[s] = (float)(1.0 / (2.0 * pixel[s]));
    float* d_inv2p = nullptr;
    hipError_t e = hipMallocAsync((void**)&d_inv2p, sizeof(h_inv2p), stream);
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(d_inv2p, h_inv2p, sizeof(float) * n_scales, hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) return e;
    const int64_t total = (int64_t)n_layers * n_scales * n * n;
    const int block = 256;
    const int64_t grid = (total + block - 1) / block;
    hipLaunchKernelGGL(gradient_kernel, dim3((unsigned)grid), dim3(block), 0, stream, opd, grad, n,
                       n_scales, d_inv2p, total);
    e = hipGetLastError();
    (void)hipFreeAsync(d_inv2p, stream);
    return e;
}

}  // namespace phx
