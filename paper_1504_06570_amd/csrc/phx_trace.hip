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

#include <mutex>

#include "phx_internal.h"
#include "phx_rng.h"

namespace phx {
namespace {

constexpr double kHcEvM = 1.2398419843320026e-6;  // h c / e in eV m
constexpr double kPi = 3.141592653589793;
// Newton stops once a step is at most 1e-12 m (the paper's criterion is 0.01 um).  The root is
// then exact to rounding (convergence is quadratic), but the slope that gives the surface normal
// is the one evaluated before the last step, a step away from the hit point: with a 1e-9 m stop
// the normal of the secondary carried an error of about c x 1e-9 rad, which moved the hit on the
// next mirror by up to 8e-10 m; at 1e-12 m that error is below 1e-13 m.
constexpr double kNewtonTol = 1e-12;             // m
constexpr int kNewtonMax = 16;
constexpr int kBlock = kThreads;
constexpr int kTimeBuckets = kTimeBucketsMax;   // time buckets of the survivor sort
static_assert(kTimeBuckets <= 64, "bucket ids are stored in one byte and queued in six bits");

// Reciprocal and reciprocal square root for well-scaled operands (no zeros, infinities or
// denormals): the hardware estimate refined by two Newton steps, about 1 ulp; used for the
// continuous geometry (decisions that quantise, like the pixel index, keep IEEE division).
__device__ __forceinline__ double rcp_fast(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}
__device__ __forceinline__ double rsq_fast(double x) {
    double y = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x;
    double e = fma(-h * y, y, 0.5);
    y = fma(y, e, y);
    e = fma(-h * y, y, 0.5);
    return fma(y, e, y);
}
// sqrt(x) for x >= 0 via the reciprocal square root (0 maps to 0).
__device__ __forceinline__ double sqrt_fast(double x) { return x > 0.0 ? x * rsq_fast(x) : 0.0; }

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

// Zernike deformation as a bivariate polynomial of degree 4 in (u, v) = (x, y)/R: the host
// expands the Noll Z4..Z15 amplitudes into monomial coefficients c[] ordered (0,0) (1,0) (0,1)
// (2,0) (1,1) (0,2) (3,0) (2,1) (1,2) (0,3) (4,0) (3,1) (2,2) (1,3) (0,4).  Returns the value and
// the partial derivatives in u and v (Horner in u within each power of v).
__device__ __forceinline__ void zernike_poly(const double* c, double u, double v, double& s,
                                             double& du, double& dv) {
    const double p0 = c[0] + u * (c[1] + u * (c[3] + u * (c[6] + u * c[10])));
    const double p1 = c[2] + u * (c[4] + u * (c[7] + u * c[11]));
    const double p2 = c[5] + u * (c[8] + u * c[12]);
    const double p3 = c[9] + u * c[13];
    const double p4 = c[14];
    s = p0 + v * (p1 + v * (p2 + v * (p3 + v * p4)));
    const double q0 = c[1] + u * (2.0 * c[3] + u * (3.0 * c[6] + u * 4.0 * c[10]));
    const double q1 = c[4] + u * (2.0 * c[7] + u * 3.0 * c[11]);
    const double q2 = c[8] + u * 2.0 * c[12];
    const double q3 = c[13];
    du = q0 + v * (q1 + v * (q2 + v * q3));
    dv = p1 + v * (2.0 * p2 + v * (3.0 * p3 + v * 4.0 * p4));
}

// Sag S(x, y) and g with (dS/dx, dS/dy) = (x g, y g) + zernike gradient.  Returns false outside
// the conic's domain.
template <bool ZERN>
__device__ __forceinline__ bool sag(const DevParams& P, const DevSurface& s, double x, double y,
                                    double& S, double& gx, double& gy) {
    const double r2 = x * x + y * y;
    const double arg = 1.0 - s.kappa1 * s.c * s.c * r2;
    if (arg < 0.0) return false;
    // conic: S = c r^2 / (1 + root), dS/dr / r = c / root, root = sqrt(arg); one reciprocal
    // square root and one reciprocal
    const double inv_root = rsq_fast(arg);
    const double root = arg * inv_root;
    S = s.c * r2 * rcp_fast(1.0 + root);
    double g = s.c * inv_root;
    if (s.asphere == 1) {
        // even terms only: Horner in r^2
        const double* a = s.alpha;
        S += r2 * r2 * (a[1] + r2 * (a[3] + r2 * (a[5] + r2 * a[7])));
        g += r2 * (4.0 * a[1] + r2 * (6.0 * a[3] + r2 * (8.0 * a[5] + r2 * 10.0 * a[7])));
    } else if (s.asphere == 2) {
        // general: sum alpha_i r^i and sum i alpha_i r^(i-2), i = 3..10
        const double r = sqrt_fast(r2);
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
    if (ZERN && s.zernike) {
        double zs, zu, zv;
        zernike_poly(P.zern, x * P.zern_inv_r, y * P.zern_inv_r, zs, zu, zv);
        S += zs;
        gx += zu * P.zern_inv_r;
        gy += zv * P.zern_inv_r;
    }
    return true;
}

// Intersection of the ray q + l d with the surface: exact conic root, then Newton on
// f(l) = q_z + l d_z - S(q_x + l d_x, q_y + l d_y).  Returns 0 or a status; gx, gy receive the
// sag gradient at the last evaluation.
template <bool ZERN>
__device__ int intersect(const DevParams& P, const DevSurface& s, const double q[3],
                         const double d[3], double& l, double& gx, double& gy, int& iters) {
    if (s.c == 0.0 && s.asphere == 0 && !(ZERN && s.zernike)) {
        // a plane (the conic root below with c = 0: l = q_z / -d_z), slope zero
        if (d[2] == 0.0) return PHX_MISSED;
        l = -q[2] * rcp_fast(d[2]);
        gx = 0.0;
        gy = 0.0;
        return 0;
    }
    const double A = s.c * (d[0] * d[0] + d[1] * d[1] + s.kappa1 * d[2] * d[2]);
    const double B = s.c * (q[0] * d[0] + q[1] * d[1] + s.kappa1 * q[2] * d[2]) - d[2];
    const double C = s.c * (q[0] * q[0] + q[1] * q[1] + s.kappa1 * q[2] * q[2]) - 2.0 * q[2];
    const double disc = B * B - A * C;
    if (disc < 0.0) return PHX_MISSED;
    const double sq = sqrt_fast(disc);
    const double den = B >= 0.0 ? B + sq : B - sq;
    if (den == 0.0) return PHX_MISSED;
    l = -C * rcp_fast(den);
    if (s.asphere == 0 && !(ZERN && s.zernike)) {
        // a plain conic: the root is the intersection (a Newton update would be rounding-sized,
        // far below the tolerance); only the slope at the hit point is needed
        const double x = q[0] + l * d[0], y = q[1] + l * d[1];
        const double arg = 1.0 - s.kappa1 * s.c * s.c * (x * x + y * y);
        if (arg < 0.0) return PHX_MISSED;
        const double g = s.c * rsq_fast(arg);
        gx = x * g;
        gy = y * g;
        return 0;
    }
#pragma unroll 1
    for (int it = 1; it <= kNewtonMax; ++it) {
        const double x = q[0] + l * d[0], y = q[1] + l * d[1], z = q[2] + l * d[2];
        double S;
        if (!sag<ZERN>(P, s, x, y, S, gx, gy)) return PHX_MISSED;
        const double fp = d[2] - (gx * d[0] + gy * d[1]);
        if (fp == 0.0) return PHX_NONCONV;
        const double dl = (z - S) * rcp_fast(fp);
        l -= dl;
        iters += 1;
        if (fabs(dl) <= kNewtonTol) return 0;
    }
    return PHX_NONCONV;
}

// Position of a wavelength on the coating tables' uniform wavelength axis (clamped at the ends):
// column il and weight b of column il + 1.  Computed once per photon.
struct LamCol {
    int il;
    double b;
};
__device__ __forceinline__ LamCol lambda_column(const DevParams& P, double lam) {
    double fl = (lam - P.lam0) * P.inv_dlam;
    fl = fmin(fmax(fl, 0.0), (double)(P.n_lam - 1));
    const int il = min((int)floor(fl), P.n_lam - 2);
    return LamCol{il, fl - il};
}

// Coating transmission (section 2.4.2): bilinear in s = sin^2(incidence) and wavelength.
__device__ __forceinline__ double coating(const DevParams& P, int c, double s, const LamCol& lc,
                                          const float* table = nullptr) {
    double fs = s * P.inv_s_step;
    fs = fmin(fmax(fs, 0.0), (double)(P.n_s - 1));
    const int is = min((int)floor(fs), P.n_s - 2);
    const double a = fs - is, b = lc.b;
    const float* r0 = (table ? table : P.coat) + ((size_t)c * P.n_s + is) * P.n_lam + lc.il;
    const float* r1 = r0 + P.n_lam;
    return (1.0 - a) * ((1.0 - b) * (double)r0[0] + b * (double)r0[1]) +
           a * ((1.0 - b) * (double)r1[0] + b * (double)r1[1]);
}


// Bilinear interpolation of one gradient screen at screen-pixel coordinates (xs, ys): one
// 32-byte record per cell holds the four corner gradients.
__device__ __forceinline__ void screen_tap(const float4* g, int64_t N, double xs, double ys,
                                           double& ax, double& ay) {
    const double fx = floor(xs), fy = floor(ys);
    const double a = xs - fx, b = ys - fy;
    const int64_t m = N - 1;
    const int64_t i0 = (int64_t)fx & m, j0 = (int64_t)fy & m;
    const float4* rec = g + 2 * (j0 * N + i0);
    const float4 lo = rec[0], hi = rec[1];   // (i,j) (i+1,j) | (i,j+1) (i+1,j+1)
    ax = (1.0 - b) * ((1.0 - a) * (double)lo.x + a * (double)lo.z) +
         b * ((1.0 - a) * (double)hi.x + a * (double)hi.z);
    ay = (1.0 - b) * ((1.0 - a) * (double)lo.y + a * (double)lo.w) +
         b * ((1.0 - a) * (double)hi.y + a * (double)hi.w);
}

__device__ __forceinline__ void normalise(double n[3]) {
    const double inv = 1.0 / sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    n[0] *= inv; n[1] *= inv; n[2] *= inv;
}

// Gamma(shape) by Marsaglia & Tsang, trial t on stream 1 block t.
__device__ double gamma_sample(const Rng& rng, double shape) {
    const double a = shape < 1.0 ? shape + 1.0 : shape;
    const double dd = a - 1.0 / 3.0, cc = 1.0 / sqrt(9.0 * dd);
#pragma unroll 1
    for (uint32_t t = 0; t < 64; ++t) {
        const uint4 w = rng.block(t, 1);
        const double u0 = u01(w.x), u1 = u01(w.y), u2 = u01(w.z);
        const double x = sqrt(-2.0 * log(u0)) * cospi(2.0 * u1);
        double v = 1.0 + cc * x;
        if (v <= 0.0) continue;
        v = v * v * v;
        const double x2 = x * x;
        bool accept = u2 < 1.0 - 0.0331 * x2 * x2;
        if (!accept) accept = log(u2) < 0.5 * x2 + dd * (1.0 - v + log(v));
        if (accept) {
            double g = dd * v;
            if (shape < 1.0) g *= exp(log(u01(w.w)) / shape);
            return g;
        }
    }
    return shape;
}

// Wavelength (section 2.2): flat photon spectrum, or the SED's photon CDF (first bin k with
// CDF[k+1] > u, found by bisection between two entries of a guide table) blurred uniformly
// across the bin; then (1 + z).
__device__ __forceinline__ double wavelength(const DevParams& P, const DevSource& src,
                                             const uint4& w0, const uint4& w1) {
    double lam;
    if (src.sed < 0) {
        lam = src.lambda_lo + u01(w0.w) * src.lambda_span;
    } else {
        const double* cdf = P.sed_cdf + (size_t)src.sed * (P.sed_k + 1);
        const double u = u01(w0.w);
        // the answer lies between the guide entries around u (u kSedGuide is exact)
        const uint16_t* guide = P.sed_guide + (size_t)src.sed * (kSedGuide + 1);
        const int j = min((int)(u * kSedGuide), kSedGuide - 1);
        int lo = guide[j], hi = guide[j + 1];
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (cdf[mid + 1] > u) hi = mid; else lo = mid + 1;
        }
        lam = P.sed_edges[lo] + u01(w1.x) * (P.sed_edges[lo + 1] - P.sed_edges[lo]);
    }
    return lam * src.redshift1;
}

// Pre-roll test (section 3.2): a photon is culled when a coated surface's roulette draw exceeds
// the largest transmission that coating has at this wavelength for any angle, so it cannot
// survive.  The coated surfaces are tested in order of decreasing selectivity.  preroll_draw
// gives the wavelength (and the time and radius words) from the photon's first Philox blocks.
__device__ __forceinline__ double preroll_draw(const DevParams& P, const Rng& rng,
                                               const DevSource& src, uint32_t& w_time,
                                               uint32_t& w_radius) {
    const uint4 w0 = rng.block(0);
    w_time = w0.z;
    w_radius = w0.x;
    uint4 w1 = make_uint4(0, 0, 0, 0);
    if (src.sed >= 0) w1 = rng.block(1);
    return wavelength(P, src, w0, w1);
}

__device__ __forceinline__ uint32_t word_of(const uint4& w, int m) {
    return m == 0 ? w.x : (m == 1 ? w.y : (m == 2 ? w.z : w.w));
}

// The first (most selective) test, at wavelength column il; only surfaces below k_lim are
// tested (with ghosts: the coated surfaces every photon passes sequentially).
template <bool GHOST>
__device__ __forceinline__ bool preroll_first(const DevParams& P, const Rng& rng, int il,
                                              int k_lim) {
    const int k = P.cull_order[0];
    if (GHOST && k >= k_lim) return false;
    const uint32_t wk = word_of(rng.block(2 + (k >> 2)), k & 3);
    return (int64_t)wk > P.coat_thr[(size_t)P.surf[k].coating * P.n_lam + il];
}

// Tests 1..n_tests-1 in order, stopping at the first that culls; a roulette block is drawn when
// the next test's surface needs a different one.
template <bool GHOST>
__device__ __forceinline__ bool preroll_rest(const DevParams& P, const Rng& rng, int il,
                                             int n_tests, int k_lim) {
    int blk = -1;
    uint4 w = make_uint4(0, 0, 0, 0);
    for (int j = 1; j < n_tests; ++j) {
        const int k = P.cull_order[j];
        if (GHOST && k >= k_lim) continue;
        if (2 + (k >> 2) != blk) {
            blk = 2 + (k >> 2);
            w = rng.block(blk);
        }
        if ((int64_t)word_of(w, k & 3) > P.coat_thr[(size_t)P.surf[k].coating * P.n_lam + il])
            return true;
    }
    return false;
}

// Pre-roll escape test (section 3.2 with the silicon stage): the photon converts deeper than the
// silicon whatever its path, since its conversion distance (the silicon stage's draw) times the
// smallest cosine a ray refracted into silicon can have exceeds the thickness.  The ray reaches
// silicon from vacuum or glass, so sin(theta) in silicon is at most n_in / n_Si with n_in the
// glass index when the optics hold glass; the relative margin 1e-12 covers the rounding of the
// optics stage's refracted direction.  Kept out of line: it runs for few photons, and inlined it
// raises the register count of the whole pre-roll.
__device__ __noinline__ bool escape_certain(const DevParams& P, double lam, uint32_t w_conv) {
    const double alpha = absorption(P, lam);
    const double L_conv = alpha > 0.0 ? -log(u01(w_conv)) / alpha : INFINITY;
    const double q = (P.has_glass ? sellmeier(P, lam) : 1.0) / n_silicon(lam);
    if (!(q < 1.0)) return false;
    const double cos_min = sqrt(1.0 - q * q);
    return L_conv * cos_min * (1.0 - 1e-12) > P.t_si;
}

// ---------------------------------------------------------------------------------------------
// Per-photon physics beyond the core path.  Only the sky and optics kernel instantiations with
// EXTRA = true contain this code (the launch picks them when one of its flags is set), so the
// registers and occupancy of the other instantiations do not depend on it.

__device__ __forceinline__ double3 unit3(double3 v) {
    const double inv = 1.0 / sqrt(v.x * v.x + v.y * v.y + v.z * v.z);
    return make_double3(v.x * inv, v.y * inv, v.z * inv);
}

// Atmospheric dispersion (section 2.3.3): the direction moves by R(lambda) - R(lambda0) along the
// zenith direction in (n_x, n_y), R = (n_air - 1) tan z, n_air from the Filippenko formula with
// its pressure-temperature and water factors precomputed; the difference of the dry brackets and
// of the water terms is taken before scaling, so no 1 + 3e-4 is formed.
__device__ __forceinline__ double3 disperse(const DevParams& P, double lam, double3 n) {
    const DevPhysics& X = P.ph;
    const double lu = lam * 1e6;
    const double s = 1.0 / (lu * lu);
    const double b = 64.328 + 29498.1 / (146.0 - s) + 255.4 / (41.0 - s);
    const double dR =
        1e-6 * (X.disp_pt * (b - X.disp_b0) + 0.000680 * X.disp_w * (s - X.disp_s0)) * X.disp_tanz;
    n.x += dR * X.disp_cx;
    n.y += dR * X.disp_cy;
    return unit3(n);
}

// Dome seeing and the micro-roughness halo (section 2.4.2), kicks of the direction on the start
// plane.  Dome: a normal kick of dome_sigma per axis (Box-Muller on block 8).  Halo: with
// probability f (block 7, word y) an angle r0 x toward the azimuth of block 7 word z; x has
// density proportional to x / (1 + x^n) on [0, x_max], drawn by rejection from the density
// x (1 + x^2)^(-n/2), whose CDF 1 - (1 + x^2)^(1 - n/2) inverts in closed form, keeping a trial
// when u < (1 + x^2)^(n/2) / (1 + x^n) / 2^(n/2 - 1) (the ratio's maximum, at x = 1); trial t
// reads stream 2 block t (proposal x, acceptance y); after 32 rejections no kick.
__device__ __forceinline__ double3 entrance_kicks(const DevParams& P, uint32_t flags, Rng rng,
                                               double3 n) {
    const DevPhysics& X = P.ph;
    if (flags & PHX_F_DOME) {
        const uint4 w = rng.block(8);
        const double rad = sqrt(-2.0 * log(u01(w.x)));
        double sa, ca;
        sincospi(2.0 * u01(w.y), &sa, &ca);
        n.x += X.dome_sigma * rad * ca;
        n.y += X.dome_sigma * rad * sa;
        n = unit3(n);
    }
    if (flags & PHX_F_HALO) {
        const uint4 w7 = rng.block(7);
        if (u01(w7.y) < X.halo_f) {
            double x = -1.0;
#pragma unroll 1
            for (uint32_t t = 0; t < 32; ++t) {
                const uint4 w = rng.block(t, 2);
                const double xt = sqrt(exp(log(1.0 - u01(w.x) * X.halo_fq) / X.halo_e) - 1.0);
                const double ratio =
                    exp(0.5 * X.halo_n * log(1.0 + xt * xt)) / (1.0 + exp(X.halo_n * log(xt)));
                if (u01(w.y) < ratio * X.halo_inv_m) {
                    x = xt;
                    break;
                }
            }
            if (x >= 0.0) {
                const double r = X.halo_r0 * x;
                double sa, ca;
                sincospi(2.0 * u01(w7.z), &sa, &ca);
                n.x += r * ca;
                n.y += r * sa;
                n = unit3(n);
            }
        }
    }
    return n;
}

// Second kick of the hybrid atmosphere at layer i (section 2.3.2): the long-exposure PSF of the
// layer's modes above kappa_crit, exp(-D/2) in the pupil, is the compound Poisson law of
// K ~ Poisson(s2_i) scatterings (count word wk; K = the smallest k whose cumulative probability
// exceeds the uniform, at most 8), each a deflection lambda_ref kappa / (2 pi) toward a uniform
// azimuth with kappa from the phase spectrum on [kappa_crit, kappa_max] by inverting
// (A(kappa_crit) - A(kappa)) / dA, A = (kappa^2 + kappa0^2)^(-5/6) (stream 3, block 8 i + j:
// wavenumber x, azimuth y).  Adds the deflection to (gx, gy).
__device__ __forceinline__ void second_kick(const DevParams& P, const Rng& rng, int i,
                                            uint32_t wk, double& gx, double& gy) {
    const DevPhysics& X = P.ph;
    const double uk = u01(wk);
    double p = X.kick_p0[i], cum = p;
    if (uk < cum) return;
    const double s2 = X.kick_s2[i];
    int K = 0;
    while (!(uk < cum) && K < 8) {
        ++K;
        p *= s2 / K;
        cum += p;
    }
#pragma unroll 1
    for (int j = 0; j < K; ++j) {
        const uint4 w = rng.block((uint32_t)(8 * i + j), 3);
        const double A = X.kick_A0 - u01(w.x) * X.kick_dA;
        const double kappa = sqrt(exp(-1.2 * log(A)) - X.kick_k02);
        const double th = P.lambda_ref * kappa / (2.0 * kPi);
        double sa, ca;
        sincospi(2.0 * u01(w.y), &sa, &ca);
        gx += th * ca;
        gy += th * sa;
    }
}

// Aerosol extinction (section 2.3.3) and the spider (sections 2.4.1-2.4.2) at the telescope
// entrance.  status 0: the photon lives (a ray that passes the spider is moved to the vanes'
// mid-height and turned); PHX_EXTINCT with p the start-plane point; PHX_OBSCURED with p the first
// point along the ray inside a vane.
struct Entry {
    double3 p, n;
    int status;
};

// One slab of the ray-box test: narrows [t0, t1] to the parameters where o + t d lies in [lo, hi].
__device__ __forceinline__ void slab(double o, double d, double lo, double hi, double& t0,
                                     double& t1, bool& inside) {
    if (d == 0.0) {
        if (o < lo || o > hi) inside = false;
        return;
    }
    double ta = (lo - o) / d, tb = (hi - o) / d;
    if (ta > tb) {
        const double tmp = ta;
        ta = tb;
        tb = tmp;
    }
    t0 = fmax(t0, ta);
    t1 = fmin(t1, tb);
}

// Aerosol: survival with probability exp(-tau sec z), tau = tau0 (lambda / 500 nm)^gamma (block 7
// word x).  Spider: vane k is the box u in [r_in, r_out], |v| <= w/2, z in [z_lo, z_hi] along
// u = (c_k, s_k, 0), v = (-s_k, c_k, 0).  A ray that passes every box turns by
// lambda / (4 pi max(d, lambda)) along +v or -v of the nearest vane (block 7 word w), d = the
// smallest distance between the ray's line and a vane's long edge (segment along u at v = +-w/2,
// z = z_lo or z_hi: the closest point of the infinite edge line, clamped to the segment, then its
// distance to the ray's line).
__device__ __forceinline__ Entry entrance_extra(const DevParams& P, uint32_t flags, Rng rng,
                                             double lam, double3 p, double3 n) {
    const DevPhysics& X = P.ph;
    const uint4 w7 = rng.block(7);
    if (flags & PHX_F_AEROSOL) {
        const double tau = X.tau0 * exp(X.gamma * log(lam / 500e-9)) * X.airmass;
        if (!(u01(w7.x) < exp(-tau))) return Entry{p, n, PHX_EXTINCT};
    }
    if ((flags & PHX_F_SPIDER) && X.vanes > 0) {
        double best = INFINITY, t_hit = INFINITY;
        int bk = -1;
#pragma unroll 1
        for (int k = 0; k < X.vanes; ++k) {
            const double c = X.vane_c[k], s = X.vane_s[k];
            double t0 = -INFINITY, t1 = INFINITY;
            bool inside = true;
            slab(p.x * c + p.y * s, n.x * c + n.y * s, X.vane_r0, X.vane_r1, t0, t1, inside);
            slab(-p.x * s + p.y * c, -n.x * s + n.y * c, -X.vane_hw, X.vane_hw, t0, t1, inside);
            slab(p.z, n.z, X.vane_z0, X.vane_z1, t0, t1, inside);
            if (inside && t0 <= t1 && t1 >= 0.0) {
                t_hit = fmin(t_hit, fmax(t0, 0.0));
                continue;
            }
            const double b = c * n.x + s * n.y;
            const double inv = 1.0 / (1.0 - b * b);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const double ve = (e & 1) ? X.vane_hw : -X.vane_hw;
                const double ze = (e & 2) ? X.vane_z1 : X.vane_z0;
                const double w0x = -ve * s - p.x, w0y = ve * c - p.y, w0z = ze - p.z;
                const double dw = c * w0x + s * w0y;
                const double ew = n.x * w0x + n.y * w0y + n.z * w0z;
                const double sc = fmin(fmax((b * ew - dw) * inv, X.vane_r0), X.vane_r1);
                const double rx = w0x + sc * c, ry = w0y + sc * s, rz = w0z;
                const double rn = rx * n.x + ry * n.y + rz * n.z;
                const double cx = rx - rn * n.x, cy = ry - rn * n.y, cz = rz - rn * n.z;
                const double dist = sqrt(cx * cx + cy * cy + cz * cz);
                if (dist < best) {
                    best = dist;
                    bk = k;
                }
            }
        }
        if (t_hit < INFINITY)
            return Entry{make_double3(p.x + n.x * t_hit, p.y + n.y * t_hit, p.z + n.z * t_hit), n,
                         PHX_OBSCURED};
        if (bk >= 0) {
            const double l = (X.vane_zm - p.z) / n.z;
            p = make_double3(p.x + n.x * l, p.y + n.y * l, X.vane_zm);
            double delta = lam / (4.0 * kPi * fmax(best, lam));
            if (!(u01(w7.w) < 0.5)) delta = -delta;
            n.x -= delta * X.vane_s[bk];
            n.y += delta * X.vane_c[bk];
            n = unit3(n);
        }
    }
    return Entry{p, n, 0};
}

struct Outcome {
    int status, surface, newton;
    int pix_i, pix_j;
    double x, y, z, xe, ye, lam;
};

// The whole per-photon path.  `culled` photons return PHX_CULLED without being traced.
// Photon state at the start plane above the optics.
struct Front {
    double p[3], n[3], lam;
};

// Sky sampling (sections 2.2, 2.2.1) and the atmosphere (sections 2.3.1-2.3.2), ending on the
// start plane above every optic.
template <bool SERSIC, bool EXTRA>
__device__ void photon_front(const DevParams& P, const Launch& L, int si, uint64_t idx, Front& f) {
    const DevSource& src = P.src[si];
    const Rng rng{L.seed, (uint32_t)si, (uint32_t)idx, (uint32_t)(idx >> 32)};
    const uint4 w0 = rng.block(0);
    uint4 w1 = make_uint4(0, 0, 0, 0);
    if (src.sed >= 0 || (SERSIC && src.kind == 1)) w1 = rng.block(1);
    const double lam = wavelength(P, src, w0, w1);

    // direction (section 2.2) and extended-source perturbation (section 2.2.1)
    double n[3] = {src.xi, src.eta, src.nz};
    if (SERSIC && src.kind == 1) {
        const double g = gamma_sample(rng, 2.0 * src.sersic_n);
        const double rr = exp(src.sersic_n * log(g / src.sersic_bn));
        double sp, cp;
        sincospi(2.0 * u01(w1.y), &sp, &cp);
        const double dmaj = src.sersic_a * rr * cp, dmin = src.sersic_b * rr * sp;
        n[0] += dmaj * src.cos_pa - dmin * src.sin_pa;
        n[1] += dmaj * src.sin_pa + dmin * src.cos_pa;
        normalise(n);
    }
    if (EXTRA && (L.flags & PHX_F_DISPERSION)) {
        const double3 m = disperse(P, lam, make_double3(n[0], n[1], n[2]));
        n[0] = m.x; n[1] = m.y; n[2] = m.z;
    }
    const double t = L.exposure * u01(w0.z);

    // pupil sample on the first surface (section 2.2)
    double p[3];
    {
        const double ro = P.pupil_r_out + L.pupil_margin;
        const double ri = fmax(P.pupil_r_in - L.pupil_margin, 0.0);
        const double r = sqrt(u01(w0.x) * (ro * ro - ri * ri) + ri * ri);
        double sphi, cphi;
        sincospi(2.0 * u01(w0.y), &sphi, &cphi);
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
        const double kick = exp(-0.2 * log(lam / P.lambda_ref));
        const int64_t N = P.screen_n;
        const bool second = EXTRA && (L.flags & PHX_F_SECOND_KICK);
        uint4 kw0 = make_uint4(0, 0, 0, 0), kw1 = make_uint4(0, 0, 0, 0);
        if (second) {
            kw0 = rng.block(9);
            if (P.n_layers > 4) kw1 = rng.block(10);
        }
#pragma unroll 1
        for (int i = P.n_layers - 1; i >= 0; --i) {
            const double h = P.height[i];
            const double l = (h - p[2]) * rcp_fast(n[2]);
            p[0] += n[0] * l;
            p[1] += n[1] * l;
            p[2] = h;
            const double sx = p[0] - P.wind[i][0] * t;
            const double sy = p[1] - P.wind[i][1] * t;
            double gx = 0.0, gy = 0.0;
#pragma unroll 1
            for (int s = 0; s < P.n_scales; ++s) {
                const float4* g = P.grad + ((size_t)(i * P.n_scales + s)) * N * N * 2;
                double ax, ay;
                screen_tap(g, N, sx * P.inv_pix[s], sy * P.inv_pix[s], ax, ay);
                gx += ax;
                gy += ay;
            }
            if (second) {
                // select by value: a select between the two blocks' addresses would keep them in
                // scratch memory
                const uint4 kw = i < 4 ? kw0 : kw1;
                second_kick(P, rng, i, word_of(kw, i & 3), gx, gy);
            }
            n[0] += kick * gx;
            n[1] += kick * gy;
            const double inv = rsq_fast(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
            n[0] *= inv;
            n[1] *= inv;
            n[2] *= inv;
        }
    }
    {
        const double l = (P.z_start - p[2]) * rcp_fast(n[2]);
        p[0] += n[0] * l;
        p[1] += n[1] * l;
        p[2] = P.z_start;
    }
    if (EXTRA && (L.flags & (PHX_F_DOME | PHX_F_HALO))) {
        const double3 m = entrance_kicks(P, L.flags, rng, make_double3(n[0], n[1], n[2]));
        n[0] = m.x; n[1] = m.y; n[2] = m.z;
    }
    f.p[0] = p[0]; f.p[1] = p[1]; f.p[2] = p[2];
    f.n[0] = n[0]; f.n[1] = n[1]; f.n[2] = n[2];
    f.lam = lam;
}

// Field model of the diffusion width (section 2.4.3): sigma^2 interpolated linearly in the
// library's table against depth below the entrance surface (zero beyond the collection height);
// `slope` = d sigma / d depth of the interpolant.
__device__ __forceinline__ double field_sigma(const DevParams& P, double depth, double& slope) {
    const DevPhysics& X = P.ph;
    slope = 0.0;
    if (!(depth < X.sig2_dmax)) return 0.0;
    const double f = depth * X.sig2_inv_step;
    const int k = min((int)f, X.n_sig2 - 1);
    const double a = f - k;
    const double s2 = (1.0 - a) * X.sig2[k] + a * X.sig2[k + 1];
    if (!(s2 > 0.0)) return 0.0;
    const double sigma = sqrt(s2);
    slope = (X.sig2[k + 1] - X.sig2[k]) * X.sig2_inv_step / (2.0 * sigma);
    return sigma;
}

// Silicon (sections 2.4.2-2.4.3): conversion after a path of mean free path x Exp(1) along the
// refracted direction d; escape if deeper than the silicon; Gaussian diffusion with sigma
// proportional to the drift distance to the collecting surface.  With PHX_F_DEAD_LAYER an
// electron converted less than `dead` below the entrance surface is removed (section 2.4.2
// field-free layer).  Moves (xc, yc) from the landing point to the electron position; returns 0,
// PHX_ESCAPED or PHX_DEAD.  Inlined: it raises the optics kernel's spills (20 -> 65 words), but a
// call would give the kernel a stack frame and register saves around it, which cost more
// (headline step 49.9 -> 48.5 ms inlined).
__device__ __forceinline__ int sensor_stage(const DevParams& P, const Launch& L, const Rng& rng,
                                         double lam, const double* d, double& xc, double& yc) {
    if (L.flags & PHX_F_SILICON) {
        const double alpha = absorption(P, lam);
        const double L_conv = alpha > 0.0 ? -log(u01(rng.block(1).z)) / alpha : INFINITY;
        const double depth = L_conv * fabs(d[2]);
        if (!(depth <= P.t_si)) return PHX_ESCAPED;
        if ((L.flags & PHX_F_DEAD_LAYER) && depth < P.ph.dead) return PHX_DEAD;
        xc += d[0] * L_conv;
        yc += d[1] * L_conv;
        if (L.flags & PHX_F_DIFFUSION) {
            const uint4 wd = rng.block(6);
            double slope;
            const double sigma = (L.flags & PHX_F_FIELD_DIFFUSION)
                                     ? field_sigma(P, depth, slope)
                                     : P.sigma_max * (P.t_si - depth) / P.t_si;
            const double rad = sqrt(-2.0 * log(u01(wd.x)));
            double sa, ca;
            sincospi(2.0 * u01(wd.y), &sa, &ca);
            xc += sigma * rad * ca;
            yc += sigma * rad * sa;
        }
    }
    return 0;
}

// Central obscuration, the surfaces (sections 2.4.1-2.4.2), silicon (sections 2.4.2-2.4.3) and
// the pixel, from the start-plane state.
struct Hit {
    double q[3], d[3], N[3];
    double dn, l;
};

// Transform into surface k's frame, intersect, clip to the clear aperture, take the normal and
// play the coating roulette (sections 2.4.1-2.4.2).  Returns 0 to continue or the photon's fate.
// Returned by hit_surface when a filter or anti-reflection coating reflects the photon (ghosts).
constexpr int kGhostReflect = 1000;

// Geometry of a surface passage: transform into surface k's frame, intersect, clip to the clear
// aperture, take the normal (facing the incoming ray).  Returns 0 or the photon's fate.
template <bool ZERN, bool TAPE = false>
__device__ __forceinline__ int hit_geometry(const DevParams& P, int k, const double p[3],
                                            const double n[3], Hit& h, int& newton) {
    const DevSurface& s = P.surf[k];
    if (s.moved) {
        const double r0 = p[0] - s.t[0], r1 = p[1] - s.t[1], r2 = p[2] - s.t[2];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            h.q[i] = s.R[i] * r0 + s.R[3 + i] * r1 + s.R[6 + i] * r2;
            h.d[i] = s.R[i] * n[0] + s.R[3 + i] * n[1] + s.R[6 + i] * n[2];
        }
    } else {
        h.q[0] = p[0]; h.q[1] = p[1]; h.q[2] = p[2] - s.t[2];
        h.d[0] = n[0]; h.d[1] = n[1]; h.d[2] = n[2];
    }
    double l, gx = 0.0, gy = 0.0;
    int st = intersect<ZERN>(P, s, h.q, h.d, l, gx, gy, newton);
    if (st == 0 && !(l > 0.0)) st = PHX_MISSED;
    if (st != 0) return st;
    if (TAPE) h.l = l;
    h.q[0] += h.d[0] * l; h.q[1] += h.d[1] * l; h.q[2] += h.d[2] * l;
    const double rq2 = h.q[0] * h.q[0] + h.q[1] * h.q[1];
    if (rq2 < s.r_in2 || rq2 > s.r_out2) return PHX_VIGNETTED;
    if (s.c == 0.0 && s.asphere == 0 && !(ZERN && s.zernike)) {
        h.N[0] = 0.0; h.N[1] = 0.0; h.N[2] = 1.0;   // a plane
    } else {
        const double inv = rsq_fast(gx * gx + gy * gy + 1.0);
        h.N[0] = -gx * inv; h.N[1] = -gy * inv; h.N[2] = inv;
    }
    h.dn = h.d[0] * h.N[0] + h.d[1] * h.N[1] + h.d[2] * h.N[2];
    if (h.dn > 0.0) { h.N[0] = -h.N[0]; h.N[1] = -h.N[1]; h.N[2] = -h.N[2]; h.dn = -h.dn; }
    return 0;
}

template <bool ZERN, bool TAPE = false, bool GHOST = false>
__device__ __forceinline__ int hit_surface(const DevParams& P, const Launch& L, const Rng& rng,
                                           int k, const double p[3], const double n[3],
                                           const LamCol& lc, uint4& wc, int& wc_block, Hit& h,
                                           int& newton) {
    const int g = hit_geometry<ZERN, TAPE>(P, k, p, n, h, newton);
    if (g != 0) return g;
    const DevSurface& s = P.surf[k];
    if ((L.flags & PHX_F_COATINGS) && s.coating >= 0) {
        const int blk = 2 + (k >> 2);
        if (blk != wc_block) { wc = rng.block(blk); wc_block = blk; }
        const int j = k & 3;
        const uint32_t w = j == 0 ? wc.x : (j == 1 ? wc.y : (j == 2 ? wc.z : wc.w));
        const double T = coating(P, s.coating, 1.0 - h.dn * h.dn, lc);
        if (!(u01(w) < T)) {
            if (GHOST && (L.flags & PHX_F_GHOSTS) && s.kind != PHX_MIRROR &&
                u01(w) < T + coating(P, s.coating, 1.0 - h.dn * h.dn, lc, P.coat_r))
                return kGhostReflect;
            return PHX_ABSORBED;
        }
    }
    return 0;
}

// Refraction by the vector form of Snell's law (section 2.4.2); false on total internal
// reflection.
__device__ __forceinline__ bool refract(Hit& h, double mu) {
    const double cosi = -h.dn;
    const double kk = 1.0 - mu * mu * (1.0 - cosi * cosi);
    if (kk < 0.0) return false;
    const double f = mu * cosi - sqrt_fast(kk);
    h.d[0] = mu * h.d[0] + f * h.N[0];
    h.d[1] = mu * h.d[1] + f * h.N[1];
    h.d[2] = mu * h.d[2] + f * h.N[2];
    return true;
}

// Tape of one surface passage for the adjoint: hit point and incoming direction in the
// element frame, and the path length from the previous surface, at tp[(k * kTapeFields + i) * ts].
__device__ __forceinline__ void tape_put(double* tp, uint64_t ts, int k, const Hit& h) {
    double* t = tp + (uint64_t)k * kTapeFields * ts;
    t[0] = h.q[0]; t[ts] = h.q[1]; t[2 * ts] = h.q[2];
    t[3 * ts] = h.d[0]; t[4 * ts] = h.d[1]; t[5 * ts] = h.d[2];
    t[6 * ts] = h.l;
}

// A photon between surfaces, in the global frame: position, direction and the index of the
// medium it travels in.
struct Ray {
    double p[3], n[3], n_cur;
};

// Per-photon constants of the optics stage: the glass index and the coating tables' wavelength
// column at the photon's wavelength.
struct Optics {
    double lam, n_glass;
    LamCol lc;
};
__device__ __forceinline__ Optics optics_of(const DevParams& P, const Launch& L, double lam) {
    Optics c;
    c.lam = lam;
    c.n_glass = P.has_glass ? sellmeier(P, lam) : 1.0;
    c.lc = (L.flags & PHX_F_COATINGS) && P.n_lam > 1 ? lambda_column(P, lam) : LamCol{0, 0.0};
    return c;
}

__device__ __forceinline__ void outcome_init(Outcome& o, double lam) {
    o.status = PHX_MISSED; o.surface = -1; o.newton = 0; o.pix_i = -1; o.pix_j = -1;
    o.x = o.y = o.z = o.xe = o.ye = 0.0;
    o.lam = lam;
}

// Central obscuration (section 2.4.1): true, with the outcome filled, if the ray meets it.
__device__ __forceinline__ bool obscured(const DevParams& P, const Ray& ray, Outcome& o) {
    if (!(P.obsc_r > 0.0)) return false;
    const double l = (P.obsc_z - ray.p[2]) / ray.n[2];
    const double x = ray.p[0] + ray.n[0] * l, y = ray.p[1] + ray.n[1] * l;
    if (!(sqrt(x * x + y * y) < P.obsc_r)) return false;
    o.status = PHX_OBSCURED;
    o.x = x; o.y = y; o.z = P.obsc_z;
    return true;
}

// Before the first surface: aerosol extinction and the spider (when their flags are set), then
// the central obscuration.  True while the photon lives, else the outcome is filled.
template <bool EXTRA>
__device__ __forceinline__ bool entrance(const DevParams& P, const Launch& L, const Rng& rng,
                                         Ray& ray, Outcome& o) {
    if (EXTRA && (L.flags & (PHX_F_AEROSOL | PHX_F_SPIDER))) {
        const Entry e = entrance_extra(P, L.flags, rng, o.lam,
                                       make_double3(ray.p[0], ray.p[1], ray.p[2]),
                                       make_double3(ray.n[0], ray.n[1], ray.n[2]));
        if (e.status != 0) {
            o.status = e.status;
            o.x = e.p.x; o.y = e.p.y; o.z = e.p.z;
            return false;
        }
        ray.p[0] = e.p.x; ray.p[1] = e.p.y; ray.p[2] = e.p.z;
        ray.n[0] = e.n.x; ray.n[1] = e.n.y; ray.n[2] = e.n.z;
    }
    return !obscured(P, ray, o);
}

// Surfaces k0..k1-1 before the detector (sections 2.4.1-2.4.2): returns true while the photon
// lives, else fills the outcome.  wc / wc_block cache the roulette block of the last coated
// surface (wc_block = -1: none).
// A ghost branch met in the surface loop, kept for later: the hit at the reflecting surface k
// (k = -1: none) and the refractive index of the medium the photon travelled in.  The optics
// kernel appends it to the chunk's ghost list; a second pass of the kernel runs the branches,
// started at different surfaces or by different photons, together.
struct GhostStart {
    Hit h;
    int k;
    double n_cur;
};

// The chunk's list of ghost starts in device memory: cap entries of kGhostFields 8-byte fields,
// field-major (field f of entry e at f * cap + e): the hit (q, d, N, dn), the index of the
// medium, the wavelength, (surface << 32 | Newton steps so far) and the photon's position in the
// survivor list.  ghost_get reads one entry.
__device__ __forceinline__ void ghost_get(const double* q, uint64_t cap, uint64_t e, GhostStart& gs,
                                          double& lam, uint32_t& r, int& newton) {
    const double* f = q + e;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        gs.h.q[i] = f[(0 + i) * cap];
        gs.h.d[i] = f[(3 + i) * cap];
        gs.h.N[i] = f[(6 + i) * cap];
    }
    gs.h.dn = f[9 * cap];
    gs.h.l = 0.0;   // not used by the branch
    gs.n_cur = f[10 * cap];
    lam = f[11 * cap];
    const uint64_t kn = (uint64_t)__double_as_longlong(f[12 * cap]);
    gs.k = (int)(kn >> 32);
    newton = (int)(uint32_t)kn;
    r = (uint32_t)__double_as_longlong(f[13 * cap]);
}
// Where the sequential pass leaves a lane's ghost start: the hit's fields are written to the
// lane's column of the wavefront's LDS staging area at the reflecting surface (field i at
// f[i * 64]), so that no register carries them out of the surface loop, and k records the
// surface (-1: none).
constexpr int kGhostStage = 11;   // q, d, N, dn, index of the medium
struct GhostSink {
    double* f;
    int k;
};
__device__ __forceinline__ void ghost_stage(GhostSink* gs, const Hit& h, int k, double n_cur) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        gs->f[(0 + i) * 64] = h.q[i];
        gs->f[(3 + i) * 64] = h.d[i];
        gs->f[(6 + i) * 64] = h.N[i];
    }
    gs->f[9 * 64] = h.dn;
    gs->f[10 * 64] = n_cur;
    gs->k = k;
}
// Appends the lanes holding a ghost start (gs.k >= 0) to the list (ctr[0] counts the entries;
// an entry beyond cap, which the list's size rules out, is not written).  Every lane of the
// wavefront must call it.
__device__ __forceinline__ void ghost_append(double* q, uint64_t cap, unsigned long long* ctr,
                                             const GhostSink& gs, const Outcome& o, uint32_t r) {
    const bool pend = gs.k >= 0;
    const uint64_t pm = __ballot(pend);
    if (!pm) return;
    unsigned long long base = 0;
    if (__lane_id() == 0) base = atomicAdd(&ctr[0], (unsigned long long)__popcll(pm));
    base = __shfl(base, 0);
    const uint64_t e = base + __popcll(pm & ((1ull << __lane_id()) - 1ull));
    if (pend && e < cap) {
        double* f = q + e;
#pragma unroll
        for (int i = 0; i < kGhostStage; ++i) f[i * cap] = gs.f[i * 64];
        f[11 * cap] = o.lam;
        f[12 * cap] = __longlong_as_double((long long)(((uint64_t)(uint32_t)gs.k << 32) |
                                                       (uint32_t)o.newton));
        f[13 * cap] = __longlong_as_double((long long)r);
    }
}

template <bool ZERN, bool TAPE = false, bool GHOST = false>
__device__ __forceinline__ bool trace_surfaces(const DevParams& P, const Launch& L, const Rng& rng,
                                               const Optics& oc, Ray& ray, int k0, int k1,
                                               uint4& wc, int& wc_block, Outcome& o,
                                               double* tp = nullptr, uint64_t ts = 0,
                                               GhostSink* gs = nullptr) {
    Hit h;
#pragma unroll 1
    for (int k = k0; k < k1; ++k) {
        const DevSurface& s = P.surf[k];
        int st = hit_surface<ZERN, TAPE, GHOST>(P, L, rng, k, ray.p, ray.n, oc.lc, wc, wc_block,
                                                h, o.newton);
        if (GHOST && st == kGhostReflect) {   // GHOST callers pass gs
            ghost_stage(gs, h, k, ray.n_cur);
            return false;
        }
        if (st == 0) {
            if (TAPE) tape_put(tp, ts, k, h);
            if (s.kind == PHX_MIRROR) {
                // reflection across the normal (section 2.4.2)
                h.d[0] -= 2.0 * h.dn * h.N[0];
                h.d[1] -= 2.0 * h.dn * h.N[1];
                h.d[2] -= 2.0 * h.dn * h.N[2];
            } else {
                const double n2 = s.medium == PHX_GLASS ? oc.n_glass : 1.0;
                if (refract(h, ray.n_cur / n2)) ray.n_cur = n2; else st = PHX_TIR;
            }
        }
        if (st != 0) {
            o.status = st; o.surface = k; o.x = h.q[0]; o.y = h.q[1]; o.z = h.q[2];
            return false;
        }
        if (s.moved) {
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                ray.p[i] = s.R[3 * i] * h.q[0] + s.R[3 * i + 1] * h.q[1] + s.R[3 * i + 2] * h.q[2] +
                           s.t[i];
                ray.n[i] = s.R[3 * i] * h.d[0] + s.R[3 * i + 1] * h.d[1] + s.R[3 * i + 2] * h.d[2];
            }
        } else {
            ray.p[0] = h.q[0]; ray.p[1] = h.q[1]; ray.p[2] = h.q[2] + s.t[2];
            ray.n[0] = h.d[0]; ray.n[1] = h.d[1]; ray.n[2] = h.d[2];
        }
    }
    return true;
}

// Landing on the detector after its coating and the refraction into silicon: conversion,
// diffusion and the pixel (sections 2.4.2-2.4.3); fills the outcome.
__device__ __forceinline__ void land(const DevParams& P, const Launch& L, const Rng& rng,
                                     const Optics& oc, const Hit& h, Outcome& o) {
    o.surface = P.n_surf - 1;
    o.x = h.q[0]; o.y = h.q[1]; o.z = h.q[2];
    double xc = h.q[0], yc = h.q[1];
    const int ss = sensor_stage(P, L, rng, oc.lam, h.d, xc, yc);
    if (ss != 0) {
        o.status = ss;
        return;
    }
    o.xe = xc; o.ye = yc;
    // pixel quantisation (section 2.4.3)
    const double fx = (xc - P.chip_x0) / P.pixel, fy = (yc - P.chip_y0) / P.pixel;
    const double ix = floor(fx), iy = floor(fy);
    o.status = PHX_OFF_CHIP;
    if (ix >= 0.0 && ix < (double)P.nx && iy >= 0.0 && iy < (double)P.ny) {
        o.status = PHX_DETECTED;
        o.pix_i = (int)ix;
        o.pix_j = (int)iy;
    }
}

// Medium codes on either side of surface k in travel order and their indices.
__device__ __forceinline__ int medium_before(const DevParams& P, int k) {
    return k > 0 ? P.surf[k - 1].medium : PHX_VACUUM;
}
__device__ __forceinline__ double medium_index(const Optics& oc, int m) {
    return m == PHX_GLASS ? oc.n_glass : (m == PHX_SILICON ? n_silicon(oc.lam) : 1.0);
}

// A ghost (section 2.4.2): the photon was reflected by the coating of refracting surface k (hit
// h, element frame) and propagates backwards; from here on its next surface is the nearest one
// ahead along the ray among all surfaces but the current one (intersection distance above
// 1e-9 m), where it is transmitted into the medium on the other side, reflected (a mirror, or a
// coating's reflection), absorbed or vignetted, for at most kGhostMax interactions (interaction
// i draws its roulette word from stream 4, block i).  Reaching the detector it lands as usual.
// ghost_begin sets up the branch, ghost_step performs one interaction.
constexpr int kGhostMax = 16;
struct GhostRay {
    double p[3], n[3];   // global frame
    double n_cur;        // index of the medium the photon travels in
    int medium, from, inter;
};

__device__ __forceinline__ void ghost_begin(const DevParams& P, Hit h, int k, double n_cur,
                                            GhostRay& gr) {
    gr.medium = medium_before(P, k);
    gr.n_cur = n_cur;
    gr.from = k;
    gr.inter = 0;
    // reflect at k and return to the global frame
    h.d[0] -= 2.0 * h.dn * h.N[0];
    h.d[1] -= 2.0 * h.dn * h.N[1];
    h.d[2] -= 2.0 * h.dn * h.N[2];
    const DevSurface& s = P.surf[k];
    if (s.moved) {
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            gr.p[i] = s.R[3 * i] * h.q[0] + s.R[3 * i + 1] * h.q[1] + s.R[3 * i + 2] * h.q[2] +
                      s.t[i];
            gr.n[i] = s.R[3 * i] * h.d[0] + s.R[3 * i + 1] * h.d[1] + s.R[3 * i + 2] * h.d[2];
        }
    } else {
        gr.p[0] = h.q[0]; gr.p[1] = h.q[1]; gr.p[2] = h.q[2] + s.t[2];
        gr.n[0] = h.d[0]; gr.n[1] = h.d[1]; gr.n[2] = h.d[2];
    }
}

// One interaction of a ghost branch; true when the photon's fate is settled (o filled).
template <bool ZERN>
__device__ __forceinline__ bool ghost_step(const DevParams& P, const Launch& L, const Rng& rng,
                                        const Optics& oc, GhostRay& gr, Outcome& o) {
    // the nearest surface ahead; the search keeps the best candidate's frame coordinates, path
    // length, slope and Newton steps, so that its hit is finished without intersecting again
    double best = INFINITY;
    int bk = -1;
    Hit h;
    double bgx = 0.0, bgy = 0.0;
    int bit = 0;
    if (gr.inter < kGhostMax) {
#pragma unroll 1
        for (int j = 0; j < P.n_surf; ++j) {
            if (j == gr.from) continue;
            const DevSurface& s = P.surf[j];
            double q[3], d[3];
            if (s.moved) {
                const double r0 = gr.p[0] - s.t[0], r1 = gr.p[1] - s.t[1], r2 = gr.p[2] - s.t[2];
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    q[i] = s.R[i] * r0 + s.R[3 + i] * r1 + s.R[6 + i] * r2;
                    d[i] = s.R[i] * gr.n[0] + s.R[3 + i] * gr.n[1] + s.R[6 + i] * gr.n[2];
                }
            } else {
                q[0] = gr.p[0]; q[1] = gr.p[1]; q[2] = gr.p[2] - s.t[2];
                d[0] = gr.n[0]; d[1] = gr.n[1]; d[2] = gr.n[2];
            }
            double l, gx, gy;
            int it = 0;
            if (intersect<ZERN>(P, s, q, d, l, gx, gy, it) == 0 && l > 1e-9 && l < best) {
                best = l;
                bk = j;
                h.q[0] = q[0]; h.q[1] = q[1]; h.q[2] = q[2];
                h.d[0] = d[0]; h.d[1] = d[1]; h.d[2] = d[2];
                bgx = gx;
                bgy = gy;
                bit = it;
            }
        }
    }
    if (bk < 0) {   // leaves the optics, or the interaction limit is reached
        o.status = PHX_MISSED;
        o.surface = gr.from;
        o.x = gr.p[0]; o.y = gr.p[1]; o.z = gr.p[2];
        return true;
    }
    const DevSurface& s = P.surf[bk];
    // the interaction: the hit point, aperture and normal (as the sequential passage takes
    // them), then the roulette with this interaction's own word
    o.newton += bit;
    h.q[0] += h.d[0] * best; h.q[1] += h.d[1] * best; h.q[2] += h.d[2] * best;
    {
        const double rq2 = h.q[0] * h.q[0] + h.q[1] * h.q[1];
        if (rq2 < s.r_in2 || rq2 > s.r_out2) {
            o.status = PHX_VIGNETTED; o.surface = bk; o.x = h.q[0]; o.y = h.q[1]; o.z = h.q[2];
            return true;
        }
        if (s.c == 0.0 && s.asphere == 0 && !(ZERN && s.zernike)) {
            h.N[0] = 0.0; h.N[1] = 0.0; h.N[2] = 1.0;   // a plane
        } else {
            const double inv = rsq_fast(bgx * bgx + bgy * bgy + 1.0);
            h.N[0] = -bgx * inv; h.N[1] = -bgy * inv; h.N[2] = inv;
        }
        h.dn = h.d[0] * h.N[0] + h.d[1] * h.N[1] + h.d[2] * h.N[2];
        if (h.dn > 0.0) { h.N[0] = -h.N[0]; h.N[1] = -h.N[1]; h.N[2] = -h.N[2]; h.dn = -h.dn; }
    }
    bool reflect = s.kind == PHX_MIRROR;
    if ((L.flags & PHX_F_COATINGS) && s.coating >= 0) {
        const double u = u01(rng.block((uint32_t)gr.inter, 4).x);
        const double sv = 1.0 - h.dn * h.dn;
        const double T = coating(P, s.coating, sv, oc.lc);
        if (!(u < T)) {
            const double R = s.kind != PHX_MIRROR ? coating(P, s.coating, sv, oc.lc, P.coat_r) : 0.0;
            if (!(u < T + R)) {
                o.status = PHX_ABSORBED; o.surface = bk;
                o.x = h.q[0]; o.y = h.q[1]; o.z = h.q[2];
                return true;
            }
            reflect = true;
        }
    }
    const bool det = s.kind == PHX_DETECTOR;
    if (reflect) {
        h.d[0] -= 2.0 * h.dn * h.N[0];
        h.d[1] -= 2.0 * h.dn * h.N[1];
        h.d[2] -= 2.0 * h.dn * h.N[2];
    } else if (!det || (L.flags & PHX_F_SILICON)) {
        const int after = s.medium, before = medium_before(P, bk);
        const int m2 = gr.medium == after ? before : after;
        const double n2 = medium_index(oc, m2);
        if (!refract(h, gr.n_cur / n2)) {
            o.status = PHX_TIR; o.surface = bk; o.x = h.q[0]; o.y = h.q[1]; o.z = h.q[2];
            return true;
        }
        gr.n_cur = n2;
        gr.medium = m2;
    }
    if (det && !reflect) {
        land(P, L, rng, oc, h, o);
        return true;
    }
    if (s.moved) {
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            gr.p[i] = s.R[3 * i] * h.q[0] + s.R[3 * i + 1] * h.q[1] + s.R[3 * i + 2] * h.q[2] +
                      s.t[i];
            gr.n[i] = s.R[3 * i] * h.d[0] + s.R[3 * i + 1] * h.d[1] + s.R[3 * i + 2] * h.d[2];
        }
    } else {
        gr.p[0] = h.q[0]; gr.p[1] = h.q[1]; gr.p[2] = h.q[2] + s.t[2];
        gr.n[0] = h.d[0]; gr.n[1] = h.d[1]; gr.n[2] = h.d[2];
    }
    gr.from = bk;
    gr.inter += 1;
    return false;
}

// The detector surface: its coating, the refraction into silicon, then the landing (sections
// 2.4.2-2.4.3); fills the outcome.  GHOST: a reflection by the detector's coating starts a ghost.
template <bool ZERN, bool TAPE = false, bool GHOST = false>
__device__ __forceinline__ void finish_detector(const DevParams& P, const Launch& L,
                                                const Rng& rng, const Optics& oc, Ray& ray,
                                                uint4& wc, int& wc_block, Outcome& o,
                                                double* tp = nullptr, uint64_t ts = 0,
                                                GhostSink* gs = nullptr) {
    const int kdet = P.n_surf - 1;
    Hit h;
    int st = hit_surface<ZERN, TAPE, GHOST>(P, L, rng, kdet, ray.p, ray.n, oc.lc, wc, wc_block, h,
                                            o.newton);
    if (GHOST && st == kGhostReflect) {   // GHOST callers pass gs
        ghost_stage(gs, h, kdet, ray.n_cur);
        return;
    }
    if (TAPE && st == 0) tape_put(tp, ts, kdet, h);
    if (st == 0 && (L.flags & PHX_F_SILICON) && !refract(h, ray.n_cur / n_silicon(oc.lam)))
        st = PHX_TIR;
    if (st != 0) {
        o.status = st;
        o.surface = kdet;
        o.x = h.q[0]; o.y = h.q[1]; o.z = h.q[2];
        return;
    }
    land(P, L, rng, oc, h, o);
}

// Central obscuration, the surfaces (sections 2.4.1-2.4.2), silicon (sections 2.4.2-2.4.3) and
// the pixel, from the start-plane state.  With TAPE, every surface passage is recorded for the
// adjoint sweep.
template <bool ZERN, bool TAPE = false>
__device__ Outcome photon_back(const DevParams& P, const Launch& L, int si, uint64_t idx,
                               const Front& f, double* tp = nullptr, uint64_t ts = 0) {
    Outcome o;
    outcome_init(o, f.lam);
    const Rng rng{L.seed, (uint32_t)si, (uint32_t)idx, (uint32_t)(idx >> 32)};
    Ray ray{{f.p[0], f.p[1], f.p[2]}, {f.n[0], f.n[1], f.n[2]}, 1.0};
    if (!entrance<true>(P, L, rng, ray, o)) return o;
    const Optics oc = optics_of(P, L, f.lam);
    uint4 wc = make_uint4(0, 0, 0, 0);
    int wc_block = -1;
    if (!trace_surfaces<ZERN, TAPE>(P, L, rng, oc, ray, 0, P.n_surf - 1, wc, wc_block, o, tp, ts))
        return o;
    finish_detector<ZERN, TAPE>(P, L, rng, oc, ray, wc, wc_block, o, tp, ts);
    return o;
}

// Wavefront-aggregated increment: lanes with the same pixel elect one leader that adds the
// group's count.  Every lane of the wavefront must call it.
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

// Flattened launch index g -> (source, photon index).
__device__ __forceinline__ void decode(const Launch& L, uint64_t g, int& si, uint64_t& idx) {
    int s;
    uint64_t local;
    if (L.n_src == 1) {
        s = 0;
        local = g;
    } else if (L.uniform_count) {
        s = (int)(g / L.uniform_count);
        local = g - (uint64_t)s * L.uniform_count;
    } else {
        // largest s with prefix[s] <= g, between the sources of the guide blocks around g
        const uint64_t b = g >> L.guide_shift;
        int lo = L.src_guide[b], hi = L.src_guide[b + 1];
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (L.prefix[mid] <= g) lo = mid; else hi = mid - 1;
        }
        s = lo;
        local = g - L.prefix[s];
    }
    si = L.src_begin + s;
    idx = L.photon_begin + local;
}

__device__ __forceinline__ void write_event(const Launch& L, uint64_t g, int si, uint64_t idx,
                                            const Outcome& o) {
    phx_event& e = L.events[g / L.event_stride];
    e.photon = idx; e.source = si; e.status = o.status; e.surface = o.surface;
    e.pix_i = o.pix_i; e.pix_j = o.pix_j; e.newton = o.newton;
    e.x = o.x; e.y = o.y; e.z = o.z; e.xe = o.xe; e.ye = o.ye; e.lambda = o.lam;
}

// Book-keeping of one traced photon: event record; returns the pixel to bin (-1 for none).
__device__ __forceinline__ int account(const DevParams& P, const Launch& L, uint64_t g, int si,
                                       uint64_t idx, const Outcome& o) {
    if ((L.flags & PHX_F_EVENTS) && (g % L.event_stride) == 0) write_event(L, g, si, idx, o);
    return o.status == PHX_DETECTED ? o.pix_j * P.nx + o.pix_i : -1;
}

__device__ __forceinline__ int stat_slot(const Outcome& o) {
    return o.status * PHX_STAT_COLS + min(o.surface + 1, PHX_STAT_COLS - 1);
}

// Wavefront-aggregated status count: lanes with the same (status, surface) slot add their count
// with one LDS atomic.  Every lane of the wavefront must call it.
__device__ __forceinline__ void count_stat(uint32_t* s_stats, int slot, bool active) {
    uint64_t pending = __ballot(active);
    const int lane = __lane_id();
    while (pending) {
        const int leader = __ffsll((unsigned long long)pending) - 1;
        const int key = __shfl(slot, leader);
        const uint64_t same = __ballot(active && slot == key);
        if (lane == leader) atomicAdd(&s_stats[key], (uint32_t)__popcll(same));
        pending &= ~same;
    }
}

// Exact per-source moments of converted photons.  Positions are quantised to 2^-44 m and the
// sums (count, X, Y, X^2, Y^2, XY) are accumulated as 128-bit integers, so the result is
// independent of the order in which photons arrive.  Lanes of the wavefront that hold the same
// source are summed with cross-lane shuffles first; the group's leader then adds the sums with
// one pair of 64-bit atomics per 128-bit word (the low word's carry goes into the high word).
// Every lane of the wavefront must call it.
__device__ __forceinline__ void wave_sum128(unsigned __int128& v) {
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) {
        const uint64_t lo = __shfl_xor((unsigned long long)(uint64_t)v, m);
        const uint64_t hi = __shfl_xor((unsigned long long)(uint64_t)(v >> 64), m);
        v += ((unsigned __int128)hi << 64) | lo;
    }
}

__device__ __forceinline__ void atomic_add128(unsigned long long* w, unsigned __int128 v) {
    const unsigned long long lo = (unsigned long long)v, hi = (unsigned long long)(v >> 64);
    const unsigned long long old = atomicAdd(w, lo);
    const unsigned long long carry = old + lo < old ? 1ull : 0ull;
    if (hi + carry) atomicAdd(w + 1, hi + carry);
}

// Moments of one source are first gathered in a per-workgroup LDS record (the first source the
// workgroup meets, s_src); other sources, and the record at the end of the workgroup, go to the
// global words.  Without it every wavefront of a one-source launch would add to the same twelve
// global words.
struct MomentCache {
    unsigned long long w[PHX_MOMENT_WORDS];
    int src;
};

__device__ __forceinline__ void moment_cache_init(MomentCache* mc) {
    if (threadIdx.x < PHX_MOMENT_WORDS) mc->w[threadIdx.x] = 0ull;
    if (threadIdx.x == 0) mc->src = -1;
}

// Called by one thread after the workgroup's last add_moments (and a barrier).
__device__ __forceinline__ void moment_cache_flush(const Launch& L, MomentCache* mc) {
    if (mc->src < 0) return;
    unsigned long long* w = L.moments + (size_t)mc->src * PHX_MOMENT_WORDS;
    atomicAdd(w, mc->w[0]);
    for (int i = 0; i < 5; ++i)
        atomic_add128(w + 2 + 2 * i, ((unsigned __int128)mc->w[3 + 2 * i] << 64) | mc->w[2 + 2 * i]);
}

__device__ void add_moments(const Launch& L, int si, double xe, double ye, bool active,
                            MomentCache* mc) {
    uint64_t pending = __ballot(active);
    const int lane = __lane_id();
    while (pending) {
        const int leader = __ffsll((unsigned long long)pending) - 1;
        const int key = __shfl(si, leader);
        const bool mine = active && si == key;
        const uint64_t same = __ballot(mine);
        pending &= ~same;
        const double q = 17592186044416.0;   // 2^PHX_MOMENT_Q_LOG2
        const long long X = mine ? __double2ll_rn(xe * q) : 0;
        const long long Y = mine ? __double2ll_rn(ye * q) : 0;
        unsigned __int128 v[5] = {(unsigned __int128)(__int128)X, (unsigned __int128)(__int128)Y,
                                  (unsigned __int128)((__int128)X * X),
                                  (unsigned __int128)((__int128)Y * Y),
                                  (unsigned __int128)((__int128)X * Y)};
#pragma unroll
        for (int i = 0; i < 5; ++i) wave_sum128(v[i]);
        if (lane == leader) {
            int cached = mc->src;
            if (cached < 0) {
                const int prev = atomicCAS(&mc->src, -1, key);
                cached = prev < 0 ? key : prev;
            }
            unsigned long long* w = cached == key ? mc->w
                                                  : L.moments + (size_t)key * PHX_MOMENT_WORDS;
            atomicAdd(w, (unsigned long long)__popcll(same));
#pragma unroll
            for (int i = 0; i < 5; ++i) atomic_add128(w + 2 + 2 * i, v[i]);
        }
    }
}

__device__ __forceinline__ void stats_init(uint32_t* s_stats) {
    for (int i = threadIdx.x; i < PHX_STATS_LEN; i += blockDim.x) s_stats[i] = 0;
    __syncthreads();
}

__device__ __forceinline__ void stats_flush(const Launch& L, uint32_t* s_stats, uint32_t newton,
                                            uint32_t traced) {
    atomicAdd(&s_stats[PHX_STAT_NEWTON], newton);
    atomicAdd(&s_stats[PHX_STAT_TRACED], traced);
    __syncthreads();
    if (L.stats) {
        for (int i = threadIdx.x; i < PHX_STATS_LEN; i += blockDim.x)
            if (s_stats[i]) atomicAdd(&L.stats[i], (unsigned long long)s_stats[i]);
    }
}

// Pre-roll (section 3.2, dynamic transmission optimisation).  Each workgroup takes contiguous
// ranges of kGenRange photons.  Stage one draws every photon's wavelength and pupil radius, drops
// photons whose pupil sample cannot reach the primary's aperture (the annulus is sampled wider
// than the aperture to leave room for atmospheric displacement, which the host bounds) and
// applies the most selective coating test; its survivors are queued in LDS (offset, time bucket,
// wavelength column) and stage two applies the remaining tests to them densely, so the many
// photons that fail the first test cost one test.  Stage two also flags the photons whose
// conversion word passes the escape filter, and stage three (only when any is flagged) runs the
// exact escape test on them out of the main loops' register budget.  The survivors' bits are set
// in an LDS copy of the range's bitmap words, written out once (the bitmap does not depend on the
// order of the queue), with each survivor's time bucket when requested.  An ordered compaction
// or the time-bucket sort then lists the survivors.
constexpr int kGenIters = 16;
constexpr int kGenRange = kBlock * kGenIters;   // photons per range (64 bitmap words)
static_assert(kGenRange <= 4096, "range offsets are queued in twelve bits");

__device__ __forceinline__ void culled_event(const Launch& L, uint64_t g, int si, uint64_t idx,
                                             double lam) {
    if ((L.flags & PHX_F_EVENTS) && (g % L.event_stride) == 0) {
        Outcome o;
        o.status = PHX_CULLED; o.surface = -1; o.newton = 0; o.pix_i = o.pix_j = -1;
        o.x = o.y = o.z = o.xe = o.ye = 0.0;
        o.lam = lam;
        write_event(L, g, si, idx, o);
    }
}

// ONE: every photon of the chunk belongs to source one_si, whose first photon has flattened
// index `first` (the source index and the Philox key are then uniform over the workgroup).
template <bool ONE, bool GHOST>
__global__ __launch_bounds__(kBlock) void generate_kernel(const DevParams* __restrict__ Pg,
                                                          const Launch L, uint64_t begin,
                                                          uint64_t len, int one_si,
                                                          uint64_t first,
                                                          unsigned long long* __restrict__ bits,
                                                          uint8_t* __restrict__ key) {
    __shared__ uint32_t s_stats[PHX_STATS_LEN];
    __shared__ unsigned long long s_bits[kGenRange / 64];
    // queued photon: offset | time bucket << 12 | wavelength column << 18 | escape test << 31
    __shared__ uint32_t s_q[kGenRange];
    __shared__ unsigned int s_qn, s_esc;
    stats_init(s_stats);
    const DevParams& P = *Pg;
    const int lane = __lane_id();
    // with ghosts a photon may leave the sequential path at a coated refracting surface, after
    // which the sequential roulette words no longer decide its fate: only the coated surfaces
    // ahead of the first coated refracting one (the mirrors) are tested then
    const int n_tests = P.n_cull;
    const int k_lim = GHOST ? P.ghost_cull_limit : PHX_MAX_SURF;
    // the chunk's one source, read once (the other case reads each photon's source record)
    DevSource one_src{};
    if constexpr (ONE) one_src = P.src[one_si];
    const uint64_t n_ranges = (len + kGenRange - 1) / kGenRange;
    for (uint64_t rg = blockIdx.x; rg < n_ranges; rg += gridDim.x) {   // workgroup-uniform
        const uint64_t r0 = rg * kGenRange;
        if (threadIdx.x < kGenRange / 64) s_bits[threadIdx.x] = 0ull;
        if (threadIdx.x == 0) {
            s_qn = 0;
            s_esc = 0;
        }
        __syncthreads();
        // stage one: wavelength and the first test for every photon of the range
        for (int it = 0; it < kGenIters; ++it) {
            const int rr = it * kBlock + threadIdx.x;
            const uint64_t r = r0 + rr;
            bool pass = false, culled = false;
            uint32_t entry = 0;
            if (r < len) {
                const uint64_t g = begin + r;
                int si;
                uint64_t idx;
                if constexpr (ONE) {
                    si = one_si;
                    idx = L.photon_begin + (g - first);
                } else {
                    decode(L, g, si, idx);
                }
                const Rng rng{L.seed, (uint32_t)si, (uint32_t)idx, (uint32_t)(idx >> 32)};
                uint32_t wt, wr;
                const double lam = preroll_draw(P, rng, ONE ? one_src : P.src[si], wt, wr);
                // squared pupil radius as the sky stage samples it: outside the reachable annulus
                // the photon is vignetted at the primary whatever the atmosphere does (the bounds
                // carry a margin far above the rounding of the square root)
                const double ro = P.pupil_r_out + L.pupil_margin;
                const double ri = fmax(P.pupil_r_in - L.pupil_margin, 0.0);
                const double rp2 = u01(wr) * (ro * ro - ri * ri) + ri * ri;
                const int il = lambda_column(P, lam).il;
                culled = rp2 < L.cull_r2_lo || rp2 > L.cull_r2_hi ||
                         (n_tests > 0 && preroll_first<GHOST>(P, rng, il, k_lim));
                pass = !culled;
                if (culled) culled_event(L, g, si, idx, lam);
                // time bucket of a survivor (the time stamp is t_e u01(wt))
                const int tb = min((int)(u01(wt) * kTimeBuckets), kTimeBuckets - 1);
                entry = (uint32_t)rr | ((uint32_t)tb << 12) | ((uint32_t)il << 18);
            }
            const uint64_t pm = __ballot(pass), cm = __ballot(culled);
            unsigned int base = 0;
            if (lane == 0) {
                if (pm) base = atomicAdd(&s_qn, (unsigned int)__popcll(pm));
                if (cm) atomicAdd(&s_stats[PHX_CULLED * PHX_STAT_COLS], (uint32_t)__popcll(cm));
            }
            base = __shfl(base, 0);
            if (pass) s_q[base + __popcll(pm & ((1ull << lane) - 1ull))] = entry;
        }
        __syncthreads();
        // stage two: the remaining tests for the queued photons
        const unsigned int qn = s_qn;
        for (unsigned int q0 = 0; q0 < qn; q0 += kBlock) {
            const unsigned int qi = q0 + threadIdx.x;
            bool keep = false, culled = false;
            if (qi < qn) {
                const uint32_t entry = s_q[qi];
                const int rr = (int)(entry & 0xfffu);
                const uint64_t r = r0 + rr;
                const uint64_t g = begin + r;
                int si;
                uint64_t idx;
                if constexpr (ONE) {
                    si = one_si;
                    idx = L.photon_begin + (g - first);
                } else {
                    decode(L, g, si, idx);
                }
                const Rng rng{L.seed, (uint32_t)si, (uint32_t)idx, (uint32_t)(idx >> 32)};
                const int il = (int)((entry >> 18) & 0x1fffu);
                culled = preroll_rest<GHOST>(P, rng, il, n_tests, k_lim);
                const uint32_t et = P.esc_thr && il >= P.esc_col0 ? P.esc_thr[il] : 0u;
                bool later = false;
                if (!culled && et && (L.flags & PHX_F_SILICON)) {
                    // escape: a quick filter on the conversion word here; the exact test in
                    // stage three, out of this loop's register budget
                    later = rng.block(1).z < et;
                    if (later) {
                        s_q[qi] = entry | (1u << 31);
                        s_esc = 1u;
                    }
                }
                keep = !culled && !later;
                if (keep) {
                    atomicOr(&s_bits[rr >> 6], 1ull << (rr & 63));
                    if (key) key[r] = (uint8_t)((entry >> 12) & 0x3fu);
                } else if ((L.flags & PHX_F_EVENTS) && (g % L.event_stride) == 0) {
                    uint32_t wt, wr;
                    culled_event(L, g, si, idx, preroll_draw(P, rng, ONE ? one_src : P.src[si], wt, wr));
                }
            }
            const uint64_t cm = __ballot(culled);
            if (lane == 0 && cm)
                atomicAdd(&s_stats[PHX_CULLED * PHX_STAT_COLS], (uint32_t)__popcll(cm));
        }
        // stage three: the exact escape test for the photons stage two flagged
        __syncthreads();
        if (s_esc) {
            for (unsigned int q0 = 0; q0 < qn; q0 += kBlock) {
                const unsigned int qi = q0 + threadIdx.x;
                const uint32_t entry = qi < qn ? s_q[qi] : 0u;
                bool culled = false;
                if (entry >> 31) {
                    const int rr = (int)(entry & 0xfffu);
                    const uint64_t r = r0 + rr;
                    const uint64_t g = begin + r;
                    int si;
                    uint64_t idx;
                    if constexpr (ONE) {
                        si = one_si;
                        idx = L.photon_begin + (g - first);
                    } else {
                        decode(L, g, si, idx);
                    }
                    const Rng rng{L.seed, (uint32_t)si, (uint32_t)idx, (uint32_t)(idx >> 32)};
                    uint32_t wt, wr;
                    const double lam = preroll_draw(P, rng, ONE ? one_src : P.src[si], wt, wr);
                    culled = escape_certain(P, lam, rng.block(1).z);
                    if (!culled) {
                        atomicOr(&s_bits[rr >> 6], 1ull << (rr & 63));
                        if (key) key[r] = (uint8_t)((entry >> 12) & 0x3fu);
                    } else {
                        culled_event(L, g, si, idx, lam);
                    }
                }
                const uint64_t cm = __ballot(culled);
                if (lane == 0 && cm)
                    atomicAdd(&s_stats[PHX_CULLED * PHX_STAT_COLS], (uint32_t)__popcll(cm));
            }
        }
        __syncthreads();
        if (threadIdx.x < kGenRange / 64 && r0 + (uint64_t)threadIdx.x * 64 < len)
            bits[(r0 >> 6) + threadIdx.x] = s_bits[threadIdx.x];
        __syncthreads();
    }
    stats_flush(L, s_stats, 0u, 0u);
}

// Ordered compaction of the survivor bitmap: kCompactWords words per workgroup.
constexpr int kWordsPerThread = 16;
constexpr uint64_t kCompactWords = (uint64_t)kBlock * kWordsPerThread;

__device__ __forceinline__ unsigned int block_sum_u32(unsigned int v, unsigned int* s_tmp) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
    if (__lane_id() == 0) s_tmp[threadIdx.x / 64] = v;
    __syncthreads();
    unsigned int t = 0;
    for (int w = 0; w < kBlock / 64; ++w) t += s_tmp[w];
    __syncthreads();
    return t;
}

// Survivors per workgroup range of the bitmap.
__global__ __launch_bounds__(kBlock) void compact_count(const unsigned long long* __restrict__ bits,
                                                        uint64_t n_words,
                                                        unsigned int* __restrict__ bsum) {
    __shared__ unsigned int s_tmp[kBlock / 64];
    const uint64_t w0 = (uint64_t)blockIdx.x * kCompactWords;
    unsigned int c = 0;
    for (int i = 0; i < kWordsPerThread; ++i) {
        const uint64_t w = w0 + (uint64_t)i * kBlock + threadIdx.x;
        if (w < n_words) c += __popcll(bits[w]);
    }
    const unsigned int t = block_sum_u32(c, s_tmp);
    if (threadIdx.x == 0) bsum[blockIdx.x] = t;
}

// Survivor offsets in photon order; the last workgroup stores the total in *count.
__global__ __launch_bounds__(kBlock) void compact_scatter(const unsigned long long* __restrict__ bits,
                                                          uint64_t n_words,
                                                          const unsigned int* __restrict__ bsum,
                                                          uint32_t* __restrict__ surv,
                                                          unsigned int* __restrict__ count) {
    __shared__ unsigned int s_tmp[kBlock / 64];
    __shared__ unsigned int s_scan[kBlock];
    // survivors before this workgroup's range
    unsigned int pre = 0;
    for (unsigned int b = threadIdx.x; b < blockIdx.x; b += blockDim.x) pre += bsum[b];
    const unsigned int base = block_sum_u32(pre, s_tmp);
    // this thread's words: a contiguous run, so that offsets follow photon order
    const uint64_t w0 = (uint64_t)blockIdx.x * kCompactWords + (uint64_t)threadIdx.x * kWordsPerThread;
    unsigned long long wv[kWordsPerThread];
    unsigned int c = 0;
#pragma unroll
    for (int i = 0; i < kWordsPerThread; ++i) {
        wv[i] = w0 + i < n_words ? bits[w0 + i] : 0ull;
        c += __popcll(wv[i]);
    }
    // inclusive scan of the per-thread counts (Hillis-Steele over the workgroup)
    s_scan[threadIdx.x] = c;
    __syncthreads();
    for (int d = 1; d < kBlock; d <<= 1) {
        const unsigned int v = threadIdx.x >= (unsigned)d ? s_scan[threadIdx.x - d] : 0u;
        __syncthreads();
        s_scan[threadIdx.x] += v;
        __syncthreads();
    }
    unsigned int o = base + s_scan[threadIdx.x] - c;
#pragma unroll
    for (int i = 0; i < kWordsPerThread; ++i) {
        unsigned long long m = wv[i];
        while (m) {
            const int bit = __ffsll(m) - 1;
            surv[o++] = (uint32_t)((w0 + i) * 64 + bit);
            m &= m - 1;
        }
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == kBlock - 1) *count = base + s_scan[kBlock - 1];
}

// Time-bucketed compaction (with the atmosphere): a stable counting sort of the survivors by
// time bucket, so that photons traced together see the same wind-shifted stretch of every phase
// screen and share its cache lines.  Within a bucket survivors keep photon order; the result is
// the same on every run.  Each workgroup takes kBucketWords bitmap words; a word's 64 bucket
// bytes are read with four 16-byte loads before its set bits are visited (in photon order).
constexpr uint64_t kBucketWords = (uint64_t)kBlock * kBucketWordsPerThread;

template <class F>
__device__ __forceinline__ void for_each_survivor(unsigned long long m, const uint8_t* key_word,
                                                  F f) {
    if (!m) return;
    const uint4* kp = reinterpret_cast<const uint4*>(key_word);
    const uint4 k0 = kp[0], k1 = kp[1], k2 = kp[2], k3 = kp[3];
    const uint32_t kw[16] = {k0.x, k0.y, k0.z, k0.w, k1.x, k1.y, k1.z, k1.w,
                             k2.x, k2.y, k2.z, k2.w, k3.x, k3.y, k3.z, k3.w};
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        uint32_t mj = (uint32_t)(m >> (4 * j)) & 0xfu;
        while (mj) {
            const int b = __ffs(mj) - 1;
            f(4 * j + b, (int)((kw[j] >> (8 * b)) & 0xffu));
            mj &= mj - 1;
        }
    }
}

__global__ __launch_bounds__(kBlock) void bucket_count(const unsigned long long* __restrict__ bits,
                                                       const uint8_t* __restrict__ key,
                                                       uint64_t n_words,
                                                       unsigned int* __restrict__ hist) {
    __shared__ unsigned int s_h[kTimeBuckets];
    if (threadIdx.x < kTimeBuckets) s_h[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t w0 = (uint64_t)blockIdx.x * kBucketWords;
    for (int i = 0; i < kBucketWordsPerThread; ++i) {
        const uint64_t w = w0 + (uint64_t)i * kBlock + threadIdx.x;
        if (w >= n_words) continue;
        for_each_survivor(bits[w], key + w * 64, [&](int, int b) { atomicAdd(&s_h[b], 1u); });
    }
    __syncthreads();
    if (threadIdx.x < kTimeBuckets) hist[(uint64_t)blockIdx.x * kTimeBuckets + threadIdx.x] = s_h[threadIdx.x];
}

// Per bucket, the exclusive prefix of its survivors over the sort's workgroups (pre[g][b]) and
// its total (tot[b]): one workgroup per bucket.
__global__ __launch_bounds__(kBlock) void bucket_scan(const unsigned int* __restrict__ hist,
                                                      unsigned int n_groups,
                                                      unsigned int* __restrict__ pre,
                                                      unsigned int* __restrict__ tot) {
    __shared__ unsigned int s_scan[kBlock];
    const int b = blockIdx.x, t = threadIdx.x;
    unsigned int carry = 0;
    for (unsigned int g0 = 0; g0 < n_groups; g0 += kBlock) {
        const unsigned int g = g0 + t;
        const unsigned int v = g < n_groups ? hist[(uint64_t)g * kTimeBuckets + b] : 0u;
        s_scan[t] = v;
        __syncthreads();
        for (int d = 1; d < kBlock; d <<= 1) {
            const unsigned int x = t >= d ? s_scan[t - d] : 0u;
            __syncthreads();
            s_scan[t] += x;
            __syncthreads();
        }
        if (g < n_groups) pre[(uint64_t)g * kTimeBuckets + b] = carry + s_scan[t] - v;
        carry += s_scan[kBlock - 1];
        __syncthreads();
    }
    if (t == 0) tot[b] = carry;
}

// Each workgroup's survivors of bucket b start after the survivors of all earlier buckets and
// those of bucket b in earlier workgroups; the last workgroup stores the total in *count.
__global__ __launch_bounds__(kBlock) void bucket_scatter(const unsigned long long* __restrict__ bits,
                                                         const uint8_t* __restrict__ key,
                                                         uint64_t n_words,
                                                         const unsigned int* __restrict__ pre,
                                                         const unsigned int* __restrict__ tot,
                                                         uint32_t* __restrict__ surv,
                                                         unsigned int* __restrict__ count) {
    // per bucket, per thread: count, then slot (a thread holds at most 4 x 64 survivors)
    __shared__ uint16_t s_c[kTimeBuckets][kBlock];
    __shared__ unsigned int s_off[kTimeBuckets];
    static_assert(kBucketWordsPerThread * 64 < 65536, "per-thread counts fit 16 bits");
    const int t = threadIdx.x;
    if (t < kTimeBuckets) {
        unsigned int base = 0, all = 0;
        for (int c = 0; c < kTimeBuckets; ++c) {
            const unsigned int tc = tot[c];
            if (c < t) base += tc;
            all += tc;
        }
        s_off[t] = base + pre[(uint64_t)blockIdx.x * kTimeBuckets + t];
        if (blockIdx.x == gridDim.x - 1 && t == 0) *count = all;
    }
    __syncthreads();
    for (int b = 0; b < kTimeBuckets; ++b) s_c[b][t] = 0;
    const uint64_t w0 = (uint64_t)blockIdx.x * kBucketWords + (uint64_t)t * kBucketWordsPerThread;
    for (int i = 0; i < kBucketWordsPerThread; ++i) {
        if (w0 + i >= n_words) break;
        for_each_survivor(bits[w0 + i], key + (w0 + i) * 64,
                          [&](int, int b) { s_c[b][t] += 1; });
    }
    __syncthreads();
    if (t < kTimeBuckets) {   // exclusive scan of bucket t over the threads, in thread order
        unsigned int run = 0;
        for (int u = 0; u < kBlock; ++u) {
            const unsigned int v = s_c[t][u];
            s_c[t][u] = (uint16_t)run;   // a thread's slot within its workgroup's bucket run
            run += v;
        }
    }
    __syncthreads();
    // slots within the workgroup's run of a bucket: below 4 x 64 x 256 = 65536
    const unsigned int* o = s_off;
    for (int i = 0; i < kBucketWordsPerThread; ++i) {
        if (w0 + i >= n_words) break;
        const uint64_t base = (w0 + i) * 64;
        for_each_survivor(bits[w0 + i], key + base, [&](int bit, int b) {
            surv[o[b] + s_c[b][t]] = (uint32_t)(base + bit);
            s_c[b][t] += 1;
        });
    }
}

// Block-uniform work distribution over [0, n): static (tile = block, block + grid, ...) or
// dynamic (tiles of kTileIters x blockDim elements claimed from a device counter).
struct Tiles {
    unsigned long long* ctr;   // null: static
    uint64_t tile, sub, n;
    __device__ bool next(unsigned long long* s_tile) {
        if (!ctr) {
            if (sub) tile += gridDim.x;
            sub = 1;
            return tile * blockDim.x < n;
        }
        if (sub == 0 || sub == kTileIters) {
            __syncthreads();
            if (threadIdx.x == 0) *s_tile = atomicAdd(ctr, 1ull);
            __syncthreads();
            tile = *s_tile * kTileIters;
            sub = 0;
        } else {
            tile += 1;
        }
        sub += 1;
        return tile * blockDim.x < n;
    }
    __device__ uint64_t index() const { return tile * blockDim.x + threadIdx.x; }
};

// Front half of the trace for the chunk's photons (the survivor list, or every photon when
// surv is null): sky sampling and the atmosphere, leaving the start-plane state in SoA arrays
// st[0..6][i] = p_x, p_y, p_z, n_x, n_y, n_z, lambda.
template <bool SERSIC, bool EXTRA>
__global__ __launch_bounds__(kBlock) void front_kernel(const DevParams* __restrict__ Pg,
                                                       const Launch L, uint64_t begin,
                                                       const uint32_t* __restrict__ surv,
                                                       const unsigned int* __restrict__ count,
                                                       uint64_t n_all, double* __restrict__ st,
                                                       uint64_t st_stride,
                                                       unsigned long long* tile_ctr) {
    __shared__ unsigned long long s_tile;
    const DevParams& P = *Pg;
    const uint64_t n = surv ? (uint64_t)*count : n_all;
    Tiles T{tile_ctr, blockIdx.x, 0, n};
    while (T.next(&s_tile)) {
        const uint64_t r = T.index();
        if (r >= n) continue;
        const uint64_t g = begin + (surv ? (uint64_t)surv[r] : r);
        int si;
        uint64_t idx;
        decode(L, g, si, idx);
        Front f;
        photon_front<SERSIC, EXTRA>(P, L, si, idx, f);
        st[0 * st_stride + r] = f.p[0];
        st[1 * st_stride + r] = f.p[1];
        st[2 * st_stride + r] = f.p[2];
        st[3 * st_stride + r] = f.n[0];
        st[4 * st_stride + r] = f.n[1];
        st[5 * st_stride + r] = f.n[2];
        st[6 * st_stride + r] = f.lam;
    }
}

// Book-keeping of finished photons, one per lane where act (every lane of the wavefront calls
// it): the event record, the pixel (through the workgroup's LDS window of win x win pixels placed
// at the first detection, else a wavefront-aggregated global atomic), the status count and the
// moment words.
__device__ __forceinline__ void book(const DevParams& P, const Launch& L, bool act, uint64_t g,
                                     int si, uint64_t idx, const Outcome& o, uint32_t* s_stats,
                                     uint32_t* s_win, int win, int* s_org, MomentCache* s_mc) {
    int pix = -1, slot = 0;
    bool m_on = false;
    if (act) {
        m_on = (L.flags & PHX_F_MOMENTS) && o.status <= PHX_OFF_CHIP;
        slot = stat_slot(o);
        if (account(P, L, g, si, idx, o) >= 0) {
            int org = *s_org;
            if (org < 0) {
                const int want = (max(o.pix_i - win / 2, 0) << 16) | max(o.pix_j - win / 2, 0);
                const int prev = atomicCAS(s_org, -1, want);
                org = prev < 0 ? want : prev;
            }
            const int wi = o.pix_i - (org >> 16), wj = o.pix_j - (org & 0xffff);
            if (wi >= 0 && wi < win && wj >= 0 && wj < win)
                atomicAdd(&s_win[wj * win + wi], 1u);
            else
                pix = o.pix_j * P.nx + o.pix_i;
        }
    }
    bin_photon(L.image, pix, pix >= 0);
    count_stat(s_stats, slot, act);
    if (L.flags & PHX_F_MOMENTS) add_moments(L, si, o.xe, o.ye, m_on, s_mc);
}

// Back half, the optics stage with refill (sections 2.4.1-2.4.3), from the start-plane state:
// each wavefront takes 64 photons at a time
// through the central obscuration and the first surface, queues the survivors in LDS, and runs
// the rest of the optics, the silicon and the pixel on 64 queued photons at a time, so lanes
// whose photon was vignetted or absorbed at the first surface are refilled instead of idling
// through the remaining surfaces.  Work units of 64 photons: static (unit w of the grid's
// wavefronts, then every grid-size-th unit) or from a device counter.
constexpr int kWin = 32;                  // LDS pixel window of the optics kernel
constexpr int kQueue = 128;               // queued photons per wavefront (64 + 63 carried)
constexpr int kWaves = kBlock / 64;
// EXTRA: aerosol and the spider at the entrance.  GH, the ghost branch of the roulette (with
// ghosts the kernel runs twice per chunk): 0 none; 1 the sequential pass, which appends the
// photons a coating reflects to the chunk's ghost list (ghost_list, cap entries, ghost_ctr[0]
// their number) instead of booking them; 2 the branches of the listed photons, claimed 64 at a
// time through ghost_ctr[1], with every lane refilled from the claimed entries as its photon is
// settled.  Keeping the branches out of the sequential pass keeps its registers those of the
// kernel without ghosts.
// Register budget for three waves per SIMD (168 VGPRs): alone the kernel runs about 7 % slower
// than with four (128 VGPRs and more spills), but beside the sky stage the whole step is faster,
// the launch then placing fewer of its workgroups on a compute unit.
template <bool ZERN, bool EXTRA, int GH>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3, 8))) void back_kernel(
        const DevParams* __restrict__ Pg, const Launch L, uint64_t begin,
        const uint32_t* __restrict__ surv, const unsigned int* __restrict__ count, uint64_t n_all,
        const double* __restrict__ st, uint64_t st_stride, unsigned long long* unit_ctr,
        double* __restrict__ ghost_list, uint64_t ghost_cap, unsigned long long* ghost_ctr) {
    constexpr bool GHOST = GH == 1;
    __shared__ uint32_t s_stats[PHX_STATS_LEN];
    __shared__ uint32_t s_win[kWin * kWin];
    __shared__ int s_org;   // window origin: (i0 << 16) | j0, or -1 before the first detection
    __shared__ MomentCache s_mc;
    __shared__ double s_q[kWaves][7][kQueue];   // p, n (global frame) and wavelength
    __shared__ uint32_t s_qr[kWaves][kQueue];   // position in the survivor list
    __shared__ int32_t s_qk[kWaves][kQueue];    // Newton steps so far << 1 | travelling in glass
    // GH == 1: each wavefront's staging area of ghost starts (kGhostStage fields x 64 lanes)
    __shared__ double s_gs[GH == 1 ? kWaves * kGhostStage * 64 : 1];
    for (int i = threadIdx.x; i < kWin * kWin; i += blockDim.x) s_win[i] = 0;
    if (threadIdx.x == 0) s_org = -1;
    moment_cache_init(&s_mc);
    stats_init(s_stats);   // ends with a barrier
    const DevParams& P = *Pg;
    const uint64_t n = surv ? (uint64_t)*count : n_all;
    const int wave = threadIdx.x >> 6, lane = __lane_id();
    double (*q)[kQueue] = s_q[wave];
    uint32_t* qr = s_qr[wave];
    int32_t* qk = s_qk[wave];
    const uint64_t n_units = (n + 63) / 64;
    const uint64_t n_waves = (uint64_t)gridDim.x * kWaves;
    uint64_t unit = (uint64_t)blockIdx.x * kWaves + wave;
    if (unit_ctr) {
        unsigned long long u = 0;
        if (lane == 0) u = atomicAdd(unit_ctr, 1ull);
        unit = __shfl(u, 0);
    }
    const int kdet = P.n_surf - 1;
    const int k_first = kdet < 1 ? kdet : 1;   // surfaces of the first pass: [0, k_first)
    int qn = 0;                                // queued photons (wavefront-uniform)
    uint32_t newton = 0, traced = 0;
    if (GH == 2) {
        // the branches: the wavefront claims 64 listed starts at a time; a lane whose photon is
        // settled takes the next claimed start, so that the lanes stay busy until the list is
        // exhausted
        const uint64_t total = min((uint64_t)ghost_ctr[0], ghost_cap);
        uint64_t wbase = 0, wend = 0;   // the wavefront's claimed, not yet started entries
        bool claims = true;
        bool busy = false;
        GhostRay gr;
        Outcome o;
        outcome_init(o, 0.0);
        Optics oc{0.0, 1.0, LamCol{0, 0.0}};
        Rng rng{0u, 0u, 0u, 0u};
        uint64_t g = 0, idx = 0;
        int si = 0;
        for (;;) {
            const uint64_t idle = __ballot(!busy);
            if (claims && idle && wbase == wend) {
                unsigned long long b = 0;
                if (lane == 0) b = atomicAdd(&ghost_ctr[1], 64ull);
                b = __shfl(b, 0);
                wbase = b < total ? b : total;
                wend = b + 64 < total ? b + 64 : total;
                claims = wbase < wend;
            }
            const uint64_t avail = wend - wbase;
            const int take = (int)min((uint64_t)__popcll(idle), avail);
            const int rank = __popcll(idle & ((1ull << lane) - 1ull));
            if (!busy && rank < take) {
                GhostStart gs;
                double lam;
                uint32_t r;
                int nw;
                ghost_get(ghost_list, ghost_cap, wbase + rank, gs, lam, r, nw);
                g = begin + (surv ? (uint64_t)surv[r] : (uint64_t)r);
                decode(L, g, si, idx);
                rng = Rng{L.seed, (uint32_t)si, (uint32_t)idx, (uint32_t)(idx >> 32)};
                outcome_init(o, lam);
                o.newton = nw;
                oc = optics_of(P, L, lam);
                ghost_begin(P, gs.h, gs.k, gs.n_cur, gr);
                busy = true;
            }
            wbase += take;
            if (__ballot(busy) == 0) break;
            bool fin = false;
            if (busy) fin = ghost_step<ZERN>(P, L, rng, oc, gr, o);
            if (fin) {
                newton += o.newton;
                busy = false;
            }
            book(P, L, fin, g, si, idx, o, s_stats, s_win, kWin, &s_org, &s_mc);
        }
    }
    for (;;) {
        if (GH == 2) break;
        const bool more = unit < n_units;
        if (qn >= 64 || (!more && qn > 0)) {
            // second pass: up to 64 queued photons through the remaining surfaces
            const int take = qn < 64 ? qn : 64;
            const bool act = lane < take;
            Outcome o;
            outcome_init(o, 0.0);
            uint64_t g = 0, idx = 0;
            int si = 0;
            uint32_t r = 0;
            GhostSink gs{s_gs + (GH == 1 ? wave * kGhostStage * 64 + lane : 0), -1};
            if (act) {
                const int e = qn - take + lane;
                r = qr[e];
                const int32_t kq = qk[e];
                g = begin + (surv ? (uint64_t)surv[r] : (uint64_t)r);
                decode(L, g, si, idx);
                const Rng rng{L.seed, (uint32_t)si, (uint32_t)idx, (uint32_t)(idx >> 32)};
                const double lam = q[6][e];
                outcome_init(o, lam);
                o.newton = kq >> 1;
                const Optics oc = optics_of(P, L, lam);
                Ray ray{{q[0][e], q[1][e], q[2][e]}, {q[3][e], q[4][e], q[5][e]},
                        (kq & 1) ? oc.n_glass : 1.0};
                uint4 wc = make_uint4(0, 0, 0, 0);
                int wc_block = -1;
                GhostSink* gp = GHOST ? &gs : nullptr;
                if (trace_surfaces<ZERN, false, GHOST>(P, L, rng, oc, ray, k_first, kdet, wc,
                                                       wc_block, o, nullptr, 0, gp))
                    finish_detector<ZERN, false, GHOST>(P, L, rng, oc, ray, wc, wc_block, o,
                                                        nullptr, 0, gp);
            }
            const bool fin = act && !(GHOST && gs.k >= 0);
            if (GHOST) ghost_append(ghost_list, ghost_cap, ghost_ctr, gs, o, r);
            if (fin) newton += o.newton;
            book(P, L, fin, g, si, idx, o, s_stats, s_win, kWin, &s_org, &s_mc);
            qn -= take;
            __builtin_amdgcn_wave_barrier();
            continue;
        }
        if (!more) break;
        // first pass: the next 64 photons through the central obscuration and the first surface
        const uint64_t r = unit * 64 + lane;
        const bool valid = r < n;
        bool alive = false;
        Outcome o;
        outcome_init(o, 0.0);
        uint64_t g = 0, idx = 0;
        int si = 0;
        Ray ray{{0.0, 0.0, 0.0}, {0.0, 0.0, 1.0}, 1.0};
        GhostSink gs{s_gs + (GH == 1 ? wave * kGhostStage * 64 + lane : 0), -1};
        if (valid) {
            g = begin + (surv ? (uint64_t)surv[r] : r);
            decode(L, g, si, idx);
            const double lam = st[6 * st_stride + r];
            outcome_init(o, lam);
            ray.p[0] = st[0 * st_stride + r];
            ray.p[1] = st[1 * st_stride + r];
            ray.p[2] = st[2 * st_stride + r];
            ray.n[0] = st[3 * st_stride + r];
            ray.n[1] = st[4 * st_stride + r];
            ray.n[2] = st[5 * st_stride + r];
            const Rng rng{L.seed, (uint32_t)si, (uint32_t)idx, (uint32_t)(idx >> 32)};
            if (entrance<EXTRA>(P, L, rng, ray, o)) {
                const Optics oc = optics_of(P, L, lam);
                uint4 wc = make_uint4(0, 0, 0, 0);
                int wc_block = -1;
                alive = trace_surfaces<ZERN, false, GHOST>(P, L, rng, oc, ray, 0, k_first, wc,
                                                           wc_block, o, nullptr, 0,
                                                           GHOST ? &gs : nullptr);
            }
            traced += 1;
        }
        if (GHOST) ghost_append(ghost_list, ghost_cap, ghost_ctr, gs, o, (uint32_t)r);
        const uint64_t am = __ballot(alive);
        if (alive) {
            const int e = qn + __popcll(am & ((1ull << lane) - 1ull));
            q[0][e] = ray.p[0]; q[1][e] = ray.p[1]; q[2][e] = ray.p[2];
            q[3][e] = ray.n[0]; q[4][e] = ray.n[1]; q[5][e] = ray.n[2];
            q[6][e] = o.lam;
            qr[e] = (uint32_t)r;
            qk[e] = (o.newton << 1) | (ray.n_cur != 1.0 ? 1 : 0);
        }
        qn += __popcll(am);
        const bool done = valid && !alive && !(GHOST && gs.k >= 0);
        if (done) newton += o.newton;
        book(P, L, done, g, si, idx, o, s_stats, s_win, kWin, &s_org, &s_mc);
        if (unit_ctr) {
            unsigned long long u = 0;
            if (lane == 0) u = atomicAdd(unit_ctr, 1ull);
            unit = __shfl(u, 0);
        } else {
            unit += n_waves;
        }
        __builtin_amdgcn_wave_barrier();
    }
    stats_flush(L, s_stats, newton, traced);   // ends with a barrier
    if (threadIdx.x == 0 && (L.flags & PHX_F_MOMENTS)) moment_cache_flush(L, &s_mc);
    const int org = s_org;
    if (org >= 0) {
        const int i0 = org >> 16, j0 = org & 0xffff;
        for (int k = threadIdx.x; k < kWin * kWin; k += blockDim.x) {
            const uint32_t c = s_win[k];
            const int i = i0 + (k % kWin), j = j0 + (k / kWin);
            if (c && i < P.nx && j < P.ny) atomicAdd(&L.image[(size_t)j * P.nx + i], c);
        }
    }
}

// ---------------------------------------------------------------------------------------------
// Adjoint trace: pathwise derivative of per-source moments with respect to the rigid-body
// parameters of the two perturbation groups and the Zernike amplitudes of the primary, with
// every discrete decision (pupil, coatings, apertures, conversion, escape) held at its forward
// value.  Each converted photon is traced again with a tape of its surface passages, then swept
// from the electron position back to the primary: the intersection by the implicit-function
// rule (the path length solves q_z + l d_z = S(q_x + l d_x, q_y + l d_y)), the normal through
// the sag Hessian, reflection and Snell refraction through their Jacobians, and each group
// transform g = R q + t with t = pivot + R (vertex - pivot) + shift.

// Monomials u^a v^b of the Zernike expansion (order of zernike_poly).
__device__ constexpr int kMonoA[kNZernPoly] = {0, 1, 0, 2, 1, 0, 3, 2, 1, 0, 4, 3, 2, 1, 0};
__device__ constexpr int kMonoB[kNZernPoly] = {0, 0, 1, 0, 1, 2, 0, 1, 2, 3, 0, 1, 2, 3, 4};

__device__ __forceinline__ double ipow(const double* pw, int e) { return e > 0 ? pw[e] : 1.0; }

// Sag slopes and Hessian in the element frame at (x, y).
template <bool ZERN>
__device__ __forceinline__ void sag_hessian(const DevParams& P, const DevSurface& s, int k,
                                            double x, double y, double& Sx, double& Sy,
                                            double& Hxx, double& Hxy, double& Hyy) {
    const double r2 = x * x + y * y;
    const double arg = fmax(1.0 - s.kappa1 * s.c * s.c * r2, 0.0);
    const double root = sqrt(arg);
    const double iroot = root > 0.0 ? 1.0 / root : 0.0;
    double g = s.c * iroot;                                       // dS/dr / r
    double gp = 0.5 * s.c * s.kappa1 * s.c * s.c * iroot * iroot * iroot;   // dg / d(r^2)
    if (s.asphere == 1) {
        const double* a = s.alpha;
        g += r2 * (4.0 * a[1] + r2 * (6.0 * a[3] + r2 * (8.0 * a[5] + r2 * 10.0 * a[7])));
        gp += 4.0 * a[1] + r2 * (12.0 * a[3] + r2 * (24.0 * a[5] + r2 * 40.0 * a[7]));
    } else if (s.asphere == 2) {
        const double r = sqrt(r2);
        const double ir = r > 0.0 ? 1.0 / r : 0.0;
        double pw = r;   // r^(i-2)
        for (int i = 3; i <= 10; ++i) {
            const double a = s.alpha[i - 3];
            g += (double)i * a * pw;
            gp += 0.5 * (double)(i * (i - 2)) * a * pw * ir * ir;   // i (i-2) a r^(i-4) / 2
            pw *= r;
        }
    }
    Sx = x * g;
    Sy = y * g;
    Hxx = g + 2.0 * x * x * gp;
    Hxy = 2.0 * x * y * gp;
    Hyy = g + 2.0 * y * y * gp;
    if (ZERN && k == 0 && s.zernike) {
        const double ir = P.zern_inv_r;
        const double u = x * ir, v = y * ir;
        double pu[5], pv[5];
        pu[0] = pv[0] = 1.0;
        for (int e = 1; e < 5; ++e) { pu[e] = pu[e - 1] * u; pv[e] = pv[e - 1] * v; }
        double zu = 0, zv = 0, zuu = 0, zuv = 0, zvv = 0;
#pragma unroll
        for (int m = 0; m < kNZernPoly; ++m) {
            const int a = kMonoA[m], b = kMonoB[m];
            const double c = P.zern[m];
            if (a >= 1) zu += c * a * ipow(pu, a - 1) * pv[b];
            if (b >= 1) zv += c * b * pu[a] * ipow(pv, b - 1);
            if (a >= 2) zuu += c * a * (a - 1) * ipow(pu, a - 2) * pv[b];
            if (a >= 1 && b >= 1) zuv += c * a * b * ipow(pu, a - 1) * ipow(pv, b - 1);
            if (b >= 2) zvv += c * b * (b - 1) * pu[a] * ipow(pv, b - 2);
        }
        Sx += zu * ir;
        Sy += zv * ir;
        Hxx += zuu * ir * ir;
        Hxy += zuv * ir * ir;
        Hyy += zvv * ir * ir;
    }
}

__device__ __forceinline__ void group_rotation_derivs(const DevParams& P, int g, double dRx[9],
                                                      double dRy[9]) {
    const double cx = P.group_cs[g][0], sx = P.group_cs[g][1];
    const double cy = P.group_cs[g][2], sy = P.group_cs[g][3];
    // R = R_x(t_x) R_y(t_y) = [[cy, 0, sy], [sx sy, cx, -sx cy], [-cx sy, sx, cx cy]]
    dRx[0] = 0.0;      dRx[1] = 0.0; dRx[2] = 0.0;
    dRx[3] = cx * sy;  dRx[4] = -sx; dRx[5] = -cx * cy;
    dRx[6] = sx * sy;  dRx[7] = cx;  dRx[8] = -sx * cy;
    dRy[0] = -sy;      dRy[1] = 0.0; dRy[2] = cy;
    dRy[3] = sx * cy;  dRy[4] = 0.0; dRy[5] = sx * sy;
    dRy[6] = -cx * cy; dRy[7] = 0.0; dRy[8] = -cx * sy;
}

// The sweep for NC cotangent columns at once: seeds (xb, yb) of the electron position, results
// added to acc[c][0..kAdj).
template <bool ZERN, int NC>
__device__ void adjoint_sweep(const DevParams& P, const Launch& L, const Rng& rng, double lam,
                              const double* tp, uint64_t ts, const double* xb, const double* yb,
                              double (*acc)[kAdj]) {
    const int kdet = P.n_surf - 1;
    const double n_glass = P.has_glass ? sellmeier(P, lam) : 1.0;
    double pb[NC][3], nb[NC][3];   // global-frame cotangents of the ray leaving surface k
#pragma unroll 1
    for (int k = kdet; k >= 0; --k) {
        const DevSurface& s = P.surf[k];
        const double* t = tp + (uint64_t)k * kTapeFields * ts;
        const double q1[3] = {t[0], t[ts], t[2 * ts]};
        const double d0[3] = {t[3 * ts], t[4 * ts], t[5 * ts]};
        const double l = t[6 * ts];
        double Sx, Sy, Hxx, Hxy, Hyy;
        sag_hessian<ZERN>(P, s, k, q1[0], q1[1], Sx, Sy, Hxx, Hxy, Hyy);
        const double inv = 1.0 / sqrt(Sx * Sx + Sy * Sy + 1.0);
        const double Nr[3] = {-Sx * inv, -Sy * inv, inv};
        const double dnr = d0[0] * Nr[0] + d0[1] * Nr[1] + d0[2] * Nr[2];
        const double sg = dnr > 0.0 ? -1.0 : 1.0;
        const double N[3] = {sg * Nr[0], sg * Nr[1], sg * Nr[2]};
        const double dn = sg * dnr;
        const double n_in = s.glass_in ? n_glass : 1.0;
        // 0: no outgoing direction, 1: reflection, 2: refraction
        int mode;
        double mu = 1.0;
        if (k == kdet) {
            mode = (L.flags & PHX_F_SILICON) ? 2 : 0;
            mu = n_in / n_silicon(lam);
        } else if (s.kind == PHX_MIRROR) {
            mode = 1;
        } else {
            mode = 2;
            mu = n_in / (s.medium == PHX_GLASS ? n_glass : 1.0);
        }
        double d1[3] = {d0[0], d0[1], d0[2]};
        double f = 0.0, fpr = 0.0;
        if (mode == 1) {
#pragma unroll
            for (int i = 0; i < 3; ++i) d1[i] = d0[i] - 2.0 * dn * N[i];
        } else if (mode == 2) {
            const double cosi = -dn;
            const double kk = 1.0 - mu * mu * (1.0 - cosi * cosi);
            const double w = sqrt(fmax(kk, 0.0));
            f = mu * cosi - w;
            fpr = mu - (w > 0.0 ? mu * mu * cosi / w : 0.0);
#pragma unroll
            for (int i = 0; i < 3; ++i) d1[i] = mu * d0[i] + f * N[i];
        }
        double qb[NC][3], db[NC][3];
        double Rb[NC][9], tb[NC][3];
        const bool grp = s.group != 0;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
#pragma unroll
            for (int i = 0; i < 9; ++i) Rb[c][i] = 0.0;
            tb[c][0] = tb[c][1] = tb[c][2] = 0.0;
        }
        if (k == kdet) {
            // electron position from the landing point (sections 2.4.2-2.4.3)
            double Lc = 0.0, kz = 0.0, ca = 0.0, sa = 0.0;
            if (L.flags & PHX_F_SILICON) {
                Lc = -log(u01(rng.block(1).z)) / absorption(P, lam);
                if (L.flags & PHX_F_DIFFUSION) {
                    const uint4 wd = rng.block(6);
                    const double rad = sqrt(-2.0 * log(u01(wd.x)));
                    sincospi(2.0 * u01(wd.y), &sa, &ca);
                    ca *= rad;
                    sa *= rad;
                    // d sigma / d d1z through the depth Lc |d1z|
                    double slope = -P.sigma_max / P.t_si;
                    if (L.flags & PHX_F_FIELD_DIFFUSION) field_sigma(P, Lc * fabs(d1[2]), slope);
                    kz = slope * Lc * (d1[2] >= 0.0 ? 1.0 : -1.0);
                }
            }
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                qb[c][0] = xb[c]; qb[c][1] = yb[c]; qb[c][2] = 0.0;
                db[c][0] = Lc * xb[c]; db[c][1] = Lc * yb[c];
                db[c][2] = kz * (ca * xb[c] + sa * yb[c]);
            }
        } else {
            // leaving surface k: p' = R q1 + t, n' = R d1
#pragma unroll
            for (int c = 0; c < NC; ++c) {
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    qb[c][j] = s.R[j] * pb[c][0] + s.R[3 + j] * pb[c][1] + s.R[6 + j] * pb[c][2];
                    db[c][j] = s.R[j] * nb[c][0] + s.R[3 + j] * nb[c][1] + s.R[6 + j] * nb[c][2];
                }
                if (grp) {
#pragma unroll
                    for (int i = 0; i < 3; ++i) {
#pragma unroll
                        for (int j = 0; j < 3; ++j)
                            Rb[c][3 * i + j] += pb[c][i] * q1[j] + nb[c][i] * d1[j];
                        tb[c][i] += pb[c][i];
                    }
                }
            }
        }
        const double mv[3] = {-Sx, -Sy, 1.0};
        const double fpn = d0[2] - Sx * d0[0] - Sy * d0[1];
        double mono[kNZernPoly], mu_[kNZernPoly], mv_[kNZernPoly];
        if (k == 0) {
            const double ir = P.zern_inv_r;
            const double u = q1[0] * ir, v = q1[1] * ir;
            double pu[5], pv[5];
            pu[0] = pv[0] = 1.0;
            for (int e = 1; e < 5; ++e) { pu[e] = pu[e - 1] * u; pv[e] = pv[e - 1] * v; }
#pragma unroll
            for (int m = 0; m < kNZernPoly; ++m) {
                const int a = kMonoA[m], b = kMonoB[m];
                mono[m] = pu[a] * pv[b];
                mu_[m] = a >= 1 ? a * ipow(pu, a - 1) * pv[b] * ir : 0.0;
                mv_[m] = b >= 1 ? b * pu[a] * ipow(pv, b - 1) * ir : 0.0;
            }
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            // reflection / refraction: cotangents of the incoming direction and of the normal
            double d0b[3] = {0.0, 0.0, 0.0}, Nb[3] = {0.0, 0.0, 0.0};
            const double tN = N[0] * db[c][0] + N[1] * db[c][1] + N[2] * db[c][2];
            if (mode == 1) {
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    d0b[i] = db[c][i] - 2.0 * tN * N[i];
                    Nb[i] = -2.0 * (dn * db[c][i] + tN * d0[i]);
                }
            } else if (mode == 2) {
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    d0b[i] = mu * db[c][i] - tN * fpr * N[i];
                    Nb[i] = f * db[c][i] - tN * fpr * d0[i];
                }
            }
            // N = sg (-Sx, -Sy, 1) / sqrt(Sx^2 + Sy^2 + 1)
            const double nn = sg * (Nb[0] * Nr[0] + Nb[1] * Nr[1] + Nb[2] * Nr[2]);
            const double Sxb = -sg * Nb[0] * inv - nn * Sx * inv * inv;
            const double Syb = -sg * Nb[1] * inv - nn * Sy * inv * inv;
            double qc[3] = {qb[c][0] + Sxb * Hxx + Syb * Hxy, qb[c][1] + Sxb * Hxy + Syb * Hyy,
                            qb[c][2]};
            // intersection: q1 = q0 + l d0 with F(l) = q1_z - S(q1_x, q1_y) = 0
            const double lb = qc[0] * d0[0] + qc[1] * d0[1] + qc[2] * d0[2];
            const double coef = -lb / fpn;
            double q0b[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                q0b[i] = qc[i] + coef * mv[i];
                d0b[i] += l * qc[i] + coef * l * mv[i];
            }
            if (k == 0) {
#pragma unroll
                for (int m = 0; m < kNZernPoly; ++m)
                    acc[c][10 + m] += Sxb * mu_[m] + Syb * mv_[m] - coef * mono[m];
            }
            // entering surface k: q0 = R^T (p - t), d0 = R^T n
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                pb[c][i] = s.R[3 * i] * q0b[0] + s.R[3 * i + 1] * q0b[1] + s.R[3 * i + 2] * q0b[2];
                nb[c][i] = s.R[3 * i] * d0b[0] + s.R[3 * i + 1] * d0b[1] + s.R[3 * i + 2] * d0b[2];
            }
            if (grp) {
                const double q0[3] = {q1[0] - l * d0[0], q1[1] - l * d0[1], q1[2] - l * d0[2]};
                double pt[3], nw[3];   // p - t = R q0 and n = R d0 (global frame)
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    pt[i] = s.R[3 * i] * q0[0] + s.R[3 * i + 1] * q0[1] + s.R[3 * i + 2] * q0[2];
                    nw[i] = s.R[3 * i] * d0[0] + s.R[3 * i + 1] * d0[1] + s.R[3 * i + 2] * d0[2];
                }
#pragma unroll
                for (int i = 0; i < 3; ++i) {
#pragma unroll
                    for (int j = 0; j < 3; ++j) Rb[c][3 * i + j] += pt[i] * q0b[j] + nw[i] * d0b[j];
                    tb[c][i] -= pb[c][i];
                }
                // t = pivot + R (vertex - pivot) + shift
                const double* Pv = P.group_pivot[s.group];
                const double vp[3] = {-Pv[0], -Pv[1], s.z_vertex - Pv[2]};
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int j = 0; j < 3; ++j) Rb[c][3 * i + j] += tb[c][i] * vp[j];
                double dRx[9], dRy[9];
                group_rotation_derivs(P, s.group, dRx, dRy);
                double gx = 0.0, gy = 0.0;
#pragma unroll
                for (int i = 0; i < 9; ++i) {
                    gx += Rb[c][i] * dRx[i];
                    gy += Rb[c][i] * dRy[i];
                }
                const int b = 5 * (s.group - 1);
                acc[c][b + 0] += tb[c][0];
                acc[c][b + 1] += tb[c][1];
                acc[c][b + 2] += gx;
                acc[c][b + 3] += gy;
                acc[c][b + 4] += tb[c][2];
            }
        }
    }
}

// Wavefront then workgroup sum of the per-lane accumulators in a fixed order; thread 0..kAdj-1
// write the workgroup's row.
__device__ void block_sum_rows(double* acc, double* row) {
    __shared__ double s_part[kBlock / 64][kAdj];
    const int lane = __lane_id(), wave = threadIdx.x / 64;
#pragma unroll
    for (int j = 0; j < kAdj; ++j) {
        double v = acc[j];
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
        if (lane == 0) s_part[wave][j] = v;
    }
    __syncthreads();
    if (threadIdx.x < kAdj) {
        double v = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) v += s_part[w][threadIdx.x];
        row[threadIdx.x] = v;
    }
}

template <bool ZERN, bool JAC>
__global__ __launch_bounds__(kBlock) void adjoint_kernel(const DevParams* __restrict__ Pg,
                                                         const Launch L, uint64_t begin,
                                                         const uint32_t* __restrict__ surv,
                                                         const unsigned int* __restrict__ count,
                                                         uint64_t n_all,
                                                         const double* __restrict__ st,
                                                         uint64_t st_stride, const Adjoint A,
                                                         uint64_t row0) {
    const DevParams& P = *Pg;
    const uint64_t n = surv ? (uint64_t)*count : n_all;
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double* tp = A.tape + tid;
    const uint64_t ts = A.tape_stride;
    double acc[1][kAdj];
#pragma unroll
    for (int j = 0; j < kAdj; ++j) acc[0][j] = 0.0;
    for (uint64_t r = tid; r < n; r += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t g = begin + (surv ? (uint64_t)surv[r] : r);
        int si;
        uint64_t idx;
        decode(L, g, si, idx);
        Front f;
        f.p[0] = st[0 * st_stride + r];
        f.p[1] = st[1 * st_stride + r];
        f.p[2] = st[2 * st_stride + r];
        f.n[0] = st[3 * st_stride + r];
        f.n[1] = st[4 * st_stride + r];
        f.n[2] = st[5 * st_stride + r];
        f.lam = st[6 * st_stride + r];
        const Outcome o = photon_back<ZERN, true>(P, L, si, idx, f, tp, ts);
        const bool conv = o.status <= PHX_OFF_CHIP;
        const bool sampled = JAC && A.jac && (g % A.jac_stride) == 0;
        if (!conv) {
            if (sampled) {
                double* J = A.jac + (g / A.jac_stride) * 2 * PHX_N_THETA;
                for (int j = 0; j < 2 * PHX_N_THETA; ++j) J[j] = 0.0;
            }
            continue;
        }
        const double* sd = A.seed + (size_t)(si - L.src_begin) * 8;
        const double dx = o.xe - sd[5], dy = o.ye - sd[6];
        const double sxb = sd[0] + sd[2] * dx + sd[4] * dy;
        const double syb = sd[1] + sd[3] * dy + sd[4] * dx;
        const Rng rng{L.seed, (uint32_t)si, (uint32_t)idx, (uint32_t)(idx >> 32)};
        if (!JAC) {
            adjoint_sweep<ZERN, 1>(P, L, rng, o.lam, tp, ts, &sxb, &syb, acc);
        } else {
            double jl[2][kAdj];
#pragma unroll
            for (int c = 0; c < 2; ++c)
#pragma unroll
                for (int j = 0; j < kAdj; ++j) jl[c][j] = 0.0;
            const double xs[2] = {1.0, 0.0}, ys[2] = {0.0, 1.0};
            adjoint_sweep<ZERN, 2>(P, L, rng, o.lam, tp, ts, xs, ys, jl);
#pragma unroll
            for (int j = 0; j < kAdj; ++j) acc[0][j] += sxb * jl[0][j] + syb * jl[1][j];
            if (sampled) {
                double* J = A.jac + (g / A.jac_stride) * 2 * PHX_N_THETA;
                for (int c = 0; c < 2; ++c) {
                    for (int j = 0; j < 10; ++j) J[c * PHX_N_THETA + j] = jl[c][j];
                    for (int z = 0; z < kNZern; ++z) {
                        double v = 0.0;
                        for (int m = 0; m < kNZernPoly; ++m) v += P.zern_basis[z][m] * jl[c][10 + m];
                        J[c * PHX_N_THETA + 10 + z] = v;
                    }
                }
            }
        }
    }
    block_sum_rows(acc[0], A.partial + (row0 + blockIdx.x) * kAdj);
}

// Column sums of the partial rows (fixed order: each thread a strided share, then a tree).
__global__ __launch_bounds__(256) void adjoint_columns(const double* __restrict__ partial,
                                                       uint64_t rows, double* __restrict__ colsum) {
    __shared__ double s[256];
    const int j = blockIdx.x;
    double v = 0.0;
    for (uint64_t r = threadIdx.x; r < rows; r += blockDim.x) v += partial[r * kAdj + j];
    s[threadIdx.x] = v;
    __syncthreads();
    for (int h = 128; h >= 1; h >>= 1) {
        if (threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) colsum[j] = s[0];
}

// Rigid-body columns as they are; monomial columns mapped to the Zernike amplitudes.
__global__ void adjoint_finish(const DevParams* __restrict__ Pg, const double* __restrict__ colsum,
                               double* __restrict__ grad) {
    const int j = threadIdx.x;
    if (j >= PHX_N_THETA) return;
    if (j < 10) {
        grad[j] = colsum[j];
        return;
    }
    double v = 0.0;
    for (int m = 0; m < kNZernPoly; ++m) v += Pg->zern_basis[j - 10][m] * colsum[10 + m];
    grad[j] = v;
}

__global__ void fill_u32(unsigned int* p, uint64_t n, unsigned int v) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Centred-difference gradients of periodic OPD screens (the refractive kick of section 2.3.2 is
// the phase gradient), single precision: g_x = (W[j][i+1] - W[j][i-1]) * (1/(2p)), likewise g_y.
// Thread (plane, j, i) writes the cell record: gradients at (i, j), (i+1, j), (i, j+1), (i+1, j+1).
__device__ __forceinline__ float2 grad_at(const float* w, int n, int i, int j, float f) {
    const int ip = i + 1 == n ? 0 : i + 1, im = i == 0 ? n - 1 : i - 1;
    const int jp = j + 1 == n ? 0 : j + 1, jm = j == 0 ? n - 1 : j - 1;
    const float dx = w[(int64_t)j * n + ip] - w[(int64_t)j * n + im];
    const float dy = w[(int64_t)jp * n + i] - w[(int64_t)jm * n + i];
    return make_float2(dx * f, dy * f);
}

// Also records, per screen, the largest gradient norm of any cell (as float bits: the order of
// non-negative floats is that of their bits), from which the host bounds how far the atmosphere
// can displace a photon at the primary.
__global__ void gradient_kernel(const float* __restrict__ opd, float4* __restrict__ grad, int n,
                                int n_scales, const float* inv2p, int64_t total,
                                unsigned int* __restrict__ gmax) {
    const int64_t id0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = id0 < total;
    const int64_t id = live ? id0 : total - 1;
    const int64_t nn = (int64_t)n * n;
    const int64_t plane = id / nn;
    const int64_t r = id - plane * nn;
    const int j = (int)(r / n), i = (int)(r - (int64_t)j * n);
    const float* w = opd + plane * nn;
    const float f = inv2p[plane % n_scales];
    const int i1 = i + 1 == n ? 0 : i + 1, j1 = j + 1 == n ? 0 : j + 1;
    const float2 g00 = grad_at(w, n, i, j, f), g10 = grad_at(w, n, i1, j, f);
    const float2 g01 = grad_at(w, n, i, j1, f), g11 = grad_at(w, n, i1, j1, f);
    if (live) {
        grad[2 * id] = make_float4(g00.x, g00.y, g10.x, g10.y);
        grad[2 * id + 1] = make_float4(g01.x, g01.y, g11.x, g11.y);
    }
    if (!gmax) return;
    // a non-finite gradient (from a NaN or infinite optical path) records an infinite maximum
    // (fmaxf would drop a NaN), which the host refuses
    const bool finite = isfinite(g00.x) && isfinite(g00.y);
    float m = live ? (finite ? sqrtf(g00.x * g00.x + g00.y * g00.y) : INFINITY) : 0.0f;
    const int p0 = __shfl((int)plane, 0);
    if (__ballot((int)plane != p0) == 0) {   // the whole wavefront is on one screen
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
        if (__lane_id() == 0) atomicMax(&gmax[plane], __float_as_uint(m));
    } else if (live) {
        atomicMax(&gmax[plane], __float_as_uint(m));
    }
}

}  // namespace

// Pre-roll of one chunk, first half: the survivor bitmap `bits` (and each survivor's time bucket
// in `key` when the chunk's survivors are sorted by time).
static void preroll_generate(const DevParams* dparams, const Launch& L, int n_cu,
                             const LaunchConfig& cfg, const ChunkSpan& sp,
                             unsigned long long* bits, uint8_t* key, hipStream_t stream) {
    const uint64_t want = (sp.len + kGenRange - 1) / kGenRange;
    const uint64_t cap = (uint64_t)n_cu * cfg.generate_per_cu;
    const dim3 gg((unsigned)(want < cap ? want : cap));
    const bool ghost = (L.flags & PHX_F_GHOSTS) != 0;
    if (sp.src >= 0) {
        const auto gk = ghost ? generate_kernel<true, true> : generate_kernel<true, false>;
        hipLaunchKernelGGL(gk, gg, dim3(kBlock), 0, stream, dparams, L, sp.begin, sp.len,
                           L.src_begin + sp.src, sp.first, bits, key);
    } else {
        const auto gk = ghost ? generate_kernel<false, true> : generate_kernel<false, false>;
        hipLaunchKernelGGL(gk, gg, dim3(kBlock), 0, stream, dparams, L, sp.begin, sp.len, 0,
                           (uint64_t)0, bits, key);
    }
}

// Second half: the survivor list (in photon order, or sorted by time bucket when key is given)
// and its count.
static void preroll_compact(const Workspace& W, const ChunkSpan& sp, uint64_t c,
                            const unsigned long long* bits, const uint8_t* key, uint32_t* surv,
                            hipStream_t stream) {
    const uint64_t n_words = (sp.len + 63) / 64;
    if (key) {
        const unsigned nbb = (unsigned)((n_words + kBucketWords - 1) / kBucketWords);
        // hist: [nbb][buckets] counts, then [nbb][buckets] prefixes, then [buckets] totals
        unsigned int* pre = W.hist + (uint64_t)nbb * kTimeBuckets;
        unsigned int* tot = pre + (uint64_t)nbb * kTimeBuckets;
        hipLaunchKernelGGL(bucket_count, dim3(nbb), dim3(kBlock), 0, stream, bits, key, n_words,
                           W.hist);
        hipLaunchKernelGGL(bucket_scan, dim3(kTimeBuckets), dim3(kBlock), 0, stream,
                           (const unsigned int*)W.hist, nbb, pre, tot);
        hipLaunchKernelGGL(bucket_scatter, dim3(nbb), dim3(kBlock), 0, stream, bits, key, n_words,
                           (const unsigned int*)pre, (const unsigned int*)tot, surv, W.counts + c);
        return;
    }
    const unsigned nb = (unsigned)((n_words + kCompactWords - 1) / kCompactWords);
    hipLaunchKernelGGL(compact_count, dim3(nb), dim3(kBlock), 0, stream, bits, n_words, W.bsum);
    hipLaunchKernelGGL(compact_scatter, dim3(nb), dim3(kBlock), 0, stream, bits, n_words,
                       (const unsigned int*)W.bsum, surv, W.counts + c);
}

// Chunks are pipelined over two streams when the pipe gives a second one: the arithmetic-bound
// pre-roll bitmap and optics stage run on pipe.aux, in the order pre-roll(0), pre-roll(1),
// optics(0), pre-roll(2), optics(1), ..., and the survivor compaction and the bandwidth-bound
// sky stage on `stream`, so the two kinds of work share the compute units and neither stream
// carries much more than the other.  Bitmaps, time keys, survivor lists and states alternate
// between two buffers; events order the hand-offs (bitmap -> compaction and sky -> optics, and
// buffer reuse: a chunk's compaction waits for the optics stage two chunks back, and its bitmap
// is rewritten only by the pre-roll issued after the optics stage that follows the sky stage
// that read it), the host issues every event record before the waits on it, and the caller's
// stream waits for the last optics stage before returning work to it.  Without a second stream
// each chunk's stages run in order on `stream`.
namespace {
struct Stages {
    const DevParams* dparams;
    const Launch& L;
    const Workspace& W;
    int n_cu;
    const LaunchConfig& cfg;
    hipStream_t stream;
    const Pipe& pipe;
    const Timing& T;
    bool piped() const { return pipe.aux && pipe.ev; }
    // events per chunk: 0 pre-roll done, 1 sky done, 2 optics done; then one fork event
    hipEvent_t ev(int kind, uint64_t c) const { return pipe.ev[3 * c + kind]; }
    void mark(int kind, int edge, hipStream_t s) const {
        if (T.on) T.record(T.self, kind, edge, s);
    }
    bool preroll() const { return (L.flags & PHX_F_CULL) && (L.flags & PHX_F_COATINGS); }
    hipStream_t arith() const { return piped() ? pipe.aux : stream; }
    uint32_t* surv_buf(uint64_t c) const { return W.survivors + (piped() ? c % 2 : 0) * W.chunk; }
    double* state_buf(uint64_t c) const { return W.state + (piped() ? c % 2 : 0) * 7 * W.chunk; }
    unsigned long long* bits_buf(uint64_t c) const {
        return W.bits + (piped() ? c % 2 : 0) * ((W.chunk + 63) / 64);
    }
    // time keys of chunk c, or null when its survivors keep photon order
    uint8_t* key_buf(uint64_t c) const {
        return (W.plan[c].sort && W.key && W.hist) ? W.key + (piped() ? c % 2 : 0) * W.chunk
                                                   : nullptr;
    }
    const uint32_t* surv(uint64_t c) const { return preroll() ? surv_buf(c) : nullptr; }
    const unsigned int* cnt(uint64_t c) const { return preroll() ? W.counts + c : nullptr; }

    // pre-roll bitmap of chunk c
    void pre(uint64_t c) const {
        const hipStream_t s = arith();
        if (preroll()) {
            mark(0, 0, s);
            preroll_generate(dparams, L, n_cu, cfg, W.plan[c], bits_buf(c), key_buf(c), s);
            mark(0, 1, s);
        }
        if (piped()) (void)hipEventRecord(ev(0, c), s);
    }
    // survivor compaction and sky stage of chunk c on `stream`
    void sky(uint64_t c, unsigned long long* ft) const {
        const ChunkSpan& sp = W.plan[c];
        if (piped()) {
            (void)hipStreamWaitEvent(stream, ev(0, c), 0);
            if (c >= 2) (void)hipStreamWaitEvent(stream, ev(2, c - 2), 0);
        }
        if (preroll()) {
            mark(3, 0, stream);
            preroll_compact(W, sp, c, bits_buf(c), key_buf(c), surv_buf(c), stream);
            mark(3, 1, stream);
        }
        const uint64_t want = (sp.len + kBlock - 1) / kBlock;
        const uint64_t fcap = (uint64_t)n_cu * cfg.front_per_cu;
        const dim3 fg((unsigned)(want < fcap ? want : fcap));
        mark(1, 0, stream);
        const bool extra = (L.flags & kFrontExtra) != 0;
        const auto fk = L.any_sersic ? (extra ? front_kernel<true, true> : front_kernel<true, false>)
                                     : (extra ? front_kernel<false, true> : front_kernel<false, false>);
        hipLaunchKernelGGL(fk, fg, dim3(kBlock), 0, stream, dparams, L, sp.begin, surv(c), cnt(c),
                           sp.len, state_buf(c), W.chunk, ft);
        mark(1, 1, stream);
        if (piped()) (void)hipEventRecord(ev(1, c), stream);
    }
    // the optics stage's stream after waiting for the sky stage of chunk c
    hipStream_t optics_begin(uint64_t c) const {
        if (piped()) (void)hipStreamWaitEvent(pipe.aux, ev(1, c), 0);
        return arith();
    }
    void optics_end(uint64_t c) const {
        if (piped()) (void)hipEventRecord(ev(2, c), pipe.aux);
    }
    void fork(uint64_t n_chunks) const {
        if (!piped()) return;
        (void)hipEventRecord(pipe.ev[3 * n_chunks], stream);
        (void)hipStreamWaitEvent(pipe.aux, pipe.ev[3 * n_chunks], 0);
    }
    void join(uint64_t n_chunks) const {
        if (piped() && n_chunks) (void)hipStreamWaitEvent(stream, ev(2, n_chunks - 1), 0);
    }
    bool valid() const {
        if (!W.state || !W.survivors || !W.counts || !W.bits || !W.bsum) return false;
        if ((W.n_plan && !W.plan) || W.n_plan > W.n_chunks) return false;
        if (piped() && (W.buffers < 2 || pipe.n_ev < 3 * W.n_plan + 1)) return false;
        for (uint64_t c = 0; c < W.n_plan; ++c)
            if (W.plan[c].len > W.chunk) return false;
        return true;
    }
    // Issue every chunk's stages; optics(c) is the caller's callback for the optics stage.
    template <class Optics>
    void run(uint64_t n_chunks, bool dynamic, Optics optics) const {
        fork(n_chunks);
        if (!piped()) {
            for (uint64_t c = 0; c < n_chunks; ++c) {
                pre(c);
                sky(c, dynamic ? W.tiles + 2 * c : nullptr);
                optics(c, optics_begin(c));
                optics_end(c);
            }
            return;
        }
        for (uint64_t c = 0; c < n_chunks; ++c) {
            pre(c);
            sky(c, dynamic ? W.tiles + 2 * c : nullptr);
            if (c >= 1) {
                optics(c - 1, optics_begin(c - 1));
                optics_end(c - 1);
            }
        }
        if (n_chunks) {
            optics(n_chunks - 1, optics_begin(n_chunks - 1));
            optics_end(n_chunks - 1);
        }
        join(n_chunks);
    }
};
}  // namespace

hipError_t launch_trace(const DevParams* dparams, const Launch& L, const Workspace& W, int n_cu,
                        const LaunchConfig& cfg, hipStream_t stream, const Pipe& pipe,
                        const Timing& T) {
    if (L.total == 0) return hipSuccess;
    const Stages S{dparams, L, W, n_cu, cfg, stream, pipe, T};
    if (!S.valid()) return hipErrorInvalidValue;
    // with ghosts every chunk's traced photons may each leave one ghost start in the list
    if ((L.flags & PHX_F_GHOSTS) && (!W.ghost_list || !W.ghost_ctr || W.ghost_cap < W.chunk))
        return hipErrorInvalidValue;
    const uint64_t n_chunks = W.n_plan;
    if (cfg.dynamic)
        hipLaunchKernelGGL(fill_u32, dim3((unsigned)((4 * n_chunks + 255) / 256)), dim3(256), 0,
                           stream, (unsigned int*)W.tiles, 4 * n_chunks, 0u);
    S.run(n_chunks, cfg.dynamic != 0, [&](uint64_t c, hipStream_t bs) {
        const ChunkSpan& sp = W.plan[c];
        const uint64_t want = (sp.len + kBlock - 1) / kBlock;
        const uint64_t bcap = (uint64_t)n_cu * cfg.back_per_cu;
        const dim3 bg((unsigned)(want < bcap ? want : bcap));
        unsigned long long* bt = cfg.dynamic ? W.tiles + 2 * c + 1 : nullptr;
        S.mark(2, 0, bs);
        const bool extra = (L.flags & kBackExtra) != 0, ghost = (L.flags & PHX_F_GHOSTS) != 0;
        if (ghost) {
            // the sequential pass lists the chunk's ghost starts, the second pass runs them (the
            // list is reused by the next chunk, whose optics stage follows on this stream)
            hipLaunchKernelGGL(fill_u32, dim3(1), dim3(64), 0, bs, (unsigned int*)W.ghost_ctr, 4,
                               0u);
            const auto k1 = L.any_zernike ? back_kernel<true, true, 1> : back_kernel<false, true, 1>;
            const auto k2 = L.any_zernike ? back_kernel<true, true, 2> : back_kernel<false, true, 2>;
            hipLaunchKernelGGL(k1, bg, dim3(kBlock), 0, bs, dparams, L, sp.begin, S.surv(c),
                               S.cnt(c), sp.len, (const double*)S.state_buf(c), W.chunk, bt,
                               W.ghost_list, W.ghost_cap, W.ghost_ctr);
            hipLaunchKernelGGL(k2, dim3((unsigned)bcap), dim3(kBlock), 0, bs, dparams, L,
                               sp.begin, S.surv(c), S.cnt(c), sp.len,
                               (const double*)S.state_buf(c), W.chunk,
                               (unsigned long long*)nullptr, W.ghost_list, W.ghost_cap,
                               W.ghost_ctr);
        } else {
            const auto bk = L.any_zernike
                                    ? (extra ? back_kernel<true, true, 0> : back_kernel<true, false, 0>)
                                    : (extra ? back_kernel<false, true, 0> : back_kernel<false, false, 0>);
            hipLaunchKernelGGL(bk, bg, dim3(kBlock), 0, bs, dparams, L, sp.begin, S.surv(c),
                               S.cnt(c), sp.len, (const double*)S.state_buf(c), W.chunk, bt,
                               (double*)nullptr, (uint64_t)0, (unsigned long long*)nullptr);
        }
        S.mark(2, 1, bs);
    });
    return hipGetLastError();
}

hipError_t launch_adjoint(const DevParams* dparams, const Launch& L, const Workspace& W, int n_cu,
                          const LaunchConfig& cfg, const Adjoint& A, double* colsum, double* grad,
                          hipStream_t stream, const Pipe& pipe, const Timing& T) {
    const Stages S{dparams, L, W, n_cu, cfg, stream, pipe, T};
    if (!S.valid()) return hipErrorInvalidValue;
    const uint64_t grid = (uint64_t)n_cu * A.per_cu;
    if (grid * kBlock > A.tape_stride) return hipErrorInvalidValue;
    const uint64_t n_chunks = W.n_plan;
    const bool jac = A.jac != nullptr;
    S.run(n_chunks, false, [&](uint64_t c, hipStream_t bs) {
        const ChunkSpan& sp = W.plan[c];
        const uint64_t row0 = c * grid;
        const dim3 ag((unsigned)grid);
        const double* cst = S.state_buf(c);
        const uint32_t* sv = S.surv(c);
        const unsigned int* cn = S.cnt(c);
        S.mark(2, 0, bs);
        if (L.any_zernike) {
            if (jac)
                hipLaunchKernelGGL((adjoint_kernel<true, true>), ag, dim3(kBlock), 0, bs, dparams,
                                   L, sp.begin, sv, cn, sp.len, cst, W.chunk, A, row0);
            else
                hipLaunchKernelGGL((adjoint_kernel<true, false>), ag, dim3(kBlock), 0, bs, dparams,
                                   L, sp.begin, sv, cn, sp.len, cst, W.chunk, A, row0);
        } else {
            if (jac)
                hipLaunchKernelGGL((adjoint_kernel<false, true>), ag, dim3(kBlock), 0, bs, dparams,
                                   L, sp.begin, sv, cn, sp.len, cst, W.chunk, A, row0);
            else
                hipLaunchKernelGGL((adjoint_kernel<false, false>), ag, dim3(kBlock), 0, bs,
                                   dparams, L, sp.begin, sv, cn, sp.len, cst, W.chunk, A, row0);
        }
        S.mark(2, 1, bs);
    });
    const uint64_t rows = n_chunks * grid;
    hipLaunchKernelGGL(adjoint_columns, dim3(kAdj), dim3(256), 0, stream, A.partial, rows, colsum);
    hipLaunchKernelGGL(adjoint_finish, dim3(1), dim3(64), 0, stream, dparams,
                       (const double*)colsum, grad);
    return hipGetLastError();
}

// Workspace of the entry point without allocation (phx_trace_noalloc), one per GPU for the life
// of the process.  Host code never passes this name to a kernel: it is a host-side stand-in for
// the symbol, and scratch_address gives the device address to use instead.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

hipError_t scratch_address(int device, void** out) {
    static std::mutex mu;
    static void* addr[64] = {};
    if (!out || device < 0 || device >= 64) return hipErrorInvalidValue;
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[device] = p;
    }
    *out = addr[device];
    return hipSuccess;
}

namespace {
// Exclusive prefix of the sources' photon counts: each of 256 lanes sums a contiguous slice, a
// workgroup scan of the slice sums gives each slice its start, and the lane writes its slice.
__global__ __launch_bounds__(256) void prefix_kernel(const DevSource* __restrict__ src,
                                                     int src_begin, int n_src,
                                                     uint64_t* __restrict__ prefix) {
    __shared__ uint64_t s_sum[256];
    const int t = threadIdx.x;
    const int per = (n_src + 255) / 256;
    const int a = min(n_src, t * per), b = min(n_src, a + per);
    uint64_t sum = 0;
    for (int i = a; i < b; ++i) sum += src[src_begin + i].n_photons;
    s_sum[t] = sum;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        const uint64_t v = t >= o ? s_sum[t - o] : 0;
        __syncthreads();
        s_sum[t] += v;
        __syncthreads();
    }
    uint64_t run = t ? s_sum[t - 1] : 0;
    for (int i = a; i < b; ++i) {
        prefix[i] = run;
        run += src[src_begin + i].n_photons;
    }
    if (t == 255) prefix[n_src] = s_sum[255];
}

// guide[b] = the source holding flattened photon b << shift: the number of j in [1, n_src) with
// prefix[j] <= b << shift (the prefix does not decrease); guide[n_blocks] = n_src - 1.
__global__ __launch_bounds__(256) void guide_kernel(const uint64_t* __restrict__ prefix,
                                                    int n_src, int32_t* __restrict__ guide,
                                                    uint64_t n_blocks, uint32_t shift) {
    const uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b > n_blocks) return;
    if (b == n_blocks) {
        guide[b] = n_src - 1;
        return;
    }
    const uint64_t g = b << shift;
    int lo = 1, hi = n_src;   // first j in [1, n_src) with prefix[j] > g, else n_src
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (prefix[mid] <= g) lo = mid + 1; else hi = mid;
    }
    guide[b] = lo - 1;
}
}  // namespace

hipError_t launch_prefix(const DevSource* src, int src_begin, int n_src, uint64_t* prefix,
                         int32_t* guide, uint64_t n_blocks, uint32_t shift, hipStream_t stream) {
    if (!src || !prefix || !guide || n_src < 1 || src_begin < 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(prefix_kernel, dim3(1), dim3(256), 0, stream, src, src_begin, n_src, prefix);
    hipLaunchKernelGGL(guide_kernel, dim3((unsigned)((n_blocks + 1 + 255) / 256)), dim3(256), 0,
                       stream, (const uint64_t*)prefix, n_src, guide, n_blocks, shift);
    return hipGetLastError();
}

hipError_t launch_gradients(const float* opd, float4* grad, int n_layers, int n_scales, int n,
                            const double* pixel, unsigned int* gmax, hipStream_t stream) {
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
                       n_scales, d_inv2p, total, gmax);
    e = hipGetLastError();
    (void)hipFreeAsync(d_inv2p, stream);
    return e;
}

}  // namespace phx
