/*
 * Photon Monte Carlo oracle -- TEST INFRASTRUCTURE ONLY (see phx_oracle.h).
 *
 * Plain double-precision C, compiled with -O2 -ffp-contract=off -fno-fast-math.  Each function
 * names the passage of the PhoSim paper (Peterson et al., ApJS 2015) it follows.  Where the paper
 * is silent or garbled, the reading taken is stated at the function.
 *
 * Random numbers: Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11), keyed per photon so that any
 * photon can be recomputed alone.  key = (seed, source), counter = (photon_lo, photon_hi, block,
 * stream).  Block/word map of stream 0:
 *   block 0: pupil radius, pupil angle, time, wavelength
 *   block 1: wavelength blur within an SED bin, Sersic angle, silicon conversion length, (spare)
 *   blocks 2..5: coating roulette for surfaces 4(b-2) .. 4(b-2)+3
 *   block 6: diffusion Box-Muller pair, (spare, spare)
 *   block 7: aerosol extinction, halo selection, halo azimuth, spider diffraction sign
 *   block 8: dome-seeing Box-Muller pair, (spare, spare)
 * Stream 1, block t: Sersic Gamma sampler trial t (normal pair words 0-1, acceptance word 2).
 *   blocks 9, 10: second-kick scattering count of layers 0-3, 4-7 (one word per layer)
 * Stream 2, block t: micro-roughness halo trial t (proposal word 0, acceptance word 1).
 * Stream 3, block 8 i + j: scattering j of layer i's second kick (wavenumber word 0, azimuth 1).
 *
 * Parity pins (tests/test_oracle_*.py): Philox vs an independent implementation (rocRAND, compiled
 * on the host); uniform conversion exhaustive bounds; pupil density; Sersic radius median and
 * Gamma law; paraboloid focus; ellipsoid foci; Cassegrain focus; Snell invariants and the tilted
 * plate shift; Sellmeier and silicon index values; Rajkanan absorption against published silicon
 * data (order of magnitude); Zernike orthonormality; screen deflection closed forms; coating
 * roulette binomial; conversion depth exponential law; diffusion normal law; photometry integral;
 * air refractivity against standard-air values and its pressure, temperature and water laws;
 * dispersion image shift; aerosol survival exp(-tau sec z); dome-seeing normal law; halo radius
 * against the incomplete-beta CDF; spider shadow area and the lambda / (4 pi d) kick; dead-layer
 * fraction 1 - exp(-alpha t); second kick against exp(-D/2); field diffusion closed forms;
 * readout chain: bleeding conservation and spread, defect and dark statistics, negative-binomial
 * transfer trails, segment geometry, the ideal digitiser, non-linearity, read noise, bit errors.
 */
#include "phx_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* Hooks of the counting build (count.cpp includes this file with every double replaced by a
 * type that counts its arithmetic): the trace stage being counted, a pause around arithmetic that
 * is not the method's (decision margins, per-device constants), Philox blocks and screen bytes
 * read.  Empty in the oracle itself. */
#ifndef ORC_STAGE
#define ORC_STAGE(s)
#define ORC_COUNT_PAUSE()
#define ORC_COUNT_RESUME()
#define ORC_COUNT_PHILOX()
#define ORC_COUNT_GATHER(bytes)
#endif
#define NOTE_MARGIN(m, v)        \
    do {                         \
        ORC_COUNT_PAUSE();       \
        note_margin((m), (v));   \
        ORC_COUNT_RESUME();      \
    } while (0)

/* The tests' boundary band: a photon with a decision margin below ORC_MARGIN_UNIT is one whose
 * decision a rounding-level difference between two implementations may change.  Margins are
 * absolute or relative differences from the decision's threshold, except the SED bin choice,
 * whose distance ORC_SED_MARGIN_ABS is scaled to ORC_MARGIN_UNIT (see trace_one). */
#define ORC_MARGIN_UNIT 1e-7
#define ORC_SED_MARGIN_ABS 1e-12

#define TWO_PI 6.283185307179586476925286766559
#define HC_EV_M 1.2398419843320026e-6 /* h c / e (eV m), SI-exact constants */
#define K_B_EV 8.617333262e-5         /* Boltzmann constant (eV/K) */
#define NEWTON_TOL 1e-12              /* m: |delta l| at convergence (paper: 0.01 um) */
#define NEWTON_MAX 16

/* ------------------------------------------------------------------------------------------ */
/* Philox4x32-10 from its published definition: 10 rounds of
 *   (L0, R0, L1, R1) -> (hi(M1*L1) ^ R0 ^ k0, lo(M1*L1), hi(M0*L0) ^ R1 ^ k1, lo(M0*L0))
 * with the counter words read as (L0, R0, L1, R1) = (c0, c1, c2, c3), multipliers
 * M0 = 0xD2511F53, M1 = 0xCD9E8D57 and the key bumped by the Weyl constants
 * (0x9E3779B9, 0xBB67AE85) between rounds. */
void orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    ORC_COUNT_PHILOX();
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* u = (w + 1/2) 2^-32: exact in double, strictly inside (0, 1). */
double orc_u01(uint32_t w) { return ((double)w + 0.5) * (1.0 / 4294967296.0); }

static void draw(const orc_scene* sc, int32_t src, uint64_t photon, uint32_t block,
                 uint32_t stream, double u[4]) {
    uint32_t ctr[4] = {(uint32_t)photon, (uint32_t)(photon >> 32), block, stream};
    uint32_t key[2] = {sc->seed, (uint32_t)src};
    uint32_t w[4];
    orc_philox(ctr, key, w);
    for (int i = 0; i < 4; ++i) u[i] = orc_u01(w[i]);
}

static void note_margin(double* m, double v) {
    v = fabs(v);
    if (v < *m) *m = v;
}

/* ------------------------------------------------------------------------------------------ */
/* Materials.                                                                                 */

/* Sellmeier equation (section 2.4.1), lambda in micrometres inside the formula. */
double orc_sellmeier(const orc_scene* sc, double lambda_m) {
    double l2 = (lambda_m * 1e6) * (lambda_m * 1e6);
    double s = 1.0;
    for (int i = 0; i < 3; ++i) s += sc->glass_b[i] * l2 / (l2 - sc->glass_c[i]);
    return sqrt(s);
}

/* Silicon index n = 3.36 + 0.211 E + 2.79 exp((E - 3.30)/0.398), E in eV (section 2.4.1). */
double orc_n_silicon(double lambda_m) {
    double e = HC_EV_M / lambda_m;
    return 3.36 + 0.211 * e + 2.79 * exp((e - 3.30) / 0.398);
}

/* Rajkanan absorption coefficient (section 2.4.2), cm^-1.  Reading: the printed "C_i A_i" is
 * C_i A_j (phonon i, indirect gap j), and each squared term contributes only where its base is
 * positive (photon energy above the phonon-assisted threshold); the direct term only above E_gd. */
double orc_rajkanan(double lambda_m, double T) {
    const double beta = 7.021e-4, gam = 1108.0;
    const double eg0[2] = {1.1557, 2.5}, egd0 = 3.2;
    const double ep[2] = {1.827e-2, 5.773e-2};
    const double C[2] = {5.5, 4.0};
    const double A[2] = {3.231e2, 7.237e3};
    const double Ad = 1.052e6;
    /* constants of the device temperature (not counted per photon by the counting build) */
    ORC_COUNT_PAUSE();
    double shift = beta * T * T / (T + gam);
    double absorb[2], emit[2], eg[2], CA[2][2];
    for (int i = 0; i < 2; ++i) {
        absorb[i] = exp(ep[i] / (K_B_EV * T)) - 1.0;
        emit[i] = 1.0 - exp(-ep[i] / (K_B_EV * T));
        eg[i] = eg0[i] - shift;
        for (int j = 0; j < 2; ++j) CA[i][j] = C[i] * A[j];
    }
    double egd = egd0 - shift;
    ORC_COUNT_RESUME();
    double e = HC_EV_M / lambda_m;
    double alpha = 0.0;
    for (int i = 0; i < 2; ++i) {
        for (int j = 0; j < 2; ++j) {
            double a = e - eg[j] + ep[i];
            double b = e - eg[j] - ep[i];
            double term = 0.0;
            if (a > 0.0) term += a * a / absorb[i];
            if (b > 0.0) term += b * b / emit[i];
            alpha += CA[i][j] * term;
        }
    }
    if (e > egd) alpha += Ad * sqrt(e - egd);
    return alpha;
}

static double medium_index(const orc_scene* sc, int medium, double lambda_m) {
    if (medium == ORC_GLASS) return orc_sellmeier(sc, lambda_m);
    if (medium == ORC_SILICON) return orc_n_silicon(lambda_m);
    return 1.0;
}

/* ------------------------------------------------------------------------------------------ */
/* Surfaces (section 2.4.1): conic + polynomial asphere, plus Zernike deformation on M1.        */

/* Noll-indexed Zernike polynomials j = 4..15, RMS-normalised on the unit disk, in Cartesian form
 * (u, v) = (x, y)/R.  Reading of "Zernike expansion up to 5th order" (section 2.4.1): Noll 1976
 * ordering; the perturbation vector carries Z4..Z15. */
double orc_zernike(int j, double u, double v) {
    double r2 = u * u + v * v;
    switch (j) {
    case 1: return 1.0;
    case 2: return 2.0 * u;
    case 3: return 2.0 * v;
    case 4: return sqrt(3.0) * (2.0 * r2 - 1.0);
    case 5: return sqrt(6.0) * (2.0 * u * v);
    case 6: return sqrt(6.0) * (u * u - v * v);
    case 7: return sqrt(8.0) * (3.0 * r2 - 2.0) * v;
    case 8: return sqrt(8.0) * (3.0 * r2 - 2.0) * u;
    case 9: return sqrt(8.0) * (3.0 * u * u * v - v * v * v);
    case 10: return sqrt(8.0) * (u * u * u - 3.0 * u * v * v);
    case 11: return sqrt(5.0) * (6.0 * r2 * r2 - 6.0 * r2 + 1.0);
    case 12: return sqrt(10.0) * (4.0 * r2 - 3.0) * (u * u - v * v);
    case 13: return sqrt(10.0) * (4.0 * r2 - 3.0) * (2.0 * u * v);
    case 14: return sqrt(10.0) * (u * u * u * u - 6.0 * u * u * v * v + v * v * v * v);
    case 15: return sqrt(10.0) * (4.0 * u * u * u * v - 4.0 * u * v * v * v);
    default: return 0.0;
    }
}

/* Partial derivatives of orc_zernike with respect to u and v. */
void orc_zernike_grad(int j, double u, double v, double* du, double* dv) {
    double r2 = u * u + v * v;
    double a = 0.0, b = 0.0;
    switch (j) {
    case 2: a = 2.0; break;
    case 3: b = 2.0; break;
    case 4: a = sqrt(3.0) * 4.0 * u; b = sqrt(3.0) * 4.0 * v; break;
    case 5: a = sqrt(6.0) * 2.0 * v; b = sqrt(6.0) * 2.0 * u; break;
    case 6: a = sqrt(6.0) * 2.0 * u; b = -sqrt(6.0) * 2.0 * v; break;
    case 7: a = sqrt(8.0) * 6.0 * u * v; b = sqrt(8.0) * (3.0 * u * u + 9.0 * v * v - 2.0); break;
    case 8: a = sqrt(8.0) * (9.0 * u * u + 3.0 * v * v - 2.0); b = sqrt(8.0) * 6.0 * u * v; break;
    case 9: a = sqrt(8.0) * 6.0 * u * v; b = sqrt(8.0) * (3.0 * u * u - 3.0 * v * v); break;
    case 10: a = sqrt(8.0) * (3.0 * u * u - 3.0 * v * v); b = -sqrt(8.0) * 6.0 * u * v; break;
    case 11: a = sqrt(5.0) * (24.0 * r2 - 12.0) * u; b = sqrt(5.0) * (24.0 * r2 - 12.0) * v; break;
    case 12:
        a = sqrt(10.0) * (8.0 * u * (u * u - v * v) + (4.0 * r2 - 3.0) * 2.0 * u);
        b = sqrt(10.0) * (8.0 * v * (u * u - v * v) - (4.0 * r2 - 3.0) * 2.0 * v);
        break;
    case 13:
        a = sqrt(10.0) * (16.0 * u * u * v + (4.0 * r2 - 3.0) * 2.0 * v);
        b = sqrt(10.0) * (16.0 * u * v * v + (4.0 * r2 - 3.0) * 2.0 * u);
        break;
    case 14: a = sqrt(10.0) * (4.0 * u * u * u - 12.0 * u * v * v); b = sqrt(10.0) * (4.0 * v * v * v - 12.0 * u * u * v); break;
    case 15: a = sqrt(10.0) * (12.0 * u * u * v - 4.0 * v * v * v); b = sqrt(10.0) * (4.0 * u * u * u - 12.0 * u * v * v); break;
    default: break;
    }
    *du = a;
    *dv = b;
}

/* Surface sag S(x, y) in the element frame and its gradient (sx, sy); returns NAN outside the
 * conic's domain. */
double orc_sag(const orc_scene* sc, int k, double x, double y, double* sx, double* sy) {
    const orc_surface* s = &sc->surf[k];
    double r2 = x * x + y * y;
    double arg = 1.0 - (1.0 + s->kappa) * s->c * s->c * r2;
    if (arg < 0.0) return NAN;
    double root = sqrt(arg);
    double sag = s->c * r2 / (1.0 + root);
    double dsdr_over_r = s->c / root;
    double r = sqrt(r2);
    for (int i = 3; i <= 10; ++i) {
        double a = s->alpha[i - 3];
        if (a == 0.0) continue;
        sag += a * pow(r, (double)i);
        dsdr_over_r += (double)i * a * pow(r, (double)(i - 2));
    }
    double gx = x * dsdr_over_r, gy = y * dsdr_over_r;
    if (k == 0 && sc->zernike_r > 0.0) {
        double R = sc->zernike_r;
        for (int j = 4; j <= 15; ++j) {
            double amp = sc->theta[10 + (j - 4)];
            if (amp == 0.0) continue;
            double du, dv;
            sag += amp * orc_zernike(j, x / R, y / R);
            orc_zernike_grad(j, x / R, y / R, &du, &dv);
            gx += amp * du / R;
            gy += amp * dv / R;
        }
    }
    if (sx) *sx = gx;
    if (sy) *sy = gy;
    return sag;
}

/* Ray-surface intersection (section 2.4.2).  The paper starts from a parabolic approximation and
 * iterates l <- l0 + delta/n_z to 0.01 um.  Reading: the result is the root of
 * f(l) = q_z + l d_z - S(q_x + l d_x, q_y + l d_y) nearest the vertex sheet; this oracle takes the
 * exact conic root as the start (the root of the conic part, continuous as the quadratic
 * coefficient vanishes) and runs Newton on f to |delta l| <= 1e-12 m.  Returns 0 on success,
 * ORC_MISSED or ORC_NONCONV. */
int orc_intersect(const orc_scene* sc, int k, const double q[3], const double d[3], double* l_out,
                  int* iters) {
    const orc_surface* s = &sc->surf[k];
    double ck = 1.0 + s->kappa;
    double A = s->c * (d[0] * d[0] + d[1] * d[1] + ck * d[2] * d[2]);
    double B = s->c * (q[0] * d[0] + q[1] * d[1] + ck * q[2] * d[2]) - d[2];
    double C = s->c * (q[0] * q[0] + q[1] * q[1] + ck * q[2] * q[2]) - 2.0 * q[2];
    double disc = B * B - A * C;
    *iters = 0;
    if (disc < 0.0) return ORC_MISSED;
    double den = B + (B >= 0.0 ? sqrt(disc) : -sqrt(disc));
    if (den == 0.0) return ORC_MISSED;
    double l = -C / den;
    for (int it = 1; it <= NEWTON_MAX; ++it) {
        double x = q[0] + l * d[0], y = q[1] + l * d[1], z = q[2] + l * d[2];
        double sx, sy;
        double S = orc_sag(sc, k, x, y, &sx, &sy);
        if (isnan(S)) return ORC_MISSED;
        double f = z - S;
        double fp = d[2] - (sx * d[0] + sy * d[1]);
        if (fp == 0.0) return ORC_NONCONV;
        double dl = f / fp;
        l -= dl;
        *iters = it;
        if (fabs(dl) <= NEWTON_TOL) {
            *l_out = l;
            return 0;
        }
    }
    return ORC_NONCONV;
}

/* ------------------------------------------------------------------------------------------ */
/* Coatings (section 2.4.2): transmission probability against incidence angle and wavelength,
 * bilinear on the uniform (s = sin^2 theta, lambda) grid of the input table, clamped at its edges. */
static double coating_table(const orc_scene* sc, const float* table, int coat, double s,
                            double lambda_m);
double orc_coating(const orc_scene* sc, int coat, double s, double lambda_m) {
    return coating_table(sc, sc->coat, coat, s, lambda_m);
}

/* Reflection probability of a coating (section 2.4.2: the four-column description carries
 * reflection and transmission), on the transmission tables' grid. */
static double coating_reflect(const orc_scene* sc, int coat, double s, double lambda_m) {
    return sc->coat_r ? coating_table(sc, sc->coat_r, coat, s, lambda_m) : 0.0;
}

static double coating_table(const orc_scene* sc, const float* table, int coat, double s,
                            double lambda_m) {
    const float* t = table + (size_t)coat * sc->n_s * sc->n_lam;
    /* the grid step is a per-scene constant and the wavelength's grid position a per-photon one:
     * the counting build leaves both out of the per-surface work (same arithmetic either way) */
    ORC_COUNT_PAUSE();
    const double s_step = sc->s_max / (double)(sc->n_s - 1);
    double fl = (lambda_m - sc->lam0) / sc->dlam;
    ORC_COUNT_RESUME();
    double fs = s / s_step;
    if (fs < 0.0) fs = 0.0;
    if (fs > (double)(sc->n_s - 1)) fs = (double)(sc->n_s - 1);
    if (fl < 0.0) fl = 0.0;
    if (fl > (double)(sc->n_lam - 1)) fl = (double)(sc->n_lam - 1);
    int is = (int)floor(fs), il = (int)floor(fl);
    if (is > sc->n_s - 2) is = sc->n_s - 2;
    if (il > sc->n_lam - 2) il = sc->n_lam - 2;
    double a = fs - is, b = fl - il;
    double t00 = t[(size_t)is * sc->n_lam + il], t01 = t[(size_t)is * sc->n_lam + il + 1];
    double t10 = t[(size_t)(is + 1) * sc->n_lam + il], t11 = t[(size_t)(is + 1) * sc->n_lam + il + 1];
    return (1.0 - a) * ((1.0 - b) * t00 + b * t01) + a * ((1.0 - b) * t10 + b * t11);
}

/* ------------------------------------------------------------------------------------------ */
/* Atmosphere (sections 2.3.1-2.3.2).                                                          */

static int64_t wrap(int64_t i, int64_t n) {
    int64_t r = i % n;
    return r < 0 ? r + n : r;
}

/* Phase-gradient screens: the refractive kick is the gradient of the phase (section 2.3.2); with
 * screens holding optical path W (m) the kick is grad W.  Reading: centred differences on the
 * periodic grid, in single precision, g_x[j][i] = (W[j][i+1] - W[j][i-1]) * (1/(2p)). */
static void derive_gradients(orc_scene* sc) {
    int64_t N = sc->screen_n;
    for (int l = 0; l < sc->n_layers; ++l)
        for (int s = 0; s < sc->n_scales; ++s) {
            const float* w = sc->opd + ((size_t)l * sc->n_scales + s) * N * N;
            float* g = sc->grad + ((size_t)l * sc->n_scales + s) * N * N * 2;
            float inv2p = (float)(1.0 / (2.0 * sc->pix[s]));
            for (int64_t j = 0; j < N; ++j)
                for (int64_t i = 0; i < N; ++i) {
                    float dx = w[j * N + wrap(i + 1, N)] - w[j * N + wrap(i - 1, N)];
                    float dy = w[wrap(j + 1, N) * N + i] - w[wrap(j - 1, N) * N + i];
                    g[(j * N + i) * 2 + 0] = dx * inv2p;
                    g[(j * N + i) * 2 + 1] = dy * inv2p;
                }
        }
}

/* Bilinear interpolation of one gradient screen at screen-pixel coordinates. */
static void screen_lookup(const orc_scene* sc, int l, int s, double xs, double ys, double* gx,
                          double* gy) {
    int64_t N = sc->screen_n;
    const float* g = sc->grad + ((size_t)l * sc->n_scales + s) * N * N * 2;
    ORC_COUNT_GATHER(32);   /* the four corners' (g_x, g_y) float pairs */
    double fx = floor(xs), fy = floor(ys);
    double a = xs - fx, b = ys - fy;
    int64_t i0 = wrap((int64_t)fx, N), j0 = wrap((int64_t)fy, N);
    int64_t i1 = wrap(i0 + 1, N), j1 = wrap(j0 + 1, N);
    for (int c = 0; c < 2; ++c) {
        double v00 = g[(j0 * N + i0) * 2 + c], v10 = g[(j0 * N + i1) * 2 + c];
        double v01 = g[(j1 * N + i0) * 2 + c], v11 = g[(j1 * N + i1) * 2 + c];
        double v = (1.0 - b) * ((1.0 - a) * v00 + a * v10) + b * ((1.0 - a) * v01 + a * v11);
        if (c == 0) *gx = v; else *gy = v;
    }
}

void orc_screen_gradient(const orc_scene* sc, int layer, int scale, double x, double y,
                         double* gx, double* gy) {
    screen_lookup(sc, layer, scale, x / sc->pix[scale], y / sc->pix[scale], gx, gy);
}

/* ------------------------------------------------------------------------------------------ */
/* Rigid-body misalignments (section 2.4.1: decenter (2), defocus, Euler rotations).  Reading:
 * rotation R = R_x(t_x) R_y(t_y) about the group's pivot, then translation (dx, dy, dz); a point q in
 * a surface's nominal frame maps to global g = R q + t with t = P + R (v - P) + d, v the vertex. */
static void prepare_transforms(orc_scene* sc) {
    for (int k = 0; k < sc->n_surf; ++k) {
        const orc_surface* s = &sc->surf[k];
        double dx = 0, dy = 0, dz = 0, tx = 0, ty = 0;
        const double* P = sc->pivot[0];
        if (s->group == 1 || s->group == 2) {
            const double* th = sc->theta + 5 * (s->group - 1);
            dx = th[0]; dy = th[1]; tx = th[2]; ty = th[3]; dz = th[4];
            P = sc->pivot[s->group];
        }
        double cx = cos(tx), sxn = sin(tx), cy = cos(ty), syn = sin(ty);
        double Rx[3][3] = {{1, 0, 0}, {0, cx, -sxn}, {0, sxn, cx}};
        double Ry[3][3] = {{cy, 0, syn}, {0, 1, 0}, {-syn, 0, cy}};
        double R[3][3];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                R[i][j] = 0.0;
                for (int m = 0; m < 3; ++m) R[i][j] += Rx[i][m] * Ry[m][j];
            }
        double v[3] = {0.0, 0.0, s->z};
        double vp[3] = {v[0] - P[0], v[1] - P[1], v[2] - P[2]};
        double d[3] = {dx, dy, dz};
        for (int i = 0; i < 3; ++i) {
            sc->trans[k][i] = P[i] + (R[i][0] * vp[0] + R[i][1] * vp[1] + R[i][2] * vp[2]) + d[i];
            for (int j = 0; j < 3; ++j) sc->rot[k][i][j] = R[i][j];
        }
    }
}

static void to_local(const orc_scene* sc, int k, const double p[3], const double n[3], double q[3],
                     double d[3]) {
    double r[3] = {p[0] - sc->trans[k][0], p[1] - sc->trans[k][1], p[2] - sc->trans[k][2]};
    for (int i = 0; i < 3; ++i) {
        q[i] = sc->rot[k][0][i] * r[0] + sc->rot[k][1][i] * r[1] + sc->rot[k][2][i] * r[2];
        d[i] = sc->rot[k][0][i] * n[0] + sc->rot[k][1][i] * n[1] + sc->rot[k][2][i] * n[2];
    }
}

static void to_global(const orc_scene* sc, int k, const double q[3], const double d[3], double p[3],
                      double n[3]) {
    for (int i = 0; i < 3; ++i) {
        p[i] = sc->rot[k][i][0] * q[0] + sc->rot[k][i][1] * q[1] + sc->rot[k][i][2] * q[2] +
               sc->trans[k][i];
        n[i] = sc->rot[k][i][0] * d[0] + sc->rot[k][i][1] * d[1] + sc->rot[k][i][2] * d[2];
    }
}

/* ------------------------------------------------------------------------------------------ */
/* SED cumulative distributions (section 2.2): bin probability = f_lambda x bin width / photon
 * energy at the bin centre, accumulated in order, normalised so that CDF[K] = 1 exactly. */
static void build_cdfs(orc_scene* sc) {
    int K = sc->sed_k;
    for (int s = 0; s < sc->n_sed; ++s) {
        double* cdf = sc->sed_cdf + (size_t)s * (K + 1);
        const double* f = sc->sed_flux + (size_t)s * K;
        cdf[0] = 0.0;
        for (int k = 0; k < K; ++k) {
            double lo = sc->sed_edges[k], hi = sc->sed_edges[k + 1];
            cdf[k + 1] = cdf[k] + f[k] * (hi - lo) * (0.5 * (lo + hi));
        }
        double total = cdf[K];
        for (int k = 1; k < K; ++k) cdf[k] = cdf[k] / total;
        cdf[K] = 1.0;
    }
}

int orc_prepare(orc_scene* sc) {
    sc->grad = NULL;
    sc->sed_cdf = NULL;
    if (sc->n_layers > 0 && sc->opd) {
        size_t n = (size_t)sc->n_layers * sc->n_scales * sc->screen_n * sc->screen_n * 2;
        sc->grad = (float*)malloc(n * sizeof(float));
        if (!sc->grad) return -1;
        derive_gradients(sc);
    }
    if (sc->n_sed > 0) {
        sc->sed_cdf = (double*)malloc((size_t)sc->n_sed * (sc->sed_k + 1) * sizeof(double));
        if (!sc->sed_cdf) return -1;
        build_cdfs(sc);
    }
    prepare_transforms(sc);
    return 0;
}

void orc_release(orc_scene* sc) {
    free(sc->grad);
    free(sc->sed_cdf);
    sc->grad = NULL;
    sc->sed_cdf = NULL;
}

/* ------------------------------------------------------------------------------------------ */
/* Sersic radius (section 2.2.1).  With I(r) = I0 exp(-b_n (r/r0)^(1/n)) the radial density is
 * proportional to r I(r); the substitution G = b_n (r/r0)^(1/n) makes G ~ Gamma(2n, 1), so
 * r/r0 = (G/b_n)^n.  Gamma(a >= 1) by Marsaglia & Tsang (2000); a < 1 by Gamma(a+1) U^(1/a).
 * Reading: the paper does not name a sampler.  Trial t draws from stream 1, block t. */
static int gamma_sample(uint32_t seed, int32_t src, uint64_t photon, double shape, double* out,
                        double* margin) {
    orc_scene tmp;
    tmp.seed = seed;
    double dummy = 1e300;
    if (!margin) margin = &dummy;
    double a = shape < 1.0 ? shape + 1.0 : shape;
    double dd = a - 1.0 / 3.0, cc = 1.0 / sqrt(9.0 * dd);
    for (uint32_t t = 0; t < 64; ++t) {
        double u[4];
        draw(&tmp, src, photon, t, 1, u);
        double x = sqrt(-2.0 * log(u[0])) * cos(TWO_PI * u[1]);
        double v = 1.0 + cc * x;
        NOTE_MARGIN(margin, v);
        if (v <= 0.0) continue;
        v = v * v * v;
        double x2 = x * x;
        double t1 = 1.0 - 0.0331 * x2 * x2;
        NOTE_MARGIN(margin, u[2] - t1);
        int accept = u[2] < t1;
        if (!accept) {
            double t2 = 0.5 * x2 + dd * (1.0 - v + log(v));
            NOTE_MARGIN(margin, log(u[2]) - t2);
            accept = log(u[2]) < t2;
        }
        if (accept) {
            double g = dd * v;
            if (shape < 1.0) g *= pow(u[3], 1.0 / shape);
            *out = g;
            return (int)t;
        }
    }
    *out = shape; /* 64 rejections in a row: deterministic fallback to the mean */
    return -1;
}

int orc_gamma(uint32_t seed, int32_t src, uint64_t photon, double shape, double* out) {
    return gamma_sample(seed, src, photon, shape, out, NULL);
}

static void renormalise(double n[3]) {
    double m = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    n[0] /= m; n[1] /= m; n[2] /= m;
}

/* ------------------------------------------------------------------------------------------ */
/* Field model of the charge diffusion (section 2.4.3).                                        */
#define Q_E 1.602176634e-19      /* C */
#define K_B_J 1.380649e-23       /* J/K */
#define EPS0 8.8541878128e-12    /* F/m */
#define EPS_SI 11.7              /* relative permittivity of silicon (the paper gives none) */

/* E_z(z) = V / t_Si + q / (eps0 eps_Si) int_{t_Si}^{z} n_d(z') dz' with
 * n_d(z) = n_bulk + n_b exp(-(t_Si - z)/s_b) + n_f exp(-z/s_f), z the height above the front
 * (collecting) surface; the integral written out in closed form.  Pinned against quadrature of
 * n_d and the uniform-field and uniform-doping closed forms of the diffusion width. */
double orc_field(const orc_scene* sc, double z) {
    const orc_extra* x = &sc->ex;
    double t = sc->t_si;
    double integral = x->si_n_bulk * (z - t);
    if (x->si_s_back > 0.0)
        integral += x->si_n_back * x->si_s_back * (exp(-(t - z) / x->si_s_back) - 1.0);
    if (x->si_s_front > 0.0)
        integral += x->si_n_front * x->si_s_front * (exp(-t / x->si_s_front) - exp(-z / x->si_s_front));
    return x->si_voltage / t + Q_E / (EPS0 * EPS_SI) * integral;
}

/* Electron mobility with velocity saturation (section 2.4.3): v_m = 1.53e9 T^-0.87 cm/s,
 * E_c = 1.01 T^1.55 V/cm, beta = 2.57e-2 T^0.66, mu = (v_m / E_c) / (1 + (E/E_c)^beta)^(1/beta)
 * (E in V/cm, mu in cm^2/Vs, returned in m^2/Vs).  Reading: the printed outer exponent beta is
 * 1/beta, the form whose drift velocity mu E tends to v_m at high field (pinned: the low-field
 * mobility and the saturation velocity of electrons in silicon at 300 K). */
double orc_mobility(double E, double T) {
    double vm = 1.53e9 * pow(T, -0.87);
    double Ec = 1.01 * pow(T, 1.55);
    double beta = 2.57e-2 * pow(T, 0.66);
    double Ecm = fabs(E) * 1e-2;
    double mu = (vm / Ec) / pow(1.0 + pow(Ecm / Ec, beta), 1.0 / beta);
    return mu * 1e-4;
}

/* Diffusion width of an electron converted at depth d below the entrance (back) surface of a
 * back-illuminated device, i.e. at height z = t_Si - d above the front surface (section 2.4.3):
 * sigma = sqrt(2 D t_c), D = mu(E(z), T) k T / q at the conversion height, collection time
 * t_c = int_{z_c}^{z} dz' / |mu(E(z'), T) E(z')| to the collection height z_c.  Reading: D is taken
 * at the conversion height, as the paper writes it; an electron converted at or below z_c is not
 * spread.  The integral: composite Simpson rule with 8192 panels. */
double orc_field_sigma(const orc_scene* sc, double depth) {
    const orc_extra* x = &sc->ex;
    double T = sc->temp_k;
    double z = sc->t_si - depth, zc = x->si_z_collect;
    if (!(z > zc)) return 0.0;
    const int n = 8192;
    double h = (z - zc) / n, sum = 0.0;
    for (int i = 0; i <= n; ++i) {
        double zi = zc + h * i;
        double E = orc_field(sc, zi);
        double f = 1.0 / fabs(orc_mobility(E, T) * E);
        double w = (i == 0 || i == n) ? 1.0 : ((i & 1) ? 4.0 : 2.0);
        sum += w * f;
    }
    double tc = sum * h / 3.0;
    double D = orc_mobility(orc_field(sc, z), T) * K_B_J * T / Q_E;
    return sqrt(2.0 * D * tc);
}

/* ------------------------------------------------------------------------------------------ */
/* Per-photon physics beyond the core path.                                                    */

/* Refractivity n - 1 of air (section 2.3.3, the Filippenko formula): lambda in metres (the
 * formula takes micrometres), pressure P and water-vapour pressure W in mmHg, temperature T in
 * deg C.  Reading: the printed water term ends in a division by W, which would make the term grow
 * without bound in dry air; it is taken as a product with W (humid air is less refractive).
 * Pinned: the refractivity of dry air at 15 C, 760 mmHg near the sodium D line, the 0 C value,
 * pressure scaling and the sign and size of the water term. */
double orc_air_refractivity(double lambda_m, double P, double T, double W) {
    double lam_um = lambda_m * 1e6;
    double s2 = 1.0 / (lam_um * lam_um);
    double dry = 64.328 + 29498.1 / (146.0 - s2) + 255.4 / (41.0 - s2);
    double pt = P * (1.0 + (1.049 - 0.0157 * T) * 1e-6 * P) / (720.883 * (1.0 + 0.003661 * T));
    double wet = (0.0624 - 0.000680 * s2) / (1.0 + 0.003661 * T) * W;
    return 1e-6 * (dry * pt - wet);
}

/* Micro-roughness halo radius (section 2.4.2): the scattered light has surface brightness
 * 1/(1 + (r/r0)^n) on the sky, so x = r/r0 has density proportional to x/(1 + x^n) (per unit x),
 * here truncated at x_max (reading: the paper does not bound the angle; a bound keeps kicks
 * physical).  Reading: the paper names no sampler.  Rejection from the proposal density
 * proportional to x (1 + x^2)^(-n/2), whose CDF 1 - (1 + x^2)^(1 - n/2) inverts in closed form;
 * the ratio (1 + x^2)^(n/2) / (1 + x^n) never exceeds its value 2^(n/2 - 1) at x = 1 (power-mean
 * inequality, n >= 2), so a proposal x is kept when u < ratio / 2^(n/2 - 1).  Trial t reads stream
 * 2, block t (proposal word 0, acceptance word 1); after 32 rejected trials the photon is not
 * scattered (returns -1).  Requires 2 < n <= 6.  Pinned: Kolmogorov-Smirnov against the exact
 * CDF (n = 4: (2/pi) atan(x^2); any n: the regularised incomplete beta I_s(2/n, 1 - 2/n) with
 * s = x^n / (1 + x^n)). */
static int halo_sample(uint32_t seed, int32_t src, uint64_t photon, double n, double x_max,
                       double* x_out, double* margin) {
    double dummy = 1e300;
    if (!margin) margin = &dummy;
    double e = 1.0 - 0.5 * n; /* < 0 */
    double Fq = 1.0 - pow(1.0 + x_max * x_max, e);
    double M = pow(2.0, 0.5 * n - 1.0);
    for (uint32_t t = 0; t < 32; ++t) {
        uint32_t ctr[4] = {(uint32_t)photon, (uint32_t)(photon >> 32), t, 2u};
        uint32_t key[2] = {seed, (uint32_t)src};
        uint32_t w[4];
        orc_philox(ctr, key, w);
        double v = orc_u01(w[0]), u = orc_u01(w[1]);
        /* (1 + x^2)^e = 1 - v Fq */
        double x = sqrt(pow(1.0 - v * Fq, 1.0 / e) - 1.0);
        double ratio = pow(1.0 + x * x, 0.5 * n) / (1.0 + pow(x, n));
        NOTE_MARGIN(margin, u - ratio / M);
        if (u < ratio / M) {
            *x_out = x;
            return (int)t;
        }
    }
    *x_out = 0.0;
    return -1;
}

int orc_halo_sample(uint32_t seed, int32_t src, uint64_t photon, double n, double x_max,
                    double* x_out) {
    return halo_sample(seed, src, photon, n, x_max, x_out, NULL);
}

/* Second kick of the hybrid atmosphere (section 2.3.2): the modes of a layer above kappa_crit
 * act through their long-exposure PSF_>, the Fourier transform of B_>(rho) = exp(-D(rho)/2) with
 * D(rho) = 4 pi int_{kappa_crit} [1 - J0(kappa rho)] Phi(kappa) kappa dkappa.  Writing
 * D = 2 (s2 - C(rho)), with C the correlation of the high-frequency phase (the transform of Phi
 * restricted to kappa > kappa_crit) and s2 = C(0) its variance, gives
 * B_> = exp(-s2) sum_k C^k / k!: PSF_> is a compound Poisson law, K ~ Poisson(s2) scatterings,
 * each a deflection by lambda_ref kappa / (2 pi) toward a uniform azimuth with kappa drawn from
 * the density proportional to Phi(kappa) kappa on [kappa_crit, kappa_max].  Phi is the paper's
 * phase spectrum, 0.033 (2 pi) k^2 C_n^2 kappa^(-11/3), with the Fried parameter of the paper
 * (k^2 int C_n^2 = r0^(-5/3) / 0.423), in the von Karman form of the screens
 * (kappa^2 + kappa0^2)^(-11/6), kappa0 = 2 pi / L0, for the layer's share of the turbulence
 * integral (r0_i^(-5/3) = fraction_i r0^(-5/3)).  Readings: kappa_max is the finest screen's
 * Nyquist wavenumber (the paper's high-frequency screens end there; its integral to infinity would
 * give kicks of radians); at most 8 scatterings per layer (probability of more < 1e-14 for
 * s2 < 0.2); the kicks are scaled by (lambda / lambda_ref)^(-1/5) like the refractive ones.
 * Pinned: the characteristic function of the sampled kick against exp(-D(rho)/2) from the
 * paper's Bessel integral at several rho; the fraction of unkicked photons exp(-s2). */
static double kick_A(const orc_extra* x, double kappa) {
    double k0 = TWO_PI / x->kick_L0;
    return pow(kappa * kappa + k0 * k0, -5.0 / 6.0);
}

double orc_kick_variance(const orc_scene* sc, int layer) {
    const orc_extra* x = &sc->ex;
    double c = 0.033 * TWO_PI / 0.423 * x->kick_fraction[layer] * pow(x->kick_r0, -5.0 / 3.0);
    /* 2 pi int kappa Phi dkappa, int kappa (kappa^2 + k0^2)^(-11/6) = -(3/5) (.)^(-5/6) */
    return TWO_PI * c * 0.6 * (kick_A(x, x->kick_kappa_crit) - kick_A(x, x->kick_kappa_max));
}

static int second_kick(const orc_scene* sc, int32_t si, uint64_t photon, int layer, double* kx,
                       double* ky, double* margin) {
    const orc_extra* x = &sc->ex;
    double u[4];
    draw(sc, si, photon, (uint32_t)(9 + layer / 4), 0, u);
    double uk = u[layer % 4];
    double s2 = orc_kick_variance(sc, layer);
    /* K = the smallest k with P(K <= k) > u */
    double p = exp(-s2), cum = p;
    int K = 0;
    NOTE_MARGIN(margin, uk - cum);
    while (!(uk < cum) && K < 8) {
        ++K;
        p *= s2 / K;
        cum += p;
        NOTE_MARGIN(margin, uk - cum);
    }
    *kx = 0.0;
    *ky = 0.0;
    double A0 = kick_A(x, x->kick_kappa_crit);
    double dA = A0 - kick_A(x, x->kick_kappa_max);
    double k0 = TWO_PI / x->kick_L0;
    for (int j = 0; j < K; ++j) {
        double w[4];
        draw(sc, si, photon, (uint32_t)(8 * layer + j), 3, w);
        /* invert the wavenumber CDF (A(kappa_crit) - A(kappa)) / dA = w0 */
        double A = A0 - w[0] * dA;
        double kappa = sqrt(pow(A, -6.0 / 5.0) - k0 * k0);
        double th = sc->lambda_ref * kappa / TWO_PI;
        *kx += th * cos(TWO_PI * w[1]);
        *ky += th * sin(TWO_PI * w[1]);
    }
    return K;
}

int orc_second_kick(const orc_scene* sc, int32_t src, uint64_t photon, int layer, double* kx,
                    double* ky) {
    double m = 1e300;
    return second_kick(sc, src, photon, layer, kx, ky, &m);
}

/* Spider (section 2.4.1: rectangular volumes; section 2.4.2: edge diffraction after Freniere et
 * al.).  Vane k is the box u in [r_in, r_out], |v| <= w/2, z in [z_lo, z_hi] in the frame of the
 * unit vectors u = (cos a_k, sin a_k, 0), v = (-sin a_k, cos a_k, 0), a_k = a_0 + 2 pi k / vanes.
 * Returns 1 if the incoming ray meets a vane (q = the first entry point along the ray).  Otherwise d is the smallest
 * distance between the ray's line and a long edge of any vane (the four segments along u at
 * v = +-w/2, z = z_lo or z_hi; for a segment, the distance of the line to its nearest point), the
 * ray moves to the vanes' mid-height and turns by lambda / (4 pi d) across the nearest vane,
 * along +v or -v by the sign word.  Readings: only the incoming pass is tested (as for the central
 * obscuration); the deflection is perpendicular to the edge in the horizontal plane with a random
 * sign (the spread of the uncertainty-principle picture), added to (n_x, n_y) with
 * renormalisation like the other kicks; d is floored at lambda (the formula diverges at the
 * edge).  Pinned: the shadowed fraction of a vertical beam against the vanes' exact area inside
 * the annulus; the focal-plane offset against lambda / (4 pi d) for vertical rays. */
static int spider(const orc_scene* sc, double p[3], double n[3], double lam, double u_sign,
                  double q[3], double* margin, double* cond) {
    const orc_extra* x = &sc->ex;
    double hw = 0.5 * x->vane_width;
    double best = INFINITY, second = INFINITY, dk[8], t_hit = INFINITY;
    int best_k = -1;
    for (int k = 0; k < x->vanes; ++k) {
        dk[k] = INFINITY;
        double a = x->vane_angle + TWO_PI * k / x->vanes;
        double U[3] = {cos(a), sin(a), 0.0}, V[3] = {-sin(a), cos(a), 0.0};
        /* ray in the vane frame */
        double pu = p[0] * U[0] + p[1] * U[1], pv = p[0] * V[0] + p[1] * V[1], pz = p[2];
        double nu = n[0] * U[0] + n[1] * U[1], nv = n[0] * V[0] + n[1] * V[1], nz = n[2];
        double lo[3] = {x->vane_r_in, -hw, x->vane_z_lo}, hi[3] = {x->vane_r_out, hw, x->vane_z_hi};
        double o[3] = {pu, pv, pz}, dd[3] = {nu, nv, nz};
        double t0 = -INFINITY, t1 = INFINITY;
        int inside = 1;
        for (int i = 0; i < 3; ++i) {
            if (dd[i] == 0.0) {
                if (o[i] < lo[i] || o[i] > hi[i]) inside = 0;
            } else {
                double ta = (lo[i] - o[i]) / dd[i], tb = (hi[i] - o[i]) / dd[i];
                if (ta > tb) { double tmp = ta; ta = tb; tb = tmp; }
                if (ta > t0) t0 = ta;
                if (tb < t1) t1 = tb;
            }
        }
        if (inside && t0 <= t1 && t1 >= 0.0) {
            if (t0 < 0.0) t0 = 0.0;
            NOTE_MARGIN(margin, (t1 - t0) / (fabs(t0) + fabs(t1)));
            if (t0 < t_hit) t_hit = t0;
            continue;
        }
        /* distance of the ray's line to the four long edges */
        for (int e = 0; e < 4; ++e) {
            double ve = (e & 1) ? hw : -hw, ze = (e & 2) ? x->vane_z_hi : x->vane_z_lo;
            /* edge point E(s) = s U + ve V + ze z; w0 = E(0) - p */
            double w0[3] = {ve * V[0] - p[0], ve * V[1] - p[1], ze - p[2]};
            double b = U[0] * n[0] + U[1] * n[1];
            double dw = U[0] * w0[0] + U[1] * w0[1];
            double ew = n[0] * w0[0] + n[1] * w0[1] + n[2] * w0[2];
            double s = (b * ew - dw) / (1.0 - b * b);
            if (s < x->vane_r_in) s = x->vane_r_in;
            if (s > x->vane_r_out) s = x->vane_r_out;
            double r[3] = {w0[0] + s * U[0], w0[1] + s * U[1], w0[2]};
            double rn = r[0] * n[0] + r[1] * n[1] + r[2] * n[2];
            double c[3] = {r[0] - rn * n[0], r[1] - rn * n[1], r[2] - rn * n[2]};
            double dist = sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
            if (dist < dk[k]) dk[k] = dist;
        }
    }
    if (t_hit < INFINITY) {
        for (int i = 0; i < 3; ++i) q[i] = p[i] + n[i] * t_hit;
        return 1;
    }
    for (int k = 0; k < x->vanes; ++k)
        if (dk[k] < best) { best = dk[k]; best_k = k; }
    if (best_k < 0) return 0;
    for (int k = 0; k < x->vanes; ++k)
        if (k != best_k && dk[k] < second) second = dk[k];
    NOTE_MARGIN(margin, best / x->vane_width);
    if (second < INFINITY) NOTE_MARGIN(margin, (second - best) / best);
    NOTE_MARGIN(margin, u_sign - 0.5);
    double zm = 0.5 * (x->vane_z_lo + x->vane_z_hi);
    double l = (zm - p[2]) / n[2];
    p[0] += n[0] * l;
    p[1] += n[1] * l;
    p[2] = zm;
    double a = x->vane_angle + TWO_PI * best_k / x->vanes;
    double delta = lam / (2.0 * TWO_PI * (best > lam ? best : lam));
    /* conditioning of the rest of the path: a difference dd in the edge distance turns the ray by
     * delta / d x dd (zero where d is floored at lambda) */
    ORC_COUNT_PAUSE();
    *cond = best > lam ? delta / best : 0.0;
    ORC_COUNT_RESUME();
    if (!(u_sign < 0.5)) delta = -delta;
    n[0] += delta * -sin(a);
    n[1] += delta * cos(a);
    renormalise(n);
    return 0;
}

/* ------------------------------------------------------------------------------------------ */
/* The per-photon trace.                                                                       */

static void set_event(orc_event* ev, int status, int surface, const double p[3]) {
    ev->status = status;
    ev->surface = surface;
    ev->x = p[0]; ev->y = p[1]; ev->z = p[2];
}


#define GHOST_MAX 16

/* The surface a ray meets first (ghost mode, section 2.4.2): the smallest intersection distance
 * l > 1e-9 m among all surfaces other than `from` whose intersection converges; -1 if none. */
static int nearest_surface(const orc_scene* sc, const double p[3], const double n[3], int from,
                           double* margin) {
    double best = INFINITY, second = INFINITY;
    int bk = -1;
    for (int j = 0; j < sc->n_surf; ++j) {
        if (j == from) continue;
        double q[3], d[3], l;
        int it;
        to_local(sc, j, p, n, q, d);
        if (orc_intersect(sc, j, q, d, &l, &it) != 0 || !(l > 1e-9)) continue;
        if (l < best) { second = best; best = l; bk = j; }
        else if (l < second) second = l;
    }
    if (bk >= 0 && second < INFINITY) NOTE_MARGIN(margin, (second - best) / best);
    return bk;
}

/* The detector (sections 2.4.2-2.4.3): conversion after the mean free path x Exp(1) along the
 * refracted direction d, escape, the dead layer, diffusion and the pixel. */
static void land(const orc_scene* sc, int32_t si, uint64_t photon, int k, const double q[3],
                 const double d[3], double lam, const double u1[4], double* margin_p,
                 orc_event* ev, uint32_t* image) {
    const orc_extra* ex = &sc->ex;
    double margin = *margin_p;
    ORC_STAGE(2);   /* sensor: silicon, diffusion, pixel */
    ev->x = q[0]; ev->y = q[1]; ev->z = q[2];
    double xc = q[0], yc = q[1];
    if (sc->physics & ORC_SILICON_PHYS) {
        /* conversion length = mean free path x Exp(1) (section 2.4.2) */
        double alpha = orc_rajkanan(lam, sc->temp_k) * 100.0; /* m^-1 */
        double L = alpha > 0.0 ? -log(u1[2]) / alpha : INFINITY;
        double depth = L * fabs(d[2]);
        NOTE_MARGIN(&margin, (depth - sc->t_si) / sc->t_si);
        if (!(depth <= sc->t_si)) {
            set_event(ev, ORC_ESCAPED, k, q);
            ev->margin = margin;
            return;
        }
        if (sc->physics & ORC_DEAD_LAYER) {
            /* field-free dead layer (section 2.4.2): electrons converted within `dead` of the
             * surface the light enters are removed.  Reading: the paper's "back surface" of a
             * back-illuminated device is the illuminated one. */
            NOTE_MARGIN(&margin, (depth - ex->dead) / sc->t_si);
            if (depth < ex->dead) {
                set_event(ev, ORC_DEAD, k, q);
                ev->margin = margin;
                return;
            }
        }
        xc = q[0] + d[0] * L;
        yc = q[1] + d[1] * L;
        if (sc->physics & ORC_DIFFUSION) {
            /* Gaussian diffusion with sigma proportional to the drift distance (section 2.4.3
             * simplified: sigma = sigma_max (t_Si - depth)/t_Si), or the field model */
            double ud[4];
            draw(sc, si, photon, 6, 0, ud);
            double sigma = (sc->physics & ORC_FIELD_DIFFUSION)
                               ? orc_field_sigma(sc, depth)
                               : sc->sigma_max * (sc->t_si - depth) / sc->t_si;
            double rad = sqrt(-2.0 * log(ud[0]));
            xc += sigma * rad * cos(TWO_PI * ud[1]);
            yc += sigma * rad * sin(TWO_PI * ud[1]);
        }
    }
    ev->xe = xc;
    ev->ye = yc;
    /* pixel quantisation (section 2.4.3, last step) */
    double fx = (xc - sc->chip_x0) / sc->pixel, fy = (yc - sc->chip_y0) / sc->pixel;
    double ix = floor(fx), iy = floor(fy);
    NOTE_MARGIN(&margin, fx - ix);
    NOTE_MARGIN(&margin, 1.0 - (fx - ix));
    NOTE_MARGIN(&margin, fy - iy);
    NOTE_MARGIN(&margin, 1.0 - (fy - iy));
    ev->status = ORC_OFF_CHIP;
    ev->surface = k;
    if (ix >= 0.0 && ix < (double)sc->nx && iy >= 0.0 && iy < (double)sc->ny) {
        ev->status = ORC_DETECTED;
        ev->pix_i = (int32_t)ix;
        ev->pix_j = (int32_t)iy;
        if (image) image[(size_t)ev->pix_j * sc->nx + ev->pix_i] += 1u;
    }
    ev->margin = margin;
}

static void trace_one(const orc_scene* sc, int32_t si, uint64_t photon, uint32_t* image,
                      orc_event* ev) {
    const orc_source* src = &sc->src[si];
    double margin = 1e300;
    double u0[4], u1[4];
    ORC_STAGE(0);   /* sky: source, atmosphere, start plane */
    draw(sc, si, photon, 0, 0, u0);
    draw(sc, si, photon, 1, 0, u1);
    memset(ev, 0, sizeof(*ev));
    ev->photon = photon;
    ev->source = si;
    ev->pix_i = ev->pix_j = -1;

    /* Direction from the source (section 2.2): tangent coordinates as n_x, n_y,
     * n_z = -sqrt(1 - n_x^2 - n_y^2). */
    double n[3] = {src->xi, src->eta, -sqrt(1.0 - src->xi * src->xi - src->eta * src->eta)};
    if (src->kind == 1) {
        /* Ellipsoidal Sersic (section 2.2.1): distance a r/r0 and b r/r0 along the axes at a
         * uniform angle, rotated by the position angle, applied paraxially to n_x, n_y. */
        double g;
        gamma_sample(sc->seed, si, photon, 2.0 * src->sersic_n, &g, &margin);
        double rr = pow(g / src->sersic_bn, src->sersic_n);
        double psi = TWO_PI * u1[1];
        double dmaj = src->sersic_a * rr * cos(psi), dmin = src->sersic_b * rr * sin(psi);
        double cp = cos(src->sersic_pa), sp = sin(src->sersic_pa);
        n[0] += dmaj * cp - dmin * sp;
        n[1] += dmaj * sp + dmin * cp;
        renormalise(n);
    }
    /* Time stamp t = t0 + t_e u (section 2.2), t0 = 0. */
    double t = sc->exposure * u0[2];
    /* Wavelength (section 2.2): top-hat flat in photon number, or the SED's photon CDF with a
     * uniform blur across the chosen bin; then (1 + z). */
    double lam;
    if (src->sed < 0) {
        lam = src->lam_lo + u0[3] * (src->lam_hi - src->lam_lo);
    } else {
        const double* cdf = sc->sed_cdf + (size_t)src->sed * (sc->sed_k + 1);
        int k = 0;
        while (k < sc->sed_k - 1 && !(cdf[k + 1] > u0[3])) ++k;
        /* Margin of the bin choice, on the common scale of the other margins: any implementation
         * compares the same uniform with a CDF summed in the same order, whose entries then
         * agree with these to K eps (1.7e-13 for the 761 bins of a blackbody table, counting
         * both sides), so only a uniform within ORC_SED_MARGIN_ABS of an edge can change bin;
         * that distance is recorded as ORC_MARGIN_UNIT.  (Taken as it stands, |u - CDF[k]| below
         * 1e-7 would hold 2e-7 K = 1.5e-4 of the photons, none of them near a change of bin.) */
        NOTE_MARGIN(&margin, (u0[3] - cdf[k]) * (ORC_MARGIN_UNIT / ORC_SED_MARGIN_ABS));
        NOTE_MARGIN(&margin, (u0[3] - cdf[k + 1]) * (ORC_MARGIN_UNIT / ORC_SED_MARGIN_ABS));
        lam = sc->sed_edges[k] + u1[0] * (sc->sed_edges[k + 1] - sc->sed_edges[k]);
    }
    lam = lam * (1.0 + src->redshift);
    ev->lambda = lam;
    const orc_extra* ex = &sc->ex;
    if (sc->physics & ORC_DISPERSION) {
        /* Atmospheric dispersion (section 2.3.3): refraction (n_air - 1) tan z toward the zenith,
         * less that of the reference wavelength lam0, applied to (n_x, n_y) like the Sersic
         * offset.  Reading: plane-parallel refraction R = (n - 1) tan z. */
        double dR = (orc_air_refractivity(lam, ex->pressure, ex->temperature, ex->water) -
                     orc_air_refractivity(ex->lam0, ex->pressure, ex->temperature, ex->water)) *
                    tan(ex->zenith);
        n[0] += dR * cos(ex->zenith_pa);
        n[1] += dR * sin(ex->zenith_pa);
        renormalise(n);
    }

    /* Pupil (section 2.2): r = sqrt(u (r_o^2 - r_i^2) + r_i^2), phi = 2 pi v on the (slightly
     * enlarged) annulus of the first mirror, z from its nominal surface. */
    double ro = sc->pupil_r_out + sc->pupil_margin;
    double ri = sc->pupil_r_in - sc->pupil_margin;
    if (ri < 0.0) ri = 0.0;
    double r = sqrt(u0[0] * (ro * ro - ri * ri) + ri * ri);
    double phi = TWO_PI * u0[1];
    double p[3] = {r * cos(phi), r * sin(phi), 0.0};
    ev->t = t;
    ev->px = p[0];
    ev->py = p[1];
    {
        /* nominal sag of the first surface: conic + asphere only */
        const orc_surface* s0 = &sc->surf[0];
        double r2 = p[0] * p[0] + p[1] * p[1];
        double arg = 1.0 - (1.0 + s0->kappa) * s0->c * s0->c * r2;
        double z = s0->z + (arg >= 0.0 ? s0->c * r2 / (1.0 + sqrt(arg)) : 0.0);
        for (int i = 3; i <= 10; ++i)
            if (s0->alpha[i - 3] != 0.0) z += s0->alpha[i - 3] * pow(sqrt(r2), (double)i);
        p[2] = z;
    }

    if ((sc->physics & ORC_ATMOSPHERE) && sc->n_layers > 0) {
        /* Up to the highest layer along the ray (reading of the top-of-atmosphere move: the ray
         * is moved up, l = (h - z)/n_z), then down through the layers (section 2.3.1:
         * x <- x + n l, l = (h_i - h_{i+1})/(-n_z)), deflecting by the screen gradients at the
         * wind-shifted position (section 2.3.1 frozen flow; section 2.3.2 kick = grad of phase)
         * scaled by (lambda/lambda_ref)^(-1/5) (section 2.3.2). */
        double scale = pow(lam / sc->lambda_ref, -0.2);
        for (int i = sc->n_layers - 1; i >= 0; --i) {
            double h = sc->height[i];
            double l = (h - p[2]) / n[2];
            p[0] += n[0] * l;
            p[1] += n[1] * l;
            p[2] = h;
            double gx = 0.0, gy = 0.0;
            for (int s = 0; s < sc->n_scales; ++s) {
                double ax, ay;
                double xs = (p[0] - sc->wind[i][0] * t) / sc->pix[s];
                double ys = (p[1] - sc->wind[i][1] * t) / sc->pix[s];
                screen_lookup(sc, i, s, xs, ys, &ax, &ay);
                gx += ax;
                gy += ay;
            }
            if (sc->physics & ORC_SECOND_KICK) {
                double kx, ky;
                second_kick(sc, si, photon, i, &kx, &ky, &margin);
                gx += kx;
                gy += ky;
            }
            n[0] += scale * gx;
            n[1] += scale * gy;
            renormalise(n);
        }
    }
    /* Back along the ray to the start plane above every optic. */
    {
        double l = (sc->z_start - p[2]) / n[2];
        p[0] += n[0] * l;
        p[1] += n[1] * l;
        p[2] = sc->z_start;
    }
    ORC_STAGE(1);   /* optics: entrance effects, obscuration, surfaces */
    double u7[4] = {0.5, 0.5, 0.5, 0.5};
    if (sc->physics & (ORC_AEROSOL | ORC_HALO | ORC_SPIDER)) draw(sc, si, photon, 7, 0, u7);
    if (sc->physics & ORC_AEROSOL) {
        /* Aerosol opacity (section 2.3.3): tau = tau0 (lambda / 500 nm)^gamma at the zenith, times
         * the airmass sec z along the path; the photon survives with probability exp(-tau).
         * Reading: the printed destruction probability exp(-tau) is the survival probability. */
        double tau = ex->tau0 * pow(lam / 500e-9, ex->gamma) / cos(ex->zenith);
        double keep = exp(-tau);
        NOTE_MARGIN(&margin, u7[0] - keep);
        if (!(u7[0] < keep)) {
            set_event(ev, ORC_EXTINCT, -1, p);
            ev->margin = margin;
            return;
        }
    }
    if (sc->physics & ORC_DOME) {
        /* Dome seeing (section 2.4.2): an isotropic Gaussian kick of the direction, standard
         * deviation dome_sigma per axis (Box-Muller), at the entrance of the telescope. */
        double ud[4];
        draw(sc, si, photon, 8, 0, ud);
        double rad = sqrt(-2.0 * log(ud[0]));
        n[0] += ex->dome_sigma * rad * cos(TWO_PI * ud[1]);
        n[1] += ex->dome_sigma * rad * sin(TWO_PI * ud[1]);
        renormalise(n);
    }
    if (sc->physics & ORC_HALO) {
        /* Micro-roughness halo (section 2.4.2): with probability f, a kick of angle r0 x
         * (halo_sample) toward a uniform azimuth, at the start of the telescope. */
        NOTE_MARGIN(&margin, u7[1] - ex->halo_f);
        if (u7[1] < ex->halo_f) {
            double xh;
            if (halo_sample(sc->seed, si, photon, ex->halo_n, ex->halo_max / ex->halo_r0, &xh,
                            &margin) >= 0) {
                double r = ex->halo_r0 * xh;
                n[0] += r * cos(TWO_PI * u7[2]);
                n[1] += r * sin(TWO_PI * u7[2]);
                renormalise(n);
            }
        }
    }
    if ((sc->physics & ORC_SPIDER) && ex->vanes > 0) {
        double q[3], cond = 0.0;
        if (spider(sc, p, n, lam, u7[3], q, &margin, &cond)) {
            set_event(ev, ORC_OBSCURED, -1, q);
            ev->margin = margin;
            return;
        }
        ev->cond = cond;
    }
    /* Central obscuration (shadow of the secondary; section 2.4.1 obscuring structure). */
    if (sc->obsc_r > 0.0) {
        double l = (sc->obsc_z - p[2]) / n[2];
        double x = p[0] + n[0] * l, y = p[1] + n[1] * l;
        double rr = sqrt(x * x + y * y);
        NOTE_MARGIN(&margin, (rr - sc->obsc_r) / sc->obsc_r);
        if (rr < sc->obsc_r) {
            double q[3] = {x, y, sc->obsc_z};
            set_event(ev, ORC_OBSCURED, -1, q);
            ev->margin = margin;
            return;
        }
    }

    /* The surfaces in travel order (section 2.4.2).  With ghosts, a photon reflected by a filter
     * or anti-reflection coating propagates backwards (section 2.4.2): from then on the next
     * surface is the nearest one ahead along the ray among all the others (the paper loops
     * through all surfaces by their intersection distance), at most GHOST_MAX interactions. */
    double n_cur = 1.0;
    int medium = ORC_VACUUM;
    double n_index[3] = {1.0, -1.0, -1.0};   /* vacuum, glass, silicon: formed on first use */
    double ucoat[4];
    int coat_block = -1;
    int ghost = 0, from = -1, inter = 0, next = 0;
    for (;;) {
        int k;
        if (!ghost) {
            if (next >= sc->n_surf) {
                /* ran out of surfaces without a detector */
                set_event(ev, ORC_MISSED, sc->n_surf, p);
                ev->margin = margin;
                return;
            }
            k = next;
        } else {
            if (inter >= GHOST_MAX) {
                set_event(ev, ORC_MISSED, from, p);
                ev->margin = margin;
                return;
            }
            k = nearest_surface(sc, p, n, from, &margin);
            if (k < 0) {   /* leaves the optics */
                set_event(ev, ORC_MISSED, from, p);
                ev->margin = margin;
                return;
            }
            ++inter;
        }
        const orc_surface* s = &sc->surf[k];
        double q[3], d[3];
        to_local(sc, k, p, n, q, d);
        double l;
        int it;
        int st = orc_intersect(sc, k, q, d, &l, &it);
        ev->newton += it;
        if (st == 0 && !(l > 0.0)) st = ORC_MISSED;
        if (st != 0) {
            set_event(ev, st, k, q);
            ev->margin = margin;
            return;
        }
        q[0] += d[0] * l; q[1] += d[1] * l; q[2] += d[2] * l;
        /* clear aperture (paper Table 1: outer and inner radii) */
        double rq = sqrt(q[0] * q[0] + q[1] * q[1]);
        if (s->r_in > 0.0) NOTE_MARGIN(&margin, (rq - s->r_in) / s->r_in);
        NOTE_MARGIN(&margin, (rq - s->r_out) / s->r_out);
        if (rq < s->r_in || rq > s->r_out) {
            set_event(ev, ORC_VIGNETTED, k, q);
            ev->margin = margin;
            return;
        }
        /* surface normal from the analytic sag gradient */
        double gx, gy;
        orc_sag(sc, k, q[0], q[1], &gx, &gy);
        double N[3] = {-gx, -gy, 1.0};
        renormalise(N);
        double dn = d[0] * N[0] + d[1] * N[1] + d[2] * N[2];
        if (dn > 0.0) { N[0] = -N[0]; N[1] = -N[1]; N[2] = -N[2]; dn = -dn; }
        double cosi = -dn;
        int is_det = (s->kind == ORC_DETECTOR);
        int reflect = s->kind == ORC_MIRROR;
        /* coating roulette (section 2.4.2): transmitted with probability T(angle, lambda) (for a
         * mirror: reflected); with ghosts a filter or anti-reflection coating reflects with
         * probability R; otherwise the photon is absorbed.  Sequential passage: the surface's own
         * word (block 2 + k/4); in ghost mode stream 4, block = interaction number. */
        if ((sc->physics & ORC_COATINGS) && s->coating >= 0) {
            double uk;
            if (!ghost) {
                int blk = 2 + k / 4;
                if (blk != coat_block) { draw(sc, si, photon, (uint32_t)blk, 0, ucoat); coat_block = blk; }
                uk = ucoat[k % 4];
            } else {
                double ug[4];
                draw(sc, si, photon, (uint32_t)(inter - 1), 4, ug);
                uk = ug[0];
            }
            double T = orc_coating(sc, s->coating, 1.0 - cosi * cosi, lam);
            NOTE_MARGIN(&margin, uk - T);
            if (!(uk < T)) {
                double R = 0.0;
                if ((sc->physics & ORC_GHOSTS) && s->kind != ORC_MIRROR) {
                    R = coating_reflect(sc, s->coating, 1.0 - cosi * cosi, lam);
                    NOTE_MARGIN(&margin, uk - (T + R));
                }
                if (!(uk < T + R)) {
                    set_event(ev, ORC_ABSORBED, k, q);
                    ev->margin = margin;
                    return;
                }
                reflect = 1;      /* a ghost: reflected by a refracting surface's coating */
                ghost = 1;
            }
        }
        if (reflect) {
            /* reflection across the normal (section 2.4.2) */
            for (int i = 0; i < 3; ++i) d[i] = d[i] - 2.0 * dn * N[i];
        } else if (!is_det || (sc->physics & ORC_SILICON_PHYS)) {
            /* refraction by the vector form of Snell's law (section 2.4.2) into the medium on the
             * other side of the surface (in travel order the surface's own medium), indices from
             * the Sellmeier / silicon formulas (section 2.4.1); vacuum elsewhere */
            int after = s->medium, before = k > 0 ? sc->surf[k - 1].medium : ORC_VACUUM;
            int m2 = medium == after ? before : after;
            /* each index once per photon (it depends on the wavelength only) */
            if (n_index[m2] < 0.0) n_index[m2] = medium_index(sc, m2, lam);
            double n2 = n_index[m2];
            double mu = n_cur / n2;
            double kk = 1.0 - mu * mu * (1.0 - cosi * cosi);
            NOTE_MARGIN(&margin, kk);
            if (kk < 0.0) {
                set_event(ev, ORC_TIR, k, q);
                ev->margin = margin;
                return;
            }
            double f = mu * cosi - sqrt(kk);
            for (int i = 0; i < 3; ++i) d[i] = mu * d[i] + f * N[i];
            n_cur = n2;
            medium = m2;
        }
        if (is_det && !reflect) {
            land(sc, si, photon, k, q, d, lam, u1, &margin, ev, image);
            return;
        }
        to_global(sc, k, q, d, p, n);
        from = k;
        next = k + 1;
    }
}

int orc_trace(const orc_scene* sc, int32_t src, uint64_t begin, uint64_t count, uint32_t* image,
              orc_event* events) {
    if (src < 0 || src >= sc->n_src) return -1;
    orc_event tmp;
    for (uint64_t i = 0; i < count; ++i) {
        orc_event* ev = events ? &events[i] : &tmp;
        trace_one(sc, src, begin + i, image, ev);
    }
    return 0;
}

/* The photons photon[0 .. count) of source src, one by one (a sample of a launch). */
int orc_trace_list(const orc_scene* sc, int32_t src, const uint64_t* photon, uint64_t count,
                   uint32_t* image, orc_event* events) {
    if (src < 0 || src >= sc->n_src || (count && !photon)) return -1;
    orc_event tmp;
    for (uint64_t i = 0; i < count; ++i) trace_one(sc, src, photon[i], image, events ? &events[i] : &tmp);
    return 0;
}

/* ------------------------------------------------------------------------------------------ */
/* Derivative of each photon's electron position (xe, ye) with respect to the 22 perturbation
 * parameters.  The paper has no derivative; this is the plain limit definition of one: central
 * differences f'(t) ~ D(h) = (f(t + h) - f(t - h)) / 2h, taken at h and h/2 and combined by one
 * Richardson step (4 D(h/2) - D(h)) / 3, whose error is O(h^4).  The photon keeps its random
 * numbers (they are keyed by photon index), and every discrete decision is held fixed: a photon
 * counts only if it is converted (DETECTED or OFF_CHIP) in the nominal trace and in all four
 * perturbed traces of every parameter, with the same deciding surface.  frozen[i] = 1 for such
 * photons and 0 otherwise (their rows are zero).  jac is [count][2][22]. */
int orc_jacobian(const orc_scene* sc, int32_t src, uint64_t begin, uint64_t count,
                 const double* h, double* jac, int32_t* frozen) {
    if (src < 0 || src >= sc->n_src) return -1;
    orc_scene w = *sc;
    static const double off[4] = {1.0, -1.0, 0.5, -0.5};
    for (uint64_t i = 0; i < count; ++i) {
        double* J = jac + i * 2 * ORC_N_THETA;
        memset(J, 0, 2 * ORC_N_THETA * sizeof(double));
        frozen[i] = 0;
        orc_event e0;
        trace_one(sc, src, begin + i, NULL, &e0);
        if (e0.status != ORC_DETECTED && e0.status != ORC_OFF_CHIP) continue;
        int ok = 1;
        for (int j = 0; j < ORC_N_THETA && ok; ++j) {
            double f[4][2];
            for (int m = 0; m < 4; ++m) {
                memcpy(w.theta, sc->theta, sizeof(w.theta));
                w.theta[j] += off[m] * h[j];
                prepare_transforms(&w);
                orc_event e;
                trace_one(&w, src, begin + i, NULL, &e);
                if ((e.status != ORC_DETECTED && e.status != ORC_OFF_CHIP) ||
                    e.surface != e0.surface) {
                    ok = 0;
                    break;
                }
                f[m][0] = e.xe;
                f[m][1] = e.ye;
            }
            if (!ok) break;
            for (int c = 0; c < 2; ++c) {
                double d1 = (f[0][c] - f[1][c]) / (2.0 * h[j]);
                double d2 = (f[2][c] - f[3][c]) / h[j];
                J[c * ORC_N_THETA + j] = (4.0 * d2 - d1) / 3.0;
            }
        }
        if (!ok) {
            memset(J, 0, 2 * ORC_N_THETA * sizeof(double));
            continue;
        }
        frozen[i] = 1;
    }
    return 0;
}

/* ------------------------------------------------------------------------------------------ */
/* Readout chain of a sensor image (section 2.4.3 saturation and bleeding; section 2.5
 * electronic readout).  Random numbers: Philox keyed (seed, stage) with counter (index low,
 * index high, draw block, 0): stage 1 defects and dark current per pixel, stage 2 hot-column
 * ends per pixel, stage 3 parallel transfers per pixel, stage 4 serial transfers per packet,
 * stage 5 read noise and bit errors per output value.                                          */

static void readout_draw(uint32_t seed, uint32_t stage, uint64_t idx, uint32_t block,
                         double u[4]) {
    uint32_t ctr[4] = {(uint32_t)idx, (uint32_t)(idx >> 32), block, 0u};
    uint32_t key[2] = {seed, stage};
    uint32_t w[4];
    orc_philox(ctr, key, w);
    for (int i = 0; i < 4; ++i) u[i] = orc_u01(w[i]);
}

/* Saturation and bleeding (section 2.4.3): a pixel holds at most w electrons; the excess moves
 * along its row to the closest pixel below full well, never past the implant at the middle of the
 * row; once the half-row is full the rest is removed.  Readings: the pixels of a half-row are
 * treated in index order, each one's excess placed in the closest unfilled pixels in turn (a tie
 * goes toward the row's end, away from the implant); a pixel filled by bleeding does not bleed
 * again.  Pinned: conservation min(total, n w) per half-row, the symmetric spread of one
 * saturated pixel, no pixel above w. */
int orc_bleed(const orc_readout_params* rp, uint32_t* image, int32_t nx, int32_t ny) {
    const uint64_t w = (uint64_t)rp->full_well;
    for (int32_t j = 0; j < ny; ++j) {
        uint32_t* row = image + (size_t)j * nx;
        for (int half = 0; half < 2; ++half) {
            int32_t a = half == 0 ? 0 : nx / 2, b = half == 0 ? nx / 2 : nx;   /* [a, b) */
            for (int32_t p = a; p < b; ++p) {
                if (row[p] <= w) continue;
                uint64_t excess = row[p] - w;
                row[p] = (uint32_t)w;
                int32_t L = p - 1, R = p + 1;
                while (excess > 0) {
                    while (L >= a && row[L] >= w) --L;
                    while (R < b && row[R] >= w) ++R;
                    int has_l = L >= a, has_r = R < b;
                    if (!has_l && !has_r) break;   /* half-row full: the rest is removed */
                    int32_t t;
                    if (has_l && has_r) {
                        int32_t dl = p - L, dr = R - p;
                        if (dl != dr) t = dl < dr ? L : R;
                        else t = half == 0 ? L : R;   /* toward the row's end */
                    } else {
                        t = has_l ? L : R;
                    }
                    uint64_t room = w - row[t];
                    uint64_t put = excess < room ? excess : room;
                    row[t] += (uint32_t)put;
                    excess -= put;
                }
            }
        }
    }
    return 0;
}

/* Delay of one electron in a transfer chain of m transfers with charge transfer efficiency cte
 * (section 2.5): every transfer succeeds with probability cte, a failure leaves the electron in
 * the packet behind, which is read one slot later; the slot delay is the number of failures
 * before m successes, a negative binomial law, drawn by inversion of u (at most 64). */
static int transfer_delay(double u, int64_t m, double eps) {
    double p = pow(1.0 - eps, (double)m), cum = p;
    int f = 0;
    while (!(u < cum) && f < 64) {
        ++f;
        p *= (double)(m + f - 1) / f * eps;
        cum += p;
    }
    return f;
}

/* Segment geometry: segment (ax, ay) covers columns [ax sw, (ax+1) sw) and rows [ay sh, (ay+1) sh);
 * its serial register lies along the device edge (below row 0 for ay = 0, above row ny - 1 for
 * ay = 1) and its amplifier at the segment's low-column end.  Parallel index r = rows from the
 * register, serial index c = columns from the amplifier. */
static void seg_coords(const orc_readout_params* rp, int32_t nx, int32_t ny, int32_t x, int32_t y,
                       int* amp, int32_t* r, int32_t* c) {
    int32_t sw = nx / rp->amp_nx, sh = ny / rp->amp_ny;
    int32_t ax = x / sw, ay = y / sh;
    *amp = ay * rp->amp_nx + ax;
    *c = x - ax * sw;
    *r = ay == 0 ? y : (ny - 1 - y);
}

/* The readout chain after bleeding (section 2.5): (1) dark current, a normal number of electrons
 * with mean and variance rate x exposure, rounded and floored at zero (reading: the paper's
 * "Gaussian error" read as the Poisson-like width sqrt(mean)); hot pixels set to w; dead pixels
 * emptied (after the dark current); hot columns: a fraction of pixels are column ends, and the end
 * and every pixel behind it in the readout chain (farther from the register) are set to w.
 * (2) Parallel transfers: an electron at parallel index r takes r + 1 transfers and lands in slot
 * r + delay; slots at or beyond sh + over_y are lost.  (3) Serial transfers of every slot of the
 * register: an electron at serial index c lands in slot c + delay of c + 1 transfers; beyond
 * sw + over_x lost.  (4) Read noise (a normal of sigma read_noise electrons, reading: the paper's
 * "mean equal to the read noise" is its width), then ADU = e / (G (1 + N e / W)) + B clamped to
 * [0, 65535], then each bit i = floor(ADU / 2^i + sigma_i g_i) mod 2, ADU = sum bit_i 2^i.
 * Pinned: defect and dark statistics, the negative-binomial trail of one pixel, charge
 * conservation, the ideal digitiser floor(e / G + B), the non-linearity closed form, read-noise
 * variance, bit-error independence. */
int orc_readout(const orc_readout_params* rp, const uint32_t* image, int32_t nx, int32_t ny,
                uint16_t* out, double* margin, uint32_t* work, uint32_t* par, uint32_t* ser) {
    if (rp->amp_nx < 1 || rp->amp_ny < 1 || rp->amp_ny > 2 || nx % rp->amp_nx || ny % rp->amp_ny ||
        rp->amp_nx * rp->amp_ny > ORC_MAX_AMPS)
        return -1;
    const int32_t sw = nx / rp->amp_nx, sh = ny / rp->amp_ny;
    const int32_t ph = sh + rp->over_y, pw = sw + rp->over_x;
    const int n_amp = rp->amp_nx * rp->amp_ny;
    const double w = rp->full_well;
    size_t n = (size_t)nx * ny;
    /* (1) bleeding, dark current, defects */
    memcpy(work, image, n * sizeof(uint32_t));
    orc_bleed(rp, work, nx, ny);
    double mu = rp->dark_rate * rp->exposure;
    for (int32_t y = 0; y < ny; ++y)
        for (int32_t x = 0; x < nx; ++x) {
            uint64_t i = (uint64_t)y * nx + x;
            double u[4];
            readout_draw(rp->seed, 1, i, 0, u);
            uint64_t e = work[i];
            if (mu > 0.0) {
                double g = sqrt(-2.0 * log(u[2])) * cos(TWO_PI * u[3]);
                double d = floor(mu + sqrt(mu) * g + 0.5);
                if (d > 0.0) e += (uint64_t)d;
            }
            if (u[0] < rp->hot_fraction) e = (uint64_t)w;
            else if (u[0] < rp->hot_fraction + rp->dead_fraction) e = 0;
            work[i] = (uint32_t)(e > 0xffffffffull ? 0xffffffffull : e);
        }
    if (rp->hot_column_fraction > 0.0) {
        for (int32_t x = 0; x < nx; ++x)
            for (int half = 0; half < rp->amp_ny; ++half) {
                /* walk the column segment away from its register */
                int hot = 0;
                for (int32_t r = 0; r < sh; ++r) {
                    int32_t y = half == 0 ? r : ny - 1 - r;
                    uint64_t i = (uint64_t)y * nx + x;
                    double u[4];
                    readout_draw(rp->seed, 2, i, 0, u);
                    if (u[0] < rp->hot_column_fraction) hot = 1;
                    if (hot) work[i] = (uint32_t)w;
                }
            }
    }
    /* (2) parallel transfers */
    memset(par, 0, (size_t)n_amp * ph * sw * sizeof(uint32_t));
    double ep = 1.0 - rp->cte_parallel, es = 1.0 - rp->cte_serial;
    for (int32_t y = 0; y < ny; ++y)
        for (int32_t x = 0; x < nx; ++x) {
            uint64_t i = (uint64_t)y * nx + x;
            int amp;
            int32_t r, c;
            seg_coords(rp, nx, ny, x, y, &amp, &r, &c);
            uint32_t* col = par + (size_t)amp * ph * sw + c;
            uint32_t ne = work[i];
            double u[4];
            for (uint32_t e = 0; e < ne; ++e) {
                if ((e & 3) == 0) readout_draw(rp->seed, 3, i, e >> 2, u);
                int64_t s = r + (ep > 0.0 ? transfer_delay(u[e & 3], r + 1, ep) : 0);
                if (s < ph) col[(size_t)s * sw] += 1;
            }
        }
    /* (3) serial transfers */
    memset(ser, 0, (size_t)n_amp * ph * pw * sizeof(uint32_t));
    for (int amp = 0; amp < n_amp; ++amp)
        for (int32_t s = 0; s < ph; ++s)
            for (int32_t c = 0; c < sw; ++c) {
                uint64_t i = ((uint64_t)amp * ph + s) * sw + c;
                uint32_t ne = par[i];
                uint32_t* row = ser + ((size_t)amp * ph + s) * pw;
                double u[4];
                for (uint32_t e = 0; e < ne; ++e) {
                    if ((e & 3) == 0) readout_draw(rp->seed, 4, i, e >> 2, u);
                    int64_t t = c + (es > 0.0 ? transfer_delay(u[e & 3], c + 1, es) : 0);
                    if (t < pw) row[t] += 1;
                }
            }
    /* (4) read noise and digitisation */
    int any_bit = 0;
    for (int b = 0; b < 16; ++b) any_bit |= rp->bit_sigma[b] > 0.0;
    for (int amp = 0; amp < n_amp; ++amp)
        for (int32_t s = 0; s < ph; ++s)
            for (int32_t c = 0; c < pw; ++c) {
                uint64_t i = ((uint64_t)amp * ph + s) * pw + c;
                double u[4];
                readout_draw(rp->seed, 5, i, 0, u);
                double e = (double)ser[i];
                e += rp->read_noise[amp] * sqrt(-2.0 * log(u[0])) * cos(TWO_PI * u[1]);
                double adu = e / (rp->gain[amp] * (1.0 + rp->nonlinearity * e / w)) + rp->bias[amp];
                if (adu < 0.0) adu = 0.0;
                if (adu > 65535.0) adu = 65535.0;
                double m = 1e300;
                uint32_t val = 0;
                double gb[16] = {0};
                if (any_bit)
                    for (int k = 0; k < 4; ++k) {
                        double v[4];
                        readout_draw(rp->seed, 5, i, 1 + k, v);
                        double r0 = sqrt(-2.0 * log(v[0])), r1 = sqrt(-2.0 * log(v[2]));
                        gb[4 * k + 0] = r0 * cos(TWO_PI * v[1]);
                        gb[4 * k + 1] = r0 * sin(TWO_PI * v[1]);
                        gb[4 * k + 2] = r1 * cos(TWO_PI * v[3]);
                        gb[4 * k + 3] = r1 * sin(TWO_PI * v[3]);
                    }
                for (int b = 0; b < 16; ++b) {
                    double a = adu / (double)(1u << b) + rp->bit_sigma[b] * gb[b];
                    double f = floor(a);
                    double dist = a - f < 1.0 - (a - f) ? a - f : 1.0 - (a - f);
                    if (dist < m) m = dist;
                    int64_t k = (int64_t)f;
                    if (((k % 2) + 2) % 2) val |= 1u << b;
                }
                out[i] = (uint16_t)val;
                if (margin) margin[i] = m;
            }
    return 0;
}
