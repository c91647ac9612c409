/*
 * Photon Monte Carlo oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, double-precision CPU implementation of the per-photon trace of Peterson et al.,
 * "Simulation of astronomical images from optical survey telescopes using a comprehensive photon
 * Monte Carlo approach" (the PhoSim paper): sky photon sampling (section 2.2), frozen-flow screen
 * deflection (section 2.3.1-2.3.2), optics (section 2.4.1-2.4.2), silicon conversion and diffusion
 * (section 2.4.2-2.4.3), pixel binning.  It exists to check the GPU implementation: only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may load it.  It shares no code with
 * the GPU library.
 *
 * Parity status per function is listed in phx_oracle.c next to each function.
 */
#ifndef PHX_ORACLE_H
#define PHX_ORACLE_H
#include <stdint.h>

#define ORC_MAX_SURF 16
#define ORC_MAX_LAYERS 8
#define ORC_MAX_SCALES 4
#define ORC_N_THETA 22

enum { ORC_MIRROR = 0, ORC_REFRACT = 1, ORC_DETECTOR = 2 };
enum { ORC_VACUUM = 0, ORC_GLASS = 1, ORC_SILICON = 2 };
enum { ORC_ATMOSPHERE = 1, ORC_COATINGS = 2, ORC_SILICON_PHYS = 4, ORC_DIFFUSION = 8,
       ORC_AEROSOL = 16, ORC_DISPERSION = 32, ORC_DOME = 64, ORC_HALO = 128,
       ORC_SPIDER = 2048, ORC_DEAD_LAYER = 4096, ORC_SECOND_KICK = 8192,
       ORC_FIELD_DIFFUSION = 16384, ORC_GHOSTS = 32768 };
enum {
    ORC_DETECTED = 0, ORC_OFF_CHIP = 1, ORC_VIGNETTED = 2, ORC_ABSORBED = 3, ORC_MISSED = 4,
    ORC_NONCONV = 5, ORC_TIR = 6, ORC_ESCAPED = 7, ORC_OBSCURED = 8,
    ORC_EXTINCT = 10, ORC_DEAD = 11
};

typedef struct {
    int32_t kind, medium, coating, group;
    double z, c, kappa;
    double alpha[8]; /* alpha_3 .. alpha_10 */
    double r_in, r_out;
} orc_surface;

typedef struct {
    double xi, eta;
    int32_t kind, sed;
    double lam_lo, lam_hi, redshift;
    double sersic_n, sersic_bn, sersic_a, sersic_b, sersic_pa;
    uint64_t n_photons;
} orc_source;

/* Per-photon physics beyond the core path (sections 2.3.2, 2.3.3, 2.4.1, 2.4.2); angles in radians,
 * lengths in metres.  Each part is used only when its physics bit is set. */
typedef struct {
    double zenith, zenith_pa;          /* zenith angle; refraction moves (n_x, n_y) along
                                          (cos zenith_pa, sin zenith_pa)                     */
    double tau0, gamma;                /* aerosol: tau = tau0 (lambda / 500 nm)^gamma        */
    double pressure, water, temperature; /* mmHg, mmHg, deg C                                */
    double lam0;                       /* wavelength whose refraction is taken out           */
    double dome_sigma;                 /* dome seeing: Gaussian kick per axis                */
    double halo_f, halo_n, halo_r0, halo_max; /* micro-roughness halo                        */
    double dead;                       /* field-free layer at the silicon entrance surface   */
    int32_t vanes, pad;                /* spider: vanes at vane_angle + 2 pi k / vanes       */
    double vane_angle, vane_width, vane_r_in, vane_r_out, vane_z_lo, vane_z_hi;
    /* hybrid atmosphere: second kick of the modes above kappa_crit (up to kappa_max) */
    double kick_r0, kick_L0, kick_kappa_crit, kick_kappa_max;
    double kick_fraction[ORC_MAX_LAYERS];
    /* silicon field model of the diffusion: overdepletion voltage, doping (bulk, back-surface and
     * front-surface exponentials, m^-3 and m), collection height above the front surface */
    double si_voltage, si_n_bulk, si_n_back, si_s_back, si_n_front, si_s_front, si_z_collect;
} orc_extra;

typedef struct {
    /* optics */
    int32_t n_surf;
    int32_t physics;
    orc_surface surf[ORC_MAX_SURF];
    double pupil_r_in, pupil_r_out, pupil_margin;
    double z_start, obsc_z, obsc_r;
    double glass_b[3], glass_c[3];
    double chip_x0, chip_y0, pixel;
    int32_t nx, ny;
    double t_si, temp_k, sigma_max;
    double theta[ORC_N_THETA];
    double pivot[3][3];
    double zernike_r;
    /* coatings */
    int32_t n_coat, n_s, n_lam, pad0;
    double s_max, lam0, dlam;
    const float* coat;
    const float* coat_r;   /* reflectance on the same grid (ghosts); may be NULL */
    /* atmosphere */
    int32_t n_layers, n_scales, screen_n, pad1;
    double height[ORC_MAX_LAYERS];
    double wind[ORC_MAX_LAYERS][2];
    double pix[ORC_MAX_SCALES];
    double lambda_ref;
    const float* opd;   /* [L][S][N][N] metres */
    /* sources and SEDs */
    int32_t n_src, n_sed, sed_k, pad2;
    const orc_source* src;
    const double* sed_edges; /* [sed_k + 1] */
    const double* sed_flux;  /* [n_sed][sed_k] */
    uint32_t seed;
    int32_t pad3;
    double exposure;
    orc_extra ex;
    /* derived by orc_prepare (owned by the oracle) */
    float* grad;        /* [L][S][N][N][2] */
    double* sed_cdf;    /* [n_sed][sed_k + 1] */
    double rot[ORC_MAX_SURF][3][3];
    double trans[ORC_MAX_SURF][3];
} orc_scene;

typedef struct {
    uint64_t photon;
    int32_t source, status, surface, pix_i, pix_j, newton;
    double x, y, z;       /* last position, in the frame of the deciding surface */
    double xe, ye;        /* electron position on the detector (detector frame) */
    double lambda;
    double margin;        /* smallest normalised distance of any decision from its threshold */
    double t, px, py;     /* time stamp and pupil sample */
    double cond;          /* conditioning of the path after the spider: the turn per metre of
                           * edge distance of its edge diffraction (rad/m), 0 without one */
} orc_event;

int  orc_prepare(orc_scene* sc);
void orc_release(orc_scene* sc);
/* Trace photons [begin, begin+count) of source `src`; events may be NULL; image may be NULL. */
int  orc_trace(const orc_scene* sc, int32_t src, uint64_t begin, uint64_t count,
               uint32_t* image, orc_event* events);
/* Photons photon[0 .. count) of source src (any indices, in the given order); events[i] for
 * photon[i].  Returns 0, or -1 for a bad source or a null list. */
int  orc_trace_list(const orc_scene* sc, int32_t src, const uint64_t* photon, uint64_t count,
                    uint32_t* image, orc_event* events);
/* d(xe, ye)/d(theta) of photons [begin, begin+count) by Richardson-extrapolated central
 * differences with frozen decisions; jac [count][2][22], frozen [count]. */
int  orc_jacobian(const orc_scene* sc, int32_t src, uint64_t begin, uint64_t count,
                  const double* h, double* jac, int32_t* frozen);
/* Primitives exported for the pin tests. */
void   orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double orc_u01(uint32_t w);
double orc_rajkanan(double lambda_m, double temp_k);
double orc_n_silicon(double lambda_m);
double orc_sellmeier(const orc_scene* sc, double lambda_m);
double orc_zernike(int j, double u, double v);
void   orc_zernike_grad(int j, double u, double v, double* du, double* dv);
int    orc_intersect(const orc_scene* sc, int k, const double q[3], const double d[3],
                     double* l_out, int* iters);
double orc_sag(const orc_scene* sc, int k, double x, double y, double* sx, double* sy);
double orc_coating(const orc_scene* sc, int coat, double s, double lambda_m);
void   orc_screen_gradient(const orc_scene* sc, int layer, int scale, double x, double y,
                           double* gx, double* gy);
int    orc_gamma(uint32_t seed, int32_t src, uint64_t photon, double shape, double* out);
double orc_air_refractivity(double lambda_m, double pressure, double temperature, double water);
/* Second kick of one layer: phase variance of its high-frequency modes, and the kick (angle at
 * the reference wavelength) photon `photon` receives at layer `layer`; returns the number of
 * scatterings. */
double orc_kick_variance(const orc_scene* sc, int layer);
int    orc_second_kick(const orc_scene* sc, int32_t src, uint64_t photon, int layer,
                       double* kx, double* ky);
/* Field model of the charge diffusion: E_z (V/m) at height z above the front surface, electron
 * mobility (m^2/Vs) at field E (V/m) and temperature T, and the diffusion sigma (m) of an
 * electron converted at `depth` below the entrance (back) surface. */
double orc_field(const orc_scene* sc, double z);
double orc_mobility(double E, double T);
double orc_field_sigma(const orc_scene* sc, double depth);
/* Readout chain of a sensor image (sections 2.4.3 saturation and bleeding, 2.5 electronic
 * readout).  Segments: amp_nx x amp_ny amplifiers (amp_ny 1 or 2); out [amp][sh + over_y]
 * [sw + over_x] in readout order; margin (may be NULL) per output value: the smallest distance
 * of a floor() argument of the digitisation from an integer. */
#define ORC_MAX_AMPS 32
typedef struct {
    uint32_t seed;
    int32_t amp_nx, amp_ny, over_x, over_y, pad;
    double full_well, exposure, dark_rate;
    double hot_fraction, dead_fraction, hot_column_fraction;
    double cte_parallel, cte_serial, nonlinearity;
    double gain[ORC_MAX_AMPS], bias[ORC_MAX_AMPS], read_noise[ORC_MAX_AMPS];
    double bit_sigma[16];
} orc_readout_params;
int    orc_bleed(const orc_readout_params* rp, uint32_t* image, int32_t nx, int32_t ny);
int    orc_readout(const orc_readout_params* rp, const uint32_t* image, int32_t nx, int32_t ny,
                   uint16_t* out, double* margin, uint32_t* stage_work, uint32_t* stage_par,
                   uint32_t* stage_ser);
int    orc_halo_sample(uint32_t seed, int32_t src, uint64_t photon, double n, double x_max,
                       double* x_out);
#endif
