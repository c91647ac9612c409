/*
 * phx -- photon Monte Carlo trace on AMD Instinct MI355X (gfx950).
 *
 * C ABI of the per-photon trace of the photon Monte Carlo image simulator described by
 * Peterson et al., "Simulation of Astronomical Images from Optical Survey Telescopes using a
 * Comprehensive Photon Monte Carlo Approach" (ApJS 218:14, 2015):
 *
 *   sky photon sampling                                    (section 2.2, 2.2.1)
 *   -> frozen-flow phase-screen deflection, layer by layer (sections 2.3.1, 2.3.2)
 *   -> conic + polynomial-asphere surfaces: Newton intersection, reflection, refraction with
 *      Sellmeier / silicon indices, coating-transmission roulette  (sections 2.4.1, 2.4.2)
 *   -> silicon conversion at an exponentially distributed depth, charge diffusion, pixel binning
 *                                                          (sections 2.4.2, 2.4.3)
 *
 * Conventions shared by every entry point:
 *   - Return value: PHX_OK (0) or a negative phx_status.  On error the context's message
 *     (phx_last_error) says what was wrong; nothing is enqueued.  Errors never abort the process.
 *   - Pointers named *_host are host memory, read during the call only.  Pointers named *_dev are
 *     device memory on the context's GPU, owned by the caller; the library never frees them.
 *     Output buffers are accumulated into, never cleared.
 *   - Work is enqueued asynchronously on the given HIP stream (NULL = the legacy default stream);
 *     caller-owned device buffers must stay valid until that stream has completed the work.
 *   - A context belongs to one device and must not be used from two threads at once.
 *   - Per-photon anomalies (no intersection, Newton non-convergence, total internal reflection)
 *     are outcomes counted in the statistics buffer, not errors.
 *
 * Units: metres, seconds, radians.  Global frame: z towards the sky, photons arrive travelling
 * towards -z, the first surface's vertex at the origin.
 */
#ifndef PHX_H
#define PHX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t phx_status;
enum {
    PHX_OK = 0,
    PHX_ERR_INVALID = -1,   /* bad argument: null pointer, size, NaN, out-of-range value */
    PHX_ERR_STATE = -2,     /* a required load (prescription, sources, screens) is missing */
    PHX_ERR_HIP = -3,       /* a HIP runtime call failed; message holds hipGetErrorString */
    PHX_ERR_NOMEM = -4,     /* device or host allocation failed */
    PHX_ERR_CAPACITY = -5   /* an output buffer is too small for the request */
};

#define PHX_MAX_SURF 16
#define PHX_MAX_LAYERS 8
#define PHX_MAX_SCALES 4
#define PHX_N_THETA 22
#define PHX_N_STATUS 12

/* Surface kinds and media (section 2.4.1: mirrors have one surface, lenses two; the detector
 * is an optical surface like a lens surface). */
enum { PHX_MIRROR = 0, PHX_REFRACT = 1, PHX_DETECTOR = 2 };
enum { PHX_VACUUM = 0, PHX_GLASS = 1, PHX_SILICON = 2 };

/* Photon fates.  The statistics buffer counts them per (status, surface). */
enum {
    PHX_DETECTED = 0,   /* converted in silicon and binned on the chip            */
    PHX_OFF_CHIP = 1,   /* reached the focal plane outside the chip's pixels      */
    PHX_VIGNETTED = 2,  /* outside a surface's clear aperture                      */
    PHX_ABSORBED = 3,   /* lost to a coating (transmission roulette)               */
    PHX_MISSED = 4,     /* ray does not meet the surface                           */
    PHX_NONCONV = 5,    /* intersection iteration did not converge                 */
    PHX_TIR = 6,        /* total internal reflection at a refracting surface       */
    PHX_ESCAPED = 7,    /* crossed the silicon without converting                  */
    PHX_OBSCURED = 8,   /* blocked by the central obscuration                      */
    PHX_CULLED = 9,     /* removed before tracing by the transmission pre-roll     */
    PHX_EXTINCT = 10,   /* destroyed by aerosol opacity (PHX_F_AEROSOL)            */
    PHX_DEAD = 11       /* converted in the field-free dead layer (PHX_F_DEAD_LAYER) */
};

/* Physics and execution flags (phx_trace_args.flags). */
enum {
    PHX_F_ATMOSPHERE = 1u << 0, /* screen deflections (needs phx_load_screens)             */
    PHX_F_COATINGS = 1u << 1,   /* coating roulette (needs phx_load_coatings)              */
    PHX_F_SILICON = 1u << 2,    /* refraction into silicon, conversion depth, escape       */
    PHX_F_DIFFUSION = 1u << 3,  /* Gaussian charge diffusion                               */
    /* Per-photon physics beyond the core path; each needs phx_load_physics.  With PHX_F_DOME,
       PHX_F_HALO or PHX_F_SPIDER the pre-roll keeps every pupil sample (the kicks at the
       telescope entrance have no bound on the displacement at the primary). */
    PHX_F_AEROSOL = 1u << 4,    /* aerosol extinction (section 2.3.3)                      */
    PHX_F_DISPERSION = 1u << 5, /* atmospheric dispersion (section 2.3.3)                  */
    PHX_F_DOME = 1u << 6,       /* dome seeing (section 2.4.2)                             */
    PHX_F_HALO = 1u << 7,       /* micro-roughness halo (section 2.4.2)                    */
    PHX_F_SPIDER = 1u << 11,    /* spider shadow and edge diffraction (2.4.1-2.4.2)        */
    PHX_F_DEAD_LAYER = 1u << 12,/* field-free dead layer (section 2.4.2; needs SILICON)    */
    PHX_F_SECOND_KICK = 1u << 13,/* hybrid atmosphere: second kick per layer (2.3.2; needs
                                   ATMOSPHERE; the pre-roll then keeps every pupil sample)   */
    PHX_F_FIELD_DIFFUSION = 1u << 14,/* diffusion width from the silicon field model (2.4.3;
                                   with DIFFUSION, in place of sigma_max x drift fraction)   */
    PHX_F_GHOSTS = 1u << 15,    /* ghost reflections (section 2.4.2; needs COATINGS and
                                   phx_load_reflectance): a filter or anti-reflection coating
                                   that does not transmit reflects with probability R; the
                                   photon then propagates backwards, its next surface being the
                                   nearest one ahead among all surfaces (at most 16
                                   interactions, stream 4 block i for interaction i), crossing
                                   into the medium on the other side of each surface it passes;
                                   the pre-roll tests only the coated surfaces ahead of the
                                   first coated refracting one; the context then holds a list of
                                   112 bytes per photon of a chunk (7.5 GB for chunks of 2^26);
                                   phx_adjoint and phx_trace_noalloc refuse it */
    PHX_F_CULL = 1u << 8,       /* pre-roll: skip photons whose roulette draws exceed the
                                   worst-case transmission of any coated surface (section 3.2,
                                   dynamic transmission optimisation), pupil samples whose
                                   radius lies farther outside the primary's clear annulus than
                                   the largest atmospheric displacement, and (flat silicon
                                   detector) photons whose conversion distance times the smallest
                                   refracted cosine exceeds the silicon thickness; images and
                                   moments are unchanged, culled photons are counted as
                                   PHX_CULLED */
    PHX_F_EVENTS = 1u << 9,     /* write per-photon records for sampled photons            */
    PHX_F_MOMENTS = 1u << 10    /* accumulate per-source moments of converted photons      */
};

typedef struct phx_ctx_s* phx_ctx;

/* One optical surface (section 2.4.1 surface equation; paper Table 1 rows "optic type",
 * "radius of curvature", "position", "outer/inner radius", "conic constant", "aspheric
 * coefficients", "medium"):
 *   z = z_vertex + c r^2 / (1 + sqrt(1 - (1 + kappa) c^2 r^2)) + sum_{i=3..10} alpha[i-3] r^i.
 * medium is the medium the photon enters at this surface; coating is a table index or -1;
 * group is the rigid-body perturbation group (0 none, 1 = theta[0..4], 2 = theta[5..9]). */
typedef struct {
    int32_t kind, medium, coating, group;
    double z_vertex, curvature, conic;
    double alpha[8];
    double r_inner, r_outer;
} phx_surface;

/* Optical prescription + focal plane (paper Table 1).  Surfaces are in travel order; the last
 * one must be the detector.  The chip is a rectangular device of nx x ny square pixels whose
 * pixel (0,0) starts at (chip_x0, chip_y0) in the detector's frame (section 2.4.1); nx, ny are at
 * most 32767. */
typedef struct {
    int32_t n_surfaces, nx, ny, pad;
    phx_surface surf[PHX_MAX_SURF];
    double pupil_r_inner, pupil_r_outer;  /* sampling annulus on the first surface (section 2.2) */
    double z_start;                       /* plane above every optic where the optics trace starts */
    double obscuration_z, obscuration_r;  /* central obscuration disk (r = 0: none) */
    double sellmeier_b[3], sellmeier_c[3];/* glass: n^2 = 1 + sum B l^2/(l^2 - C), l in um */
    double chip_x0, chip_y0, pixel;
    double si_thickness, si_temperature, sigma_max; /* silicon (sections 2.4.2-2.4.3) */
    double group_pivot[3][3];             /* rotation pivots of perturbation groups 0..2 */
} phx_prescription;

/* Turbulence layers (section 2.3.1): heights above the first surface's vertex, wind vectors,
 * screen pixel sizes per nested scale (coarse to fine), screen side, reference wavelength of
 * the (lambda/lambda_ref)^(-1/5) kick scaling (section 2.3.2). */
typedef struct {
    int32_t n_layers, n_scales, screen_n, pad;
    double height[PHX_MAX_LAYERS];
    double wind[PHX_MAX_LAYERS][2];
    double pixel[PHX_MAX_SCALES];
    double lambda_ref;
} phx_atmosphere;

/* A source (section 2.2): nominal direction n_x = xi, n_y = eta, n_z = -sqrt(1-xi^2-eta^2).
 * kind 0 point, 1 ellipsoidal Sersic (section 2.2.1: index n, b_n, semi-axis scales a >= b in
 * radians, position angle).  sed = -1: photon spectrum flat on [lambda_lo, lambda_hi]; sed >= 0:
 * row of the tabulated SEDs.  Wavelengths are multiplied by (1 + redshift). */
typedef struct {
    double xi, eta;
    int32_t kind, sed;
    double lambda_lo, lambda_hi, redshift;
    double sersic_n, sersic_bn, sersic_a, sersic_b, sersic_pa;
    uint64_t n_photons;
} phx_source;

/* Parameters of the per-photon physics beyond the core path.  Angles in radians, lengths in
 * metres, all in the global frame of the prescription.  Random numbers: Philox block 7 (aerosol,
 * halo selection, halo azimuth, spider sign), block 8 (dome-seeing normal pair), stream 2 block t
 * (halo rejection trial t).
 *  - Aerosol (section 2.3.3): a photon survives with probability exp(-tau sec z),
 *    tau = tau0 (lambda / 500 nm)^gamma; else PHX_EXTINCT at the start plane.
 *  - Dispersion (section 2.3.3): the source direction moves by (R(lambda) - R(lambda0)) along
 *    (cos zenith_pa, sin zenith_pa) in (n_x, n_y), R = (n_air - 1) tan z with the Filippenko
 *    index of air at pressure, water-vapour pressure (mmHg) and temperature (deg C), the water
 *    term taken as a product with W.
 *  - Dome seeing (section 2.4.2): a normal kick of standard deviation dome_sigma per axis added
 *    to (n_x, n_y) on the start plane.
 *  - Halo (section 2.4.2): with probability halo_fraction, a kick of angle r0 x toward a uniform
 *    azimuth, x with density proportional to x / (1 + x^n) on [0, halo_max / r0]
 *    (2 < n <= 6), drawn by rejection (at most 32 trials, then no kick).
 *  - Spider (section 2.4.1 rectangular volumes, 2.4.2 edge diffraction): spider_vanes boxes
 *    (at most 8), vane k along azimuth spider_angle + 2 pi k / spider_vanes, spanning radii
 *    [r_inner, r_outer], width spider_width across and heights [z_low, z_high] (z_high at most
 *    the start plane).  A ray that meets a box is PHX_OBSCURED; any other turns, at the vanes'
 *    mid-height, by lambda / (4 pi max(d, lambda)) across the nearest vane (sign from its random
 *    word), d = the closest distance between the ray and a long edge of a vane.
 *  - Dead layer (section 2.4.2): an electron converted less than dead_layer below the surface the
 *    light enters is removed (PHX_DEAD).
 *  - Second kick (section 2.3.2, hybrid two-kick atmosphere): the screens carry the modes below
 *    kick_kappa_crit (rad/m); at layer i the modes above it deflect the photon by a draw from
 *    their long-exposure PSF, the Fourier transform of exp(-D(rho)/2): K ~ Poisson(s2_i)
 *    scatterings (at most 8), each lambda_ref kappa / (2 pi) toward a uniform azimuth with kappa
 *    from the phase spectrum 0.033 (2 pi) / 0.423 r0_i^(-5/3) (kappa^2 + (2 pi / L0)^2)^(-11/6)
 *    on [kappa_crit, kappa_max], r0_i = kick_fraction[i]^(-3/5) kick_r0 (at lambda_ref), s2_i its
 *    integral; the sum is added to the layer's refractive kick and scaled with it by
 *    (lambda / lambda_ref)^(-1/5).  Random numbers: block 9 + i/4 word i%4 (count), stream 3
 *    block 8 i + j (scattering j: wavenumber, azimuth).
 *  - Field diffusion (section 2.4.3): an electron converted at height z above the front
 *    (collecting) surface of the back-illuminated device spreads with sigma = sqrt(2 D t_c),
 *    D = mu(E(z), T) k T / q, t_c = int_{z_collect}^{z} dz' / |mu E|, with
 *    E_z(z) = si_voltage / t_Si + q / (eps0 11.7) int_{t_Si}^{z} n_d, n_d = si_n_bulk +
 *    si_n_back exp(-(t_Si - z)/si_s_back) + si_n_front exp(-z/si_s_front) (m^-3, m) and the
 *    velocity-saturation mobility mu = (v_m/E_c) / (1 + (E/E_c)^beta)^(1/beta), v_m = 1.53e9
 *    T^-0.87 cm/s, E_c = 1.01 T^1.55 V/cm, beta = 2.57e-2 T^0.66; no spread at or below
 *    z_collect.  The library tabulates sigma^2 against depth (131073 points) when the
 *    parameters are loaded (and again when a prescription is loaded after them); a trace with
 *    PHX_F_FIELD_DIFFUSION fails with PHX_ERR_INVALID if E_z is not positive across the device. */
typedef struct {
    double zenith_angle, zenith_pa;
    double aerosol_tau0, aerosol_gamma;
    double air_pressure, air_water, air_temperature;
    double dispersion_lambda0;
    double dome_sigma;
    double halo_fraction, halo_index, halo_r0, halo_max;
    double dead_layer;
    int32_t spider_vanes, pad;
    double spider_angle, spider_width, spider_r_inner, spider_r_outer;
    double spider_z_low, spider_z_high;
    double kick_r0, kick_L0, kick_kappa_crit, kick_kappa_max;
    double kick_fraction[PHX_MAX_LAYERS];
    double si_voltage, si_n_bulk, si_n_back, si_s_back, si_n_front, si_s_front, si_z_collect;
} phx_physics;

/* Per-photon record written for sampled photons (PHX_F_EVENTS). */
typedef struct {
    uint64_t photon;
    int32_t source, status, surface, pix_i, pix_j, newton;
    double x, y, z;    /* last position, in the frame of the deciding surface (detector frame
                          for photons that reached the detector)                             */
    double xe, ye;     /* electron position in the detector frame (after diffusion)         */
    double lambda;
} phx_event;

/* Statistics buffer layout (uint64): counts[status][surface + 1] for status < PHX_N_STATUS and
 * surface in -1..PHX_MAX_SURF-1 (column 0 = before any surface), followed by PHX_STAT_NEWTON
 * (total Newton iterations) and PHX_STAT_TRACED (photons traced past the pre-roll). */
#define PHX_STAT_COLS (PHX_MAX_SURF + 1)
#define PHX_STAT_NEWTON (PHX_N_STATUS * PHX_STAT_COLS)
#define PHX_STAT_TRACED (PHX_STAT_NEWTON + 1)
#define PHX_STATS_LEN (PHX_STAT_TRACED + 1)

/* Moments buffer layout (uint64 words): per source PHX_MOMENT_WORDS words holding exact sums
 * over the photons that converted in silicon (status DETECTED or OFF_CHIP) of their electron
 * position (x, y) in the detector frame, quantised to X = round(x * 2^PHX_MOMENT_Q_LOG2),
 * Y likewise (round half to even; requires |x|, |y| < 1 m):
 *   word 0        n (number of converted photons), word 1 zero,
 *   words 2-3     sum X      words 4-5   sum Y      words 6-7   sum X^2
 *   words 8-9     sum Y^2    words 10-11 sum X Y
 * each sum a two's-complement 128-bit integer, low word first.  Integer addition is exact and
 * associative, so the words do not depend on launch shape, batching or execution order. */
#define PHX_MOMENT_WORDS 12
#define PHX_MOMENT_Q_LOG2 44

typedef struct {
    uint32_t seed;          /* Philox key word 0 (key word 1 = source index)                  */
    uint32_t flags;         /* PHX_F_* */
    int32_t src_begin;      /* sources [src_begin, src_end) of the loaded catalogue           */
    int32_t src_end;
    uint64_t photon_begin;  /* first photon index traced for every source                      */
    uint64_t photon_count;  /* photons per source; 0 = each source's n_photons                 */
    double exposure;        /* t_e (section 2.2 time stamp t = t_e u)                          */
    double pupil_margin;    /* annulus enlargement (section 2.2: slightly larger aperture)      */
    uint32_t* image_dev;    /* [ny][nx], accumulated (+1 per detected photon); required        */
    uint64_t* stats_dev;    /* [PHX_STATS_LEN], accumulated; may be NULL                        */
    uint64_t* moments_dev;  /* [n_sources][PHX_MOMENT_WORDS], accumulated; NULL unless MOMENTS */
    phx_event* events_dev;  /* NULL unless EVENTS                                               */
    uint64_t event_stride;  /* photon g of the launch (sources concatenated in order, photons
                               in index order) is recorded at slot g / stride iff g % stride == 0 */
    uint64_t event_capacity;/* slots available; PHX_ERR_CAPACITY if too small                   */
} phx_trace_args;

/* Library version string (static storage). */
const char* phx_version(void);

/* Create a context on HIP device `device`.  *out receives the handle.  Allocates the context's
 * small device tables.  Errors: PHX_ERR_INVALID (null out, bad device), PHX_ERR_HIP. */
phx_status phx_create(int32_t device, phx_ctx* out);

/* Free the context and every device buffer it owns.  NULL is ignored.  Synchronises the device. */
void phx_destroy(phx_ctx ctx);

/* Message of the last failed call on ctx (context-owned, valid until the next call). */
const char* phx_last_error(phx_ctx ctx);

/* Load the optical prescription (section 2.4.1, paper Table 1), copied from host memory.
 * Validates surface count (1..PHX_MAX_SURF, last = detector), finite values, apertures,
 * chip size.  Keeps the current perturbation.  Errors: PHX_ERR_INVALID. */
phx_status phx_load_prescription(phx_ctx ctx, const phx_prescription* p_host);

/* Set the misalignment/deformation vector (section 2.4.1: decenter, defocus and rotations per
 * rigid group; Zernike deformation of the first surface):
 *   theta[0..4]  group 1: dx, dy, tilt_x, tilt_y, dz      theta[5..9] group 2: same
 *   theta[10..21] Noll Z4..Z15 amplitudes (m) on surface 0, normalised to its outer radius.
 * A group is rotated by R = R_x(tilt_x) R_y(tilt_y) about its pivot, then translated.
 * n must be PHX_N_THETA.  Takes effect for work enqueued afterwards.  Errors: PHX_ERR_INVALID. */
phx_status phx_set_perturbation(phx_ctx ctx, const double* theta_host, int32_t n);

/* Load coating tables (section 2.4.2 transmission probability vs angle and wavelength):
 * float32 [n_coat][n_s][n_lambda], transmission on a uniform grid of s = sin^2(incidence angle)
 * from 0 to s_max and wavelength lambda0 + k dlambda (2 <= n_lambda <= 8192).  Copied to device
 * memory.
 * Errors: PHX_ERR_INVALID, PHX_ERR_NOMEM, PHX_ERR_HIP. */
phx_status phx_load_coatings(phx_ctx ctx, const float* tables_host, int32_t n_coat, int32_t n_s,
                             int32_t n_lambda, double s_max, double lambda0, double dlambda);

/* Load the reflection probabilities of the coatings for ghosts (section 2.4.2: the coating
 * description carries reflection and transmission against angle and wavelength): float32
 * [n_coat][n_s][n_lambda] on the grid of the loaded transmission tables (same sizes), with
 * 0 <= R <= 1 - T (+1e-6).  Copied.  Mirrors ignore it (their table is the reflection).
 * Errors: PHX_ERR_INVALID, PHX_ERR_STATE (no coatings loaded), PHX_ERR_NOMEM, PHX_ERR_HIP. */
phx_status phx_load_reflectance(phx_ctx ctx, const float* tables_host, int32_t n_coat,
                                int32_t n_s, int32_t n_lambda);

/* Load turbulence screens (sections 2.3.1-2.3.2).  opd_dev: float32 [L][S][N][N] optical path
 * (m), row j along y, column i along x, periodic; read only by work enqueued on `stream` during
 * this call.  The context derives and owns the gradient screens (centred differences).  A screen
 * holding a NaN or infinite value is refused with PHX_ERR_INVALID, and the context then has no
 * usable screens (PHX_F_ATMOSPHERE fails with PHX_ERR_STATE until a good load).
 * Errors: PHX_ERR_INVALID, PHX_ERR_NOMEM, PHX_ERR_HIP. */
phx_status phx_load_screens(phx_ctx ctx, const phx_atmosphere* atm_host, const float* opd_dev,
                            int64_t n_floats, void* stream);

/* Load the source catalogue (section 2.2) and tabulated SEDs (f_lambda per wavelength bin on the
 * shared grid sed_edges_host[0..sed_k]; flux_host [n_sed][sed_k]).  Both copied; the context
 * builds each SED's photon cumulative distribution (section 2.2: flux / photon energy x bin
 * width) and a search guide for it.  n_sed may be 0; 1 <= sed_k <= 65535.  Errors:
 * PHX_ERR_INVALID, PHX_ERR_NOMEM, PHX_ERR_HIP. */
phx_status phx_load_sources(phx_ctx ctx, const phx_source* src_host, int32_t n_src,
                            const double* sed_edges_host, const double* sed_flux_host,
                            int32_t n_sed, int32_t sed_k);

/* Load the parameters of the per-photon physics beyond the core path (the PHX_F_AEROSOL ..
 * PHX_F_DEAD_LAYER flags; a trace with one of them set before this call fails with
 * PHX_ERR_STATE).  Copied.  Validates 0 <= zenith_angle < pi/2, tau0 >= 0, pressures >= 0,
 * temperature > -273.15, lambda0 > 0.16 um, dome_sigma >= 0, 0 <= halo_fraction <= 1,
 * 2 < halo_index <= 6, 0 < halo_r0, 0 < halo_max < pi/2, dead_layer >= 0, 0 <= spider_vanes <= 8
 * and (with vanes) width > 0, r_inner < r_outer, z_low < z_high <= the prescription's start
 * plane (load the prescription first), kick_r0 > 0, kick_L0 > 0,
 * 0 < kick_kappa_crit < kick_kappa_max, 0 <= kick_fraction[i] with a phase variance of at most 2
 * per layer, si_voltage > 0, doping densities >= 0 with positive depths, 0 <= si_z_collect < t_Si.
 * Errors: PHX_ERR_INVALID, PHX_ERR_STATE, PHX_ERR_NOMEM, PHX_ERR_HIP. */
phx_status phx_load_physics(phx_ctx ctx, const phx_physics* physics_host);

/* Sensor readout chain (section 2.4.3 saturation and bleeding; section 2.5 electronic readout),
 * applied to an image of electrons (for instance the trace's image).  Segments: amp_nx x amp_ny
 * amplifiers (amp_ny 1 or 2, at most PHX_MAX_AMPS, nx % amp_nx == ny % amp_ny == 0); segment
 * (ax, ay) covers columns [ax sw, (ax+1) sw) and rows [ay sh, (ay+1) sh), sw = nx / amp_nx,
 * sh = ny / amp_ny; its serial register lies along the device edge (below row 0 for ay = 0, above
 * row ny - 1 for ay = 1) and its amplifier at the segment's low-column end; a pixel's parallel
 * index r counts rows from the register, its serial index c columns from the amplifier.
 * Steps, in order:
 *  1. bleeding: each half-row (split at column nx / 2, the implant) holds at most full_well per
 *     pixel; treating its pixels in index order, a pixel's excess goes to the closest pixels
 *     below full well (a tie toward the row's end), the rest is removed once the half-row is full;
 *  2. dark current: + max(0, round(mu + sqrt(mu) g)), mu = dark_rate x exposure; hot pixels set
 *     to full_well, dead pixels emptied (Philox key (seed, 1), counter (pixel, 0): word 0 selects,
 *     words 2, 3 the normal); hot columns: a pixel is a hot-column end with probability
 *     hot_column_fraction (key (seed, 2) word 0) and it and every pixel behind it (larger r in its
 *     segment column) are set to full_well;
 *  3. parallel transfers: each electron of a pixel at parallel index r is read in slot
 *     r + F, F the failures before r + 1 successes at probability cte_parallel (negative binomial,
 *     drawn by inversion, at most 64; electron e uses key (seed, 3), counter (pixel, e / 4) word
 *     e % 4); slots >= sh + over_y are lost;
 *  4. serial transfers of every slot row likewise with c + 1 transfers at cte_serial (key
 *     (seed, 4), counter (packet index in the [amp][sh + over_y][sw] layout, e / 4));
 *  5. digitisation per output value: e + read_noise[amp] g (key (seed, 5), counter (index, 0));
 *     ADU = e / (gain (1 + nonlinearity e / full_well)) + bias, clamped to [0, 65535]; bit i =
 *     floor(ADU / 2^i + bit_sigma[i] g_i) mod 2 (g_i from counters (index, 1..4)); the output is
 *     sum bit_i 2^i.
 * electrons_dev: [ny][nx] uint32 (device; read only).  adu_dev: [amp][sh + over_y][sw + over_x]
 * uint16 (device; adu_capacity elements at least).  work_dev [ny][nx], parallel_dev
 * [amp][sh + over_y][sw] and serial_dev [amp][sh + over_y][sw + over_x] (uint32, device) receive
 * the electrons after steps 2, 3 and 4 when not NULL; otherwise context-owned buffers are used
 * (allocated or grown on first use: that call may synchronise the device).  Limits (the transfer
 * stages draw one delay per electron): 1 <= full_well <= 1e7, dark_rate x exposure <= 1e6.
 * Enqueued on `stream`.  Errors: PHX_ERR_INVALID, PHX_ERR_CAPACITY, PHX_ERR_NOMEM, PHX_ERR_HIP. */
#define PHX_MAX_AMPS 32
typedef struct {
    uint32_t seed;
    int32_t amp_nx, amp_ny, over_x, over_y, pad;
    double full_well, exposure, dark_rate;
    double hot_fraction, dead_fraction, hot_column_fraction;
    double cte_parallel, cte_serial, nonlinearity;
    double gain[PHX_MAX_AMPS], bias[PHX_MAX_AMPS], read_noise[PHX_MAX_AMPS];
    double bit_sigma[16];
} phx_readout_params;

phx_status phx_readout(phx_ctx ctx, const phx_readout_params* params_host,
                       const uint32_t* electrons_dev, int32_t nx, int32_t ny, uint16_t* adu_dev,
                       uint64_t adu_capacity, uint32_t* work_dev, uint32_t* parallel_dev,
                       uint32_t* serial_dev, void* stream);

/* Trace photons: for every source s in [src_begin, src_end), photons photon_begin ..
 * photon_begin + count - 1, each keyed by Philox4x32-10 (key = (seed, s), counter = (photon
 * index, block, stream)), so any photon's history is reproducible independently of the launch.
 * Enqueued on `stream`.  Errors: PHX_ERR_INVALID, PHX_ERR_STATE, PHX_ERR_CAPACITY, PHX_ERR_HIP. */
phx_status phx_trace(phx_ctx ctx, const phx_trace_args* args, void* stream);

/* The same trace as phx_trace for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): phx_trace_noalloc calls
 * no hipMalloc or hipFree and creates no stream or event.  Its workspace is a file-scope device
 * array of 40 MiB per GPU (held until the process ends), whose address the library looks up
 * once per device when a context is created; the caller still passes the image, statistics,
 * moments and event buffers.  Photons, results and error behaviour are those of phx_trace with
 * the same arguments (the launch is cut into chunks of at most 2^19 photons, run on `stream`
 * alone).  Limits: at most 65536 sources and 16384 chunks (about 8.6e9 photons); PHX_F_GHOSTS
 * is refused (PHX_ERR_INVALID: the ghost list needs context memory); beyond a limit
 * PHX_ERR_CAPACITY, nothing enqueued.  Every call on one GPU shares that GPU's workspace, so
 * calls that overlap on one GPU (two streams, two threads or two contexts) race: serialise them.
 * The parameter block is uploaded on `stream` when a load changed it (that call synchronises
 * `stream`). */
phx_status phx_trace_noalloc(phx_ctx ctx, const phx_trace_args* args, void* stream);

/* Launch shape of phx_trace / phx_trace_batched / phx_adjoint.  chunk_log2: photons per chunk =
 * 2^chunk_log2 (16..27; the context keeps survivor lists and 56-byte states for two chunks);
 * *_blocks_per_cu: workgroups of 256 lanes per compute unit for the pre-roll, sky+atmosphere and
 * optics kernels (1..64); dynamic_tiles: 0 = static grid-stride, 1 = the sky kernel claims tiles of
 * 2048 photons and each optics wavefront units of 64 from device counters; pipeline: 1 = each
 * chunk's pre-roll bitmap and optics stages run on a context-owned second stream, overlapping
 * the survivor compaction and sky stage of the next chunk on the caller's stream (ordered by
 * events; the caller's stream waits for the last optics stage), 0 = everything on the caller's
 * stream.  Graphs captured by phx_trace_batched follow the same setting.
 * Defaults: 26, 16, 48, 2, 0, 1 (the shape the autotuner settles on for one star of 1e9 photons). */
typedef struct {
    int32_t chunk_log2;
    int32_t generate_blocks_per_cu, front_blocks_per_cu, back_blocks_per_cu;
    int32_t dynamic_tiles;
    int32_t pipeline;
} phx_launch_config;

phx_status phx_set_launch_config(phx_ctx ctx, const phx_launch_config* cfg_host);
phx_status phx_get_launch_config(phx_ctx ctx, phx_launch_config* cfg_host);

/* Batched trace (the many-source schedule): the same photons and results as phx_trace with the
 * same arguments, but the whole launch -- every chunk's pre-roll, sky and optics kernels over the
 * concatenated photon ranges of all sources in [src_begin, src_end) -- is captured once into a HIP
 * graph (keyed by the arguments and launch shape) and replayed with a single graph launch on
 * `stream`.  The first call with a new key prepares (uploads tables, may synchronise `stream`)
 * and captures on a context-owned stream; later calls only launch the graph.  Errors as phx_trace. */
phx_status phx_trace_batched(phx_ctx ctx, const phx_trace_args* args, void* stream);

/* Autotuner: times `sample` for candidate launch shapes (coordinate descent over the chunk size,
 * the schedule and the optics, sky and pre-roll workgroups per CU, in that order, up to three
 * passes; each shape's time is the best of three runs; the pipeline setting is kept and
 * selects what is timed: eager phx_trace launches when it is 1, phx_trace_batched graph replays
 * on one stream when it is 0), writing into context-owned scratch outputs (the sample's output
 * pointers are ignored), sets the fastest shape on the context and returns it in *best_host (may
 * be NULL).  Synchronises `stream`.  Errors as phx_trace, plus PHX_ERR_NOMEM. */
phx_status phx_autotune(phx_ctx ctx, const phx_trace_args* sample, void* stream,
                        phx_launch_config* best_host);

/* The same for phx_trace_batched graph replays in the context's pipeline setting (with the
 * pipeline on, the captured graph holds both streams' stages and their hand-offs). */
phx_status phx_autotune_batched(phx_ctx ctx, const phx_trace_args* sample, void* stream,
                                phx_launch_config* best_host);

/* Adjoint trace: the gradient of a weighted sum of per-source moments with respect to the
 * PHX_N_THETA perturbation parameters (section 2.4.1 misalignments: group 1 and group 2 shift
 * x, y, tilt x, y, piston; then the primary's Zernike Z4..Z15 amplitudes, section 2.4.1 surface
 * perturbations), as the pathwise derivative of the electron positions with every discrete
 * decision held at its forward value.  `args` names the same photons as the forward trace (its
 * output pointers are ignored; the pre-roll is switched on with coatings: it removes no
 * converted photon).  Only converted photons (DETECTED or OFF_CHIP) contribute, photon i of
 * source s with cotangents
 *     xbar = g[0] + g[2] (x_i - g[5]) + g[4] (y_i - g[6])
 *     ybar = g[1] + g[3] (y_i - g[6]) + g[4] (x_i - g[5]),  g = seed_dev + 8 (s - src_begin)
 * (for mean and central second moments: g = (dL/dmx, dL/dmy, 2 dL/dIxx, 2 dL/dIyy, dL/dIxy) / n
 * and (mx, my) the source's mean position).  seed_dev: device [src_end - src_begin][8] doubles.
 * grad_dev: device [PHX_N_THETA] doubles, overwritten with sum_i xbar_i dx_i/dtheta +
 * ybar_i dy_i/dtheta; the sum is taken in a fixed order for a fixed launch shape.  jac_dev:
 * optional device [slots][2][PHX_N_THETA] doubles; photon g of the launch (indexed as events)
 * with g % jac_stride == 0 gets its own (dx/dtheta, dy/dtheta), zero if not converted.
 * Enqueued on `stream`; may synchronise it to grow the context's tape.  Errors: as phx_trace,
 * PHX_ERR_CAPACITY if jac_capacity < ceil(total / jac_stride). */
phx_status phx_adjoint(phx_ctx ctx, const phx_trace_args* args, const double* seed_dev,
                       double* grad_dev, double* jac_dev, uint64_t jac_stride,
                       uint64_t jac_capacity, void* stream);

/* Per-source moments of the converted photons (paper section 3.1 outputs: per-source counts and
 * centroids; the moments of section 4 read as unweighted moments of the electron positions):
 * from the moment words of a trace with PHX_F_MOMENTS, moments_dev [n_src][PHX_MOMENT_WORDS]
 * (device), writes out_dev [n_src][6] (device doubles) = (n, mean x, mean y, Ixx, Iyy, Ixy),
 * mean x = SX / n, Ixx = (n SXX - SX^2) / n^2, Ixy = (n SXY - SX SY) / n^2 over the quantised
 * sums, each evaluated in exact integer arithmetic and rounded once to the nearest double (ties
 * to even); a source with n = 0 gets a zero row.  Enqueued on `stream`.  Errors:
 * PHX_ERR_INVALID (null buffer with n_src > 0, n_src < 0), PHX_ERR_HIP. */
phx_status phx_moments(phx_ctx ctx, const uint64_t* moments_dev, int32_t n_src, double* out_dev,
                       void* stream);

/* Adjoint of a loss of the per-source moments (the gradient of section 2.4.1's perturbation
 * parameters, as phx_adjoint): moments_dev is the forward trace's moment-word buffer
 * [n_sources][PHX_MOMENT_WORDS] (device; the rows of sources [src_begin, src_end) are read) and
 * dmom_dev [src_end - src_begin][5] (device doubles) the loss gradient with respect to
 * (mean x, mean y, Ixx, Iyy, Ixy) of each source.  The library forms the cotangent coefficients
 * of phx_adjoint on the device -- g = (dL/dmx, dL/dmy, 2 dL/dIxx, 2 dL/dIyy, dL/dIxy) / n and the
 * means from the words (zero for a source without converted photons) -- into a context-owned
 * buffer (grown on first use: that call may synchronise `stream`) and runs phx_adjoint with
 * them.  Other arguments, results and errors as phx_adjoint. */
phx_status phx_adjoint_moments(phx_ctx ctx, const phx_trace_args* args,
                               const uint64_t* moments_dev, const double* dmom_dev,
                               double* grad_dev, double* jac_dev, uint64_t jac_stride,
                               uint64_t jac_capacity, void* stream);

/* Copy a trace image (section 2.4.3 pixel counts) to host memory: image_dev [ny][nx] uint32
 * (device) into image_host (host, n = nx ny of the loaded prescription elements), enqueued on
 * `stream`, which is then synchronised.  Errors: PHX_ERR_STATE (no prescription),
 * PHX_ERR_INVALID (null pointer, n not nx ny), PHX_ERR_HIP. */
phx_status phx_read_image(phx_ctx ctx, const uint32_t* image_dev, uint32_t* image_host, int64_t n,
                          void* stream);

/* Kernel timing for profiling.  While on, phx_trace brackets each kernel it launches with HIP
 * events on the trace stream; phx_get_timing waits for them and returns the accumulated
 * milliseconds per kernel kind since timing was switched on:
 *   out[0] pre-roll bitmap (generate)   out[1] sky + atmosphere (front)
 *   out[2] optics + silicon (back)      out[3] number of chunks launched
 *   out[4] pre-roll survivor compaction (ordered or by time bucket).
 * n is the capacity of out (at most 5 values are written).  Switching on resets the totals.
 * Errors: PHX_ERR_INVALID, PHX_ERR_HIP. */
phx_status phx_set_timing(phx_ctx ctx, int32_t on);
phx_status phx_get_timing(phx_ctx ctx, double* out_host, int32_t n);

#ifdef __cplusplus
}
#endif
#endif
