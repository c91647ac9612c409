// Internal layout shared by the host API (phx_api.cpp) and the HIP kernels (phx_trace.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/phx.h"

namespace phx {

constexpr int kNZern = 12;  // Noll Z4..Z15
constexpr int kThreads = 256;   // workgroup size of every trace kernel
constexpr int kSedGuide = 1024;   // guide entries per SED for the wavelength search
constexpr int kNZernPoly = 15;  // monomials u^a v^b, a + b <= 4

// One surface as the kernels read it.  The element frame maps to the global frame by
// g = R q + t (R row-major); `moved` = 0 means R = identity and t = (0, 0, z_vertex).
struct DevSurface {
    int32_t kind, medium, coating, moved;
    int32_t asphere, zernike;              // asphere: 0 none, 1 even terms only, 2 general
    int32_t group;                         // rigid-body perturbation group (0 = fixed)
    int32_t glass_in;                      // the ray arrives through glass (else vacuum)
    double R[9];
    double t[3];
    double c, kappa1;      // curvature, 1 + kappa
    double alpha[8];       // alpha_3 .. alpha_10
    double r_in, r_out;
    double r_in2, r_out2;  // squared aperture radii
    double z_vertex;       // nominal vertex height (the group transform acts about a pivot)
};

struct DevSource {
    double xi, eta, nz;
    double lambda_lo, lambda_span, redshift1;
    double sersic_n, sersic_bn, sersic_a, sersic_b, cos_pa, sin_pa;
    int32_t kind, sed;
    uint64_t n_photons;
};

// Per-photon physics beyond the core path, as the kernels use it (derived from phx_physics).
struct DevPhysics {
    double airmass;                  // sec z
    double tau0, gamma;              // aerosol tau = tau0 (lambda / 500 nm)^gamma
    double disp_tanz, disp_cx, disp_cy;  // tan z and the direction of the shift in (n_x, n_y)
    double disp_pt, disp_w;          // Filippenko pressure-temperature factor, water factor
    double disp_b0, disp_s0;         // standard-air bracket and 1/lambda0^2 (um^-2) at lambda0
    double dome_sigma;
    double halo_f, halo_n, halo_r0;
    double halo_e, halo_fq, halo_inv_m;  // 1 - n/2, proposal CDF at x_max, 2^(1 - n/2)
    double dead;
    int32_t vanes, pad;
    double vane_c[8], vane_s[8];     // unit vector of each vane
    double vane_hw, vane_r0, vane_r1, vane_z0, vane_z1, vane_zm, vane_w;
    // second kick: per-layer phase variance above kappa_crit and exp(-variance); the wavenumber
    // CDF through A(kappa) = (kappa^2 + kappa0^2)^(-5/6): A0 = A(kappa_crit), dA = A0 - A(kappa_max)
    double kick_s2[PHX_MAX_LAYERS], kick_p0[PHX_MAX_LAYERS];
    double kick_A0, kick_dA, kick_k02;
    // field diffusion: sigma^2 at depths k dmax / n_sig2 below the entrance, k = 0..n_sig2
    const double* sig2;
    double sig2_inv_step, sig2_dmax;
    int32_t n_sig2, sig2_pad;
};
constexpr int kSig2Cells = 131072;   // cells of 0.75 nm over 98 um: sigma within 2e-14 m

// Everything the trace kernel reads that does not change between launches with the same loads.
struct DevParams {
    int32_t n_surf, nx, ny, n_layers;
    int32_t n_scales, screen_n, n_coat, n_s;
    int32_t n_lam, sed_k, has_glass, pad;
    DevSurface surf[PHX_MAX_SURF];
    double zern[kNZernPoly];   // Zernike deformation of surface 0 as monomial coefficients
    double zern_inv_r;
    double zern_basis[kNZern][kNZernPoly];  // Noll Z4..Z15 as monomial coefficients
    double group_pivot[3][3];
    double group_cs[3][4];     // cos t_x, sin t_x, cos t_y, sin t_y of each group's rotation
    double pupil_r_in, pupil_r_out;
    double z_start, obsc_z, obsc_r;
    double sell_b[3], sell_c[3];
    double chip_x0, chip_y0, pixel;
    double t_si, sigma_max;
    // Rajkanan constants at the device temperature (section 2.4.2)
    double eg[2], egd, absorb[2], emit[2];
    // coatings: uniform grid in s = sin^2(theta) and wavelength
    double inv_s_step, lam0, inv_dlam;
    int32_t cull_order[PHX_MAX_SURF]; // coated surfaces, most selective coating first
    // pre-roll escape test per wavelength column: a conversion word at or above esc_thr[il]
    // cannot mean a certain escape (a quick filter; the exact test follows below it); null: off
    const uint32_t* esc_thr;
    int32_t esc_col0;          // first column whose esc_thr is not 0 (n_lam when none)
    int32_t esc_pad;
    int32_t n_cull;
    int32_t ghost_cull_limit;  // first coated refracting surface (n_surf if none): with ghosts the
                               // pre-roll tests only coated surfaces ahead of it
    const float* coat;       // [n_coat][n_s][n_lam]
    const float* coat_r;     // [n_coat][n_s][n_lam] reflection probability (ghosts), or null
    const int64_t* coat_thr; // [n_coat][n_lam]: pre-roll threshold of wavelength column pair
                             // (il, il + 1): the largest roulette word w whose uniform
                             // (w + 1/2) 2^-32 does not exceed the larger of the two columns'
                             // maxima over s (plus 1e-12); -1 when every word exceeds it
    // atmosphere
    double height[PHX_MAX_LAYERS];
    double wind[PHX_MAX_LAYERS][2];
    double inv_pix[PHX_MAX_SCALES];
    double lambda_ref;
    const float4* grad;      // [L][S][N][N][2]: per cell (i, j) the gradients (g_x, g_y) at
                             // (i, j), (i+1, j) then (i, j+1), (i+1, j+1): one 32-byte record
                             // holds a bilinear footprint
    // sources
    const DevSource* src;
    const double* sed_cdf;   // [n_sed][sed_k + 1]
    const double* sed_edges; // [sed_k + 1]
    const uint16_t* sed_guide; // [n_sed][kSedGuide + 1]: guide[j] = the first bin k with
                               // CDF[k + 1] > j / kSedGuide (guide[kSedGuide] = sed_k - 1)
    DevPhysics ph;
};

// Per-launch arguments.
struct Launch {
    uint32_t seed, flags;
    int32_t src_begin, n_src;      // sources [src_begin, src_begin + n_src)
    uint64_t photon_begin;
    uint64_t uniform_count;        // > 0: every source traces this many photons
    const uint64_t* prefix;        // else: exclusive prefix of per-source counts [n_src + 1]
    const int32_t* src_guide;      // with prefix: src_guide[b] = the source holding flattened
                                   // photon b << guide_shift ([blocks + 1], last = n_src - 1)
    uint32_t guide_shift, guide_pad;
    uint64_t total;
    double exposure, pupil_margin;
    uint32_t* image;
    unsigned long long* stats;
    unsigned long long* moments;
    phx_event* events;
    uint64_t event_stride;
    int32_t any_sersic;            // an extended source is in the range
    int32_t any_zernike;           // the first surface carries a Zernike deformation
    // pre-roll geometric cull: a pupil sample at radius r with r^2 < cull_r2_lo or
    // r^2 > cull_r2_hi cannot
    // reach the primary's clear aperture (its atmospheric displacement is bounded)
    double cull_r2_lo, cull_r2_hi;
};

// Scratch of the staged trace: the launch's photon range is processed in chunks; per chunk the
// pre-roll survivor bitmap, the survivors (offsets within the chunk, in photon order), a
// survivor counter, and the start-plane state of every traced photon (7 doubles each,
// structure of arrays).
constexpr uint64_t kChunk = 1ull << 26;
// One chunk of a launch: photons [begin, begin + len) of the flattened launch index, and whether
// its pre-roll survivors are sorted by time bucket.  A chunk inside one source's range names it
// (src: index relative to the launch's first source, first: the flattened index of that source's
// first photon); src = -1 for a chunk that spans several sources.
struct ChunkSpan {
    uint64_t begin, len, first;
    int32_t sort, src;
};
struct Workspace {
    uint32_t* survivors;       // [buffers][chunk]
    unsigned int* counts;      // [n_chunks]
    uint64_t n_chunks;
    double* state;             // [buffers][7][chunk]
    uint64_t chunk;
    unsigned long long* tiles; // [n_chunks][2] tile counters of the dynamic schedule
    unsigned long long* bits;  // [buffers][chunk / 64] survivor bitmap
    unsigned int* bsum;        // [compact_groups(chunk)] survivors per compaction workgroup
    uint8_t* key;              // [buffers][chunk] time bucket of each survivor
    unsigned int* hist;        // [2 bucket_groups(chunk) + 1][kTimeBucketsMax]: survivors per
                               // bucket and workgroup, their prefixes over workgroups, totals
    const ChunkSpan* plan;     // host array: the launch's chunks in order
    uint64_t n_plan;
    int buffers;               // bitmaps, keys, survivors and states hold this many chunks
                               // (1 or 2)
    double* ghost_list = nullptr;          // [kGhostFields][ghost_cap] ghost starts of a chunk
    uint64_t ghost_cap = 0;                 // (with ghosts: at least chunk entries)
    unsigned long long* ghost_ctr = nullptr; // [2] entries listed, entries claimed
};
// Workspace of phx_trace_noalloc: a file-scope device array of kScratchBytes on each GPU (its
// address is looked up once per device when a context is created), carved into the buffers of
// one chunk of at most 2^kNoAllocChunkLog2 photons (one buffer set: no pipeline), the per-chunk
// counters of at most kNoAllocMaxChunks chunks, and the prefix table and source guide of at
// most kNoAllocMaxSources sources (built on the device).  Offsets in bytes, each 256-aligned.
constexpr int kNoAllocChunkLog2 = 19;
constexpr uint64_t kNoAllocMaxChunks = 16384;
constexpr int kNoAllocMaxSources = 65536;
constexpr uint64_t kNoAllocGuideMax = 8ull * kNoAllocMaxSources + 2;   // guide blocks + 1
constexpr uint64_t kScratchBytes = 40ull << 20;
struct ScratchLayout {
    uint64_t survivors, state, bits, bsum, key, hist, counts, tiles, prefix, guide, end;
};
constexpr uint64_t align256(uint64_t x) { return (x + 255) & ~uint64_t(255); }
constexpr ScratchLayout scratch_layout() {
    const uint64_t chunk = 1ull << kNoAllocChunkLog2;
    const uint64_t groups = ((chunk + 63) / 64 + 4095) / 4096;            // compaction
    const uint64_t bgroups = ((chunk + 63) / 64 + 1023) / 1024;           // time-bucket sort
    ScratchLayout s{};
    s.survivors = 0;
    s.state = align256(s.survivors + chunk * 4);
    s.bits = align256(s.state + 7 * chunk * 8);
    s.bsum = align256(s.bits + (chunk + 63) / 64 * 8);
    s.key = align256(s.bsum + groups * 4);
    s.hist = align256(s.key + chunk);
    s.counts = align256(s.hist + (2 * bgroups + 1) * 64 * 4);
    s.tiles = align256(s.counts + kNoAllocMaxChunks * 4);
    s.prefix = align256(s.tiles + 2 * kNoAllocMaxChunks * 8);
    s.guide = align256(s.prefix + (kNoAllocMaxSources + 1) * 8);
    s.end = align256(s.guide + kNoAllocGuideMax * 4);
    return s;
}
static_assert(scratch_layout().end <= kScratchBytes, "no-allocation workspace exceeds the scratch");
// Device address of this GPU's scratch array (the calling thread's current device must be
// `device`); looked up once per device and cached.
hipError_t scratch_address(int device, void** out);
// Exclusive prefix of the photon counts of sources [src_begin, src_begin + n_src) into
// prefix[0 .. n_src] and the photon-block guide (Launch::src_guide) guide[0 .. n_blocks] for
// blocks of 2^shift photons, computed on the device from the source table.
hipError_t launch_prefix(const DevSource* src, int src_begin, int n_src, uint64_t* prefix,
                         int32_t* guide, uint64_t n_blocks, uint32_t shift, hipStream_t stream);

// 8-byte fields of one entry of the ghost list (the optics kernel's ghost starts of a chunk).
constexpr int kGhostFields = 14;

// Second stream and events for pipelining chunks (aux null: everything on the caller's stream).
struct Pipe {
    hipStream_t aux = nullptr;   // pre-roll and optics stages
    hipEvent_t* ev = nullptr;    // at least 3 n_chunks + 1 events
    uint64_t n_ev = 0;
};
constexpr int kTimeBucketsMax = 64;
// Workgroups of the ordered compaction for a chunk of n photons (64 photons per bitmap word,
// 4096 words per workgroup).
inline uint64_t compact_groups(uint64_t n) { return ((n + 63) / 64 + 4095) / 4096; }
// Workgroups of the time-bucket sort for a chunk of n photons (1024 bitmap words each).
constexpr int kBucketWordsPerThread = 4;
inline uint64_t bucket_groups(uint64_t n) {
    return ((n + 63) / 64 + kThreads * kBucketWordsPerThread - 1) / (kThreads * kBucketWordsPerThread);
}

// Launch shape (tunable): workgroups per compute unit of each stage, and the schedule of the
// sky and optics stages (static grid-stride, or tiles of kTileIters x 256 photons taken from a
// device counter).
struct LaunchConfig {
    int generate_per_cu = 16;
    int front_per_cu = 48;
    int back_per_cu = 2;
    int dynamic = 0;
    int pipeline = 1;
};
constexpr int kTileIters = 8;
// Flags that select the sky and optics kernels carrying the per-photon physics beyond the core
// path (the other instantiations hold none of its code).
constexpr uint32_t kFrontExtra = PHX_F_DISPERSION | PHX_F_DOME | PHX_F_HALO | PHX_F_SECOND_KICK;
constexpr uint32_t kBackExtra = PHX_F_AEROSOL | PHX_F_SPIDER | PHX_F_GHOSTS;

// Optional per-kernel timing: events recorded before/after each kernel launch.
struct Timing {
    bool on = false;
    // event pairs per kernel kind (0 generate, 1 front, 2 back, 3 survivor compaction),
    // appended per chunk
    void (*record)(void* self, int kind, int edge, hipStream_t stream) = nullptr;
    void* self = nullptr;
};

hipError_t launch_trace(const DevParams* dparams, const Launch& L, const Workspace& W, int n_cu,
                        const LaunchConfig& cfg, hipStream_t stream, const Pipe& pipe,
                        const Timing& T);
// Adjoint of the per-source moments (pathwise derivative, decisions frozen).  Per-lane
// accumulators: the ten rigid-body parameters, then the fifteen monomial coefficients of the
// primary's deformation (mapped to Zernike amplitudes by the final reduction).
constexpr int kAdj = 10 + kNZernPoly;
constexpr int kTapeFields = 7;   // per surface: hit point (3), incoming direction (3), path length
struct Adjoint {
    const double* seed;      // [n_src][8]: gx, gy, gxx, gyy, gxy, mean x, mean y, unused
    double* partial;         // [rows][kAdj], one row per (chunk, workgroup)
    double* tape;            // [n_surf * kTapeFields][tape_stride]
    uint64_t tape_stride;    // threads of one adjoint launch
    double* jac;             // optional [slots][2][PHX_N_THETA]
    uint64_t jac_stride, jac_cap;
    int per_cu;              // workgroups per compute unit of the adjoint kernel
};

hipError_t launch_adjoint(const DevParams* dparams, const Launch& L, const Workspace& W, int n_cu,
                          const LaunchConfig& cfg, const Adjoint& A, double* colsum, double* grad,
                          hipStream_t stream, const Pipe& pipe, const Timing& T);
// One readout of a sensor image (phx_readout): parameters, the input electrons and the
// buffers of each step (device pointers).
struct ReadoutJob {
    phx_readout_params p;
    const uint32_t* in;
    int32_t nx, ny;
    uint32_t* work;     // [ny][nx] after bleeding, dark current and defects
    uint32_t* par;      // [amp][sh + over_y][sw] after the parallel transfers
    uint32_t* ser;      // [amp][sh + over_y][sw + over_x] after the serial transfers
    uint16_t* out;      // [amp][sh + over_y][sw + over_x] ADU
    uint32_t* heavy;    // packets with many electrons, handled one workgroup each
                        // [max(ny nx, amp (sh + over_y) sw)]
    uint32_t* heavy_count;
};
hipError_t launch_readout(const ReadoutJob& J, hipStream_t stream);

// Per-source (n, mean x, mean y, Ixx, Iyy, Ixy) from moment words [n_src][PHX_MOMENT_WORDS]
// into out [n_src][6], each rounded once from exact integer arithmetic (phx_moments).
hipError_t launch_moments(const unsigned long long* words, int n_src, double* out,
                          hipStream_t stream);
// The adjoint's cotangent coefficients [n_src][8] from the moment words and a loss gradient
// dmom [n_src][5] with respect to (mean x, mean y, Ixx, Iyy, Ixy).
hipError_t launch_seeds(const unsigned long long* words, int n_src, const double* dmom,
                        double* seed, hipStream_t stream);

hipError_t launch_gradients(const float* opd, float4* grad, int n_layers, int n_scales, int n,
                            const double* pixel, unsigned int* gmax, hipStream_t stream);

}  // namespace phx
