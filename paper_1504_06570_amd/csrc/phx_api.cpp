// C ABI of the photon trace library (declarations and contracts in include/phx.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "phx_internal.h"

using phx::DevParams;
using phx::DevSource;
using phx::DevSurface;

struct phx_ctx_s {
    int device = 0;
    int n_cu = 256;
    std::string err;
    bool have_presc = false, have_src = false, have_coat = false, have_screens = false;
    bool have_phys = false;
    bool have_refl = false;
    float* d_coat_r = nullptr;           // reflection probabilities (ghosts)
    phx_physics phys{};                  // last loaded physics parameters (re-derived on a new
                                         // prescription)
    bool field_ok = false;               // E_z > 0 across the device (field diffusion usable)
    double* d_sig2 = nullptr;            // sigma^2 against depth [kSig2Cells + 1]
    // readout chain scratch (phx_readout without caller buffers)
    // work, parallel slots, serial slots, heavy-packet list (+ its counter)
    uint32_t* d_ro[4] = {nullptr, nullptr, nullptr, nullptr};
    uint64_t ro_cap[4] = {0, 0, 0, 0};
    phx_prescription presc{};
    double theta[PHX_N_THETA] = {0};
    DevParams host{};          // host image of the device parameter block
    DevParams* dparams = nullptr;
    bool dirty = true;
    float* d_coat = nullptr;
    int64_t* d_coat_thr = nullptr;
    uint32_t* d_esc_thr = nullptr;       // pre-roll escape filter per wavelength column
    float4* d_grad = nullptr;
    size_t grad_elems = 0;
    DevSource* d_src = nullptr;
    std::vector<phx_source> src;
    std::vector<float> coat_max;   // host copy of the per-wavelength worst-case transmission
    double* d_cdf = nullptr;
    uint16_t* d_guide = nullptr;          // SED search guide [n_sed][kSedGuide + 1]
    double* d_edges = nullptr;
    uint64_t* d_prefix = nullptr;
    size_t prefix_cap = 0;
    int32_t* d_src_guide = nullptr;       // photon-block -> source guide of the prefix table
    size_t src_guide_cap = 0;
    uint32_t guide_shift = 0;
    uint32_t* d_survivors = nullptr;     // pre-roll survivors of one chunk
    unsigned int* d_counts = nullptr;    // survivor count per chunk
    uint64_t counts_cap = 0;
    double* d_state = nullptr;           // start-plane state of one chunk [7][ws_chunk]
    uint64_t ws_chunk = 0;
    double* d_ghost = nullptr;           // ghost list of a chunk (with ghosts) and its counters
    uint64_t ghost_cap = 0;
    unsigned long long* d_ghost_ctr = nullptr;
    // kernel timing (phx_set_timing)
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<int, std::pair<size_t, size_t>>> ev_pairs;   // kind, (start, stop)
    size_t ev_used = 0;
    long pending_start[4] = {-1, -1, -1, -1};
    double timing_ms[4] = {0, 0, 0, 0};   // pre-roll bitmap, sky, optics, compaction
    double timing_chunks = 0;
    // launch shape, prefix-table cache, captured graphs (phx_trace_batched)
    phx::LaunchConfig cfg;
    int chunk_log2 = 26;
    uint64_t* d_tiles = nullptr;
    bool prefix_valid = false;
    int prefix_begin = 0, prefix_end = 0;
    uint64_t src_version = 0, prefix_version = 0;
    hipStream_t cap_stream = nullptr;
    hipStream_t aux_stream = nullptr;       // optics stage of the chunk pipeline
    std::vector<hipEvent_t> pipe_ev;        // hand-off events of the chunk pipeline
    std::map<std::string, hipGraphExec_t> graphs;
    float autotune_ms = 0.0f;
    // adjoint workspace
    int adj_per_cu = 2;
    double* d_tape = nullptr;
    uint64_t tape_cap = 0;
    double* d_partial = nullptr;
    uint64_t rows_cap = 0;
    double* d_colsum = nullptr;
    double* d_seed = nullptr;            // cotangent coefficients of phx_adjoint_moments
    uint64_t seed_cap = 0;
    uint64_t* d_bits = nullptr;
    unsigned int* d_bsum = nullptr;
    uint8_t* d_key = nullptr;
    unsigned int* d_hist = nullptr;
    std::vector<phx::ChunkSpan> plan;   // reserved for kNoAllocMaxChunks chunks at creation
    void* scratch = nullptr;            // device address of this GPU's no-allocation workspace
    double sed_lo = 0.0;                    // lowest SED bin edge (m)
    std::vector<double> grad_max;           // [layer][scale] largest gradient norm of a screen
    void graphs_clear() {
        for (auto& g : graphs) (void)hipGraphExecDestroy(g.second);
        graphs.clear();
    }
};

namespace {
void timing_record(void* self, int kind, int edge, hipStream_t stream) {
    phx_ctx c = (phx_ctx)self;
    if (c->ev_used == c->ev_pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return;
        c->ev_pool.push_back(e);
    }
    const size_t i = c->ev_used++;
    if (hipEventRecord(c->ev_pool[i], stream) != hipSuccess) return;
    if (edge == 0) {
        c->pending_start[kind] = (long)i;
    } else if (c->pending_start[kind] >= 0) {
        c->ev_pairs.push_back({kind, {(size_t)c->pending_start[kind], i}});
        c->pending_start[kind] = -1;
        if (kind == 2) c->timing_chunks += 1;
    }
}
}  // namespace

namespace {

phx_status fail(phx_ctx c, phx_status code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return code;
}

phx_status hip_fail(phx_ctx c, hipError_t e, const char* what) {
    return fail(c, PHX_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

bool finite_all(const double* v, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(v[i])) return false;
    return true;
}

template <class T>
void free_dev(T*& p) {
    if (p) (void)hipFree((void*)p);
    p = nullptr;
}

// Rigid-body transforms of the surfaces from the perturbation vector.  A group's elements are
// rotated by R = R_x(tx) R_y(ty) about the group's pivot P and translated by (dx, dy, dz): an
// element-frame point q maps to g = R q + t with t = P + R (v - P) + d, v = (0, 0, z_vertex).
void build_surfaces(phx_ctx c) {
    const phx_prescription& p = c->presc;
    DevParams& H = c->host;
    H.n_surf = p.n_surfaces;
    for (int k = 0; k < p.n_surfaces; ++k) {
        const phx_surface& s = p.surf[k];
        DevSurface& d = H.surf[k];
        std::memset(&d, 0, sizeof(d));
        d.kind = s.kind;
        d.medium = s.medium;
        d.coating = s.coating;
        d.c = s.curvature;
        d.kappa1 = 1.0 + s.conic;
        d.asphere = 0;
        for (int i = 0; i < 8; ++i) {
            d.alpha[i] = s.alpha[i];
            if (s.alpha[i] != 0.0) d.asphere = (i & 1) ? 1 : 2;   // alpha[i] is alpha_{i+3}
        }
        for (int i = 0; i < 8; i += 2)
            if (s.alpha[i] != 0.0) d.asphere = 2;                  // an odd power is present
        d.r_in = s.r_inner;
        d.r_out = s.r_outer;
        d.z_vertex = s.z_vertex;
        d.group = (s.group == 1 || s.group == 2) ? s.group : 0;
        d.r_in2 = s.r_inner * s.r_inner;
        d.r_out2 = s.r_outer * s.r_outer;
        double dx = 0, dy = 0, dz = 0, tx = 0, ty = 0;
        const double* P = p.group_pivot[0];
        if (s.group == 1 || s.group == 2) {
            const double* th = c->theta + 5 * (s.group - 1);
            dx = th[0]; dy = th[1]; tx = th[2]; ty = th[3]; dz = th[4];
            P = p.group_pivot[s.group];
        }
        d.moved = (dx != 0 || dy != 0 || dz != 0 || tx != 0 || ty != 0) ? 1 : 0;
        const double cx = std::cos(tx), sx = std::sin(tx), cy = std::cos(ty), sy = std::sin(ty);
        // R_x(tx) R_y(ty)
        const double R[9] = {cy, 0.0, sy, sx * sy, cx, -sx * cy, -cx * sy, sx, cx * cy};
        const double v[3] = {0.0, 0.0, s.z_vertex};
        const double dd[3] = {dx, dy, dz};
        for (int i = 0; i < 3; ++i) {
            const double rv = R[3 * i] * (v[0] - P[0]) + R[3 * i + 1] * (v[1] - P[1]) +
                              R[3 * i + 2] * (v[2] - P[2]);
            d.t[i] = d.moved ? P[i] + rv + dd[i] : v[i];
        }
        for (int i = 0; i < 9; ++i) d.R[i] = R[i];
    }
    // medium in front of each surface, in travel order (mirrors keep it, lenses set it)
    bool glass = false;
    for (int k = 0; k < p.n_surfaces; ++k) {
        H.surf[k].glass_in = glass ? 1 : 0;
        if (p.surf[k].kind == PHX_REFRACT) glass = p.surf[k].medium == PHX_GLASS;
    }
    for (int g = 0; g < 3; ++g) {
        double tx = 0.0, ty = 0.0;
        if (g > 0) {
            tx = c->theta[5 * (g - 1) + 2];
            ty = c->theta[5 * (g - 1) + 3];
        }
        H.group_cs[g][0] = std::cos(tx);
        H.group_cs[g][1] = std::sin(tx);
        H.group_cs[g][2] = std::cos(ty);
        H.group_cs[g][3] = std::sin(ty);
        for (int i = 0; i < 3; ++i) H.group_pivot[g][i] = p.group_pivot[g][i];
    }
    // Zernike deformation of surface 0 (Noll Z4..Z15, amplitudes theta[10..21]) expanded into the
    // monomials u^a v^b of degree <= 4, ordered as the kernel's zernike_poly expects.
    enum { C00, C10, C01, C20, C11, C02, C30, C21, C12, C03, C40, C31, C22, C13, C04 };
    const double s3 = std::sqrt(3.0), s5 = std::sqrt(5.0), s6 = std::sqrt(6.0);
    const double s8 = std::sqrt(8.0), s10 = std::sqrt(10.0);
    double (*B)[phx::kNZernPoly] = H.zern_basis;
    std::memset(H.zern_basis, 0, sizeof(H.zern_basis));
    B[0][C00] = -s3;  B[0][C20] = 2 * s3;  B[0][C02] = 2 * s3;                    // Z4
    B[1][C11] = 2 * s6;                                                          // Z5
    B[2][C20] = s6;   B[2][C02] = -s6;                                            // Z6
    B[3][C21] = 3 * s8; B[3][C03] = 3 * s8; B[3][C01] = -2 * s8;                  // Z7
    B[4][C30] = 3 * s8; B[4][C12] = 3 * s8; B[4][C10] = -2 * s8;                  // Z8
    B[5][C21] = 3 * s8; B[5][C03] = -s8;                                         // Z9
    B[6][C30] = s8;   B[6][C12] = -3 * s8;                                        // Z10
    B[7][C40] = 6 * s5; B[7][C22] = 12 * s5; B[7][C04] = 6 * s5;                  // Z11
    B[7][C20] = -6 * s5; B[7][C02] = -6 * s5; B[7][C00] = s5;
    B[8][C40] = 4 * s10; B[8][C04] = -4 * s10;                                   // Z12
    B[8][C20] = -3 * s10; B[8][C02] = 3 * s10;
    B[9][C31] = 8 * s10; B[9][C13] = 8 * s10; B[9][C11] = -6 * s10;              // Z13
    B[10][C40] = s10; B[10][C22] = -6 * s10; B[10][C04] = s10;                   // Z14
    B[11][C31] = 4 * s10; B[11][C13] = -4 * s10;                                 // Z15
    const double* a = c->theta + 10;
    double z[phx::kNZernPoly] = {0};
    for (int j = 0; j < phx::kNZern; ++j)
        for (int m = 0; m < phx::kNZernPoly; ++m) z[m] += B[j][m] * a[j];
    bool any = false;
    for (int j = 0; j < phx::kNZern; ++j) any |= a[j] != 0.0;
    for (int j = 0; j < phx::kNZernPoly; ++j) H.zern[j] = z[j];
    H.surf[0].zernike = any ? 1 : 0;
    H.zern_inv_r = 1.0 / p.surf[0].r_outer;
}

phx_status set_device(phx_ctx c);

// Host copies of the silicon and glass optics the pre-roll escape filter is built from (the
// filter only needs to be approximately right: a low value skips culls, never adds one).
double host_absorption(const DevParams& H, double lam) {
    const double e = 1.2398419843320026e-6 / lam;
    const double C[2] = {5.5, 4.0}, A[2] = {3.231e2, 7.237e3}, ep[2] = {1.827e-2, 5.773e-2};
    double alpha = 0.0;
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
            const double a = e - H.eg[j] + ep[i], b = e - H.eg[j] - ep[i];
            double term = 0.0;
            if (a > 0.0) term += a * a / H.absorb[i];
            if (b > 0.0) term += b * b / H.emit[i];
            alpha += C[i] * A[j] * term;
        }
    if (e > H.egd) alpha += 1.052e6 * std::sqrt(e - H.egd);
    return alpha * 100.0;
}
double host_n_silicon(double lam) {
    const double e = 1.2398419843320026e-6 / lam;
    return 3.36 + 0.211 * e + 2.79 * std::exp((e - 3.30) / 0.398);
}
double host_sellmeier(const DevParams& H, double lam) {
    const double l2 = (lam * 1e6) * (lam * 1e6);
    double s = 1.0;
    for (int i = 0; i < 3; ++i) s += H.sell_b[i] * l2 / (l2 - H.sell_c[i]);
    return std::sqrt(s);
}

// Pre-roll escape filter (section 3.2 with the silicon stage): a photon whose conversion distance
// L = -ln(u) / alpha exceeds t_Si / cos_min, with cos_min the smallest cosine a ray refracted into
// silicon can have, escapes whatever its path: u < E(lambda) = exp(-alpha t_Si / cos_min).  Per
// wavelength column the table holds the first word whose uniform reaches 1.5 x max E over the
// column (sampled; the first column also stands for every bluer wavelength, whose absorption is
// stronger), so that words at or above it skip the exact test (0: the column never takes it); the
// last column stands for every redder wavelength and always takes it.
phx_status build_escape_table(phx_ctx c) {
    DevParams& H = c->host;
    H.esc_thr = nullptr;
    H.esc_col0 = H.n_lam;
    if (!c->have_presc || !c->have_coat) return PHX_OK;
    // a flat silicon detector: the depth is measured along the surface normal
    const phx_surface& det = c->presc.surf[c->presc.n_surfaces - 1];
    if (det.medium != PHX_SILICON || det.curvature != 0.0) return PHX_OK;
    for (int i = 0; i < 8; ++i)
        if (det.alpha[i] != 0.0) return PHX_OK;
    std::vector<uint32_t> t((size_t)H.n_lam, 0xFFFFFFFFu);
    const double dlam = 1.0 / H.inv_dlam;
    for (int il = 0; il + 2 < H.n_lam; ++il) {
        double emax = 0.0;
        for (int k = 0; k <= 32; ++k) {
            const double lam = il == 0 ? H.lam0 * (0.5 + k / 64.0) + k / 32.0 * dlam
                                       : H.lam0 + (il + k / 32.0) * dlam;
            const double n_in = H.has_glass ? host_sellmeier(H, lam) : 1.0;
            const double q = n_in / host_n_silicon(lam);
            const double cmin = q < 1.0 ? std::sqrt(1.0 - q * q) : 0.0;
            const double alpha = host_absorption(H, lam);
            const double e = cmin > 0.0 ? std::exp(-alpha * H.t_si / cmin) : 0.0;
            emax = std::max(emax, e);
        }
        // u01(w) < x  <=>  w < x 2^32 - 1/2: no word passes below ceil(x 2^32 - 1/2).  A column
        // whose escape chance stays below 1e-3 skips the test: its Philox block would cost more
        // than the culls save (skipping a cull never changes a result).
        const double x = emax * 1.5;
        const double w = std::ceil(x * 4294967296.0 - 0.5);
        t[(size_t)il] = x < 1e-3 ? 0u : (w >= 4294967295.0 ? 0xFFFFFFFFu : (uint32_t)w);
    }
    int col0 = H.n_lam;
    for (int il = H.n_lam - 1; il >= 0; --il)
        if (t[(size_t)il]) col0 = il;
    if (set_device(c) != PHX_OK) return PHX_ERR_HIP;
    free_dev(c->d_esc_thr);
    hipError_t e = hipMalloc((void**)&c->d_esc_thr, t.size() * sizeof(uint32_t));
    if (e != hipSuccess) return fail(c, PHX_ERR_NOMEM, "escape table: %s", hipGetErrorString(e));
    e = hipMemcpy(c->d_esc_thr, t.data(), t.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(c, e, "hipMemcpy(escape table)");
    H.esc_thr = c->d_esc_thr;
    H.esc_col0 = col0;
    return PHX_OK;
}

// Largest 32-bit roulette word w whose uniform (w + 1/2) 2^-32 does not exceed r, or -1 when
// none does: u01(w) > r  <=>  w > word_threshold(r), since u01 is increasing and exact.
int64_t word_threshold(double r) {
    const auto u = [](int64_t w) {
        return std::fma((double)w, 2.3283064365386963e-10, 1.1641532182693481e-10);
    };
    const int64_t top = 0xFFFFFFFFll;
    if (!(u(0) <= r)) return -1;
    if (u(top) <= r) return top;
    int64_t w = (int64_t)std::floor(r * 4294967296.0 - 0.5);
    w = std::min(std::max(w, (int64_t)0), top);
    while (w < top && u(w + 1) <= r) ++w;
    while (w > 0 && u(w) > r) --w;
    return w;
}

// Pre-roll order: coated surfaces sorted by the mean (over wavelength) of their coating's
// worst-case transmission, most selective first; ties keep the surface order.
void build_cull_order(phx_ctx c) {
    DevParams& H = c->host;
    H.n_cull = 0;
    H.ghost_cull_limit = 0;
    if (!c->have_presc || !c->have_coat) return;
    H.ghost_cull_limit = c->presc.n_surfaces;
    for (int k = 0; k < c->presc.n_surfaces; ++k)
        if (c->presc.surf[k].kind != PHX_MIRROR && c->presc.surf[k].coating >= 0) {
            H.ghost_cull_limit = k;
            break;
        }
    std::vector<std::pair<double, int>> v;
    for (int k = 0; k < c->presc.n_surfaces; ++k) {
        const int co = c->presc.surf[k].coating;
        if (co < 0 || co >= H.n_coat) continue;
        double m = 0.0;
        for (int l = 0; l < H.n_lam; ++l) m += c->coat_max[(size_t)co * H.n_lam + l];
        v.push_back({m / H.n_lam, k});
    }
    std::stable_sort(v.begin(), v.end(),
                     [](const std::pair<double, int>& a, const std::pair<double, int>& b) {
                         return a.first < b.first;
                     });
    for (size_t i = 0; i < v.size(); ++i) H.cull_order[i] = v[i].second;
    H.n_cull = (int)v.size();
}

phx_status set_device(phx_ctx c) {
    const hipError_t e = hipSetDevice(c->device);
    return e == hipSuccess ? PHX_OK : hip_fail(c, e, "hipSetDevice");
}

phx_status upload_params(phx_ctx c, hipStream_t stream) {
    if (!c->dirty) return PHX_OK;
    hipError_t e = hipMemcpyAsync(c->dparams, &c->host, sizeof(DevParams), hipMemcpyHostToDevice,
                                  stream);
    if (e != hipSuccess) return hip_fail(c, e, "hipMemcpyAsync(params)");
    // the host image may change before the copy runs: wait for it
    e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(c, e, "hipStreamSynchronize");
    c->dirty = false;
    return PHX_OK;
}

}  // namespace

extern "C" {

const char* phx_version(void) { return "phx 0.1 (gfx950)"; }

phx_status phx_create(int32_t device, phx_ctx* out) {
    if (!out) return PHX_ERR_INVALID;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return PHX_ERR_INVALID;
    phx_ctx c = new (std::nothrow) phx_ctx_s();
    if (!c) return PHX_ERR_NOMEM;
    c->device = device;
    hipError_t e = hipSetDevice(device);
    if (e == hipSuccess) {
        hipDeviceProp_t prop;
        e = hipGetDeviceProperties(&prop, device);
        if (e == hipSuccess) c->n_cu = prop.multiProcessorCount;
    }
    if (e == hipSuccess) e = hipMalloc((void**)&c->dparams, sizeof(DevParams));
    // the device address of this GPU's phx_trace_noalloc workspace (looked up once per device,
    // with the device current)
    if (e == hipSuccess) e = phx::scratch_address(device, &c->scratch);
    if (e != hipSuccess) {
        free_dev(c->dparams);
        delete c;
        return PHX_ERR_HIP;
    }
    try {
        c->plan.reserve(phx::kNoAllocMaxChunks);
    } catch (...) {
        free_dev(c->dparams);
        delete c;
        return PHX_ERR_NOMEM;
    }
    *out = c;
    return PHX_OK;
}

void phx_destroy(phx_ctx c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    free_dev(c->dparams);
    free_dev(c->d_coat);
    free_dev(c->d_coat_thr);
    free_dev(c->d_esc_thr);
    free_dev(c->d_sig2);
    free_dev(c->d_coat_r);
    for (int k = 0; k < 4; ++k) free_dev(c->d_ro[k]);
    free_dev(c->d_grad);
    free_dev(c->d_src);
    free_dev(c->d_cdf);
    free_dev(c->d_guide);
    free_dev(c->d_edges);
    free_dev(c->d_prefix);
    free_dev(c->d_src_guide);
    free_dev(c->d_survivors);
    free_dev(c->d_counts);
    free_dev(c->d_state);
    free_dev(c->d_ghost);
    free_dev(c->d_ghost_ctr);
    free_dev(c->d_tiles);
    free_dev(c->d_tape);
    free_dev(c->d_partial);
    free_dev(c->d_colsum);
    free_dev(c->d_seed);
    free_dev(c->d_bits);
    free_dev(c->d_bsum);
    free_dev(c->d_key);
    free_dev(c->d_hist);
    c->graphs_clear();
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    if (c->aux_stream) (void)hipStreamDestroy(c->aux_stream);
    for (hipEvent_t e : c->pipe_ev) (void)hipEventDestroy(e);
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    delete c;
}

const char* phx_last_error(phx_ctx c) { return c ? c->err.c_str() : "null context"; }

phx_status phx_load_prescription(phx_ctx c, const phx_prescription* p) {
    if (!c) return PHX_ERR_INVALID;
    if (!p) return fail(c, PHX_ERR_INVALID, "null prescription");
    if (p->n_surfaces < 1 || p->n_surfaces > PHX_MAX_SURF)
        return fail(c, PHX_ERR_INVALID, "n_surfaces %d outside 1..%d", p->n_surfaces, PHX_MAX_SURF);
    if (p->surf[p->n_surfaces - 1].kind != PHX_DETECTOR)
        return fail(c, PHX_ERR_INVALID, "the last surface must be the detector");
    for (int k = 0; k < p->n_surfaces; ++k) {
        const phx_surface& s = p->surf[k];
        if (s.kind < PHX_MIRROR || s.kind > PHX_DETECTOR)
            return fail(c, PHX_ERR_INVALID, "surface %d: bad kind %d", k, s.kind);
        if (s.kind == PHX_DETECTOR && k != p->n_surfaces - 1)
            return fail(c, PHX_ERR_INVALID, "surface %d: detector before the last surface", k);
        if (s.medium < PHX_VACUUM || s.medium > PHX_SILICON)
            return fail(c, PHX_ERR_INVALID, "surface %d: bad medium %d", k, s.medium);
        if (s.group < 0 || s.group > 2)
            return fail(c, PHX_ERR_INVALID, "surface %d: bad group %d", k, s.group);
        const double v[4] = {s.z_vertex, s.curvature, s.conic, s.r_inner};
        if (!finite_all(v, 4) || !finite_all(s.alpha, 8) || !std::isfinite(s.r_outer) ||
            !(s.r_outer > 0.0) || s.r_inner < 0.0 || s.r_inner >= s.r_outer)
            return fail(c, PHX_ERR_INVALID, "surface %d: non-finite value or bad aperture", k);
    }
    if (p->nx <= 0 || p->ny <= 0 || p->nx > 32767 || p->ny > 32767)
        return fail(c, PHX_ERR_INVALID, "chip %d x %d out of range", p->nx, p->ny);
    const double g[] = {p->pupil_r_inner, p->pupil_r_outer, p->z_start, p->obscuration_z,
                        p->obscuration_r, p->chip_x0, p->chip_y0, p->pixel, p->si_thickness,
                        p->si_temperature, p->sigma_max};
    if (!finite_all(g, sizeof(g) / sizeof(g[0])) || !(p->pixel > 0) || !(p->si_thickness > 0) ||
        !(p->si_temperature > 0) || p->sigma_max < 0 || !(p->pupil_r_outer > p->pupil_r_inner) ||
        p->pupil_r_inner < 0)
        return fail(c, PHX_ERR_INVALID, "bad pupil, chip or silicon parameters");
    if (!finite_all(p->sellmeier_b, 3) || !finite_all(p->sellmeier_c, 3) ||
        !finite_all(&p->group_pivot[0][0], 9))
        return fail(c, PHX_ERR_INVALID, "non-finite Sellmeier coefficients or pivots");
    c->presc = *p;
    DevParams& H = c->host;
    H.nx = p->nx;
    H.ny = p->ny;
    H.pupil_r_in = p->pupil_r_inner;
    H.pupil_r_out = p->pupil_r_outer;
    H.z_start = p->z_start;
    H.obsc_z = p->obscuration_z;
    H.obsc_r = p->obscuration_r;
    for (int i = 0; i < 3; ++i) {
        H.sell_b[i] = p->sellmeier_b[i];
        H.sell_c[i] = p->sellmeier_c[i];
    }
    H.has_glass = 0;
    for (int k = 0; k < p->n_surfaces; ++k) H.has_glass |= p->surf[k].medium == PHX_GLASS;
    H.chip_x0 = p->chip_x0;
    H.chip_y0 = p->chip_y0;
    H.pixel = p->pixel;
    H.t_si = p->si_thickness;
    H.sigma_max = p->sigma_max;
    // Rajkanan temperature-dependent constants (section 2.4.2)
    const double T = p->si_temperature, kB = 8.617333262e-5;
    const double shift = 7.021e-4 * T * T / (T + 1108.0);
    H.eg[0] = 1.1557 - shift;
    H.eg[1] = 2.5 - shift;
    H.egd = 3.2 - shift;
    const double ep[2] = {1.827e-2, 5.773e-2};
    for (int i = 0; i < 2; ++i) {
        H.absorb[i] = std::exp(ep[i] / (kB * T)) - 1.0;
        H.emit[i] = 1.0 - std::exp(-ep[i] / (kB * T));
    }
    build_surfaces(c);
    c->have_presc = true;
    build_cull_order(c);
    c->dirty = true;
    const phx_status st = build_escape_table(c);
    if (st != PHX_OK || !c->have_phys) return st;
    // the physics parameters' derived tables depend on the silicon and the start plane
    const phx_physics keep = c->phys;
    c->have_phys = false;
    return phx_load_physics(c, &keep);
}

phx_status phx_set_perturbation(phx_ctx c, const double* theta, int32_t n) {
    if (!c) return PHX_ERR_INVALID;
    if (!theta || n != PHX_N_THETA)
        return fail(c, PHX_ERR_INVALID, "perturbation needs %d values", PHX_N_THETA);
    if (!finite_all(theta, PHX_N_THETA)) return fail(c, PHX_ERR_INVALID, "non-finite theta");
    std::memcpy(c->theta, theta, sizeof(c->theta));
    if (c->have_presc) build_surfaces(c);
    c->dirty = true;
    return PHX_OK;
}

phx_status phx_load_coatings(phx_ctx c, const float* t, int32_t n_coat, int32_t n_s,
                             int32_t n_lam, double s_max, double lam0, double dlam) {
    if (!c) return PHX_ERR_INVALID;
    if (!t || n_coat <= 0 || n_s < 2 || n_lam < 2 || n_lam > 8192 || !(s_max > 0) || !(dlam > 0) ||
        !std::isfinite(lam0) || !std::isfinite(s_max) || !std::isfinite(dlam))
        return fail(c, PHX_ERR_INVALID, "bad coating table description");
    const size_t n = (size_t)n_coat * n_s * n_lam;
    std::vector<float> mx((size_t)n_coat * n_lam, 0.0f);
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(t[i]) || t[i] < 0.0f || t[i] > 1.0f)
            return fail(c, PHX_ERR_INVALID, "coating value %zu not in [0, 1]", i);
    for (int k = 0; k < n_coat; ++k)
        for (int s = 0; s < n_s; ++s)
            for (int l = 0; l < n_lam; ++l) {
                float v = t[((size_t)k * n_s + s) * n_lam + l];
                float& m = mx[(size_t)k * n_lam + l];
                if (v > m) m = v;
            }
    // pre-roll thresholds per wavelength column pair (the test compares the roulette word)
    std::vector<int64_t> thr(mx.size());
    for (int k = 0; k < n_coat; ++k)
        for (int l = 0; l < n_lam; ++l) {
            const int l0 = std::min(l, n_lam - 2);
            const double m = std::fmax((double)mx[(size_t)k * n_lam + l0],
                                       (double)mx[(size_t)k * n_lam + l0 + 1]);
            thr[(size_t)k * n_lam + l] = word_threshold(m + 1e-12);
        }
    if (set_device(c) != PHX_OK) return PHX_ERR_HIP;
    free_dev(c->d_coat);
    free_dev(c->d_coat_thr);
    hipError_t e = hipMalloc((void**)&c->d_coat, n * sizeof(float));
    if (e == hipSuccess) e = hipMalloc((void**)&c->d_coat_thr, thr.size() * sizeof(int64_t));
    if (e != hipSuccess) return fail(c, PHX_ERR_NOMEM, "coating tables: %s", hipGetErrorString(e));
    e = hipMemcpy(c->d_coat, t, n * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(c->d_coat_thr, thr.data(), thr.size() * sizeof(int64_t),
                      hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(c, e, "hipMemcpy(coatings)");
    DevParams& H = c->host;
    H.n_coat = n_coat;
    H.n_s = n_s;
    H.n_lam = n_lam;
    H.inv_s_step = (double)(n_s - 1) / s_max;
    H.lam0 = lam0;
    H.inv_dlam = 1.0 / dlam;
    H.coat = c->d_coat;
    H.coat_thr = c->d_coat_thr;
    H.coat_r = nullptr;        // new tables: the reflectances must be loaded again
    c->have_refl = false;
    c->coat_max = mx;
    c->have_coat = true;
    build_cull_order(c);
    c->dirty = true;
    return build_escape_table(c);
}

phx_status phx_load_physics(phx_ctx c, const phx_physics* x) {
    if (!c) return PHX_ERR_INVALID;
    if (!x) return fail(c, PHX_ERR_INVALID, "null physics parameters");
    if (!c->have_presc) return fail(c, PHX_ERR_STATE, "load a prescription first");
    const double half_pi = 0.5 * M_PI;
    const double v[] = {x->zenith_angle, x->zenith_pa, x->aerosol_tau0, x->aerosol_gamma,
                        x->air_pressure, x->air_water, x->air_temperature,
                        x->dispersion_lambda0, x->dome_sigma, x->halo_fraction, x->halo_index,
                        x->halo_r0, x->halo_max, x->dead_layer};
    if (!finite_all(v, (int)(sizeof(v) / sizeof(v[0]))))
        return fail(c, PHX_ERR_INVALID, "non-finite physics parameter");
    if (!(x->zenith_angle >= 0.0 && x->zenith_angle < half_pi))
        return fail(c, PHX_ERR_INVALID, "zenith angle outside [0, pi/2)");
    if (!(x->aerosol_tau0 >= 0.0) || !(x->air_pressure >= 0.0) || !(x->air_water >= 0.0) ||
        !(x->air_temperature > -273.15) || !(x->dispersion_lambda0 > 0.16e-6))
        return fail(c, PHX_ERR_INVALID, "bad aerosol or air parameters");
    if (!(x->dome_sigma >= 0.0) || !(x->halo_fraction >= 0.0 && x->halo_fraction <= 1.0) ||
        !(x->halo_index > 2.0 && x->halo_index <= 6.0) || !(x->halo_r0 > 0.0) ||
        !(x->halo_max > 0.0 && x->halo_max < half_pi) || !(x->dead_layer >= 0.0))
        return fail(c, PHX_ERR_INVALID, "bad dome, halo or dead-layer parameters");
    if (x->spider_vanes < 0 || x->spider_vanes > 8)
        return fail(c, PHX_ERR_INVALID, "spider vanes %d outside 0..8", x->spider_vanes);
    if (x->spider_vanes > 0) {
        const double g[] = {x->spider_angle, x->spider_width, x->spider_r_inner,
                            x->spider_r_outer, x->spider_z_low, x->spider_z_high};
        if (!finite_all(g, 6) || !(x->spider_width > 0.0) ||
            !(x->spider_r_inner < x->spider_r_outer) || !(x->spider_z_low < x->spider_z_high) ||
            !(x->spider_z_high <= c->presc.z_start))
            return fail(c, PHX_ERR_INVALID, "bad spider geometry");
    }
    {
        const double g[] = {x->kick_r0, x->kick_L0, x->kick_kappa_crit, x->kick_kappa_max};
        if (!finite_all(g, 4) || !finite_all(x->kick_fraction, PHX_MAX_LAYERS) ||
            !(x->kick_r0 > 0.0) || !(x->kick_L0 > 0.0) || !(x->kick_kappa_crit > 0.0) ||
            !(x->kick_kappa_crit < x->kick_kappa_max))
            return fail(c, PHX_ERR_INVALID, "bad second-kick parameters");
        for (int i = 0; i < PHX_MAX_LAYERS; ++i)
            if (!(x->kick_fraction[i] >= 0.0))
                return fail(c, PHX_ERR_INVALID, "negative second-kick fraction %d", i);
    }
    {
        const double g[] = {x->si_voltage, x->si_n_bulk, x->si_n_back, x->si_s_back,
                            x->si_n_front, x->si_s_front, x->si_z_collect};
        if (!finite_all(g, 7) || !(x->si_voltage > 0.0) || !(x->si_n_bulk >= 0.0) ||
            !(x->si_n_back >= 0.0) || !(x->si_n_front >= 0.0) || !(x->si_s_back > 0.0) ||
            !(x->si_s_front > 0.0) || !(x->si_z_collect >= 0.0) ||
            !(x->si_z_collect < c->presc.si_thickness))
            return fail(c, PHX_ERR_INVALID, "bad silicon field parameters");
    }
    phx::DevPhysics X{};   // assigned to the parameter block only once every check passed
    {
        // phase variance of each layer's modes in [kappa_crit, kappa_max]: 2 pi int Phi kappa
        const double k0 = 2.0 * M_PI / x->kick_L0;
        const double A0 = std::pow(x->kick_kappa_crit * x->kick_kappa_crit + k0 * k0, -5.0 / 6.0);
        const double A1 = std::pow(x->kick_kappa_max * x->kick_kappa_max + k0 * k0, -5.0 / 6.0);
        X.kick_A0 = A0;
        X.kick_dA = A0 - A1;
        X.kick_k02 = k0 * k0;
        for (int i = 0; i < PHX_MAX_LAYERS; ++i) {
            const double cphi = 0.033 * (2.0 * M_PI) / 0.423 * x->kick_fraction[i] *
                                std::pow(x->kick_r0, -5.0 / 3.0);
            X.kick_s2[i] = (2.0 * M_PI) * cphi * 0.6 * (A0 - A1);
            X.kick_p0[i] = std::exp(-X.kick_s2[i]);
            if (!(X.kick_s2[i] <= 2.0))
                return fail(c, PHX_ERR_INVALID, "second-kick phase variance %g of layer %d above 2",
                            X.kick_s2[i], i);
        }
    }
    X.airmass = 1.0 / std::cos(x->zenith_angle);
    X.tau0 = x->aerosol_tau0;
    X.gamma = x->aerosol_gamma;
    // Filippenko index of air: factors of the dry bracket and of the water term
    const double T = x->air_temperature, P = x->air_pressure;
    X.disp_tanz = std::tan(x->zenith_angle);
    X.disp_cx = std::cos(x->zenith_pa);
    X.disp_cy = std::sin(x->zenith_pa);
    X.disp_pt = P * (1.0 + (1.049 - 0.0157 * T) * 1e-6 * P) / (720.883 * (1.0 + 0.003661 * T));
    X.disp_w = x->air_water / (1.0 + 0.003661 * T);
    const double lu = x->dispersion_lambda0 * 1e6;
    X.disp_s0 = 1.0 / (lu * lu);
    X.disp_b0 = 64.328 + 29498.1 / (146.0 - X.disp_s0) + 255.4 / (41.0 - X.disp_s0);
    X.dome_sigma = x->dome_sigma;
    // halo: proposal density x (1 + x^2)^(-n/2) truncated at x_max, acceptance bound 2^(n/2 - 1)
    const double n = x->halo_index, xmax = x->halo_max / x->halo_r0;
    X.halo_f = x->halo_fraction;
    X.halo_n = n;
    X.halo_r0 = x->halo_r0;
    X.halo_e = 1.0 - 0.5 * n;
    X.halo_fq = 1.0 - std::pow(1.0 + xmax * xmax, X.halo_e);
    X.halo_inv_m = std::pow(2.0, 1.0 - 0.5 * n);
    X.dead = x->dead_layer;
    X.vanes = x->spider_vanes;
    for (int k = 0; k < x->spider_vanes; ++k) {
        const double a = x->spider_angle + 2.0 * M_PI * k / x->spider_vanes;
        X.vane_c[k] = std::cos(a);
        X.vane_s[k] = std::sin(a);
    }
    X.vane_w = x->spider_width;
    X.vane_hw = 0.5 * x->spider_width;
    X.vane_r0 = x->spider_r_inner;
    X.vane_r1 = x->spider_r_outer;
    X.vane_z0 = x->spider_z_low;
    X.vane_z1 = x->spider_z_high;
    X.vane_zm = 0.5 * (x->spider_z_low + x->spider_z_high);
    // field diffusion: sigma^2 against depth, the collection time accumulated from the
    // collection height upward by 4-point Gauss-Legendre per table cell
    std::vector<double> sig2(phx::kSig2Cells + 1, 0.0);
    bool ok = true;
    {
        const double t = c->presc.si_thickness, T = c->presc.si_temperature, zc = x->si_z_collect;
        const double qe = 1.602176634e-19, kT_q = 1.380649e-23 * T / qe;
        const double k_eps = qe / (8.8541878128e-12 * 11.7);
        auto field = [&](double z) {
            return x->si_voltage / t +
                   k_eps * (x->si_n_bulk * (z - t) +
                            x->si_n_back * x->si_s_back * (std::exp((z - t) / x->si_s_back) - 1.0) +
                            x->si_n_front * x->si_s_front *
                                (std::exp(-t / x->si_s_front) - std::exp(-z / x->si_s_front)));
        };
        const double vm = 1.53e9 * std::pow(T, -0.87), Ec = 1.01 * std::pow(T, 1.55);
        const double beta = 2.57e-2 * std::pow(T, 0.66);
        auto mobility = [&](double E) {   // m^2/Vs at |E| V/m
            const double r = std::fabs(E) * 1e-2 / Ec;
            return 1e-4 * (vm / Ec) / std::pow(1.0 + std::pow(r, beta), 1.0 / beta);
        };
        const double gx[4] = {-0.8611363115940526, -0.3399810435848563, 0.3399810435848563,
                              0.8611363115940526};
        const double gw[4] = {0.3478548451374538, 0.6521451548625461, 0.6521451548625461,
                              0.3478548451374538};
        const int N = phx::kSig2Cells;
        const double dmax = t - zc, h = dmax / N;
        double tc = 0.0;   // collection time from height zc
        for (int k = N; k >= 0; --k) {
            const double z = t - h * k;   // height of table entry k (depth h k)
            if (k < N) {
                const double mid = z - 0.5 * h;   // the cell between heights z - h and z
                double cell = 0.0;
                for (int i = 0; i < 4; ++i) {
                    const double zi = mid + 0.5 * h * gx[i];
                    const double E = field(zi);
                    if (!(E > 0.0)) ok = false;
                    cell += gw[i] / (mobility(E) * E);
                }
                tc += 0.5 * h * cell;
            }
            const double E = field(z);
            if (!(E > 0.0)) ok = false;
            sig2[k] = 2.0 * mobility(E) * kT_q * tc;
        }
        X.n_sig2 = N;
        X.sig2_dmax = dmax;
        X.sig2_inv_step = N / dmax;
    }
    if (set_device(c) != PHX_OK) return PHX_ERR_HIP;
    if (!c->d_sig2) {
        const hipError_t e = hipMalloc((void**)&c->d_sig2, sig2.size() * sizeof(double));
        if (e != hipSuccess) return fail(c, PHX_ERR_NOMEM, "sigma table: %s", hipGetErrorString(e));
    }
    {
        const hipError_t e = hipMemcpy(c->d_sig2, sig2.data(), sig2.size() * sizeof(double),
                                       hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(c, e, "hipMemcpy(sigma table)");
    }
    X.sig2 = c->d_sig2;
    c->host.ph = X;
    c->phys = *x;
    c->field_ok = ok;
    c->have_phys = true;
    c->dirty = true;
    return PHX_OK;
}

phx_status phx_load_reflectance(phx_ctx c, const float* r, int32_t n_coat, int32_t n_s,
                                int32_t n_lam) {
    if (!c) return PHX_ERR_INVALID;
    if (!c->have_coat) return fail(c, PHX_ERR_STATE, "load the coatings first");
    if (!r || n_coat != c->host.n_coat || n_s != c->host.n_s || n_lam != c->host.n_lam)
        return fail(c, PHX_ERR_INVALID, "reflectance tables must match the coating tables");
    const size_t n = (size_t)n_coat * n_s * n_lam;
    std::vector<float> t(n);
    if (set_device(c) != PHX_OK) return PHX_ERR_HIP;
    hipError_t e = hipMemcpy(t.data(), c->d_coat, n * sizeof(float), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(c, e, "hipMemcpy(coatings)");
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(r[i]) || r[i] < 0.0f || (double)r[i] > 1.0 - (double)t[i] + 1e-6)
            return fail(c, PHX_ERR_INVALID, "reflectance %zu outside [0, 1 - T]", i);
    if (!c->d_coat_r) {
        e = hipMalloc((void**)&c->d_coat_r, n * sizeof(float));
        if (e != hipSuccess) {
            c->d_coat_r = nullptr;
            return fail(c, PHX_ERR_NOMEM, "reflectance tables: %s", hipGetErrorString(e));
        }
    }
    e = hipMemcpy(c->d_coat_r, r, n * sizeof(float), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(c, e, "hipMemcpy(reflectance)");
    c->host.coat_r = c->d_coat_r;
    c->have_refl = true;
    c->dirty = true;
    return PHX_OK;
}

phx_status phx_load_screens(phx_ctx c, const phx_atmosphere* a, const float* opd, int64_t n_floats,
                            void* stream) {
    if (!c) return PHX_ERR_INVALID;
    if (!a || !opd) return fail(c, PHX_ERR_INVALID, "null atmosphere or screen pointer");
    if (a->n_layers < 1 || a->n_layers > PHX_MAX_LAYERS || a->n_scales < 1 ||
        a->n_scales > PHX_MAX_SCALES)
        return fail(c, PHX_ERR_INVALID, "layers %d / scales %d out of range", a->n_layers,
                    a->n_scales);
    const int N = a->screen_n;
    if (N < 4 || (N & (N - 1)) != 0)
        return fail(c, PHX_ERR_INVALID, "screen side %d must be a power of two >= 4", N);
    const int64_t want = (int64_t)a->n_layers * a->n_scales * N * N;
    if (n_floats != want)
        return fail(c, PHX_ERR_INVALID, "screen buffer has %lld floats, expected %lld",
                    (long long)n_floats, (long long)want);
    for (int i = 0; i < a->n_layers; ++i) {
        const double v[3] = {a->height[i], a->wind[i][0], a->wind[i][1]};
        if (!finite_all(v, 3)) return fail(c, PHX_ERR_INVALID, "layer %d not finite", i);
        if (i > 0 && !(a->height[i] > a->height[i - 1]))
            return fail(c, PHX_ERR_INVALID, "layer heights must increase");
    }
    for (int s = 0; s < a->n_scales; ++s)
        if (!(a->pixel[s] > 0) || !std::isfinite(a->pixel[s]))
            return fail(c, PHX_ERR_INVALID, "scale %d pixel not positive", s);
    if (!(a->lambda_ref > 0)) return fail(c, PHX_ERR_INVALID, "lambda_ref not positive");
    if (set_device(c) != PHX_OK) return PHX_ERR_HIP;
    hipStream_t st = (hipStream_t)stream;
    if ((size_t)want != c->grad_elems) {
        free_dev(c->d_grad);
        c->grad_elems = 0;
        hipError_t e = hipMalloc((void**)&c->d_grad, (size_t)want * 2 * sizeof(float4));
        if (e != hipSuccess) return fail(c, PHX_ERR_NOMEM, "gradient screens: %s",
                                         hipGetErrorString(e));
        c->grad_elems = (size_t)want;
    }
    const int planes = a->n_layers * a->n_scales;
    unsigned int* d_gmax = nullptr;
    hipError_t e = hipMalloc((void**)&d_gmax, planes * sizeof(unsigned int));
    if (e != hipSuccess) return fail(c, PHX_ERR_NOMEM, "screen maxima");
    e = hipMemsetAsync(d_gmax, 0, planes * sizeof(unsigned int), st);
    if (e == hipSuccess)
        e = phx::launch_gradients(opd, c->d_grad, a->n_layers, a->n_scales, N, a->pixel, d_gmax, st);
    std::vector<unsigned int> gm(planes, 0u);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e == hipSuccess)
        e = hipMemcpy(gm.data(), d_gmax, planes * sizeof(unsigned int), hipMemcpyDeviceToHost);
    free_dev(d_gmax);
    if (e != hipSuccess) return hip_fail(c, e, "gradient kernel");
    c->grad_max.assign(planes, 0.0);
    for (int i = 0; i < planes; ++i) {
        float f;
        std::memcpy(&f, &gm[i], sizeof(f));
        if (!std::isfinite(f)) {
            // the gradient screens now hold this load's values: no screens are usable
            c->have_screens = false;
            c->grad_max.clear();
            return fail(c, PHX_ERR_INVALID,
                        "screen plane %d (layer %d, scale %d) holds a NaN or infinite value", i,
                        i / a->n_scales, i % a->n_scales);
        }
        c->grad_max[i] = (double)f;
    }
    DevParams& H = c->host;
    H.n_layers = a->n_layers;
    H.n_scales = a->n_scales;
    H.screen_n = N;
    for (int i = 0; i < a->n_layers; ++i) {
        H.height[i] = a->height[i];
        H.wind[i][0] = a->wind[i][0];
        H.wind[i][1] = a->wind[i][1];
    }
    for (int s = 0; s < a->n_scales; ++s) H.inv_pix[s] = 1.0 / a->pixel[s];
    H.lambda_ref = a->lambda_ref;
    H.grad = c->d_grad;
    c->have_screens = true;
    c->dirty = true;
    return PHX_OK;
}

phx_status phx_load_sources(phx_ctx c, const phx_source* src, int32_t n_src, const double* edges,
                            const double* flux, int32_t n_sed, int32_t sed_k) {
    if (!c) return PHX_ERR_INVALID;
    if (!src || n_src <= 0) return fail(c, PHX_ERR_INVALID, "no sources");
    if (n_sed < 0 || (n_sed > 0 && (!edges || !flux || sed_k < 1 || sed_k > 65535)))
        return fail(c, PHX_ERR_INVALID, "bad SED table");
    std::vector<DevSource> ds(n_src);
    for (int i = 0; i < n_src; ++i) {
        const phx_source& s = src[i];
        const double v[] = {s.xi, s.eta, s.lambda_lo, s.lambda_hi, s.redshift, s.sersic_n,
                            s.sersic_bn, s.sersic_a, s.sersic_b, s.sersic_pa};
        if (!finite_all(v, sizeof(v) / sizeof(v[0])))
            return fail(c, PHX_ERR_INVALID, "source %d: non-finite field", i);
        if (!(s.xi * s.xi + s.eta * s.eta < 1.0))
            return fail(c, PHX_ERR_INVALID, "source %d: direction outside the unit disk", i);
        if (s.kind != 0 && s.kind != 1) return fail(c, PHX_ERR_INVALID, "source %d: kind", i);
        if (s.kind == 1 && !(s.sersic_n > 0 && s.sersic_bn > 0 && s.sersic_a >= 0 && s.sersic_b >= 0))
            return fail(c, PHX_ERR_INVALID, "source %d: Sersic parameters", i);
        if (s.sed >= n_sed || s.sed < -1) return fail(c, PHX_ERR_INVALID, "source %d: sed index", i);
        if (s.sed < 0 && !(s.lambda_lo > 0 && s.lambda_hi >= s.lambda_lo))
            return fail(c, PHX_ERR_INVALID, "source %d: wavelength band", i);
        if (!(s.redshift > -1.0)) return fail(c, PHX_ERR_INVALID, "source %d: redshift", i);
        DevSource& d = ds[i];
        d.xi = s.xi;
        d.eta = s.eta;
        d.nz = -std::sqrt(1.0 - s.xi * s.xi - s.eta * s.eta);
        d.lambda_lo = s.lambda_lo;
        d.lambda_span = s.lambda_hi - s.lambda_lo;
        d.redshift1 = 1.0 + s.redshift;
        d.sersic_n = s.sersic_n;
        d.sersic_bn = s.sersic_bn;
        d.sersic_a = s.sersic_a;
        d.sersic_b = s.sersic_b;
        d.cos_pa = std::cos(s.sersic_pa);
        d.sin_pa = std::sin(s.sersic_pa);
        d.kind = s.kind;
        d.sed = s.sed;
        d.n_photons = s.n_photons;
    }
    // SED photon CDFs (section 2.2): bin weight = f_lambda x width x centre wavelength (flux over
    // photon energy), accumulated in order and normalised; CDF[K] = 1 exactly.
    std::vector<double> cdf;
    std::vector<uint16_t> guide;
    if (n_sed > 0) {
        for (int k = 0; k < sed_k; ++k)
            if (!(edges[k + 1] > edges[k]) || !(edges[k] > 0))
                return fail(c, PHX_ERR_INVALID, "SED edges must be positive and increasing");
        c->sed_lo = edges[0];
        cdf.assign((size_t)n_sed * (sed_k + 1), 0.0);
        for (int s = 0; s < n_sed; ++s) {
            double* C = cdf.data() + (size_t)s * (sed_k + 1);
            const double* f = flux + (size_t)s * sed_k;
            C[0] = 0.0;
            for (int k = 0; k < sed_k; ++k) {
                if (!(f[k] >= 0) || !std::isfinite(f[k]))
                    return fail(c, PHX_ERR_INVALID, "SED %d bin %d negative or not finite", s, k);
                const double lo = edges[k], hi = edges[k + 1];
                C[k + 1] = C[k] + f[k] * (hi - lo) * (0.5 * (lo + hi));
            }
            const double total = C[sed_k];
            if (!(total > 0)) return fail(c, PHX_ERR_INVALID, "SED %d is zero", s);
            for (int k = 1; k < sed_k; ++k) C[k] = C[k] / total;
            C[sed_k] = 1.0;
        }
        // search guide: the first bin k with CDF[k + 1] > j / kSedGuide (the same predicate as
        // the device search, so the guided search returns the same bin)
        guide.assign((size_t)n_sed * (phx::kSedGuide + 1), 0);
        for (int s = 0; s < n_sed; ++s) {
            const double* C = cdf.data() + (size_t)s * (sed_k + 1);
            uint16_t* G = guide.data() + (size_t)s * (phx::kSedGuide + 1);
            int k = 0;
            for (int j = 0; j < phx::kSedGuide; ++j) {
                const double u = (double)j / phx::kSedGuide;
                while (k < sed_k - 1 && !(C[k + 1] > u)) ++k;
                G[j] = (uint16_t)k;
            }
            G[phx::kSedGuide] = (uint16_t)(sed_k - 1);
        }
    }
    if (set_device(c) != PHX_OK) return PHX_ERR_HIP;
    free_dev(c->d_src);
    free_dev(c->d_cdf);
    free_dev(c->d_guide);
    free_dev(c->d_edges);
    hipError_t e = hipMalloc((void**)&c->d_src, ds.size() * sizeof(DevSource));
    if (e == hipSuccess && n_sed > 0) e = hipMalloc((void**)&c->d_cdf, cdf.size() * sizeof(double));
    if (e == hipSuccess && n_sed > 0)
        e = hipMalloc((void**)&c->d_guide, guide.size() * sizeof(uint16_t));
    if (e == hipSuccess && n_sed > 0)
        e = hipMalloc((void**)&c->d_edges, (size_t)(sed_k + 1) * sizeof(double));
    if (e != hipSuccess) return fail(c, PHX_ERR_NOMEM, "sources: %s", hipGetErrorString(e));
    e = hipMemcpy(c->d_src, ds.data(), ds.size() * sizeof(DevSource), hipMemcpyHostToDevice);
    if (e == hipSuccess && n_sed > 0)
        e = hipMemcpy(c->d_cdf, cdf.data(), cdf.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess && n_sed > 0)
        e = hipMemcpy(c->d_guide, guide.data(), guide.size() * sizeof(uint16_t),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess && n_sed > 0)
        e = hipMemcpy(c->d_edges, edges, (size_t)(sed_k + 1) * sizeof(double),
                      hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(c, e, "hipMemcpy(sources)");
    c->src.assign(src, src + n_src);
    c->src_version += 1;
    c->graphs_clear();
    DevParams& H = c->host;
    H.src = c->d_src;
    H.sed_cdf = c->d_cdf;
    H.sed_guide = c->d_guide;
    H.sed_edges = c->d_edges;
    H.sed_k = n_sed > 0 ? sed_k : 0;
    c->have_src = true;
    c->dirty = true;
    return PHX_OK;
}

}  // extern "C"

namespace {

constexpr uint32_t kExtraFlags = PHX_F_AEROSOL | PHX_F_DISPERSION | PHX_F_DOME | PHX_F_HALO |
                                 PHX_F_SPIDER | PHX_F_DEAD_LAYER | PHX_F_SECOND_KICK |
                                 PHX_F_FIELD_DIFFUSION;

// Radii of the pupil annulus outside which a photon cannot reach the primary's clear aperture:
// the aperture widened by a bound on the atmospheric displacement at the primary.  Each layer i
// turns the ray by at most kick_max x (sum over scales of the screen's largest gradient norm; a
// bilinear value never exceeds its corners), and the turn displaces the landing point by at most
// that angle x (h_i + |z| of the primary) / min |n_z|; the sum over layers is taken with a factor
// 1.1 for the second-order terms (renormalisation, the sag slope at the displaced point, each
// below 1 %).
void set_cull_radii(phx_ctx c, const phx_trace_args* a, phx::Launch& L) {
    L.cull_r2_lo = -1.0;
    L.cull_r2_hi = INFINITY;
    // kicks at the telescope entrance (unbounded normal dome kick, halo, spider diffraction) and
    // the second kick (up to 8 scatterings per layer, each up to lambda_ref kappa_max / 2 pi)
    // move the landing point on the primary without a useful bound
    if (a->flags & (PHX_F_DOME | PHX_F_HALO | PHX_F_SPIDER | PHX_F_SECOND_KICK)) return;
    const phx::DevSurface& s0 = c->host.surf[0];
    if (s0.moved || c->presc.n_surfaces < 2) return;
    double D = 1e-6;
    if (a->flags & PHX_F_ATMOSPHERE) {
        if (!c->have_screens || c->grad_max.empty()) return;
        double lam_min = INFINITY, nz_min = 1.0;
        for (int s = a->src_begin; s < a->src_end; ++s) {
            const phx_source& q = c->src[s];
            const double lo = (q.sed >= 0 ? c->sed_lo : q.lambda_lo) * (1.0 + q.redshift);
            lam_min = std::min(lam_min, lo);
            nz_min = std::min(nz_min, std::sqrt(std::max(0.0, 1.0 - q.xi * q.xi - q.eta * q.eta)));
        }
        if (!(lam_min > 0.0) || !(nz_min > 0.5)) return;
        const double kick = std::pow(lam_min / c->host.lambda_ref, -0.2);
        // |z| of the primary over the sampled annulus
        const double R = s0.r_out + a->pupil_margin;
        const double arg = std::max(0.0, 1.0 - s0.kappa1 * s0.c * s0.c * R * R);
        double zmax = std::fabs(s0.t[2]) + std::fabs(s0.c) * R * R / (1.0 + std::sqrt(arg));
        for (int i = 0; i < 8; ++i) zmax += std::fabs(s0.alpha[i]) * std::pow(R, i + 3);
        for (int j = 0; j < phx::kNZern; ++j) zmax += 8.0 * std::fabs(c->theta[10 + j]);
        double sum = 0.0;
        const int S = c->host.n_scales;
        for (int i = 0; i < c->host.n_layers; ++i) {
            double g = 0.0;
            for (int k = 0; k < S; ++k) g += c->grad_max[(size_t)i * S + k];
            sum += kick * g * (std::fabs(c->host.height[i]) + zmax) / nz_min;
        }
        if (!std::isfinite(sum)) return;
        D += 1.1 * sum;
    }
    const double lo = s0.r_in - D, hi = s0.r_out + D;
    L.cull_r2_lo = lo > 0.0 ? lo * lo : -1.0;
    L.cull_r2_hi = hi * hi;
}

// Validation and the launch description (no device allocation, no upload): the sources, the
// photon total and the event capacity.  The prefix table is not set here.
phx_status validate_launch(phx_ctx c, const phx_trace_args* a, phx::Launch& L, bool need_image) {
    if (!a) return fail(c, PHX_ERR_INVALID, "null trace arguments");
    if (!c->have_presc || !c->have_src)
        return fail(c, PHX_ERR_STATE, "load a prescription and sources first");
    if ((a->flags & PHX_F_ATMOSPHERE) && !c->have_screens)
        return fail(c, PHX_ERR_STATE, "PHX_F_ATMOSPHERE without loaded screens");
    if ((a->flags & kExtraFlags) && !c->have_phys)
        return fail(c, PHX_ERR_STATE, "per-photon physics flags without phx_load_physics");
    if ((a->flags & PHX_F_GHOSTS) && !c->have_refl)
        return fail(c, PHX_ERR_STATE, "PHX_F_GHOSTS without loaded reflectance tables");
    if ((a->flags & PHX_F_FIELD_DIFFUSION) && !c->field_ok)
        return fail(c, PHX_ERR_INVALID, "silicon field model: E_z not positive across the device");
    if (a->flags & PHX_F_COATINGS)
        for (int k = 0; k < c->presc.n_surfaces; ++k) {
            const int co = c->presc.surf[k].coating;
            if (co >= 0 && !c->have_coat)
                return fail(c, PHX_ERR_STATE, "PHX_F_COATINGS without loaded coatings");
            if (co >= 0 && co >= c->host.n_coat)
                return fail(c, PHX_ERR_INVALID, "surface %d uses coating %d beyond the tables", k,
                            co);
        }
    const int n_src_all = (int)c->src.size();
    if (a->src_begin < 0 || a->src_end > n_src_all || a->src_begin >= a->src_end)
        return fail(c, PHX_ERR_INVALID, "source range [%d, %d) outside [0, %d)", a->src_begin,
                    a->src_end, n_src_all);
    if (need_image && !a->image_dev) return fail(c, PHX_ERR_INVALID, "null image");
    if (need_image && (a->flags & PHX_F_MOMENTS) && !a->moments_dev)
        return fail(c, PHX_ERR_INVALID, "PHX_F_MOMENTS without a moments buffer");
    if ((a->flags & PHX_F_MOMENTS) && c->presc.surf[c->presc.n_surfaces - 1].r_outer > 0.5)
        return fail(c, PHX_ERR_INVALID, "PHX_F_MOMENTS needs a detector radius <= 0.5 m");
    if (!std::isfinite(a->exposure) || a->exposure < 0 || !std::isfinite(a->pupil_margin) ||
        a->pupil_margin < 0)
        return fail(c, PHX_ERR_INVALID, "bad exposure or pupil margin");
    if (set_device(c) != PHX_OK) return PHX_ERR_HIP;
    L = phx::Launch{};
    L.seed = a->seed;
    L.flags = a->flags;
    L.src_begin = a->src_begin;
    L.n_src = a->src_end - a->src_begin;
    L.photon_begin = a->photon_begin;
    L.exposure = a->exposure;
    L.pupil_margin = a->pupil_margin;
    L.image = a->image_dev;
    L.stats = (unsigned long long*)a->stats_dev;
    L.moments = (unsigned long long*)a->moments_dev;
    L.events = a->events_dev;
    L.event_stride = a->event_stride;
    L.any_sersic = 0;
    for (int s = a->src_begin; s < a->src_end; ++s) L.any_sersic |= c->src[s].kind == 1;
    L.any_zernike = c->host.surf[0].zernike;
    set_cull_radii(c, a, L);
    if (a->photon_count > 0) {
        L.uniform_count = a->photon_count;
        if (a->photon_count > UINT64_MAX / (uint64_t)L.n_src)
            return fail(c, PHX_ERR_INVALID, "photon total overflows");
        L.total = a->photon_count * (uint64_t)L.n_src;
    } else {
        uint64_t total = 0;
        for (int s = 0; s < L.n_src; ++s) {
            const uint64_t n = c->src[a->src_begin + s].n_photons;
            if (total > UINT64_MAX - n) return fail(c, PHX_ERR_INVALID, "photon total overflows");
            total += n;
        }
        L.total = total;
    }
    if (a->photon_begin > UINT64_MAX - (L.total ? L.total : 0))
        return fail(c, PHX_ERR_INVALID, "photon index overflows");
    if (need_image && (a->flags & PHX_F_EVENTS)) {
        if (!a->events_dev || a->event_stride == 0)
            return fail(c, PHX_ERR_INVALID, "PHX_F_EVENTS needs events_dev and event_stride > 0");
        const uint64_t need = (L.total + a->event_stride - 1) / a->event_stride;
        if (need > a->event_capacity)
            return fail(c, PHX_ERR_CAPACITY, "events need %llu slots, capacity %llu",
                        (unsigned long long)need, (unsigned long long)a->event_capacity);
    }
    return PHX_OK;
}

// Blocks of 2^shift photons for the source guide: about four per source.
uint32_t guide_shift_of(uint64_t total, int n_src) {
    uint32_t shift = 0;
    while (shift < 40 && (total >> (shift + 1)) >= 4 * (uint64_t)n_src) ++shift;
    return shift;
}

// Chunk plan.  With the atmosphere every chunk has its survivors sorted by time (screen
// locality; a chunk of many sources keeps their order within a time bucket); traces of big
// sources are cut at source boundaries, traces of many small sources and adjoints evenly (the
// adjoint's optics kernel is the heavy stage and wants few, full chunks).  Returns the number of
// chunks; fills c->plan only if that is at most max_chunks.
uint64_t make_plan(phx_ctx c, const phx_trace_args* a, const phx::Launch& L, uint64_t chunk,
                   bool need_image, uint64_t max_chunks) {
    const bool atm = (a->flags & PHX_F_ATMOSPHERE) != 0;
    const bool per_source = need_image && atm && L.n_src > 1 &&
                            L.total / (uint64_t)L.n_src >= chunk / 8;
    uint64_t n = 0;
    if (per_source) {
        for (int s = 0; s < L.n_src; ++s) {
            const uint64_t n_s = L.uniform_count ? L.uniform_count
                                                 : c->src[a->src_begin + s].n_photons;
            n += (n_s + chunk - 1) / chunk;
        }
    } else {
        n = (L.total + chunk - 1) / chunk;
    }
    if (n > max_chunks) return n;
    c->plan.clear();
    if (per_source) {
        uint64_t start = 0;
        for (int s = 0; s < L.n_src; ++s) {
            const uint64_t n_s = L.uniform_count ? L.uniform_count
                                                 : c->src[a->src_begin + s].n_photons;
            for (uint64_t o = 0; o < n_s; o += chunk)
                c->plan.push_back({start + o, std::min(chunk, n_s - o), start, 1, s});
            start += n_s;
        }
    } else {
        for (uint64_t b = 0; b < L.total; b += chunk)
            c->plan.push_back({b, std::min(chunk, L.total - b), 0, atm ? 1 : 0,
                               L.n_src == 1 ? 0 : -1});
    }
    return n;
}

// Validation, uploads and workspace for a trace; fills the launch description.  May synchronise
// `st` (new prefix table, growing workspace, changed parameter block).
phx_status prepare(phx_ctx c, const phx_trace_args* a, hipStream_t st, phx::Launch& L,
                   phx::Workspace& W, bool need_image = true) {
    phx_status r = validate_launch(c, a, L, need_image);
    if (r != PHX_OK) return r;
    if (a->photon_count == 0) {
        std::vector<uint64_t> pre(L.n_src + 1, 0);
        for (int s = 0; s < L.n_src; ++s) pre[s + 1] = pre[s] + c->src[a->src_begin + s].n_photons;
        const bool same = c->prefix_valid && c->prefix_begin == a->src_begin &&
                          c->prefix_end == a->src_end && c->prefix_version == c->src_version;
        if (!same) {
            const uint32_t shift = guide_shift_of(L.total, L.n_src);
            const uint64_t nb = L.total ? ((L.total - 1) >> shift) + 1 : 1;
            std::vector<int32_t> guide(nb + 1);
            int s = 0;
            for (uint64_t b = 0; b < nb; ++b) {
                const uint64_t g = b << shift;
                while (s + 1 < L.n_src && pre[s + 1] <= g) ++s;
                guide[b] = s;
            }
            guide[nb] = L.n_src - 1;
            if (guide.size() > c->src_guide_cap) {
                hipError_t e = hipStreamSynchronize(st);
                if (e != hipSuccess) return hip_fail(c, e, "hipStreamSynchronize");
                free_dev(c->d_src_guide);
                c->src_guide_cap = 0;
                e = hipMalloc((void**)&c->d_src_guide, guide.size() * sizeof(int32_t));
                if (e != hipSuccess) return fail(c, PHX_ERR_NOMEM, "source guide");
                c->src_guide_cap = guide.size();
            }
            hipError_t e = hipStreamSynchronize(st);
            if (e == hipSuccess)
                e = hipMemcpy(c->d_src_guide, guide.data(), guide.size() * sizeof(int32_t),
                              hipMemcpyHostToDevice);
            if (e != hipSuccess) return hip_fail(c, e, "source guide upload");
            c->guide_shift = shift;
            if ((size_t)(L.n_src + 1) > c->prefix_cap) {
                hipError_t e = hipStreamSynchronize(st);
                if (e != hipSuccess) return hip_fail(c, e, "hipStreamSynchronize");
                free_dev(c->d_prefix);
                c->prefix_cap = 0;
                e = hipMalloc((void**)&c->d_prefix, (L.n_src + 1) * sizeof(uint64_t));
                if (e != hipSuccess) return fail(c, PHX_ERR_NOMEM, "prefix table");
                c->prefix_cap = L.n_src + 1;
            }
            // enqueued work may still read the previous table; the host vector must outlive
            // the copy: both are handled by doing it synchronously after the stream drains
            e = hipStreamSynchronize(st);
            if (e == hipSuccess)
                e = hipMemcpy(c->d_prefix, pre.data(), pre.size() * sizeof(uint64_t),
                              hipMemcpyHostToDevice);
            if (e != hipSuccess) return hip_fail(c, e, "prefix upload");
            c->prefix_valid = true;
            c->prefix_begin = a->src_begin;
            c->prefix_end = a->src_end;
            c->prefix_version = c->src_version;
        }
        L.prefix = c->d_prefix;
        L.src_guide = c->d_src_guide;
        L.guide_shift = c->guide_shift;
    }
    // Workspace: chunk = min(2^chunk_log2, total rounded up to a power of two); grows only
    const uint64_t max_chunk = 1ull << c->chunk_log2;
    uint64_t chunk = 1024;
    while (chunk < L.total && chunk < max_chunk) chunk <<= 1;
    if (chunk > c->ws_chunk) {
        hipError_t e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail(c, e, "hipStreamSynchronize");
        free_dev(c->d_survivors);
        free_dev(c->d_state);
        free_dev(c->d_bits);
        free_dev(c->d_bsum);
        free_dev(c->d_key);
        free_dev(c->d_hist);
        c->ws_chunk = 0;
        c->graphs_clear();
        e = hipMalloc((void**)&c->d_survivors, 2 * chunk * sizeof(uint32_t));
        if (e == hipSuccess) e = hipMalloc((void**)&c->d_state, 2 * 7 * chunk * sizeof(double));
        if (e == hipSuccess)
            e = hipMalloc((void**)&c->d_bits, 2 * ((chunk + 63) / 64) * sizeof(uint64_t));
        if (e == hipSuccess)
            e = hipMalloc((void**)&c->d_bsum, phx::compact_groups(chunk) * sizeof(unsigned int));
        if (e == hipSuccess) e = hipMalloc((void**)&c->d_key, 2 * chunk);
        if (e == hipSuccess)
            e = hipMalloc((void**)&c->d_hist, (2 * phx::bucket_groups(chunk) + 1) *
                                                  phx::kTimeBucketsMax * sizeof(unsigned int));
        if (e != hipSuccess) return fail(c, PHX_ERR_NOMEM, "trace workspace: %s",
                                         hipGetErrorString(e));
        c->ws_chunk = chunk;
    }
    chunk = std::min<uint64_t>(c->ws_chunk, max_chunk);
    const uint64_t n_chunks = make_plan(c, a, L, chunk, need_image, UINT64_MAX);
    if (n_chunks > c->counts_cap) {
        hipError_t e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail(c, e, "hipStreamSynchronize");
        free_dev(c->d_counts);
        free_dev(c->d_tiles);
        c->counts_cap = 0;
        c->graphs_clear();
        e = hipMalloc((void**)&c->d_counts, n_chunks * sizeof(unsigned int));
        if (e == hipSuccess) e = hipMalloc((void**)&c->d_tiles, 2 * n_chunks * sizeof(uint64_t));
        if (e != hipSuccess) return fail(c, PHX_ERR_NOMEM, "chunk counters");
        c->counts_cap = n_chunks;
    }
    W = phx::Workspace{c->d_survivors, c->d_counts, c->counts_cap, c->d_state, chunk,
                       (unsigned long long*)c->d_tiles, (unsigned long long*)c->d_bits,
                       c->d_bsum, c->d_key, c->d_hist, c->plan.data(), (uint64_t)c->plan.size(),
                       2};
    if (a->flags & PHX_F_GHOSTS) {
        // every traced photon of a chunk may leave one ghost start: a list of chunk entries
        // (14 doubles each; 7.5 GB for chunks of 2^26 photons); grows only
        if (chunk > c->ghost_cap || !c->d_ghost_ctr) {
            hipError_t e = hipStreamSynchronize(st);
            if (e != hipSuccess) return hip_fail(c, e, "hipStreamSynchronize");
            free_dev(c->d_ghost);
            c->ghost_cap = 0;
            c->graphs_clear();
            e = hipMalloc((void**)&c->d_ghost, chunk * phx::kGhostFields * sizeof(double));
            if (e == hipSuccess && !c->d_ghost_ctr)
                e = hipMalloc((void**)&c->d_ghost_ctr, 2 * sizeof(unsigned long long));
            if (e != hipSuccess) return fail(c, PHX_ERR_NOMEM, "ghost list: %s",
                                             hipGetErrorString(e));
            c->ghost_cap = chunk;
        }
        W.ghost_list = c->d_ghost;
        W.ghost_cap = c->ghost_cap;
        W.ghost_ctr = c->d_ghost_ctr;
    }
    if (c->cfg.pipeline) {
        if (!c->aux_stream) {
            hipError_t e = hipStreamCreateWithFlags(&c->aux_stream, hipStreamNonBlocking);
            if (e != hipSuccess) return hip_fail(c, e, "hipStreamCreate");
        }
        while (c->pipe_ev.size() < 3 * c->plan.size() + 1) {
            hipEvent_t ev = nullptr;
            hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
            if (e != hipSuccess) return hip_fail(c, e, "hipEventCreate");
            c->pipe_ev.push_back(ev);
        }
    }
    return upload_params(c, st);
}

phx::Pipe pipe_of(phx_ctx c) {
    phx::Pipe p;
    if (c->cfg.pipeline && c->aux_stream) {
        p.aux = c->aux_stream;
        p.ev = c->pipe_ev.data();
        p.n_ev = c->pipe_ev.size();
    }
    return p;
}

// Launches pipeline chunks over the context's two streams when the launch shape says so; in a
// launch being captured into a graph the second stream joins the capture through the pipeline's
// fork event and rejoins it through the final wait, so the hand-off events become graph edges.
// Only eager launches are timed.
phx_status enqueue(phx_ctx c, const phx::Launch& L, const phx::Workspace& W, hipStream_t st,
                   bool eager) {
    phx::Timing T;
    T.on = eager && c->timing;
    T.record = timing_record;
    T.self = c;
    hipError_t e = phx::launch_trace(c->dparams, L, W, c->n_cu, c->cfg, st, pipe_of(c), T);
    if (e != hipSuccess) return hip_fail(c, e, "trace kernel launch");
    return PHX_OK;
}

}  // namespace

extern "C" {

phx_status phx_trace(phx_ctx c, const phx_trace_args* a, void* stream) {
    if (!c) return PHX_ERR_INVALID;
    hipStream_t st = (hipStream_t)stream;
    phx::Launch L;
    phx::Workspace W;
    phx_status r = prepare(c, a, st, L, W);
    if (r != PHX_OK) return r;
    return enqueue(c, L, W, st, true);
}

phx_status phx_trace_noalloc(phx_ctx c, const phx_trace_args* a, void* stream) {
    if (!c) return PHX_ERR_INVALID;
    hipStream_t st = (hipStream_t)stream;
    phx::Launch L;
    phx_status r = validate_launch(c, a, L, true);
    if (r != PHX_OK) return r;
    if (a->flags & PHX_F_GHOSTS)
        return fail(c, PHX_ERR_INVALID,
                    "phx_trace_noalloc does not trace ghosts (their list needs context memory)");
    if (L.n_src > phx::kNoAllocMaxSources)
        return fail(c, PHX_ERR_CAPACITY, "phx_trace_noalloc traces at most %d sources, not %d",
                    phx::kNoAllocMaxSources, L.n_src);
    if (!c->scratch) return fail(c, PHX_ERR_STATE, "no scratch address for this device");
    if (L.total == 0) return upload_params(c, st);
    uint64_t chunk = 1024;
    const uint64_t max_chunk = 1ull << std::min(c->chunk_log2, phx::kNoAllocChunkLog2);
    while (chunk < L.total && chunk < max_chunk) chunk <<= 1;
    const uint64_t n_chunks = make_plan(c, a, L, chunk, true, phx::kNoAllocMaxChunks);
    if (n_chunks > phx::kNoAllocMaxChunks)
        return fail(c, PHX_ERR_CAPACITY,
                    "phx_trace_noalloc handles at most %llu chunks of %llu photons, not %llu",
                    (unsigned long long)phx::kNoAllocMaxChunks, (unsigned long long)chunk,
                    (unsigned long long)n_chunks);
    constexpr phx::ScratchLayout S = phx::scratch_layout();
    unsigned char* base = (unsigned char*)c->scratch;
    if (a->photon_count == 0 && L.n_src > 1) {
        // prefix table and source guide of this launch, built on the device in the scratch
        const uint32_t shift = guide_shift_of(L.total, L.n_src);
        const uint64_t nb = ((L.total - 1) >> shift) + 1;
        if (nb + 1 > phx::kNoAllocGuideMax)
            return fail(c, PHX_ERR_CAPACITY, "source guide of %llu blocks",
                        (unsigned long long)nb);
        L.prefix = (const uint64_t*)(base + S.prefix);
        L.src_guide = (const int32_t*)(base + S.guide);
        L.guide_shift = shift;
        const hipError_t e = phx::launch_prefix(c->d_src, a->src_begin, L.n_src,
                                                (uint64_t*)(base + S.prefix),
                                                (int32_t*)(base + S.guide), nb, shift, st);
        if (e != hipSuccess) return hip_fail(c, e, "prefix kernels");
    }
    const phx::Workspace W{(uint32_t*)(base + S.survivors), (unsigned int*)(base + S.counts),
                           phx::kNoAllocMaxChunks, (double*)(base + S.state), chunk,
                           (unsigned long long*)(base + S.tiles),
                           (unsigned long long*)(base + S.bits), (unsigned int*)(base + S.bsum),
                           (uint8_t*)(base + S.key), (unsigned int*)(base + S.hist),
                           c->plan.data(), (uint64_t)c->plan.size(), 1};
    r = upload_params(c, st);
    if (r != PHX_OK) return r;
    // every stage on the caller's stream, one buffer set, no timing events
    const hipError_t e = phx::launch_trace(c->dparams, L, W, c->n_cu, c->cfg, st, phx::Pipe{},
                                           phx::Timing{});
    if (e != hipSuccess) return hip_fail(c, e, "trace kernel launch");
    return PHX_OK;
}

phx_status phx_trace_batched(phx_ctx c, const phx_trace_args* a, void* stream) {
    if (!c) return PHX_ERR_INVALID;
    hipStream_t st = (hipStream_t)stream;
    phx::Launch L;
    phx::Workspace W;
    phx_status r = prepare(c, a, st, L, W);
    if (r != PHX_OK) return r;
    // graph key: the launch description, the workspace and the launch shape
    // (the launch description is value-initialised, so its padding is zero; the workspace
    // fields are appended one by one)
    std::string key((const char*)&L, sizeof(L));
    auto put = [&key](const void* p, size_t n) { key.append((const char*)p, n); };
    const void* ptrs[] = {W.survivors, W.counts, W.state, W.tiles, W.bits, W.bsum, W.key, W.hist,
                          W.ghost_list, W.ghost_ctr};
    put(ptrs, sizeof(ptrs));
    const uint64_t sizes[] = {W.n_chunks, W.chunk, W.n_plan, (uint64_t)W.buffers, W.ghost_cap};
    put(sizes, sizeof(sizes));
    put(W.plan, W.n_plan * sizeof(phx::ChunkSpan));
    put(&c->cfg, sizeof(c->cfg));
    auto it = c->graphs.find(key);
    if (it == c->graphs.end()) {
        if (c->graphs.size() >= 32) c->graphs_clear();
        if (!c->cap_stream) {
            hipError_t e = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking);
            if (e != hipSuccess) return hip_fail(c, e, "hipStreamCreate");
        }
        hipError_t e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed);
        if (e != hipSuccess) return hip_fail(c, e, "hipStreamBeginCapture");
        phx_status q = enqueue(c, L, W, c->cap_stream, false);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(c->cap_stream, &g);
        if (q != PHX_OK) {
            if (g) (void)hipGraphDestroy(g);
            return q;
        }
        if (e != hipSuccess) return hip_fail(c, e, "hipStreamEndCapture");
        hipGraphExec_t x = nullptr;
        e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return hip_fail(c, e, "hipGraphInstantiate");
        it = c->graphs.emplace(key, x).first;
    }
    hipError_t e = hipGraphLaunch(it->second, st);
    if (e != hipSuccess) return hip_fail(c, e, "hipGraphLaunch");
    return PHX_OK;
}

phx_status phx_adjoint(phx_ctx c, const phx_trace_args* a, const double* seed_dev,
                       double* grad_dev, double* jac_dev, uint64_t jac_stride,
                       uint64_t jac_capacity, void* stream) {
    if (!c) return PHX_ERR_INVALID;
    if (!a) return fail(c, PHX_ERR_INVALID, "null trace arguments");
    if (!seed_dev || !grad_dev) return fail(c, PHX_ERR_INVALID, "null seed or gradient buffer");
    if (a->flags & PHX_F_GHOSTS)
        return fail(c, PHX_ERR_INVALID, "the adjoint follows the sequential path: no ghosts");
    hipStream_t st = (hipStream_t)stream;
    phx_trace_args b = *a;
    // outputs of the forward trace are not produced; the pre-roll changes no converted photon
    b.flags &= ~(uint32_t)(PHX_F_EVENTS | PHX_F_MOMENTS);
    if (b.flags & PHX_F_COATINGS) b.flags |= PHX_F_CULL;
    b.image_dev = nullptr;
    b.stats_dev = nullptr;
    b.moments_dev = nullptr;
    b.events_dev = nullptr;
    phx::Launch L;
    phx::Workspace W;
    phx_status r = prepare(c, &b, st, L, W, false);
    if (r != PHX_OK) return r;
    if (jac_dev) {
        if (jac_stride == 0) return fail(c, PHX_ERR_INVALID, "jacobian stride 0");
        const uint64_t need = (L.total + jac_stride - 1) / jac_stride;
        if (need > jac_capacity)
            return fail(c, PHX_ERR_CAPACITY, "jacobian needs %llu slots, capacity %llu",
                        (unsigned long long)need, (unsigned long long)jac_capacity);
    }
    // Adjoint workspace: tape for every thread of one launch, one partial row per workgroup
    const uint64_t grid = (uint64_t)c->n_cu * c->adj_per_cu;
    const uint64_t threads = grid * phx::kThreads;
    const uint64_t n_chunks = W.n_plan;
    const uint64_t tape_need = (uint64_t)c->presc.n_surfaces * phx::kTapeFields * threads;
    const uint64_t rows_need = std::max<uint64_t>(n_chunks * grid, 1);
    if (tape_need > c->tape_cap || rows_need > c->rows_cap || !c->d_colsum) {
        hipError_t e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail(c, e, "hipStreamSynchronize");
        if (tape_need > c->tape_cap) {
            free_dev(c->d_tape);
            c->tape_cap = 0;
            e = hipMalloc((void**)&c->d_tape, tape_need * sizeof(double));
            if (e != hipSuccess) return fail(c, PHX_ERR_NOMEM, "adjoint tape");
            c->tape_cap = tape_need;
        }
        if (rows_need > c->rows_cap) {
            free_dev(c->d_partial);
            c->rows_cap = 0;
            e = hipMalloc((void**)&c->d_partial, rows_need * phx::kAdj * sizeof(double));
            if (e != hipSuccess) return fail(c, PHX_ERR_NOMEM, "adjoint partial sums");
            c->rows_cap = rows_need;
        }
        if (!c->d_colsum) {
            e = hipMalloc((void**)&c->d_colsum, phx::kAdj * sizeof(double));
            if (e != hipSuccess) return fail(c, PHX_ERR_NOMEM, "adjoint column sums");
        }
    }
    phx::Adjoint A;
    A.seed = seed_dev;
    A.partial = c->d_partial;
    A.tape = c->d_tape;
    A.tape_stride = threads;
    A.jac = jac_dev;
    A.jac_stride = jac_dev ? jac_stride : 1;
    A.jac_cap = jac_capacity;
    A.per_cu = c->adj_per_cu;
    phx::Timing T;
    T.on = c->timing;
    T.record = timing_record;
    T.self = c;
    hipError_t e = phx::launch_adjoint(c->dparams, L, W, c->n_cu, c->cfg, A, c->d_colsum, grad_dev,
                                       st, pipe_of(c), T);
    if (e != hipSuccess) return hip_fail(c, e, "adjoint kernel launch");
    return PHX_OK;
}

phx_status phx_adjoint_moments(phx_ctx c, const phx_trace_args* a, const uint64_t* moments_dev,
                               const double* dmom_dev, double* grad_dev, double* jac_dev,
                               uint64_t jac_stride, uint64_t jac_capacity, void* stream) {
    if (!c) return PHX_ERR_INVALID;
    if (!a) return fail(c, PHX_ERR_INVALID, "null trace arguments");
    if (!moments_dev || !dmom_dev)
        return fail(c, PHX_ERR_INVALID, "null moment words or moment gradient");
    const int n_src_all = (int)c->src.size();
    if (a->src_begin < 0 || a->src_end > n_src_all || a->src_begin >= a->src_end)
        return fail(c, PHX_ERR_INVALID, "source range [%d, %d) outside [0, %d)", a->src_begin,
                    a->src_end, n_src_all);
    if (set_device(c) != PHX_OK) return PHX_ERR_HIP;
    hipStream_t st = (hipStream_t)stream;
    const uint64_t n = (uint64_t)(a->src_end - a->src_begin);
    if (n > c->seed_cap) {
        hipError_t e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail(c, e, "hipStreamSynchronize");
        free_dev(c->d_seed);
        c->seed_cap = 0;
        e = hipMalloc((void**)&c->d_seed, n * 8 * sizeof(double));
        if (e != hipSuccess) return fail(c, PHX_ERR_NOMEM, "adjoint seeds");
        c->seed_cap = n;
    }
    hipError_t e = phx::launch_seeds((const unsigned long long*)moments_dev +
                                         (size_t)a->src_begin * PHX_MOMENT_WORDS,
                                     (int)n, dmom_dev, c->d_seed, st);
    if (e != hipSuccess) return hip_fail(c, e, "seed kernel launch");
    return phx_adjoint(c, a, c->d_seed, grad_dev, jac_dev, jac_stride, jac_capacity, stream);
}

phx_status phx_moments(phx_ctx c, const uint64_t* moments_dev, int32_t n_src, double* out_dev,
                       void* stream) {
    if (!c) return PHX_ERR_INVALID;
    if (n_src < 0 || (n_src > 0 && (!moments_dev || !out_dev)))
        return fail(c, PHX_ERR_INVALID, "null buffer or negative source count");
    if (set_device(c) != PHX_OK) return PHX_ERR_HIP;
    const hipError_t e = phx::launch_moments((const unsigned long long*)moments_dev, n_src,
                                             out_dev, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "moments kernel launch");
    return PHX_OK;
}

phx_status phx_read_image(phx_ctx c, const uint32_t* image_dev, uint32_t* image_host, int64_t n,
                          void* stream) {
    if (!c) return PHX_ERR_INVALID;
    if (!c->have_presc) return fail(c, PHX_ERR_STATE, "load a prescription first");
    const int64_t npix = (int64_t)c->presc.nx * c->presc.ny;
    if (!image_dev || !image_host || n != npix)
        return fail(c, PHX_ERR_INVALID, "null image or n = %lld, not nx ny = %lld", (long long)n,
                    (long long)npix);
    if (set_device(c) != PHX_OK) return PHX_ERR_HIP;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(image_host, image_dev, (size_t)n * sizeof(uint32_t),
                                  hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(c, e, "image copy");
    return PHX_OK;
}

phx_status phx_set_launch_config(phx_ctx c, const phx_launch_config* cfg) {
    if (!c) return PHX_ERR_INVALID;
    if (!cfg) return fail(c, PHX_ERR_INVALID, "null launch config");
    if (cfg->chunk_log2 < 16 || cfg->chunk_log2 > 27 || cfg->generate_blocks_per_cu < 1 ||
        cfg->generate_blocks_per_cu > 64 || cfg->front_blocks_per_cu < 1 ||
        cfg->front_blocks_per_cu > 64 || cfg->back_blocks_per_cu < 1 ||
        cfg->back_blocks_per_cu > 64 || (cfg->dynamic_tiles != 0 && cfg->dynamic_tiles != 1) ||
        (cfg->pipeline != 0 && cfg->pipeline != 1))
        return fail(c, PHX_ERR_INVALID, "launch config out of range");
    c->chunk_log2 = cfg->chunk_log2;
    c->cfg.generate_per_cu = cfg->generate_blocks_per_cu;
    c->cfg.front_per_cu = cfg->front_blocks_per_cu;
    c->cfg.back_per_cu = cfg->back_blocks_per_cu;
    c->cfg.dynamic = cfg->dynamic_tiles;
    c->cfg.pipeline = cfg->pipeline;
    return PHX_OK;
}

phx_status phx_get_launch_config(phx_ctx c, phx_launch_config* cfg) {
    if (!c) return PHX_ERR_INVALID;
    if (!cfg) return fail(c, PHX_ERR_INVALID, "null launch config");
    cfg->chunk_log2 = c->chunk_log2;
    cfg->generate_blocks_per_cu = c->cfg.generate_per_cu;
    cfg->front_blocks_per_cu = c->cfg.front_per_cu;
    cfg->back_blocks_per_cu = c->cfg.back_per_cu;
    cfg->dynamic_tiles = c->cfg.dynamic;
    cfg->pipeline = c->cfg.pipeline;
    return PHX_OK;
}

namespace {
// graph: time phx_trace_batched graph replays, else eager phx_trace launches
phx_status autotune(phx_ctx c, const phx_trace_args* sample, void* stream,
                    phx_launch_config* best, bool graph) {
    if (!c) return PHX_ERR_INVALID;
    if (!sample) return fail(c, PHX_ERR_INVALID, "null sample");
    if (!c->have_presc) return fail(c, PHX_ERR_STATE, "load a prescription first");
    if (set_device(c) != PHX_OK) return PHX_ERR_HIP;
    hipStream_t st = (hipStream_t)stream;
    // scratch outputs
    uint32_t* img = nullptr;
    unsigned long long* stats = nullptr;
    uint64_t* mom = nullptr;
    const size_t npix = (size_t)c->presc.nx * c->presc.ny;
    hipError_t e = hipMalloc((void**)&img, npix * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMalloc((void**)&stats, PHX_STATS_LEN * sizeof(uint64_t));
    if (e == hipSuccess && (sample->flags & PHX_F_MOMENTS))
        e = hipMalloc((void**)&mom, c->src.size() * PHX_MOMENT_WORDS * sizeof(uint64_t));
    if (e != hipSuccess) {
        free_dev(img);
        free_dev(stats);
        free_dev(mom);
        return fail(c, PHX_ERR_NOMEM, "autotune scratch");
    }
    phx_trace_args a = *sample;
    a.flags &= ~(uint32_t)PHX_F_EVENTS;
    a.image_dev = img;
    a.stats_dev = (uint64_t*)stats;
    a.moments_dev = mom;
    a.events_dev = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    phx_launch_config cur;
    phx_get_launch_config(c, &cur);
    phx_status status = PHX_OK;
    // the path the shape is for: eager launches or graph replays
    auto launch = [&]() -> phx_status {
        return graph ? phx_trace_batched(c, &a, st) : phx_trace(c, &a, st);
    };
    auto measure = [&](const phx_launch_config& k, float& ms_out) -> phx_status {
        phx_status r = phx_set_launch_config(c, &k);
        if (r != PHX_OK) return r;
        r = launch();   // warm-up (prepares, and captures a graph)
        if (r != PHX_OK) return r;
        float best_ms = 1e30f;
        for (int rep = 0; rep < 3; ++rep) {
            (void)hipEventRecord(e0, st);
            r = launch();
            if (r != PHX_OK) return r;
            (void)hipEventRecord(e1, st);
            if (hipEventSynchronize(e1) != hipSuccess) return fail(c, PHX_ERR_HIP, "sync");
            float ms = 0.0f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            best_ms = std::min(best_ms, ms);
        }
        ms_out = best_ms;
        return PHX_OK;
    };
    float cur_ms = 0.0f;
    status = measure(cur, cur_ms);
    // coordinate descent over the knobs, the chunk size and the schedule first (they set how
    // many chunks overlap and how the work is split, which the best optics and sky widths then
    // depend on); up to three passes, ending after a pass that changes nothing
    const int backs[] = {2, 3, 4, 6, 8, 12};
    const int fronts[] = {8, 16, 24, 32, 48, 64};
    const int gens[] = {2, 4, 8, 16};
    const int chunks[] = {24, 25, 26};
    for (int pass = 0; pass < 3 && status == PHX_OK; ++pass) {
        bool changed = false;
        for (int knob = 0; knob < 5 && status == PHX_OK; ++knob) {
            std::vector<phx_launch_config> cand;
            if (knob == 0) for (int v : chunks) { auto k = cur; k.chunk_log2 = v; cand.push_back(k); }
            if (knob == 1) for (int v = 0; v < 2; ++v) { auto k = cur; k.dynamic_tiles = v; cand.push_back(k); }
            if (knob == 2) for (int v : backs) { auto k = cur; k.back_blocks_per_cu = v; cand.push_back(k); }
            if (knob == 3) for (int v : fronts) { auto k = cur; k.front_blocks_per_cu = v; cand.push_back(k); }
            if (knob == 4) for (int v : gens) { auto k = cur; k.generate_blocks_per_cu = v; cand.push_back(k); }
            for (const auto& k : cand) {
                if (std::memcmp(&k, &cur, sizeof(k)) == 0) continue;
                float ms = 0.0f;
                status = measure(k, ms);
                if (status != PHX_OK) break;
                if (ms < cur_ms) {
                    cur_ms = ms;
                    cur = k;
                    changed = true;
                }
            }
        }
        if (!changed) break;
    }
    (void)hipStreamSynchronize(st);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    free_dev(img);
    free_dev(stats);
    free_dev(mom);
    c->graphs_clear();
    if (status != PHX_OK) return status;
    phx_set_launch_config(c, &cur);
    c->autotune_ms = cur_ms;
    if (best) *best = cur;
    return PHX_OK;
}
}  // namespace

phx_status phx_autotune(phx_ctx c, const phx_trace_args* sample, void* stream,
                        phx_launch_config* best) {
    return autotune(c, sample, stream, best, c && !c->cfg.pipeline);
}

phx_status phx_autotune_batched(phx_ctx c, const phx_trace_args* sample, void* stream,
                                phx_launch_config* best) {
    return autotune(c, sample, stream, best, true);
}

phx_status phx_readout(phx_ctx c, const phx_readout_params* p, const uint32_t* in, int32_t nx,
                       int32_t ny, uint16_t* adu, uint64_t adu_capacity, uint32_t* work,
                       uint32_t* par, uint32_t* ser, void* stream) {
    if (!c) return PHX_ERR_INVALID;
    if (!p || !in || !adu) return fail(c, PHX_ERR_INVALID, "null readout argument");
    if (nx < 2 || ny < 1 || (nx & 1)) return fail(c, PHX_ERR_INVALID, "bad image size %d x %d", nx, ny);
    if (p->amp_nx < 1 || p->amp_ny < 1 || p->amp_ny > 2 || p->amp_nx * p->amp_ny > PHX_MAX_AMPS ||
        nx % p->amp_nx || ny % p->amp_ny || p->over_x < 0 || p->over_y < 0 ||
        p->over_x > 65536 || p->over_y > 65536)
        return fail(c, PHX_ERR_INVALID, "bad amplifier layout");
    const int n_amp = p->amp_nx * p->amp_ny;
    const double v[] = {p->full_well, p->exposure, p->dark_rate, p->hot_fraction,
                        p->dead_fraction, p->hot_column_fraction, p->cte_parallel,
                        p->cte_serial, p->nonlinearity};
    if (!finite_all(v, 9) || !finite_all(p->gain, n_amp) || !finite_all(p->bias, n_amp) ||
        !finite_all(p->read_noise, n_amp) || !finite_all(p->bit_sigma, 16))
        return fail(c, PHX_ERR_INVALID, "non-finite readout parameter");
    // the transfer stages draw one delay per electron: bound the electrons per pixel (a full
    // well of 1e7 is far above real devices)
    if (!(p->full_well >= 1.0 && p->full_well <= 1e7) || !(p->exposure >= 0.0) ||
        !(p->dark_rate >= 0.0) || !(p->dark_rate * p->exposure <= 1e6) || !(p->hot_fraction >= 0.0) || !(p->dead_fraction >= 0.0) ||
        !(p->hot_fraction + p->dead_fraction <= 1.0) || !(p->hot_column_fraction >= 0.0) ||
        !(p->hot_column_fraction <= 1.0) || !(p->cte_parallel > 0.0 && p->cte_parallel <= 1.0) ||
        !(p->cte_serial > 0.0 && p->cte_serial <= 1.0) || !(p->nonlinearity >= 0.0))
        return fail(c, PHX_ERR_INVALID, "readout parameter out of range");
    for (int a = 0; a < n_amp; ++a)
        if (!(p->gain[a] > 0.0) || !(p->read_noise[a] >= 0.0))
            return fail(c, PHX_ERR_INVALID, "amplifier %d: gain must be > 0, read noise >= 0", a);
    for (int b = 0; b < 16; ++b)
        if (!(p->bit_sigma[b] >= 0.0)) return fail(c, PHX_ERR_INVALID, "negative bit_sigma");
    const uint64_t sw = (uint64_t)(nx / p->amp_nx), sh = (uint64_t)(ny / p->amp_ny);
    const uint64_t ph = sh + p->over_y, pw = sw + p->over_x;
    const uint64_t need[4] = {(uint64_t)nx * ny, n_amp * ph * sw, n_amp * ph * pw,
                              std::max((uint64_t)nx * ny, n_amp * ph * sw) + 1};
    if (adu_capacity < need[2])
        return fail(c, PHX_ERR_CAPACITY, "adu capacity %llu < %llu",
                    (unsigned long long)adu_capacity, (unsigned long long)need[2]);
    if (set_device(c) != PHX_OK) return PHX_ERR_HIP;
    hipStream_t st = (hipStream_t)stream;
    uint32_t* bufs[4] = {work, par, ser, nullptr};
    for (int k = 0; k < 4; ++k) {
        if (bufs[k]) continue;
        if (c->ro_cap[k] < need[k]) {
            if (c->d_ro[k]) {
                const hipError_t e = hipStreamSynchronize(st);
                if (e != hipSuccess) return hip_fail(c, e, "hipStreamSynchronize");
                free_dev(c->d_ro[k]);
                c->ro_cap[k] = 0;
            }
            const hipError_t e = hipMalloc((void**)&c->d_ro[k], need[k] * sizeof(uint32_t));
            if (e != hipSuccess) {
                c->d_ro[k] = nullptr;
                return fail(c, PHX_ERR_NOMEM, "readout scratch: %s", hipGetErrorString(e));
            }
            c->ro_cap[k] = need[k];
        }
        bufs[k] = c->d_ro[k];
    }
    phx::ReadoutJob J;
    J.p = *p;
    J.in = in;
    J.nx = nx;
    J.ny = ny;
    J.work = bufs[0];
    J.par = bufs[1];
    J.ser = bufs[2];
    J.out = adu;
    J.heavy_count = bufs[3];
    J.heavy = bufs[3] + 1;
    const hipError_t e = phx::launch_readout(J, st);
    if (e != hipSuccess) return hip_fail(c, e, "readout launch");
    return PHX_OK;
}

phx_status phx_set_timing(phx_ctx c, int32_t on) {
    if (!c) return PHX_ERR_INVALID;
    c->timing = on != 0;
    c->ev_pairs.clear();
    c->ev_used = 0;
    for (int k = 0; k < 4; ++k) {
        c->pending_start[k] = -1;
        c->timing_ms[k] = 0.0;
    }
    c->timing_chunks = 0;
    return PHX_OK;
}

phx_status phx_get_timing(phx_ctx c, double* out, int32_t n) {
    if (!c) return PHX_ERR_INVALID;
    if (!out || n < 1) return fail(c, PHX_ERR_INVALID, "null or empty output");
    for (const auto& pr : c->ev_pairs) {
        hipError_t e = hipEventSynchronize(c->ev_pool[pr.second.second]);
        if (e != hipSuccess) return hip_fail(c, e, "hipEventSynchronize");
        float ms = 0.0f;
        e = hipEventElapsedTime(&ms, c->ev_pool[pr.second.first], c->ev_pool[pr.second.second]);
        if (e != hipSuccess) return hip_fail(c, e, "hipEventElapsedTime");
        c->timing_ms[pr.first] += ms;
    }
    c->ev_pairs.clear();
    c->ev_used = 0;
    const double v[5] = {c->timing_ms[0], c->timing_ms[1], c->timing_ms[2], c->timing_chunks,
                         c->timing_ms[3]};
    for (int i = 0; i < n && i < 5; ++i) out[i] = v[i];
    return PHX_OK;
}

}  // extern "C"
