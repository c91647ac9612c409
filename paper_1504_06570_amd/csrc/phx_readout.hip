// Sensor readout chain (section 2.4.3 saturation and bleeding; section 2.5 electronic readout):
// bleeding along half-rows, dark current and defects, per-electron parallel and serial charge
// transfer, and digitisation with read noise, gain, non-linearity, bias and bit errors.
//
// Every random draw is keyed by the pixel (or packet, or output value) it belongs to, so the
// result does not depend on the launch shape.  Floating-point contraction is off in this file: the
// decisions that quantise (transfer delays, rounding of the dark current, the digitiser's floors)
// are taken with the plain IEEE operations written.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "phx_internal.h"
#include "phx_rng.h"

#pragma clang fp contract(off)

namespace phx {
namespace {

constexpr int kRoBlock = 256;
constexpr double kTwoPi = 6.283185307179586;

__device__ __forceinline__ uint4 ro_draw(uint32_t seed, uint32_t stage, uint64_t idx,
                                         uint32_t block) {
    return philox(make_uint4((uint32_t)idx, (uint32_t)(idx >> 32), block, 0u), seed, stage);
}

__device__ __forceinline__ uint32_t ro_word(const uint4& w, int k) {
    return k == 0 ? w.x : k == 1 ? w.y : k == 2 ? w.z : w.w;
}

// Step 1: one wavefront per half-row copies it (coalesced) into the work image; if a pixel exceeds
// the full well, lane 0 then bleeds the half-row: pixels in index order, each excess to the
// closest pixels below full well (ties toward the row's end), the rest removed once it is full.
// With `lds` the half-row is also staged in LDS (kRoBlock / 64 half-rows of nx / 2 words per
// workgroup), lane 0 bleeds it there and the wavefront writes it back.
__device__ __forceinline__ void bleed_half_row(uint32_t* row, int64_t a, int64_t b, int half,
                                               uint64_t w) {
    for (int64_t p = a; p < b; ++p) {
        if (row[p] <= w) continue;
        uint64_t excess = row[p] - w;
        row[p] = (uint32_t)w;
        int64_t L = p - 1, R = p + 1;
        while (excess > 0) {
            while (L >= a && row[L] >= w) --L;
            while (R < b && row[R] >= w) ++R;
            const bool hl = L >= a, hr = R < b;
            if (!hl && !hr) break;
            int64_t t;
            if (hl && hr) {
                const int64_t dl = p - L, dr = R - p;
                t = dl != dr ? (dl < dr ? L : R) : (half == 0 ? L : R);
            } else {
                t = hl ? L : R;
            }
            const uint64_t room = w - row[t];
            const uint64_t put = excess < room ? excess : room;
            row[t] += (uint32_t)put;
            excess -= put;
        }
    }
}

__global__ __launch_bounds__(kRoBlock) void ro_bleed(const ReadoutJob J, int lds) {
    extern __shared__ uint32_t s_half[];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint64_t h = (uint64_t)blockIdx.x * (kRoBlock / 64) + wave;
    if (h >= 2ull * (uint64_t)J.ny) return;
    const int64_t j = (int64_t)(h >> 1);
    const int half = (int)(h & 1);
    const int64_t a = half ? J.nx / 2 : 0, b = half ? J.nx : J.nx / 2;
    const uint64_t w = (uint64_t)J.p.full_well;
    const uint32_t* src = J.in + j * J.nx;
    uint32_t* row = J.work + j * J.nx;
    uint32_t* buf = s_half + (int64_t)wave * (J.nx / 2);   // buf[x - a] holds pixel x
    bool sat = false;
    for (int64_t x = a + lane; x < b; x += 64) {
        const uint32_t v = src[x];
        row[x] = v;
        if (lds) buf[x - a] = v;
        sat |= v > w;
    }
    if (__ballot(sat) == 0) return;
    if (lds) {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        if (lane == 0) bleed_half_row(buf, 0, b - a, half, w);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        for (int64_t x = a + lane; x < b; x += 64) row[x] = buf[x - a];
    } else {
        __threadfence();
        __builtin_amdgcn_wave_barrier();
        if (lane == 0) bleed_half_row(row, a, b, half, w);
    }
}

// Step 2: dark current (normal with mean and variance mu, rounded, floored at zero), then hot
// pixels set to the full well and dead pixels emptied.
__global__ __launch_bounds__(kRoBlock) void ro_defects(const ReadoutJob J) {
    const uint64_t n = (uint64_t)J.nx * J.ny;
    const double mu = J.p.dark_rate * J.p.exposure;
    const double fh = J.p.hot_fraction, fd = J.p.dead_fraction;
    const uint64_t w = (uint64_t)J.p.full_well;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint4 r = ro_draw(J.p.seed, 1, i, 0);
        uint64_t e = J.work[i];
        if (mu > 0.0) {
            const double g = sqrt(-2.0 * log(u01(r.z))) * cos(kTwoPi * u01(r.w));
            const double d = floor(mu + sqrt(mu) * g + 0.5);
            if (d > 0.0) e += (uint64_t)d;
        }
        const double u = u01(r.x);
        if (u < fh) e = w;
        else if (u < fh + fd) e = 0;
        J.work[i] = (uint32_t)(e > 0xffffffffull ? 0xffffffffull : e);
    }
}

// Step 2, hot columns: one wavefront per segment column draws the end flags of 64 rows at a
// time, walking away from the register; from the first end on, every pixel is set to the full
// well.
__global__ __launch_bounds__(kRoBlock) void ro_hot_columns(const ReadoutJob J) {
    const int lane = threadIdx.x & 63;
    const uint64_t t = (uint64_t)blockIdx.x * (kRoBlock / 64) + (threadIdx.x >> 6);
    if (t >= (uint64_t)J.nx * J.p.amp_ny) return;
    const int64_t x = (int64_t)(t % J.nx);
    const int half = (int)(t / J.nx);
    const int64_t sh = J.ny / J.p.amp_ny;
    const uint32_t w = (uint32_t)J.p.full_well;
    int64_t first = sh;
    for (int64_t r0 = 0; r0 < sh; r0 += 64) {
        const int64_t r = r0 + lane;
        bool end = false;
        if (r < sh) {
            const int64_t y = half == 0 ? r : J.ny - 1 - r;
            end = u01(ro_draw(J.p.seed, 2, (uint64_t)y * J.nx + x, 0).x) < J.p.hot_column_fraction;
        }
        const uint64_t mask = __ballot(end);
        if (mask) {
            first = r0 + __ffsll((unsigned long long)mask) - 1;
            break;
        }
    }
    for (int64_t r = first + lane; r < sh; r += 64) {
        const int64_t y = half == 0 ? r : J.ny - 1 - r;
        J.work[(uint64_t)y * J.nx + x] = w;
    }
}

__global__ __launch_bounds__(kRoBlock) void ro_zero(uint32_t* p, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// Failures before m successes of probability 1 - eps, by inversion of u above P(0) = p0 (at most
// 64).
__device__ __forceinline__ int ro_delay(double u, int64_t m, double eps, double p0) {
    double p = p0, cum = p0;
    int f = 0;
    while (!(u < cum) && f < 64) {
        ++f;
        p *= (double)(m + f - 1) / f * eps;
        cum += p;
    }
    return f;
}

// Number of 32-bit words w with u01(w) < c: ceil(c 2^32 - 1/2) clamped to [0, 2^32].
__device__ __forceinline__ uint64_t word_bound(double c) {
    const double x = ceil(c * 4294967296.0 - 0.5);
    return x <= 0.0 ? 0ull : (x >= 4294967296.0 ? 4294967296ull : (uint64_t)x);
}

// Steps 3 and 4: the electrons of one packet at transfer index m - 1 (m transfers), each drawn
// a delay; electron e reads word e % 4 of draw block e / 4.  Blocks b0, b0 + db, ... are handled
// here; the kept electrons and those delayed by one slot are counted (the caller adds them to
// slots m - 1 and m), longer delays are added one by one (rare).
struct Kept {
    uint32_t k0, k1;
};
__device__ __forceinline__ Kept ro_transfer(uint32_t ne, uint64_t idx, int64_t m, double eps,
                                            double p0, uint32_t seed, uint32_t stage,
                                            uint32_t* dst, int64_t stride, int64_t n_slots,
                                            uint32_t b0, uint32_t db) {
    uint32_t kept = 0, one = 0;
    // the first two cumulative probabilities of the delay, as the inversion forms them, and the
    // word thresholds they imply: u01(w) = (w + 1/2) 2^-32 < c exactly when w < ceil(c 2^32 - 1/2)
    // (every step exact in double), so the decisions are integer compares
    const double cum1 = p0 + p0 * ((double)m / 1 * eps);
    const uint64_t t0 = word_bound(p0), t1 = word_bound(cum1);
    const uint32_t nb = (ne + 3) >> 2;
    for (uint32_t b = b0; b < nb; b += db) {
        const uint4 r = ro_draw(seed, stage, idx, b);
        const uint32_t left = ne - 4 * b;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const bool live = (uint32_t)q < left;
            const uint64_t w = ro_word(r, q);
            kept += live && w < t0;
            one += live && w >= t0 && w < t1;
            if (live && w >= t1) {   // a delay of two slots or more: rare
                const int64_t s = m - 1 + ro_delay(u01((uint32_t)w), m, eps, p0);
                if (s < n_slots) atomicAdd(dst + s * stride, 1u);
            }
        }
    }
    return Kept{kept, one};
}

// A packet with more electrons than this is handed to a whole wavefront (the heavy list).
constexpr uint32_t kHeavy = 1024;

// Where packet i of a transfer stage sits: its electrons, transfer count m, destination column
// or row and slot stride / count.
struct Packet {
    uint32_t ne;
    int64_t m;
    uint32_t* dst;
    int64_t stride, n_slots;
};

template <int STAGE>
__device__ __forceinline__ Packet packet_of(const ReadoutJob& J, uint64_t i) {
    const int64_t sw = J.nx / J.p.amp_nx, sh = J.ny / J.p.amp_ny;
    const int64_t ph = sh + J.p.over_y, pw = sw + J.p.over_x;
    Packet k;
    if (STAGE == 3) {
        const int64_t y = (int64_t)(i / J.nx), x = (int64_t)(i % J.nx);
        const int64_t ax = x / sw, ay = y / sh;
        const int64_t amp = ay * J.p.amp_nx + ax, c = x - ax * sw;
        const int64_t r = ay == 0 ? y : J.ny - 1 - y;
        k = Packet{J.work[i], r + 1, J.par + amp * ph * sw + c, sw, ph};
    } else {
        const int64_t c = (int64_t)(i % sw), rowi = (int64_t)(i / sw);   // rowi = amp ph + s
        k = Packet{J.par[i], c + 1, J.ser + rowi * pw, 1, pw};
    }
    return k;
}

// One thread per packet; packets above kHeavy electrons are appended to the heavy list instead.
template <int STAGE>
__global__ __launch_bounds__(kRoBlock) void ro_transfer_light(const ReadoutJob J, uint64_t n,
                                                              double eps) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const Packet k = packet_of<STAGE>(J, i);
        if (k.ne == 0) continue;
        if (!(eps > 0.0)) {
            atomicAdd(k.dst + (k.m - 1) * k.stride, k.ne);
            continue;
        }
        if (k.ne > kHeavy) {
            J.heavy[atomicAdd(J.heavy_count, 1u)] = (uint32_t)i;
            continue;
        }
        const double p0 = pow(1.0 - eps, (double)k.m);
        const Kept kk = ro_transfer(k.ne, i, k.m, eps, p0, J.p.seed, STAGE, k.dst, k.stride,
                                    k.n_slots, 0, 1);
        if (kk.k0) atomicAdd(k.dst + (k.m - 1) * k.stride, kk.k0);
        if (kk.k1 && k.m < k.n_slots) atomicAdd(k.dst + k.m * k.stride, kk.k1);
    }
}

// kSplit wavefronts per heavy packet: wavefront `sub` takes the draw blocks sub * 64 + lane +
// j * kSplit * 64, and each sums its kept electrons (a few hundred saturated pixels would
// otherwise leave most SIMDs with one long dependent chain each).
constexpr uint32_t kSplit = 4;
__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

template <int STAGE>
__global__ __launch_bounds__(kRoBlock) void ro_transfer_heavy(const ReadoutJob J, double eps) {
    const uint64_t n = (uint64_t)*J.heavy_count * kSplit;
    const int lane = threadIdx.x & 63;
    const uint64_t waves = (uint64_t)gridDim.x * (kRoBlock / 64);
    for (uint64_t t = (uint64_t)blockIdx.x * (kRoBlock / 64) + (threadIdx.x >> 6); t < n;
         t += waves) {
        const uint64_t i = J.heavy[t / kSplit];
        const uint32_t sub = (uint32_t)(t % kSplit);
        const Packet k = packet_of<STAGE>(J, i);
        const double p0 = pow(1.0 - eps, (double)k.m);
        const Kept kk = ro_transfer(k.ne, i, k.m, eps, p0, J.p.seed, STAGE, k.dst, k.stride,
                                    k.n_slots, sub * 64u + (uint32_t)lane, 64u * kSplit);
        const uint32_t k0 = wave_sum(kk.k0), k1 = wave_sum(kk.k1);
        if (lane == 0) {
            if (k0) atomicAdd(k.dst + (k.m - 1) * k.stride, k0);
            if (k1 && k.m < k.n_slots) atomicAdd(k.dst + k.m * k.stride, k1);
        }
    }
}

// Step 5: read noise, gain, non-linearity, bias, clamp, bit errors.
__global__ __launch_bounds__(kRoBlock) void ro_digitise(const ReadoutJob J, int any_bit) {
    const int64_t sw = J.nx / J.p.amp_nx, sh = J.ny / J.p.amp_ny;
    const int64_t ph = sh + J.p.over_y, pw = sw + J.p.over_x;
    const uint64_t n = (uint64_t)J.p.amp_nx * J.p.amp_ny * ph * pw;
    const double W = J.p.full_well;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const int amp = (int)(i / (uint64_t)(ph * pw));
        const uint4 r = ro_draw(J.p.seed, 5, i, 0);
        double e = (double)J.ser[i];
        e += J.p.read_noise[amp] * sqrt(-2.0 * log(u01(r.x))) * cos(kTwoPi * u01(r.y));
        double adu = e / (J.p.gain[amp] * (1.0 + J.p.nonlinearity * e / W)) + J.p.bias[amp];
        adu = adu < 0.0 ? 0.0 : (adu > 65535.0 ? 65535.0 : adu);
        uint32_t val = 0;
#pragma unroll 1
        for (int k = 0; k < 4; ++k) {
            double g[4] = {0.0, 0.0, 0.0, 0.0};
            // a block whose four widths are zero contributes nothing (0 x g): not drawn
            const bool need = J.p.bit_sigma[4 * k] > 0.0 || J.p.bit_sigma[4 * k + 1] > 0.0 ||
                              J.p.bit_sigma[4 * k + 2] > 0.0 || J.p.bit_sigma[4 * k + 3] > 0.0;
            if (any_bit && need) {
                const uint4 v = ro_draw(J.p.seed, 5, i, 1 + k);
                const double r0 = sqrt(-2.0 * log(u01(v.x))), r1 = sqrt(-2.0 * log(u01(v.z)));
                g[0] = r0 * cos(kTwoPi * u01(v.y));
                g[1] = r0 * sin(kTwoPi * u01(v.y));
                g[2] = r1 * cos(kTwoPi * u01(v.w));
                g[3] = r1 * sin(kTwoPi * u01(v.w));
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int bit = 4 * k + q;
                // ldexp by -bit equals the division by 2^bit exactly
                const double a = ldexp(adu, -bit) + J.p.bit_sigma[bit] * g[q];
                const int64_t f = (int64_t)floor(a);
                if (((f % 2) + 2) % 2) val |= 1u << bit;
            }
        }
        J.out[i] = (uint16_t)val;
    }
}

unsigned grid_for(uint64_t n) {
    const uint64_t g = (n + kRoBlock - 1) / kRoBlock;
    return (unsigned)(g < (1ull << 20) ? (g ? g : 1) : (1ull << 20));
}

}  // namespace

hipError_t launch_readout(const ReadoutJob& J, hipStream_t s) {
    const uint64_t npix = (uint64_t)J.nx * J.ny;
    const int64_t sw = J.nx / J.p.amp_nx, sh = J.ny / J.p.amp_ny;
    const int64_t ph = sh + J.p.over_y, pw = sw + J.p.over_x;
    const uint64_t n_amp = (uint64_t)J.p.amp_nx * J.p.amp_ny;
    const uint64_t n_par = n_amp * ph * sw, n_ser = n_amp * ph * pw;
    int any_bit = 0;
    for (int b = 0; b < 16; ++b) any_bit |= J.p.bit_sigma[b] > 0.0;
    const uint64_t half_rows = 2ull * (uint64_t)J.ny;
    const size_t lds_bytes = (size_t)(kRoBlock / 64) * (J.nx / 2) * sizeof(uint32_t);
    const int lds = lds_bytes <= 64 * 1024 ? 1 : 0;
    hipLaunchKernelGGL(ro_bleed, dim3((unsigned)((half_rows + 3) / 4)), dim3(kRoBlock),
                       lds ? lds_bytes : 0, s, J, lds);
    hipLaunchKernelGGL(ro_defects, dim3(grid_for(npix)), dim3(kRoBlock), 0, s, J);
    if (J.p.hot_column_fraction > 0.0)
        hipLaunchKernelGGL(ro_hot_columns,
                           dim3((unsigned)(((uint64_t)J.nx * J.p.amp_ny + 3) / 4)),
                           dim3(kRoBlock), 0, s, J);
    const double ep = 1.0 - J.p.cte_parallel, es = 1.0 - J.p.cte_serial;
    const unsigned heavy_grid = 2048;
    hipLaunchKernelGGL(ro_zero, dim3(grid_for(n_par)), dim3(kRoBlock), 0, s, J.par, n_par);
    hipLaunchKernelGGL(ro_zero, dim3(1), dim3(kRoBlock), 0, s, J.heavy_count, (uint64_t)1);
    hipLaunchKernelGGL(ro_transfer_light<3>, dim3(grid_for(npix)), dim3(kRoBlock), 0, s, J, npix,
                       ep);
    hipLaunchKernelGGL(ro_transfer_heavy<3>, dim3(heavy_grid), dim3(kRoBlock), 0, s, J, ep);
    hipLaunchKernelGGL(ro_zero, dim3(grid_for(n_ser)), dim3(kRoBlock), 0, s, J.ser, n_ser);
    hipLaunchKernelGGL(ro_zero, dim3(1), dim3(kRoBlock), 0, s, J.heavy_count, (uint64_t)1);
    hipLaunchKernelGGL(ro_transfer_light<4>, dim3(grid_for(n_par)), dim3(kRoBlock), 0, s, J, n_par,
                       es);
    hipLaunchKernelGGL(ro_transfer_heavy<4>, dim3(heavy_grid), dim3(kRoBlock), 0, s, J, es);
    hipLaunchKernelGGL(ro_digitise, dim3(grid_for(n_ser)), dim3(kRoBlock), 0, s, J, any_bit);
    return hipGetLastError();
}

}  // namespace phx
