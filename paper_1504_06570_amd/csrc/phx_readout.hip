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
__global__ __launch_bounds__(kRoBlock) void ro_bleed(const ReadoutJob J) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint64_t h = (uint64_t)blockIdx.x * (kRoBlock / 64) + wave;
    if (h >= 2ull * (uint64_t)J.ny) return;
    const int64_t j = (int64_t)(h >> 1);
    const int half = (int)(h & 1);
    const int64_t a = half ? J.nx / 2 : 0, b = half ? J.nx : J.nx / 2;
    const uint64_t w = (uint64_t)J.p.full_well;
    const uint32_t* src = J.in + j * J.nx;
    uint32_t* row = J.work + j * J.nx;
    bool sat = false;
    for (int64_t x = a + lane; x < b; x += 64) {
        const uint32_t v = src[x];
        row[x] = v;
        sat |= v > w;
    }
    if (__ballot(sat) == 0) return;
    __threadfence();
    __builtin_amdgcn_wave_barrier();
    if (lane != 0) return;
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

// Step 2, hot columns: one thread per segment column walks away from its register; from the first
// hot-column end on, every pixel is set to the full well.
__global__ __launch_bounds__(kRoBlock) void ro_hot_columns(const ReadoutJob J) {
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (uint64_t)J.nx * J.p.amp_ny) return;
    const int64_t x = (int64_t)(t % J.nx);
    const int half = (int)(t / J.nx);
    const int64_t sh = J.ny / J.p.amp_ny;
    const uint32_t w = (uint32_t)J.p.full_well;
    bool hot = false;
    for (int64_t r = 0; r < sh; ++r) {
        const int64_t y = half == 0 ? r : J.ny - 1 - r;
        const uint64_t i = (uint64_t)y * J.nx + x;
        if (!hot) hot = u01(ro_draw(J.p.seed, 2, i, 0).x) < J.p.hot_column_fraction;
        if (hot) J.work[i] = w;
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

// Steps 3 and 4: the electrons of one packet at transfer index m - 1 (m transfers), each drawn
// a delay; kept electrons are added to slot m - 1 at once, delayed ones one by one (rare).
__device__ __forceinline__ void ro_transfer(uint32_t ne, int64_t idx, int64_t m, double eps,
                                            uint32_t seed, uint32_t stage, uint32_t* dst,
                                            int64_t stride, int64_t n_slots) {
    if (ne == 0) return;
    if (!(eps > 0.0)) {
        atomicAdd(dst + (m - 1) * stride, ne);
        return;
    }
    const double p0 = pow(1.0 - eps, (double)m);
    uint32_t kept = 0;
    uint4 r = make_uint4(0, 0, 0, 0);
    for (uint32_t e = 0; e < ne; ++e) {
        if ((e & 3) == 0) r = ro_draw(seed, stage, (uint64_t)idx, e >> 2);
        const double u = u01(ro_word(r, (int)(e & 3)));
        if (u < p0) {
            ++kept;
            continue;
        }
        const int64_t s = m - 1 + ro_delay(u, m, eps, p0);
        if (s < n_slots) atomicAdd(dst + s * stride, 1u);
    }
    if (kept) atomicAdd(dst + (m - 1) * stride, kept);
}

__global__ __launch_bounds__(kRoBlock) void ro_parallel(const ReadoutJob J) {
    const uint64_t n = (uint64_t)J.nx * J.ny;
    const int64_t sw = J.nx / J.p.amp_nx, sh = J.ny / J.p.amp_ny, ph = sh + J.p.over_y;
    const double eps = 1.0 - J.p.cte_parallel;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const int64_t y = (int64_t)(i / J.nx), x = (int64_t)(i % J.nx);
        const int64_t ax = x / sw, ay = y / sh;
        const int64_t amp = ay * J.p.amp_nx + ax, c = x - ax * sw;
        const int64_t r = ay == 0 ? y : J.ny - 1 - y;
        ro_transfer(J.work[i], (int64_t)i, r + 1, eps, J.p.seed, 3, J.par + amp * ph * sw + c, sw,
                    ph);
    }
}

__global__ __launch_bounds__(kRoBlock) void ro_serial(const ReadoutJob J) {
    const int64_t sw = J.nx / J.p.amp_nx, sh = J.ny / J.p.amp_ny;
    const int64_t ph = sh + J.p.over_y, pw = sw + J.p.over_x;
    const uint64_t n = (uint64_t)J.p.amp_nx * J.p.amp_ny * ph * sw;
    const double eps = 1.0 - J.p.cte_serial;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const int64_t c = (int64_t)(i % sw), rowi = (int64_t)(i / sw);   // rowi = amp ph + s
        ro_transfer(J.par[i], (int64_t)i, c + 1, eps, J.p.seed, 4, J.ser + rowi * pw, 1, pw);
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
            if (any_bit) {
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
                const double a = adu / (double)(1u << bit) + J.p.bit_sigma[bit] * g[q];
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
    hipLaunchKernelGGL(ro_bleed, dim3((unsigned)((half_rows + 3) / 4)), dim3(kRoBlock), 0, s, J);
    hipLaunchKernelGGL(ro_defects, dim3(grid_for(npix)), dim3(kRoBlock), 0, s, J);
    if (J.p.hot_column_fraction > 0.0)
        hipLaunchKernelGGL(ro_hot_columns, dim3(grid_for((uint64_t)J.nx * J.p.amp_ny)),
                           dim3(kRoBlock), 0, s, J);
    hipLaunchKernelGGL(ro_zero, dim3(grid_for(n_par)), dim3(kRoBlock), 0, s, J.par, n_par);
    hipLaunchKernelGGL(ro_parallel, dim3(grid_for(npix)), dim3(kRoBlock), 0, s, J);
    hipLaunchKernelGGL(ro_zero, dim3(grid_for(n_ser)), dim3(kRoBlock), 0, s, J.ser, n_ser);
    hipLaunchKernelGGL(ro_serial, dim3(grid_for(n_par)), dim3(kRoBlock), 0, s, J);
    hipLaunchKernelGGL(ro_digitise, dim3(grid_for(n_ser)), dim3(kRoBlock), 0, s, J, any_bit);
    return hipGetLastError();
}

}  // namespace phx
