// Probes for the benchmark's rooflines (not part of the trace library).
//
// probe_gather: random gathers of 32-byte records, the size and alignment of one screen-cell
// record of the sky stage, over a table of a chosen size.  Each thread makes `rounds` dependent rounds of `width` independent
// gathers (the next round's addresses depend on the loaded values, as a layer's taps depend on
// the direction left by the layer above); the record indices come from a 32-bit integer hash of
// the thread and round, scaled to the table by a multiply-high.  The loaded words are folded into
// one word per thread so that no load can be dropped.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "phx_rng.h"

namespace {

__device__ __forceinline__ uint32_t mix32(uint32_t x) {
    // a 32-bit finaliser (xor-shift-multiply rounds)
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

constexpr int kMaxWidth = 4;

__global__ __launch_bounds__(256) void gather_kernel(const uint4* __restrict__ table,
                                                     uint64_t n_rec, uint32_t* __restrict__ out,
                                                     uint64_t n_threads, int rounds, int width,
                                                     uint32_t seed) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_threads) return;
    uint32_t h = mix32((uint32_t)i ^ mix32((uint32_t)(i >> 32) + seed));
    uint32_t acc = 0;
    for (int r = 0; r < rounds; ++r) {
        uint4 lo[kMaxWidth], hi[kMaxWidth];
#pragma unroll
        for (int k = 0; k < kMaxWidth; ++k) {
            if (k < width) {
                const uint32_t u = mix32(h + (uint32_t)(r * kMaxWidth + k) * 0x9e3779b9u + acc);
                const uint64_t rec = ((uint64_t)u * n_rec) >> 32;   // below n_rec
                lo[k] = table[2 * rec];
                hi[k] = table[2 * rec + 1];
            }
        }
#pragma unroll
        for (int k = 0; k < kMaxWidth; ++k) {
            if (k < width)
                acc ^= lo[k].x ^ lo[k].y ^ lo[k].z ^ lo[k].w ^ hi[k].x ^ hi[k].y ^ hi[k].z ^
                       hi[k].w;
        }
    }
    out[i] = acc;
}

}  // namespace

// table: n_rec records of 32 bytes (16-byte aligned device memory); out: n_threads words.
// Returns 0, or -1 for an invalid argument, or the HIP error code of the launch.
extern "C" __attribute__((visibility("default"))) int probe_gather(
        const void* table, uint64_t n_rec, uint32_t* out, uint64_t n_threads, int rounds,
        int width, uint32_t seed, hipStream_t stream) {
    if (!table || !out || n_rec == 0 || n_rec > (1ull << 32) || n_threads == 0 || rounds < 1 ||
        width < 1 || width > kMaxWidth || ((uintptr_t)table & 15u) != 0)
        return -1;
    const uint64_t blocks = (n_threads + 255) / 256;
    if (blocks > 0x7fffffffull) return -1;
    hipLaunchKernelGGL(gather_kernel, dim3((unsigned)blocks), dim3(256), 0, stream,
                       (const uint4*)table, n_rec, out, n_threads, rounds, width, seed);
    return (int)hipGetLastError();
}

// probe_fp64: the issue rate of one class of FP64 operation as hipcc compiles it for this GPU --
// fused multiply-add, IEEE division and square root, exp, log, sin, and the refined reciprocal
// and square root of the trace kernels -- the classes the oracle's counting build tallies.
// Every thread runs kChains independent dependency chains for `iters` steps (enough chains in
// flight that the rate, not the latency, is measured); each step maps a value in [1/2, 2] back
// into that range.  One result word per thread keeps the work alive.
namespace {
constexpr int kChains = 8;

// The hardware reciprocal (square-root) estimate refined by two Newton steps, to about one ulp:
// the form the trace kernels use for quotients and roots in continuous quantities.
__device__ __forceinline__ double refined_rcp(double x) {
    double r = __builtin_amdgcn_rcp(x);
    for (int k = 0; k < 2; ++k) r = fma(r, fma(-x, r, 1.0), r);
    return r;
}
__device__ __forceinline__ double refined_sqrt(double x) {
    double y = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x;
    for (int k = 0; k < 2; ++k) y = fma(y, fma(-h * y, y, 0.5), y);
    return x * y;
}

template <int KIND>
__device__ __forceinline__ double op_step(double a) {
    if (KIND == 0) return fma(a, 0.999999999, 1.0e-9);   // stays near 1
    if (KIND == 1) return 1.0000001 / a;                   // a -> 1/a
    if (KIND == 2) return sqrt(a) * 1.0000001;             // a -> ~sqrt(a), towards 1
    if (KIND == 3) return exp(0.5 - 0.5 * a);              // in [1/2, 2] for a in [1/2, 2]
    if (KIND == 4) return 1.0 + 0.5 * log(a);              // a -> 1 + log(a) / 2
    if (KIND == 5) return 1.0 + 0.5 * sin(a);              // in [1/2, 3/2]
    if (KIND == 6) return 1.0000001 * refined_rcp(a);      // as kind 1
    return refined_sqrt(a) * 1.0000001;                     // as kind 2
}

template <int KIND>
__global__ __launch_bounds__(256) void op_kernel(double* __restrict__ out, uint64_t n_threads,
                                                 int iters) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_threads) return;
    double a[kChains];
#pragma unroll
    for (int k = 0; k < kChains; ++k) a[k] = 1.0 + 1e-7 * (double)((i + k) & 1023);
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < kChains; ++k) a[k] = op_step<KIND>(a[k]);
    }
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < kChains; ++k) s += a[k];
    out[i] = s;
}
}  // namespace

// kind: 0 fma, 1 IEEE division, 2 IEEE square root, 3 exp, 4 log, 5 sin, 6 refined reciprocal,
// 7 refined square root; out: n_threads doubles.  The
// operations performed are n_threads x iters x 8.  Returns 0, -1 for an invalid argument, or the
// HIP error code of the launch.
extern "C" __attribute__((visibility("default"))) int probe_fp64(int kind, double* out,
                                                                 uint64_t n_threads, int iters,
                                                                 hipStream_t stream) {
    if (!out || n_threads == 0 || iters < 1 || kind < 0 || kind > 7) return -1;
    const uint64_t blocks = (n_threads + 255) / 256;
    if (blocks > 0x7fffffffull) return -1;
    const dim3 g((unsigned)blocks), b(256);
    switch (kind) {
    case 0: hipLaunchKernelGGL(op_kernel<0>, g, b, 0, stream, out, n_threads, iters); break;
    case 1: hipLaunchKernelGGL(op_kernel<1>, g, b, 0, stream, out, n_threads, iters); break;
    case 2: hipLaunchKernelGGL(op_kernel<2>, g, b, 0, stream, out, n_threads, iters); break;
    case 3: hipLaunchKernelGGL(op_kernel<3>, g, b, 0, stream, out, n_threads, iters); break;
    case 4: hipLaunchKernelGGL(op_kernel<4>, g, b, 0, stream, out, n_threads, iters); break;
    case 5: hipLaunchKernelGGL(op_kernel<5>, g, b, 0, stream, out, n_threads, iters); break;
    case 6: hipLaunchKernelGGL(op_kernel<6>, g, b, 0, stream, out, n_threads, iters); break;
    default: hipLaunchKernelGGL(op_kernel<7>, g, b, 0, stream, out, n_threads, iters); break;
    }
    return (int)hipGetLastError();
}

// probe_philox: the rate of Philox4x32-10 blocks as the trace kernels compute them (the pre-roll's
// unit of work).  Every thread computes `iters` blocks of kChains independent counters; the
// words are folded into one word per thread.
namespace {
__global__ __launch_bounds__(256) void philox_kernel(uint32_t* __restrict__ out,
                                                     uint64_t n_threads, int iters) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_threads) return;
    uint32_t acc = 0;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < kChains; ++k) {
            const uint4 w = phx::philox(make_uint4((uint32_t)i, (uint32_t)(i >> 32),
                                                   (uint32_t)(it * kChains + k), acc & 1u),
                                        0x1234567u, (uint32_t)k);
            acc ^= w.x ^ w.y ^ w.z ^ w.w;
        }
    }
    out[i] = acc;
}
}  // namespace

// out: n_threads words; the blocks computed are n_threads x iters x 8.  Returns 0, -1 for an
// invalid argument, or the HIP error code of the launch.
extern "C" __attribute__((visibility("default"))) int probe_philox(uint32_t* out,
                                                                   uint64_t n_threads, int iters,
                                                                   hipStream_t stream) {
    if (!out || n_threads == 0 || iters < 1) return -1;
    const uint64_t blocks = (n_threads + 255) / 256;
    if (blocks > 0x7fffffffull) return -1;
    hipLaunchKernelGGL(philox_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, out,
                       n_threads, iters);
    return (int)hipGetLastError();
}
