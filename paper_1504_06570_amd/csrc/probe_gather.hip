// Memory-system probe for the benchmark (not part of the trace library): random gathers of
// 32-byte records, the size and alignment of one screen-cell record of the sky stage, over a
// table of a chosen size.  Each thread makes `rounds` dependent rounds of `width` independent
// gathers (the next round's addresses depend on the loaded values, as a layer's taps depend on
// the direction left by the layer above); the record indices come from a 32-bit integer hash of
// the thread and round, scaled to the table by a multiply-high.  The loaded words are folded into
// one word per thread so that no load can be dropped.
#include <hip/hip_runtime.h>

#include <cstdint>

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
