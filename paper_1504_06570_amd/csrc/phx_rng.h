// Counter-based random numbers shared by the library's kernels (trace and readout).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace phx {

// Philox4x32-10 (Salmon et al., SC'11).  Each round's two 32x32 -> 64-bit products come from one
// v_mad_u64_u32 each, and each three-way xor from one v_bitop3 (truth table 0x96).
__device__ __forceinline__ uint4 philox(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
        c = make_uint4(__builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c.y, k0, 0x96),
                       (uint32_t)p1,
                       __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c.w, k1, 0x96),
                       (uint32_t)p0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// (w + 1/2) 2^-32, exact in double.
__device__ __forceinline__ double u01(uint32_t w) {
    return fma((double)w, 2.3283064365386963e-10, 1.1641532182693481e-10);
}

}  // namespace phx
