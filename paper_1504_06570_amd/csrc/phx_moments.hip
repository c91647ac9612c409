// Per-source centroids and second moments from the trace's exact moment words (the per-source
// outputs of the paper's section 3.1: counts and centroids of the sources; "weighted moments" of
// section 4 read as unweighted moments of the converted photons' electron positions), and the
// adjoint's per-photon cotangent coefficients from a loss gradient with respect to those moments.
//
// The words hold n and the 128-bit sums SX, SY, SXX, SYY, SXY of positions quantised to
// X = x 2^44.  Each result is a ratio of integers,
//   mean x = SX / (n 2^44),   Ixx = (n SXX - SX^2) / (n^2 2^88),   Ixy = (n SXY - SX SY) / (n^2 2^88),
// formed here in exact multiword integer arithmetic (six 64-bit limbs) and rounded once to the
// nearest double (ties to even), so the small central moments of a far-off-axis source lose
// nothing to cancellation.  One thread per source.
#include <hip/hip_runtime.h>

#include "phx_internal.h"

namespace phx {
namespace {

constexpr int kLimbs = 6;   // 384 bits: n SXX < 2^192, SX^2 < 2^256
struct Big {
    uint64_t w[kLimbs];
};

__device__ Big big_zero() {
    Big r;
#pragma unroll
    for (int i = 0; i < kLimbs; ++i) r.w[i] = 0;
    return r;
}

__device__ Big big_from(uint64_t lo, uint64_t hi) {
    Big r = big_zero();
    r.w[0] = lo;
    r.w[1] = hi;
    return r;
}

__device__ bool big_is_zero(const Big& a) {
    uint64_t o = 0;
#pragma unroll
    for (int i = 0; i < kLimbs; ++i) o |= a.w[i];
    return o == 0;
}

// -1, 0, 1 as a < b, a == b, a > b
__device__ int big_cmp(const Big& a, const Big& b) {
    for (int i = kLimbs - 1; i >= 0; --i) {
        if (a.w[i] != b.w[i]) return a.w[i] < b.w[i] ? -1 : 1;
    }
    return 0;
}

// a - b for a >= b
__device__ Big big_sub(const Big& a, const Big& b) {
    Big r;
    uint64_t borrow = 0;
#pragma unroll
    for (int i = 0; i < kLimbs; ++i) {
        const uint64_t d = a.w[i] - b.w[i];
        const uint64_t b1 = a.w[i] < b.w[i];
        r.w[i] = d - borrow;
        const uint64_t b2 = d < borrow;
        borrow = b1 | b2;
    }
    return r;
}

// a x b, the operands below 2^192 each (so the product fits)
__device__ Big big_mul(const Big& a, const Big& b) {
    Big r = big_zero();
    for (int i = 0; i < kLimbs / 2; ++i) {
        uint64_t carry = 0;
        for (int j = 0; j < kLimbs - i; ++j) {
            const uint64_t lo = a.w[i] * b.w[j];
            const uint64_t hi = __umul64hi(a.w[i], b.w[j]);
            uint64_t s = r.w[i + j] + lo;
            uint64_t c = s < lo;
            s += carry;
            c += s < carry;
            r.w[i + j] = s;
            carry = hi + c;
        }
    }
    return r;
}

__device__ int big_bits(const Big& a) {
    for (int i = kLimbs - 1; i >= 0; --i)
        if (a.w[i]) return 64 * i + 64 - __clzll(a.w[i]);
    return 0;
}

__device__ Big big_shl(const Big& a, int s) {
    Big r = big_zero();
    const int q = s / 64, b = s % 64;
    for (int i = kLimbs - 1; i >= q; --i) {
        uint64_t v = a.w[i - q] << b;
        if (b && i - q - 1 >= 0) v |= a.w[i - q - 1] >> (64 - b);
        r.w[i] = v;
    }
    return r;
}

__device__ bool big_bit(const Big& a, int i) { return (a.w[i / 64] >> (i % 64)) & 1u; }

// num / den x 2^e2 rounded once to the nearest double (ties to even); num, den > 0 with at most
// 320 bits.  The quotient q = floor(num 2^sh / den) is formed with 64 or 65 bits by restoring
// long division; its bits below the double's 53 and the remainder decide the rounding.
__device__ double big_ratio(const Big& num, const Big& den, int e2) {
    const int ln = big_bits(num), ld = big_bits(den);
    // num 2^sh lies in [2^(63 + ld), 2^(64 + ld)) and den in [2^(ld - 1), 2^ld)
    const int sh = 64 + ld - ln;
    const Big n2 = sh >= 0 ? big_shl(num, sh) : num;
    const Big d2 = sh >= 0 ? den : big_shl(den, -sh);
    Big rem = big_zero();
    uint64_t qlo = 0, qhi = 0;
    for (int i = big_bits(n2) - 1; i >= 0; --i) {
        rem = big_shl(rem, 1);
        rem.w[0] |= big_bit(n2, i) ? 1u : 0u;
        qhi = (qhi << 1) | (qlo >> 63);
        qlo <<= 1;
        if (big_cmp(rem, d2) >= 0) {
            rem = big_sub(rem, d2);
            qlo |= 1u;
        }
    }
    const bool sticky = !big_is_zero(rem);
    // q has 64 or 65 bits: drop its low 11 or 12 bits
    const int drop = (qhi ? 65 : 64) - 53;
    uint64_t m = (qlo >> drop) | (qhi << (64 - drop));
    const uint64_t low = qlo & ((1ull << drop) - 1);
    const uint64_t halfbit = 1ull << (drop - 1);
    const bool half = (low & halfbit) != 0;
    const bool below = (low & (halfbit - 1)) != 0 || sticky;
    if (half && (below || (m & 1u))) m += 1;   // 2^53 after a carry is still exact
    return ldexp((double)m, e2 - sh + drop);
}

struct Signed {
    bool neg;
    Big mag;
};

__device__ Signed s128(uint64_t lo, uint64_t hi) {
    Signed r;
    r.neg = (hi >> 63) != 0;
    if (r.neg) {   // two's complement magnitude
        lo = ~lo;
        hi = ~hi;
        lo += 1;
        hi += lo == 0;
    }
    r.mag = big_from(lo, hi);
    return r;
}

// a - b for signed magnitudes
__device__ Signed s_sub(const Signed& a, const Signed& b) {
    Signed r;
    if (a.neg != b.neg) {   // a - b = sign(a) (|a| + |b|)
        Big s = big_zero();
        uint64_t carry = 0;
        for (int i = 0; i < kLimbs; ++i) {
            uint64_t v = a.mag.w[i] + carry;
            uint64_t c = v < carry;
            v += b.mag.w[i];
            c += v < b.mag.w[i];
            s.w[i] = v;
            carry = c;
        }
        r.neg = a.neg;
        r.mag = s;
        return r;
    }
    const int c = big_cmp(a.mag, b.mag);
    if (c >= 0) {
        r.neg = a.neg;
        r.mag = big_sub(a.mag, b.mag);
    } else {
        r.neg = !a.neg;
        r.mag = big_sub(b.mag, a.mag);
    }
    return r;
}

__device__ double s_ratio(const Signed& num, const Big& den, int e2) {
    if (big_is_zero(num.mag)) return 0.0;
    const double v = big_ratio(num.mag, den, e2);
    return num.neg ? -v : v;
}

__device__ Signed s_mul(const Signed& a, const Signed& b) {
    Signed r;
    r.neg = a.neg != b.neg;
    r.mag = big_mul(a.mag, b.mag);
    return r;
}

// (n, mean x, mean y, Ixx, Iyy, Ixy) of the source's words
__device__ void source_moments(const unsigned long long* w, double out[6]) {
    const uint64_t n = w[0];
    out[0] = (double)n;
    if (n == 0) {
        for (int i = 1; i < 6; ++i) out[i] = 0.0;
        return;
    }
    const Signed sx = s128(w[2], w[3]), sy = s128(w[4], w[5]);
    const Signed sxx = s128(w[6], w[7]), syy = s128(w[8], w[9]), sxy = s128(w[10], w[11]);
    Signed nn;
    nn.neg = false;
    nn.mag = big_from(n, 0);
    const Big n2 = big_mul(nn.mag, nn.mag);
    constexpr int q = PHX_MOMENT_Q_LOG2;
    out[1] = s_ratio(sx, nn.mag, -q);
    out[2] = s_ratio(sy, nn.mag, -q);
    out[3] = s_ratio(s_sub(s_mul(nn, sxx), s_mul(sx, sx)), n2, -2 * q);
    out[4] = s_ratio(s_sub(s_mul(nn, syy), s_mul(sy, sy)), n2, -2 * q);
    out[5] = s_ratio(s_sub(s_mul(nn, sxy), s_mul(sx, sy)), n2, -2 * q);
}

__global__ void moments_kernel(const unsigned long long* __restrict__ words, int n_src,
                               double* __restrict__ out) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_src) return;
    double m[6];
    source_moments(words + (size_t)s * PHX_MOMENT_WORDS, m);
    for (int i = 0; i < 6; ++i) out[(size_t)s * 6 + i] = m[i];
}

// Cotangent coefficients of the adjoint for a loss L(mean x, mean y, Ixx, Iyy, Ixy) per source:
// d mean/d x_i = 1/n, d Ixx/d x_i = 2 (x_i - mean x)/n, d Ixy/d x_i = (y_i - mean y)/n, so that
// xbar_i = g0 + g2 (x_i - g5) + g4 (y_i - g6) and ybar_i = g1 + g3 (y_i - g6) + g4 (x_i - g5)
// with g = (dL/dmx, dL/dmy, 2 dL/dIxx, 2 dL/dIyy, dL/dIxy) / n and (g5, g6) the mean; a source
// without converted photons gets a zero row.
__global__ void seed_kernel(const unsigned long long* __restrict__ words, int n_src,
                            const double* __restrict__ dmom, double* __restrict__ seed) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_src) return;
    double m[6];
    source_moments(words + (size_t)s * PHX_MOMENT_WORDS, m);
    double* g = seed + (size_t)s * 8;
    const double* d = dmom + (size_t)s * 5;
    if (m[0] == 0.0) {
        for (int i = 0; i < 8; ++i) g[i] = 0.0;
        return;
    }
    const double inv = 1.0 / m[0];
    g[0] = d[0] * inv;
    g[1] = d[1] * inv;
    g[2] = 2.0 * d[2] * inv;
    g[3] = 2.0 * d[3] * inv;
    g[4] = d[4] * inv;
    g[5] = m[1];
    g[6] = m[2];
    g[7] = 0.0;
}

}  // namespace

hipError_t launch_moments(const unsigned long long* words, int n_src, double* out,
                          hipStream_t stream) {
    if (n_src <= 0) return hipSuccess;
    hipLaunchKernelGGL(moments_kernel, dim3((unsigned)((n_src + 63) / 64)), dim3(64), 0, stream,
                       words, n_src, out);
    return hipGetLastError();
}

hipError_t launch_seeds(const unsigned long long* words, int n_src, const double* dmom,
                        double* seed, hipStream_t stream) {
    if (n_src <= 0) return hipSuccess;
    hipLaunchKernelGGL(seed_kernel, dim3((unsigned)((n_src + 63) / 64)), dim3(64), 0, stream,
                       words, n_src, dmom, seed);
    return hipGetLastError();
}

}  // namespace phx
