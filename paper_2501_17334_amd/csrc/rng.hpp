// Counter-based random numbers for the chain kernels (gfx950).
//
// Philox4x64-10 (Salmon, Moraes, Dror & Shaw, "Parallel random numbers: as
// easy as 1, 2, 3", SC'11): ten rounds of the two-multiply bijection, the key
// bumped by the two Weyl constants between rounds.  Every random number a
// chain uses is a pure function of (seed, chain, step, block, tag), so a chain
// needs no stored generator state and any subset of chains, any batch layout
// and any split of a run into several calls reproduce the same numbers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fastmath.hpp"

namespace qst {

constexpr uint64_t kPhiloxM0 = 0xD2E7470EE14C6C93ULL;
constexpr uint64_t kPhiloxM1 = 0xCA5A826395121157ULL;
constexpr uint64_t kPhiloxW0 = 0x9E3779B97F4A7C15ULL;
constexpr uint64_t kPhiloxW1 = 0xBB67AE8584CAA73BULL;

// Stream tags (counter word 3, bits 56..63).
constexpr int kTagNormal = 0;
constexpr int kTagMH = 1;
constexpr int kTagDA = 2;

struct Block4 {
    uint64_t w[4];
};

// Full 64 x 64 -> 128-bit product from four 32 x 32 + 64 multiply-adds
// (v_mad_u64_u32): with a = a1:a0 and b = b1:b0, t = a0 b1 + hi(a0 b0) and
// u = a1 b0 + lo(t) cannot overflow 64 bits, and
// a b = lo(a0 b0) + 2^32 lo(u) + 2^64 (a1 b1 + hi(t) + hi(u)).
__device__ __forceinline__ void mulhilo64(uint64_t a, uint64_t b, uint64_t& lo, uint64_t& hi)
{
    const uint64_t a0 = static_cast<uint32_t>(a), a1 = a >> 32;
    const uint64_t b0 = static_cast<uint32_t>(b), b1 = b >> 32;
    const uint64_t p00 = a0 * b0;
    const uint64_t t = a0 * b1 + (p00 >> 32);
    const uint64_t u = a1 * b0 + static_cast<uint32_t>(t);
    hi = a1 * b1 + ((t >> 32) + (u >> 32));
    lo = (u << 32) | static_cast<uint32_t>(p00);
}

__device__ __forceinline__ Block4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                                 uint64_t k0, uint64_t k1)
{
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += kPhiloxW0;
            k1 += kPhiloxW1;
        }
        uint64_t lo0, hi0, lo1, hi1;
        mulhilo64(kPhiloxM0, c0, lo0, hi0);
        mulhilo64(kPhiloxM1, c2, lo1, hi1);
        const uint64_t n0 = hi1 ^ c1 ^ k0;
        const uint64_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    Block4 b;
    b.w[0] = c0;
    b.w[1] = c1;
    b.w[2] = c2;
    b.w[3] = c3;
    return b;
}

// Uniform on the open interval (0,1): top 52 bits plus one half, times 2^-52
// (exact in FP64, so the result is never 0 or 1).  Formed without an integer
// conversion: the 52 bits as the mantissa of a number x in [1, 2), then
// x - (1 - 2^-53) = (m + 1/2) 2^-52 exactly.
__device__ __forceinline__ double uniform_open(uint64_t w)
{
    const double x = __longlong_as_double(static_cast<long long>((w >> 12) | 0x3FF0000000000000ULL));
    return x - 0x1.fffffffffffffp-1;
}

// Box-Muller (1958) on one pair of words: r = sqrt(-2 ln u_a),
// theta = 2 pi u_b -> (r cos theta, r sin theta); ln from the table-driven
// logarithm, the root by sqrt_pos, sin/cos(2 pi u_b) as sin/cos(pi x) with
// x = 2 u_b in (0, 2).  -2 ln u_a lies in [2^-52, 74]; it is clamped at its
// true minimum 2^-52 because the table logarithm of the largest uniform,
// 1 - 2^-53, may round to zero or just above, which would make the root NaN.
__device__ __forceinline__ void box_muller(uint64_t wa, uint64_t wb, double& n0, double& n1,
                                           const LogEntry* __restrict__ logtab)
{
    const double ua = uniform_open(wa);
    const double r = sqrt_pos(fmax(-2.0 * fast_log(ua, logtab), 0x1p-52));
    // 2 u_b = 2 (x - (1 - 2^-53)) for x in [1, 2) from the mantissa bits: one
    // exact FMA (the difference is exact and doubling it is too)
    const double xb = __longlong_as_double(static_cast<long long>((wb >> 12) | 0x3FF0000000000000ULL));
    double s, c;
    sincospi_0_2(__builtin_fma(2.0, xb, -0x1.fffffffffffffp0), s, c);
    n0 = r * c;
    n1 = r * s;
}

}  // namespace qst
