// FP64 elementary functions for the chain kernels, written for the
// instruction budget of gfx950's VALU.
//
// * Natural logarithm, table-driven after P. T. P. Tang, "Table-driven
//   implementation of the logarithm function in IEEE floating-point
//   arithmetic", ACM TOMS 16(4), 1990: x = m 2^e with m in [1,2);
//   the top 7 fraction bits of m pick a breakpoint with reciprocal c_j, so
//   r = m c_j - 1 satisfies |r| <= 2^-8 and ln x = e ln 2 - ln c_j + log1p(r),
//   log1p(r) by its Taylor series to r^6 (truncation < 3e-18).  The caller
//   keeps e (an exact integer) apart, so a sum of n_m ln p_m can gather the
//   e ln 2 terms exactly and multiply by ln 2 once.
// * sqrt of a positive normal argument by a refined reciprocal square root.
// * sin(pi x) and cos(pi x) for x in [0, 2): x = k/2 + r with |r| <= 1/4
//   (exact), then the Taylor series of sin(pi r) to degree 17 and of
//   cos(pi r) to degree 16 (truncation < 1e-19), rotated by the quadrant k.
// * 64-lane cross-lane exchanges by DPP for the Walsh-Hadamard butterflies.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qst {

constexpr int kLogTableSize = 128;   // breakpoints of the table-driven logarithm
constexpr double kLn2 = 0.693147180559945309417232121458176568;
constexpr double kInvLn2 = 1.442695040888963407359924681001892137;
constexpr double kPi = 3.14159265358979323846264338327950288;

// Table entry j: c2 = 2 / (1 + (j + 1/2)/128) (applied to the frexp mantissa
// in [1/2, 1)) and L = -ln(c2 / 2) = ln(1 + (j + 1/2)/128).
struct LogEntry {
    double c2;
    double L;
};

// Fill the table cooperatively (once per workgroup, before first use).
__device__ __forceinline__ void log_table_init(LogEntry* tab, int tid, int nthreads)
{
    for (int j = tid; j < kLogTableSize; j += nthreads) {
        const double mid = 1.0 + (static_cast<double>(j) + 0.5) / kLogTableSize;
        tab[j].c2 = 2.0 / mid;
        tab[j].L = -log(tab[j].c2 * 0.5);
    }
}

// ln x = e * ln2 + frac for finite x > 0 (normal or subnormal).
__device__ __forceinline__ double log_parts(double x, const LogEntry* __restrict__ tab, int& e)
{
    const double m = __builtin_amdgcn_frexp_mant(x);   // [1/2, 1)
    e = __builtin_amdgcn_frexp_exp(x) - 1;              // x = (2m) 2^e
    const uint32_t hi = static_cast<uint32_t>(__double_as_longlong(m) >> 32);
    const int j = (hi >> 13) & (kLogTableSize - 1);     // top 7 fraction bits
    const LogEntry t = tab[j];
    const double r = __builtin_fma(m, t.c2, -1.0);      // |r| <= 2^-8
    // log1p(r) = r - r^2/2 + r^3/3 - r^4/4 + r^5/5 - r^6/6
    double q = -1.0 / 6.0;
    q = __builtin_fma(q, r, 1.0 / 5.0);
    q = __builtin_fma(q, r, -1.0 / 4.0);
    q = __builtin_fma(q, r, 1.0 / 3.0);
    q = __builtin_fma(q, r, -1.0 / 2.0);
    const double r2 = r * r;
    return t.L + __builtin_fma(q, r2, r);
}

__device__ __forceinline__ double fast_log(double x, const LogEntry* __restrict__ tab)
{
    int e;
    const double f = log_parts(x, tab, e);
    return __builtin_fma(static_cast<double>(e), kLn2, f);
}

// sqrt(x) for positive normal x well inside the FP64 range (no scaling
// for denormal or huge arguments): the hardware reciprocal square root
// refined by two Newton steps r <- r + r (1 - x r^2) / 2, each squaring its
// relative error, then x r; within about one ulp of the correctly rounded
// root, in a third of the instructions of the general library routine.
__device__ __forceinline__ double sqrt_pos(double x)
{
    double r = __builtin_amdgcn_rsq(x);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const double e = __builtin_fma(-x * r, r, 1.0);
        r = __builtin_fma(0.5 * r, e, r);
    }
    return x * r;
}

// Taylor coefficients of sin(pi r) = sum_j (-1)^j pi^(2j+1) r^(2j+1) / (2j+1)!
// and cos(pi r) = sum_j (-1)^j pi^(2j) r^(2j) / (2j)!.
constexpr double taylor_pi_pow(int n) { return n == 0 ? 1.0 : kPi * taylor_pi_pow(n - 1); }
constexpr double taylor_fact(int n) { return n <= 1 ? 1.0 : n * taylor_fact(n - 1); }
constexpr double sin_coef(int j) { return (j % 2 ? -1.0 : 1.0) * taylor_pi_pow(2 * j + 1) / taylor_fact(2 * j + 1); }
constexpr double cos_coef(int j) { return (j % 2 ? -1.0 : 1.0) * taylor_pi_pow(2 * j) / taylor_fact(2 * j); }

// The coefficients as compile-time constants.
constexpr double kSin0 = sin_coef(0), kSin1 = sin_coef(1), kSin2 = sin_coef(2), kSin3 = sin_coef(3),
                 kSin4 = sin_coef(4), kSin5 = sin_coef(5), kSin6 = sin_coef(6), kSin7 = sin_coef(7),
                 kSin8 = sin_coef(8);
constexpr double kCos1 = cos_coef(1), kCos2 = cos_coef(2), kCos3 = cos_coef(3), kCos4 = cos_coef(4),
                 kCos5 = cos_coef(5), kCos6 = cos_coef(6), kCos7 = cos_coef(7), kCos8 = cos_coef(8);

// s = sin(pi x), c = cos(pi x) for 0 <= x < 2.
__device__ __forceinline__ void sincospi_0_2(double x, double& s, double& c)
{
    const double k = __builtin_rint(2.0 * x);   // quadrant 0..4
    const double r = x - 0.5 * k;               // exact, |r| <= 1/4
    const double r2 = r * r;
    double ps = kSin8;
    ps = __builtin_fma(ps, r2, kSin7);
    ps = __builtin_fma(ps, r2, kSin6);
    ps = __builtin_fma(ps, r2, kSin5);
    ps = __builtin_fma(ps, r2, kSin4);
    ps = __builtin_fma(ps, r2, kSin3);
    ps = __builtin_fma(ps, r2, kSin2);
    ps = __builtin_fma(ps, r2, kSin1);
    ps = __builtin_fma(ps, r2, kSin0);
    const double sr = ps * r;
    double pc = kCos8;
    pc = __builtin_fma(pc, r2, kCos7);
    pc = __builtin_fma(pc, r2, kCos6);
    pc = __builtin_fma(pc, r2, kCos5);
    pc = __builtin_fma(pc, r2, kCos4);
    pc = __builtin_fma(pc, r2, kCos3);
    pc = __builtin_fma(pc, r2, kCos2);
    pc = __builtin_fma(pc, r2, kCos1);
    const double cr = __builtin_fma(pc, r2, 1.0);
    // x = r + k/2: rotate by k quarter turns
    const int q = static_cast<int>(k) & 3;
    const double s0 = (q & 1) ? cr : sr;
    const double c0 = (q & 1) ? sr : cr;
    s = (q & 2) ? -s0 : s0;
    c = ((q + 1) & 2) ? -c0 : c0;
}

// ---------------------------------------------------------------------------
// cross-lane exchange: value of lane (lane ^ MASK) within a 64-lane wave
// ---------------------------------------------------------------------------
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v)
{
    // every source lane of the patterns used here exists, so the old value
    // of the destination is never kept and needs no initialisation
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp(static_cast<int>(b), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp(static_cast<int>(b >> 32), CTRL, 0xF, 0xF, true);
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<uint32_t>(lo));
}

constexpr int kDppQuadXor1 = 0xB1;     // quad_perm [1,0,3,2]
constexpr int kDppQuadXor2 = 0x4E;     // quad_perm [2,3,0,1]
constexpr int kDppQuadXor3 = 0x1B;     // quad_perm [3,2,1,0]
constexpr int kDppRowHalfMirror = 0x141;  // lane i <- lane 7-i within 8 (xor 7)
constexpr int kDppRowRor8 = 0x128;     // rotate a row of 16 by 8: lane i <- lane (i + 8) mod 16 = i ^ 8
constexpr int kDppRowNewBcast0 = 0x150;   // + n: every lane of a row of 16 <- lane n of that row

// Exchange across 16- or 32-lane halves with the gfx950 lane-swap
// instructions: permlane16_swap(v, v) leaves, in each 16-lane row, the
// row's own values in the first result where the row index is odd and the
// partner row's in the second where it is even (and the other way round);
// permlane32_swap does the same for the two 32-lane halves.  The partner of
// lane i is i ^ MASK.
template <int MASK>
__device__ __forceinline__ int xor_swap_i32(int v)
{
    static_assert(MASK == 16 || MASK == 32, "row or half swap");
    const int lane = static_cast<int>(threadIdx.x) & 63;
    if constexpr (MASK == 16) {
        const auto q = __builtin_amdgcn_permlane16_swap(v, v, false, false);
        return (lane & 16) ? q[0] : q[1];
    } else {
        const auto q = __builtin_amdgcn_permlane32_swap(v, v, false, false);
        return (lane & 32) ? q[0] : q[1];
    }
}

template <int MASK>
__device__ __forceinline__ double xor_lane(double v)
{
    if constexpr (MASK == 1) {
        return dpp_f64<kDppQuadXor1>(v);
    } else if constexpr (MASK == 2) {
        return dpp_f64<kDppQuadXor2>(v);
    } else if constexpr (MASK == 4) {
        return dpp_f64<kDppRowHalfMirror>(dpp_f64<kDppQuadXor3>(v));   // (i^3)^7 = i^4
    } else if constexpr (MASK == 8) {
        return dpp_f64<kDppRowRor8>(v);
    } else {
        const long long b = __double_as_longlong(v);
        const int lo = xor_swap_i32<MASK>(static_cast<int>(b));
        const int hi = xor_swap_i32<MASK>(static_cast<int>(b >> 32));
        return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<uint32_t>(lo));
    }
}

// -v if the sign mask is 0x80000000, v if it is 0 (one XOR of the sign bit).
__device__ __forceinline__ double flip_sign(double v, uint32_t mask)
{
    const long long b = __double_as_longlong(v);
    const uint32_t hi = static_cast<uint32_t>(b >> 32) ^ mask;
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<uint32_t>(b));
}

__device__ __forceinline__ float flip_sign(float v, uint32_t mask)
{
    return __int_as_float(static_cast<int>(static_cast<uint32_t>(__float_as_int(v)) ^ mask));
}

// FP32 forms of the same lane exchanges (one 32-bit DPP move per step).
template <int CTRL>
__device__ __forceinline__ float dpp_f32(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, true));
}

template <int MASK>
__device__ __forceinline__ float xor_lane_f32(float v)
{
    if constexpr (MASK == 1) {
        return dpp_f32<kDppQuadXor1>(v);
    } else if constexpr (MASK == 2) {
        return dpp_f32<kDppQuadXor2>(v);
    } else if constexpr (MASK == 4) {
        return dpp_f32<kDppRowHalfMirror>(dpp_f32<kDppQuadXor3>(v));
    } else if constexpr (MASK == 8) {
        return dpp_f32<kDppRowRor8>(v);
    } else {
        return __int_as_float(xor_swap_i32<MASK>(__float_as_int(v)));
    }
}

}  // namespace qst
