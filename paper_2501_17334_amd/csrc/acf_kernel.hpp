// Autocorrelation of recorded chains, Eq. (ACFrho)/(ACFa):
//   c[l] ~ sum_{n=1}^{N-l_max} Re Tr[(rho^n - rho_hat)^dag (rho^{n+l} - rho_hat)]
// for each chain around its own mean rho_hat^N, the unnormalised sums
// averaged over chains and divided by the lag-0 value.  Samples are packed
// (D*D reals); an off-diagonal packed entry stands for two entries of rho
// with equal products, so it carries weight 2.  Fixed summation order.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qst {

constexpr int kAcfThreads = 256;
constexpr int kAcfLags = 8;   // lags per workgroup

// One workgroup per (chain, group of kAcfLags lags), n_groups groups per
// chain, in a 1-D grid whose workgroup ids are mapped so that the groups of a
// chain run on one XCD (workgroups are dispatched to the 8 XCDs round-robin
// by id): the chain's records are then read through one L2.
// part[chain][l] = weighted lag sum of that chain.
constexpr int kXcds = 8;

__global__ __launch_bounds__(kAcfThreads) void k_acf_partial(const double* __restrict__ rec, int64_t N, int D,
                                                             int l_max, int n_groups, int64_t n_chains,
                                                             double* part)
{
    // id w runs on XCD w % 8 as the (w / 8)-th of that XCD's ids; the work
    // items (chain-major) are cut into 8 contiguous runs, one per XCD
    const int64_t total = n_chains * n_groups;
    const int64_t w = blockIdx.x;
    const int64_t xcd = w % kXcds, j = w / kXcds;
    const int64_t per = total / kXcds, extra = total % kXcds;   // XCD x holds per + (x < extra) items
    const int64_t item = xcd * per + (xcd < extra ? xcd : extra) + j;
    const int64_t chain = item / n_groups;
    const int l0 = static_cast<int>(item % n_groups) * kAcfLags;

    const int D2 = D * D;
    const double* x = rec + chain * N * D2;
    const int64_t n_terms = N - l_max;
    __shared__ double red[kAcfLags][kAcfThreads];
    double acc[kAcfLags];
    for (int k = 0; k < kAcfLags; ++k) acc[k] = 0.0;
    for (int i = threadIdx.x; i < D2; i += blockDim.x) {
        const int a = i / D, b = i % D;
        const double wt = (a == b) ? 1.0 : 2.0;
        double mean = 0.0;
        for (int64_t n = 0; n < N; ++n) mean += x[n * D2 + i];
        mean /= static_cast<double>(N);
        // sliding window x[n + l0 .. n + l0 + kAcfLags - 1]: two loads per
        // sample for all the group's lags (indices past the last sample,
        // which only lags beyond l_max would use, are clamped and discarded)
        auto at = [&](int64_t n) { return x[(n < N ? n : N - 1) * D2 + i]; };
        double win[kAcfLags], s[kAcfLags];
#pragma unroll
        for (int k = 0; k < kAcfLags; ++k) {
            win[k] = at(l0 + k);
            s[k] = 0.0;
        }
        for (int64_t n = 0; n < n_terms; ++n) {
            const double d0 = x[n * D2 + i] - mean;
#pragma unroll
            for (int k = 0; k < kAcfLags; ++k) s[k] += d0 * (win[k] - mean);
#pragma unroll
            for (int k = 0; k + 1 < kAcfLags; ++k) win[k] = win[k + 1];
            win[kAcfLags - 1] = at(n + l0 + kAcfLags);
        }
#pragma unroll
        for (int k = 0; k < kAcfLags; ++k)
            if (l0 + k <= l_max) acc[k] += wt * s[k];
    }
    for (int k = 0; k < kAcfLags; ++k) red[k][threadIdx.x] = acc[k];
    __syncthreads();
    if (threadIdx.x < kAcfLags) {
        const int l = l0 + threadIdx.x;
        double sum = 0.0;
        for (int t = 0; t < kAcfThreads; ++t) sum += red[threadIdx.x][t];
        if (l <= l_max) part[chain * (l_max + 1) + l] = sum;
    }
}

// out[l] = (sum over chains of part[.][l]) / (same at l = 0), one thread per lag
__global__ __launch_bounds__(kAcfThreads) void k_acf_final(const double* __restrict__ part, int64_t n_chains,
                                                           int l_max, double* out)
{
    for (int l = threadIdx.x; l <= l_max; l += blockDim.x) {
        double s = 0.0, s0 = 0.0;
        for (int64_t c = 0; c < n_chains; ++c) {
            s += part[c * (l_max + 1) + l];
            s0 += part[c * (l_max + 1)];
        }
        out[l] = s / s0;
    }
}

}  // namespace qst
