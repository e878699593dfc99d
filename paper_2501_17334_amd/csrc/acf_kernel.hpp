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

// grid: (lag chunks, chains); part[chain][l] = weighted lag sum of that chain
__global__ __launch_bounds__(kAcfThreads) void k_acf_partial(const double* __restrict__ rec, int64_t N, int D,
                                                             int l_max, double* part)
{
    const int D2 = D * D;
    const int64_t chain = blockIdx.y;
    const int l0 = blockIdx.x * kAcfLags;
    const double* x = rec + chain * N * D2;
    const int64_t n_terms = N - l_max;
    __shared__ double red[kAcfLags][kAcfThreads];
    double acc[kAcfLags];
    for (int k = 0; k < kAcfLags; ++k) acc[k] = 0.0;
    for (int i = threadIdx.x; i < D2; i += blockDim.x) {
        const int a = i / D, b = i % D;
        const double w = (a == b) ? 1.0 : 2.0;
        double mean = 0.0;
        for (int64_t n = 0; n < N; ++n) mean += x[n * D2 + i];
        mean /= static_cast<double>(N);
        for (int k = 0; k < kAcfLags; ++k) {
            const int l = l0 + k;
            if (l > l_max) break;
            double s = 0.0;
            for (int64_t n = 0; n < n_terms; ++n) s += (x[n * D2 + i] - mean) * (x[(n + l) * D2 + i] - mean);
            acc[k] += w * s;
        }
    }
    for (int k = 0; k < kAcfLags; ++k) red[k][threadIdx.x] = acc[k];
    __syncthreads();
    if (threadIdx.x < kAcfLags) {
        const int l = l0 + threadIdx.x;
        double s = 0.0;
        for (int t = 0; t < kAcfThreads; ++t) s += red[threadIdx.x][t];
        if (l <= l_max) part[chain * (l_max + 1) + l] = s;
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
