// Pooling of the per-chain moment sums into the estimate of Eq. (BME2)
// (Step 6 with phi(rho) = rho), with second moments and the between-chain
// standard error.  Two passes in a fixed order (chunks of chains, then the
// chunks in index order), so the result is bitwise reproducible.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qst {

constexpr int kPoolThreads = 256;

// part layout: [chunk][5][D2] sums of (S1, S2, m, m^2, has-samples) with
// m = S1_r / N_r the chain mean (chains without samples contribute 0), plus
// [chunk] sample totals in nsum.
__global__ __launch_bounds__(kPoolThreads) void k_pool_partial(const double* __restrict__ s1,
                                                               const double* __restrict__ s2,
                                                               const int64_t* __restrict__ nst,
                                                               int64_t R, int D2, int64_t chunk,
                                                               double* part, int64_t* nsum)
{
    const int64_t r0 = static_cast<int64_t>(blockIdx.x) * chunk;
    const int64_t r1 = r0 + chunk < R ? r0 + chunk : R;
    for (int i = threadIdx.x; i < D2; i += blockDim.x) {
        double a = 0.0, b = 0.0, m = 0.0, mm = 0.0, cnt = 0.0;
        // unrolled so that the loads of several chains are in flight at
        // once; every sum still runs over the chains in index order
#pragma unroll 8
        for (int64_t r = r0; r < r1; ++r) {
            const double x1 = s1[r * D2 + i];
            a += x1;
            b += s2[r * D2 + i];
            const int64_t n = nst[r];
            if (n > 0) {
                const double mean = x1 / static_cast<double>(n);
                m += mean;
                mm += mean * mean;
                cnt += 1.0;
            }
        }
        double* o = part + static_cast<int64_t>(blockIdx.x) * 5 * D2;
        o[i] = a;
        o[D2 + i] = b;
        o[2 * D2 + i] = m;
        o[3 * D2 + i] = mm;
        o[4 * D2 + i] = cnt;
    }
    if (threadIdx.x == 0) {
        int64_t n = 0;
        for (int64_t r = r0; r < r1; ++r) n += nst[r];
        nsum[blockIdx.x] = n;
    }
}

// out layout (doubles): mean [D2*2] interleaved complex, second [D2*2]
// (E[(Re a)^2], E[(Im a)^2]), se [D2*2]; nout[0] = total samples.  One
// thread per matrix element, ceil(D2 / kPoolThreads) workgroups.
__global__ __launch_bounds__(kPoolThreads) void k_pool_final(const double* __restrict__ part,
                                                             const int64_t* __restrict__ nsum,
                                                             int nchunks, int D, double* out,
                                                             int64_t* nout)
{
    const int D2 = D * D;
    __shared__ int64_t ntot_s;
    if (threadIdx.x == 0) {
        int64_t n = 0;
        for (int c = 0; c < nchunks; ++c) n += nsum[c];
        ntot_s = n;
        if (blockIdx.x == 0) nout[0] = n;
    }
    __syncthreads();
    const double ntot = static_cast<double>(ntot_s);
    const int p = static_cast<int>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p < D2) {
        const int a = p / D, b = p % D;
        const int up = (a <= b) ? a * D + b : b * D + a;   // packed slot of Re rho_ab
        const int lo = (a <= b) ? b * D + a : a * D + b;   // packed slot of Im of the upper element
        double sums[2][5] = {};
        const int slots[2] = {up, lo};
        // the ten sums side by side (their loads overlap), each over the
        // chunks in index order
#pragma unroll 4
        for (int c = 0; c < nchunks; ++c) {
            const double* pc = part + static_cast<int64_t>(c) * 5 * D2;
#pragma unroll
            for (int s = 0; s < 2; ++s)
#pragma unroll
                for (int k = 0; k < 5; ++k) sums[s][k] += pc[k * D2 + slots[s]];
        }
        const double im_sign = (a < b) ? 1.0 : -1.0;
        const bool diag = (a == b);
        // mean
        out[2 * p] = sums[0][0] / ntot;
        out[2 * p + 1] = diag ? 0.0 : im_sign * sums[1][0] / ntot;
        // second moments
        out[2 * D2 + 2 * p] = sums[0][1] / ntot;
        out[2 * D2 + 2 * p + 1] = diag ? 0.0 : sums[1][1] / ntot;
        // between-chain standard error of the chain means
        for (int s = 0; s < 2; ++s) {
            const double R = sums[s][4];
            double se = 0.0;
            if (R > 1.0) {
                const double var = (sums[s][3] - sums[s][2] * sums[s][2] / R) / (R - 1.0);
                se = sqrt(fmax(var, 0.0) / R);
            }
            out[4 * D2 + 2 * p + s] = (s == 1 && diag) ? 0.0 : se;
        }
    }
}

}  // namespace qst
