// Delayed acceptance (Christen & Fox, J. Comput. Graph. Stat. 2005) for the
// pCN chains: a cheap surrogate s(x) of log L screens every proposal before
// the exact likelihood is computed.  The pCN proposal leaves the N(0, I)
// prior invariant, so the prior terms cancel and the two stages are
//   stage 1: pass iff log u1 < s(y') - s(y);
//   stage 2: accept iff log u  < [log L(y') - log L(y)] - [s(y') - s(y)],
// which keeps the posterior exact whatever the surrogate.  u is the plain
// method's Metropolis-Hastings uniform, u1 an independent one (stream tag 2).
//
// One step of all chains is four launches: propose (y', BF16 copy for the
// network, the two uniforms), the network on every proposal (mlp_kernels.hpp),
// stage 1 (survivors appended to a list), and the exact likelihood plus
// stage 2 on the survivors only, one team per survivor.  The per-step state
// lives in HBM between launches.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "chain_kernel.hpp"
#include "mlp_kernels.hpp"

namespace qst {

struct DaArgs {
    ChainArgs A;            // chain state and run parameters
    double* s_cur;          // [R] surrogate value of the current state
    int64_t* n_stage1;      // [R] proposals that passed stage 1 in this call
    double* yprop;          // [R][d] proposal
    uint16_t* xb;           // [R][dp] proposal in BF16, zero padded to the network width dp
    int32_t dp;
    const float* smlp;      // [R] surrogate value of the proposal
    double* u_mh;           // [R] uniform of stage 2 (the Metropolis-Hastings uniform)
    double* u_da;           // [R] uniform of stage 1
    int32_t* surv;          // [R] chains that passed stage 1
    int32_t* n_surv;        // [1]
    int64_t chain0;         // the handle's chain offset (local chain c draws the numbers of chain0 + c)
    int64_t j;              // global index of the step (1-based)
    int64_t t;              // its index within this call
};

// Bookkeeping after the decision of step j for chain c, by one team of G
// lanes: adaptation window, moments, trace, record.
template <int Q, int G>
__device__ __forceinline__ void da_finish(const DaArgs& P, int64_t c, int lane, bool accept, double llprop,
                                          double logu)
{
    const ChainArgs& A = P.A;
    constexpr int D2 = Dims<Q>::D2;
    if (A.adapt_every > 0 && P.j % A.adapt_every == 0 && lane == 0) {
        double beta = A.beta[c];
        if (A.adapt_until < 0 || P.j <= A.adapt_until) {
            const double rate = static_cast<double>(A.acc_win[c]) / static_cast<double>(A.adapt_every);
            if (rate > A.adapt_hi) beta = fmin(beta * A.adapt_factor, 1.0);
            if (rate < A.adapt_lo) beta = beta / A.adapt_factor;
        }
        A.beta[c] = beta;
        A.acc_win[c] = 0;
    }
    if (P.j > A.burn_in && P.j % A.thin == 0) {
        for (int p = lane; p < D2; p += G) {
            const double r = A.rho_cur[c * D2 + p];
            A.s1[c * D2 + p] += r;
            A.s2[c * D2 + p] = __builtin_fma(r, r, A.s2[c * D2 + p]);
        }
        if (lane == 0) A.n_stored[c] += 1;
    }
    if (c < A.trace_chains && lane == 0) {
        const int64_t o = c * A.n_steps + P.t;
        if (A.tr_ll) A.tr_ll[o] = llprop;
        if (A.tr_lu) A.tr_lu[o] = logu;
        if (A.tr_acc) A.tr_acc[o] = accept ? 1 : 0;
    }
    if (A.record_every > 0 && c < A.record_chains && (P.t + 1) % A.record_every == 0) {
        const int64_t n_rec = A.n_steps / A.record_every;
        const int64_t slot = (P.t + 1) / A.record_every - 1;
        for (int p = lane; p < D2; p += G) A.rec[(c * n_rec + slot) * D2 + p] = A.rho_cur[c * D2 + p];
    }
}

// Launch 1: y' = sqrt(1 - beta^2) y + beta eta, its BF16 copy, the uniforms.
template <int Q, int G, int WG>
__global__ __launch_bounds__(WG) void k_da_propose(DaArgs P)
{
    using Dm = Dims<Q>;
    constexpr int d = Dm::d, NB = Dm::NB;
    constexpr int NJL = (NB + 2 + G - 1) / G;
    extern __shared__ double lds[];
    LogEntry* logtab = reinterpret_cast<LogEntry*>(lds);
    log_table_init(logtab, threadIdx.x, WG);
    __syncthreads();
    const ChainArgs& A = P.A;
    const int team = threadIdx.x / G, lane = threadIdx.x % G;
    const int64_t chain = static_cast<int64_t>(blockIdx.x) * (WG / G) + team;
    const bool live = chain < A.R;
    const int64_t c = live ? chain : 0;
    double* eta = lds + 2 * kLogTableSize + team * (d + 4);
#pragma unroll 1
    for (int e = 0; e < NJL; ++e) {
        const int job = lane + G * e;
        if (job < NB + 2) {
            const bool normal = job < NB;
            const uint64_t c0 = normal ? static_cast<uint64_t>(job) : 0;
            const uint64_t tag = normal ? kTagNormal : (job == NB ? kTagMH : kTagDA);
            const Block4 B = philox4x64_10(c0, static_cast<uint64_t>(P.j), static_cast<uint64_t>(P.chain0 + c), tag << 56,
                                           A.seed, 0);
            if (normal) {
                double n0, n1, n2, n3;
                box_muller(B.w[0], B.w[1], n0, n1, logtab);
                box_muller(B.w[2], B.w[3], n2, n3, logtab);
                const int i = 4 * job;
                eta[i] = n0;
                if (i + 1 < d) eta[i + 1] = n1;
                if (i + 2 < d) eta[i + 2] = n2;
                if (i + 3 < d) eta[i + 3] = n3;
            } else if (live) {
                (job == NB ? P.u_mh : P.u_da)[c] = uniform_open(B.w[0]);
            }
        }
    }
    __syncthreads();
    if (!live) return;
    const double beta = A.beta[c];
    const double a = sqrt(1.0 - beta * beta);
    for (int i = lane; i < d; i += G) {
        const double yp = __builtin_fma(beta, eta[i], a * A.x[c * d + i]);
        P.yprop[c * d + i] = yp;
        P.xb[c * P.dp + i] = bf16_bits(static_cast<float>(yp));
    }
    for (int i = d + lane; i < P.dp; i += G) P.xb[c * P.dp + i] = 0;
}

// Launch 3: stage 1, one wavefront per chain.
template <int Q>
__global__ __launch_bounds__(256) void k_da_stage1(DaArgs P)
{
    __shared__ LogEntry logtab[kLogTableSize];
    log_table_init(logtab, threadIdx.x, 256);
    __syncthreads();
    const ChainArgs& A = P.A;
    const int64_t c = static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (c >= A.R) return;
    const double dsh = static_cast<double>(P.smlp[c]) - P.s_cur[c];
    const bool pass = fast_log(P.u_da[c], logtab) < dsh;
    if (pass) {
        if (lane == 0) {
            const int k = atomicAdd(P.n_surv, 1);
            P.surv[k] = static_cast<int32_t>(c);
            P.n_stage1[c] += 1;
        }
        return;
    }
    da_finish<Q, 64>(P, c, lane, false, NAN, fast_log(P.u_mh[c], logtab));
}

// Launch 4: exact likelihood and stage 2 for the survivors, one team each.
template <int Q, int G, int WG>
__global__ __launch_bounds__(WG, (chain_min_waves<Q, G>())) void k_da_exact(DaArgs P)
{
    using Dm = Dims<Q>;
    using S = TeamShape<Q, G>;
    constexpr int d = Dm::d, D2 = Dm::D2;
    const ChainArgs& A = P.A;
    const int n = *P.n_surv;
    const int64_t first = static_cast<int64_t>(blockIdx.x) * (WG / G);
    if (first >= n) return;   // the whole workgroup has no survivor
    extern __shared__ double lds_all[];
    wg_tables_init<Q>(lds_all, threadIdx.x, WG);
    double* tables = lds_all;
    double* lds = lds_all + WgTables<Q>::kDoubles;
    const LogEntry* logtab = reinterpret_cast<const LogEntry*>(tables);
    const int team = threadIdx.x / G, lane = threadIdx.x % G;
    const int64_t k = first + team;
    const bool live = k < n;
    const int64_t c = live ? P.surv[k] : P.surv[0];
    double* base = lds + team * S::kLds;
    double* ybuf = base;
    double* pauli = base + S::kOffPauli;
    double* rhoP = base + S::kOffRho;
    double* wt = base + S::kOffWt;
    double* misc = base + S::kOffMisc;
    for (int i = lane; i < d; i += G) ybuf[i] = P.yprop[c * d + i];
    __syncthreads();
    double rp[S::NPL];
    stage_rho<Q, G>(ybuf, ybuf + 2 * D2, wt, rhoP, rp, lane);
    __syncthreads();
    stage_pauli<Q, G>(rhoP, pauli, lane);
    __syncthreads();
    double part_e = 0.0, part_f = 0.0;
    int bad = 0;
    stage_loglik<Q, G>(pauli, A.nd, A.mu, A.ndv, A.muv, tables, lane, part_e, part_f, bad);
    const double llp = team_loglik<G>(part_e, part_f, bad, misc + 4, lane);
    // teams without a survivor (the tail of the last workgroup) run along to
    // the barrier below but write nothing
    const double logu = fast_log(P.u_mh[c], logtab);
    const double sp = static_cast<double>(P.smlp[c]);
    const double delta = (llp - A.ll[c]) - (sp - P.s_cur[c]);
    const bool accept = logu < delta;
    if (live && accept) {
        for (int i = lane; i < d; i += G) A.x[c * d + i] = ybuf[i];
#pragma unroll
        for (int e = 0; e < S::NPL; ++e) {
            const int p = packed_slot<Q, G>(lane, e);
            if (p < D2) A.rho_cur[c * D2 + p] = rp[e];
        }
    }
    // every lane has read A.ll[c] and P.s_cur[c]; lane 0 owns the scalars
    __syncthreads();
    if (live && lane == 0) {
        if (accept) {
            A.ll[c] = llp;
            P.s_cur[c] = sp;
            A.acc_win[c] += 1;
            A.n_acc[c] += 1;
        }
        if (fabs(logu - delta) < 1e-8) A.n_near[c] += 1;
    }
    // the team's rho_cur writes are visible to its own moment update after the barrier
    __syncthreads();
    if (live) da_finish<Q, G>(P, c, lane, accept, llp, logu);
}

// x (FP64 [R][d]) -> BF16 [R][dp] zero padded; and s_cur = (double) smlp
__global__ void k_rows_to_bf16(const double* __restrict__ x, int64_t R, int d, int dp, uint16_t* __restrict__ xb)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= R * dp) return;
    const int64_t r = i / dp;
    const int k = static_cast<int>(i % dp);
    xb[i] = k < d ? bf16_bits(static_cast<float>(x[r * d + k])) : 0;
}

template <typename T>
__global__ void k_fill_zero(T* p, int64_t n)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = T(0);
}

__global__ void k_f32_to_f64(const float* __restrict__ in, int64_t n, double* __restrict__ out)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) out[i] = static_cast<double>(in[i]);
}

}  // namespace qst
