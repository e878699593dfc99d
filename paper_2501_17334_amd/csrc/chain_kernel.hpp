// The fused pCN chain step on gfx950: Algorithm 2 of the paper for a tile of
// independent chains, every step of every chain inside one kernel launch.
//
// Work decomposition.  A "team" of G consecutive threads owns one chain; a
// workgroup of WG threads holds WG/G teams (G <= 64 keeps a team inside one
// 64-wide wavefront, G = 128/256/512 spreads a large chain over several).
// The chain state y (d = 2D^2+D doubles), the packed rho of the current
// state and its moment sums stay in registers for the whole launch; the only
// global-memory traffic of the step loop is the count vector and the Pauli
// index table (read-only, L2 resident) and the optional traces and records.
// LDS holds, per team, the proposal y' (read back as the matrix Z), the
// column weights, the packed rho', the Pauli coefficients and a ring of
// Philox values drawn ahead for the next steps; per workgroup, the logarithm
// table.  Teams of at most one wavefront synchronise with
// wavefront-scope fences only.
//
// One step, per team (sections of the paper in brackets):
//  1. Philox jobs: normal block b -> 4 normals of eta (Box-Muller), plus one
//     job for the Metropolis-Hastings uniform; y' = sqrt(1-beta^2) y + beta eta
//     [Alg. 2, proposal]
//  2. w_j = v_j^2 / sum v^2 / |z_j|^2 and packed rho(y') = sum_j w_j z_j z_j^dag,
//     on FP64 MFMA from 4 qubits up [parameterisation]
//  3. Pauli coefficients c_mu = Tr(rho sigma_mu), 4^Q of them, each a signed
//     sum of D entries of rho (sigma_mu has one non-zero per row)
//  4. per setting k, p_kl = 2^-Q sum_t c_mu(k,t) (-1)^popcount(l&t): a
//     2^Q-point Walsh-Hadamard transform across the lanes of a D-lane group
//     (Tr(sigma_mu Lambda_kl) factorises over qubits) [Step 1, Eq. (likelihood)]
//  5. log L(y') = sum_{c>0} c log p, team-reduced in a fixed order [Eq. (likelihood)]
//  6. accept iff log u < log L(y') - log L(y) [Alg. 2]; adaptation every M_A
//     steps; thinning and the moment sums [Alg. 2; Eq. (BME2)].
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <type_traits>

#include "fastmath.hpp"
#include "rng.hpp"

namespace qst {

__host__ __device__ constexpr int pow3(int q) { return q == 0 ? 1 : 3 * pow3(q - 1); }

template <int Q>
struct Dims {
    static constexpr int D = 1 << Q;
    static constexpr int D2 = D * D;
    static constexpr int d = 2 * D2 + D;   // parameters of rho(x)
    static constexpr int K = pow3(Q);      // Pauli settings
    static constexpr int KD = K * D;       // projectors
    static constexpr int NB = (d + 3) / 4; // Philox blocks of normals per step
};

// Everything a chain launch needs; plain pointers into the problem's buffers.
struct ChainArgs {
    const double* nd;       // [KD] counts as doubles
    const uint16_t* mu;     // [KD] Pauli index of every (setting, transform position)
    const double* ndv;      // [KD] counts, task-major order of the likelihood transforms (LikSplit)
    const uint16_t* muv;    // [KD] Pauli indices in the same order
    const void* mfrag;      // dense path: the Pauli matrix in MFMA fragment order
    // Chains c < R.  The chain kernels use problem-wide indices c in
    // [chain0, R) with chain0 the handle's chain offset (a kernel argument of
    // its own): the host passes every per-chain array (and the trace and
    // record buffers) shifted back by chain0 rows, so that row c is chain c's,
    // and the trace/record bounds as problem-wide indices; c is also the
    // Philox counter word.  Delayed acceptance passes unshifted arrays and
    // local indices in [0, R), and adds its chain0 for the counter word.
    int64_t R;
    double* x;              // [R][d] current state
    double* ll;             // [R] log L of the current state
    double* beta;           // [R]
    int32_t* acc_win;       // [R] acceptances in the current adaptation window
    double* rho_cur;        // [R][D2] packed rho of the current state
    double* s1;             // [R][D2] sum of stored packed rho
    double* s2;             // [R][D2] sum of squares
    int64_t* n_stored;      // [R]
    int64_t* n_acc;         // [R] accepts in this call
    int64_t* n_near;        // [R] near-threshold decisions in this call
    int64_t step_begin;     // this call runs steps step_begin+1 .. step_begin+n_steps
    int64_t n_steps;
    int64_t burn_in;
    int64_t adapt_until;
    int32_t thin;
    int32_t adapt_every;
    int32_t init;           // 1: draw y^0 (step 0) and evaluate it first
                            //    (log L, packed rho) and keep the rest of it
    int32_t poisson;        // 1: Poisson counts: log L -= sum_p W[p] rho_p, W = nd + KD (packed)
    double beta0;
    double adapt_lo, adapt_hi, adapt_factor;
    uint64_t seed;
    double alpha, lg_alpha;  // Dirichlet weights: concentration and lgamma(alpha)
    int32_t trace_chains;
    double* tr_ll;
    double* tr_lu;
    int8_t* tr_acc;
    int32_t record_every;
    int32_t record_chains;
    double* rec;
    // training pairs for the surrogate: every pair_every steps, the proposal
    // y' (BF16, zero padded to pair_width) and its log L of the first
    // pair_chains chains, row slot * pair_chains + chain
    int32_t pair_every;
    int32_t pair_chains;
    int32_t pair_width;
    uint16_t* pair_x;
    double* pair_ll;
};

// How p = Tr(Lambda rho) is formed inside the chain step.
enum : int { kPathKron = 0, kPathDense = 1 };
// Parameterisation rho(x): the Gaussian/gamma form (d = 2D^2 + D), the
// paper's Algorithm 1, the Bures draw (d = 4D^2), or the Gaussian/gamma form
// with Dirichlet(alpha) weights (d = 2D^2 + D).
enum : int { kParamGamma = 0, kParamBures = 1, kParamDirichlet = 2 };

template <int Q, int PARAM>
struct ParamDims {
    static constexpr int D = 1 << Q, D2 = D * D;
    static constexpr int d = PARAM == kParamBures ? 4 * D2 : 2 * D2 + D;
    static constexpr int NB = (d + 3) / 4;   // Philox blocks of normals per step
};
// Arithmetic of the dense contraction (the log-likelihood sum is FP64 always).
enum : int { kPrecF64 = 0, kPrecF32 = 1, kPrecBF16x3 = 2 };

// Sizes of the dense contraction p = M vec(rho) for one workgroup of 16
// chains: M is KD x D^2 (rows padded to 16 for the MFMA tiles, columns to
// 32 for the BF16 k-steps).
template <int Q>
struct DenseShape {
    static constexpr int KD = Dims<Q>::KD;
    static constexpr int KDP = (KD + 15) / 16 * 16;
    static constexpr int NT = KDP / 16;              // 16-row output tiles
    static constexpr int K = Dims<Q>::D2;
    static constexpr int KS4 = K / 4;                // k-steps of the 16x16x4 FP64/FP32 MFMA
    static constexpr int KP32 = (K + 31) / 32 * 32;
    static constexpr int KS32 = KP32 / 32;           // k-steps of the 16x16x32 BF16 MFMA
    static constexpr int kChains = 16;               // MFMA N dimension = chains per workgroup
    // B-operand staging per chain: FP32 copy or three BF16 parts (in doubles)
    static constexpr int kStageDoubles = (6 * KP32 + 7) / 8;
};

template <int Q, int G, int PATH = kPathKron, int PARAM = kParamGamma>
struct TeamShape {
    using Dm = Dims<Q>;
    static_assert(G >= Dm::D, "a team must hold one D-lane transform group");
    static_assert(G <= 64 ? (64 % G == 0) : (G % 64 == 0), "team size must tile wavefronts");
    static constexpr int d = ParamDims<Q, PARAM>::d;     // parameters of rho(x)
    static constexpr int NB = ParamDims<Q, PARAM>::NB;   // Philox blocks of normals per step
    static constexpr int NJL = (NB + 1 + G - 1) / G;      // Philox jobs per lane (normals + MH uniform)
    static constexpr int NYL = (d + G - 1) / G;           // state entries per lane (strided)
    static constexpr int NPL = (Dm::D2 + G - 1) / G;      // packed rho entries per lane (strided)
    static constexpr int NFL = (Dm::KD + G - 1) / G;      // projector outputs per lane
    static constexpr int kMisc = 24;                      // per-team scratch doubles
    // the Pauli-coefficient region doubles as the dense path's B-operand staging
    static constexpr int kPauliDoubles =
        PATH == kPathDense && DenseShape<Q>::kStageDoubles > Dm::D2 ? DenseShape<Q>::kStageDoubles : Dm::D2;
    // per-team LDS (doubles): y' | Pauli coefficients | packed rho' | column weights | scratch.
    // Algorithm 1 uses the Pauli and rho' regions (2 D^2 doubles) as its QR
    // and product workspace before rho' is formed.
    static constexpr int kOffPauli = d;
    static constexpr int kOffRho = kOffPauli + kPauliDoubles;
    static constexpr int kOffWt = kOffRho + Dm::D2;
    static constexpr int kOffMisc = kOffWt + Dm::D;
    static constexpr int kLdsRaw = kOffMisc + kMisc;
    // dense path: 16 teams are read side by side; a stride of 16k+1 doubles
    // keeps the 16 lanes of an MFMA column group on distinct LDS banks
    static constexpr int kLds = PATH == kPathDense ? (kLdsRaw + 14) / 16 * 16 + 1 : kLdsRaw;
    // Philox jobs of a step: whole passes over the team, then a tail of kTail
    // jobs.  On the Kronecker path the tails of kRing consecutive steps are
    // drawn together in one pass into an LDS ring behind the team's area, so
    // that a step does not pay a whole pass for a few lanes (kRing = 1: no
    // ring).  kRing is capped so that the ring does not lower the number of
    // workgroups per CU of the tuned launch shape (LDS is the limit there).
    static constexpr int kJobs = NB + 1;
    static constexpr int kFullJobs = kJobs / G * G;
    static constexpr int kTail = kJobs - kFullJobs;
    static constexpr int kRingCap = Q == 1 ? 2 : Q == 2 ? 3 : Q == 3 ? 10 : Q == 4 ? 6 : Q == 5 ? 18 : 30;
    static constexpr int kRingFit = kTail > 0 ? G / kTail : 1;
    static constexpr int kRing =
        PATH == kPathKron && kTail > 0 ? (kRingFit < kRingCap ? kRingFit : kRingCap) : 1;
    static constexpr int kRingDoubles = kRing > 1 ? 4 * kTail * kRing : 0;
    static constexpr int kLdsChain = kLds + kRingDoubles;   // per team, in the chain kernels
};

// Per-workgroup tables at the start of LDS, ahead of the teams: the
// logarithm breakpoints (and, on the dense path, the per-wave partial
// log-likelihoods).  The Pauli index of every (setting, transform position)
// comes from a per-problem table in global memory (ChainArgs::mu), loaded one
// iteration ahead in the likelihood loop; in LDS it would cost two dependent
// reads per projector and, at 5 qubits, a quarter of the workgroup's LDS.
template <int Q, int PATH = kPathKron>
struct WgTables {
    static constexpr int kLogDoubles = 2 * kLogTableSize;
    // dense path: per-wave partial log-likelihoods [16 waves][16 chains][3]
    static constexpr int kRedDoubles = PATH == kPathDense ? 16 * 16 * 3 : 0;
    static constexpr int kOffRed = kLogDoubles;
    static constexpr int kDoubles = kOffRed + kRedDoubles;
};

template <int Q, int PATH = kPathKron>
__device__ __forceinline__ void wg_tables_init(double* lds, int tid, int nthreads)
{
    log_table_init(reinterpret_cast<LogEntry*>(lds), tid, nthreads);
}

// ---------------------------------------------------------------------------
// team collectives (deterministic: every lane ends with the same bits)
// ---------------------------------------------------------------------------
// v + its partners across lane bits O, O/2, ..., 1 (in that order)
template <int O>
__device__ __forceinline__ double butterfly_sum(double v)
{
    v += xor_lane<O>(v);
    if constexpr (O > 1) return butterfly_sum<O / 2>(v);
    else return v;
}

template <int G>
__device__ __forceinline__ double team_sum(double v, double* scratch, int lane)
{
    if constexpr (G == 1) {
        return v;
    } else if constexpr (G <= 64) {
        return butterfly_sum<G / 2>(v);
    } else {
        v = butterfly_sum<32>(v);
        if ((lane & 63) == 0) scratch[lane >> 6] = v;
        __syncthreads();
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < G / 64; ++w) s += scratch[w];
        __syncthreads();
        return s;
    }
}

// 1/sqrt(x) for x > 0 in FP64: the hardware reciprocal square root refined by
// two Newton steps r <- r + r (1 - x r^2) / 2, which square its relative
// error each time.
__device__ __forceinline__ double rsqrt_f64(double x)
{
    double r = __builtin_amdgcn_rsq(x);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const double e = __builtin_fma(-x * r, r, 1.0);
        r = __builtin_fma(0.5 * r, e, r);
    }
    return r;
}

// log L of a team from the lanes' shares (sum c e, sum c frac, any p <= 0 with
// a count): one reduction of e ln2 + frac per lane, -inf if a lane saw a bad
// probability.
template <int G>
__device__ __forceinline__ double team_loglik(double part_e, double part_f, int bad, double* scratch, int lane)
{
    const double part = bad ? -INFINITY : __builtin_fma(part_e, kLn2, part_f);
    return team_sum<G>(part, scratch, lane);
}

// The linear part of the Poisson log-likelihood, sum_m lambda_m p_m =
// Tr(rho Lambda) with Lambda = sum_m lambda_m Pi_m, as the dot product of
// packed rho with the packed weights W of Lambda (W[a][a] = Lambda_aa,
// W[a][b] = 2 Re Lambda_ab and W[b][a] = 2 Im Lambda_ab for a < b): this
// lane's share, p = lane, lane + G, ...
template <int Q, int G>
__device__ __forceinline__ double linear_share(const double* __restrict__ W, const double* rhoP, int lane)
{
    double s = 0.0;
    for (int p = lane; p < Dims<Q>::D2; p += G) s = __builtin_fma(W[p], rhoP[p], s);
    return s;
}

// Synchronisation of one team's LDS traffic.  A team of at most 64 lanes
// lives inside one wavefront and its LDS region is its own; the LDS performs
// a wavefront's operations in issue order, so ordering the compiler with a
// wavefront-scope fence is enough and the team never waits for the other
// wavefronts of its workgroup.  Wider teams take the workgroup barrier.
template <int G>
__device__ __forceinline__ void team_sync()
{
    if constexpr (G <= 64) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// stages on LDS
// ---------------------------------------------------------------------------

// The packed-rho entries a lane owns: p = lane + G e, except on the MFMA
// path, where rho is formed by 16x16x4 FP64 MFMAs tile by tile: the D x D
// result is (D/16)^2 tiles of 16 x 16, the team's wavefronts take equal
// shares of them, and a lane owns, per tile, the four entries of the MFMA
// result layout (row lane % 64 / 16 + 4 r, column lane % 16 of the tile).
// Used for one-wave 4-qubit teams and for 5- and 6-qubit teams whose
// wavefront count divides the tile count.
template <int Q, int G>
struct RhoLayout {
    static constexpr int kTileDim = Q >= 4 ? (1 << (Q - 4)) : 0;   // tiles per row of rho
    static constexpr int kTiles = kTileDim * kTileDim;
    static constexpr int kWaves = G >= 64 ? G / 64 : 0;
    static constexpr bool kMfma =
        (Q == 4 && G == 64) || (Q >= 5 && kWaves > 0 && kTiles % (kWaves > 0 ? kWaves : 1) == 0);
    static constexpr int kTilesPerWave = kMfma ? kTiles / kWaves : 0;
};

template <int Q, int G>
__device__ __forceinline__ int packed_slot(int lane, int e)
{
    using L = RhoLayout<Q, G>;
    if constexpr (L::kMfma) {
        constexpr int D = 1 << Q;
        const int tile = (lane >> 6) * L::kTilesPerWave + (e >> 2);
        const int rb = tile / L::kTileDim, cb = tile % L::kTileDim;
        const int l = lane & 63;
        return (16 * rb + (l >> 4) + 4 * (e & 3)) * D + 16 * cb + (l & 15);
    } else {
        return lane + G * e;
    }
}

// ---------------------------------------------------------------------------
// Dirichlet(alpha) weights: gamma_j = P^{-1}(alpha, Phi(v_j)), the Gamma(alpha)
// quantile of the normal probability of v_j, so that x ~ N(0, I) maps to
// Dirichlet(alpha) weights w_j = gamma_j / sum_k gamma_k and the pCN ratio of
// Algorithm 2 stays exact.
// ---------------------------------------------------------------------------
// Regularised incomplete gamma at x = e^t (a > 0): P by its power series
// below x = a + 1, Q = 1 - P by the Legendre continued fraction (modified
// Lentz) above it; returns the one that is accurate (P below, Q above) with
// `upper` telling which.
__device__ __forceinline__ double gamma_pq_dev(double a, double t, double lg_a, bool& upper)
{
    const double x = exp(t);
    const double pre = exp(a * t - x - lg_a);   // x^a e^-x / Gamma(a)
    if (x < a + 1.0) {
        upper = false;
        double term = 1.0 / a, sum = term;
        for (int n = 1; n < 500; ++n) {
            term *= x / (a + n);
            sum += term;
            if (term < sum * 1e-17) break;
        }
        return sum * pre;
    }
    upper = true;
    // Q = pre / (b1 - 1(1-a) / (b2 - 2(2-a) / (b3 - ...))), b_n = x + 2n - 1 - a
    const double tiny = 1e-300;
    double b = x + 1.0 - a, c = 1.0 / tiny, dd = 1.0 / b, h = dd;
    for (int n = 1; n < 500; ++n) {
        const double an = -n * (n - a);
        b += 2.0;
        dd = an * dd + b;
        if (fabs(dd) < tiny) dd = tiny;
        c = b + an / c;
        if (fabs(c) < tiny) c = tiny;
        dd = 1.0 / dd;
        const double del = dd * c;
        h *= del;
        if (fabs(del - 1.0) < 1e-16) break;
    }
    return pre * h;
}

// log x of the Gamma(a) quantile at probability Phi(v): Halley steps on
// t = log x for P(a, e^t) = Phi(v) (v <= 0) or Q(a, e^t) = Phi(-v) (v > 0),
// both increasing in t with first derivative g = x^a e^-x / Gamma(a) and
// g'/g = a - x; started from the Wilson-Hilferty cube (whose normal quantile
// is v itself) or, where that is not positive, from the leading term of the
// series or of the tail.  Convergence is cubic: once a step is below 1e-5
// one more step reaches full precision, and the iteration stops there.
__device__ __forceinline__ double gamma_quantile_log(double a, double v, double lg_a)
{
    const double target = 0.5 * erfc((v <= 0.0 ? -v : v) * 0.70710678118654752440);   // Phi(-|v|)
    const double c = 1.0 / (9.0 * a);
    const double wh = 1.0 - c + v * sqrt(c);
    double t = wh > 0.1 ? log(a) + 3.0 * log(wh)
                        : (v <= 0.0 ? (log(target) + lg_a + log(a)) / a : log(a + 1.0) - log(target));
    bool last = false;
    for (int it = 0; it < 40; ++it) {
        bool upper;
        const double f = gamma_pq_dev(a, t, lg_a, upper);
        // residual of the increasing function of t: P - u, or (1 - Q) - (1 - q) = q - Q
        double r;
        if (v <= 0.0) r = upper ? (1.0 - f) - target : f - target;
        else r = upper ? target - f : (f - (1.0 - target));
        const double x = exp(t);
        const double newton = r / exp(a * t - x - lg_a);
        const double corr = 1.0 - 0.5 * newton * (a - x);   // Halley: divide by 1 - f f'' / (2 f'^2)
        double step = corr > 0.5 ? newton / corr : newton;
        step = fmax(fmin(step, 2.0), -2.0);
        t -= step;
        if (last) break;
        last = fabs(step) < 1e-5 * fmax(1.0, fabs(t));
    }
    return t;
}

// v_j = sqrt(gamma_j / sum_k gamma_k) into vbuf (the team's LDS), so that the
// weights of stage_rho, v_j^2 / sum_k v_k^2, are the Dirichlet weights.
template <int Q, int G>
__device__ __forceinline__ void stage_dirichlet_v(const double* ybuf, double* vbuf, double alpha, double lg_alpha,
                                                  double* scratch, int lane)
{
    constexpr int D = 1 << Q, D2 = D * D;
    for (int j = lane; j < D; j += G) vbuf[j] = exp(gamma_quantile_log(alpha, ybuf[2 * D2 + j], lg_alpha));
    team_sync<G>();
    double part = 0.0;
    for (int j = lane; j < D; j += G) part += vbuf[j];
    const double gs = team_sum<G>(part, scratch, lane);
    team_sync<G>();
    for (int j = lane; j < D; j += G) vbuf[j] = sqrt(vbuf[j] / gs);
    team_sync<G>();
}

// Column weights w_j = (v_j^2 / sum_k v_k^2) / |z_j|^2 from Z in ybuf (x
// layout) and v in vbuf.
template <int Q, int G>
__device__ __forceinline__ void stage_weights(const double* ybuf, const double* vbuf, double* wt, int lane)
{
    using Dm = Dims<Q>;
    constexpr int D = Dm::D, D2 = Dm::D2;
    double V = 0.0;
#pragma unroll 4
    for (int j = 0; j < D; ++j) {
        const double v = vbuf[j];
        V += v * v;
    }
    for (int j = lane; j < D; j += G) {
        double nz = 0.0;
        for (int i = 0; i < D; ++i) {
            const double re = ybuf[j * D + i];
            const double im = ybuf[D2 + j * D + i];
            nz += re * re + im * im;
        }
        const double v = vbuf[j];
        const double w = (v * v / V) / nz;
        wt[j] = w;
    }
}

// Packed rho = sum_j w_j z_j z_j^dag into rhoP (LDS) and rp (this lane's
// slots): entry (a, b) is sum_j w_j Re(z_aj conj z_bj) for a <= b and
// sum_j w_j Im(z_bj conj z_aj) for a > b.  Z from ybuf (x layout), the
// weight parameters v_j from vbuf (x[2D^2 + j], or their Dirichlet form).
// F32 (the mixed-precision Kronecker form, whose likelihood reads rho'
// rounded to FP32): at 4 qubits the Gram products run on the FP32 matrix
// pipe, at twice the rate of the FP64 one.
template <int Q, int G, bool F32 = false, bool RP = true>
__device__ __forceinline__ void stage_rho(const double* ybuf, const double* vbuf, double* wt, double* rhoP,
                                          double (&rp)[TeamShape<Q, G>::NPL], int lane)
{
    using Dm = Dims<Q>;
    using S = TeamShape<Q, G>;
    constexpr int D = Dm::D, D2 = Dm::D2;
    if constexpr (RhoLayout<Q, G>::kMfma && Q >= 5) {
        // The same Gram products tile by tile.  Column weights first: G / D
        // lanes share a column, sum |z_ij|^2 over their rows and combine by
        // butterflies; sqrt(w_j) goes to LDS for the operand loads.
        using L = RhoLayout<Q, G>;
        constexpr int LPC = G / D;          // lanes per column: 2, 4, 8 or 16
        constexpr int RPL = D / LPC;        // rows per lane
        static_assert(LPC >= 2 && LPC <= 16, "column groups must sit inside a DPP row");
        static_assert(D == 32 || D == 64, "one wavefront spans the v_j");
        // V = sum_j v_j^2 within each wavefront: lane l squares v_(l mod D)
        double V;
        {
            const double v = vbuf[lane & (D - 1)];
            V = butterfly_sum<D / 2>(v * v);
        }
        {
            // lane (j, q) sums rows q RPL .. q RPL + RPL - 1 of column j.  At
            // 6 qubits it starts at row offset j mod RPL, so that the columns
            // of a wavefront (eight in a 512-thread team, four in a 1024-thread
            // one) read different LDS banks at every r (unrotated, all of them
            // read the same bank pairs: 6 qubits 163 -> 157 ns per
            // chain-step); at 5 qubits the rotation's address arithmetic cost
            // more than its fewer conflicts saved
            const int j = lane / LPC, q = lane % LPC;
            const int rot = Q >= 6 ? j : 0;
            double nz = 0.0;
#pragma unroll 4
            for (int r = 0; r < RPL; ++r) {
                const int i = q * RPL + ((r + rot) & (RPL - 1));
                const double re = ybuf[j * D + i];
                const double im = ybuf[D2 + j * D + i];
                nz += re * re + im * im;
            }
            nz += xor_lane<1>(nz);
            if constexpr (LPC >= 4) nz += xor_lane<2>(nz);
            if constexpr (LPC >= 8) nz += xor_lane<4>(nz);
            if constexpr (LPC >= 16) nz += xor_lane<8>(nz);
            if (q == 0) {
                const double v = vbuf[j];
                wt[j] = sqrt((v * v / V) / nz);
            }
        }
        __syncthreads();
        typedef double double4_t __attribute__((ext_vector_type(4)));
        typedef float float4_t __attribute__((ext_vector_type(4)));
        using acc_t = std::conditional_t<F32, float4_t, double4_t>;
        const int l = lane & 63, i = l & 15, kq = l >> 4;
#pragma unroll
        for (int m = 0; m < L::kTilesPerWave; ++m) {
            const int tile = (lane >> 6) * L::kTilesPerWave + m;
            const int r0 = 16 * (tile / L::kTileDim), c0 = 16 * (tile % L::kTileDim);
            acc_t re = {}, im = {};
            // the packed form keeps Re above the diagonal and Im below it, so
            // a tile off the diagonal needs one of the two products
            auto gram = [&](auto want_re, auto want_im) {
#pragma unroll 4
                for (int s = 0; s < D / 4; ++s) {
                    const int j = 4 * s + kq;
                    const double sj = wt[j];
                    const double ar = ybuf[j * D + r0 + i] * sj;
                    const double ai = ybuf[D2 + j * D + r0 + i] * sj;
                    const double br = ybuf[j * D + c0 + i] * sj;
                    const double bi = ybuf[D2 + j * D + c0 + i] * sj;
                    if constexpr (F32) {
                        const float far = static_cast<float>(ar), fai = static_cast<float>(ai);
                        const float fbr = static_cast<float>(br), fbi = static_cast<float>(bi);
                        if constexpr (decltype(want_re)::value) {
                            re = __builtin_amdgcn_mfma_f32_16x16x4f32(far, fbr, re, 0, 0, 0);
                            re = __builtin_amdgcn_mfma_f32_16x16x4f32(fai, fbi, re, 0, 0, 0);
                        }
                        if constexpr (decltype(want_im)::value) {
                            im = __builtin_amdgcn_mfma_f32_16x16x4f32(fai, fbr, im, 0, 0, 0);
                            im = __builtin_amdgcn_mfma_f32_16x16x4f32(-far, fbi, im, 0, 0, 0);
                        }
                    } else {
                        if constexpr (decltype(want_re)::value) {
                            re = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, br, re, 0, 0, 0);
                            re = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, bi, re, 0, 0, 0);
                        }
                        if constexpr (decltype(want_im)::value) {
                            im = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, br, im, 0, 0, 0);
                            im = __builtin_amdgcn_mfma_f64_16x16x4f64(-ar, bi, im, 0, 0, 0);
                        }
                    }
                }
            };
            using yes = std::true_type;
            using no = std::false_type;
            // result register r of lane l: row l/16 + 4 r (FP64) or 4 (l/16) + r
            // (FP32) of the tile, column l%16
            auto row_of = [&](int r) { return F32 ? 4 * kq + r : kq + 4 * r; };
            if (r0 != c0) {
                if (r0 < c0) gram(yes{}, no{});
                else gram(no{}, yes{});
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int a = r0 + row_of(r), b = c0 + i;
                    const double v = a <= b ? static_cast<double>(re[r]) : -static_cast<double>(im[r]);
                    if constexpr (!F32) rp[4 * m + r] = v;
                    rhoP[a * D + b] = v;
                }
            } else {
                // a diagonal tile: Im = X - X^T with X = Zi Zr^T over the tile's
                // rows (one product instead of two), X transposed through the
                // tile's own LDS slots, which only this wavefront writes.  Re
                // comes from the same X: with Zp = Zr + Zi, Zp Zp^T =
                // Re + X + X^T, so Re = Zp Zp^T - X - X^T (two products per
                // tile instead of three)
                acc_t x = {};
#pragma unroll 4
                for (int s = 0; s < D / 4; ++s) {
                    const int j = 4 * s + kq;
                    const double sj = wt[j];
                    const double ar = ybuf[j * D + r0 + i] * sj;
                    const double ai = ybuf[D2 + j * D + r0 + i] * sj;
                    if constexpr (F32) {
                        const float far = static_cast<float>(ar), fai = static_cast<float>(ai);
                        const float fap = far + fai;
                        re = __builtin_amdgcn_mfma_f32_16x16x4f32(fap, fap, re, 0, 0, 0);
                        x = __builtin_amdgcn_mfma_f32_16x16x4f32(fai, far, x, 0, 0, 0);
                    } else {
                        const double ap = ar + ai;
                        re = __builtin_amdgcn_mfma_f64_16x16x4f64(ap, ap, re, 0, 0, 0);
                        x = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, ar, x, 0, 0, 0);
                    }
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) rhoP[(r0 + row_of(r)) * D + c0 + i] = static_cast<double>(x[r]);
                team_sync<64>();
                double xt[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) xt[r] = rhoP[(r0 + i) * D + c0 + row_of(r)];   // X at (column, row)
                team_sync<64>();
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int a = r0 + row_of(r), b = c0 + i;
                    // P[a][b] = Im rho_ba = X_ba - X_ab below the diagonal
                    const double xr = static_cast<double>(x[r]);
                    const double v = a <= b ? (static_cast<double>(re[r]) - xr) - xt[r] : xt[r] - xr;
                    if constexpr (!F32) rp[4 * m + r] = v;
                    rhoP[a * D + b] = v;
                }
            }
        }
        if constexpr (F32 && RP) {   // this lane's packed slots, written by other lanes
            __syncthreads();
#pragma unroll
            for (int e = 0; e < S::NPL; ++e) rp[e] = rhoP[packed_slot<Q, G>(lane, e)];
        }
    } else if constexpr (RhoLayout<Q, G>::kMfma) {
        // rho = Zs Zs^dag with Zs = Z diag(sqrt w): Re rho = Zr Zr^T + Zi Zi^T and
        // Im rho = Zi Zr^T - Zr Zi^T, 16x16 real products with K = 16, four
        // v_mfma_f64_16x16x4f64 each.  Operand lane l carries
        // A[l % 16][k0 + l / 16]; for a Gram product the B operand is the same
        // value.  The lane already holds z_ij for its four columns j, so the
        // column norms |z_j|^2 are butterfly sums over the 16 lanes of its row
        // group and the weights never pass through LDS.
        const int i = lane & 15, kq = lane >> 4;
        // V = sum_j v_j^2 by a butterfly over each row of 16 lanes
        double V;
        {
            const double v = vbuf[i];
            V = butterfly_sum<8>(v * v);
        }
        double zr[4], zi[4], nzt[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int j = 4 * t + kq;
            zr[t] = ybuf[j * D + i];
            zi[t] = ybuf[D2 + j * D + i];
            double nz = zr[t] * zr[t] + zi[t] * zi[t];
            nz += xor_lane<1>(nz);
            nz += xor_lane<2>(nz);
            nz += xor_lane<4>(nz);
            nz += xor_lane<8>(nz);
            nzt[t] = nz;
        }
        // sqrt(w_j) = |v_j| / sqrt(V |z_j|^2) once per column: lane i of a row
        // computes column 4 (i mod 4) + kq, and lane t of the row hands
        // column 4 t + kq to the others
        const int tm = i & 3;
        const double nzm = tm == 0 ? nzt[0] : (tm == 1 ? nzt[1] : (tm == 2 ? nzt[2] : nzt[3]));
        const double sm = fabs(vbuf[4 * tm + kq]) * rsqrt_f64(V * nzm);
        const double sj[4] = {dpp_f64<kDppRowNewBcast0 + 0>(sm), dpp_f64<kDppRowNewBcast0 + 1>(sm),
                              dpp_f64<kDppRowNewBcast0 + 2>(sm), dpp_f64<kDppRowNewBcast0 + 3>(sm)};
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            zr[t] *= sj[t];
            zi[t] *= sj[t];
        }
        if constexpr (F32) {
            // the same products in FP32; result register e of lane l is row
            // 4 (l/16) + e, column l%16
            typedef float float4_t __attribute__((ext_vector_type(4)));
            float4_t g = {0.0f, 0.0f, 0.0f, 0.0f}, x = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const float ar = static_cast<float>(zr[t]), ai = static_cast<float>(zi[t]);
                const float ap = ar + ai;
                g = __builtin_amdgcn_mfma_f32_16x16x4f32(ap, ap, g, 0, 0, 0);
                x = __builtin_amdgcn_mfma_f32_16x16x4f32(ai, ar, x, 0, 0, 0);
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) rhoP[(4 * kq + e) * 16 + i] = static_cast<double>(x[e]);
            team_sync<G>();
            double xt[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) xt[e] = rhoP[i * 16 + 4 * kq + e];
            team_sync<G>();
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int row = 4 * kq + e, col = i;
                const double xe = static_cast<double>(x[e]);
                rhoP[row * 16 + col] = row <= col ? (static_cast<double>(g[e]) - xe) - xt[e] : xt[e] - xe;
            }
            if constexpr (RP) {   // this lane's packed slots, written by other lanes
                team_sync<G>();
#pragma unroll
                for (int e = 0; e < 4; ++e) rp[e] = rhoP[packed_slot<Q, G>(lane, e)];
            }
            return;
        }
        typedef double double4_t __attribute__((ext_vector_type(4)));
        // Im rho = Zi Zr^T - Zr Zi^T = X - X^T with X = Zi Zr^T: four products
        // for X and a transpose through LDS instead of eight for Im rho.  Re
        // rho from the same X: Zp Zp^T = Re + X + X^T, so
        // four products for Zp Zp^T (Zp = Zr + Zi) instead of eight for
        // Zr Zr^T + Zi Zi^T
        double4_t g = {0.0, 0.0, 0.0, 0.0}, x = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const double zp = zr[t] + zi[t];
            g = __builtin_amdgcn_mfma_f64_16x16x4f64(zp, zp, g, 0, 0, 0);
            x = __builtin_amdgcn_mfma_f64_16x16x4f64(zi[t], zr[t], x, 0, 0, 0);
        }
        // result register e of lane l: row l/16 + 4e, column l%16
#pragma unroll
        for (int e = 0; e < 4; ++e) rhoP[(kq + 4 * e) * 16 + i] = x[e];
        team_sync<G>();
        double xt[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) xt[e] = rhoP[i * 16 + kq + 4 * e];   // X at (column, row)
        team_sync<G>();
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int row = kq + 4 * e, col = i;
            // P[a][b] = Im rho_ba = X_ba - X_ab below the diagonal
            const double v = row <= col ? (g[e] - x[e]) - xt[e] : xt[e] - x[e];
            rp[e] = v;
            rhoP[row * 16 + col] = v;
        }
    } else {
        stage_weights<Q, G>(ybuf, vbuf, wt, lane);
        team_sync<G>();
#pragma unroll 1
        for (int e = 0; e < S::NPL; ++e) {
            const int p = lane + G * e;
            double acc = 0.0;
            if (p < D2) {
                const int a = p / D, b = p % D;
                const int r = a <= b ? a : b;   // row of the upper-triangle element
                const int c = a <= b ? b : a;
                const bool want_re = a <= b;
#pragma unroll 4
                for (int j = 0; j < D; ++j) {
                    const double zr_r = ybuf[j * D + r], zi_r = ybuf[D2 + j * D + r];
                    const double zr_c = ybuf[j * D + c], zi_c = ybuf[D2 + j * D + c];
                    // z_r conj(z_c): real part and imaginary part
                    const double re = zr_r * zr_c + zi_r * zi_c;
                    const double im = zi_r * zr_c - zr_r * zi_c;
                    acc += wt[j] * (want_re ? re : im);
                }
                rhoP[p] = acc;
            }
            rp[e] = acc;
        }
    }
}

// The same without the register copy: packed rho' stays in rhoP only, where
// each lane finds its own slots p = packed_slot(lane, e) again.
template <int Q, int G, bool F32 = false>
__device__ __forceinline__ void stage_rho(const double* ybuf, const double* vbuf, double* wt, double* rhoP, int lane)
{
    double unused[TeamShape<Q, G>::NPL];
    stage_rho<Q, G, F32, false>(ybuf, vbuf, wt, rhoP, unused, lane);
}

// ---------------------------------------------------------------------------
// Algorithm 1 (the Bures draw): rho(x) = W W^dag / Tr(W W^dag), W = (U + I) G
// ---------------------------------------------------------------------------
// Sum over lanes xor M, 2M, ... below G (the lanes of one matrix column);
// every lane of the group gets the same bits.
template <int M, int G>
__device__ __forceinline__ double column_sum(double v)
{
    if constexpr (M < G) {
        v += xor_lane<M>(v);
        return column_sum<2 * M, G>(v);
    } else {
        return v;
    }
}

// U = Q Lambda of H = QR with Lambda = diag(r_kk / |r_kk|), i.e. the unitary
// factor whose triangular factor has a positive real diagonal: the one that
// Gram-Schmidt orthonormalisation of H's columns produces, whatever sign
// convention a Householder QR would take.  Modified Gram-Schmidt across the
// team: lane NG j + g holds rows g + NG r (NG = G / D) of column j, so a
// column's lanes are neighbours and its sums are quad exchanges; column k is
// normalised by its own lanes and broadcast through LDS (two alternating
// buffers of 2D doubles in ubuf), then every later column loses its
// component along it.  On return the lane holds U's entries of its rows.
template <int Q, int G>
struct BuresLayout {
    static constexpr int D = 1 << Q, NG = G / D, RPL = (D + NG - 1) / NG;
};

template <int Q, int G>
__device__ __forceinline__ void bures_unitary(const double* hbuf, double* ubuf, double (&ar)[BuresLayout<Q, G>::RPL],
                                              double (&ai)[BuresLayout<Q, G>::RPL], int lane)
{
    using BL = BuresLayout<Q, G>;
    constexpr int D = BL::D, D2 = D * D, NG = BL::NG, RPL = BL::RPL;
    const int j = lane / NG, g = lane % NG;
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
        const int i = g + NG * r;
        ar[r] = i < D ? hbuf[j * D + i] : 0.0;
        ai[r] = i < D ? hbuf[D2 + j * D + i] : 0.0;
    }
#pragma unroll 1
    for (int k = 0; k < D; ++k) {
        double* ub = ubuf + (k & 1) * 2 * D;
        // every lane takes part in the column sums (lane exchanges run with
        // the whole wavefront active); only column k's lanes use this one
        double n2 = 0.0;
#pragma unroll
        for (int r = 0; r < RPL; ++r) n2 += ar[r] * ar[r] + ai[r] * ai[r];
        n2 = column_sum<1, NG>(n2);
        if (j == k) {
            const double inv = 1.0 / sqrt(n2);
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
                const int i = g + NG * r;
                ar[r] *= inv;
                ai[r] *= inv;
                if (i < D) {
                    ub[i] = ar[r];
                    ub[D + i] = ai[r];
                }
            }
        }
        team_sync<G>();   // with two buffers, one wait per column suffices
        // c = u_k^dag a_j, then a_j -= c u_k for the columns j > k
        double ur[RPL], ui[RPL];
        double cr = 0.0, ci = 0.0;
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            const int i = g + NG * r;
            ur[r] = i < D ? ub[i] : 0.0;
            ui[r] = i < D ? ub[D + i] : 0.0;
            cr = __builtin_fma(ur[r], ar[r], __builtin_fma(ui[r], ai[r], cr));
            ci = __builtin_fma(ur[r], ai[r], __builtin_fma(-ui[r], ar[r], ci));
        }
        cr = column_sum<1, NG>(cr);
        ci = column_sum<1, NG>(ci);
        if (j > k) {
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
                ar[r] -= cr * ur[r] - ci * ui[r];
                ai[r] -= cr * ui[r] + ci * ur[r];
            }
        }
    }
}

// rho(x) of Algorithm 1 into rhoP (packed).  ws: the team's 2 D^2 doubles of
// workspace (the Pauli and rho' regions, which the later stages overwrite);
// matrices in ws are stored column by column, entry (a, b) at b D + a (real
// parts) and D^2 + b D + a (imaginary parts), the layout of x.
template <int Q, int G>
__device__ __forceinline__ void stage_rho_bures(const double* ybuf, double* ws, double* rhoP, double* misc, int lane)
{
    using BL = BuresLayout<Q, G>;
    using S = TeamShape<Q, G>;
    constexpr int D = BL::D, D2 = D * D, NG = BL::NG, RPL = BL::RPL;
    const double* gbuf = ybuf;            // G: x[0 : 2D^2]
    const double* hbuf = ybuf + 2 * D2;   // H: x[2D^2 : 4D^2]
    double ar[RPL], ai[RPL];
    bures_unitary<Q, G>(hbuf, ws, ar, ai, lane);
    team_sync<G>();
    {
        const int j = lane / NG, g = lane % NG;
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            const int i = g + NG * r;
            if (i < D) {
                ws[j * D + i] = ar[r] + (i == j ? 1.0 : 0.0);   // U + I
                ws[D2 + j * D + i] = ai[r];
            }
        }
    }
    team_sync<G>();
    double tpart = 0.0;
    if constexpr (Q == 4 && G == 64) {
        // W = (U + I) G on MFMA: Re W = Ar Gr - Ai Gi, Im W = Ar Gi + Ai Gr with
        // K = 16 in four k-steps; operand lane l carries A[l % 16][4 ks + l / 16]
        // and B[4 ks + l / 16][l % 16]; result register e of lane l is entry
        // (l / 16 + 4 e, l % 16).
        typedef double double4_t __attribute__((ext_vector_type(4)));
        const int i = lane & 15, kq = lane >> 4;
        double4_t wr = {0.0, 0.0, 0.0, 0.0}, wi = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const int kk = 4 * ks + kq;
            const double a_r = ws[kk * D + i], a_i = ws[D2 + kk * D + i];
            const double b_r = gbuf[i * D + kk], b_i = gbuf[D2 + i * D + kk];
            wr = __builtin_amdgcn_mfma_f64_16x16x4f64(a_r, b_r, wr, 0, 0, 0);
            wr = __builtin_amdgcn_mfma_f64_16x16x4f64(-a_i, b_i, wr, 0, 0, 0);
            wi = __builtin_amdgcn_mfma_f64_16x16x4f64(a_r, b_i, wi, 0, 0, 0);
            wi = __builtin_amdgcn_mfma_f64_16x16x4f64(a_i, b_r, wi, 0, 0, 0);
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) tpart = __builtin_fma(wr[e], wr[e], __builtin_fma(wi[e], wi[e], tpart));
        team_sync<G>();
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int a = kq + 4 * e, b = i;
            ws[b * D + a] = wr[e];
            ws[D2 + b * D + a] = wi[e];
        }
    } else {
        constexpr int NW = (D2 + G - 1) / G;
        double wr[NW], wi[NW];
#pragma unroll
        for (int e = 0; e < NW; ++e) {
            const int p = lane + G * e;
            const int a = p % D, b = p / D;
            double sr = 0.0, si = 0.0;
            if (p < D2) {
#pragma unroll 4
                for (int m = 0; m < D; ++m) {
                    const double u_r = ws[m * D + a], u_i = ws[D2 + m * D + a];
                    const double g_r = gbuf[b * D + m], g_i = gbuf[D2 + b * D + m];
                    sr = __builtin_fma(u_r, g_r, __builtin_fma(-u_i, g_i, sr));
                    si = __builtin_fma(u_r, g_i, __builtin_fma(u_i, g_r, si));
                }
            }
            wr[e] = sr;
            wi[e] = si;
            tpart = __builtin_fma(sr, sr, __builtin_fma(si, si, tpart));
        }
        team_sync<G>();
#pragma unroll
        for (int e = 0; e < NW; ++e) {
            const int p = lane + G * e;
            if (p < D2) {
                ws[(p / D) * D + p % D] = wr[e];
                ws[D2 + (p / D) * D + p % D] = wi[e];
            }
        }
    }
    const double inv_t = 1.0 / team_sum<G>(tpart, misc + 4, lane);   // 1 / Tr(W W^dag)
    team_sync<G>();
    // packed rho = Gram product of W's columns, scaled; the operands are read
    // before any result is written, since rhoP lies inside ws
    if constexpr (RhoLayout<Q, G>::kMfma) {
        typedef double double4_t __attribute__((ext_vector_type(4)));
        const int i = lane & 15, kq = lane >> 4;
        double zr[4], zi[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int j = 4 * t + kq;
            zr[t] = ws[j * D + i];
            zi[t] = ws[D2 + j * D + i];
        }
        double4_t re = {0.0, 0.0, 0.0, 0.0}, im = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            re = __builtin_amdgcn_mfma_f64_16x16x4f64(zr[t], zr[t], re, 0, 0, 0);
            re = __builtin_amdgcn_mfma_f64_16x16x4f64(zi[t], zi[t], re, 0, 0, 0);
            im = __builtin_amdgcn_mfma_f64_16x16x4f64(zi[t], zr[t], im, 0, 0, 0);
            im = __builtin_amdgcn_mfma_f64_16x16x4f64(-zr[t], zi[t], im, 0, 0, 0);
        }
        team_sync<G>();
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int row = kq + 4 * e, col = i;
            rhoP[row * 16 + col] = (row <= col ? re[e] : -im[e]) * inv_t;
        }
    } else {
        double acc[S::NPL];
#pragma unroll
        for (int e = 0; e < S::NPL; ++e) {
            const int p = lane + G * e;
            acc[e] = 0.0;
            if (p < D2) {
                const int a = p / D, b = p % D;
                const int r = a <= b ? a : b, c = a <= b ? b : a;
                const bool want_re = a <= b;
#pragma unroll 4
                for (int j = 0; j < D; ++j) {
                    const double zr_r = ws[j * D + r], zi_r = ws[D2 + j * D + r];
                    const double zr_c = ws[j * D + c], zi_c = ws[D2 + j * D + c];
                    acc[e] += want_re ? zr_r * zr_c + zi_r * zi_c : zi_r * zr_c - zr_r * zi_c;
                }
            }
        }
        team_sync<G>();
#pragma unroll
        for (int e = 0; e < S::NPL; ++e) {
            const int p = lane + G * e;
            if (p < D2) rhoP[p] = acc[e] * inv_t;
        }
    }
}

// Pauli coefficients c_mu = Tr(rho sigma_mu), mu = sum_q mu_q 4^(Q-1-q) with
// mu_q in {I=0, X=1, Y=2, Z=3}.  sigma_mu has one non-zero per row:
// (sigma_mu)_{a^m, a} = i^nY (-1)^popcount(a & zy), with m marking the X/Y
// qubits, zy the Z/Y qubits and nY = popcount(m & zy).  For one flip mask m,
// the coefficients of all 2^Q masks zy are therefore a Walsh-Hadamard
// transform over a of the generalised diagonal v_m[a] = rho_{a, a^m}:
// c = Re(i^nY W_m[zy]).  Lanes hold (m, a), butterflies run across the D-lane
// group, and lane position a ends holding zy = a.
__device__ __forceinline__ int spread_bits(int x)   // bit q -> bit 2q (x < 256)
{
    x = (x | (x << 4)) & 0x0F0F;
    x = (x | (x << 2)) & 0x3333;
    x = (x | (x << 1)) & 0x5555;
    return x;
}

template <int Q>
__device__ __forceinline__ double xor_lane_stage(double v, int s)
{
    switch (s) {
        case 0: return xor_lane<1>(v);
        case 1: return xor_lane<2>(v);
        case 2: return xor_lane<4>(v);
        case 3: return xor_lane<8>(v);
        case 4: return xor_lane<16>(v);
        default: return xor_lane<32>(v);
    }
}

__device__ __forceinline__ float xor_lane_stage_f32(float v, int s)
{
    switch (s) {
        case 0: return xor_lane_f32<1>(v);
        case 1: return xor_lane_f32<2>(v);
        case 2: return xor_lane_f32<4>(v);
        case 3: return xor_lane_f32<8>(v);
        case 4: return xor_lane_f32<16>(v);
        default: return xor_lane_f32<32>(v);
    }
}

// In-register butterflies over the V values of a lane (position bits
// log2 L and log2 L + 1): lower output a + b, upper a - b.
template <int V, typename T>
__device__ __forceinline__ void wht_in_lane(T (&v)[V])
{
    if constexpr (V >= 2) {
#pragma unroll
        for (int j = 0; j < V; j += 2) {
            const T a = v[j], b = v[j + 1];
            v[j] = a + b;
            v[j + 1] = a - b;
        }
    }
    if constexpr (V == 4) {
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const T a = v[j], b = v[j + 2];
            v[j] = a + b;
            v[j + 2] = a - b;
        }
    }
}

// Work split of the Pauli-coefficient transforms: a lane holds V positions
// a = al + L j (j < V, L = D / V) of generalised diagonal m (task u = m L +
// al), V at most D^2 / G so that the tasks still fill the team; the top
// log2 V butterfly stages are then register adds.  V = 2 up to 4 qubits
// (four positions, with re and im of each in registers, ran slower there)
// and 4 from 5 qubits on.
template <int Q, int G>
struct PauliSplit {
    static constexpr int D = 1 << Q, D2 = D * D;
    static constexpr int kFill = D2 / G;
    static constexpr int V = (Q >= 5 && kFill >= 4) ? 4 : (kFill >= 2 ? 2 : 1);
    static constexpr int L = D / V;
    static constexpr int kLogL = L == 1 ? 0 : L == 2 ? 1 : L == 4 ? 2 : L == 8 ? 3 : L == 16 ? 4 : 5;
    static constexpr int kTasks = D * L;
    static constexpr int kPasses = (kTasks + G - 1) / G;
    static_assert(G % L == 0 || L % G == 0, "transform groups tile the team");
};

// The Pauli coefficients of packed rho' (Re rho_ab at (a, b) for a <= b,
// Im rho_ba at (a, b) for a > b): for each generalised diagonal m, the
// D-point Walsh-Hadamard transform of rho_{a, a^m} over a gives, at output z,
// Tr(rho Z^z X^m) up to the phase i^{popcount(m & z)}.
template <int Q, int G, typename T>
__device__ __forceinline__ void stage_pauli_t(const double* rhoP, T* pauli, int lane)
{
    using PS = PauliSplit<Q, G>;
    constexpr int D = PS::D, V = PS::V, L = PS::L;
    const int al = lane & (L - 1);
#pragma unroll 1
    for (int e = 0; e < PS::kPasses; ++e) {
        const int u = lane + G * e;          // u = m L + al
        const bool valid = (PS::kPasses * G == PS::kTasks) || u < PS::kTasks;
        const int m = valid ? (u / L) : 0;
        T re[V], im[V];
#pragma unroll
        for (int j = 0; j < V; ++j) {
            const int a = al + L * j;
            const int b = a ^ m;
            const int lo = a < b ? a : b, hi = a < b ? b : a;
            re[j] = static_cast<T>(rhoP[lo * D + hi]);
            const T pim = static_cast<T>(rhoP[hi * D + lo]);   // Im of the upper element (a != b)
            im[j] = (a == b) ? T(0) : (a < b ? pim : -pim);
        }
#pragma unroll
        for (int s = 0; s < PS::kLogL; ++s) {
            // upper butterfly output other - own, lower own + other
            const uint32_t sg = ((al >> s) & 1u) << 31;
#pragma unroll
            for (int j = 0; j < V; ++j) {
                T ore, oim;
                if constexpr (sizeof(T) == 8) {
                    ore = xor_lane_stage<Q>(re[j], s);
                    oim = xor_lane_stage<Q>(im[j], s);
                } else {
                    ore = xor_lane_stage_f32(re[j], s);
                    oim = xor_lane_stage_f32(im[j], s);
                }
                re[j] = flip_sign(re[j], sg) + ore;
                im[j] = flip_sign(im[j], sg) + oim;
            }
        }
        wht_in_lane<V>(re);
        wht_in_lane<V>(im);
#pragma unroll
        for (int j = 0; j < V; ++j) {
            const int zy = al + L * j;
            const int r4 = __popc(m & zy) & 3;
            const T c = r4 == 0 ? re[j] : (r4 == 1 ? -im[j] : (r4 == 2 ? -re[j] : im[j]));
            // digit (m_q, zy_q): (0,0) -> I, (1,0) -> X, (1,1) -> Y, (0,1) -> Z
            const int mu = (spread_bits(zy) << 1) | spread_bits(m ^ zy);
            if (valid) pauli[mu] = c;
        }
    }
}

template <int Q, int G>
__device__ __forceinline__ void stage_pauli(const double* rhoP, double* pauli, int lane)
{
    stage_pauli_t<Q, G, double>(rhoP, pauli, lane);
}

// The same Pauli coefficients with the transform in FP32 (the mixed-precision
// Kronecker form): rho' is rounded to FP32 as it is read.
template <int Q, int G>
__device__ __forceinline__ void stage_pauli_f32(const double* rhoP, float* pauli, int lane)
{
    stage_pauli_t<Q, G, float>(rhoP, pauli, lane);
}

// Work split of the per-setting transforms.  A lane holds V = min(4, D)
// positions t = tl + L j (j < V) of one setting, L = D / V lanes per
// setting, so the top log2 V butterfly stages are register adds and only the
// lower ones cross lanes.  Task u = k L + tl covers setting k; the counts and
// Pauli indices are also stored task-major (ndv, muv: entry u V + j is
// position tl + L j of setting k), so a lane loads its V entries at once.
// Settings left over after the passes in which every lane is busy run in the
// one-value layout (D lanes per setting, entries nd / mu in natural order)
// when they fit one pass of it, else as a last partial pass of tasks.
template <int Q, int G>
struct LikSplit {
    static constexpr int D = 1 << Q, K = pow3(Q), KD = K * D;
    static constexpr int V = D < 4 ? D : 4;
    static constexpr int L = D / V;
    static constexpr int kLogL = L == 1 ? 0 : L == 2 ? 1 : L == 4 ? 2 : L == 8 ? 3 : 4;
    static constexpr int kTasks = K * L;
    static constexpr int kWhole = kTasks / G;
    static constexpr int kRemSettings = (kTasks - kWhole * G) / L;
    static constexpr bool kRemFlat = kRemSettings > 0 && kRemSettings * D <= G;
    static constexpr int kPasses = kWhole + (kRemSettings > 0 && !kRemFlat ? 1 : 0);
    static constexpr int kFlat0 = kWhole * (G / L);   // first setting of the one-value pass
    static_assert(G % L == 0, "a team holds whole settings");
};

// Probabilities of every projector by a 2^Q-point Walsh-Hadamard transform
// per setting, and this lane's share of sum c log p, kept as
// (sum c e, sum c frac) with log p = e ln2 + frac.
template <int Q, int G>
__device__ __forceinline__ void stage_loglik(const double* pauli, const double* __restrict__ nd,
                                             const uint16_t* __restrict__ mug, const double* __restrict__ ndv,
                                             const uint16_t* __restrict__ muv, const double* tables, int lane,
                                             double& part_e, double& part_f, int& bad)
{
    using LS = LikSplit<Q, G>;
    constexpr int D = LS::D, V = LS::V, L = LS::L;
    const LogEntry* tab = reinterpret_cast<const LogEntry*>(tables);
    // log p with p = val 2^-Q: the table logarithm of val, its exponent less Q
    auto term = [&](double val, double n) {
        const bool pos = val > 0.0;
        bad |= (n > 0.0 && !pos) ? 1 : 0;
        int ex;
        const double fr = log_parts(pos ? val : 1.0, tab, ex);
        part_e = __builtin_fma(n, static_cast<double>(ex - Q), part_e);
        part_f = __builtin_fma(n, fr, part_f);
    };
    const int tl = lane & (L - 1);
    if constexpr (LS::kPasses > 0) {
        // indices of the next task loaded one pass ahead (clamped into range)
        uint16_t mu_next[V];
        {
            const int u = lane < LS::kTasks ? lane : 0;
#pragma unroll
            for (int j = 0; j < V; ++j) mu_next[j] = muv[u * V + j];
        }
#pragma unroll 1
        for (int e = 0; e < LS::kPasses; ++e) {
            const int u = lane + G * e;
            const bool valid = LS::kPasses * G <= LS::kTasks || u < LS::kTasks;
            const int uc = valid ? u : 0;
            double n[V];
#pragma unroll
            for (int j = 0; j < V; ++j) n[j] = ndv[uc * V + j];
            double v[V];
#pragma unroll
            for (int j = 0; j < V; ++j) v[j] = pauli[mu_next[j]];
            if (e + 1 < LS::kPasses) {
                const int un = u + G < LS::kTasks ? u + G : 0;
#pragma unroll
                for (int j = 0; j < V; ++j) mu_next[j] = muv[un * V + j];
            }
#pragma unroll
            for (int s = 0; s < LS::kLogL; ++s) {
#pragma unroll
                for (int j = 0; j < V; ++j) {
                    const double other = xor_lane_stage<Q>(v[j], s);
                    v[j] = flip_sign(v[j], ((tl >> s) & 1u) << 31) + other;
                }
            }
            wht_in_lane<V>(v);
#pragma unroll
            for (int j = 0; j < V; ++j) term(v[j], valid ? n[j] : 0.0);
        }
    }
    if constexpr (LS::kRemFlat) {
        const int i = lane & (D - 1);
        const bool valid = lane < (LS::K - LS::kFlat0) * D;
        const int f = valid ? LS::kFlat0 * D + lane : 0;
        const double n = nd[f];
        double val = pauli[mug[f]];
#pragma unroll
        for (int s = 0; s < Q; ++s) {
            const double other = xor_lane_stage<Q>(val, s);
            val = flip_sign(val, ((i >> s) & 1u) << 31) + other;
        }
        term(val, valid ? n : 0.0);
    }
}

// The mixed-precision Kronecker form of stage_loglik: the transform and
// log2 p (hardware logarithm) in FP32, the count-weighted sum of log2 p in
// FP64.  A probability that rounds below the smallest normal FP32 value is
// taken at that value.
template <int Q, int G>
__device__ __forceinline__ void stage_loglik_f32(const float* pauli, const double* __restrict__ nd,
                                                 const uint16_t* __restrict__ mug, const double* __restrict__ ndv,
                                                 const uint16_t* __restrict__ muv, int lane, double& part)
{
    using LS = LikSplit<Q, G>;
    constexpr int D = LS::D, V = LS::V, L = LS::L;
    auto term = [&](float val, double n) {
        const float p = fmaxf(val * (1.0f / D), 0x1.0p-126f);
        part = __builtin_fma(n, static_cast<double>(__builtin_amdgcn_logf(p)), part);
    };
    const int tl = lane & (L - 1);
    if constexpr (LS::kPasses > 0) {
        uint16_t mu_next[V];
        {
            const int u = lane < LS::kTasks ? lane : 0;
#pragma unroll
            for (int j = 0; j < V; ++j) mu_next[j] = muv[u * V + j];
        }
#pragma unroll 1
        for (int e = 0; e < LS::kPasses; ++e) {
            const int u = lane + G * e;
            const bool valid = LS::kPasses * G <= LS::kTasks || u < LS::kTasks;
            const int uc = valid ? u : 0;
            double n[V];
#pragma unroll
            for (int j = 0; j < V; ++j) n[j] = ndv[uc * V + j];
            float v[V];
#pragma unroll
            for (int j = 0; j < V; ++j) v[j] = pauli[mu_next[j]];
            if (e + 1 < LS::kPasses) {
                const int un = u + G < LS::kTasks ? u + G : 0;
#pragma unroll
                for (int j = 0; j < V; ++j) mu_next[j] = muv[un * V + j];
            }
#pragma unroll
            for (int s = 0; s < LS::kLogL; ++s) {
#pragma unroll
                for (int j = 0; j < V; ++j) {
                    const float other = xor_lane_stage_f32(v[j], s);
                    v[j] = flip_sign(v[j], ((tl >> s) & 1u) << 31) + other;
                }
            }
            wht_in_lane<V>(v);
#pragma unroll
            for (int j = 0; j < V; ++j) term(v[j], valid ? n[j] : 0.0);
        }
    }
    if constexpr (LS::kRemFlat) {
        const int i = lane & (D - 1);
        const bool valid = lane < (LS::K - LS::kFlat0) * D;
        const int f = valid ? LS::kFlat0 * D + lane : 0;
        const double n = nd[f];
        float val = pauli[mug[f]];
#pragma unroll
        for (int s = 0; s < Q; ++s) {
            const float other = xor_lane_stage_f32(val, s);
            val = flip_sign(val, ((i >> s) & 1u) << 31) + other;
        }
        term(val, valid ? n : 0.0);
    }
}

// ---------------------------------------------------------------------------
// dense contraction on MFMA: p = M vec(rho) for the 16 chains of a workgroup
// ---------------------------------------------------------------------------
// M (KD x D^2, exact entries 0 or +-2^-a in every precision) is stored in the
// order the MFMA A operand is consumed: for output tile nt and k-step ks,
// 64 lanes' fragments back to back (FP64/FP32: lane l holds M[16 nt + l%16]
// [4 ks + l/16]; BF16: lane l holds M[16 nt + l%16][32 ks + 8 (l/16) + v],
// v = 0..7).  The B operand is packed rho of chain l%16 at the same k, read
// from that chain's team region in LDS.  Results: FP64 lane l register r is
// row l/16 + 4r; FP32/BF16 lane l register r is row 4 (l/16) + r; the column
// is the chain l % 16 in both.
typedef double dense_f64x4 __attribute__((ext_vector_type(4)));
typedef float dense_f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 dense_bf16x8 __attribute__((ext_vector_type(8)));

// Reduced-precision B operands: the FP32 rounding of packed rho, or its
// three-part BF16 split x = hi + mid + lo (each part the BF16 rounding of
// what the previous parts leave), written into the team's staging region.
template <int Q, int G, int PREC>
__device__ __forceinline__ void stage_dense_operands(const double* rhoP, double* stage, int lane)
{
    using DS = DenseShape<Q>;
    if constexpr (PREC == kPrecF32) {
        float* f = reinterpret_cast<float*>(stage);
        for (int k = lane; k < DS::K; k += G) f[k] = static_cast<float>(rhoP[k]);
    } else if constexpr (PREC == kPrecBF16x3) {
        __bf16* h = reinterpret_cast<__bf16*>(stage);
        for (int k = lane; k < DS::KP32; k += G) {
            const double x = k < DS::K ? rhoP[k] : 0.0;
            const __bf16 hi = static_cast<__bf16>(static_cast<float>(x));
            const double r1 = x - static_cast<double>(static_cast<float>(hi));
            const __bf16 mid = static_cast<__bf16>(static_cast<float>(r1));
            const double r2 = r1 - static_cast<double>(static_cast<float>(mid));
            const __bf16 lo = static_cast<__bf16>(static_cast<float>(r2));
            h[k] = hi;
            h[DS::KP32 + k] = mid;
            h[2 * DS::KP32 + k] = lo;
        }
    }
}

// Partial sums of c log p for the 16 chains of the workgroup; the calling
// thread's wave covers output tiles wave, wave + nwaves, ...  Each lane keeps
// the sums of its column chain (l % 16).
template <int Q, int PREC, int NWAVES, int TEAM_LDS>
__device__ __forceinline__ void dense_partials(const double* lds_teams, int off_rho, int off_stage,
                                               const void* __restrict__ mfrag, const double* __restrict__ nd,
                                               const LogEntry* logtab, int wave, int l, double& part_e,
                                               double& part_f, int& bad)
{
    using DS = DenseShape<Q>;
    const int col = l & 15, kq = l >> 4;
    const double* team_base = lds_teams + col * TEAM_LDS;
#pragma unroll 1
    for (int nt = wave; nt < DS::NT; nt += NWAVES) {
        double pr[4];
        float pr32[4];
        if constexpr (PREC == kPrecF64) {
            const double* A = static_cast<const double*>(mfrag) + static_cast<size_t>(nt) * DS::KS4 * 64;
            const double* B = team_base + off_rho;
            dense_f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
            for (int ks = 0; ks < DS::KS4; ++ks)
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(A[ks * 64 + l], B[4 * ks + kq], acc, 0, 0, 0);
#pragma unroll
            for (int r = 0; r < 4; ++r) pr[r] = acc[r];
        } else if constexpr (PREC == kPrecF32) {
            const float* A = static_cast<const float*>(mfrag) + static_cast<size_t>(nt) * DS::KS4 * 64;
            const float* B = reinterpret_cast<const float*>(team_base + off_stage);
            dense_f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll 4
            for (int ks = 0; ks < DS::KS4; ++ks)
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(A[ks * 64 + l], B[4 * ks + kq], acc, 0, 0, 0);
#pragma unroll
            for (int r = 0; r < 4; ++r) pr32[r] = acc[r];
        } else {
            const dense_bf16x8* A = static_cast<const dense_bf16x8*>(mfrag) + static_cast<size_t>(nt) * DS::KS32 * 64;
            const __bf16* B = reinterpret_cast<const __bf16*>(team_base + off_stage);
            dense_f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int ks = 0; ks < DS::KS32; ++ks) {
                const dense_bf16x8 a = A[ks * 64 + l];
                const int k0 = 32 * ks + 8 * kq;
#pragma unroll
                for (int part = 0; part < 3; ++part) {
                    const dense_bf16x8 b = *reinterpret_cast<const dense_bf16x8*>(B + part * DS::KP32 + k0);
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
                }
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) pr32[r] = acc[r];
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = PREC == kPrecF64 ? kq + 4 * r : 4 * kq + r;
            const int kl = 16 * nt + row;
            const double n = kl < DS::KD ? nd[kl] : 0.0;
            if constexpr (PREC == kPrecF64) {
                const double p = pr[r];
                const bool pos = p > 0.0;
                bad |= (n > 0.0 && !pos) ? 1 : 0;
                int ex;
                const double fr = log_parts(pos ? p : 1.0, logtab, ex);
                part_e = __builtin_fma(n, static_cast<double>(ex), part_e);
                part_f = __builtin_fma(n, fr, part_f);
            } else {
                // reduced precision: log2 p by the hardware FP32 logarithm of
                // the FP32 probability (one that rounds below the smallest
                // normal FP32 value taken at that value), summed in FP64 in
                // units of ln 2 beside the FP64 form's exponents
                const float p = fmaxf(pr32[r], 0x1.0p-126f);
                part_e = __builtin_fma(n, static_cast<double>(__builtin_amdgcn_logf(p)), part_e);
            }
        }
    }
    // fold the four row groups of each column (lanes l, l^16, l^32, l^48)
    part_e += __shfl_xor(part_e, 16, 64);
    part_f += __shfl_xor(part_f, 16, 64);
    bad |= __shfl_xor(bad, 16, 64);
    part_e += __shfl_xor(part_e, 32, 64);
    part_f += __shfl_xor(part_f, 32, 64);
    bad |= __shfl_xor(bad, 32, 64);
}

// log L of the 16 chains of a workgroup of 16 one-wave teams (G = 64);
// returns the calling team's value.  All threads of the workgroup call it.
template <int Q, int PREC>
__device__ __forceinline__ double dense_loglik_wg(double* lds_teams, double* red, const void* mfrag,
                                                  const double* nd, const LogEntry* logtab, int tid)
{
    using S = TeamShape<Q, 64, kPathDense>;
    constexpr int NW = 16;
    const int wave = tid >> 6, l = tid & 63;
    stage_dense_operands<Q, 64, PREC>(lds_teams + wave * S::kLds + S::kOffRho, lds_teams + wave * S::kLds + S::kOffPauli,
                                      l);
    __syncthreads();
    double pe = 0.0, pf = 0.0;
    int bad = 0;
    dense_partials<Q, PREC, NW, S::kLds>(lds_teams, S::kOffRho, S::kOffPauli, mfrag, nd, logtab, wave, l, pe, pf,
                                         bad);
    if (l < 16) {
        red[(wave * 16 + l) * 3 + 0] = pe;
        red[(wave * 16 + l) * 3 + 1] = pf;
        red[(wave * 16 + l) * 3 + 2] = static_cast<double>(bad);
    }
    __syncthreads();
    double te = 0.0, tf = 0.0;
    int tb = 0;
#pragma unroll 4
    for (int w = 0; w < NW; ++w) {
        te += red[(w * 16 + wave) * 3 + 0];
        tf += red[(w * 16 + wave) * 3 + 1];
        tb |= static_cast<int>(red[(w * 16 + wave) * 3 + 2]);
    }
    __syncthreads();
    return tb ? -INFINITY : __builtin_fma(te, kLn2, tf);
}

// ---------------------------------------------------------------------------
// the chain tile
// ---------------------------------------------------------------------------
template <int Q, int G, int WG, int PATH, int PREC, int PARAM = kParamGamma, bool RESTORE = false>
__device__ __forceinline__ void chain_tile(const ChainArgs& A, int64_t tile_chain0, double* tables, double* lds)
{
    using Dm = Dims<Q>;
    using S = TeamShape<Q, G, PATH, PARAM>;
    static_assert(PARAM != kParamBures || (PATH == kPathKron && Q <= 4 && G <= 64),
                  "Algorithm 1 runs on the Kronecker path with one-wavefront teams");
    static_assert(PATH == kPathKron ? (PREC == kPrecF64 || PREC == kPrecF32) : (G == 64 && WG == 1024),
                  "unsupported path");
    constexpr int D2 = Dm::D2, d = S::d, NB = S::NB;
    static_assert(WG % G == 0, "workgroup must hold whole teams");

    const int tid = threadIdx.x;
    const int team = tid / G;
    const int lane = tid % G;
    const int64_t chain = tile_chain0 + team;     // problem-wide index
    const bool live = chain < A.R;
    const int64_t c = live ? chain : A.R - 1;     // a valid row for the loads of idle teams

    const LogEntry* logtab = reinterpret_cast<const LogEntry*>(tables);
    double* base = lds + team * S::kLdsChain;
    double* ybuf = base;                 // proposal y' (x layout), kept until the decision
    double* pauli = base + S::kOffPauli;
    double* rhoP = base + S::kOffRho;
    double* wt = base + S::kOffWt;
    double* misc = base + S::kOffMisc;

    // registers: state entries i = lane + G e, packed-rho entries p = lane + G e
    double y[S::NYL];
    double rc[S::NPL], s1[S::NPL], s2[S::NPL];
    double ll, beta;
    int acc_w;
    int64_t nst, nacc = 0, nnear = 0;

    // Philox job `job` of step `step`: normal block b -> eta[4b..4b+3], job
    // NB -> the Metropolis-Hastings uniform (in v[0])
    auto job_values = [&](int job, uint64_t step, double v[4]) {
        const bool normal = job < NB;
        const uint64_t c0 = normal ? static_cast<uint64_t>(job) : 0;
        const uint64_t c3 = normal ? 0 : (static_cast<uint64_t>(kTagMH) << 56);
        const Block4 B = philox4x64_10(c0, step, static_cast<uint64_t>(c), c3, A.seed, 0);
        if (normal) {
            box_muller(B.w[0], B.w[1], v[0], v[1], logtab);
            box_muller(B.w[2], B.w[3], v[2], v[3], logtab);
        } else {
            v[0] = uniform_open(B.w[0]);
            v[1] = v[2] = v[3] = 0.0;
        }
    };
    // eta into ybuf, the uniform into misc[0]
    auto store_job = [&](int job, const double v[4]) {
        if (job < NB) {
            const int i = 4 * job;
            ybuf[i] = v[0];
            if (i + 1 < d) ybuf[i + 1] = v[1];
            if (i + 2 < d) ybuf[i + 2] = v[2];
            if (i + 3 < d) ybuf[i + 3] = v[3];
        } else {
            misc[0] = v[0];
        }
    };

    // every job of one step, directly
    auto draw_all = [&](uint64_t step) {
#pragma unroll 1
        for (int e = 0; e < S::NJL; ++e) {
            const int job = lane + G * e;
            if (job <= NB) {
                double v[4];
                job_values(job, step, v);
                store_job(job, v);
            }
        }
    };

    // One step of the loop.  Without a ring: draw_all.  With one: the whole
    // passes, then at k = 0 (the first step of a group of kRing) one pass
    // draws the tails of steps step .. step + kRing - 1 into the ring, and
    // every step copies its own tail (k = its position in the group) into
    // place.  Separate loops for the two cases: one loop with a ring pass
    // folded in spills more and runs slower.
    double* ring = base + S::kLds;
    auto draw = [&](uint64_t step, int k) {
        if constexpr (S::kRing == 1) {
            draw_all(step);
        } else {
#pragma unroll 1
            for (int e = 0; e < S::kFullJobs / G; ++e) {
                const int job = lane + G * e;
                double v[4];
                job_values(job, step, v);
                store_job(job, v);
            }
            if (k == 0) {
                if (lane < S::kTail * S::kRing) {
                    // ring[(k' kTail + r) 4 + m] = value m of tail job r of step + k'
                    double v[4];
                    job_values(S::kFullJobs + lane % S::kTail, step + static_cast<uint64_t>(lane / S::kTail), v);
                    double* dst = ring + 4 * lane;
                    dst[0] = v[0];
                    dst[1] = v[1];
                    dst[2] = v[2];
                    dst[3] = v[3];
                }
                team_sync<G>();
            }
            for (int m = lane; m < 4 * S::kTail; m += G) {   // 4 kTail can exceed a small team
                const double v = ring[4 * S::kTail * k + m];
                const int job = S::kFullJobs + m / 4;
                const int i = 4 * S::kFullJobs + m;
                if (job < NB) {
                    if (i < d) ybuf[i] = v;
                } else if ((m & 3) == 0) {
                    misc[0] = v;
                }
            }
        }
    };

    // log L at the parameters in ybuf (team-uniform result); leaves packed rho in rhoP
    // the dense contraction shares work across the workgroup's teams
    auto sync = [&]() {
        if constexpr (PATH == kPathDense) __syncthreads();
        else team_sync<G>();
    };

    auto evaluate = [&]() -> double {
        if constexpr (PARAM == kParamBures) {
            stage_rho_bures<Q, G>(ybuf, pauli, rhoP, misc, lane);
        } else if constexpr (PARAM == kParamDirichlet) {
            // v in the Pauli region; misc[0] holds the uniform, the sum uses misc[4..]
            stage_dirichlet_v<Q, G>(ybuf, pauli, A.alpha, A.lg_alpha, misc + 4, lane);
            stage_rho<Q, G, PATH == kPathKron && PREC == kPrecF32>(ybuf, pauli, wt, rhoP, lane);
        } else {
            stage_rho<Q, G, PATH == kPathKron && PREC == kPrecF32>(ybuf, ybuf + 2 * D2, wt, rhoP, lane);
        }
        sync();
        double llv;
        if constexpr (PATH == kPathDense) {
            llv = dense_loglik_wg<Q, PREC>(lds, tables + WgTables<Q, PATH>::kOffRed, A.mfrag, A.nd, logtab, tid);
        } else if constexpr (PREC == kPrecF32) {
            float* pauli32 = reinterpret_cast<float*>(pauli);
            stage_pauli_f32<Q, G>(rhoP, pauli32, lane);
            sync();
            double part = 0.0;
            stage_loglik_f32<Q, G>(pauli32, A.nd, A.mu, A.ndv, A.muv, lane, part);
            // Poisson counts: minus sum_m lambda_m p_m (FP64, from packed rho),
            // in the same team reduction
            if (A.poisson) part -= kInvLn2 * linear_share<Q, G>(A.nd + Dm::KD, rhoP, lane);
            llv = kLn2 * team_sum<G>(part, misc + 4, lane);
        } else {
            stage_pauli<Q, G>(rhoP, pauli, lane);
            sync();
            double part_e = 0.0, part_f = 0.0;
            int bad = 0;
            stage_loglik<Q, G>(pauli, A.nd, A.mu, A.ndv, A.muv, tables, lane, part_e, part_f, bad);
            if (A.poisson) part_f -= linear_share<Q, G>(A.nd + Dm::KD, rhoP, lane);   // as above
            llv = team_loglik<G>(part_e, part_f, bad, misc + 4, lane);
        }
        if constexpr (PATH == kPathDense) {
            if (A.poisson)   // Poisson counts: minus sum_m lambda_m p_m, in FP64 from packed rho
                llv -= team_sum<G>(linear_share<Q, G>(A.nd + Dm::KD, rhoP, lane), misc + 4, lane);
        }
        return llv;
    };

    if constexpr (RESTORE) {
        // a state set from outside (checkpoint, restart): log L and packed
        // rho of the stored y, with the team shape and code of the step
        // kernel, so they are the values a run would have carried; nothing
        // else is touched.  (A kernel of its own: the same branch inside the
        // step kernel cost it scalar-register spills in the step loop.)
        for (int i = lane; i < d; i += G) ybuf[i] = A.x[c * d + i];
        sync();
        const double llv = evaluate();
        if (live) {
            for (int p = lane; p < D2; p += G) A.rho_cur[c * D2 + p] = rhoP[p];
            if (lane == 0) A.ll[c] = llv;
        }
        return;
    }

    // ---- load or initialise the chain state ----
    if (A.init) {
        draw_all(0);                     // y^0 ~ N(0, I): Algorithm 2, first line
        __syncthreads();
        ll = evaluate();
#pragma unroll
        for (int e = 0; e < S::NYL; ++e) {
            const int i = lane + G * e;
            y[e] = i < d ? ybuf[i] : 0.0;
        }
#pragma unroll
        for (int e = 0; e < S::NPL; ++e) {
            const int p = packed_slot<Q, G>(lane, e);
            rc[e] = p < D2 ? rhoP[p] : 0.0;
            s1[e] = 0.0;
            s2[e] = 0.0;
        }
        beta = A.beta0;
        acc_w = 0;
        nst = 0;
        __syncthreads();
    } else {
#pragma unroll
        for (int e = 0; e < S::NYL; ++e) {
            const int i = lane + G * e;
            y[e] = i < d ? A.x[c * d + i] : 0.0;
        }
#pragma unroll
        for (int e = 0; e < S::NPL; ++e) {
            const int p = packed_slot<Q, G>(lane, e);
            const bool ok = p < D2;
            rc[e] = ok ? A.rho_cur[c * D2 + p] : 0.0;
            s1[e] = ok ? A.s1[c * D2 + p] : 0.0;
            s2[e] = ok ? A.s2[c * D2 + p] : 0.0;
        }
        ll = A.ll[c];
        beta = A.beta[c];
        acc_w = A.acc_win[c];
        nst = A.n_stored[c];
    }

    const int64_t n_rec = A.record_every > 0 ? A.n_steps / A.record_every : 0;

    // ---- Algorithm 2 ----
    int kr = 0;   // position of the step in its group of kRing steps
    double a = sqrt(1.0 - beta * beta);   // the pCN contraction, recomputed when beta changes
    // j mod M_A and j mod T, carried from step to step (no 64-bit remainder
    // in the loop)
    const int32_t ma = A.adapt_every > 0 ? A.adapt_every : 1;
    int32_t ja = static_cast<int32_t>((A.step_begin + 1) % ma);
    int32_t jt = static_cast<int32_t>((A.step_begin + 1) % A.thin);
    for (int64_t t = 0; t < A.n_steps; ++t) {
        const int64_t j = A.step_begin + 1 + t;
        draw(static_cast<uint64_t>(j), kr);
        kr = kr + 1 == S::kRing ? 0 : kr + 1;
        sync();
        // pCN proposal y' = sqrt(1 - beta^2) y + beta eta, in place over eta
#pragma unroll
        for (int e = 0; e < S::NYL; ++e) {
            const int i = lane + G * e;
            if (i < d) ybuf[i] = __builtin_fma(beta, ybuf[i], a * y[e]);
        }
        sync();
        const double llp = evaluate();
        if (A.pair_every > 0 && live && chain < A.pair_chains && (t + 1) % A.pair_every == 0) {
            const int64_t slot = (t + 1) / A.pair_every - 1;   // rows are slot-major: [slot][chain]
            const int64_t row = slot * A.pair_chains + chain;
            uint16_t* dst = A.pair_x + row * A.pair_width;
            for (int i = lane; i < A.pair_width; i += G) {
                const float v = i < d ? static_cast<float>(ybuf[i]) : 0.0f;
                dst[i] = __builtin_bit_cast(uint16_t, static_cast<__bf16>(v));
            }
            if (lane == 0) A.pair_ll[row] = llp;
        }
        const double logu = fast_log(misc[0], logtab);
        const double delta = llp - ll;
        const bool accept = logu < delta;
        nnear += fabs(logu - delta) < 1e-8 ? 1 : 0;
        if (accept) {
#pragma unroll
            for (int e = 0; e < S::NYL; ++e) {
                const int i = lane + G * e;
                if (i < d) y[e] = ybuf[i];
            }
#pragma unroll
            for (int e = 0; e < S::NPL; ++e) {
                const int p = packed_slot<Q, G>(lane, e);   // this lane's own writes in stage_rho
                rc[e] = p < D2 ? rhoP[p] : 0.0;
            }
            ll = llp;
            ++acc_w;
            ++nacc;
        }
        if (A.adapt_every > 0 && ja == 0) {
            if (A.adapt_until < 0 || j <= A.adapt_until) {
                const double rate = static_cast<double>(acc_w) / static_cast<double>(A.adapt_every);
                if (rate > A.adapt_hi) beta = fmin(beta * A.adapt_factor, 1.0);
                if (rate < A.adapt_lo) beta = beta / A.adapt_factor;
                a = sqrt(1.0 - beta * beta);
            }
            acc_w = 0;
        }
        if (j > A.burn_in && jt == 0) {
#pragma unroll
            for (int e = 0; e < S::NPL; ++e) {
                s1[e] += rc[e];
                s2[e] = __builtin_fma(rc[e], rc[e], s2[e]);
            }
            ++nst;
        }
        ja = ja + 1 == ma ? 0 : ja + 1;
        jt = jt + 1 == A.thin ? 0 : jt + 1;
        if (live && chain < A.trace_chains && lane == 0) {
            const int64_t o = chain * A.n_steps + t;
            if (A.tr_ll) A.tr_ll[o] = llp;
            if (A.tr_lu) A.tr_lu[o] = logu;
            if (A.tr_acc) A.tr_acc[o] = accept ? 1 : 0;
        }
        if (A.record_every > 0 && live && chain < A.record_chains && (t + 1) % A.record_every == 0) {
            const int64_t slot = (t + 1) / A.record_every - 1;
            double* dst = A.rec + (chain * n_rec + slot) * D2;
#pragma unroll
            for (int e = 0; e < S::NPL; ++e) {
                const int p = packed_slot<Q, G>(lane, e);
                if (p < D2) dst[p] = rc[e];
            }
        }
        sync();
    }

    // ---- write the state back ----
    if (live) {
#pragma unroll
        for (int e = 0; e < S::NYL; ++e) {
            const int i = lane + G * e;
            if (i < d) A.x[c * d + i] = y[e];
        }
#pragma unroll
        for (int e = 0; e < S::NPL; ++e) {
            const int p = packed_slot<Q, G>(lane, e);
            if (p < D2) {
                A.rho_cur[c * D2 + p] = rc[e];
                A.s1[c * D2 + p] = s1[e];
                A.s2[c * D2 + p] = s2[e];
            }
        }
        if (lane == 0) {
            A.ll[c] = ll;
            A.beta[c] = beta;
            A.acc_win[c] = acc_w;
            A.n_stored[c] = nst;
            A.n_acc[c] = nacc;
            A.n_near[c] = nnear;
        }
    }
}

// Waves per SIMD the register allocation aims at: the per-lane state
// (NYL + 4 NPL doubles) plus about 64 registers of temporaries, within the
// 512-register file of a SIMD lane, at most 4.
template <int Q, int G>
constexpr int chain_min_waves()
{
    using S = TeamShape<Q, G>;
    const int regs = 2 * (S::NYL + 4 * S::NPL) + 64;
    const int w = 512 / regs;
    return w < 1 ? 1 : (w > 4 ? 4 : w);
}

// The same capped by what the workgroup's LDS allows on a CU (160 KiB): a
// shape that fits fewer wavefronts per SIMD than its registers would allow
// gets the registers of the wavefronts that actually run (fewer spills).
template <int Q, int G, int WG, int PATH, int PARAM>
constexpr int chain_waves()
{
    using S = TeamShape<Q, G, PATH, PARAM>;
    constexpr long lds = (static_cast<long>(WG / G) * S::kLdsChain + WgTables<Q, PATH>::kDoubles) * 8;
    constexpr long wgs = (160L * 1024) / lds;
    constexpr int w_lds = static_cast<int>((wgs * (WG / 64) + 3) / 4);
    constexpr int w_reg = chain_min_waves<Q, G>();
    return w_lds < 1 ? 1 : (w_lds < w_reg ? w_lds : w_reg);
}

template <int Q, int G, int WG, int PATH = kPathKron, int PREC = kPrecF64, int PARAM = kParamGamma>
__global__ __launch_bounds__(WG, (chain_waves<Q, G, WG, PATH, PARAM>())) void k_chains(ChainArgs A, int64_t chain0)
{
    extern __shared__ double lds[];
    wg_tables_init<Q, PATH>(lds, threadIdx.x, WG);
    __syncthreads();
    chain_tile<Q, G, WG, PATH, PREC, PARAM>(A, chain0 + static_cast<int64_t>(blockIdx.x) * (WG / G), lds,
                                            lds + WgTables<Q, PATH>::kDoubles);
}

// log L and packed rho of restored states (qst_set_chain_state), written to
// ll and rho_cur; same template arguments as the step kernel they precede.
template <int Q, int G, int WG, int PATH = kPathKron, int PREC = kPrecF64, int PARAM = kParamGamma>
__global__ __launch_bounds__(WG, (chain_waves<Q, G, WG, PATH, PARAM>())) void k_chains_restore(ChainArgs A,
                                                                                     int64_t chain0)
{
    extern __shared__ double lds[];
    wg_tables_init<Q, PATH>(lds, threadIdx.x, WG);
    __syncthreads();
    chain_tile<Q, G, WG, PATH, PREC, PARAM, true>(A, chain0 + static_cast<int64_t>(blockIdx.x) * (WG / G), lds,
                                                  lds + WgTables<Q, PATH>::kDoubles);
}

// Eq. (likelihood) for n given density matrices (complex, interleaved,
// row-major), one team per matrix.
template <int Q, int G, int WG, int PREC = kPrecF64>
__global__ __launch_bounds__(WG) void k_loglik(const double* __restrict__ nd, const uint16_t* __restrict__ mug,
                                               const double* __restrict__ ndv, const uint16_t* __restrict__ muv,
                                               const double* rho, int64_t n, double* ll_out, int poisson)
{
    using Dm = Dims<Q>;
    using S = TeamShape<Q, G>;
    constexpr int D = Dm::D, D2 = Dm::D2;
    extern __shared__ double lds_all[];
    wg_tables_init<Q>(lds_all, threadIdx.x, WG);
    double* tables = lds_all;
    double* lds = lds_all + WgTables<Q>::kDoubles;
    const int tid = threadIdx.x, team = tid / G, lane = tid % G;
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * (WG / G) + team;
    const bool live = idx < n;
    const int64_t c = live ? idx : 0;
    double* base = lds + team * S::kLds;
    double* pauli = base + S::kOffPauli;
    double* rhoP = base + S::kOffRho;
    double* misc = base + S::kOffMisc;
    for (int p = lane; p < D2; p += G) {
        const int a = p / D, b = p % D;
        // packed: Re rho_ab above/on the diagonal, Im rho_ba below it
        rhoP[p] = a <= b ? rho[(c * D2 + a * D + b) * 2] : rho[(c * D2 + b * D + a) * 2 + 1];
    }
    __syncthreads();
    if constexpr (PREC == kPrecF32) {
        float* pauli32 = reinterpret_cast<float*>(pauli);
        stage_pauli_f32<Q, G>(rhoP, pauli32, lane);
        __syncthreads();
        double part = 0.0;
        stage_loglik_f32<Q, G>(pauli32, nd, mug, ndv, muv, lane, part);
        double ll = kLn2 * team_sum<G>(part, misc + 4, lane);
        if (poisson) ll -= team_sum<G>(linear_share<Q, G>(nd + Dm::KD, rhoP, lane), misc + 4, lane);
        if (live && lane == 0) ll_out[idx] = ll;
    } else {
        stage_pauli<Q, G>(rhoP, pauli, lane);
        __syncthreads();
        double part_e = 0.0, part_f = 0.0;
        int bad = 0;
        stage_loglik<Q, G>(pauli, nd, mug, ndv, muv, tables, lane, part_e, part_f, bad);
        double ll = team_loglik<G>(part_e, part_f, bad, misc + 4, lane);
        if (poisson) ll -= team_sum<G>(linear_share<Q, G>(nd + Dm::KD, rhoP, lane), misc + 4, lane);
        if (live && lane == 0) ll_out[idx] = ll;
    }
}

// ---------------------------------------------------------------------------
// Eq. (likelihood) for n given density matrices on the dense path, alone
// (qst_loglik), 1..5 qubits: 64 matrices per 1024-thread workgroup (48 for
// BF16x3; at 5 qubits 32 in FP32, 16 otherwise, what LDS holds), so
// that each fragment of M, streamed from L2, feeds four (three) MFMAs, one
// per 16-column block of matrices, instead of one.  Their B operands sit in
// LDS in the precision's format, one padded row per matrix; wave w computes
// the output tiles w, w + 16, ... of all the workgroup's matrices and keeps
// per-lane sums of c log p for its columns; the 16 waves' sums are added in
// wave order.  BF16x3 takes 48 matrices so that its three-part operands
// (76 KB) leave room for a second workgroup per CU, whose HBM reads of rho
// then overlap the first one's MFMAs.
// ---------------------------------------------------------------------------
template <int Q, int PREC>
struct DenseAloneShape {
    using DS = DenseShape<Q>;
    // matrices per workgroup: as many 16-column blocks as the operands of all
    // D^2 values of k leave room for in LDS (5 qubits: 1024 values per matrix)
    static constexpr int kStates = Q <= 4 ? (PREC == kPrecBF16x3 ? 48 : 64) : (PREC == kPrecF32 ? 32 : 16);
    static constexpr int kBlocks = kStates / 16;       // 16-column MFMA blocks
    // B row stride in elements of the operand type, padded against LDS bank
    // conflicts between the 16 rows one MFMA reads
    static constexpr int kStrideF64 = DS::K + 1;       // doubles
    static constexpr int kStrideF32 = DS::K + 1;       // floats
    static constexpr int kStrideBF16 = 3 * DS::KP32 + 8;   // bf16: hi | mid | lo parts
    static constexpr size_t kOperandBytes =
        PREC == kPrecF64 ? size_t(kStates) * kStrideF64 * 8
                         : (PREC == kPrecF32 ? size_t(kStates) * kStrideF32 * 4 : size_t(kStates) * kStrideBF16 * 2);
    static constexpr size_t kRedBytes = size_t(16) * kStates * 3 * 8;   // [wave][matrix] (e, f, bad)
    static constexpr size_t kBodyBytes = kOperandBytes > kRedBytes ? kOperandBytes : kRedBytes;
    static constexpr size_t kLdsBytes = size_t(2 * kLogTableSize) * 8 + (kBodyBytes + 15) / 16 * 16;
};

template <int Q, int PREC>
__global__ __launch_bounds__(1024) void k_loglik_dense(const double* __restrict__ nd, const void* mfrag,
                                                       const double* rho, int64_t n, double* ll_out, int poisson)
{
    using Dm = Dims<Q>;
    using DS = DenseShape<Q>;
    using SH = DenseAloneShape<Q, PREC>;
    constexpr int D = Dm::D, D2 = Dm::D2, NS = SH::kStates;
    extern __shared__ double lds_all[];
    const LogEntry* logtab = reinterpret_cast<const LogEntry*>(lds_all);
    log_table_init(reinterpret_cast<LogEntry*>(lds_all), threadIdx.x, 1024);
    char* body = reinterpret_cast<char*>(lds_all + 2 * kLogTableSize);
    const int tid = threadIdx.x, wave = tid >> 6, l = tid & 63, col = l & 15, kq = l >> 4;
    const int64_t first = static_cast<int64_t>(blockIdx.x) * NS;

    // B operands: packed rho (Re rho_ab for a <= b, Im rho_ba for a > b) of
    // each matrix, zero for matrices past n
    for (int e = tid; e < NS * DS::KP32; e += 1024) {
        const int sidx = e / DS::KP32, k = e % DS::KP32;
        const int64_t idx = first + sidx;
        double x = 0.0;
        if (idx < n && k < D2) {
            const int a = k / D, b = k % D;
            x = a <= b ? rho[(idx * D2 + a * D + b) * 2] : rho[(idx * D2 + b * D + a) * 2 + 1];
        }
        if constexpr (PREC == kPrecF64) {
            if (k < D2) reinterpret_cast<double*>(body)[sidx * SH::kStrideF64 + k] = x;
        } else if constexpr (PREC == kPrecF32) {
            if (k < D2) reinterpret_cast<float*>(body)[sidx * SH::kStrideF32 + k] = static_cast<float>(x);
        } else {
            // three BF16 parts, each the rounding of what the previous leave
            __bf16* h = reinterpret_cast<__bf16*>(body) + sidx * SH::kStrideBF16;
            const __bf16 hi = static_cast<__bf16>(static_cast<float>(x));
            const double r1 = x - static_cast<double>(static_cast<float>(hi));
            const __bf16 mid = static_cast<__bf16>(static_cast<float>(r1));
            const double r2 = r1 - static_cast<double>(static_cast<float>(mid));
            h[k] = hi;
            h[DS::KP32 + k] = mid;
            h[2 * DS::KP32 + k] = static_cast<__bf16>(static_cast<float>(r2));
        }
    }
    __syncthreads();

    double pe[SH::kBlocks], pf[SH::kBlocks];
    int bad[SH::kBlocks];                             // per column block: a p <= 0 that carries a count
#pragma unroll
    for (int cb = 0; cb < SH::kBlocks; ++cb) {
        pe[cb] = pf[cb] = 0.0;
        bad[cb] = 0;
    }
    // BF16x3 takes two output tiles per pass, so that every B fragment read
    // from LDS feeds two MFMAs (its LDS traffic, not the MFMA pipe, was the
    // bound with one)
    constexpr int TPG = PREC == kPrecBF16x3 ? 2 : 1;
#pragma unroll 1
    for (int nt0 = wave; nt0 < DS::NT; nt0 += 16 * TPG) {
        if constexpr (PREC == kPrecF64) {
            const int nt = nt0;
            const double* A = static_cast<const double*>(mfrag) + static_cast<size_t>(nt) * DS::KS4 * 64;
            const double* B = reinterpret_cast<const double*>(body) + col * SH::kStrideF64 + kq;
            dense_f64x4 acc[SH::kBlocks];
#pragma unroll
            for (int cb = 0; cb < SH::kBlocks; ++cb) acc[cb] = dense_f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
            for (int ks = 0; ks < DS::KS4; ++ks) {
                const double a = A[ks * 64 + l];
#pragma unroll
                for (int cb = 0; cb < SH::kBlocks; ++cb)
                    acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, B[16 * cb * SH::kStrideF64 + 4 * ks], acc[cb],
                                                                   0, 0, 0);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int kl = 16 * nt + kq + 4 * r;          // FP64 result register r: row l/16 + 4r
                const double c = kl < DS::KD ? nd[kl] : 0.0;
#pragma unroll
                for (int cb = 0; cb < SH::kBlocks; ++cb) {
                    const double p = acc[cb][r];
                    const bool pos = p > 0.0;
                    bad[cb] |= (c > 0.0 && !pos) ? 1 : 0;
                    int ex;
                    const double fr = log_parts(pos ? p : 1.0, logtab, ex);
                    pe[cb] = __builtin_fma(c, static_cast<double>(ex), pe[cb]);
                    pf[cb] = __builtin_fma(c, fr, pf[cb]);
                }
            }
        } else {
            dense_f32x4 acc[TPG][SH::kBlocks];
#pragma unroll
            for (int t = 0; t < TPG; ++t)
#pragma unroll
                for (int cb = 0; cb < SH::kBlocks; ++cb) acc[t][cb] = dense_f32x4{0.0f, 0.0f, 0.0f, 0.0f};
            if constexpr (PREC == kPrecF32) {
                const float* A = static_cast<const float*>(mfrag) + static_cast<size_t>(nt0) * DS::KS4 * 64;
                const float* B = reinterpret_cast<const float*>(body) + col * SH::kStrideF32 + kq;
#pragma unroll 4
                for (int ks = 0; ks < DS::KS4; ++ks) {
                    const float a = A[ks * 64 + l];
#pragma unroll
                    for (int cb = 0; cb < SH::kBlocks; ++cb)
                        acc[0][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, B[16 * cb * SH::kStrideF32 + 4 * ks],
                                                                          acc[0][cb], 0, 0, 0);
                }
            } else {
                const bool second = nt0 + 16 < DS::NT;        // the pass's second tile exists (wave-uniform)
                const dense_bf16x8* A0 =
                    static_cast<const dense_bf16x8*>(mfrag) + static_cast<size_t>(nt0) * DS::KS32 * 64;
                const dense_bf16x8* A1 = A0 + static_cast<size_t>(16) * DS::KS32 * 64;
                const __bf16* B = reinterpret_cast<const __bf16*>(body) + col * SH::kStrideBF16 + 8 * kq;
                // one k-step at a time: its B fragments already fill 36 registers
#pragma unroll 1
                for (int ks = 0; ks < DS::KS32; ++ks) {
                    const dense_bf16x8 a0 = A0[ks * 64 + l];
                    const dense_bf16x8 a1 = second ? A1[ks * 64 + l] : a0;
#pragma unroll
                    for (int cb = 0; cb < SH::kBlocks; ++cb)
#pragma unroll
                        for (int part = 0; part < 3; ++part) {
                            const dense_bf16x8 b = *reinterpret_cast<const dense_bf16x8*>(
                                B + 16 * cb * SH::kStrideBF16 + part * DS::KP32 + 32 * ks);
                            acc[0][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b, acc[0][cb], 0, 0, 0);
                            if (second)
                                acc[TPG - 1][cb] =
                                    __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b, acc[TPG - 1][cb], 0, 0, 0);
                        }
                }
            }
#pragma unroll
            for (int t = 0; t < TPG; ++t) {
                const int nt = nt0 + 16 * t;
                if (nt >= DS::NT) break;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int kl = 16 * nt + 4 * kq + r;      // FP32 result register r: row 4 (l/16) + r
                    const double c = kl < DS::KD ? nd[kl] : 0.0;
#pragma unroll
                    for (int cb = 0; cb < SH::kBlocks; ++cb) {
                        // log2 p by the hardware FP32 logarithm (p clamped at the
                        // smallest normal FP32 value), summed in FP64
                        const float p = fmaxf(acc[t][cb][r], 0x1.0p-126f);
                        pe[cb] = __builtin_fma(c, static_cast<double>(__builtin_amdgcn_logf(p)), pe[cb]);
                    }
                }
            }
        }
    }
    // fold the four row groups of each column (lanes l, l^16, l^32, l^48)
#pragma unroll
    for (int cb = 0; cb < SH::kBlocks; ++cb) {
        pe[cb] += __shfl_xor(pe[cb], 16, 64);
        pf[cb] += __shfl_xor(pf[cb], 16, 64);
        pe[cb] += __shfl_xor(pe[cb], 32, 64);
        pf[cb] += __shfl_xor(pf[cb], 32, 64);
        bad[cb] |= __shfl_xor(bad[cb], 16, 64);
        bad[cb] |= __shfl_xor(bad[cb], 32, 64);
    }
    __syncthreads();                                  // the operand region becomes the reduction area
    double* red = reinterpret_cast<double*>(body);
    if (l < 16) {
#pragma unroll
        for (int cb = 0; cb < SH::kBlocks; ++cb) {
            double* o = red + (static_cast<size_t>(wave) * NS + 16 * cb + col) * 3;
            o[0] = pe[cb];
            o[1] = pf[cb];
            o[2] = static_cast<double>(bad[cb]);
        }
    }
    __syncthreads();
    if (tid < NS && first + tid < n) {
        double te = 0.0, tf = 0.0;
        int tb = 0;
        for (int w = 0; w < 16; ++w) {
            const double* o = red + (static_cast<size_t>(w) * NS + tid) * 3;
            te += o[0];
            tf += o[1];
            tb |= static_cast<int>(o[2]);
        }
        double ll = tb ? -INFINITY : __builtin_fma(te, kLn2, tf);
        if (poisson) {
            // minus sum_m lambda_m p_m = Tr(rho Lambda), packed weights after the counts
            const double* W = nd + Dm::KD;
            const int64_t idx = first + tid;
            double lin = 0.0;
            for (int k = 0; k < D2; ++k) {
                const int a = k / D, b = k % D;
                const double x = a <= b ? rho[(idx * D2 + a * D + b) * 2] : rho[(idx * D2 + b * D + a) * 2 + 1];
                lin = __builtin_fma(W[k], x, lin);
            }
            ll -= lin;
        }
        ll_out[first + tid] = ll;
    }
}

}  // namespace qst
