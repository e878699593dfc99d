/* Drives every entry point of the CPU oracle on small problems, built with
 * AddressSanitizer and UndefinedBehaviorSanitizer by
 * tests/test_oracle_sanitize.py (test infrastructure: any out-of-bounds
 * access, leak, misaligned or overflowing operation in the oracle aborts the
 * run with a report).  The oracle is included as one translation unit. */
#include "../../oracle/qst_oracle.c"

#include <stdio.h>

static void fill(double* a, int n, uint64_t seed)
{
    orc_normals(seed, 0, 1, n, a);
}

static void run_chains(int Q, int param, int use_povm, int poisson, int surrogate)
{
    const int D = 1 << Q, D2 = D * D, K = orc_K(Q), KD = K * D, d = orc_param_dim(Q, param);
    const int R = 5, T = 40;
    int64_t* counts = calloc(KD, sizeof(int64_t));
    for (int m = 0; m < KD; ++m) counts[m] = (m * 7) % 13;
    double* povm = NULL;
    int n_povm = 0;
    if (use_povm) {
        /* the Pauli projectors written out as POVM elements, first half only */
        n_povm = KD / 2;
        povm = calloc((size_t)n_povm * 2 * D2, sizeof(double));
        double complex* e = malloc(sizeof(double complex) * D);
        for (int m = 0; m < n_povm; ++m) {
            orc_eigvec(Q, m / D, m % D, e);
            for (int a = 0; a < D; ++a)
                for (int b = 0; b < D; ++b) {
                    const double complex v = e[a] * conj(e[b]);
                    povm[(size_t)m * 2 * D2 + 2 * (a * D + b)] = creal(v);
                    povm[(size_t)m * 2 * D2 + 2 * (a * D + b) + 1] = cimag(v);
                }
        }
        free(e);
        for (int m = n_povm; m < KD; ++m) counts[m] = 0;   /* padding elements carry no counts */
    }
    double* lambda = NULL;
    if (poisson) {
        lambda = malloc(sizeof(double) * KD);
        for (int m = 0; m < KD; ++m) lambda[m] = 10.0 + m;
    }
    orc_mlp mlp;
    double *W1 = NULL, *b1 = NULL, *W2 = NULL, *b2 = NULL, *w3 = NULL;
    if (surrogate) {
        const int h = 6;
        W1 = malloc(sizeof(double) * h * d);
        W2 = malloc(sizeof(double) * h * h);
        b1 = malloc(sizeof(double) * h);
        b2 = malloc(sizeof(double) * h);
        w3 = malloc(sizeof(double) * h);
        fill(W1, h * d, 3);
        fill(W2, h * h, 4);
        fill(b1, h, 5);
        fill(b2, h, 6);
        fill(w3, h, 7);
        mlp = (orc_mlp){d, h, h, W1, b1, W2, b2, w3, 0.1, 0.5, 0.0};
    }
    orc_run_desc rd;
    memset(&rd, 0, sizeof rd);
    rd.n_qubits = Q;
    rd.counts = counts;
    rd.n_chains = R;
    rd.chain_offset = 3;
    rd.thin = 3;
    rd.burn_in = 5;
    rd.beta0 = 0.2;
    rd.adapt_every = 10;
    rd.adapt_lo = 0.2;
    rd.adapt_hi = 0.6;
    rd.adapt_factor = 1.1;
    rd.adapt_until = -1;
    rd.seed = 11;
    rd.surrogate = surrogate ? &mlp : NULL;
    rd.trace_chains = 2;
    rd.record_every = 4;
    rd.record_chains = 2;
    rd.param = param;
    rd.povm = povm;
    rd.n_povm = n_povm;
    rd.alpha = 0.7;
    rd.intensity = lambda;
    orc_state st;
    memset(&st, 0, sizeof st);
    st.x = malloc(sizeof(double) * R * d);
    st.ll = malloc(sizeof(double) * R);
    st.beta = malloc(sizeof(double) * R);
    st.acc_win = malloc(sizeof(int32_t) * R);
    st.rho_cur = malloc(sizeof(double) * R * D2);
    st.s1 = malloc(sizeof(double) * R * D2);
    st.s2 = malloc(sizeof(double) * R * D2);
    st.n_stored = malloc(sizeof(int64_t) * R);
    st.n_accepted = malloc(sizeof(int64_t) * R);
    st.n_stage1 = malloc(sizeof(int64_t) * R);
    st.n_near = malloc(sizeof(int64_t) * R);
    st.tr_llprop = malloc(sizeof(double) * 2 * T);
    st.tr_logu = malloc(sizeof(double) * 2 * T);
    st.tr_accept = malloc(2 * T);
    st.rec = malloc(sizeof(double) * 2 * (T / 4) * D2);
    st.s_cur = malloc(sizeof(double) * R);
    orc_init_chains(&rd, &st);
    for (int half = 0; half < 2; ++half) {
        rd.step_begin = half * T;
        rd.n_steps = T;
        orc_run_chains(&rd, &st);
    }
    double* mean = malloc(sizeof(double) * D2);
    double* second = malloc(sizeof(double) * D2);
    orc_pool(Q, R, st.s1, st.s2, st.n_stored, mean, second);
    printf("Q=%d param=%d povm=%d poisson=%d surrogate=%d: ll[0]=%.6g mean[0]=%.6g\n", Q, param, use_povm, poisson,
           surrogate, st.ll[0], mean[0]);
    free(mean);
    free(second);
    free(st.x); free(st.ll); free(st.beta); free(st.acc_win); free(st.rho_cur); free(st.s1); free(st.s2);
    free(st.n_stored); free(st.n_accepted); free(st.n_stage1); free(st.n_near); free(st.tr_llprop);
    free(st.tr_logu); free(st.tr_accept); free(st.rec); free(st.s_cur);
    free(W1); free(b1); free(W2); free(b2); free(w3);
    free(lambda);
    free(povm);
    free(counts);
}

int main(void)
{
    /* elementary pieces */
    uint64_t ctr[4] = {1, 2, 3, 4}, key[2] = {5, 6}, out[4];
    orc_philox4x64_10(ctr, key, out);
    for (int Q = 1; Q <= 3; ++Q) {
        const int D = 1 << Q, D2 = D * D, KD = orc_K(Q) * D;
        const int nx = 3 * (2 * D2 + D) > 4 * D2 ? 3 * (2 * D2 + D) : 4 * D2;   /* 3 rows for eval_batch */
        double* x = malloc(sizeof(double) * nx);
        double* rho = malloc(sizeof(double) * 2 * D2);
        double* packed = malloc(sizeof(double) * D2);
        double* p = malloc(sizeof(double) * KD);
        int64_t* counts = calloc(KD, sizeof(int64_t));
        fill(x, nx, 9);
        orc_rho(Q, x, rho);
        orc_pack(Q, rho, packed);
        orc_unpack(Q, packed, rho);
        orc_probs(Q, rho, p);
        (void)orc_loglik(Q, counts, p);
        orc_rho_bures(Q, x, rho);
        orc_bures_unitary(Q, x, rho);
        orc_rho_dirichlet(Q, x, 0.3, rho);
        double* ll = malloc(sizeof(double) * 3);
        double* rp = malloc(sizeof(double) * 3 * D2);
        orc_eval_batch(Q, counts, 3, x, ll, rp);
        free(ll); free(rp); free(x); free(rho); free(packed); free(p); free(counts);
    }
    double P, Qc;
    orc_gamma_pq(0.4, 2.0, &P, &Qc);
    (void)orc_gamma_quantile(2.5, -1.3);
    /* chains in every mode */
    for (int Q = 1; Q <= 2; ++Q) {
        run_chains(Q, 0, 0, 0, 0);
        run_chains(Q, 1, 0, 0, 0);
        run_chains(Q, 2, 0, 0, 0);
        run_chains(Q, 0, 1, 0, 0);
        run_chains(Q, 0, 0, 1, 0);
        run_chains(Q, 0, 1, 1, 0);
        run_chains(Q, 0, 0, 0, 1);
    }
    run_chains(3, 0, 0, 1, 1);
    printf("oracle driver done\n");
    return 0;
}
