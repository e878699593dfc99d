/*
 * qst_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 CPU implementation of the parallel pooled pCN sampler
 * for Bayesian quantum state tomography (Nguyen, Law & Lukens, "Unorthodox
 * parallelization for Bayesian quantum state estimation", arXiv 2501.17334).
 * It exists so that the GPU library can be checked against it; only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark may load
 * it.  It shares no source with the GPU library: its own Philox, its own
 * density-matrix construction and a direct Tr(rho Pi) with no measurement
 * matrix.
 *
 * What is computed, and where it comes from:
 *   - Philox4x64-10 (Salmon, Moraes, Dror & Shaw, SC'11) as the counter-based
 *     source of every random number; uniforms on the open interval (0,1) from
 *     the top 52 bits of a word; normals by the Box-Muller transform (1958).
 *   - rho(x) = sum_j w_j z_j z_j^dag / (z_j^dag z_j) with z_j the j-th column
 *     of a complex Gaussian matrix and w_j = v_j^2 / sum_k v_k^2 (Dirichlet
 *     weights with concentration 1/2): the Gaussian/gamma-derived
 *     parameterisation that replaces the Bures draw of Algorithm 1, with the
 *     real/imaginary block order of Algorithm 1 (Steps 2-3); and, as an
 *     option, Algorithm 1 itself (the Bures draw: complex Householder QR of
 *     a Gaussian H, the phase fix U = Q Lambda, W = (U + I) G).
 *   - p_kl = Tr(Lambda_kl rho) for all 3^Q Pauli settings and 2^Q outcomes
 *     (Section "Steps", step 1; all Pauli settings as in Section "Simulated
 *     Results"), evaluated as <e_kl| rho |e_kl> from the product vector e_kl.
 *   - log L = sum_{kl} c_kl log p_kl (Eq. (likelihood)), dropping terms with
 *     c_kl = 0 and returning -inf if any p_kl <= 0 with c_kl > 0.
 *   - Algorithm 2 (pCN for a single chain): proposal, Metropolis-Hastings
 *     test with a strict "<", step-size adaptation every M_A steps, thinning.
 *     The likelihood of the current state is cached instead of recomputed,
 *     which gives the same decisions.
 *   - Pooled first and second moments (Eq. (BME2); Step 6 with phi(rho)=rho).
 *   - Delayed acceptance (Christen & Fox, J. Comput. Graph. Stat. 2005) with
 *     a surrogate s(x) given by an MLP evaluated here in FP64.
 *
 * Index conventions (the paper leaves them open):
 *   setting k <-> (s_1..s_Q), s in {X=0,Y=1,Z=2}, k = sum_q s_q 3^(Q-q);
 *   outcome l <-> bits (b_1..b_Q), l = sum_q b_q 2^(Q-q); qubit 1 is the most
 *   significant bit and the leftmost Kronecker factor; b = 0 is eigenvalue +1.
 *   x (length 2D^2+D): Re Z_ij = x[jD+i], Im Z_ij = x[D^2+jD+i], v_j = x[2D^2+j].
 *   Packed real form of a Hermitian D x D matrix ("packed rho", D^2 reals,
 *   row-major): P[a][b] = Re rho_ab for a <= b, P[a][b] = Im rho_ba for a > b.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

/* ----------------------------------------------------------------------- */
/* Philox4x64-10 (Salmon et al., SC'11): 10 rounds of the two-multiply      */
/* Feistel-like bijection, key bumped by the Weyl constants between rounds. */
/* ----------------------------------------------------------------------- */
static const uint64_t PHX_M0 = 0xD2E7470EE14C6C93ULL;
static const uint64_t PHX_M1 = 0xCA5A826395121157ULL;
static const uint64_t PHX_W0 = 0x9E3779B97F4A7C15ULL;
static const uint64_t PHX_W1 = 0xBB67AE8584CAA73BULL;

void orc_philox4x64_10(const uint64_t ctr_in[4], const uint64_t key_in[2], uint64_t out[4])
{
    uint64_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
    uint64_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHX_W0;
            k1 += PHX_W1;
        }
        unsigned __int128 prod0 = (unsigned __int128)PHX_M0 * c[0];
        unsigned __int128 prod1 = (unsigned __int128)PHX_M1 * c[2];
        uint64_t hi0 = (uint64_t)(prod0 >> 64), lo0 = (uint64_t)prod0;
        uint64_t hi1 = (uint64_t)(prod1 >> 64), lo1 = (uint64_t)prod1;
        uint64_t n0 = hi1 ^ c[1] ^ k0;
        uint64_t n1 = lo1;
        uint64_t n2 = hi0 ^ c[3] ^ k1;
        uint64_t n3 = lo0;
        c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
    }
    out[0] = c[0]; out[1] = c[1]; out[2] = c[2]; out[3] = c[3];
}

/* Stream tags: which use a Philox block serves. */
enum { ORC_TAG_NORMAL = 0, ORC_TAG_MH = 1, ORC_TAG_DA = 2 };

/* One Philox block of stream `tag`: counter = (block, step, chain, tag<<56),
 * key = (seed, 0). */
static void orc_block(uint64_t seed, int tag, uint64_t block, uint64_t step,
                      uint64_t chain, uint64_t out[4])
{
    uint64_t ctr[4] = {block, step, chain, ((uint64_t)tag) << 56};
    uint64_t key[2] = {seed, 0};
    orc_philox4x64_10(ctr, key, out);
}

/* Uniform on the open interval (0,1): the top 52 bits of the word plus one
 * half, times 2^-52.  Every such value is exactly representable (53 bits), so
 * the result lies in [2^-53, 1 - 2^-53]. */
double orc_u53(uint64_t w)
{
    return ((double)(w >> 12) + 0.5) * 0x1.0p-52;
}

/* n normals of step `step` of chain `chain`: normal i comes from block i/4,
 * words (0,1) -> normals (0,1) and words (2,3) -> normals (2,3) of that
 * block through Box-Muller: r = sqrt(-2 ln u_a), theta = 2 pi u_b,
 * (r cos theta, r sin theta). */
void orc_normals(uint64_t seed, uint64_t chain, uint64_t step, int n, double* out)
{
    for (int b = 0; 4 * b < n; ++b) {
        uint64_t w[4];
        orc_block(seed, ORC_TAG_NORMAL, (uint64_t)b, step, chain, w);
        for (int pair = 0; pair < 2; ++pair) {
            double ua = orc_u53(w[2 * pair]);
            double ub = orc_u53(w[2 * pair + 1]);
            double r = sqrt(-2.0 * log(ua));
            double theta = 2.0 * M_PI * ub;
            int i0 = 4 * b + 2 * pair;
            if (i0 < n) out[i0] = r * cos(theta);
            if (i0 + 1 < n) out[i0 + 1] = r * sin(theta);
        }
    }
}

/* The uniform of the Metropolis-Hastings test of step `step`. */
double orc_mh_uniform(uint64_t seed, uint64_t chain, uint64_t step)
{
    uint64_t w[4];
    orc_block(seed, ORC_TAG_MH, 0, step, chain, w);
    return orc_u53(w[0]);
}

/* The uniform of the first (surrogate) stage of delayed acceptance. */
double orc_da_uniform(uint64_t seed, uint64_t chain, uint64_t step)
{
    uint64_t w[4];
    orc_block(seed, ORC_TAG_DA, 0, step, chain, w);
    return orc_u53(w[0]);
}

/* ----------------------------------------------------------------------- */
/* rho(x) = sum_j w_j z_j z_j^dag / (z_j^dag z_j), w_j = v_j^2 / sum v^2.    */
/* Output: D x D complex, row-major, interleaved (re, im).                   */
/* ----------------------------------------------------------------------- */
void orc_rho(int Q, const double* x, double* rho_out)
{
    const int D = 1 << Q, D2 = D * D;
    double complex* Z = malloc(sizeof(double complex) * D2);
    double* v2 = malloc(sizeof(double) * D);
    double* nz = malloc(sizeof(double) * D);
    for (int j = 0; j < D; ++j)
        for (int i = 0; i < D; ++i)
            Z[i * D + j] = x[j * D + i] + I * x[D2 + j * D + i];
    double vsum = 0.0;
    for (int j = 0; j < D; ++j) {
        v2[j] = x[2 * D2 + j] * x[2 * D2 + j];
        vsum += v2[j];
        double s = 0.0;
        for (int i = 0; i < D; ++i) s += creal(Z[i * D + j] * conj(Z[i * D + j]));
        nz[j] = s;
    }
    for (int a = 0; a < D; ++a) {
        for (int b = 0; b < D; ++b) {
            double complex acc = 0.0;
            for (int j = 0; j < D; ++j) {
                const double wj = v2[j] / vsum;               /* Dirichlet weight */
                acc += (wj / nz[j]) * (Z[a * D + j] * conj(Z[b * D + j]));
            }
            rho_out[2 * (a * D + b)] = creal(acc);
            rho_out[2 * (a * D + b) + 1] = cimag(acc);
        }
    }
    free(Z);
    free(v2);
    free(nz);
}

/* ----------------------------------------------------------------------- */
/* The paper's own parameterisation, Algorithm 1 (Bures draw): x of length   */
/* 4D^2, G = x[0:D^2] + i x[D^2:2D^2], H = x[2D^2:3D^2] + i x[3D^2:4D^2],     */
/* both filled column by column (entry (i, j) at offset jD + i); H = QR;     */
/* U = Q Lambda with Lambda = diag(r_kk / |r_kk|) (Mezzadri 2007), which is  */
/* the unitary factor whose R has a positive real diagonal and so does not   */
/* depend on the sign convention of the QR; W = (U + I) G; rho = W W^dag /   */
/* Tr(W W^dag) (Al Osipov, Sommers & Zyczkowski 2010).                      */
/* ----------------------------------------------------------------------- */
int orc_param_dim(int Q, int param)
{
    const int D = 1 << Q, D2 = D * D;
    return param == 1 ? 4 * D2 : 2 * D2 + D;   /* param 2 (Dirichlet alpha) as 0 */
}

/* Householder QR of the D x D complex matrix A (row-major, overwritten by R
 * in its upper triangle) with Q formed explicitly (row-major); textbook
 * complex Householder reflections P_k = I - 2 v v^dag / (v^dag v) with
 * v = x + e^{i arg x_0} |x| e_1, so that P_k x = -e^{i arg x_0} |x| e_1. */
static void householder_qr(int D, double complex* A, double complex* Qm)
{
    double complex* V = calloc((size_t)D * D, sizeof(double complex));   /* v_k in column k, rows k.. */
    double* vn = calloc((size_t)D, sizeof(double));
    for (int k = 0; k < D; ++k) {
        double alpha = 0.0;
        for (int i = k; i < D; ++i) alpha += creal(A[i * D + k] * conj(A[i * D + k]));
        alpha = sqrt(alpha);
        if (alpha == 0.0) { vn[k] = 0.0; continue; }
        const double complex x0 = A[k * D + k];
        const double complex ph = cabs(x0) > 0.0 ? x0 / cabs(x0) : 1.0;
        for (int i = k; i < D; ++i) V[i * D + k] = A[i * D + k];
        V[k * D + k] += ph * alpha;
        double nv = 0.0;
        for (int i = k; i < D; ++i) nv += creal(V[i * D + k] * conj(V[i * D + k]));
        vn[k] = nv;
        for (int j = k; j < D; ++j) {
            double complex s = 0.0;
            for (int i = k; i < D; ++i) s += conj(V[i * D + k]) * A[i * D + j];
            s *= 2.0 / nv;
            for (int i = k; i < D; ++i) A[i * D + j] -= V[i * D + k] * s;
        }
    }
    /* Q = P_0 P_1 ... P_{D-1}: apply the reflections to I, last one first */
    for (int i = 0; i < D * D; ++i) Qm[i] = 0.0;
    for (int i = 0; i < D; ++i) Qm[i * D + i] = 1.0;
    for (int k = D - 1; k >= 0; --k) {
        if (vn[k] == 0.0) continue;
        for (int j = 0; j < D; ++j) {
            double complex s = 0.0;
            for (int i = k; i < D; ++i) s += conj(V[i * D + k]) * Qm[i * D + j];
            s *= 2.0 / vn[k];
            for (int i = k; i < D; ++i) Qm[i * D + j] -= V[i * D + k] * s;
        }
    }
    free(V);
    free(vn);
}

/* U = Q Lambda of Algorithm 1 for the H of x (D x D complex, row-major,
 * interleaved (re, im)). */
void orc_bures_unitary(int Q, const double* x, double* u_out)
{
    const int D = 1 << Q, D2 = D * D;
    double complex* A = malloc(sizeof(double complex) * D2);
    double complex* Qm = malloc(sizeof(double complex) * D2);
    for (int j = 0; j < D; ++j)
        for (int i = 0; i < D; ++i)
            A[i * D + j] = x[2 * D2 + j * D + i] + I * x[3 * D2 + j * D + i];
    householder_qr(D, A, Qm);
    for (int i = 0; i < D; ++i)
        for (int k = 0; k < D; ++k) {
            const double complex r = A[k * D + k];
            const double complex lam = cabs(r) > 0.0 ? r / cabs(r) : 1.0;
            const double complex u = Qm[i * D + k] * lam;
            u_out[2 * (i * D + k)] = creal(u);
            u_out[2 * (i * D + k) + 1] = cimag(u);
        }
    free(A);
    free(Qm);
}

/* rho(x) of Algorithm 1.  Output: D x D complex, row-major, interleaved. */
void orc_rho_bures(int Q, const double* x, double* rho_out)
{
    const int D = 1 << Q, D2 = D * D;
    double* u = malloc(sizeof(double) * 2 * D2);
    double complex* Gm = malloc(sizeof(double complex) * D2);
    double complex* W = malloc(sizeof(double complex) * D2);
    orc_bures_unitary(Q, x, u);
    for (int j = 0; j < D; ++j)
        for (int i = 0; i < D; ++i) Gm[i * D + j] = x[j * D + i] + I * x[D2 + j * D + i];
    /* W = (U + I) G */
    for (int a = 0; a < D; ++a)
        for (int b = 0; b < D; ++b) {
            double complex acc = 0.0;
            for (int m = 0; m < D; ++m) {
                double complex um = u[2 * (a * D + m)] + I * u[2 * (a * D + m) + 1];
                if (m == a) um += 1.0;
                acc += um * Gm[m * D + b];
            }
            W[a * D + b] = acc;
        }
    double tr = 0.0;
    for (int i = 0; i < D2; ++i) tr += creal(W[i] * conj(W[i]));
    for (int a = 0; a < D; ++a)
        for (int b = 0; b < D; ++b) {
            double complex acc = 0.0;
            for (int m = 0; m < D; ++m) acc += W[a * D + m] * conj(W[b * D + m]);
            acc /= tr;
            rho_out[2 * (a * D + b)] = creal(acc);
            rho_out[2 * (a * D + b) + 1] = cimag(acc);
        }
    free(u);
    free(Gm);
    free(W);
}

/* ----------------------------------------------------------------------- */
/* Dirichlet weights of general concentration alpha (the paper's "other      */
/* priors"): gamma_j = P^{-1}(alpha, Phi(v_j)), the Gamma(alpha) quantile of   */
/* the normal probability of v_j, so that x ~ N(0, I) still maps to the      */
/* prior; w_j = gamma_j / sum_k gamma_k.                                      */
/* ----------------------------------------------------------------------- */
/* Regularised incomplete gamma functions for a > 0, x > 0: the power series
 * P = x^a e^-x / Gamma(a+1) sum_n x^n / ((a+1)...(a+n)) below x = a + 1, the
 * Legendre continued fraction of Q = 1 - P above it (evaluated from the
 * bottom up with a fixed depth). */
static double gamma_prefactor(double a, double x) { return exp(a * log(x) - x - lgamma(a)); }

void orc_gamma_pq(double a, double x, double* P, double* Qc)
{
    if (x <= 0.0) { *P = 0.0; *Qc = 1.0; return; }
    if (x < a + 1.0) {
        double term = 1.0 / a, sum = term;
        for (int n = 1; n < 10000; ++n) {
            term *= x / (a + n);
            sum += term;
            if (term < sum * 1e-17) break;
        }
        *P = sum * gamma_prefactor(a, x);
        *Qc = 1.0 - *P;
    } else {
        /* Q = prefactor / (x + 1 - a - 1(1-a)/(x + 3 - a - 2(2-a)/(x + 5 - a - ...))) */
        double f = x + 2.0 * 400 + 1.0 - a;
        for (int n = 400; n >= 1; --n) f = x + 2.0 * n - 1.0 - a - (double)n * (n - a) / f;
        *Qc = gamma_prefactor(a, x) / f;
        *P = 1.0 - *Qc;
    }
}

/* x with P(a, x) = u (v <= 0, u = Phi(v)) or Q(a, x) = q (v > 0, q = Phi(-v)):
 * bisection on log x until the bracket stops shrinking. */
double orc_gamma_quantile(double a, double v)
{
    const double u = 0.5 * erfc(-v / sqrt(2.0));
    const double q = 0.5 * erfc(v / sqrt(2.0));
    double lo = -800.0, hi = 10.0;             /* log x */
    for (int it = 0; it < 400; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid == lo || mid == hi) break;
        double P, Qc;
        orc_gamma_pq(a, exp(mid), &P, &Qc);
        const int below = v <= 0.0 ? (P < u) : (Qc > q);
        if (below) lo = mid;
        else hi = mid;
    }
    return exp(0.5 * (lo + hi));
}

/* rho(x) = sum_j w_j z_j z_j^dag / |z_j|^2 with w_j from the Gamma(alpha)
 * quantiles of the v_j (same x layout as orc_rho). */
void orc_rho_dirichlet(int Q, const double* x, double alpha, double* rho_out)
{
    const int D = 1 << Q, D2 = D * D;
    double* y = malloc(sizeof(double) * (2 * D2 + D));
    double* g = malloc(sizeof(double) * D);
    double gs = 0.0;
    for (int j = 0; j < D; ++j) {
        g[j] = orc_gamma_quantile(alpha, x[2 * D2 + j]);
        gs += g[j];
    }
    /* orc_rho takes weights v_j^2 / sum v^2: hand it v_j = sqrt(gamma_j) */
    memcpy(y, x, sizeof(double) * 2 * D2);
    for (int j = 0; j < D; ++j) y[2 * D2 + j] = sqrt(g[j] / gs);
    orc_rho(Q, y, rho_out);
    free(y);
    free(g);
}

/* Packed real form of a Hermitian matrix given as interleaved complex. */
void orc_pack(int Q, const double* rho, double* packed)
{
    const int D = 1 << Q;
    for (int a = 0; a < D; ++a)
        for (int b = 0; b < D; ++b)
            packed[a * D + b] = (a <= b) ? rho[2 * (a * D + b)] : rho[2 * (b * D + a) + 1];
}

/* Inverse of orc_pack. */
void orc_unpack(int Q, const double* packed, double* rho)
{
    const int D = 1 << Q;
    for (int a = 0; a < D; ++a)
        for (int b = 0; b < D; ++b) {
            double re, im;
            if (a == b) { re = packed[a * D + a]; im = 0.0; }
            else if (a < b) { re = packed[a * D + b]; im = packed[b * D + a]; }
            else { re = packed[b * D + a]; im = -packed[a * D + b]; }
            rho[2 * (a * D + b)] = re;
            rho[2 * (a * D + b) + 1] = im;
        }
}

/* ----------------------------------------------------------------------- */
/* Pauli measurement: product eigenvectors and outcome probabilities.        */
/* ----------------------------------------------------------------------- */

/* Single-qubit eigenvector of setting s (X=0, Y=1, Z=2) for outcome b
 * (b = 0 <-> eigenvalue +1), component a in {0,1}. */
static double complex eig1(int s, int b, int a)
{
    const double h = 1.0 / sqrt(2.0);
    if (s == 2) return (a == b) ? 1.0 : 0.0;           /* Z: e_0, e_1 */
    if (a == 0) return h;                               /* X, Y: first comp 1/sqrt2 */
    if (s == 0) return (b == 0) ? h : -h;               /* X: (1, +-1)/sqrt2 */
    return (b == 0) ? I * h : -I * h;                   /* Y: (1, +-i)/sqrt2 */
}

/* The product vector e_kl (length D). */
void orc_eigvec(int Q, int k, int l, double complex* e)
{
    const int D = 1 << Q;
    int s[8], b[8];
    for (int q = Q - 1, kk = k; q >= 0; --q) { s[q] = kk % 3; kk /= 3; }
    for (int q = 0; q < Q; ++q) b[q] = (l >> (Q - 1 - q)) & 1;
    for (int a = 0; a < D; ++a) {
        double complex val = 1.0;
        for (int q = 0; q < Q; ++q) val *= eig1(s[q], b[q], (a >> (Q - 1 - q)) & 1);
        e[a] = val;
    }
}

/* p[k*D + l] = Re <e_kl| rho |e_kl> for all K*D projectors. */
void orc_probs(int Q, const double* rho, double* p)
{
    const int D = 1 << Q;
    int K = 1;
    for (int q = 0; q < Q; ++q) K *= 3;
    double complex* e = malloc(sizeof(double complex) * D);
    for (int k = 0; k < K; ++k) {
        for (int l = 0; l < D; ++l) {
            orc_eigvec(Q, k, l, e);
            double complex acc = 0.0;
            for (int a = 0; a < D; ++a)
                for (int b = 0; b < D; ++b) {
                    double complex r = rho[2 * (a * D + b)] + I * rho[2 * (a * D + b) + 1];
                    acc += conj(e[a]) * r * e[b];
                }
            p[k * D + l] = creal(acc);
        }
    }
    free(e);
}

/* log L = sum_{c>0} c log p; -inf if some p <= 0 carries a count. */
/* p_m = Tr(Pi_m rho) for n given POVM elements (n complex D x D matrices,
 * row-major, interleaved), written to p[0..n); p[n..3^Q 2^Q) = 0 (padding
 * elements, which carry no counts). */
void orc_probs_povm(int Q, const double* rho, int n, const double* povm, double* p)
{
    const int D = 1 << Q, D2 = D * D;
    int K = 1;
    for (int q = 0; q < Q; ++q) K *= 3;
    for (int m = 0; m < K * D; ++m) {
        double acc = 0.0;
        if (m < n) {
            const double* P = povm + (size_t)m * 2 * D2;
            for (int a = 0; a < D; ++a)
                for (int b = 0; b < D; ++b) {
                    /* Re(Pi_ab rho_ba) */
                    const double pr = P[2 * (a * D + b)], pi = P[2 * (a * D + b) + 1];
                    const double rr = rho[2 * (b * D + a)], ri = rho[2 * (b * D + a) + 1];
                    acc += pr * rr - pi * ri;
                }
        }
        p[m] = acc;
    }
}

double orc_loglik(int Q, const int64_t* counts, const double* p)
{
    const int D = 1 << Q;
    int K = 1;
    for (int q = 0; q < Q; ++q) K *= 3;
    double ll = 0.0;
    for (int m = 0; m < K * D; ++m) {
        if (counts[m] == 0) continue;
        if (!(p[m] > 0.0)) return -INFINITY;
        ll += (double)counts[m] * log(p[m]);
    }
    return ll;
}

/* Poisson counts, a likelihood other than the multinomial one (Section
 * "Proposed Approach": other likelihoods change only the likelihood steps of
 * Algorithm 2): the count of projector m is Poisson with mean lambda_m p_m,
 * independently of the others, with known intensities lambda_m >= 0 (shots
 * of the setting times the efficiency of the outcome's detector, say).  Up to
 * the constant sum_m (n_m ln lambda_m - ln n_m!),
 *   log L = sum_{n_m > 0} n_m ln p_m - sum_m lambda_m p_m,
 * the second sum over every projector; -inf if a p <= 0 carries a count. */
double orc_loglik_poisson(int Q, const int64_t* counts, const double* lambda, const double* p)
{
    const int D = 1 << Q;
    int K = 1;
    for (int q = 0; q < Q; ++q) K *= 3;
    double ll = 0.0, lin = 0.0;
    for (int m = 0; m < K * D; ++m) {
        lin += lambda[m] * p[m];
        if (counts[m] == 0) continue;
        if (!(p[m] > 0.0)) return -INFINITY;
        ll += (double)counts[m] * log(p[m]);
    }
    return ll - lin;
}

/* ----------------------------------------------------------------------- */
/* MLP surrogate s(x) for delayed acceptance, FP64:                          */
/* h1 = gelu(W1 x + b1), h2 = gelu(W2 h1 + b2), s = out_scale*(w3.h2 + b3)   */
/* + out_shift, with gelu(t) = t * (1 + erf(t/sqrt2)) / 2 (Hendrycks &       */
/* Gimpel 2016, exact form).  Weights row-major: W1[H1][d], W2[H2][H1].      */
/* ----------------------------------------------------------------------- */
typedef struct {
    int d_in, h1, h2;
    const double *W1, *b1, *W2, *b2, *w3;
    double b3, out_scale, out_shift;
} orc_mlp;

static double gelu(double t) { return 0.5 * t * (1.0 + erf(t / sqrt(2.0))); }

double orc_mlp_forward(const orc_mlp* m, const double* x)
{
    double* a1 = malloc(sizeof(double) * m->h1);
    double* a2 = malloc(sizeof(double) * m->h2);
    for (int i = 0; i < m->h1; ++i) {
        double s = m->b1[i];
        for (int t = 0; t < m->d_in; ++t) s += m->W1[(size_t)i * m->d_in + t] * x[t];
        a1[i] = gelu(s);
    }
    for (int i = 0; i < m->h2; ++i) {
        double s = m->b2[i];
        for (int t = 0; t < m->h1; ++t) s += m->W2[(size_t)i * m->h1 + t] * a1[t];
        a2[i] = gelu(s);
    }
    double s = m->b3;
    for (int t = 0; t < m->h2; ++t) s += m->w3[t] * a2[t];
    free(a1);
    free(a2);
    return m->out_scale * s + m->out_shift;
}

/* ----------------------------------------------------------------------- */
/* Algorithm 2 for R independent chains, pooled afterwards.                  */
/* ----------------------------------------------------------------------- */
typedef struct {
    int32_t n_qubits;
    const int64_t* counts;      /* K*D */
    int64_t n_chains;           /* chains handled by this call */
    int64_t chain_offset;       /* id of the first chain (streams are keyed by id) */
    int64_t step_begin;         /* steps step_begin+1 .. step_begin+n_steps run here */
    int64_t n_steps;
    int32_t thin;
    int64_t burn_in;
    double beta0;
    int32_t adapt_every;        /* M_A; 0 = fixed beta */
    double adapt_lo, adapt_hi, adapt_factor;
    int64_t adapt_until;        /* -1 = whole run */
    uint64_t seed;
    const orc_mlp* surrogate;   /* NULL = plain pCN */
    int32_t trace_chains;       /* first chains whose per-step values are traced */
    int32_t record_every, record_chains;
    int32_t param;              /* 0: Gaussian/gamma form (2D^2+D); 1: Algorithm 1 (4D^2) */
    const double* povm;         /* NULL: the Pauli settings; else n_povm POVM elements (counts padded) */
    int32_t n_povm;
    double alpha;               /* param 2: Dirichlet concentration of the weights */
    const double* intensity;    /* NULL: multinomial counts; else Poisson means lambda_m p_m (K*D, padded) */
} orc_run_desc;

/* Per-chain state; arrays are indexed by local chain index r in [0, n_chains). */
typedef struct {
    double* x;          /* n_chains * d: current state y */
    double* ll;         /* n_chains: log L of the current state */
    double* beta;       /* n_chains */
    int32_t* acc_win;   /* n_chains: A, acceptances in the current window */
    double* rho_cur;    /* n_chains * D^2: packed rho of the current state */
    double* s1;         /* n_chains * D^2: sum of packed rho over stored samples */
    double* s2;         /* n_chains * D^2: sum of squares */
    int64_t* n_stored;  /* n_chains */
    int64_t* n_accepted;/* n_chains: total accepts in this call */
    int64_t* n_stage1;  /* n_chains: delayed acceptance, proposals passing stage 1 */
    int64_t* n_near;    /* n_chains: |log u - dlogL| < 1e-8 events */
    /* traces, [trace_chains][n_steps] */
    double* tr_llprop;
    double* tr_logu;
    int8_t* tr_accept;
    /* records, [record_chains][n_steps/record_every][D^2] */
    double* rec;
    /* surrogate values of the current state (delayed acceptance) */
    double* s_cur;
} orc_state;

static int orc_K(int Q) { int K = 1; for (int q = 0; q < Q; ++q) K *= 3; return K; }

/* Evaluate rho, packed rho and log L at x. */
static double eval_state(const orc_run_desc* rd, const double* x, double* rho, double* packed, double* p)
{
    const int Q = rd->n_qubits;
    if (rd->param == 1) orc_rho_bures(Q, x, rho);
    else if (rd->param == 2) orc_rho_dirichlet(Q, x, rd->alpha, rho);
    else orc_rho(Q, x, rho);
    orc_pack(Q, rho, packed);
    if (rd->povm) orc_probs_povm(Q, rho, rd->n_povm, rd->povm, p);
    else orc_probs(Q, rho, p);
    return rd->intensity ? orc_loglik_poisson(Q, rd->counts, rd->intensity, p) : orc_loglik(Q, rd->counts, p);
}

/* Initialise chains: Algorithm 2, line 1 (y^0 ~ N(0,I) from step 0's normals). */
void orc_init_chains(const orc_run_desc* rd, orc_state* st)
{
    const int Q = rd->n_qubits, D = 1 << Q, D2 = D * D, d = orc_param_dim(Q, rd->param), K = orc_K(Q);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < rd->n_chains; ++r) {
        uint64_t chain = (uint64_t)(rd->chain_offset + r);
        double* x = st->x + (size_t)r * d;
        double* rho = malloc(sizeof(double) * 2 * D2);
        double* p = malloc(sizeof(double) * K * D);
        orc_normals(rd->seed, chain, 0, d, x);
        st->ll[r] = eval_state(rd, x, rho, st->rho_cur + (size_t)r * D2, p);
        st->beta[r] = rd->beta0;
        st->acc_win[r] = 0;
        memset(st->s1 + (size_t)r * D2, 0, sizeof(double) * D2);
        memset(st->s2 + (size_t)r * D2, 0, sizeof(double) * D2);
        st->n_stored[r] = 0;
        if (rd->surrogate && st->s_cur) st->s_cur[r] = orc_mlp_forward(rd->surrogate, x);
        free(rho);
        free(p);
    }
}

/* Run steps step_begin+1 .. step_begin+n_steps of Algorithm 2 on every chain. */
void orc_run_chains(const orc_run_desc* rd, orc_state* st)
{
    const int Q = rd->n_qubits, D = 1 << Q, D2 = D * D, d = orc_param_dim(Q, rd->param), K = orc_K(Q);
    const int64_t n_rec_per_chain = rd->record_every > 0 ? rd->n_steps / rd->record_every : 0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < rd->n_chains; ++r) {
        uint64_t chain = (uint64_t)(rd->chain_offset + r);
        double* y = st->x + (size_t)r * d;
        double* rho_c = st->rho_cur + (size_t)r * D2;
        double* s1 = st->s1 + (size_t)r * D2;
        double* s2 = st->s2 + (size_t)r * D2;
        double* eta = malloc(sizeof(double) * d);
        double* yp = malloc(sizeof(double) * d);
        double* rho = malloc(sizeof(double) * 2 * D2);
        double* packed = malloc(sizeof(double) * D2);
        double* p = malloc(sizeof(double) * K * D);
        double ll = st->ll[r];
        double beta = st->beta[r];
        int32_t A = st->acc_win[r];
        int64_t n_acc = 0, n_s1 = 0, n_near = 0;
        double s_cur = (rd->surrogate && st->s_cur) ? st->s_cur[r] : 0.0;

        for (int64_t t = 0; t < rd->n_steps; ++t) {
            const int64_t j = rd->step_begin + 1 + t;
            /* lines 3-4: eta ~ N(0,I); y' = sqrt(1-beta^2) y + beta eta */
            orc_normals(rd->seed, chain, (uint64_t)j, d, eta);
            const double a = sqrt(1.0 - beta * beta);
            for (int i = 0; i < d; ++i) yp[i] = a * y[i] + beta * eta[i];
            /* line 6: alpha ~ U(0,1) */
            const double logu = log(orc_mh_uniform(rd->seed, chain, (uint64_t)j));
            int accept = 0;
            double llp = NAN;
            int evaluated = 1;
            double s_prop = 0.0;
            if (rd->surrogate) {
                /* delayed acceptance: stage 1 on the surrogate */
                s_prop = orc_mlp_forward(rd->surrogate, yp);
                const double logu1 = log(orc_da_uniform(rd->seed, chain, (uint64_t)j));
                if (logu1 < s_prop - s_cur) {
                    ++n_s1;
                    llp = eval_state(rd, yp, rho, packed, p);
                    const double delta = (llp - ll) - (s_prop - s_cur);
                    accept = logu < delta;
                    if (fabs(logu - delta) < 1e-8) ++n_near;
                } else {
                    evaluated = 0;
                }
            } else {
                /* line 5: rho(y') and L(y'); line 7: accept iff log alpha < dlogL */
                llp = eval_state(rd, yp, rho, packed, p);
                accept = logu < llp - ll;
                if (fabs(logu - (llp - ll)) < 1e-8) ++n_near;
            }
            if (accept) {
                memcpy(y, yp, sizeof(double) * d);
                memcpy(rho_c, packed, sizeof(double) * D2);
                ll = llp;
                s_cur = s_prop;
                ++A;
                ++n_acc;
            }
            if (r < rd->trace_chains) {
                st->tr_llprop[(size_t)r * rd->n_steps + t] = evaluated ? llp : NAN;
                st->tr_logu[(size_t)r * rd->n_steps + t] = logu;
                st->tr_accept[(size_t)r * rd->n_steps + t] = (int8_t)accept;
            }
            /* lines 13-21: step-size adaptation every M_A steps */
            if (rd->adapt_every > 0 && j % rd->adapt_every == 0) {
                if (rd->adapt_until < 0 || j <= rd->adapt_until) {
                    const double rate = (double)A / (double)rd->adapt_every;
                    if (rate > rd->adapt_hi) beta = fmin(beta * rd->adapt_factor, 1.0);
                    if (rate < rd->adapt_lo) beta = beta / rd->adapt_factor;
                }
                A = 0;
            }
            /* lines 22-24: thinning; Step 6 / Eq. (BME2) accumulate the moments */
            if (j > rd->burn_in && j % rd->thin == 0) {
                for (int i = 0; i < D2; ++i) {
                    s1[i] += rho_c[i];
                    s2[i] += rho_c[i] * rho_c[i];
                }
                st->n_stored[r] += 1;
            }
            if (rd->record_every > 0 && r < rd->record_chains && (t + 1) % rd->record_every == 0) {
                const int64_t slot = (t + 1) / rd->record_every - 1;
                memcpy(st->rec + ((size_t)r * n_rec_per_chain + slot) * D2, rho_c, sizeof(double) * D2);
            }
        }
        st->ll[r] = ll;
        st->beta[r] = beta;
        st->acc_win[r] = A;
        st->n_accepted[r] = n_acc;
        if (st->n_stage1) st->n_stage1[r] = n_s1;
        st->n_near[r] = n_near;
        if (rd->surrogate && st->s_cur) st->s_cur[r] = s_cur;
        free(eta);
        free(yp);
        free(rho);
        free(packed);
        free(p);
    }
}

/* Eq. (BME2): pooled mean sum_r S1_r / sum_r N_r, returned as packed rho;
 * also the pooled second moment sum_r S2_r / sum_r N_r (packed). */
void orc_pool(int Q, int64_t n_chains, const double* s1, const double* s2,
              const int64_t* n_stored, double* mean_packed, double* second_packed)
{
    const int D2 = 1 << (2 * Q);
    int64_t n_tot = 0;
    for (int64_t r = 0; r < n_chains; ++r) n_tot += n_stored[r];
    for (int i = 0; i < D2; ++i) {
        double a = 0.0, b = 0.0;
        for (int64_t r = 0; r < n_chains; ++r) {
            a += s1[(size_t)r * D2 + i];
            b += s2[(size_t)r * D2 + i];
        }
        mean_packed[i] = n_tot > 0 ? a / (double)n_tot : NAN;
        second_packed[i] = n_tot > 0 ? b / (double)n_tot : NAN;
    }
}

/* log L and packed rho at n parameter vectors (rows of xs); used by the
 * brute-force importance sampler of the tests. */
void orc_eval_batch(int Q, const int64_t* counts, int64_t n, const double* xs,
                    double* ll_out, double* packed_out)
{
    const int D = 1 << Q, D2 = D * D, d = 2 * D2 + D, K = orc_K(Q);
    orc_run_desc rd;
    memset(&rd, 0, sizeof rd);
    rd.n_qubits = Q;
    rd.counts = counts;
#pragma omp parallel
    {
        double* rho = malloc(sizeof(double) * 2 * D2);
        double* packed = malloc(sizeof(double) * D2);
        double* p = malloc(sizeof(double) * K * D);
#pragma omp for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            ll_out[i] = eval_state(&rd, xs + (size_t)i * d, rho, packed, p);
            if (packed_out) memcpy(packed_out + (size_t)i * D2, packed, sizeof(double) * D2);
        }
        free(rho);
        free(packed);
        free(p);
    }
}

/* Threads an OpenMP parallel region of the oracle uses. */
int orc_num_threads(void)
{
    int n = 1;
#pragma omp parallel
    {
#pragma omp single
        n = omp_get_num_threads();
    }
    return n;
}

/* Set the number of threads of the oracle's parallel loops (the baseline
 * timing uses one thread for its single-core figure). */
void orc_set_num_threads(int n)
{
    omp_set_num_threads(n > 0 ? n : 1);
}
