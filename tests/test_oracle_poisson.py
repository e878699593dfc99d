"""Pins of the oracle's Poisson likelihood (a non-multinomial likelihood:
count m ~ Poisson(lambda_m p_m) independently), log L = sum_{n>0} n ln p -
sum_m lambda_m p_m up to a constant.

* With the same intensity N_k for every outcome of setting k the outcome
  probabilities of a setting sum to one, so the Poisson log L is the
  multinomial one minus the constant sum_k N_k for every rho, and chains make
  the same decisions.
* Against scipy's Poisson log-pmf: the sum of log P(n_m; lambda_m p_m) is the
  oracle's value plus sum_m (n_m ln lambda_m - ln n_m!).
* A zero probability with a count gives -inf; without a count it is fine.
* The 1-qubit posterior mean under unequal detector efficiencies matches
  brute-force importance sampling from the prior (Bayes' rule, Eq. (Bayes)),
  and differs from the multinomial posterior of the same counts.
"""
import numpy as np
import pytest
from scipy.special import gammaln
from scipy.stats import poisson

from oracle import bruteforce
from oracle import oracle as O
from paper_2501_17334_amd import synth

SX = np.array([[0, 1], [1, 0]], dtype=complex)
SY = np.array([[0, -1j], [1j, 0]])
SZ = np.array([[1, 0], [0, -1]], dtype=complex)


def _eigvecs():
    """Textbook eigenvectors (+1 first) of X, Y, Z from numpy's eigh."""
    out = []
    for s in (SX, SY, SZ):
        w, v = np.linalg.eigh(s)
        out.append([v[:, 1], v[:, 0]])          # eigenvalue +1, then -1
    return out


def lambda_operator(Q, intensity):
    """sum_kl lambda_kl Pi_kl from product eigenvectors (independent of the
    oracle's projector code)."""
    ev = _eigvecs()
    D = 2 ** Q
    L = np.zeros((D, D), dtype=complex)
    lam = np.asarray(intensity, dtype=float).reshape(3 ** Q, D)
    for k in range(3 ** Q):
        s = [(k // 3 ** (Q - 1 - q)) % 3 for q in range(Q)]
        for l in range(D):
            e = np.ones(1, dtype=complex)
            for q in range(Q):
                e = np.kron(e, ev[s[q]][(l >> (Q - 1 - q)) & 1])
            L += lam[k, l] * np.outer(e, e.conj())
    return L


@pytest.mark.parametrize("Q", [1, 2, 3])
def test_equal_intensities_give_multinomial_minus_a_constant(Q):
    D, K = 2 ** Q, 3 ** Q
    rng = np.random.default_rng(10 + Q)
    counts = rng.integers(0, 50, size=(K, D))
    N = rng.integers(100, 1000, size=K).astype(float)
    lam = np.repeat(N[:, None], D, axis=1)
    for _ in range(5):
        rho = synth.random_density_matrix(D, rng, rank=int(rng.integers(1, D + 1)))
        p = O.probs(Q, rho)
        lp = O.loglik_poisson(Q, counts, lam, p)
        lm = O.loglik(Q, counts, p)
        assert abs((lp - lm) - (-N.sum())) <= 1e-9 * abs(lp)


def test_matches_scipy_poisson_log_pmf():
    Q = 2
    prob = synth.poisson_problem(Q)
    rng = np.random.default_rng(3)
    for _ in range(5):
        rho = synth.random_density_matrix(4, rng, rank=2)
        p = O.probs(Q, rho).ravel()
        n = prob.counts.ravel()
        lam = prob.intensity.ravel()
        want = np.sum(poisson.logpmf(n, lam * p))
        got = O.loglik_poisson(Q, prob.counts, prob.intensity, p) + np.sum(n * np.log(lam) - gammaln(n + 1))
        assert abs(got - want) <= 1e-10 * abs(want), (got, want)


def test_zero_probability():
    Q = 1
    rho = np.array([[1, 0], [0, 0]], dtype=complex)    # |0><0|: p = 0 for outcome 1 of Z
    p = O.probs(Q, rho)
    lam = np.full((3, 2), 100.0)
    counts = np.zeros((3, 2), dtype=np.int64)
    counts[2, 1] = 1
    assert O.loglik_poisson(Q, counts, lam, p) == -np.inf
    counts[2, 1] = 0
    counts[0, 0] = 3
    val = O.loglik_poisson(Q, counts, lam, p)
    assert np.isfinite(val)
    assert abs(val - (3 * np.log(0.5) - 300.0)) < 1e-12      # sum_l p_kl = 1 for each of the 3 settings


def test_chains_with_equal_intensities_make_the_multinomial_decisions():
    prob = synth.make_problem("c2")
    lam = np.full(prob.counts.shape, 1000.0)
    kw = dict(n_chains=16, n_steps=0, seed=prob.seed, beta0=0.05, adapt_every=50, trace_chains=16)
    a = O.Chains(2, prob.counts, O.RunParams(intensity=lam, **kw))
    b = O.Chains(2, prob.counts, O.RunParams(**kw))
    oa, ob = a.run(600), b.run(600)
    assert np.array_equal(oa["trace_accept"], ob["trace_accept"])
    assert np.allclose(oa["trace_llprop"] - ob["trace_llprop"], -9 * 1000.0, rtol=0, atol=1e-7)
    assert np.allclose(a.x, b.x, rtol=0, atol=1e-12)


def test_one_qubit_poisson_posterior_matches_importance_sampling():
    prob = synth.poisson_problem(1)
    L = lambda_operator(1, prob.intensity)
    is_mean, is_se, ess = bruteforce.posterior_mean_is(1, prob.counts, 4_000_000, seed=98, poisson_lambda=L)
    assert ess > 300
    ch = O.Chains(1, prob.counts, O.RunParams(n_chains=512, n_steps=0, seed=8, beta0=0.1, adapt_every=100,
                                              burn_in=1500, thin=5, intensity=prob.intensity))
    ch.run(4000)
    pooled = ch.pool()
    cm = pooled["chain_means_packed"]
    mc_se = cm.std(axis=0) / np.sqrt(cm.shape[0])
    diff = np.abs(pooled["mean_packed"] - is_mean)
    assert np.all(diff < 4 * np.sqrt(is_se ** 2 + mc_se ** 2) + 1e-4), (diff, is_se, mc_se)
    # the multinomial model of the same counts ignores the unequal detectors
    m_mean, m_se, _ = bruteforce.posterior_mean_is(1, prob.counts, 1_000_000, seed=97)
    assert np.max(np.abs(m_mean - is_mean)) > 10 * np.max(np.sqrt(m_se ** 2 + is_se ** 2))
