"""Pins of the oracle's Dirichlet(alpha) weights, gamma_j = P^{-1}(alpha,
Phi(v_j)), w_j = gamma_j / sum gamma, against what is fixed independently:

* P and Q = 1 - P against scipy's regularised incomplete gamma functions,
  the quantile against scipy's inverses;
* alpha = 1: the exponential quantile -log Phi(-v) in closed form;
* the distribution: E[w_j] = 1/D, Var w_j = (D-1) / (D^2 (D alpha + 1)), and
  the prior mean purity of rho, (2 D alpha + D - alpha) / (D (D alpha + 1))
  (the weights' second moments times Haar overlaps E|<z_j, z_k>|^2 = 1/D),
  for alpha in {0.5, 1, 3} over 20000 draws;
* rho is a density matrix.
"""
import numpy as np
import pytest
import scipy.special as sp

from oracle import oracle as O


@pytest.mark.parametrize("a", [0.05, 0.3, 1.0, 2.5, 12.0])
def test_incomplete_gamma_against_scipy(a):
    for x in (1e-6, 0.01, 0.4, 1.0, a, a + 1.5, 5.0, 30.0, 120.0):
        P, Qc = O.gamma_pq(a, x)
        assert abs(P - sp.gammainc(a, x)) <= 1e-13 * max(sp.gammainc(a, x), 1e-300) + 1e-300
        assert abs(Qc - sp.gammaincc(a, x)) <= 1e-12 * max(sp.gammaincc(a, x), 1e-300) + 1e-300


@pytest.mark.parametrize("a", [0.1, 0.5, 1.0, 2.5, 10.0])
def test_quantile_against_scipy(a):
    for v in np.linspace(-6.0, 6.0, 25):
        g = O.gamma_quantile(a, v)
        ref = sp.gammaincinv(a, sp.ndtr(v)) if v <= 0 else sp.gammainccinv(a, sp.ndtr(-v))
        assert abs(g - ref) <= 1e-12 * ref, (a, v, g, ref)


def test_exponential_case():
    for v in np.linspace(-5.0, 5.0, 41):
        # -log Phi(-v), written without cancellation on either side
        want = -np.log(sp.ndtr(-v)) if v > 0 else -np.log1p(-sp.ndtr(v))
        assert abs(O.gamma_quantile(1.0, v) - want) <= 1e-13 * want


@pytest.mark.parametrize("alpha", [0.5, 1.0, 3.0])
def test_prior_moments(alpha):
    Q, D = 2, 4
    n = 20000
    rng = np.random.default_rng(int(alpha * 100))
    pur = np.empty(n)
    w = np.empty((n, D))
    for t in range(n):
        x = rng.standard_normal(2 * D * D + D)
        g = np.array([O.gamma_quantile(alpha, v) for v in x[2 * D * D:]])
        w[t] = g / g.sum()
        rho = O.rho_of_x(Q, x, "dirichlet", alpha)
        pur[t] = np.real(np.trace(rho @ rho))
        if t < 50:
            assert abs(np.trace(rho).real - 1.0) < 1e-14 and np.linalg.eigvalsh(rho).min() > -1e-14
    assert np.abs(w.mean(0) - 1.0 / D).max() < 4 * w.std(0).max() / np.sqrt(n)
    var = (D - 1) / (D * D * (D * alpha + 1))
    assert np.abs(w.var(0) - var).max() < 0.05 * var
    want = (2 * D * alpha + D - alpha) / (D * (D * alpha + 1))
    assert abs(pur.mean() - want) < 4 * pur.std() / np.sqrt(n), (pur.mean(), want)


def test_chains_with_dirichlet_weights():
    Q, D = 2, 4
    counts = np.full(9 * D, 7, dtype=np.int64)
    ch = O.Chains(Q, counts, O.RunParams(n_chains=3, n_steps=0, seed=9, beta0=0.2, param="dirichlet", alpha=2.0))
    for r in range(3):
        rho = O.rho_of_x(Q, ch.x[r], "dirichlet", 2.0)
        assert abs(ch.ll[r] - O.loglik(Q, counts, O.probs(Q, rho))) <= 1e-12 * abs(ch.ll[r])
    out = ch.run(40)
    assert np.all(np.isfinite(ch.ll)) and out["n_accepted"].sum() > 0
