"""Brute-force posterior mean by prior importance sampling (TEST INFRASTRUCTURE).

For a small problem (1 qubit: x in R^10) the posterior mean of Bayes' rule,
Eq. (Bayes), <rho> = int rho(x) L(x) pi_0(x) dx / int L(x) pi_0(x) dx, is
estimated without any Markov chain: draw x_i ~ pi_0 = N(0, I) and weight each
rho(x_i) by L(x_i) (self-normalised importance sampling).  It shares the
oracle's rho(x) and log L but none of Algorithm 2, so it pins the chain
machinery (proposal, acceptance, adaptation, pooling).
"""
from __future__ import annotations

import numpy as np

from . import oracle as O


def _trace_with(packed, lam):
    """Tr(rho Lambda) for a batch of packed rho [n, D, D] and a Hermitian D x D
    Lambda, from Re rho_ab (a <= b) and Im rho_ba (a > b)."""
    D = lam.shape[0]
    iu = np.triu_indices(D, 1)
    tot = np.einsum("naa,aa->n", packed, lam.real)
    # off-diagonal pairs (a < b): 2 Re(rho_ab conj(Lambda_ab)) = 2 (Re rho Re L + Im rho Im L)
    re = packed[:, iu[0], iu[1]]
    im = packed[:, iu[1], iu[0]]
    return tot + 2.0 * (re @ lam.real[iu] + im @ lam.imag[iu])


def posterior_mean_is(Q, counts, n_draws, seed, batch=1 << 20, poisson_lambda=None):
    """Returns (mean packed rho, standard error packed, IS effective size).
    poisson_lambda (D x D, Hermitian): Poisson counts, whose log L is the
    multinomial one minus Tr(rho Lambda) with Lambda = sum_m lambda_m Pi_m."""
    D, _, d = O.dims(Q)
    rng = np.random.default_rng(seed)
    lls, rhos = [], []
    done = 0
    while done < n_draws:
        n = min(batch, n_draws - done)
        xs = rng.standard_normal((n, d))
        ll, rp = O.eval_batch(Q, counts, xs, want_rho=True)
        if poisson_lambda is not None:
            ll = ll - _trace_with(rp, np.asarray(poisson_lambda))
        lls.append(ll)
        rhos.append(rp.reshape(n, D * D))
        done += n
    ll = np.concatenate(lls)
    rp = np.concatenate(rhos)
    w = np.exp(ll - ll.max())
    w /= w.sum()
    mean = w @ rp
    # delta-method standard error of a self-normalised IS estimate
    var = (w ** 2) @ ((rp - mean) ** 2)
    ess = 1.0 / np.sum(w ** 2)
    return mean.reshape(D, D), np.sqrt(var).reshape(D, D), float(ess)
