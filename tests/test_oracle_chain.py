"""Pins of the oracle's Algorithm 2 (pCN chain, adaptation, thinning) and of
the pooled estimate Eq. (BME2).

* zero counts: log L == 0, so every proposal is accepted (log u < 0), and
  beta grows by exactly the factor 1.1 at every window end (clamped at 1);
* zero counts: pCN leaves N(0, I) invariant, so after any number of steps
  the states are standard normal, and the pooled mean is the prior mean I/D;
  a wrong proposal coefficient (anything but sqrt(1 - beta^2)) would make the
  state variance drift away from 1;
* a sharply peaked likelihood with beta = 1 rejects almost everything, so
  beta shrinks by 1.1 at every window;
* resume and subset runs are bit-identical to one long run (streams are
  keyed by chain id and step);
* thinning and burn-in store samples at j = T, 2T, ... after the burn-in;
* the 1-qubit posterior mean agrees with brute-force importance sampling.
"""
import numpy as np
import pytest

from oracle import oracle as O
from oracle import bruteforce
from paper_2501_17334_amd import synth


def zero_counts(Q):
    return np.zeros((3 ** Q, 2 ** Q), dtype=np.int64)


def test_zero_counts_accept_all_and_beta_growth():
    Q = 2
    ch = O.Chains(Q, zero_counts(Q), O.RunParams(n_chains=8, n_steps=0, seed=3, beta0=0.1,
                                                 adapt_every=50, trace_chains=8))
    out = ch.run(1500)
    assert np.all(out["n_accepted"] == 1500)
    assert np.all(out["trace_accept"] == 1)
    assert np.all(out["trace_llprop"] == 0.0)
    beta = 0.1
    for _ in range(1500 // 50):
        beta = min(beta * 1.1, 1.0)
    assert beta == 1.0          # 30 windows pass the clamp
    assert np.all(ch.beta == beta)
    ch2 = O.Chains(Q, zero_counts(Q), O.RunParams(n_chains=2, n_steps=0, seed=3, beta0=0.1,
                                                  adapt_every=50))
    ch2.run(1000)
    assert np.all(ch2.beta == 0.1 * 1.1 ** 20) or np.allclose(ch2.beta, 0.1 * 1.1 ** 20, rtol=1e-15)


def test_pcn_preserves_prior():
    Q = 1
    ch = O.Chains(Q, zero_counts(Q), O.RunParams(n_chains=20000, n_steps=0, seed=5, beta0=0.6,
                                                 adapt_every=0))
    ch.run(40)
    x = ch.x.reshape(-1)
    n = x.size
    assert abs(x.mean()) < 5 / np.sqrt(n)
    assert abs(x.var() - 1.0) < 5 * np.sqrt(2.0 / n)
    # each chain moved: correlation with the start is (1-beta^2)^(40/2) ~ 0
    pooled = ch.pool()
    D = 2
    cm = pooled["chain_means_packed"]
    se = cm.std(axis=0) / np.sqrt(cm.shape[0])
    assert np.all(np.abs(pooled["mean_packed"] - np.eye(D) / D) < 5 * se + 1e-15)


def test_sharp_likelihood_shrinks_beta():
    prob = synth.make_problem("c3")
    ch = O.Chains(4, prob.counts, O.RunParams(n_chains=2, n_steps=0, seed=1, beta0=1.0,
                                              adapt_every=50, trace_chains=2))
    out = ch.run(150)
    # with beta = 1 each proposal is a fresh prior draw: it is accepted only
    # when it beats every earlier one (a record), about ln(50) times a window
    acc = out["trace_accept"].reshape(2, 3, 50).sum(axis=2)
    assert np.all(acc < 10)
    assert np.allclose(ch.beta, 1.0 / 1.1 ** 3, rtol=1e-15, atol=0)


def _params(**kw):
    base = dict(n_chains=6, n_steps=0, seed=11, beta0=0.3, adapt_every=25, thin=3,
                burn_in=10, trace_chains=6)
    base.update(kw)
    return O.RunParams(**base)


def test_resume_and_subset_are_bitwise():
    prob = synth.make_problem("c1")
    full = O.Chains(1, prob.counts, _params())
    a = full.run(200)
    half = O.Chains(1, prob.counts, _params())
    b1 = half.run(113)
    b2 = half.run(87)
    assert np.array_equal(full.x, half.x)
    assert np.array_equal(full.ll, half.ll)
    assert np.array_equal(full.s1, half.s1) and np.array_equal(full.s2, half.s2)
    assert np.array_equal(full.beta, half.beta)
    assert np.array_equal(a["trace_llprop"], np.concatenate([b1["trace_llprop"], b2["trace_llprop"]], 1))
    sub = O.Chains(1, prob.counts, _params(n_chains=2, chain_offset=3))
    sub.run(200)
    assert np.array_equal(sub.x, full.x[3:5])
    assert np.array_equal(sub.s1, full.s1[3:5])


def test_thinning_and_burn_in_counts():
    prob = synth.make_problem("c1")
    ch = O.Chains(1, prob.counts, _params(thin=7, burn_in=30))
    ch.run(100)
    # stored at j in {35, 42, ..., 98}
    assert np.all(ch.n_stored == len(range(35, 101, 7)))


def test_trace_is_consistent():
    prob = synth.make_problem("c1")
    ch = O.Chains(1, prob.counts, _params(adapt_every=0))
    ll0 = ch.ll.copy()
    out = ch.run(300)
    for r in range(6):
        ll = ll0[r]
        for t in range(300):
            acc = out["trace_logu"][r, t] < out["trace_llprop"][r, t] - ll
            assert acc == bool(out["trace_accept"][r, t])
            if acc:
                ll = out["trace_llprop"][r, t]
        assert ll == ch.ll[r]
    # the cached log L of the final state is that state's log L
    for r in range(6):
        assert abs(O.loglik_of_x(1, prob.counts, ch.x[r]) - ch.ll[r]) <= 1e-12 * abs(ch.ll[r])


@pytest.mark.slow
def test_one_qubit_posterior_matches_importance_sampling():
    prob = synth.make_problem("c1")
    # importance sampling from the prior, 4e6 draws
    is_mean, is_se, ess = bruteforce.posterior_mean_is(1, prob.counts, 4_000_000, seed=99)
    assert ess > 300
    # MCMC: 512 chains, adaptation on, burn-in
    ch = O.Chains(1, prob.counts, O.RunParams(n_chains=512, n_steps=0, seed=7, beta0=0.1,
                                              adapt_every=100, burn_in=1500, thin=5))
    ch.run(4000)
    pooled = ch.pool()
    cm = pooled["chain_means_packed"]
    mc_se = cm.std(axis=0) / np.sqrt(cm.shape[0])
    diff = np.abs(pooled["mean_packed"] - is_mean)
    assert np.all(diff < 4 * np.sqrt(is_se ** 2 + mc_se ** 2) + 1e-4), (diff, is_se, mc_se)
