"""Pins of the oracle's delayed-acceptance rule (Christen & Fox 2005) and of
its FP64 network forward pass, on the CPU.

* The forward pass s = out_scale (w3 . gelu(W2 gelu(W1 x + b1) + b2) + b3) +
  out_shift (exact erf GELU, Hendrycks & Gimpel 2016) against two independent
  FP64 evaluations: PyTorch's ``F.linear`` / ``F.gelu(approximate="none")`` in
  float64, and the numpy reference ``oracle/mlp_ref.py``.
* A constant surrogate passes every proposal at stage 1 (log u1 < 0), so
  stage 2 is the plain Metropolis-Hastings test of Algorithm 2: traces, final
  states and moments must equal plain chains bit for bit.
* Both stages together keep the target exact.  With zero counts the target is
  the N(0, I) prior itself, so the chains' final states must be standard
  normal for any surrogate; a surrogate close to s(x) = x_1 makes a wrong rule
  visible (leaving out the stage-2 correction would shift x_1 to N(1, 1), a
  sign error in stage 1 to N(-2, 1)).  The pooled rho must then be the prior
  mean I/D.
* On real 1-qubit data the pooled mean of delayed acceptance with a random
  network matches plain pCN within the Monte Carlo error (Eq. (BME2)).
"""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

from oracle import mlp_ref as M
from oracle import oracle as O
from paper_2501_17334_amd import synth


def _random_weights(rng, d, h1, h2, scale=1.0, shift=0.0):
    p = M.init_params(d, h1, h2, rng)
    p.b1 = rng.normal(0, 0.3, h1)
    p.b2 = rng.normal(0, 0.3, h2)
    p.b3 = 0.2
    return p, O.MlpWeights(p.W1, p.b1, p.W2, p.b2, p.w3, p.b3, scale, shift)


@pytest.mark.parametrize("d,h1,h2", [(10, 7, 5), (36, 32, 16), (528, 64, 64)])
def test_mlp_forward_matches_torch_f64(d, h1, h2):
    rng = np.random.default_rng(d)
    p, w = _random_weights(rng, d, h1, h2, scale=3.5, shift=-1.25)
    X = rng.standard_normal((25, d)) * 1.7
    got = np.array([O.mlp_forward(w, x) for x in X])
    t = lambda a: torch.from_numpy(np.asarray(a, dtype=np.float64))
    a1 = F.gelu(F.linear(t(X), t(p.W1), t(p.b1)), approximate="none")
    a2 = F.gelu(F.linear(a1, t(p.W2), t(p.b2)), approximate="none")
    s = (a2 @ t(p.w3) + p.b3).numpy()
    want_torch = 3.5 * s - 1.25
    want_ref = 3.5 * M.forward(p, X)[0] - 1.25
    scale = np.abs(want_torch) + 1.0
    assert np.all(np.abs(got - want_torch) <= 1e-13 * scale), np.max(np.abs(got - want_torch))
    assert np.all(np.abs(got - want_ref) <= 1e-13 * scale)


def test_mlp_forward_special_cases():
    d, h = 4, 3
    z = O.MlpWeights(np.zeros((h, d)), np.zeros(h), np.zeros((h, h)), np.zeros(h), np.zeros(h), 0.5, 2.0, -1.0)
    assert O.mlp_forward(z, np.arange(d, dtype=float)) == 2.0 * 0.5 - 1.0
    # one path of identities: s = gelu(gelu(x_0)); gelu(t) = t Phi(t)
    W1 = np.zeros((h, d))
    W1[0, 0] = 1.0
    W2 = np.zeros((h, h))
    W2[0, 0] = 1.0
    w3 = np.array([1.0, 0.0, 0.0])
    w = O.MlpWeights(W1, np.zeros(h), W2, np.zeros(h), w3, 0.0)
    from scipy.stats import norm
    for x0 in (-2.0, -0.3, 0.0, 0.7, 3.0):
        g1 = x0 * norm.cdf(x0)
        assert abs(O.mlp_forward(w, np.array([x0, 5.0, -1.0, 2.0])) - g1 * norm.cdf(g1)) < 1e-15


def _zero_counts(Q):
    return np.zeros((3 ** Q, 2 ** Q), dtype=np.int64)


@pytest.mark.parametrize("Q,problem", [(1, "c1"), (2, "c2")])
def test_constant_surrogate_reproduces_plain_pcn(Q, problem):
    prob = synth.make_problem(problem)
    D, K, d = O.dims(Q)
    h = 6
    const = O.MlpWeights(np.zeros((h, d)), np.zeros(h), np.zeros((h, h)), np.zeros(h), np.zeros(h), 0.0, 1.0, 7.5)
    kw = dict(n_chains=12, n_steps=0, seed=prob.seed, beta0=0.08, adapt_every=40, thin=2, burn_in=30,
              trace_chains=12, record_every=5, record_chains=3)
    a = O.Chains(Q, prob.counts, O.RunParams(surrogate=const, **kw))
    b = O.Chains(Q, prob.counts, O.RunParams(**kw))
    oa = a.run(400)
    ob = b.run(400)
    assert np.all(oa["n_stage1"] == 400)
    for k in ("trace_llprop", "trace_logu", "trace_accept", "records", "n_accepted", "n_near"):
        assert np.array_equal(oa[k], ob[k]), k
    for k in ("x", "ll", "beta", "acc_win", "rho_cur", "s1", "s2", "n_stored"):
        assert np.array_equal(getattr(a, k), getattr(b, k)), k


def _linear_surrogate(d, a):
    """An MLP equal to s(x) = a x_0 within 1e-8 while x_0 > -6: both hidden
    units see t = x_0 + 12 > 6, where gelu(t) = t Phi(t) = t (1 - O(e^{-t^2/2}))."""
    h = 2
    W1 = np.zeros((h, d))
    W1[0, 0] = 1.0
    W2 = np.zeros((h, h))
    W2[0, 0] = 1.0
    return O.MlpWeights(W1, np.array([12.0, 0.0]), W2, np.zeros(h), np.array([1.0, 0.0]), -12.0, a, 0.0)


def test_delayed_acceptance_keeps_the_prior():
    """Zero counts: log L = 0, so the exact target is N(0, I); stage 1 screens
    on s(x) ~ x_0 and stage 2 must undo it exactly."""
    Q = 1
    D, K, d = O.dims(Q)
    R, T = 4000, 60
    w = _linear_surrogate(d, 1.0)
    ch = O.Chains(Q, _zero_counts(Q), O.RunParams(n_chains=R, n_steps=0, seed=77, beta0=0.5, adapt_every=0,
                                                  surrogate=w, thin=1, burn_in=30))
    out = ch.run(T)
    x0 = ch.x[:, 0]
    # stage 1 rejects part of the proposals (the screen is not constant) ...
    assert 0.2 * R * T < out["n_stage1"].sum() < 0.95 * R * T
    # ... and stage 2 accepts every survivor that stage 1 let through downhill in s
    # only with probability e^{ds}: the states stay N(0, 1) in every coordinate
    se = 1.0 / np.sqrt(R)
    assert abs(x0.mean()) < 5 * se, x0.mean()
    assert abs(x0.var() - 1.0) < 5 * np.sqrt(2.0 / R)
    other = ch.x[:, 1:].reshape(-1)
    assert abs(other.mean()) < 5 / np.sqrt(other.size)
    # the prior mean of rho (Dirichlet(1/2) weights, Haar columns) is I/D
    pooled = ch.pool()
    cm = pooled["chain_means_packed"]
    se_rho = cm.std(axis=0) / np.sqrt(R)
    assert np.all(np.abs(pooled["mean_packed"] - np.eye(D) / D) < 5 * se_rho + 1e-15)


def test_delayed_acceptance_matches_plain_on_data():
    """1 qubit (c1 counts): pooled means of delayed acceptance and plain pCN
    agree within 5 combined between-chain standard errors."""
    Q = 1
    prob = synth.make_problem("c1")
    D, K, d = O.dims(Q)
    rng = np.random.default_rng(9)
    _, w = _random_weights(rng, d, 16, 16, scale=6.0)
    R, T, burn = 512, 3000, 1000
    kw = dict(n_chains=R, n_steps=0, beta0=0.1, adapt_every=100, burn_in=burn)
    a = O.Chains(Q, prob.counts, O.RunParams(seed=101, surrogate=w, **kw))
    b = O.Chains(Q, prob.counts, O.RunParams(seed=202, **kw))
    oa = a.run(T)
    b.run(T)
    assert oa["n_stage1"].sum() < R * T          # the screen rejected some proposals
    pa, pb = a.pool(), b.pool()
    sa = pa["chain_means_packed"].std(axis=0, ddof=1) / np.sqrt(R)
    sb = pb["chain_means_packed"].std(axis=0, ddof=1) / np.sqrt(R)
    diff = np.abs(pa["mean_packed"] - pb["mean_packed"])
    assert np.all(diff <= 5 * np.sqrt(sa ** 2 + sb ** 2) + 1e-15), (diff, sa, sb)
