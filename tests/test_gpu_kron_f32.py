"""The mixed-precision Kronecker form: the Gram products of rho, the Pauli
coefficients, per-setting Walsh-Hadamard transforms and log2 p in FP32, the
count-weighted sum in FP64.

* log L of given states against the FP64 oracle within an a-priori
  rounding bound computed from the oracle's probabilities, on 1..6 qubits;
* zero counts: log L is exactly 0 in both precisions, so an FP32 run is the
  FP64 run bit for bit;
* chains against the oracle: per-step log L within 2e-5 of the total count
  while the decisions agree, and where a decision first differs its margin
  |log u - dlog L| lies within twice that bar (the proposal's error and the
  current state's);
* the pooled mean agrees with an FP64 run within the Monte Carlo error.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2501_17334_amd import qst, synth
from tests.gpu_util import gpu_run, oracle_run

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _problem_for(Q):
    return {1: synth.make_problem("c1"), 2: synth.make_problem("c2"), 3: synth.make_problem("w_3"),
            4: synth.make_problem("c3"), 5: synth.make_problem("c4"),
            6: next(p for p in synth.mixed_batch(64) if p.n_qubits == 6)}[Q]


def _rounding_bound(Q, counts, p):
    """A-priori bound on |log L_fp32 - log L| for outcome probabilities p.
    rho' enters rounded to FP32 and every Pauli coefficient is a Q-stage FP32
    transform of a generalised diagonal whose absolute sum is at most 1, so
    |dc| <= (Q + 1) u with u = 2^-24; the per-setting transform adds Q more
    roundings of partial sums of at most D, so |dp| <= (2Q + 2) u.  Each term
    then errs by n (|dp| / p + 2 u |ln p|) (the hardware logarithm is within
    about 2 u), and the FP64 sum adds nothing at this scale."""
    u = 2.0 ** -24
    n = np.asarray(counts, dtype=np.float64).ravel()
    p = np.maximum(np.asarray(p, dtype=np.float64).ravel(), 2.0 ** -126)
    m = n > 0
    return float(np.sum(n[m] * ((2 * Q + 2) * u / p[m] + 2 * u * np.abs(np.log(p[m])))))


@pytest.mark.parametrize("Q", [1, 2, 3, 4, 5, 6])
def test_f32_loglik_of_given_states(Q):
    print(f"[kron f32 loglik] Q={Q}", flush=True)
    prob = _problem_for(Q)
    D = 2 ** Q
    rng = np.random.default_rng(3000 + Q)
    n = 37 if Q < 6 else 5
    rhos = np.stack([synth.random_density_matrix(D, rng, rank=int(rng.integers(1, D + 1))) for _ in range(n)])
    probs = [O.probs(Q, r) for r in rhos]
    want = np.array([O.loglik(Q, prob.counts, pr) for pr in probs])
    bound = np.array([_rounding_bound(Q, prob.counts, pr) for pr in probs])
    P = qst.Problem(Q, prob.counts, precision="fp32", path="kron")
    dev = torch.from_numpy(np.ascontiguousarray(np.stack([rhos.real, rhos.imag], -1))).cuda()
    out = torch.zeros(n, dtype=torch.float64, device="cuda")
    P.loglik(dev, out, path="kron", precision="fp32")
    got = out.cpu().numpy()
    err = np.abs(got - want)
    print(f"  max |dlogL| = {err.max():.3e}; max err / bound = {np.max(err / bound):.3f}", flush=True)
    assert np.all(err <= bound)


def test_f32_zero_counts_equal_fp64():
    Q = 3
    counts = np.zeros((27, 8), dtype=np.int64)
    kw = dict(n_chains=48, n_steps=200, seed=12, beta0=0.3, adapt_every=50)
    a = gpu_run(Q, counts, problem=qst.Problem(Q, counts, precision="fp64", path="kron"), **kw)["problem"]
    b = gpu_run(Q, counts, problem=qst.Problem(Q, counts, precision="fp32", path="kron"), **kw)["problem"]
    assert np.array_equal(a.state()[0], b.state()[0])
    assert np.array_equal(a.pool()["mean"], b.pool()["mean"])


def _current_ll(ll0, llprop, accept, k):
    cur = ll0
    for t in range(k):
        if accept[t]:
            cur = llprop[t]
    return cur


@pytest.mark.parametrize("Q", [1, 2, 3, 4, 5, 6])
def test_f32_chains_against_oracle(Q):
    prob = _problem_for(Q)
    R, T, beta0 = {1: (40, 400, 0.1), 2: (48, 300, 0.05), 3: (24, 150, 0.03), 4: (32, 80, 0.02),
                   5: (8, 12, 0.01), 6: (2, 3, 0.01)}[Q]
    print(f"[kron f32 chains] Q={Q} R={R} T={T}", flush=True)
    P = qst.Problem(Q, prob.counts, precision="fp32", path="kron")
    g = gpu_run(Q, prob.counts, n_chains=R, n_steps=T, seed=prob.seed, beta0=beta0, adapt_every=0, trace=R,
                problem=P)
    ch, o = oracle_run(Q, prob.counts, n_chains=R, n_steps=T, seed=prob.seed, beta0=beta0, adapt_every=0,
                       trace=R)
    bar = 2e-5 * prob.counts.sum()
    worst, firsts = 0.0, []
    for r in range(R):
        acc_o, acc_g = o["trace_accept"][r], g["trace_accept"][r]
        diff = np.nonzero(acc_o != acc_g)[0]
        k = diff[0] if diff.size else T
        s = min(k + 1, T)                    # the proposals agree up to and including step k
        err = np.abs(o["trace_llprop"][r, :s] - g["trace_llprop"][r, :s])
        worst = max(worst, float(err.max()))
        assert np.all(err <= bar), (r, err.max())
        if k < T:
            firsts.append((r, k))
    # a decision may differ only where log u lies within the error of the
    # proposal's log L plus that of the current state's, each within the bar
    band = 2.0 * bar
    for r, k in firsts:
        cur = _current_ll(o["ll0"][r], o["trace_llprop"][r], o["trace_accept"][r], k)
        margin = abs(o["trace_logu"][r, k] - (o["trace_llprop"][r, k] - cur))
        assert margin <= band, (r, k, margin, band)
    print(f"  max |dlogL| {worst:.3e}; chains parting at a near-tie: {len(firsts)} of {R}", flush=True)


def test_f32_pooled_mean_matches_fp64():
    Q = 2
    prob = _problem_for(Q)
    R, T = 4096, 3000
    kw = dict(n_chains=R, n_steps=T, beta0=0.05, adapt_every=100, burn_in=1000)
    a = gpu_run(Q, prob.counts, seed=71, problem=qst.Problem(Q, prob.counts, precision="fp32", path="kron"),
                **kw)["problem"].pool()
    b = gpu_run(Q, prob.counts, seed=72, problem=qst.Problem(Q, prob.counts, precision="fp64", path="kron"),
                **kw)["problem"].pool()
    for part, se in (("real", "se_re"), ("imag", "se_im")):
        diff = np.abs(getattr(a["mean"], part) - getattr(b["mean"], part))
        tol = 5 * np.sqrt(a[se] ** 2 + b[se] ** 2) + 1e-12
        assert np.all(diff <= tol), (part, diff, tol)
