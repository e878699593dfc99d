"""The dense MFMA contraction p = M vec(rho) (FP64, FP32, BF16x3) against the
FP64 oracle.

FP64: the same bars as the Kronecker path (log L of given states within
1e-12 relative; chains in lockstep within 1e-10).  FP32 and BF16x3: p is
accumulated in FP32, so each p carries a relative error of order
sqrt(K) 2^-24 and log L an error of order sum_m c_m |dp_m / p_m|; the tests
bound |d log L| by 1e-6 * sum(c) (about 0.08 at 4 qubits) and check the
special case that must be exact in any precision (zero counts: every
proposal accepted, the same trajectories as FP64).
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


def _problem(Q):
    return {1: synth.make_problem("c1"), 2: synth.make_problem("c2"), 3: synth.make_problem("w_3"),
            4: synth.make_problem("c3")}[Q]


def _loglik(P, rhos, precision):
    dev = torch.from_numpy(np.ascontiguousarray(np.stack([rhos.real, rhos.imag], -1))).cuda()
    out = torch.zeros(rhos.shape[0], dtype=torch.float64, device="cuda")
    P.loglik(dev, out, path="dense", precision=precision)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("Q", [1, 2, 3, 4])
@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
def test_dense_loglik_of_given_states(Q, precision):
    print(f"[dense loglik] Q={Q} {precision}", flush=True)
    prob = _problem(Q)
    D = 2 ** Q
    rng = np.random.default_rng(2000 + Q)
    n = 37
    rhos = np.stack([synth.random_density_matrix(D, rng, rank=int(rng.integers(1, D + 1))) for _ in range(n)])
    want = np.array([O.loglik(Q, prob.counts, O.probs(Q, r)) for r in rhos])
    P = qst.Problem(Q, prob.counts)
    got = _loglik(P, rhos, precision)
    err = np.abs(got - want)
    print(f"  max |dlogL| = {err.max():.3e}, max rel = {np.max(err / np.abs(want)):.3e}", flush=True)
    if precision == "fp64":
        assert np.all(err <= 1e-12 * np.abs(want))
    else:
        assert np.all(err <= 1e-6 * prob.counts.sum())


@pytest.mark.parametrize("Q", [1, 2, 3, 4])
def test_dense_fp64_chains_lockstep(Q):
    from tests.test_gpu_parity import _compare_lockstep  # noqa: F401  (same protocol)
    prob = _problem(Q)
    R, T, beta0 = {1: (40, 400, 0.1), 2: (40, 300, 0.05), 3: (33, 200, 0.05), 4: (40, 80, 0.02)}[Q]
    print(f"[dense lockstep] Q={Q}", flush=True)
    P = qst.Problem(Q, prob.counts, precision="fp64", path="dense")
    g = gpu_run(Q, prob.counts, n_chains=R, n_steps=T, seed=prob.seed, beta0=beta0, adapt_every=50, trace=R,
                problem=P)
    ch, o = oracle_run(Q, prob.counts, n_chains=R, n_steps=T, seed=prob.seed, beta0=beta0, adapt_every=50, trace=R)
    a, b = o["trace_llprop"], g["trace_llprop"]
    # compare until the first accept decision that differs (none expected)
    for r in range(R):
        diff = np.nonzero(o["trace_accept"][r] != g["trace_accept"][r])[0]
        s = diff[0] if diff.size else T
        assert s == T or abs(o["trace_logu"][r, s] - (a[r, s] - (o["ll0"][r] if s == 0 else 0))) < 1  # informative
        assert np.all(np.abs(a[r, :s] - b[r, :s]) <= 1e-10 * np.abs(a[r, :s]))
    assert np.array_equal(o["trace_accept"], g["trace_accept"])


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_reduced_precision_zero_counts_equal_fp64(precision):
    Q = 3
    counts = np.zeros((27, 8), dtype=np.int64)
    kw = dict(n_chains=48, n_steps=200, seed=12, beta0=0.3, adapt_every=50)
    a = gpu_run(Q, counts, problem=qst.Problem(Q, counts, precision="fp64", path="dense"), **kw)["problem"]
    b = gpu_run(Q, counts, problem=qst.Problem(Q, counts, precision=precision, path="dense"), **kw)["problem"]
    assert np.array_equal(a.state()[0], b.state()[0])
    assert np.array_equal(a.pool()["mean"], b.pool()["mean"])


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_reduced_precision_chain_error(precision):
    Q = 4
    prob = _problem(Q)
    R, T = 32, 60
    P = qst.Problem(Q, prob.counts, precision=precision, path="dense")
    g = gpu_run(Q, prob.counts, n_chains=R, n_steps=T, seed=prob.seed, beta0=0.02, adapt_every=0, trace=R, problem=P)
    ch, o = oracle_run(Q, prob.counts, n_chains=R, n_steps=T, seed=prob.seed, beta0=0.02, adapt_every=0, trace=R)
    worst = 0.0
    for r in range(R):
        diff = np.nonzero(o["trace_accept"][r] != g["trace_accept"][r])[0]
        s = diff[0] + 1 if diff.size else T      # proposals agree up to the first differing decision
        err = np.abs(o["trace_llprop"][r, :s] - g["trace_llprop"][r, :s])
        worst = max(worst, err.max())
    print(f"[{precision}] max |dlogL| over lockstep proposals: {worst:.3e}", flush=True)
    assert worst <= 1e-6 * prob.counts.sum()
