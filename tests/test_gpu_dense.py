"""The dense MFMA contraction p = M vec(rho) (FP64, FP32, BF16x3) against the
FP64 oracle.

FP64: the same bars as the Kronecker path (log L of given states within
1e-12 relative, 1..5 qubits; chains in lockstep within 1e-10, 1..4 qubits).  FP32 and BF16x3: p is
accumulated in FP32 and log2 p taken by the hardware FP32 logarithm; log L
of given states must lie within the a-priori rounding bound of that
arithmetic (_dense_bound), chains within 1e-6 * sum(c) (about 0.08 at 4
qubits) while their decisions agree; and the special case that must be exact
in any precision holds (zero counts: every proposal accepted, the same
trajectories as FP64).
"""
import itertools
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
            4: synth.make_problem("c3"), 5: synth.make_problem("c4")}[Q]


def _abs_eigvec(Q, k, l):
    """|e_kl| entrywise: the product eigenvector of setting k, outcome l
    (X and Y eigenvectors have entries of modulus 1/sqrt 2, Z ones 1 or 0)."""
    s = [(k // 3 ** (Q - 1 - q)) % 3 for q in range(Q)]
    b = [(l >> (Q - 1 - q)) & 1 for q in range(Q)]
    v = np.ones(1)
    for q in range(Q):
        f = np.array([2 ** -0.5, 2 ** -0.5]) if s[q] < 2 else np.eye(2)[b[q]]
        v = np.kron(v, f)
    return v


def _dense_bound(Q, counts, rho, precision):
    """A-priori bound on |log L - log L_fp64| of the reduced-precision dense
    forms: each p_m = sum_k M_mk vec(rho)_k is an FP32 sum of n_t exact
    products (n_t = D^2 for FP32, 3 D^2 padded for BF16x3) of operands
    rounded to relative 2^-24 (FP32 rounding of rho, or what the three BF16
    parts leave), so |dp_m| <= (n_t 2^-23 + 2^-24) A_m with
    A_m = sum_ab |Pi_ab| |rho_ab| = |e_m|^T |rho| |e_m| (Higham ch. 3, with
    u = 2^-23 covering truncating adds); the FP32 logarithm adds at most
    2^-22 |ln p| + 2^-24; each term contributes n_m (|dp_m| / p_m + that)."""
    D, K = 2 ** Q, 3 ** Q
    n_t = D * D if precision == "fp32" else 3 * ((D * D + 31) // 32 * 32)
    g = n_t * 2.0 ** -23 + 2.0 ** -24
    p = O.probs(Q, rho).ravel()
    c = np.asarray(counts, dtype=np.float64).ravel()
    absr = np.abs(rho)
    total = 0.0
    for k, l in itertools.product(range(K), range(D)):
        m = k * D + l
        if c[m] == 0:
            continue
        e = _abs_eigvec(Q, k, l)
        pm = max(p[m], 2.0 ** -126)
        total += c[m] * (g * (e @ absr @ e) / pm + 2.0 ** -22 * abs(np.log(pm)) + 2.0 ** -24)
    return total


def _loglik(P, rhos, precision):
    dev = torch.from_numpy(np.ascontiguousarray(np.stack([rhos.real, rhos.imag], -1))).cuda()
    out = torch.zeros(rhos.shape[0], dtype=torch.float64, device="cuda")
    P.loglik(dev, out, path="dense", precision=precision)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("Q", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
def test_dense_loglik_of_given_states(Q, precision):
    print(f"[dense loglik] Q={Q} {precision}", flush=True)
    prob = _problem(Q)
    D = 2 ** Q
    rng = np.random.default_rng(2000 + Q)
    n = 37 if Q < 5 else 21          # 21 five-qubit matrices span two workgroups of 16 (FP64, BF16x3)
    rhos = np.stack([synth.random_density_matrix(D, rng, rank=int(rng.integers(1, D + 1))) for _ in range(n)])
    want = np.array([O.loglik(Q, prob.counts, O.probs(Q, r)) for r in rhos])
    P = qst.Problem(Q, prob.counts)
    got = _loglik(P, rhos, precision)
    err = np.abs(got - want)
    print(f"  max |dlogL| = {err.max():.3e}, max rel = {np.max(err / np.abs(want)):.3e}", flush=True)
    if precision == "fp64":
        assert np.all(err <= 1e-12 * np.abs(want))
    else:
        bound = np.array([_dense_bound(Q, prob.counts, r, precision) for r in rhos])
        print(f"  max err / a-priori bound = {np.max(err / bound):.3e}", flush=True)
        assert np.all(err <= bound)
        assert np.all(err <= 1e-6 * prob.counts.sum())   # the stated tolerance of the reduced forms


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


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
def test_dense_loglik_zero_probability_marks_only_its_matrix(precision):
    """A matrix with p = 0 on a projector that carries counts has log L = -inf
    (FP64; the reduced forms clamp p at 2^-126 and stay finite); every other
    matrix of its workgroup keeps its own value.  70 matrices span two
    workgroups of 64."""
    Q = 2
    prob = _problem(Q)
    D = 2 ** Q
    rng = np.random.default_rng(77)
    rhos = np.stack([synth.random_density_matrix(D, rng, rank=2) for _ in range(70)])
    pure = np.zeros((D, D), dtype=complex)
    pure[0, 0] = 1.0                     # |00><00|: p = 0 for outcome 11 of the ZZ setting
    for i in (5, 66):
        rhos[i] = pure
    want = np.array([O.loglik(Q, prob.counts, O.probs(Q, r)) for r in rhos])
    P = qst.Problem(Q, prob.counts)
    got = _loglik(P, rhos, precision)
    ok = np.ones(70, dtype=bool)
    ok[[5, 66]] = False
    assert np.all(np.isneginf(want[~ok]))
    if precision == "fp64":
        assert np.all(np.isneginf(got[~ok]))
        assert np.all(np.abs(got[ok] - want[ok]) <= 1e-12 * np.abs(want[ok]))
    else:
        assert np.all(np.isfinite(got))
        assert np.all(np.abs(got[ok] - want[ok]) <= 1e-6 * prob.counts.sum())


def test_dense_chain_step_refused_at_five_qubits():
    """qst_loglik takes the dense path up to 5 qubits; the dense chain step
    (16 chains of a workgroup share the MFMA tiles) stops at 4."""
    prob = _problem(5)
    with pytest.raises(qst.QstError) as e:
        qst.Problem(5, prob.counts, path="dense")
    assert e.value.status == qst.QST_ERR_UNSUPPORTED
