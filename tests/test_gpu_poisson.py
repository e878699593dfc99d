"""Poisson counts on the GPU against the oracle (count m ~ Poisson(lambda_m
p_m); log L = sum_{n>0} n ln p - sum_m lambda_m p_m).

* log L of given states on every path and precision (the dense one for 1..5
  qubits): FP64 within 1e-12 relative, FP32 Kronecker within the a-priori bound of its probabilities
  (the linear part is FP64 in every form), reduced dense forms within the
  a-priori bound of their FP32 sums and logarithms;
* chains in lockstep (FP64, Kronecker and dense, Pauli settings and a POVM):
  per-step log L within 1e-10 relative, identical accept flags up to the
  first near-tie;
* a Poisson problem inside an uneven batch equals its solo run bit for bit;
* delayed acceptance refuses Poisson problems.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2501_17334_amd import qst, synth
from tests.gpu_util import first_near_step
from tests.test_gpu_dense import _dense_bound
from tests.test_gpu_kron_f32 import _rounding_bound

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _states(Q, n, seed):
    rng = np.random.default_rng(seed)
    D = 2 ** Q
    return np.stack([synth.random_density_matrix(D, rng, rank=int(rng.integers(1, D + 1))) for _ in range(n)])


@pytest.mark.parametrize("Q", [1, 2, 3, 4, 5, 6])
@pytest.mark.parametrize("path,precision", [("kron", "fp64"), ("kron", "fp32"), ("dense", "fp64"),
                                            ("dense", "fp32"), ("dense", "bf16x3")])
def test_poisson_loglik_of_given_states(Q, path, precision):
    if path == "dense" and Q > 5:
        pytest.skip("the dense contraction of given states is built for 1..5 qubits")
    prob = synth.poisson_problem(Q)
    n = 37 if Q < 5 else 5
    rhos = _states(Q, n, 500 + Q)
    probs = [O.probs(Q, r) for r in rhos]
    want = np.array([O.loglik_poisson(Q, prob.counts, prob.intensity, p) for p in probs])
    if path == "dense" and Q == 5:   # chains on the dense path stop at 4 qubits; given states go to 5
        P = qst.Problem(Q, prob.counts, intensity=prob.intensity)
    else:
        P = qst.Problem(Q, prob.counts, precision=precision, path=path, intensity=prob.intensity)
    dev = torch.from_numpy(np.ascontiguousarray(np.stack([rhos.real, rhos.imag], -1))).cuda()
    out = torch.zeros(n, dtype=torch.float64, device="cuda")
    P.loglik(dev, out, path=path, precision=precision)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    err = np.abs(got - want)
    print(f"[poisson loglik] Q={Q} {path} {precision}: max |dlogL| {err.max():.3e}", flush=True)
    if precision == "fp64":
        assert np.all(err <= 1e-12 * np.abs(want))
    elif path == "kron":
        bound = np.array([_rounding_bound(Q, prob.counts, p) for p in probs])
        assert np.all(err <= bound + 1e-12 * np.abs(want))
    else:
        bound = np.array([_dense_bound(Q, prob.counts, r, precision) for r in rhos])
        assert np.all(err <= bound)


def _lockstep(Q, counts, intensity, R, T, beta0, problem, povm=None):
    tr = dict(chains=R, llprop=torch.full((R, T), float("nan"), dtype=torch.float64, device="cuda"),
              logu=torch.zeros((R, T), dtype=torch.float64, device="cuda"),
              accept=torch.zeros((R, T), dtype=torch.int8, device="cuda"))
    seed = 4242
    problem.run(qst.RunConfig(n_chains=R, n_steps=T, seed=seed, beta0=beta0, adapt_every=50), trace=tr)
    torch.cuda.synchronize()
    ch = O.Chains(Q, counts, O.RunParams(n_chains=R, n_steps=0, seed=seed, beta0=beta0, adapt_every=50,
                                         trace_chains=R, intensity=intensity, povm=povm))
    ll0 = ch.ll.copy()
    o = ch.run(T)
    g_ll, g_acc = tr["llprop"].cpu().numpy(), tr["accept"].cpu().numpy()
    stop = first_near_step(o["trace_llprop"], g_ll, o["trace_logu"], ll0, o["trace_accept"])
    for r in range(R):
        s = stop[r]
        assert np.array_equal(o["trace_accept"][r, :s], g_acc[r, :s]), r
        assert np.all(np.abs(o["trace_llprop"][r, :s] - g_ll[r, :s]) <= 1e-10 * np.abs(o["trace_llprop"][r, :s])), r
    return stop


@pytest.mark.parametrize("Q,path", [(1, "kron"), (2, "kron"), (4, "kron"), (5, "kron"), (2, "dense"), (4, "dense")])
def test_poisson_chains_lockstep(Q, path):
    prob = synth.poisson_problem(Q)
    R, T = {1: (32, 400), 2: (32, 300), 4: (16, 80), 5: (4, 10)}[Q]
    P = qst.Problem(Q, prob.counts, path=path, intensity=prob.intensity)
    stop = _lockstep(Q, prob.counts, prob.intensity, R, T, 0.05 if Q < 4 else 0.01, P)
    print(f"[poisson lockstep] Q={Q} {path}: compared over {int(stop.sum())} chain-steps", flush=True)


def test_poisson_povm_chains_lockstep():
    bp = synth.random_bases_problem(2)
    lam = np.linspace(200.0, 900.0, bp.counts.size)
    P = qst.Problem(2, bp.counts, povm=bp.povm, intensity=lam)
    _lockstep(2, bp.counts, lam, 24, 200, 0.05, P, povm=bp.povm)


def test_poisson_problem_in_a_batch_equals_solo():
    pp = synth.poisson_problem(3)
    other = synth.make_problem("c2")
    cfg = qst.RunConfig(n_chains=40, n_steps=60, seed=pp.seed, beta0=0.03)
    ocfg = qst.RunConfig(n_chains=30, n_steps=20, seed=other.seed, beta0=0.03)
    saved = qst.get_launch_shape(3)
    try:
        qst.set_launch_shape(3, 32, 64)            # the team size of 3-qubit batch tiles
        solo = qst.Problem(3, pp.counts, intensity=pp.intensity)
        solo.run(cfg)
        b = qst.Problem(3, pp.counts, intensity=pp.intensity)
        qst.run_batch([b, qst.Problem(2, other.counts)], [cfg, ocfg])
        xs, ls, _, _ = solo.state()
        xb, lb, _, _ = b.state()
        assert np.array_equal(xs, xb) and np.array_equal(ls, lb)
    finally:
        qst.set_launch_shape(3, *saved)


def test_poisson_refuses_delayed_acceptance():
    pp = synth.poisson_problem(1)
    P = qst.Problem(1, pp.counts, intensity=pp.intensity)
    net = qst.Mlp(P.pair_width, 32, 32)
    net.set_params(np.zeros(net.n_params, dtype=np.float32))
    with pytest.raises(qst.QstError) as e:
        P.run(qst.RunConfig(n_chains=8, n_steps=4, seed=1), surrogate=net.surrogate())
    assert e.value.status == qst.QST_ERR_UNSUPPORTED
    with pytest.raises(qst.QstError) as e:
        qst.Problem(1, pp.counts, intensity=-pp.intensity)
    assert e.value.status == qst.QST_ERR_INVALID
