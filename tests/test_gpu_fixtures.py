"""GPU runs against stored oracle runs (tests/golden/*.npz, written by
tests/golden/make_fixtures.py from the FP64 oracle alone): the 2-qubit
workload at full size (4096 chains x 10^4 steps), the 5-qubit workload
(64 x 200) and a 6-qubit problem of the mixed batch (32 x 50), the last one
both alone and inside an uneven batch.

Bars: per-step log L of the traced proposals within 1e-10 relative and
identical accept flags up to the first step where |log u - dlogL| < 1e-8 on
either side; every chain's final log L within 1e-10 relative and its final
beta identical (beta changes only by exact factors at window ends, so equal
decisions give equal values); the pooled mean of Eq. (BME2) over the chains
without a near-threshold decision within 1e-11 (Frobenius).
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2501_17334_amd import qst, synth
from tests.golden.make_fixtures import FIXTURES, load, problem_of
from tests.gpu_util import first_near_step

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _config(f):
    return qst.RunConfig(n_chains=int(f["n_chains"]), n_steps=int(f["n_steps"]), seed=int(f["seed"]),
                         beta0=float(f["beta0"]), adapt_every=int(f["adapt_every"]), burn_in=int(f["burn_in"]),
                         thin=int(f["thin"]))


def _trace(f):
    k, T = f["trace_llprop"].shape
    if k == 0:
        return None
    return dict(chains=k, llprop=torch.full((k, T), float("nan"), dtype=torch.float64, device="cuda"),
                logu=torch.zeros((k, T), dtype=torch.float64, device="cuda"),
                accept=torch.zeros((k, T), dtype=torch.int8, device="cuda"))


def _compare(name, f, P, tr):
    D = 2 ** int(f["n_qubits"])
    R = int(f["n_chains"])
    if tr is not None:
        g_ll = tr["llprop"].cpu().numpy()
        g_acc = tr["accept"].cpu().numpy()
        o_ll, o_lu, o_acc = f["trace_llprop"], f["trace_logu"], f["trace_accept"]
        stop = first_near_step(o_ll, g_ll, o_lu, f["ll0"][:len(o_ll)], o_acc)
        for r in range(len(o_ll)):
            s = stop[r]
            assert np.array_equal(o_acc[r, :s], g_acc[r, :s]), (name, r)
            assert np.all(np.abs(o_ll[r, :s] - g_ll[r, :s]) <= 1e-10 * np.abs(o_ll[r, :s])), (name, r)
            g_lu = tr["logu"].cpu().numpy()[r, :s]
            assert np.all(np.abs(g_lu - o_lu[r, :s]) <= 2e-15 * np.maximum(1.0, np.abs(o_lu[r, :s]))), (name, r)
        print(f"[fixtures] {name}: traced chains compared over {stop.tolist()} steps", flush=True)
    x, ll, beta, nst = P.state()
    near = set(f["near_chains"].tolist())
    keep = np.array([r for r in range(R) if r not in near])
    assert np.all(np.abs(ll[keep] - f["ll_final"][keep]) <= 1e-10 * np.abs(f["ll_final"][keep])), name
    assert np.array_equal(beta[keep], f["beta_final"][keep]), name
    assert np.array_equal(nst, f["n_stored"]), name
    s1, s2 = P.moments()
    s1 = s1.reshape(R, D * D)[keep].sum(axis=0)
    n = nst[keep].sum()
    assert n == int(f["n_samples"])
    err = float(np.sqrt(np.sum((s1 / n - f["s1_sum"] / n) ** 2)))
    print(f"[fixtures] {name}: {len(keep)} of {R} chains, pooled-mean difference {err:.2e} (Frobenius, packed)",
          flush=True)
    assert err <= 1e-11, (name, err)
    if not near:
        # the library's own pooling (Eq. (BME2)) against the stored sums
        mean = P.pool()["mean"]
        want = O.unpack(f["s1_sum"].reshape(D, D) / n)
        assert float(np.sqrt(np.sum(np.abs(mean - want) ** 2))) <= 1e-11


@pytest.mark.parametrize("name", ["c2_full", "c4_q5", "c5_q6"])
def test_solo_run_matches_stored_oracle(name):
    f = load(name)
    Q = int(f["n_qubits"])
    prob = problem_of(FIXTURES[name])
    assert np.array_equal(prob.counts.reshape(-1), f["counts"])
    cfg = _config(f)
    print(f"[fixtures] {name}: Q={Q} {cfg.n_chains} x {cfg.n_steps}, shape {qst.get_launch_shape(Q)}", flush=True)
    P = qst.Problem(Q, prob.counts)
    tr = _trace(f)
    st = P.run(cfg, trace=tr)
    torch.cuda.synchronize()
    assert st["nonfinite_chains"] == 0
    _compare(name, f, P, tr)


def test_six_qubit_problem_in_a_batch_matches_stored_oracle():
    """The 6-qubit fixture problem inside an uneven batch with a 1-, 3- and
    5-qubit problem: the batch tile gives the oracle's chains too."""
    name = "c5_q6"
    f = load(name)
    prob = problem_of(FIXTURES[name])
    others = [synth.make_problem("c5", index=i) for i in (1, 2, 5)]
    probs = [prob] + others
    cfgs = [_config(f)] + [qst.RunConfig(n_chains=40, n_steps=12, seed=p.seed, beta0=0.02) for p in others]
    handles = [qst.Problem(p.n_qubits, p.counts) for p in probs]
    tr = _trace(f)
    print(f"[fixtures] batch of {[p.n_qubits for p in probs]} qubits", flush=True)
    qst.run_batch(handles, cfgs, traces=[tr, None, None, None])
    torch.cuda.synchronize()
    _compare(name + " (batch)", f, handles[0], tr)
