"""Uneven batches (one persistent work-queue launch per qubit count and
precision), and the launch-shape tuner.

A batch of problems of 1..6 qubits must give each problem exactly (bit for
bit) what running it alone gives with the same team size, because every
random number is keyed by (seed, problem-local chain id, step).
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2501_17334_amd import qst, synth
from tests.gpu_util import first_near_step

pytestmark = pytest.mark.gpu



@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _problems():
    by_q = {}
    for p in synth.mixed_batch(256):
        by_q.setdefault(p.n_qubits, p)
    return [by_q[q] for q in range(1, 7)]


def test_batch_equals_solo():
    probs = _problems()
    chains = {1: 70, 2: 45, 3: 21, 4: 9, 5: 3, 6: 2}
    steps = {1: 300, 2: 200, 3: 100, 4: 40, 5: 6, 6: 2}
    cfgs = [qst.RunConfig(n_chains=chains[p.n_qubits], n_steps=steps[p.n_qubits], seed=p.seed, beta0=0.05,
                          adapt_every=20, burn_in=1) for p in probs]
    batch = [qst.Problem(p.n_qubits, p.counts) for p in probs]
    print("[batch] run", flush=True)
    st_b = qst.run_batch(batch, cfgs)
    saved = {q: qst.get_launch_shape(q) for q in range(1, 7)}
    try:
        for q in range(1, 7):
            qst.set_launch_shape(q, qst.get_batch_shape(q)[0], max(64, qst.get_batch_shape(q)[0]))
        for p, cfg, b, sb in zip(probs, cfgs, batch, st_b):
            print(f"[batch] solo Q={p.n_qubits}", flush=True)
            solo = qst.Problem(p.n_qubits, p.counts)
            st = solo.run(cfg)
            xs, lls, bs, ns = solo.state()
            xb, llb, bb, nb = b.state()
            assert np.array_equal(xs, xb) and np.array_equal(lls, llb)
            assert np.array_equal(bs, bb) and np.array_equal(ns, nb)
            assert np.array_equal(solo.pool()["mean"], b.pool()["mean"])
            assert st["accepted"] == sb["accepted"]
    finally:
        for q, sh in saved.items():
            qst.set_launch_shape(q, *sh)


def test_mixed_precision_batch_equals_solo():
    """FP64 and FP32 Kronecker problems in one batch: each equals its solo
    run in its own precision with the batch team size, bit for bit."""
    probs = _problems()
    precs = ["fp32", "fp64", "fp32", "fp64", "fp32", "fp32"]
    chains = {1: 40, 2: 33, 3: 17, 4: 9, 5: 4, 6: 2}
    steps = {1: 200, 2: 120, 3: 60, 4: 30, 5: 6, 6: 2}
    cfgs = [qst.RunConfig(n_chains=chains[p.n_qubits], n_steps=steps[p.n_qubits], seed=p.seed + 5, beta0=0.05,
                          adapt_every=20) for p in probs]
    batch = [qst.Problem(p.n_qubits, p.counts, precision=pr, path="kron") for p, pr in zip(probs, precs)]
    print("[batch mixed] run", flush=True)
    qst.run_batch(batch, cfgs)
    saved = {q: qst.get_launch_shape(q) for q in range(1, 7)}
    try:
        for q in range(1, 7):
            qst.set_launch_shape(q, qst.get_batch_shape(q)[0], max(64, qst.get_batch_shape(q)[0]))
        for p, pr, cfg, b in zip(probs, precs, cfgs, batch):
            print(f"[batch mixed] solo Q={p.n_qubits} {pr}", flush=True)
            solo = qst.Problem(p.n_qubits, p.counts, precision=pr, path="kron")
            solo.run(cfg)
            xs, lls, _, _ = solo.state()
            xb, llb, _, _ = b.state()
            assert np.array_equal(xs, xb) and np.array_equal(lls, llb), (p.n_qubits, pr)
    finally:
        for q, sh in saved.items():
            qst.set_launch_shape(q, *sh)


def test_batch_matches_oracle():
    """Every problem of a 1..6-qubit batch against the oracle: per-step log L
    of the proposals to 1e-10 relative while the decisions agree."""
    probs = _problems()
    chains = {1: 6, 2: 5, 3: 4, 4: 3, 5: 3, 6: 2}
    steps = {1: 60, 2: 40, 3: 20, 4: 10, 5: 5, 6: 2}
    cfgs = [qst.RunConfig(n_chains=chains[p.n_qubits], n_steps=steps[p.n_qubits], seed=p.seed, beta0=0.05,
                          adapt_every=0) for p in probs]
    traces = [dict(chains=c.n_chains,
                   llprop=torch.full((c.n_chains, c.n_steps), float("nan"), dtype=torch.float64, device="cuda"),
                   logu=torch.zeros((c.n_chains, c.n_steps), dtype=torch.float64, device="cuda"),
                   accept=torch.zeros((c.n_chains, c.n_steps), dtype=torch.int8, device="cuda")) for c in cfgs]
    batch = [qst.Problem(p.n_qubits, p.counts) for p in probs]
    print("[batch oracle] run", flush=True)
    qst.run_batch(batch, cfgs, traces=traces)
    torch.cuda.synchronize()
    for p, c, tr in zip(probs, cfgs, traces):
        ch = O.Chains(p.n_qubits, p.counts, O.RunParams(n_chains=c.n_chains, n_steps=0, seed=p.seed, beta0=0.05,
                                                         adapt_every=0, trace_chains=c.n_chains))
        ll0 = ch.ll.copy()
        o = ch.run(c.n_steps)
        g_ll = tr["llprop"].cpu().numpy()
        g_acc = tr["accept"].cpu().numpy()
        stop = first_near_step(o["trace_llprop"], g_ll, o["trace_logu"], ll0, o["trace_accept"])
        for r in range(c.n_chains):
            k = stop[r]
            # decisions agree on every step before the first near-tie
            assert np.array_equal(g_acc[r, :k], o["trace_accept"][r, :k]), (p.n_qubits, r)
            a, b = o["trace_llprop"][r, :k], g_ll[r, :k]
            assert np.all(np.abs(a - b) <= 1e-10 * np.abs(a)), (p.n_qubits, r)
        print(f"[batch oracle] Q={p.n_qubits} ok over {stop.tolist()} steps", flush=True)


def test_batch_resume_and_stats():
    probs = _problems()[:4]
    cfgs = [qst.RunConfig(n_chains=33, n_steps=50, seed=p.seed, beta0=0.05, adapt_every=25) for p in probs]
    batch = [qst.Problem(p.n_qubits, p.counts) for p in probs]
    st = qst.run_batch(batch, cfgs)
    assert [s["proposed"] for s in st] == [33 * 50] * 4
    cfgs2 = [qst.RunConfig(n_chains=33, n_steps=30, seed=p.seed, beta0=0.05, adapt_every=25, resume=True)
             for p in probs]
    qst.run_batch(batch, cfgs2)
    for p, b in zip(probs, batch):
        one = qst.Problem(p.n_qubits, p.counts)
        qst.run_batch([one, qst.Problem(1, synth.make_problem("c1").counts)],
                      [qst.RunConfig(n_chains=33, n_steps=80, seed=p.seed, beta0=0.05, adapt_every=25),
                       qst.RunConfig(n_chains=5, n_steps=3, seed=1, beta0=0.1)])
        assert np.array_equal(one.state()[0], b.state()[0])


def test_batch_rejects_dense_and_duplicates():
    p = synth.make_problem("c3")
    a = qst.Problem(4, p.counts, precision="bf16x3", path="dense")
    b = qst.Problem(4, p.counts)
    cfg = qst.RunConfig(n_chains=4, n_steps=2, seed=1, beta0=0.1)
    with pytest.raises(qst.QstError) as e:
        qst.run_batch([a, b], [cfg, cfg])
    assert e.value.status == qst.QST_ERR_UNSUPPORTED
    with pytest.raises(qst.QstError) as e:
        qst.run_batch([b, b], [cfg, cfg])
    assert e.value.status == qst.QST_ERR_INVALID


def test_launch_shapes_roundtrip():
    for q in range(1, 7):
        shapes = qst.list_launch_shapes(q)
        assert len(shapes) >= 1
        cur = qst.get_launch_shape(q)
        assert cur in shapes
    with pytest.raises(qst.QstError):
        qst.set_launch_shape(4, 3, 64)


def test_auto_path_roundtrip():
    saved = qst.get_auto_path(3, "fp64")
    try:
        qst.set_auto_path(3, "fp64", "dense")
        assert qst.get_auto_path(3, "fp64") == "dense"
        p = synth.make_problem("w_3")
        P = qst.Problem(3, p.counts)               # path "auto": now the dense chain step
        st = P.run(qst.RunConfig(n_chains=16, n_steps=5, seed=1, beta0=0.05))
        assert st["proposed"] == 80
    finally:
        qst.set_auto_path(3, "fp64", saved)
    assert qst.get_auto_path(2, "bf16x3") == "dense"
    for q, prec, path, status in ((5, "fp64", "dense", qst.QST_ERR_UNSUPPORTED),
                                  (2, "bf16x3", "kron", qst.QST_ERR_UNSUPPORTED),
                                  (7, "fp64", "kron", qst.QST_ERR_INVALID)):
        with pytest.raises(qst.QstError) as e:
            qst.set_auto_path(q, prec, path)
        assert e.value.status == status
