"""A range of chains run alone (qst_run_desc.chain_offset) reproduces the
same range of a larger run: every random number is keyed by (seed, chain
index within the problem, step), so a failed tile can be rerun by itself.
Checked bit for bit against the full run and against the oracle's chain
offset."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2501_17334_amd import qst, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("name,R,T,k", [("c1", 64, 200, 23), ("c2", 300, 400, 137), ("c3", 96, 60, 65),
                                         ("c4", 12, 10, 9), ("c5", 5, 4, 3)])
def test_tail_of_a_run_alone(name, R, T, k):
    prob = synth.make_problem(name)
    Q = prob.n_qubits
    print(f"[offset] {name} R={R} T={T} k={k}", flush=True)
    full = qst.Problem(Q, prob.counts)
    cfg = qst.RunConfig(n_chains=R, n_steps=T, seed=prob.seed, beta0=0.02, adapt_every=50, burn_in=T // 4)
    full.run(cfg)
    tail = qst.Problem(Q, prob.counts)
    tail.run(qst.RunConfig(n_chains=R - k, n_steps=T, seed=prob.seed, beta0=0.02, adapt_every=50, burn_in=T // 4,
                           chain_offset=k))
    xf, lf, bf, nf = full.state()
    xt, lt, bt, nt = tail.state()
    assert np.array_equal(xf[k:], xt) and np.array_equal(lf[k:], lt)
    assert np.array_equal(bf[k:], bt) and np.array_equal(nf[k:], nt)
    s1f, _ = full.moments()
    s1t, _ = tail.moments()
    assert np.array_equal(s1f[k:], s1t)
    # resuming with another offset is refused
    with pytest.raises(qst.QstError) as e:
        tail.run(qst.RunConfig(n_chains=R - k, n_steps=2, seed=prob.seed, resume=True, chain_offset=k + 1))
    assert e.value.status == qst.QST_ERR_INVALID
    # the oracle's chain at the same global index
    one = O.Chains(Q, prob.counts, O.RunParams(n_chains=1, n_steps=0, seed=prob.seed, beta0=0.02, adapt_every=50,
                                               burn_in=T // 4, chain_offset=R - 1))
    one.run(T)
    assert np.allclose(xt[-1], one.x[0], rtol=1e-9, atol=1e-9)
    assert abs(lt[-1] - one.ll[0]) <= 1e-10 * abs(one.ll[0])


def _buffers(n_tr, n_rec, T, every, D):
    tr = dict(chains=n_tr, llprop=torch.full((n_tr, T), float("nan"), dtype=torch.float64, device="cuda"),
              logu=torch.zeros((n_tr, T), dtype=torch.float64, device="cuda"),
              accept=torch.zeros((n_tr, T), dtype=torch.int8, device="cuda"))
    rec = dict(every=every, chains=n_rec,
               buf=torch.zeros((n_rec, T // every, D, D), dtype=torch.float64, device="cuda"))
    return tr, rec


def test_offset_run_traces_and_records():
    """Traces and records of a range of chains are the rows of a full run's."""
    prob = synth.make_problem("c2")
    R, T, k, every = 256, 300, 100, 10
    cfg = dict(n_steps=T, seed=prob.seed, beta0=0.05, adapt_every=50)
    full = qst.Problem(2, prob.counts)
    trf, recf = _buffers(R, 200, T, every, 4)
    full.run(qst.RunConfig(n_chains=R, **cfg), trace=trf, record=recf)
    tail = qst.Problem(2, prob.counts)
    trt, rect = _buffers(R - k - 6, 200 - k, T, every, 4)
    tail.run(qst.RunConfig(n_chains=R - k, chain_offset=k, **cfg), trace=trt, record=rect)
    torch.cuda.synchronize()
    for key in ("llprop", "logu", "accept"):
        assert torch.equal(trf[key][k:R - 6], trt[key]), key
    assert torch.equal(recf["buf"][k:200], rect["buf"])


def test_offset_handle_in_a_batch():
    probs = [synth.make_problem(n) for n in ("c1", "c3", "c2")]
    offs = [5, 70, 0]
    Rs = [40, 30, 50]
    cfgs = [qst.RunConfig(n_chains=R, n_steps=25, seed=p.seed, beta0=0.03, chain_offset=o)
            for p, R, o in zip(probs, Rs, offs)]
    hs = [qst.Problem(p.n_qubits, p.counts) for p in probs]
    qst.run_batch(hs, cfgs)
    for p, R, o, h in zip(probs, Rs, offs, hs):
        full = qst.Problem(p.n_qubits, p.counts)
        full.run(qst.RunConfig(n_chains=o + R, n_steps=25, seed=p.seed, beta0=0.03))
        xf, lf, _, _ = full.state()
        xb, lb, _, _ = h.state()
        # the batch runs the 4-qubit problem with its batch team size: equal up to rounding
        assert np.allclose(xf[o:], xb, rtol=1e-12, atol=1e-12), p.name
        assert np.allclose(lf[o:], lb, rtol=1e-12), p.name
