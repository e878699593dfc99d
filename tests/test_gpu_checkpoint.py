"""Checkpoint, restore and failure detection (qst_set_chain_state).

* A checkpoint taken at an adaptation-window boundary (state, beta, moment
  sums, sample counts, step) and restored into a fresh handle gives, resumed,
  the chains of an uninterrupted run bit for bit; restoring the same state
  into the same handle does too.
* A chain whose state is set to NaN has a non-finite log L and NaN
  proposals, never accepts, and is the one chain counted by
  nonfinite_chains; every other chain is unaffected bit for bit.
"""
import numpy as np
import pytest
import torch

from paper_2501_17334_amd import qst, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _cfg(prob, R, T, resume=False):
    return qst.RunConfig(n_chains=R, n_steps=T, seed=prob.seed, beta0=0.03, adapt_every=50, burn_in=20,
                         resume=resume)


@pytest.mark.parametrize("name,R", [("c1", 64), ("c2", 200), ("c3", 96), ("c4", 8), ("c5", 3)])
def test_checkpoint_restore_into_a_fresh_handle(name, R):
    prob = synth.make_problem(name)
    Q = prob.n_qubits
    print(f"[checkpoint] {name} R={R}", flush=True)
    A = qst.Problem(Q, prob.counts)
    A.run(_cfg(prob, R, 100))
    x, ll, beta, nst = A.state()
    s1, s2 = A.moments()
    A.run(_cfg(prob, R, 100, resume=True))                      # uninterrupted: steps 101..200
    C = qst.Problem(Q, prob.counts)
    C.run(_cfg(prob, R, 0))                                     # allocate R chains
    C.set_state(x=x, beta=beta, step=100, s1=s1, s2=s2, n_stored=nst)
    C.run(_cfg(prob, R, 100, resume=True))
    xa, la, ba, na = A.state()
    xc, lc, bc, nc = C.state()
    assert np.array_equal(xa, xc) and np.array_equal(la, lc) and np.array_equal(ba, bc) and np.array_equal(na, nc)
    assert np.array_equal(A.pool()["mean"], C.pool()["mean"])
    # the same state set into the same handle is a no-op for the chains
    B = qst.Problem(Q, prob.counts)
    B.run(_cfg(prob, R, 100))
    xb, _, bb, _ = B.state()
    B.set_state(x=xb, beta=bb)
    B.run(_cfg(prob, R, 100, resume=True))
    assert np.array_equal(B.state()[0], xa) and np.array_equal(B.state()[1], la)


def test_nan_state_is_detected_and_isolated():
    prob = synth.make_problem("c2")
    R, bad = 64, 7
    ref = qst.Problem(2, prob.counts)
    ref.run(_cfg(prob, R, 50))
    ref.run(_cfg(prob, R, 50, resume=True))
    P = qst.Problem(2, prob.counts)
    P.run(_cfg(prob, R, 50))
    x, _, _, _ = P.state()
    x[bad, :] = np.nan
    P.set_state(x=x)
    tr = dict(chains=R, llprop=torch.zeros((R, 50), dtype=torch.float64, device="cuda"),
              logu=torch.zeros((R, 50), dtype=torch.float64, device="cuda"),
              accept=torch.zeros((R, 50), dtype=torch.int8, device="cuda"))
    st = P.run(_cfg(prob, R, 50, resume=True), trace=tr)
    assert st["nonfinite_chains"] == 1
    acc = tr["accept"].cpu().numpy()
    assert not acc[bad].any()                                   # a NaN state never accepts
    xp, lp, _, _ = P.state()
    xr, lr, _, _ = ref.state()
    assert not np.isfinite(lp[bad]) and np.all(np.isnan(xp[bad]))
    keep = np.arange(R) != bad
    assert np.array_equal(xp[keep], xr[keep]) and np.array_equal(lp[keep], lr[keep])


def test_set_state_refusals():
    prob = synth.make_problem("c1")
    P = qst.Problem(1, prob.counts)
    P.n_chains = 4                      # the binding's view; the library has no chains yet
    with pytest.raises(qst.QstError) as e:
        P.set_state(beta=np.full(4, 0.5))
    assert e.value.status == qst.QST_ERR_STATE
    P.run(_cfg(prob, 4, 0))
    with pytest.raises(qst.QstError) as e:
        P.set_state(beta=np.array([0.5, 0.5, 1.5, 0.5]))
    assert e.value.status == qst.QST_ERR_INVALID
