"""Dirichlet(alpha) weights on the GPU (Newton on log x from a Wilson-
Hilferty start, series / continued fraction) against the oracle's
bisection: chains in lockstep with per-step log L within 1e-10 relative,
the packed rho of every final state within 1e-12 of the oracle's rho(x),
on 1 to 6 qubits and alpha from 0.3 to 2; refusals."""
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


@pytest.mark.parametrize("Q,alpha", [(1, 0.8), (2, 0.3), (2, 2.0), (3, 1.3), (4, 1.0), (4, 0.5), (5, 1.7), (6, 0.7)])
def test_dirichlet_chains_match_oracle(Q, alpha):
    prob = {1: synth.make_problem("c1"), 2: synth.make_problem("c2"), 3: synth.make_problem("w_3"),
            4: synth.make_problem("c3"), 5: synth.make_problem("c4"),
            6: next(p for p in synth.mixed_batch(64) if p.n_qubits == 6)}[Q]
    R, T, beta0 = {1: (32, 200, 0.1), 2: (24, 150, 0.05), 3: (16, 80, 0.03), 4: (8, 50, 0.02), 5: (4, 8, 0.01),
                   6: (2, 3, 0.01)}[Q]
    D = 2 ** Q
    print(f"[dirichlet] Q={Q} alpha={alpha} R={R} T={T}", flush=True)
    P = qst.Problem(Q, prob.counts, param="dirichlet", alpha=alpha)
    tr = dict(chains=R, llprop=torch.full((R, T), float("nan"), dtype=torch.float64, device="cuda"),
              logu=torch.zeros((R, T), dtype=torch.float64, device="cuda"),
              accept=torch.zeros((R, T), dtype=torch.int8, device="cuda"))
    rec = dict(every=T, chains=R, buf=torch.zeros((R, 1, D, D), dtype=torch.float64, device="cuda"))
    P.run(qst.RunConfig(n_chains=R, n_steps=T, seed=prob.seed, beta0=beta0, adapt_every=0), trace=tr, record=rec)
    torch.cuda.synchronize()
    ch = O.Chains(Q, prob.counts, O.RunParams(n_chains=R, n_steps=0, seed=prob.seed, beta0=beta0, adapt_every=0,
                                              trace_chains=R, param="dirichlet", alpha=alpha))
    ll0 = ch.ll.copy()
    o = ch.run(T)
    g_ll, g_acc = tr["llprop"].cpu().numpy(), tr["accept"].cpu().numpy()
    stop = first_near_step(o["trace_llprop"], g_ll, o["trace_logu"], ll0, o["trace_accept"])
    worst = 0.0
    for r in range(R):
        s = stop[r]
        rel = np.abs(o["trace_llprop"][r, :s] - g_ll[r, :s]) / np.abs(o["trace_llprop"][r, :s])
        if s:
            worst = max(worst, float(rel.max()))
        assert np.all(rel <= 1e-10), (r, rel.max())
        assert np.array_equal(o["trace_accept"][r, :s], g_acc[r, :s]), r
    x = P.state()[0]
    recs = rec["buf"].cpu().numpy()
    for r in range(R):
        want = O.pack(O.rho_of_x(Q, x[r], "dirichlet", alpha))
        assert np.abs(recs[r, 0] - want).max() < 1e-12, r
    print(f"  max relative |dlogL| {worst:.2e}", flush=True)


def _current_ll(ll0, llprop, accept, k):
    cur = ll0
    for t in range(k):
        if accept[t]:
            cur = llprop[t]
    return cur


@pytest.mark.parametrize("Q,alpha", [(2, 0.6), (4, 1.4), (6, 0.9)])
def test_dirichlet_fp32_form_within_its_bar(Q, alpha):
    """The FP32 Kronecker form with Dirichlet weights against the FP64
    oracle, to the FP32 form's bars: per-step log L within 2e-5 of the total
    count while the decisions agree, and a first differing decision only
    where |log u - dlog L| lies within twice that bar."""
    prob = {2: synth.make_problem("c2"), 4: synth.make_problem("c3"),
            6: next(p for p in synth.mixed_batch(64) if p.n_qubits == 6)}[Q]
    R, T, beta0 = {2: (24, 150, 0.05), 4: (8, 50, 0.02), 6: (2, 3, 0.01)}[Q]
    print(f"[dirichlet fp32] Q={Q} alpha={alpha} R={R} T={T}", flush=True)
    P = qst.Problem(Q, prob.counts, precision="fp32", param="dirichlet", alpha=alpha)
    tr = dict(chains=R, llprop=torch.full((R, T), float("nan"), dtype=torch.float64, device="cuda"),
              logu=torch.zeros((R, T), dtype=torch.float64, device="cuda"),
              accept=torch.zeros((R, T), dtype=torch.int8, device="cuda"))
    P.run(qst.RunConfig(n_chains=R, n_steps=T, seed=prob.seed, beta0=beta0, adapt_every=0), trace=tr)
    torch.cuda.synchronize()
    ch = O.Chains(Q, prob.counts, O.RunParams(n_chains=R, n_steps=0, seed=prob.seed, beta0=beta0, adapt_every=0,
                                              trace_chains=R, param="dirichlet", alpha=alpha))
    ll0 = ch.ll.copy()
    o = ch.run(T)
    g_ll, g_acc = tr["llprop"].cpu().numpy(), tr["accept"].cpu().numpy()
    bar = 2e-5 * prob.counts.sum()
    worst = 0.0
    for r in range(R):
        diff = np.nonzero(o["trace_accept"][r] != g_acc[r])[0]
        k = diff[0] if diff.size else T
        s = min(k + 1, T)
        err = np.abs(o["trace_llprop"][r, :s] - g_ll[r, :s])
        worst = max(worst, float(err.max()))
        assert np.all(err <= bar), (r, err.max())
        if k < T:
            cur = _current_ll(ll0[r], o["trace_llprop"][r], o["trace_accept"][r], k)
            assert abs(o["trace_logu"][r, k] - (o["trace_llprop"][r, k] - cur)) <= 2.0 * bar, (r, k)
    print(f"  max |dlogL| {worst:.3e} (bar {bar:.3g})", flush=True)


def test_dirichlet_refusals():
    prob = synth.make_problem("c2")
    with pytest.raises(qst.QstError) as e:
        qst.Problem(2, prob.counts, param="dirichlet", alpha=0.0)
    assert e.value.status == qst.QST_ERR_INVALID
    with pytest.raises(qst.QstError):
        qst.Problem(2, prob.counts, param="dirichlet", alpha=1.0, path="dense")
