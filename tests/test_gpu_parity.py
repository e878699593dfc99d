"""GPU (HIP, through the C ABI) against the FP64 CPU oracle on identical
seeded inputs and identical Philox streams.

Bars: per-step log L of every traced chain within 1e-10 relative; identical
accept decisions except from the first step where |log u - dlogL| < 1e-8 on
either side (the comparison of that chain stops there); final states and the
pooled mean (Eq. (BME2)) to rounding; log L of given density matrices within
1e-12 relative.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2501_17334_amd import qst, synth
from tests.gpu_util import first_near_step, gpu_run, oracle_run

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _problem_for(Q):
    return {1: synth.make_problem("c1"), 2: synth.make_problem("c2"), 3: synth.make_problem("w_3"),
            4: synth.make_problem("c3"), 5: synth.make_problem("c4"),
            6: next(p for p in synth.mixed_batch(64) if p.n_qubits == 6)}[Q]


@pytest.mark.parametrize("Q", [1, 2, 3, 4, 5, 6])
def test_loglik_of_given_states(Q):
    print(f"[loglik] Q={Q}", flush=True)
    prob = _problem_for(Q)
    D = 2 ** Q
    rng = np.random.default_rng(1000 + Q)
    n = 37 if Q < 6 else 5
    rhos = np.stack([synth.random_density_matrix(D, rng, rank=int(rng.integers(1, D + 1))) for _ in range(n)])
    want = np.array([O.loglik(Q, prob.counts, O.probs(Q, r)) for r in rhos])
    P = qst.Problem(Q, prob.counts)
    dev = torch.from_numpy(np.ascontiguousarray(np.stack([rhos.real, rhos.imag], -1))).cuda()
    out = torch.zeros(n, dtype=torch.float64, device="cuda")
    P.loglik(dev, out)
    got = out.cpu().numpy()
    assert np.all(np.abs(got - want) <= 1e-12 * np.abs(want)), np.max(np.abs(got - want) / np.abs(want))


def test_loglik_special_values():
    Q, D = 3, 8
    pure0 = np.zeros((1, D, D), dtype=complex)
    pure0[0, 0, 0] = 1.0
    zero = np.zeros((27, 8), dtype=np.int64)
    hit = zero.copy()
    hit[26, 1] = 3   # all-Z setting, outcome 001: probability 0 for |000>
    for counts, want in ((zero, 0.0), (hit, -np.inf)):
        P = qst.Problem(Q, counts)
        dev = torch.from_numpy(np.ascontiguousarray(np.stack([pure0.real, pure0.imag], -1))).cuda()
        out = torch.zeros(1, dtype=torch.float64, device="cuda")
        P.loglik(dev, out)
        assert out.item() == want
        assert O.loglik(Q, counts, O.probs(Q, pure0[0])) == want


def _compare_lockstep(Q, counts, R, T, seed, beta0, adapt_every, trace, thin=1, burn_in=0):
    print(f"[lockstep] Q={Q} R={R} T={T} seed={seed}", flush=True)
    g = gpu_run(Q, counts, n_chains=R, n_steps=T, seed=seed, beta0=beta0, adapt_every=adapt_every,
                trace=trace, thin=thin, burn_in=burn_in)
    ch, o = oracle_run(Q, counts, n_chains=R, n_steps=T, seed=seed, beta0=beta0, adapt_every=adapt_every,
                       trace=trace, thin=thin, burn_in=burn_in)
    stop = first_near_step(o["trace_llprop"], g["trace_llprop"], o["trace_logu"], o["ll0"], o["trace_accept"])
    n_cmp = 0
    for r in range(trace):
        s = stop[r]
        a, b = o["trace_llprop"][r, :s], g["trace_llprop"][r, :s]
        fin = np.isfinite(a)
        assert np.array_equal(fin, np.isfinite(b))
        assert np.all(np.abs(a[fin] - b[fin]) <= 1e-10 * np.abs(a[fin])), (r, np.max(np.abs(a - b)))
        # log u of the same uniform: the two logarithms agree to a few ulp of max(1, |log u|)
        lu_o, lu_g = o["trace_logu"][r, :s], g["trace_logu"][r, :s]
        assert np.all(np.abs(lu_o - lu_g) <= 2e-15 * np.maximum(1.0, np.abs(lu_o)))
        assert np.array_equal(o["trace_accept"][r, :s], g["trace_accept"][r, :s])
        n_cmp += s
    x, ll, beta, nst = g["problem"].state()
    clean = stop == T
    assert np.array_equal(nst, ch.n_stored)
    if clean.all():
        assert np.allclose(x, ch.x, rtol=1e-9, atol=1e-9)
        assert np.allclose(ll, ch.ll, rtol=1e-10, atol=0)
        assert np.array_equal(beta, ch.beta)
        gp = g["problem"].pool()
        op = ch.pool()
        assert gp["n_samples"] == op["n_samples"]
        err = np.sqrt(np.sum(np.abs(gp["mean"] - op["mean"]) ** 2))
        assert err <= 1e-11, err
    return g, ch, n_cmp


def test_c1_full_trace():
    p = synth.make_problem("c1")
    g, ch, n = _compare_lockstep(1, p.counts, 64, 2000, p.seed, 0.1, 500, trace=64)
    assert n > 0.99 * 64 * 2000


def test_q2_lockstep():
    p = synth.make_problem("c2")
    _compare_lockstep(2, p.counts, 256, 600, p.seed, 0.05, 100, trace=64, thin=3, burn_in=100)


def test_q3_lockstep_ragged_tile():
    p = synth.make_problem("w_3")
    _compare_lockstep(3, p.counts, 37, 300, 5, 0.05, 50, trace=37)


def test_q4_lockstep():
    p = synth.make_problem("c3")
    _compare_lockstep(4, p.counts, 64, 120, p.seed, 0.02, 40, trace=64)


def test_q5_lockstep():
    p = synth.make_problem("c4")
    _compare_lockstep(5, p.counts, 6, 12, p.seed, 0.01, 4, trace=6)


def test_q6_lockstep():
    p = _problem_for(6)
    _compare_lockstep(6, p.counts, 3, 3, p.seed, 0.01, 0, trace=3)


@pytest.mark.parametrize("Q", [1, 2, 3, 4, 5, 6])
def test_every_compiled_launch_shape_matches_oracle(Q):
    """Each compiled (team, workgroup) of a qubit count, not only the tuned
    one, in lockstep with the oracle (short runs; chain counts that leave a
    ragged last workgroup)."""
    p = _problem_for(Q)
    R, T = {1: (19, 40), 2: (13, 30), 3: (7, 20), 4: (5, 8), 5: (3, 4), 6: (2, 2)}[Q]
    saved = qst.get_launch_shape(Q)
    try:
        for shape in qst.list_launch_shapes(Q):
            print(f"[shape] Q={Q} team={shape[0]} workgroup={shape[1]}", flush=True)
            qst.set_launch_shape(Q, *shape)
            _compare_lockstep(Q, p.counts, R, T, p.seed + 3, 0.02, 0, trace=R)
    finally:
        qst.set_launch_shape(Q, *saved)


@pytest.mark.parametrize("Q", [2, 4])
def test_independence_proposals_at_beta_one(Q):
    """beta = 1, the degenerate end of pCN: y' = eta, a fresh prior draw that
    ignores the current state (adaptation off, so beta stays 1)."""
    p = _problem_for(Q)
    R, T = {2: (32, 200), 4: (8, 30)}[Q]
    g, ch, n = _compare_lockstep(Q, p.counts, R, T, p.seed + 11, 1.0, 0, trace=R)
    assert np.all(g["problem"].state()[2] == 1.0)


def test_runs_that_store_no_sample():
    """burn-in or thinning that excludes every step: no chain stores a sample
    and pooling is refused (QST_ERR_STATE); one more step stores one."""
    p = synth.make_problem("c2")
    for kw in (dict(n_steps=30, burn_in=30), dict(n_steps=30, thin=31), dict(n_steps=30, thin=7, burn_in=28)):
        P = qst.Problem(2, p.counts)
        P.run(qst.RunConfig(n_chains=16, seed=3, beta0=0.05, **kw))
        assert np.all(P.state()[3] == 0), kw
        with pytest.raises(qst.QstError) as e:
            P.pool()
        assert e.value.status == qst.QST_ERR_STATE and "no stored samples" in str(e.value)
    P = qst.Problem(2, p.counts)
    P.run(qst.RunConfig(n_chains=16, n_steps=31, seed=3, beta0=0.05, burn_in=30))
    assert np.all(P.state()[3] == 1) and P.pool()["n_samples"] == 16


def test_resume_is_bitwise():
    p = synth.make_problem("c2")
    kw = dict(n_chains=64, seed=9, beta0=0.05, adapt_every=50, thin=2, burn_in=20)
    a = gpu_run(2, p.counts, n_steps=300, **kw)
    b = gpu_run(2, p.counts, n_steps=170, **kw)
    gpu_run(2, p.counts, n_steps=130, problem=b["problem"], resume=True, **kw)
    xa, lla, ba, na = a["problem"].state()
    xb, llb, bb, nb = b["problem"].state()
    assert np.array_equal(xa, xb) and np.array_equal(lla, llb) and np.array_equal(ba, bb)
    pa, pb = a["problem"].pool(), b["problem"].pool()
    assert np.array_equal(pa["mean"], pb["mean"]) and pa["n_samples"] == pb["n_samples"]


def test_rerun_is_deterministic():
    p = synth.make_problem("c3")
    kw = dict(n_chains=130, n_steps=20, seed=4, beta0=0.02, adapt_every=0)
    a = gpu_run(4, p.counts, **kw)["problem"]
    b = gpu_run(4, p.counts, **kw)["problem"]
    assert np.array_equal(a.state()[0], b.state()[0])
    assert np.array_equal(a.pool()["mean"], b.pool()["mean"])


def test_zero_counts_prior():
    Q, D = 3, 8
    counts = np.zeros((27, 8), dtype=np.int64)
    g = gpu_run(Q, counts, n_chains=4096, n_steps=400, seed=2, beta0=0.5, adapt_every=100)
    st = g["stats"]
    assert st["accepted"] == st["proposed"] == 4096 * 400
    x, ll, beta, nst = g["problem"].state()
    assert np.all(ll == 0.0)
    b = 0.5
    for _ in range(4):
        b = min(b * 1.1, 1.0)
    assert np.all(beta == b)
    pool = g["problem"].pool()
    se = np.sqrt(pool["se_re"] ** 2 + pool["se_im"] ** 2) + 1e-15
    assert np.all(np.abs(pool["mean"] - np.eye(D) / D) < 5 * se)
    xs = x.reshape(-1)
    assert abs(xs.mean()) < 5 / np.sqrt(xs.size) and abs(xs.var() - 1) < 5 * np.sqrt(2 / xs.size)


def test_init_only_matches_oracle():
    p = synth.make_problem("c3")
    g = gpu_run(4, p.counts, n_chains=5, n_steps=0, seed=3, beta0=0.1)
    x, ll, beta, nst = g["problem"].state()
    ch = O.Chains(4, p.counts, O.RunParams(n_chains=5, n_steps=0, seed=3))
    assert np.allclose(x, ch.x, rtol=1e-14, atol=1e-15)
    assert np.allclose(ll, ch.ll, rtol=1e-12, atol=0)
    with pytest.raises(qst.QstError) as e:
        g["problem"].pool()
    assert e.value.status == qst.QST_ERR_STATE


def test_records_match_oracle():
    p = synth.make_problem("c1")
    kw = dict(n_chains=6, n_steps=100, seed=8, beta0=0.2, adapt_every=0, record_every=5, record_chains=4)
    g = gpu_run(1, p.counts, **kw)
    ch, o = oracle_run(1, p.counts, **kw)
    assert np.allclose(g["records"].reshape(4, 20, 4), o["records"].reshape(4, 20, 4), rtol=0, atol=1e-13)


def test_invalid_run_arguments():
    p = synth.make_problem("c1")
    P = qst.Problem(1, p.counts)
    for bad in (dict(beta0=0.0), dict(beta0=1.5), dict(thin=0), dict(n_chains=0)):
        kw = dict(n_chains=4, n_steps=10, seed=1, beta0=0.1)
        kw.update(bad)
        with pytest.raises(qst.QstError) as e:
            P.run(qst.RunConfig(**kw))
        assert e.value.status == qst.QST_ERR_INVALID
    with pytest.raises(qst.QstError) as e:
        P.run(qst.RunConfig(n_chains=4, n_steps=10, seed=1, resume=True))
    assert e.value.status == qst.QST_ERR_STATE


def test_acf_matches_oracle_diagnostics():
    from oracle import diagnostics as G
    p = synth.make_problem("c2")
    g = gpu_run(2, p.counts, n_chains=12, n_steps=3000, seed=3, beta0=0.05, adapt_every=100,
                record_every=2, record_chains=10)
    rec = g["records"]
    want = G.acf(rec, l_max=60)
    got = qst.acf(torch.from_numpy(rec).cuda(), l_max=60)
    assert np.allclose(got, want, rtol=0, atol=1e-12)
    assert got[0] == 1.0
