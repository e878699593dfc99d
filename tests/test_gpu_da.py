"""Delayed acceptance (Christen & Fox 2005) with the MLP surrogate.

* A constant surrogate passes every proposal at stage 1 (log u1 < 0), so
  stage 2 is the plain Metropolis-Hastings test: the run must equal plain
  pCN bit for bit (same streams, same team shape).
* Against the oracle's delayed-acceptance rule (FP64 surrogate from the same
  BF16-rounded weights): the GPU surrogate stays within the a-priori error
  bound of its arithmetic (tests/mlp_bound.py) on random states, and
  decisions are identical except where a stage margin lies within that
  bound at the two states involved.
* Both stages keep the posterior exact: the pooled mean of a delayed-
  acceptance run agrees with plain pCN within the Monte Carlo error.
"""
import numpy as np
import pytest
import torch

from oracle import mlp_ref as M
from oracle import oracle as O
from paper_2501_17334_amd import qst, synth
from tests.gpu_util import gpu_run
from tests.mlp_bound import surrogate_error_bound

pytestmark = pytest.mark.gpu

DA_SHAPE = {1: (8, 64), 2: (16, 64), 3: (32, 64), 4: (64, 256), 5: (256, 256), 6: (512, 512)}


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(autouse=True)
def _restore_launch_shapes():
    # the tests run plain chains with the delayed-acceptance kernels' team
    # sizes; later tests get the tuned shapes back
    saved = {q: qst.get_launch_shape(q) for q in range(1, 7)}
    yield
    for q, sh in saved.items():
        qst.set_launch_shape(q, *sh)


def _problem(Q):
    return {1: synth.make_problem("c1"), 2: synth.make_problem("c2"), 3: synth.make_problem("w_3"),
            4: synth.make_problem("c3"), 5: synth.make_problem("c4"),
            6: next(p for p in synth.mixed_batch(64) if p.n_qubits == 6)}[Q]


def _run(P, cfg, surrogate=None, trace=0):
    tr = None
    if trace:
        tr = dict(chains=trace,
                  llprop=torch.full((trace, cfg.n_steps), float("nan"), dtype=torch.float64, device="cuda"),
                  logu=torch.zeros((trace, cfg.n_steps), dtype=torch.float64, device="cuda"),
                  accept=torch.zeros((trace, cfg.n_steps), dtype=torch.int8, device="cuda"))
    st = P.run(cfg, trace=tr, surrogate=surrogate)
    torch.cuda.synchronize()
    out = {"stats": st}
    if tr:
        out.update({k: tr[k].cpu().numpy() for k in ("llprop", "logu", "accept")})
    return out


@pytest.mark.parametrize("Q", [1, 2, 3, 4, 5, 6])
def test_constant_surrogate_equals_plain(Q):
    print(f"[da const] Q={Q}", flush=True)
    prob = _problem(Q)
    R, T = {1: (64, 300), 2: (48, 200), 3: (24, 100), 4: (16, 60), 5: (4, 8), 6: (2, 3)}[Q]
    qst.set_launch_shape(Q, *DA_SHAPE[Q])
    A = qst.Problem(Q, prob.counts)
    B = qst.Problem(Q, prob.counts)
    net = qst.Mlp(A.pair_width, 32, 32)
    net.set_params(np.zeros(net.n_params, dtype=np.float32), out_scale=1.0, out_shift=3.0)
    cfg = qst.RunConfig(n_chains=R, n_steps=T, seed=prob.seed, beta0=0.05 if Q < 4 else 0.01, adapt_every=25)
    a = _run(A, cfg, surrogate=net.surrogate(), trace=R)
    b = _run(B, cfg, trace=R)
    assert a["stats"]["stage1_passed"] == a["stats"]["proposed"] == R * T
    assert a["stats"]["accepted"] == b["stats"]["accepted"]
    assert np.array_equal(a["llprop"], b["llprop"])
    assert np.array_equal(a["accept"], b["accept"])
    xa, la, ba, na = A.state()
    xb, lb, bb, nb = B.state()
    assert np.array_equal(xa, xb) and np.array_equal(la, lb) and np.array_equal(ba, bb) and np.array_equal(na, nb)
    assert np.array_equal(A.pool()["mean"], B.pool()["mean"])


def _random_net(d, dp, h, rng, scale):
    p = M.init_params(dp, h, h, rng)
    p.W1[:, d:] = 0.0
    p.b1 = rng.normal(0, 0.2, h)
    p.b2 = rng.normal(0, 0.2, h)
    p.b3 = 0.1
    flat = p.flat().astype(np.float32)
    return p, flat


def _oracle_weights(flat, d, dp, h, scale, shift):
    o = 0
    def take(n):
        nonlocal o
        v = flat[o:o + n].astype(np.float64)
        o += n
        return v
    W1 = M.bf16_round(take(h * dp).reshape(h, dp))[:, :d]
    b1 = take(h)
    W2 = M.bf16_round(take(h * h).reshape(h, h))
    b2 = take(h)
    w3 = take(h)
    b3 = float(take(1)[0])
    return O.MlpWeights(np.ascontiguousarray(W1), b1, W2, b2, w3, b3, scale, shift)


def test_matches_oracle_delayed_acceptance():
    Q = 1
    prob = _problem(Q)
    R, T, h = 64, 400, 32
    qst.set_launch_shape(Q, *DA_SHAPE[Q])
    P = qst.Problem(Q, prob.counts)
    d, dp = P.d, P.pair_width
    rng = np.random.default_rng(5)
    _, flat = _random_net(d, dp, h, rng, 1.0)
    scale, shift, beta = 4.0, 0.0, 0.2
    net = qst.Mlp(dp, h, h)
    net.set_params(flat, out_scale=scale, out_shift=shift)
    cfg = qst.RunConfig(n_chains=R, n_steps=T, seed=prob.seed, beta0=beta, adapt_every=0)
    g = _run(P, cfg, surrogate=net.surrogate(), trace=R)
    w = _oracle_weights(flat, d, dp, h, scale, shift)
    ch = O.Chains(Q, prob.counts, O.RunParams(n_chains=R, n_steps=0, seed=prob.seed, beta0=beta, adapt_every=0,
                                              trace_chains=R, surrogate=w))
    o = ch.run(T)
    # the GPU surrogate (BF16 inputs, weights and activations, FP32 sums)
    # against the oracle's FP64 one, within the a-priori bound of its arithmetic
    bound = lambda X: surrogate_error_bound(w.W1, w.b1, w.W2, w.b2, w.w3, w.b3, scale, shift, X)
    xs = np.random.default_rng(8).standard_normal((512, d))
    xpad = np.zeros((512, dp))
    xpad[:, :d] = xs
    s_gpu = net.predict(torch.from_numpy(xpad).cuda()).cpu().numpy().astype(np.float64)
    s_cpu = np.array([O.mlp_forward(w, x) for x in xs])
    gap, bnd = np.abs(s_gpu - s_cpu), bound(xs)
    print(f"[da oracle] surrogate GPU-CPU max diff {gap.max():.3e}, a-priori bound max {bnd.max():.3e}",
          flush=True)
    assert np.all(gap <= bnd), np.max(gap / bnd)
    agree = 0
    a_beta = np.sqrt(1.0 - beta * beta)
    for r in range(R):
        ev_g = np.isfinite(g["llprop"][r])
        ev_o = np.isfinite(o["trace_llprop"][r])
        same = (ev_g == ev_o) & (g["accept"][r] == o["trace_accept"][r])
        k = T if same.all() else int(np.argmin(same))
        both = ev_g[:k] & ev_o[:k]
        a, b = o["trace_llprop"][r, :k][both], g["llprop"][r, :k][both]
        assert np.all(np.abs(a - b) <= 1e-10 * np.abs(a))
        agree += k
        if k < T:
            # replay the oracle chain to step k and check the decision margin
            one = O.Chains(Q, prob.counts, O.RunParams(n_chains=1, n_steps=0, seed=prob.seed, beta0=beta,
                                                       adapt_every=0, chain_offset=r, surrogate=w))
            if k:
                one.run(k)
            y = one.x[0]
            j = k + 1
            yp = a_beta * y + beta * O.normals(prob.seed, r, j, d)
            ds = O.mlp_forward(w, yp) - O.mlp_forward(w, y)
            band = float(np.sum(bound(np.stack([yp, y]))))   # |ds_gpu - ds_cpu| at most
            m1 = abs(np.log(O.da_uniform(prob.seed, r, j)) - ds)
            if ev_g[k] != ev_o[k]:
                assert m1 <= band, (r, k, m1, band)
            else:
                llp = O.loglik_of_x(Q, prob.counts, yp)
                m2 = abs(np.log(O.mh_uniform(prob.seed, r, j)) - ((llp - one.ll[0]) - ds))
                assert m2 <= band, (r, k, m2, band)
    print(f"[da oracle] steps in agreement before the first surrogate-margin flip: {agree} of {R * T}",
          flush=True)
    s = g["stats"]
    assert 0 < s["stage1_passed"] < s["proposed"]


def test_pooled_mean_matches_plain():
    Q = 1
    prob = _problem(Q)
    R, T, h = 2048, 3000, 32
    qst.set_launch_shape(Q, *DA_SHAPE[Q])
    P = qst.Problem(Q, prob.counts)
    rng = np.random.default_rng(6)
    _, flat = _random_net(P.d, P.pair_width, h, rng, 1.0)
    net = qst.Mlp(P.pair_width, h, h)
    net.set_params(flat, out_scale=2.0, out_shift=0.0)
    cfg = qst.RunConfig(n_chains=R, n_steps=T, seed=41, beta0=0.05, adapt_every=100, burn_in=1000)
    _run(P, cfg, surrogate=net.surrogate())
    pa = P.pool()
    B = qst.Problem(Q, prob.counts)
    _run(B, qst.RunConfig(n_chains=R, n_steps=T, seed=42, beta0=0.05, adapt_every=100, burn_in=1000))
    pb = B.pool()
    for part, se in (("real", "se_re"), ("imag", "se_im")):
        diff = np.abs(getattr(pa["mean"], part) - getattr(pb["mean"], part))
        tol = 5 * np.sqrt(pa[se] ** 2 + pb[se] ** 2) + 1e-12
        assert np.all(diff <= tol), (part, diff, tol)
