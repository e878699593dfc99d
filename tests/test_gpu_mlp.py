"""The surrogate MLP's GPU forward/backward/Adam kernels against the FP64
CPU reference (oracle/mlp_ref.py).

Tight check: the reference rounds to BF16 exactly where the kernels store
BF16 (inputs, weights in the products, h1, h2, the back-propagated row
gradients), so the remaining difference is FP32 accumulation (and the rare
BF16 rounding flip it causes): relative norm error <= 2e-3 per parameter
block.  Loose check against the plain FP64 network: <= 5e-2.  Adam: the first
step moves every parameter by -lr * g / (|g| + eps).
"""
import numpy as np
import pytest
import torch

from oracle import mlp_ref as M
from paper_2501_17334_amd import qst

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _case(d=96, h1=64, h2=64, n=128, seed=0):
    rng = np.random.default_rng(seed)
    p = M.init_params(d, h1, h2, rng)
    p.b1 = rng.normal(0, 0.1, h1)
    p.b2 = rng.normal(0, 0.1, h2)
    p.b3 = 0.2
    X = rng.standard_normal((n, d))
    y = rng.standard_normal(n) * 0.5
    # the GPU keeps FP32 master weights: start both sides from the same FP32 values
    flat32 = p.flat().astype(np.float32)
    return p, X, y, flat32


def _unflat(flat, d, h1, h2):
    o = 0
    out = []
    for shape in [(h1, d), (h1,), (h2, h1), (h2,), (h2,), ()]:
        k = int(np.prod(shape)) if shape else 1
        out.append(flat[o:o + k].reshape(shape).astype(np.float64) if shape else float(flat[o]))
        o += k
    return M.Params(*out)


def _blocks(flat, d, h1, h2):
    p = _unflat(flat, d, h1, h2)
    return {"W1": p.W1, "b1": p.b1, "W2": p.W2, "b2": p.b2, "w3": p.w3, "b3": np.array([p.b3])}


@pytest.mark.parametrize("d,h1,h2,n", [(96, 64, 64, 128), (2080, 512, 512, 256), (64, 96, 32, 96)])
def test_gradients_match_reference(d, h1, h2, n):
    p, X, y, flat32 = _case(d, h1, h2, n)
    net = qst.Mlp(d, h1, h2)
    net.set_params(flat32)
    xd = torch.from_numpy(X).cuda()
    yd = torch.from_numpy(y).cuda()
    g_gpu, loss_gpu = net.gradients(xd, yd)
    p32 = _unflat(flat32, d, h1, h2)
    y32 = y.astype(np.float32).astype(np.float64)
    loss_e, g_e = M.loss_and_grads(p32, X, y32, bf16_emulation=True)
    loss_f, g_f = M.loss_and_grads(p32, X, y32, bf16_emulation=False)
    assert abs(loss_gpu - loss_e) <= 1e-4 * abs(loss_e)
    got = _blocks(g_gpu, d, h1, h2)
    for name, ref_e, ref_f in zip(["W1", "b1", "W2", "b2", "w3", "b3"],
                                  [g_e.W1, g_e.b1, g_e.W2, g_e.b2, g_e.w3, np.array([g_e.b3])],
                                  [g_f.W1, g_f.b1, g_f.W2, g_f.b2, g_f.w3, np.array([g_f.b3])]):
        e_tight = np.linalg.norm(got[name] - ref_e) / np.linalg.norm(ref_e)
        e_loose = np.linalg.norm(got[name] - ref_f) / np.linalg.norm(ref_f)
        print(f"  {name}: vs BF16-emulated FP64 {e_tight:.2e}, vs FP64 {e_loose:.2e}", flush=True)
        assert e_tight <= 2e-3, name
        assert e_loose <= 5e-2, name


def test_predict_matches_reference():
    d, h1, h2, n = 2080, 512, 512, 64
    p, X, y, flat32 = _case(d, h1, h2, n, seed=4)
    net = qst.Mlp(d, h1, h2)
    net.set_params(flat32, out_scale=3.0, out_shift=-7.0)
    s = net.predict(torch.from_numpy(X).cuda()).cpu().numpy().astype(np.float64)
    s_ref, _ = M.forward(_unflat(flat32, d, h1, h2), X, bf16_emulation=True)
    want = 3.0 * s_ref - 7.0
    assert np.max(np.abs(s - want)) <= 2e-3 * np.max(np.abs(want))


def test_adam_first_step():
    d, h1, h2, n = 96, 64, 64, 128
    p, X, y, flat32 = _case(d, h1, h2, n, seed=2)
    net = qst.Mlp(d, h1, h2)
    net.set_params(flat32)
    xd = torch.from_numpy(X).cuda()
    yd = torch.from_numpy(y).cuda()
    g, _ = net.gradients(xd, yd)
    lr = 1e-3
    net.train_step(xd.to(torch.bfloat16).contiguous(), yd.to(torch.float32).contiguous(), lr)
    new = net.get_params()
    want = flat32 - lr * g / (np.abs(g) + 1e-8)
    assert np.allclose(new, want, rtol=1e-5, atol=1e-7)


def test_training_lowers_loss():
    rng = np.random.default_rng(9)
    d, h1, h2, n = 96, 64, 64, 512
    X = rng.standard_normal((n, d))
    y = np.tanh(X[:, :4].sum(axis=1)) + 0.1 * X[:, 5]
    p = M.init_params(d, h1, h2, rng)
    net = qst.Mlp(d, h1, h2)
    net.set_params(p.flat().astype(np.float32))
    xb = torch.from_numpy(X).cuda().to(torch.bfloat16).contiguous()
    yf = torch.from_numpy(y).cuda().to(torch.float32).contiguous()
    l0 = net.train_step(xb, yf, 2e-3, want_loss=True)
    for _ in range(300):
        l = net.train_step(xb, yf, 2e-3, want_loss=True)
    assert l < 0.2 * l0
