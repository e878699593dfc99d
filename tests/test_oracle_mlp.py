"""Pins of the FP64 MLP reference (surrogate of delayed acceptance).

Analytic gradients against central finite differences of the FP64 loss
(relative 1e-6 or better), the GELU derivative against finite differences,
BF16 rounding against known values, Adam's first steps against its closed
form (after one step every parameter moves by lr * sign(grad)).
"""
import numpy as np
import pytest

from oracle import mlp_ref as M


def _setup(seed=0, n=12, d=9, h1=7, h2=5):
    rng = np.random.default_rng(seed)
    p = M.init_params(d, h1, h2, rng)
    p.b1 = rng.normal(0, 0.1, h1)
    p.b2 = rng.normal(0, 0.1, h2)
    p.b3 = 0.3
    X = rng.standard_normal((n, d))
    y = rng.standard_normal(n)
    return p, X, y


@pytest.mark.parametrize("which", ["W1", "b1", "W2", "b2", "w3", "b3"])
def test_gradients_match_finite_differences(which):
    p, X, y = _setup()
    _, g = M.loss_and_grads(p, X, y)
    ga = getattr(g, which)
    rng = np.random.default_rng(1)
    size = 1 if which == "b3" else getattr(p, which).size
    for idx in rng.choice(size, size=min(6, size), replace=False):
        fd = M.finite_difference(p, X, y, which, int(idx))
        an = ga if which == "b3" else ga.flat[int(idx)]
        assert abs(fd - an) <= 1e-6 * max(1e-3, abs(an)) + 1e-9, (which, idx, fd, an)


def test_gelu_grad():
    t = np.linspace(-4, 4, 81)
    h = 1e-6
    fd = (M.gelu(t + h) - M.gelu(t - h)) / (2 * h)
    assert np.allclose(M.gelu_grad(t), fd, atol=1e-8)
    assert M.gelu(0.0) == 0.0
    assert abs(M.gelu(10.0) - 10.0) < 1e-12


def test_bf16_round():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -7, 1.0 + 3 * 2 ** -8, -2.5, 0.0, 3.14159])
    want = np.array([1.0, 1.0, 1.0 + 2 ** -7, 1.0 + 2 ** -6, -2.5, 0.0, 3.140625])
    assert np.array_equal(M.bf16_round(vals), want)


def test_adam_first_step_is_sign():
    theta = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -7.0, 1e-3])
    st = M.AdamState(np.zeros(3), np.zeros(3))
    M.adam_step(theta, g, st, lr=0.01, eps=0.0)
    assert np.allclose(theta, [0.99, -1.99, 0.49])


def test_training_reduces_loss():
    rng = np.random.default_rng(3)
    d = 6
    X = rng.standard_normal((256, d))
    y = np.sin(X[:, 0]) + 0.5 * X[:, 1] ** 2
    p = M.init_params(d, 16, 16, rng)
    theta = p.flat()
    st = M.AdamState(np.zeros_like(theta), np.zeros_like(theta))
    shapes = [(16, d), (16,), (16, 16), (16,), (16,), ()]

    def unflat(t):
        out, o = [], 0
        for s in shapes:
            n = int(np.prod(s)) if s else 1
            out.append(t[o:o + n].reshape(s) if s else float(t[o]))
            o += n
        return M.Params(*out)
    l0 = M.loss_and_grads(unflat(theta), X, y)[0]
    for _ in range(300):
        loss, g = M.loss_and_grads(unflat(theta), X, y)
        M.adam_step(theta, g.flat(), st, lr=1e-2)
    assert loss < 0.2 * l0
