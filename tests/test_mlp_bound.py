"""The a-priori surrogate error bound (tests/mlp_bound.py) against a CPU
emulation of the GPU's arithmetic: BF16 inputs, weights and activations,
FP32 products, sums and GELU.  Both bounds (deterministic and
probabilistic) must cover the emulation's deviation from FP64 on every row,
for inputs of several scales."""
import numpy as np
import pytest
from scipy.special import erf

from oracle import mlp_ref as M
from tests.mlp_bound import surrogate_error_bound


def _emulate_gpu(p, X, scale, shift):
    f = np.float32
    Xb = M.bf16_round(X).astype(f)
    W1 = M.bf16_round(p.W1).astype(f)
    W2 = M.bf16_round(p.W2).astype(f)
    g = lambda t: (f(0.5) * t * (f(1.0) + erf(t * f(0.70710678118654752)).astype(f))).astype(f)
    z1 = (Xb @ W1.T).astype(f) + p.b1.astype(f)
    h1 = M.bf16_round(g(z1)).astype(f)
    z2 = (h1 @ W2.T).astype(f) + p.b2.astype(f)
    h2 = M.bf16_round(g(z2)).astype(f)
    s = (h2 @ p.w3.astype(f)).astype(f) + f(p.b3)
    return (f(scale) * s + f(shift)).astype(np.float64), W1.astype(np.float64), W2.astype(np.float64)


@pytest.mark.parametrize("d,h,xscale", [(10, 32, 1.0), (36, 64, 0.3), (528, 128, 1.0), (2080, 64, 2.0)])
def test_bound_covers_fp32_bf16_emulation(d, h, xscale):
    rng = np.random.default_rng(d + h)
    p = M.init_params(d, h, h, rng)
    p.b1 = rng.normal(0, 0.3, h).astype(np.float32).astype(np.float64)
    p.b2 = rng.normal(0, 0.3, h).astype(np.float32).astype(np.float64)
    p.w3 = p.w3.astype(np.float32).astype(np.float64)
    p.b3 = float(np.float32(0.2))
    X = rng.standard_normal((200, d)) * xscale
    scale, shift = 4.0, -2.0
    s_emul, W1b, W2b = _emulate_gpu(p, X, scale, shift)
    q = M.Params(W1b, p.b1, W2b, p.b2, p.w3, p.b3)
    s64 = scale * M.forward(q, X)[0] + shift
    err = np.abs(s_emul - s64)
    worst = surrogate_error_bound(W1b, p.b1, W2b, p.b2, p.w3, p.b3, scale, shift, X, worst=True)
    prob = surrogate_error_bound(W1b, p.b1, W2b, p.b2, p.w3, p.b3, scale, shift, X)
    assert np.all(err <= worst), np.max(err / worst)
    assert np.all(err <= prob), np.max(err / prob)
    assert np.all(prob <= worst * (1 + 1e-12))
    # the probabilistic bound is a usable band: within 100x of the typical error
    assert np.median(prob) < 100 * np.median(err), (np.median(prob), np.median(err))
