"""FP64 reference of the MLP surrogate and its training step (TEST
INFRASTRUCTURE ONLY).

Network: h1 = gelu(W1 x + b1), h2 = gelu(W2 h1 + b2), s = w3 . h2 + b3 with
the exact GELU t (1 + erf(t / sqrt 2)) / 2 (Hendrycks & Gimpel 2016).  Loss:
mean squared error over a minibatch, L = mean_i (s_i - y_i)^2.  Optimiser:
Adam (Kingma & Ba 2015) with bias correction.

``bf16_emulation=True`` rounds to BF16 (round to nearest even) exactly where
the GPU kernels store BF16 values (the inputs, the weights used by the
products, the activations h1, h2 and the back-propagated row gradients), so
the remaining GPU/CPU difference is the FP32 accumulation order alone.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
from scipy.special import erf


def bf16_round(a):
    """Round float64 values to the nearest BF16 value (ties to even), via float32."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def gelu(t):
    return 0.5 * t * (1.0 + erf(t / np.sqrt(2.0)))


def gelu_grad(t):
    return 0.5 * (1.0 + erf(t / np.sqrt(2.0))) + t * np.exp(-0.5 * t * t) / np.sqrt(2.0 * np.pi)


@dataclass
class Params:
    W1: np.ndarray
    b1: np.ndarray
    W2: np.ndarray
    b2: np.ndarray
    w3: np.ndarray
    b3: float

    def copy(self):
        return Params(self.W1.copy(), self.b1.copy(), self.W2.copy(), self.b2.copy(), self.w3.copy(), float(self.b3))

    def flat(self):
        return np.concatenate([self.W1.ravel(), self.b1, self.W2.ravel(), self.b2, self.w3, [self.b3]])


def forward(p: Params, X, bf16_emulation=False):
    """Returns s [n] and the cache for backward."""
    r = bf16_round if bf16_emulation else (lambda a: a)
    Xr = r(X)
    z1 = Xr @ r(p.W1).T + p.b1
    h1 = r(gelu(z1))
    z2 = h1 @ r(p.W2).T + p.b2
    h2 = r(gelu(z2))
    s = h2 @ p.w3 + p.b3
    return s, (Xr, z1, h1, z2, h2)


def loss_and_grads(p: Params, X, y, bf16_emulation=False):
    """MSE loss and its gradients with respect to every parameter."""
    r = bf16_round if bf16_emulation else (lambda a: a)
    n = X.shape[0]
    s, (Xr, z1, h1, z2, h2) = forward(p, X, bf16_emulation)
    d = s - y
    loss = float(np.mean(d * d))
    ds = 2.0 * d / n                       # dL/ds
    gw3 = h2.T @ ds
    gb3 = float(np.sum(ds))
    dh2 = np.outer(ds, p.w3)
    dz2 = r(dh2 * gelu_grad(z2))
    gW2 = dz2.T @ h1
    gb2 = dz2.sum(axis=0)
    dh1 = dz2 @ r(p.W2)
    dz1 = r(dh1 * gelu_grad(z1))
    gW1 = dz1.T @ Xr
    gb1 = dz1.sum(axis=0)
    return loss, Params(gW1, gb1, gW2, gb2, gw3, gb3)


def finite_difference(p: Params, X, y, which, idx, h=1e-6):
    """Central difference of the FP64 loss in one parameter entry."""
    def loss_at(delta):
        q = p.copy()
        arr = getattr(q, which)
        if which == "b3":
            q.b3 = q.b3 + delta
        else:
            arr.flat[idx] += delta
        return loss_and_grads(q, X, y)[0]
    return (loss_at(h) - loss_at(-h)) / (2 * h)


@dataclass
class AdamState:
    m: np.ndarray
    v: np.ndarray
    t: int = 0


def adam_step(theta, grad, st: AdamState, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update of the flat parameter vector theta (in place)."""
    st.t += 1
    st.m = beta1 * st.m + (1 - beta1) * grad
    st.v = beta2 * st.v + (1 - beta2) * grad * grad
    mhat = st.m / (1 - beta1 ** st.t)
    vhat = st.v / (1 - beta2 ** st.t)
    theta -= lr * mhat / (np.sqrt(vhat) + eps)
    return theta


def init_params(d_in, h1, h2, rng):
    """He-style uniform initialisation (the GPU uses the same recipe from its own generator)."""
    def uni(shape, fan_in):
        bound = np.sqrt(6.0 / fan_in) / 2
        return rng.uniform(-bound, bound, shape)
    return Params(uni((h1, d_in), d_in), np.zeros(h1), uni((h2, h1), h1), np.zeros(h2), uni((h2,), h2), 0.0)
