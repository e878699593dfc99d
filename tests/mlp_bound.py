"""A-priori bounds on |s_gpu(x) - s_fp64(x)| for the library's surrogate
forward pass, derived from its arithmetic (not from a measured gap).

The GPU evaluates s = out_scale (w3 . h2 + b3) + out_shift with
h1 = bf16(gelu(W1 x + b1)), h2 = bf16(gelu(W2 h1 + b2)): the input x is
rounded to BF16 (through FP32: relative error at most 2^-8 + 2^-24), the
weights W1, W2 are BF16 (the FP64 side uses the same rounded values), the
layer products are BF16 x BF16 products (exact in FP32) summed in FP32 on
MFMA, the bias added in FP32, GELU evaluated in FP32 with erff, the last
layer a FP32 dot product of BF16 h2 with FP32 w3.  The FP64 side is the
exact-arithmetic network on unrounded x.

Local errors (Higham, "Accuracy and Stability of Numerical Algorithms",
ch. 3): a sum of n terms with every addition rounded to relative error u is
within gamma_n = n u / (1 - n u) of the sum of the absolute values of its
terms; u = 2^-23 is taken for the FP32 accumulations (twice the unit
roundoff, which also covers truncating adds).  The FP32 GELU
0.5 t (1 + erff(t / sqrt 2)) is within 4 u32 (|t| + |gelu(t)|) of gelu(t)
(erff to 2 ulp, four roundings), and rounding its value to BF16 adds 2^-8
relative.  Each local error travels to s through the network's Jacobian
(GELU is smooth, sup |gelu'| = gelu'(sqrt 2) < 1.1290, so second-order terms
are of relative size 2^-8 and are covered by a final factor 1.1).

worst=True adds every propagated error in absolute value: a deterministic
bound.  The default combines the errors of independent roundings (of the
inputs, and of the activations of one layer) by Hoeffding's inequality, as
in the probabilistic rounding-error analysis of Higham & Mary (SIAM J. Sci.
Comput. 41, 2019): a sum of independent zero-mean terms |e_i| <= b_i exceeds
lam * ||b||_2 with probability at most 2 exp(-lam^2 / 2), and an FP32 sum of
n terms is within lam sqrt(n) u sum|terms| under the same model.  lam = 7
gives at most 5e-11 per combined sum.
"""
import numpy as np
from scipy.special import erf

U_BF16 = 2.0 ** -8
U_F32 = 2.0 ** -24
U_ACC = 2.0 ** -23
GELU_LIP = 1.1290


def _gelu(t):
    return 0.5 * t * (1.0 + erf(t / np.sqrt(2.0)))


def _gelu_grad(t):
    return 0.5 * (1.0 + erf(t / np.sqrt(2.0))) + t * np.exp(-0.5 * t * t) / np.sqrt(2.0 * np.pi)


def surrogate_error_bound(W1, b1, W2, b2, w3, b3, out_scale, out_shift, X, worst=False, lam=7.0):
    """Per row of X [n, d] (FP64 inputs): a bound on the GPU surrogate's
    deviation from the FP64 network with the same (BF16-valued) weights."""
    X = np.atleast_2d(np.asarray(X, dtype=np.float64))
    n, d = X.shape
    W1 = np.asarray(W1, dtype=np.float64)[:, :d]
    W2 = np.asarray(W2, dtype=np.float64)
    w3 = np.asarray(w3, dtype=np.float64)
    h1n, h2n = W1.shape[0], W2.shape[0]
    ux = U_BF16 + U_F32
    z1 = X @ W1.T + b1
    h1 = _gelu(z1)
    z2 = h1 @ W2.T + b2
    h2 = _gelu(z2)
    s = h2 @ w3 + b3
    out = out_scale * s + out_shift
    # Jacobians of s
    g_z2 = _gelu_grad(z2) * w3                 # ds/dz2 [n, h2]
    g_h1 = g_z2 @ W2                           # ds/dh1 [n, h1]
    g_z1 = g_h1 * _gelu_grad(z1)               # ds/dz1 [n, h1]
    g_x = g_z1 @ W1                            # ds/dx  [n, d]
    # local error bounds
    bx = ux * np.abs(X)                                                    # input rounding
    abs1 = np.abs(X) @ np.abs(W1).T + np.abs(b1)
    abs2 = np.abs(h1) @ np.abs(W2).T + np.abs(b2)
    abs3 = np.abs(h2) @ np.abs(w3) + abs(b3)
    act1 = U_BF16 * np.abs(h1) + 4.0 * U_F32 * (np.abs(z1) + np.abs(h1))   # GELU + BF16 store
    act2 = U_BF16 * np.abs(h2) + 4.0 * U_F32 * (np.abs(z2) + np.abs(h2))
    if worst:
        g = lambda m: m * U_ACC / (1.0 - m * U_ACC)
        acc1, acc2, acc3 = g(d + 1) * abs1, g(h1n + 1) * abs2, g(2 * h2n + 1) * abs3
        es = (np.sum(np.abs(g_x) * bx, axis=1) + np.sum(np.abs(g_z1) * acc1, axis=1)
              + np.sum(np.abs(g_h1) * act1, axis=1) + np.sum(np.abs(g_z2) * acc2, axis=1)
              + np.abs(w3) @ act2.T + acc3)
        # the input rounding also scales the activations' own errors: first order covers it
    else:
        g = lambda m: lam * np.sqrt(m) * U_ACC
        acc1, acc2, acc3 = g(d + 1) * abs1, g(h1n + 1) * abs2, g(2 * h2n + 1) * abs3
        l2 = lambda a: np.sqrt(np.sum(a * a, axis=1))
        es = (lam * l2(g_x * bx) + lam * l2(g_z1 * acc1) + lam * l2(g_h1 * act1)
              + lam * l2(g_z2 * acc2) + lam * l2(w3 * act2) + acc3)
    eout = abs(out_scale) * es + U_F32 * (np.abs(out_scale * s) + np.abs(out)) + 1e-12 * (np.abs(out) + 1.0)
    if not worst:
        # few terms: the deterministic sum can be the smaller of the two
        eout = np.minimum(eout, surrogate_error_bound(W1, b1, W2, b2, w3, b3, out_scale, out_shift, X,
                                                      worst=True) / 1.1)
    return 1.1 * eout
