"""Pins of the oracle's rho(x) = sum_j w_j z_j z_j^dag / |z_j|^2.

Invariants that any density matrix satisfies (Eq. (rho) and the text around
it: Hermitian, positive semidefinite, unit trace), special inputs with a
closed-form answer, and the prior moments in closed form:
E[rho] = I/D and E[Tr rho^2] = (2 D a + D - a) / (D (D a + 1)) for Dirichlet
concentration a = 1/2 (from the Dirichlet moments and E|<z_j|z_k>|^2 = 1/D
for independent Haar vectors).
"""
import numpy as np
import pytest

from oracle import oracle as O


def x_from(Z, v):
    """Pack a complex D x D matrix Z (columns z_j) and weights v into x."""
    D = Z.shape[0]
    return np.concatenate([Z.real.T.reshape(-1), Z.imag.T.reshape(-1), np.asarray(v, float)])


@pytest.mark.parametrize("Q", [1, 2, 3, 4, 5])
def test_rho_invariants(Q):
    D, _, d = O.dims(Q)
    rng = np.random.default_rng(Q)
    for _ in range(5 if Q < 5 else 2):
        x = rng.standard_normal(d)
        r = O.rho_of_x(Q, x)
        assert np.array_equal(r, r.conj().T)                # Hermitian, exactly
        assert abs(np.trace(r) - 1.0) < 1e-14
        assert np.linalg.eigvalsh(r).min() > -1e-14
        assert np.linalg.matrix_rank(r, tol=1e-12) <= D


@pytest.mark.parametrize("Q", [1, 2, 3])
def test_rho_single_weight_gives_that_column(Q):
    # only v_j != 0: rho is the pure state of column j, whatever the others are
    D, _, d = O.dims(Q)
    rng = np.random.default_rng(10 + Q)
    Z = rng.standard_normal((D, D)) + 1j * rng.standard_normal((D, D))
    for j in range(D):
        v = np.zeros(D)
        v[j] = -1.7
        r = O.rho_of_x(Q, x_from(Z, v))
        z = Z[:, j] / np.linalg.norm(Z[:, j])
        assert np.allclose(r, np.outer(z, z.conj()), atol=1e-15, rtol=0)
        assert abs(np.trace(r @ r) - 1.0) < 1e-13


@pytest.mark.parametrize("Q", [1, 2, 3])
def test_rho_basis_columns_give_diagonal_weights(Q):
    D, _, d = O.dims(Q)
    rng = np.random.default_rng(20 + Q)
    scales = rng.uniform(0.5, 2.0, D) * np.exp(2j * np.pi * rng.uniform(size=D))
    Z = np.diag(scales)
    v = rng.standard_normal(D)
    r = O.rho_of_x(Q, x_from(Z, v))
    assert np.allclose(r, np.diag(v ** 2 / np.sum(v ** 2)), atol=1e-15, rtol=0)


def test_rho_invariances():
    # rho is unchanged by z_j -> c z_j (c complex) and v_j -> -v_j
    Q, rng = 2, np.random.default_rng(3)
    D, _, d = O.dims(Q)
    Z = rng.standard_normal((D, D)) + 1j * rng.standard_normal((D, D))
    v = rng.standard_normal(D)
    c = rng.uniform(0.3, 3, D) * np.exp(1j * rng.uniform(0, 6, D))
    r1 = O.rho_of_x(Q, x_from(Z, v))
    r2 = O.rho_of_x(Q, x_from(Z * c[None, :], -v))
    assert np.allclose(r1, r2, atol=1e-14, rtol=0)


def test_pack_roundtrip():
    rng = np.random.default_rng(0)
    for Q in (1, 2, 3):
        r = O.rho_of_x(Q, rng.standard_normal(O.dims(Q)[2]))
        P = O.pack(r)
        D = r.shape[0]
        for a in range(D):
            for b in range(D):
                assert P[a, b] == (r[a, b].real if a <= b else r[b, a].imag)
        assert np.array_equal(O.unpack(P), r)


@pytest.mark.parametrize("Q", [1, 2])
def test_prior_moments(Q):
    D, _, d = O.dims(Q)
    n = 200_000
    xs = np.random.default_rng(100 + Q).standard_normal((n, d))
    _, rp = O.eval_batch(Q, np.zeros(3 ** Q * D, dtype=np.int64), xs, want_rho=True)
    rhos = np.array([O.unpack(P) for P in rp[:20000]])
    mean = rhos.mean(axis=0)
    se = rhos.std(axis=0) / np.sqrt(rhos.shape[0])
    assert np.all(np.abs(mean - np.eye(D) / D) < 5 * se + 1e-12)
    # purity from packed entries: diagonal once, off-diagonal re/im twice
    w = np.full((D, D), 2.0)
    np.fill_diagonal(w, 1.0)
    purity = np.sum(w * rp ** 2, axis=(1, 2))
    a = 0.5
    want = (2 * D * a + D - a) / (D * (D * a + 1))
    assert abs(purity.mean() - want) < 5 * purity.std() / np.sqrt(n)
