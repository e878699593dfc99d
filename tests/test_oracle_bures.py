"""Pins of the oracle's Algorithm 1 (the Bures draw), independent of its own
code:

* an independent QR (numpy / LAPACK) with the phase fix U = Q Lambda gives
  the same U and rho: U does not depend on the QR's sign convention, because
  Lambda makes the diagonal of R positive real;
* U is unitary and U^dag H is upper triangular with a positive real diagonal;
* special cases with a known U: an upper-triangular H with positive
  diagonal gives U = I (rho = G G^dag / Tr), a diagonal H gives U = diag of
  its phases;
* the distribution: rho is Bures-distributed, whose mean purity is
  (5D^2 + 1) / (2D(D^2 + 2)) (Sommers & Zyczkowski 2004; for D = 2 the Bures
  density on the Bloch ball is proportional to r^2 / sqrt(1 - r^2), so
  E[r^2] = 3/4 and E[Tr rho^2] = (1 + 3/4) / 2 = 7/8), and E[rho] = I / D.
  Dropping the (U + I) factor gives the Hilbert-Schmidt measure instead
  (mean purity 2D / (D^2 + 1)), which the same test rejects.
"""
import numpy as np
import pytest

from oracle import oracle as O


def _blocks(Q, x):
    D = 2 ** Q
    D2 = D * D
    G = (x[:D2] + 1j * x[D2:2 * D2]).reshape(D, D).T       # entry (i, j) at offset jD + i
    H = (x[2 * D2:3 * D2] + 1j * x[3 * D2:]).reshape(D, D).T
    return G, H


def _x_of(G, H):
    Gt, Ht = G.T.reshape(-1), H.T.reshape(-1)
    return np.concatenate([Gt.real, Gt.imag, Ht.real, Ht.imag])


def _numpy_bures(Q, x):
    D = 2 ** Q
    G, H = _blocks(Q, x)
    q, r = np.linalg.qr(H)
    lam = np.diag(r) / np.abs(np.diag(r))
    U = q * lam
    W = (U + np.eye(D)) @ G
    rho = W @ W.conj().T
    return U, rho / np.trace(rho).real


@pytest.mark.parametrize("Q", [1, 2, 3, 4])
def test_matches_an_independent_qr(Q):
    rng = np.random.default_rng(100 + Q)
    D = 2 ** Q
    for _ in range(20):
        x = rng.standard_normal(4 * D * D)
        U_ref, rho_ref = _numpy_bures(Q, x)
        assert np.abs(O.bures_unitary(Q, x) - U_ref).max() < 1e-12
        assert np.abs(O.rho_of_x(Q, x, "bures") - rho_ref).max() < 1e-13


@pytest.mark.parametrize("Q", [1, 2, 3, 4])
def test_unitary_with_positive_triangular_factor(Q):
    rng = np.random.default_rng(200 + Q)
    D = 2 ** Q
    for _ in range(10):
        x = rng.standard_normal(4 * D * D)
        _, H = _blocks(Q, x)
        U = O.bures_unitary(Q, x)
        assert np.abs(U.conj().T @ U - np.eye(D)).max() < 1e-13
        R = U.conj().T @ H
        assert np.abs(np.tril(R, -1)).max() < 1e-12 * np.abs(R).max()
        assert np.all(np.abs(np.diag(R).imag) < 1e-12) and np.all(np.diag(R).real > 0)
        rho = O.rho_of_x(Q, x, "bures")
        assert np.abs(rho - rho.conj().T).max() < 1e-15
        assert abs(np.trace(rho).real - 1.0) < 1e-14
        assert np.linalg.eigvalsh(rho).min() > -1e-14


@pytest.mark.parametrize("Q", [1, 3])
def test_triangular_h_gives_identity(Q):
    rng = np.random.default_rng(300 + Q)
    D = 2 ** Q
    G = rng.standard_normal((D, D)) + 1j * rng.standard_normal((D, D))
    H = np.triu(rng.standard_normal((D, D)) + 1j * rng.standard_normal((D, D)), 1)
    H += np.diag(rng.uniform(0.5, 2.0, D))
    x = _x_of(G, H)
    assert np.abs(O.bures_unitary(Q, x) - np.eye(D)).max() < 1e-14
    want = G @ G.conj().T
    assert np.abs(O.rho_of_x(Q, x, "bures") - want / np.trace(want).real).max() < 1e-14


def test_diagonal_h_gives_its_phases():
    Q, D = 2, 4
    rng = np.random.default_rng(7)
    G = rng.standard_normal((D, D)) + 1j * rng.standard_normal((D, D))
    phases = np.exp(1j * rng.uniform(-np.pi, np.pi, D))
    H = np.diag(rng.uniform(0.5, 2.0, D) * phases)
    x = _x_of(G, H)
    assert np.abs(O.bures_unitary(Q, x) - np.diag(phases)).max() < 1e-14
    W = (np.diag(phases) + np.eye(D)) @ G
    want = W @ W.conj().T
    assert np.abs(O.rho_of_x(Q, x, "bures") - want / np.trace(want).real).max() < 1e-14


@pytest.mark.parametrize("Q", [1, 2])
def test_bures_measure_moments(Q):
    D = 2 ** Q
    n = 20000
    rng = np.random.default_rng(400 + Q)
    pur = np.empty(n)
    pur_hs = np.empty(n)
    mean = np.zeros((D, D), dtype=complex)
    for t in range(n):
        x = rng.standard_normal(4 * D * D)
        rho = O.rho_of_x(Q, x, "bures")
        pur[t] = np.real(np.trace(rho @ rho))
        mean += rho
        G, _ = _blocks(Q, x)
        hs = G @ G.conj().T
        hs /= np.trace(hs).real
        pur_hs[t] = np.real(np.trace(hs @ hs))
    mean /= n
    want = (5 * D * D + 1) / (2 * D * (D * D + 2))
    se = pur.std() / np.sqrt(n)
    assert abs(pur.mean() - want) < 4 * se, (pur.mean(), want, se)
    # the Hilbert-Schmidt measure (no (U + I) factor) is told apart
    assert abs(pur_hs.mean() - 2 * D / (D * D + 1)) < 4 * pur_hs.std() / np.sqrt(n)
    assert abs(pur_hs.mean() - want) > 10 * se
    assert np.abs(mean - np.eye(D) / D).max() < 0.01


def test_chains_take_4d2_parameters():
    Q = 2
    D = 4
    counts = np.full(9 * D, 5, dtype=np.int64)
    ch = O.Chains(Q, counts, O.RunParams(n_chains=3, n_steps=0, seed=5, beta0=0.2, param="bures"))
    assert ch.x.shape == (3, 4 * D * D)
    # step 0 of every chain: y0 = the first 4D^2 normals of step 0
    for r in range(3):
        assert np.array_equal(ch.x[r], O.normals(5, r, 0, 4 * D * D))
        rho = O.rho_of_x(Q, ch.x[r], "bures")
        assert abs(ch.ll[r] - O.loglik(Q, counts, O.probs(Q, rho))) <= 1e-12 * abs(ch.ll[r])
    out = ch.run(50)
    assert np.all(np.isfinite(ch.ll)) and out["n_accepted"].sum() > 0
