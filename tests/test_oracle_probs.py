"""Pins of the oracle's outcome probabilities p_kl = Tr(Lambda_kl rho) and of
log L (Eq. (likelihood)).

Checked against closed forms that do not use the oracle's eigenvectors:
product states rho = (x)_q (I + r_q . sigma)/2 built from the textbook Pauli
matrices, for which p_kl = prod_q (1 + (-1)^b_q r_q[s_q]) / 2; the maximally
mixed state; GHZ; normalisation over outcomes; and, for general states, the
synthetic-data module's measurement-circuit simulation (basis-change gates,
then computational-basis readout), an independent route to the same numbers.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2501_17334_amd import synth

SX = np.array([[0, 1], [1, 0]], dtype=complex)
SY = np.array([[0, -1j], [1j, 0]], dtype=complex)
SZ = np.array([[1, 0], [0, -1]], dtype=complex)


def product_state(bloch):
    rho = np.array([[1.0]], dtype=complex)
    for r in bloch:
        rho = np.kron(rho, (np.eye(2) + r[0] * SX + r[1] * SY + r[2] * SZ) / 2)
    return rho


def digits(Q, k):
    return synth.setting_digits(Q, k)


@pytest.mark.parametrize("Q", [1, 2, 3])
def test_product_states_closed_form(Q):
    rng = np.random.default_rng(Q)
    for _ in range(4):
        bloch = []
        for _q in range(Q):
            v = rng.standard_normal(3)
            bloch.append(v / np.linalg.norm(v) * rng.uniform(0.2, 1.0))
        p = O.probs(Q, product_state(bloch))
        D = 2 ** Q
        for k in range(3 ** Q):
            s = digits(Q, k)
            for l in range(D):
                b = [(l >> (Q - 1 - q)) & 1 for q in range(Q)]
                want = np.prod([(1 + (-1) ** b[q] * bloch[q][s[q]]) / 2 for q in range(Q)])
                assert abs(p[k, l] - want) < 1e-15


def test_single_qubit_eigenstates():
    # |+>, |->, |+i>, |-i>, |0>, |1>: probability 1 for their own outcome
    cases = [((1, 0, 0), 0, 0), ((-1, 0, 0), 0, 1), ((0, 1, 0), 1, 0), ((0, -1, 0), 1, 1),
             ((0, 0, 1), 2, 0), ((0, 0, -1), 2, 1)]
    for r, s, b in cases:
        p = O.probs(1, product_state([r]))
        assert abs(p[s, b] - 1.0) < 1e-15 and abs(p[s, 1 - b]) < 1e-15


@pytest.mark.parametrize("Q", [1, 2, 3, 4])
def test_maximally_mixed_and_normalisation(Q):
    D = 2 ** Q
    p = O.probs(Q, np.eye(D, dtype=complex) / D)
    assert np.allclose(p, 1.0 / D, atol=1e-15, rtol=0)
    rng = np.random.default_rng(Q)
    r = O.rho_of_x(Q, rng.standard_normal(O.dims(Q)[2]))
    p = O.probs(Q, r)
    assert np.allclose(p.sum(axis=1), 1.0, atol=1e-14, rtol=0)
    assert p.min() > 0


@pytest.mark.parametrize("Q", [2, 3, 4])
def test_ghz(Q):
    D = 2 ** Q
    g = synth.ghz_vector(Q)
    p = O.probs(Q, np.outer(g, g.conj()))
    zz = 3 ** Q - 1  # all-Z setting
    want = np.zeros(D)
    want[0] = want[-1] = 0.5
    assert np.allclose(p[zz], want, atol=1e-15)


@pytest.mark.parametrize("Q", [1, 2, 3, 4])
def test_matches_measurement_circuit(Q):
    rng = np.random.default_rng(40 + Q)
    D = 2 ** Q
    st = synth.TruthState(Q, [0.6, 0.3], [synth.haar_vector(D, rng), synth.haar_vector(D, rng)], 0.1)
    p = O.probs(Q, st.density_matrix())
    assert np.allclose(p, synth.outcome_distribution(st), atol=1e-14, rtol=0)


def test_loglik_special_cases():
    Q, D = 3, 8
    rng = np.random.default_rng(0)
    counts = rng.integers(0, 50, size=(27, 8))
    p = O.probs(Q, np.eye(D, dtype=complex) / D)
    assert abs(O.loglik(Q, counts, p) + counts.sum() * np.log(D)) < 1e-12 * counts.sum() * np.log(D)
    assert O.loglik(Q, np.zeros((27, 8), dtype=np.int64), p) == 0.0
    # a zero probability only matters where a count sits
    p0 = p.copy()
    p0[3, 2] = 0.0
    c = counts.copy()
    c[3, 2] = 0
    assert np.isfinite(O.loglik(Q, c, p0))
    c[3, 2] = 1
    assert O.loglik(Q, c, p0) == -np.inf
    # pure |0><0| on one qubit with counts only on the Z outcome 0
    c1 = np.array([[3, 5], [4, 4], [10, 0]])
    p1 = O.probs(1, product_state([(0, 0, 1)]))
    assert abs(O.loglik(1, c1, p1) - 16 * np.log(0.5)) < 1e-13
