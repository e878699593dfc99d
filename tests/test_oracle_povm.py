"""Pins of the oracle's probabilities for user POVM elements, p_m =
Tr(Pi_m rho), against what is fixed independently of that code:

* the Pauli settings written out as POVM elements (products of textbook
  Pauli eigenvectors, in the library's index order) give the oracle's
  product-eigenvector probabilities of the Pauli settings;
* the qubit SIC-POVM gives (1 + n_m . r) / 4 from the Bloch vector r;
* the projectors of complete orthonormal bases sum to the trace, 1 per basis;
* chains started on a POVM problem carry log L = sum_m c_m log Tr(Pi_m rho).
"""
import itertools

import numpy as np
import pytest

from oracle import oracle as O
from paper_2501_17334_amd import synth

_S2 = 1 / np.sqrt(2)
# eigenvectors of X, Y, Z; index 0 is the +1 eigenvalue
_EIG = {0: [np.array([_S2, _S2]), np.array([_S2, -_S2])],
        1: [np.array([_S2, 1j * _S2]), np.array([_S2, -1j * _S2])],
        2: [np.array([1.0, 0.0]), np.array([0.0, 1.0])]}


def _pauli_povm(Q):
    """Setting k = sum_q s_q 3^(Q-q), outcome l = sum_q b_q 2^(Q-q), qubit 1
    the leftmost Kronecker factor."""
    out = []
    for s in itertools.product(range(3), repeat=Q):
        for b in itertools.product(range(2), repeat=Q):
            v = np.array([1.0 + 0j])
            for q in range(Q):
                v = np.kron(v, _EIG[s[q]][b[q]])
            out.append(np.outer(v, v.conj()))
    return np.stack(out)


@pytest.mark.parametrize("Q", [1, 2, 3])
def test_pauli_settings_as_povm(Q):
    rng = np.random.default_rng(40 + Q)
    povm = _pauli_povm(Q)
    for _ in range(5):
        rho = synth.random_density_matrix(2 ** Q, rng, rank=int(rng.integers(1, 2 ** Q + 1)))
        assert np.abs(O.probs_povm(Q, rho, povm) - O.probs(Q, rho).ravel()).max() < 1e-14


def test_sic_closed_form():
    prob = synth.sic_qubit_problem()
    rng = np.random.default_rng(5)
    n = np.array([[0.0, 0.0, 1.0], [2 * np.sqrt(2) / 3, 0.0, -1 / 3],
                  [-np.sqrt(2) / 3, np.sqrt(2 / 3), -1 / 3], [-np.sqrt(2) / 3, -np.sqrt(2 / 3), -1 / 3]])
    for _ in range(5):
        rho = synth.random_density_matrix(2, rng, rank=2)
        r = np.array([2 * rho[0, 1].real, -2 * rho[0, 1].imag, (rho[0, 0] - rho[1, 1]).real])
        assert np.abs(O.probs_povm(1, rho, prob.povm) - (1 + n @ r) / 4).max() < 1e-15


@pytest.mark.parametrize("Q", [2, 3])
def test_complete_bases_sum_to_one(Q):
    prob = synth.random_bases_problem(Q)
    D = 2 ** Q
    rho = prob.truth.density_matrix()
    p = O.probs_povm(Q, rho, prob.povm).reshape(-1, D)
    assert np.abs(p.sum(1) - 1.0).max() < 1e-13
    assert p.min() >= -1e-15


def test_chains_on_a_povm_problem():
    prob = synth.random_bases_problem(2)
    ch = O.Chains(2, prob.counts, O.RunParams(n_chains=3, n_steps=0, seed=prob.seed, beta0=0.1, povm=prob.povm))
    for r in range(3):
        p = O.probs_povm(2, O.rho_of_x(2, ch.x[r]), prob.povm)
        want = float(np.sum(prob.counts * np.log(p)))
        assert abs(ch.ll[r] - want) <= 1e-12 * abs(want)
    ch.run(30)
    assert np.all(np.isfinite(ch.ll))
