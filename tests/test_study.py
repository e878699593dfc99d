"""Host pieces of the scaling study: the packed-to-complex map against the
packed form's definition, and the fidelity of Eq. (fid) against closed
forms (pure states, commuting states, the maximally mixed state)."""
import numpy as np

from paper_2501_17334_amd import study, synth


def _pack(rho):
    D = rho.shape[0]
    P = np.zeros((D, D))
    for a in range(D):
        for b in range(D):
            P[a, b] = rho[a, b].real if a <= b else rho[b, a].imag
    return P


def test_unpack_inverts_the_packed_form():
    rng = np.random.default_rng(1)
    for D in (2, 4, 8):
        rho = synth.random_density_matrix(D, rng, rank=D)
        assert np.abs(study.unpack(_pack(rho)) - rho).max() < 1e-15
    stack = np.stack([_pack(synth.random_density_matrix(4, rng)) for _ in range(3)])
    assert study.unpack(stack).shape == (3, 4, 4)


def test_fidelity_closed_forms():
    rng = np.random.default_rng(2)
    for D in (2, 4, 16):
        psi = synth.haar_vector(D, rng)
        phi = synth.haar_vector(D, rng)
        a, b = np.outer(psi, psi.conj()), np.outer(phi, phi.conj())
        assert abs(study.fidelity(a, b) - abs(np.vdot(psi, phi)) ** 2) < 1e-12
        assert abs(study.fidelity(a, np.eye(D) / D) - 1.0 / D) < 1e-12
        p, q = rng.dirichlet(np.ones(D)), rng.dirichlet(np.ones(D))
        assert abs(study.fidelity(np.diag(p), np.diag(q)) - np.sum(np.sqrt(p * q)) ** 2) < 1e-12
        r, s = synth.random_density_matrix(D, rng, rank=D), synth.random_density_matrix(D, rng, rank=2)
        f = study.fidelity(r, s)
        assert 0.0 <= f <= 1.0
        assert abs(f - study.fidelity(s, r)) < 1e-9
        assert abs(study.fidelity(r, r) - 1.0) < 1e-12


def test_chain_counts():
    assert study.chain_counts(4096) == [2 ** k for k in range(13)]
    assert study.chain_counts(3) == [1, 2, 3]
    assert study.chain_counts(1) == [1]
