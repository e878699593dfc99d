"""The synthetic-data generator: sizes and seeds of every workload."""
import numpy as np
import pytest

from paper_2501_17334_amd import synth


@pytest.mark.parametrize("name,Q,shots,chains", [("c1", 1, 1000, 64), ("c2", 2, 1000, 4096),
                                                  ("c3", 4, 1024, 65536), ("c4", 5, 1024, 16384)])
def test_configs(name, Q, shots, chains):
    p = synth.make_problem(name)
    assert p.n_qubits == Q and p.shots == shots and p.n_chains == chains
    assert p.counts.shape == (3 ** Q, 2 ** Q)
    assert np.all(p.counts.sum(axis=1) == shots)
    r = p.truth.density_matrix()
    assert abs(np.trace(r) - 1) < 1e-12
    # seeded: the same call gives the same counts
    assert np.array_equal(p.counts, synth.make_problem(name).counts)


def test_mixed_batch():
    b = synth.mixed_batch(256)
    qs = [p.n_qubits for p in b]
    assert set(qs) == {1, 2, 3, 4, 5, 6}
    assert all(p.n_chains in (256, 512, 1024, 2048, 4096) for p in b)
    assert len({p.seed for p in b}) == 256


def test_outcome_distribution_normalised():
    rng = np.random.default_rng(0)
    st = synth.TruthState(3, [1.0], [synth.haar_vector(8, rng)], 0.0)
    d = synth.outcome_distribution(st)
    assert np.allclose(d.sum(axis=1), 1.0)
    w = synth.w_vector(3)
    assert abs(np.linalg.norm(w) - 1) < 1e-15 and np.count_nonzero(w) == 3
