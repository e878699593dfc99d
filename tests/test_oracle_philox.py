"""Pins of the oracle's random streams.

Philox4x64-10 is checked bit for bit against numpy's independent
implementation of the same published generator (Salmon et al., SC'11);
numpy pre-increments its counter, so its block at counter c is ours at c+1.
The normals are checked against the standard normal law (moments, a
Kolmogorov-Smirnov test, independence of the two members of a Box-Muller pair).
"""
import numpy as np
import pytest
from scipy import stats

from oracle import oracle as O


def test_philox_known_answer_zero():
    # Known answer of Philox4x64-10 at counter 0, key 0 (Random123 KAT)
    got = O.philox4x64_10([0, 0, 0, 0], [0, 0])
    want = [0x16554d9eca36314c, 0xdb20fe9d672d0fdc, 0xd7e772cee186176b, 0x7e68b68aec7ba23b]
    assert [int(v) for v in got] == want


@pytest.mark.parametrize("trial", range(200))
def test_philox_matches_numpy(trial):
    rng = np.random.default_rng(trial)
    ctr = [int(v) for v in rng.integers(0, 2 ** 63, size=4, dtype=np.int64)]
    ctr[0] += 1  # keep ctr[0] >= 1 so that numpy's pre-increment does not carry
    key = [int(v) for v in rng.integers(0, 2 ** 63, size=2, dtype=np.int64)]
    bg = np.random.Philox(counter=[ctr[0] - 1, ctr[1], ctr[2], ctr[3]], key=key[0] | (key[1] << 64))
    want = [int(v) for v in bg.random_raw(4)]
    got = [int(v) for v in O.philox4x64_10(ctr, key)]
    assert got == want


def test_philox_high_bits_of_counter_words():
    # the stream tag lives in bits 56..63 of counter word 3
    ctr = [7, 11, 13, 1 << 56]
    bg = np.random.Philox(counter=[6, 11, 13, 1 << 56], key=42)
    assert [int(v) for v in O.philox4x64_10(ctr, [42, 0])] == [int(v) for v in bg.random_raw(4)]


def test_u53_open_interval():
    assert O.u53(0) == 2.0 ** -53
    assert O.u53(2 ** 64 - 1) == 1.0 - 2.0 ** -53
    assert O.u53(1 << 63) == 0.5 + 2.0 ** -53
    assert 0.0 < O.u53(0) < O.u53(2 ** 64 - 1) < 1.0


def test_normals_law():
    n = 4 * 250_000
    z = np.concatenate([O.normals(17, c, 3, 4000) for c in range(250)])
    assert z.size == n
    se = 1.0 / np.sqrt(n)
    assert abs(z.mean()) < 5 * se
    assert abs(z.var() - 1.0) < 5 * np.sqrt(2.0) * se
    assert abs(stats.kurtosis(z)) < 5 * np.sqrt(24.0) * se
    assert stats.kstest(z, "norm").pvalue > 1e-3
    # members of a Box-Muller pair are independent: correlation ~ 0,
    # and r^2 = n0^2 + n1^2 is chi-square with 2 degrees of freedom
    pairs = z.reshape(-1, 2)
    assert abs(np.corrcoef(pairs[:, 0], pairs[:, 1])[0, 1]) < 5 / np.sqrt(pairs.shape[0])
    r2 = (pairs ** 2).sum(axis=1)
    assert stats.kstest(r2, "chi2", args=(2,)).pvalue > 1e-3


def test_streams_are_distinct():
    a = O.normals(5, 0, 1, 16)
    assert not np.array_equal(a, O.normals(5, 1, 1, 16))   # chain
    assert not np.array_equal(a, O.normals(5, 0, 2, 16))   # step
    assert not np.array_equal(a, O.normals(6, 0, 1, 16))   # seed
    assert O.mh_uniform(5, 0, 1) != O.da_uniform(5, 0, 1)  # tag
    # a prefix of a longer draw is the shorter draw
    assert np.array_equal(O.normals(5, 0, 1, 10), O.normals(5, 0, 1, 16)[:10])


def test_uniform_law():
    u = np.array([O.mh_uniform(9, c, s) for c in range(100) for s in range(200)])
    assert stats.kstest(u, "uniform").pvalue > 1e-3
