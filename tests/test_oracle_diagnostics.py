"""Pins of the chain diagnostics (Eqs. (ACFrho), (IACT), (fro), (fid)).

* independent samples: c[l] ~ 0 for l >= 1 and tau ~ 1;
* every packed component an AR(1) series with coefficient phi: c[l] ~ phi^l
  and tau ~ 1 + 2 phi (1 - phi^l_max) / (1 - phi) (the l_max-truncated
  closed form);
* a constant offset added to every sample changes nothing (mean removed);
* the packed off-diagonal weight 2: the ACF of the packed form equals the
  ACF computed from the full complex matrices as Eq. (ACFa) writes it;
* fidelity of a state with itself is 1; with an orthogonal pure state 0.
"""
import numpy as np

from oracle import diagnostics as G
from oracle import oracle as O


def ar1(n, m, phi, rng):
    out = np.zeros((n, m))
    x = rng.standard_normal(m)
    for t in range(n):
        x = phi * x + np.sqrt(1 - phi ** 2) * rng.standard_normal(m)
        out[t] = x
    return out


def test_iid_tau_one():
    rng = np.random.default_rng(0)
    s = rng.standard_normal((20, 4000, 2, 2))
    c = G.acf(s, l_max=50)
    assert c[0] == 1.0
    assert np.all(np.abs(c[1:]) < 0.02)
    assert abs(G.iact(c) - 1.0) < 0.3


def test_ar1_closed_form():
    rng = np.random.default_rng(1)
    phi, l_max = 0.6, 200
    s = np.stack([ar1(5000, 4, phi, rng).reshape(5000, 2, 2) for _ in range(20)])
    c = G.acf(s, l_max=l_max)
    assert np.all(np.abs(c[1:6] - phi ** np.arange(1, 6)) < 0.03)
    tau_true = 1 + 2 * phi * (1 - phi ** l_max) / (1 - phi)
    assert abs(G.iact(c) - tau_true) < 0.35


def test_offset_invariance_and_full_matrix_form():
    rng = np.random.default_rng(2)
    Q = 2
    xs = [rng.standard_normal(O.dims(Q)[2]) for _ in range(300)]
    packed = np.array([O.pack(O.rho_of_x(Q, x)) for x in xs])
    c1 = G.acf(packed, l_max=20)
    c2 = G.acf(packed + 0.37, l_max=20)
    assert np.allclose(c1, c2, atol=1e-12)
    # Eq. (ACFa) on the full complex matrices
    full = np.array([O.rho_of_x(Q, x) for x in xs])
    dev = full - full.mean(axis=0)
    n = 300 - 20
    sums = np.array([np.sum((dev[:n].conj() * dev[l:l + n]).real) for l in range(21)])
    assert np.allclose(c1, sums / sums[0], atol=1e-12)


def test_fidelity_and_frobenius():
    rng = np.random.default_rng(3)
    r = O.rho_of_x(2, rng.standard_normal(O.dims(2)[2]))
    assert abs(G.fidelity(r, r) - 1.0) < 1e-10
    a = np.diag([1.0, 0, 0, 0]).astype(complex)
    b = np.diag([0, 1.0, 0, 0]).astype(complex)
    assert abs(G.fidelity(a, b)) < 1e-12
    assert G.frobenius_sq(a, b) == 2.0
