"""Chain diagnostics in plain numpy FP64 (TEST INFRASTRUCTURE ONLY).

* ``acf`` follows Eq. (ACFrho)/(ACFa): for one chain with stored samples
  rho^1..rho^N and their mean rho_hat^N, c[l] is proportional to
  sum_{n=1}^{N-l_max} Re Tr[(rho^n - rho_hat)^dag (rho^{n+l} - rho_hat)],
  normalised so that c[0] = 1.  Over several chains the unnormalised sums
  are averaged before normalising.
* ``iact``: Eq. (IACT), tau = 1 + 2 sum_{l=1}^{l_max} c[l].
* ``n_eff``: N_eff = N R / tau (Section "Simulated Results").
* ``frobenius_sq`` and ``fidelity``: Eqs. (fro) and (fid).

Samples are given in the packed real form (D x D reals, P[a][b] = Re rho_ab
for a <= b and Im rho_ba for a > b).  The trace in Eq. (ACFrho) runs over
all D^2 complex entries, so an off-diagonal packed entry stands for two
entries of rho with equal products: weight 2, diagonal weight 1.
"""
from __future__ import annotations

import numpy as np


def _weights(D):
    w = np.full((D, D), 2.0)
    np.fill_diagonal(w, 1.0)
    return w.reshape(-1)


def acf_sums(samples, l_max):
    """Unnormalised lag sums for one chain: samples (N, D, D) packed."""
    s = np.asarray(samples, dtype=np.float64)
    N, D = s.shape[0], s.shape[-1]
    if N <= l_max:
        raise ValueError("need more stored samples than l_max")
    v = s.reshape(N, D * D)
    dev = v - v.mean(axis=0)
    w = _weights(D)
    n_terms = N - l_max
    out = np.zeros(l_max + 1)
    for lag in range(l_max + 1):
        out[lag] = np.sum(w * dev[:n_terms] * dev[lag:lag + n_terms])
    return out


def acf(samples, l_max=200):
    """c[0..l_max] for one chain (N, D, D) or pooled over chains (R, N, D, D)."""
    s = np.asarray(samples, dtype=np.float64)
    if s.ndim == 3:
        sums = acf_sums(s, l_max)
    else:
        sums = np.mean([acf_sums(c, l_max) for c in s], axis=0)
    return sums / sums[0]


def iact(c):
    """Eq. (IACT)."""
    c = np.asarray(c, dtype=np.float64)
    return 1.0 + 2.0 * np.sum(c[1:])


def n_eff(n_per_chain, n_chains, tau):
    return n_per_chain * n_chains / tau


def frobenius_sq(a, b):
    """Eq. (fro): ||a - b||_F^2 for complex matrices."""
    return float(np.sum(np.abs(np.asarray(a) - np.asarray(b)) ** 2))


def _sqrtm_psd(m):
    w, v = np.linalg.eigh((m + m.conj().T) / 2)
    return (v * np.sqrt(np.clip(w, 0.0, None))) @ v.conj().T


def fidelity(a, b):
    """Eq. (fid): (Tr sqrt(sqrt(a) b sqrt(a)))^2."""
    sa = _sqrtm_psd(np.asarray(a))
    m = sa @ np.asarray(b) @ sa
    w = np.linalg.eigvalsh((m + m.conj().T) / 2)
    return float(np.sum(np.sqrt(np.clip(w, 0.0, None))) ** 2)
