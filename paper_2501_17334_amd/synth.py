"""Seeded synthetic tomography data: true states and Pauli-measurement counts.

This module is the one input source shared by the GPU library's callers and
the CPU oracle's tests.  It holds none of the sampler's arithmetic: it
simulates the experiment of the paper's Step 1 (all 3^Q Pauli settings, P
shots each, Section "Simulated Results") by applying each setting's
basis-change circuit to the pure components of the true state and reading out
in the computational basis (Born rule on the rotated amplitudes), then draws
multinomial counts.

Conventions (shared with the library and the oracle through the data layout
only): setting k = sum_q s_q 3^(Q-q) with s in {X=0, Y=1, Z=2}; outcome
l = sum_q b_q 2^(Q-q); qubit 1 is the most significant bit; b = 0 is the +1
eigenvalue.  counts has shape (3^Q, 2^Q), flattened as k*D + l.

No public data set is used: the paper's IBM ``ibmq_kyoto`` counts are not
available, so every workload below is synthetic with the sizes of the
paper's experiments and of the benchmark configurations.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

DATA_SEED = 2501
CHAIN_SEED = 17334

_H = np.array([[1.0, 1.0], [1.0, -1.0]]) / np.sqrt(2.0)
_SDAG = np.array([[1.0, 0.0], [0.0, -1.0j]])
# basis change applied before a computational-basis readout, per setting
_ROT = {0: _H.astype(complex), 1: _H @ _SDAG, 2: np.eye(2, dtype=complex)}


@dataclass
class TruthState:
    """rho = sum_i w_i |psi_i><psi_i| + white * I/D (weights sum to 1)."""
    n_qubits: int
    weights: list
    vectors: list
    white: float = 0.0

    @property
    def dim(self):
        return 2 ** self.n_qubits

    def density_matrix(self):
        D = self.dim
        rho = self.white * np.eye(D, dtype=complex) / D
        for w, v in zip(self.weights, self.vectors):
            rho = rho + w * np.outer(v, v.conj())
        return rho


def haar_vector(D, rng):
    g = rng.standard_normal(D) + 1j * rng.standard_normal(D)
    return g / np.linalg.norm(g)


def random_density_matrix(D, rng, rank=None):
    """A random density matrix: Haar vectors mixed with random weights."""
    rank = D if rank is None else rank
    w = rng.uniform(0.05, 1.0, rank)
    w /= w.sum()
    rho = np.zeros((D, D), dtype=complex)
    for i in range(rank):
        v = haar_vector(D, rng)
        rho += w[i] * np.outer(v, v.conj())
    return rho


def ghz_vector(Q):
    v = np.zeros(2 ** Q, dtype=complex)
    v[0] = v[-1] = 1.0 / np.sqrt(2.0)
    return v


def w_vector(Q):
    """|W_Q> = Q^(-1/2) sum_q |0..1_q..0> (Eq. (W))."""
    v = np.zeros(2 ** Q, dtype=complex)
    for q in range(Q):
        v[1 << (Q - 1 - q)] = 1.0
    return v / np.sqrt(Q)


def _rotate(psi, Q, setting_digits):
    t = psi.reshape((2,) * Q)
    for q, s in enumerate(setting_digits):
        t = np.moveaxis(np.tensordot(_ROT[s], t, axes=([1], [q])), 0, q)
    return t.reshape(-1)


def setting_digits(Q, k):
    digits = []
    for _ in range(Q):
        digits.append(k % 3)
        k //= 3
    return digits[::-1]


def outcome_distribution(state: TruthState):
    """(3^Q, 2^Q) outcome probabilities of every Pauli setting, from the
    measurement circuit (rotation, then computational-basis readout)."""
    Q, D = state.n_qubits, state.dim
    K = 3 ** Q
    out = np.full((K, D), state.white / D)
    for k in range(K):
        dig = setting_digits(Q, k)
        for w, v in zip(state.weights, state.vectors):
            out[k] += w * np.abs(_rotate(v, Q, dig)) ** 2
    return out


def sample_counts(dist, shots, rng):
    counts = np.zeros(dist.shape, dtype=np.int64)
    for k in range(dist.shape[0]):
        p = np.clip(dist[k], 0.0, None)
        counts[k] = rng.multinomial(shots, p / p.sum())
    return counts


@dataclass
class PovmProblem:
    """A measurement other than the Pauli settings: POVM elements [n, D, D]
    with one count each."""
    name: str
    n_qubits: int
    povm: np.ndarray
    counts: np.ndarray
    truth: TruthState
    seed: int


def random_bases_problem(Q, shots=1024, n_bases=None, white=0.1, index=0) -> PovmProblem:
    """n_bases (default 3^Q) Haar-random orthonormal bases U_k (scipy's
    unitary_group); the POVM elements are the projectors onto the columns
    u_kl of each U_k, and the counts of basis k are a multinomial sample of
    the diagonal of U_k^dag rho U_k (the state rotated into the basis and read
    out).  Truth: a Haar pure state with white noise."""
    from scipy.stats import unitary_group
    rng = np.random.default_rng([DATA_SEED, 91, Q, index])
    D = 2 ** Q
    K = n_bases or 3 ** Q
    bases = [unitary_group.rvs(D, random_state=rng) for _ in range(K)]
    st = _noisy_pure(Q, haar_vector(D, rng), white)
    rho = st.density_matrix()
    povm = np.stack([np.outer(U[:, l], U[:, l].conj()) for U in bases for l in range(D)])
    dist = np.stack([np.real(np.diag(U.conj().T @ rho @ U)) for U in bases])
    counts = sample_counts(dist, shots, rng).reshape(-1)
    return PovmProblem(f"bases_{Q}", Q, povm, counts, st, CHAIN_SEED + 200 + Q)


@dataclass
class PoissonProblem:
    """Pauli-setting counts that are independent Poisson variables with known
    intensities: count (k, l) has mean intensity[k, l] * p_kl."""
    name: str
    n_qubits: int
    counts: np.ndarray          # (3^Q, 2^Q) int64
    intensity: np.ndarray       # (3^Q, 2^Q) float64
    truth: TruthState
    seed: int


def poisson_problem(Q, shots=1000, efficiency=(0.9, 0.6), white=0.1, index=0) -> PoissonProblem:
    """Every Pauli setting runs for `shots` trials, and the detector of each
    qubit registers outcome b with efficiency efficiency[b]: count (k, l) is
    Poisson with mean shots * prod_q efficiency[b_q(l)] * p_kl, independently
    of the others (counting with unequal detectors, where the multinomial
    model of Eq. (likelihood) no longer holds).  Truth: a Haar pure state with
    white noise."""
    rng = np.random.default_rng([DATA_SEED, 93, Q, index])
    D = 2 ** Q
    st = _noisy_pure(Q, haar_vector(D, rng), white)
    eta = np.ones(D)
    for l in range(D):
        for q in range(Q):
            eta[l] *= efficiency[(l >> (Q - 1 - q)) & 1]
    intensity = np.tile(shots * eta, (3 ** Q, 1))
    mean = intensity * np.clip(outcome_distribution(st), 0.0, None)
    counts = rng.poisson(mean).astype(np.int64)
    return PoissonProblem(f"poisson_{Q}", Q, counts, intensity, st, CHAIN_SEED + 400 + Q)


def sic_qubit_problem(shots=4000, white=0.1) -> PovmProblem:
    """The qubit SIC-POVM: Pi_m = (I + n_m . sigma) / 4 with n_m the vertices
    of a regular tetrahedron; the outcome probabilities of a state with Bloch
    vector r are (1 + n_m . r) / 4.  Truth: a Haar pure state with white noise."""
    rng = np.random.default_rng([DATA_SEED, 92])
    n = np.array([[0.0, 0.0, 1.0], [2 * np.sqrt(2) / 3, 0.0, -1 / 3],
                  [-np.sqrt(2) / 3, np.sqrt(2 / 3), -1 / 3], [-np.sqrt(2) / 3, -np.sqrt(2 / 3), -1 / 3]])
    sx = np.array([[0, 1], [1, 0]], dtype=complex)
    sy = np.array([[0, -1j], [1j, 0]])
    sz = np.array([[1, 0], [0, -1]], dtype=complex)
    povm = np.stack([(np.eye(2) + v[0] * sx + v[1] * sy + v[2] * sz) / 4 for v in n])
    st = _noisy_pure(1, haar_vector(2, rng), white)
    rho = st.density_matrix()
    r = np.array([2 * rho[0, 1].real, -2 * rho[0, 1].imag, (rho[0, 0] - rho[1, 1]).real])
    p = np.clip((1 + n @ r) / 4, 0.0, None)
    counts = rng.multinomial(shots, p / p.sum()).astype(np.int64)
    return PovmProblem("sic_1", 1, povm, counts, st, CHAIN_SEED + 300)


@dataclass
class Problem:
    name: str
    n_qubits: int
    counts: np.ndarray          # (3^Q, 2^Q) int64
    truth: TruthState
    shots: int
    n_chains: int
    n_steps: int
    seed: int = CHAIN_SEED
    extra: dict = field(default_factory=dict)


def _noisy_pure(Q, vec, white):
    return TruthState(Q, [1.0 - white], [vec], white)


def make_problem(name: str, *, n_chains=None, n_steps=None, index=0) -> Problem:
    """The synthetic workloads.

    c1  1 qubit: 0.9|psi><psi| + 0.1 I/2, Haar psi; 1000 shots/setting;
        64 chains x 2000 steps, beta0 = 0.1 (Algorithm 2 as printed).
    c2  2 qubits: Haar pure state + 10% white noise; 1000 shots; 4096 x 1e4.
    c3  4 qubits: 0.95 |GHZ><GHZ| + 0.05 I/16; 1024 shots; 65536 x 1e4.
    c4  5 qubits: rank-2 WW^dag/Tr, W complex Gaussian 32x2; 1024 shots;
        16384 chains (delayed-acceptance workload).
    c5_<i>  problem i of the mixed batch: Q ~ U{1..6}, Haar pure + 10% white,
        1024 shots, chains ~ U{256, 512, 1024, 2048, 4096}, 2000 steps.
    zero_<Q> all-zero counts (the run samples the prior).
    w_<Q>   |W_Q> with 10% white noise, P = 25 * 2^Q shots (the paper's
        experimental target state and shot budget).
    """
    if name.startswith("zero_"):
        Q = int(name.split("_")[1])
        st = TruthState(Q, [], [], 1.0)
        counts = np.zeros((3 ** Q, 2 ** Q), dtype=np.int64)
        return Problem(name, Q, counts, st, 0, n_chains or 256, n_steps or 1000)
    if name.startswith("w_"):
        Q = int(name.split("_")[1])
        rng = np.random.default_rng([DATA_SEED, 77, Q])
        st = _noisy_pure(Q, w_vector(Q), 0.1)
        shots = 25 * 2 ** Q
        counts = sample_counts(outcome_distribution(st), shots, rng)
        return Problem(name, Q, counts, st, shots, n_chains or 1024, n_steps or 4096)
    if name == "c1":
        rng = np.random.default_rng(DATA_SEED)
        st = _noisy_pure(1, haar_vector(2, rng), 0.1)
        counts = sample_counts(outcome_distribution(st), 1000, rng)
        return Problem(name, 1, counts, st, 1000, n_chains or 64, n_steps or 2000,
                       extra={"beta0": 0.1})
    if name == "c2":
        rng = np.random.default_rng(DATA_SEED)
        st = _noisy_pure(2, haar_vector(4, rng), 0.1)
        counts = sample_counts(outcome_distribution(st), 1000, rng)
        return Problem(name, 2, counts, st, 1000, n_chains or 4096, n_steps or 10000)
    if name == "c3":
        rng = np.random.default_rng(DATA_SEED)
        st = _noisy_pure(4, ghz_vector(4), 0.05)
        counts = sample_counts(outcome_distribution(st), 1024, rng)
        return Problem(name, 4, counts, st, 1024, n_chains or 65536, n_steps or 10000)
    if name == "c4":
        rng = np.random.default_rng(DATA_SEED)
        W = rng.standard_normal((32, 2)) + 1j * rng.standard_normal((32, 2))
        norms = np.sum(np.abs(W) ** 2, axis=0)
        st = TruthState(5, list(norms / norms.sum()), [W[:, i] / np.sqrt(norms[i]) for i in range(2)])
        counts = sample_counts(outcome_distribution(st), 1024, rng)
        return Problem(name, 5, counts, st, 1024, n_chains or 16384, n_steps or 10000)
    if name.startswith("c5"):
        i = index if name == "c5" else int(name.split("_")[1])
        rng = np.random.default_rng([DATA_SEED, 5, i])
        Q = int(rng.integers(1, 7))
        chains = int(rng.choice([256, 512, 1024, 2048, 4096]))
        st = _noisy_pure(Q, haar_vector(2 ** Q, rng), 0.1)
        counts = sample_counts(outcome_distribution(st), 1024, rng)
        return Problem(f"c5_{i}", Q, counts, st, 1024, n_chains or chains, n_steps or 2000,
                       seed=CHAIN_SEED + 1 + i)
    raise ValueError(f"unknown workload {name!r}")


def mixed_batch(n_problems=256, n_steps=2000):
    """The 256-problem mixed batch (1..6 qubits)."""
    return [make_problem("c5", index=i, n_steps=n_steps) for i in range(n_problems)]
