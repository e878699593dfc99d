"""Python face of the FP64 CPU oracle (TEST INFRASTRUCTURE ONLY).

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import this module.  It loads ``liborc.so`` built from
``qst_oracle.c`` (``oracle/build.py``) and wraps its functions with numpy
arrays.  Everything here follows the paper's Algorithm 2, Steps 1-6 and
Eqs. (likelihood), (BME2); see the C file for the conventions.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liborc.so")
_lib = None

c_double_p = C.POINTER(C.c_double)
c_int64_p = C.POINTER(C.c_int64)
c_int32_p = C.POINTER(C.c_int32)
c_int8_p = C.POINTER(C.c_int8)
c_uint64_p = C.POINTER(C.c_uint64)


class _Mlp(C.Structure):
    _fields_ = [("d_in", C.c_int), ("h1", C.c_int), ("h2", C.c_int),
                ("W1", c_double_p), ("b1", c_double_p), ("W2", c_double_p),
                ("b2", c_double_p), ("w3", c_double_p),
                ("b3", C.c_double), ("out_scale", C.c_double), ("out_shift", C.c_double)]


class _RunDesc(C.Structure):
    _fields_ = [("n_qubits", C.c_int32), ("counts", c_int64_p), ("n_chains", C.c_int64),
                ("chain_offset", C.c_int64), ("step_begin", C.c_int64), ("n_steps", C.c_int64),
                ("thin", C.c_int32), ("burn_in", C.c_int64), ("beta0", C.c_double),
                ("adapt_every", C.c_int32), ("adapt_lo", C.c_double), ("adapt_hi", C.c_double),
                ("adapt_factor", C.c_double), ("adapt_until", C.c_int64), ("seed", C.c_uint64),
                ("surrogate", C.POINTER(_Mlp)), ("trace_chains", C.c_int32),
                ("record_every", C.c_int32), ("record_chains", C.c_int32), ("param", C.c_int32),
                ("povm", c_double_p), ("n_povm", C.c_int32), ("alpha", C.c_double),
                ("intensity", c_double_p)]


class _State(C.Structure):
    _fields_ = [("x", c_double_p), ("ll", c_double_p), ("beta", c_double_p),
                ("acc_win", c_int32_p), ("rho_cur", c_double_p), ("s1", c_double_p),
                ("s2", c_double_p), ("n_stored", c_int64_p), ("n_accepted", c_int64_p),
                ("n_stage1", c_int64_p), ("n_near", c_int64_p), ("tr_llprop", c_double_p),
                ("tr_logu", c_double_p), ("tr_accept", c_int8_p), ("rec", c_double_p),
                ("s_cur", c_double_p)]


def lib():
    """Load liborc.so (built by oracle/build.py); raise if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"oracle library not built: {_LIB_PATH} (run oracle/build.py)")
        L = C.CDLL(_LIB_PATH)
        L.orc_philox4x64_10.argtypes = [c_uint64_p, c_uint64_p, c_uint64_p]
        L.orc_u53.argtypes = [C.c_uint64]
        L.orc_u53.restype = C.c_double
        L.orc_normals.argtypes = [C.c_uint64, C.c_uint64, C.c_uint64, C.c_int, c_double_p]
        L.orc_mh_uniform.argtypes = [C.c_uint64, C.c_uint64, C.c_uint64]
        L.orc_mh_uniform.restype = C.c_double
        L.orc_da_uniform.argtypes = [C.c_uint64, C.c_uint64, C.c_uint64]
        L.orc_da_uniform.restype = C.c_double
        L.orc_rho.argtypes = [C.c_int, c_double_p, c_double_p]
        L.orc_rho_bures.argtypes = [C.c_int, c_double_p, c_double_p]
        L.orc_rho_dirichlet.argtypes = [C.c_int, c_double_p, C.c_double, c_double_p]
        L.orc_gamma_quantile.argtypes = [C.c_double, C.c_double]
        L.orc_gamma_quantile.restype = C.c_double
        L.orc_gamma_pq.argtypes = [C.c_double, C.c_double, c_double_p, c_double_p]
        L.orc_bures_unitary.argtypes = [C.c_int, c_double_p, c_double_p]
        L.orc_param_dim.argtypes = [C.c_int, C.c_int]
        L.orc_param_dim.restype = C.c_int
        L.orc_pack.argtypes = [C.c_int, c_double_p, c_double_p]
        L.orc_unpack.argtypes = [C.c_int, c_double_p, c_double_p]
        L.orc_probs.argtypes = [C.c_int, c_double_p, c_double_p]
        L.orc_probs_povm.argtypes = [C.c_int, c_double_p, C.c_int, c_double_p, c_double_p]
        L.orc_loglik.argtypes = [C.c_int, c_int64_p, c_double_p]
        L.orc_loglik.restype = C.c_double
        L.orc_loglik_poisson.argtypes = [C.c_int, c_int64_p, c_double_p, c_double_p]
        L.orc_loglik_poisson.restype = C.c_double
        L.orc_mlp_forward.argtypes = [C.POINTER(_Mlp), c_double_p]
        L.orc_mlp_forward.restype = C.c_double
        L.orc_init_chains.argtypes = [C.POINTER(_RunDesc), C.POINTER(_State)]
        L.orc_run_chains.argtypes = [C.POINTER(_RunDesc), C.POINTER(_State)]
        L.orc_eval_batch.argtypes = [C.c_int, c_int64_p, C.c_int64, c_double_p, c_double_p,
                                     c_double_p]
        L.orc_num_threads.restype = C.c_int
        L.orc_set_num_threads.argtypes = [C.c_int]
        L.orc_pool.argtypes = [C.c_int, C.c_int64, c_double_p, c_double_p, c_int64_p,
                               c_double_p, c_double_p]
        _lib = L
    return _lib


def _p(a, t=c_double_p):
    return a.ctypes.data_as(t) if a is not None else None


def num_threads():
    """OpenMP threads the oracle's parallel loops use."""
    return lib().orc_num_threads()


def set_num_threads(n):
    """Threads of the oracle's later parallel loops."""
    lib().orc_set_num_threads(int(n))


# parameterisations: the Gaussian/gamma form (2D^2+D parameters) and the
# paper's Algorithm 1, the Bures draw (4D^2 parameters)
PARAMS = {"gamma": 0, "bures": 1, "dirichlet": 2}


def dims(Q, param="gamma"):
    D = 2 ** Q
    return D, 3 ** Q, (4 * D * D if param == "bures" else 2 * D * D + D)


# --------------------------------------------------------------------------
# Elementary pieces
# --------------------------------------------------------------------------
def philox4x64_10(ctr, key):
    """One Philox4x64-10 block (Salmon et al., SC'11)."""
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib().orc_philox4x64_10(_p(c, c_uint64_p), _p(k, c_uint64_p), _p(out, c_uint64_p))
    return out


def u53(w):
    return lib().orc_u53(C.c_uint64(int(w)))


def normals(seed, chain, step, n):
    out = np.zeros(n)
    lib().orc_normals(seed, chain, step, n, _p(out))
    return out


def mh_uniform(seed, chain, step):
    return lib().orc_mh_uniform(seed, chain, step)


def da_uniform(seed, chain, step):
    return lib().orc_da_uniform(seed, chain, step)


def rho_of_x(Q, x, param="gamma", alpha=0.5):
    """rho(x) as a D x D complex matrix (param "bures": Algorithm 1;
    "dirichlet": Gamma(alpha)-quantile weights)."""
    D, _, d = dims(Q, param)
    x = np.ascontiguousarray(x, dtype=np.float64)
    assert x.shape == (d,)
    out = np.zeros(2 * D * D)
    if param == "dirichlet":
        lib().orc_rho_dirichlet(Q, _p(x), alpha, _p(out))
    else:
        (lib().orc_rho_bures if param == "bures" else lib().orc_rho)(Q, _p(x), _p(out))
    return out.reshape(D, D, 2) @ np.array([1.0, 1j])


def gamma_quantile(a, v):
    """P^{-1}(a, Phi(v)): the Gamma(a) quantile of the normal probability of v."""
    return lib().orc_gamma_quantile(a, v)


def gamma_pq(a, x):
    P, Qc = np.zeros(1), np.zeros(1)
    lib().orc_gamma_pq(a, x, _p(P), _p(Qc))
    return P[0], Qc[0]


def bures_unitary(Q, x):
    """U = Q Lambda of Algorithm 1 for the H part of x (D x D complex)."""
    D, _, d = dims(Q, "bures")
    x = np.ascontiguousarray(x, dtype=np.float64)
    assert x.shape == (d,)
    out = np.zeros(2 * D * D)
    lib().orc_bures_unitary(Q, _p(x), _p(out))
    return out.reshape(D, D, 2) @ np.array([1.0, 1j])


def pack(rho):
    """Complex Hermitian D x D -> packed real D x D (see the C file)."""
    D = rho.shape[0]
    Q = D.bit_length() - 1
    inter = np.ascontiguousarray(np.stack([rho.real, rho.imag], axis=-1).reshape(-1))
    out = np.zeros(D * D)
    lib().orc_pack(Q, _p(inter), _p(out))
    return out.reshape(D, D)


def unpack(packed):
    packed = np.ascontiguousarray(packed, dtype=np.float64)
    D = packed.shape[-1]
    Q = D.bit_length() - 1
    out = np.zeros(2 * D * D)
    lib().orc_unpack(Q, _p(packed.reshape(-1)), _p(out))
    return out.reshape(D, D, 2) @ np.array([1.0, 1j])


def probs(Q, rho):
    """p[k, l] = Tr(Lambda_kl rho) for all Pauli settings k and outcomes l."""
    D, K, _ = dims(Q)
    inter = np.ascontiguousarray(np.stack([rho.real, rho.imag], axis=-1).reshape(-1))
    out = np.zeros(K * D)
    lib().orc_probs(Q, _p(inter), _p(out))
    return out.reshape(K, D)


def _interleave(a):
    a = np.asarray(a, dtype=complex)
    return np.ascontiguousarray(np.stack([a.real, a.imag], axis=-1).reshape(-1))


def probs_povm(Q, rho, povm):
    """p_m = Tr(Pi_m rho) for the POVM elements povm [n, D, D] (returns n values)."""
    D, K, _ = dims(Q)
    povm = np.asarray(povm, dtype=complex)
    n = povm.shape[0]
    out = np.zeros(K * D)
    lib().orc_probs_povm(Q, _p(_interleave(rho)), n, _p(_interleave(povm)), _p(out))
    return out[:n]


def loglik(Q, counts, p):
    c = np.ascontiguousarray(counts, dtype=np.int64).reshape(-1)
    pp = np.ascontiguousarray(p, dtype=np.float64).reshape(-1)
    return lib().orc_loglik(Q, _p(c, c_int64_p), _p(pp))


def loglik_poisson(Q, counts, intensity, p):
    """Poisson log L = sum_{n>0} n ln p - sum lambda p (see the C file)."""
    c = np.ascontiguousarray(counts, dtype=np.int64).reshape(-1)
    lam = np.ascontiguousarray(intensity, dtype=np.float64).reshape(-1)
    pp = np.ascontiguousarray(p, dtype=np.float64).reshape(-1)
    return lib().orc_loglik_poisson(Q, _p(c, c_int64_p), _p(lam), _p(pp))


def loglik_of_x(Q, counts, x):
    return loglik(Q, counts, probs(Q, rho_of_x(Q, x)))


def eval_batch(Q, counts, xs, want_rho=False):
    """log L (and packed rho) at every row of xs."""
    D, K, d = dims(Q)
    xs = np.ascontiguousarray(xs, dtype=np.float64).reshape(-1, d)
    c = np.ascontiguousarray(counts, dtype=np.int64).reshape(-1)
    ll = np.zeros(xs.shape[0])
    rp = np.zeros((xs.shape[0], D, D)) if want_rho else None
    lib().orc_eval_batch(Q, _p(c, c_int64_p), xs.shape[0], _p(xs), _p(ll), _p(rp))
    return (ll, rp) if want_rho else ll


# --------------------------------------------------------------------------
# MLP surrogate (FP64 forward)
# --------------------------------------------------------------------------
@dataclass
class MlpWeights:
    W1: np.ndarray  # [h1, d]
    b1: np.ndarray
    W2: np.ndarray  # [h2, h1]
    b2: np.ndarray
    w3: np.ndarray  # [h2]
    b3: float
    out_scale: float = 1.0
    out_shift: float = 0.0

    def _struct(self):
        self._keep = [np.ascontiguousarray(a, dtype=np.float64)
                      for a in (self.W1, self.b1, self.W2, self.b2, self.w3)]
        W1, b1, W2, b2, w3 = self._keep
        return _Mlp(W1.shape[1], W1.shape[0], W2.shape[0], _p(W1), _p(b1), _p(W2), _p(b2),
                    _p(w3), float(self.b3), float(self.out_scale), float(self.out_shift))


def mlp_forward(w: MlpWeights, x):
    s = w._struct()
    xx = np.ascontiguousarray(x, dtype=np.float64)
    return lib().orc_mlp_forward(C.byref(s), _p(xx))


# --------------------------------------------------------------------------
# Chains
# --------------------------------------------------------------------------
@dataclass
class RunParams:
    n_chains: int
    n_steps: int
    seed: int
    beta0: float = 0.1
    thin: int = 1
    burn_in: int = 0
    adapt_every: int = 500
    adapt_lo: float = 0.2
    adapt_hi: float = 0.6
    adapt_factor: float = 1.1
    adapt_until: int = -1
    chain_offset: int = 0
    trace_chains: int = 0
    record_every: int = 0
    record_chains: int = 0
    surrogate: MlpWeights | None = None
    param: str = "gamma"            # "bures": Algorithm 1 (4D^2 parameters)
    povm: np.ndarray | None = None  # [n, D, D] POVM elements (counts then has n entries)
    alpha: float = 0.5              # param "dirichlet": concentration of the weights
    intensity: np.ndarray | None = None  # Poisson counts with means intensity * p (one per count)


class Chains:
    """R chains of Algorithm 2 held in host arrays; run() may be called
    repeatedly to continue the same chains (resume is exact because every
    random number is a function of (seed, chain, step))."""

    def __init__(self, Q, counts, params: RunParams):
        self.Q = Q
        self.D, self.K, self.d = dims(Q, params.param)
        self.counts = np.ascontiguousarray(counts, dtype=np.int64).reshape(-1)
        self._povm = None
        if params.povm is not None:
            n = params.povm.shape[0]
            assert self.counts.shape == (n,) and n <= self.K * self.D
            self._povm = _interleave(params.povm)
            self.counts = np.concatenate([self.counts, np.zeros(self.K * self.D - n, dtype=np.int64)])
        assert self.counts.shape == (self.K * self.D,)
        self._intensity = None
        if params.intensity is not None:
            lam = np.asarray(params.intensity, dtype=np.float64).reshape(-1)
            self._intensity = np.ascontiguousarray(np.concatenate([lam, np.zeros(self.K * self.D - lam.size)]))
        self.p = params
        R, D2 = params.n_chains, self.D * self.D
        self.x = np.zeros((R, self.d))
        self.ll = np.zeros(R)
        self.beta = np.zeros(R)
        self.acc_win = np.zeros(R, dtype=np.int32)
        self.rho_cur = np.zeros((R, D2))
        self.s1 = np.zeros((R, D2))
        self.s2 = np.zeros((R, D2))
        self.n_stored = np.zeros(R, dtype=np.int64)
        self.s_cur = np.zeros(R)
        self.step = 0
        self.last = {}
        lib().orc_init_chains(C.byref(self._desc(0)), C.byref(self._state(None, None)))

    def _desc(self, n_steps):
        p = self.p
        self._mlp = C.pointer(p.surrogate._struct()) if p.surrogate is not None else None
        return _RunDesc(self.Q, _p(self.counts, c_int64_p), p.n_chains, p.chain_offset,
                        self.step, n_steps, p.thin, p.burn_in, p.beta0, p.adapt_every,
                        p.adapt_lo, p.adapt_hi, p.adapt_factor, p.adapt_until, p.seed,
                        self._mlp, p.trace_chains, p.record_every, p.record_chains,
                        PARAMS[p.param], _p(self._povm),
                        0 if p.povm is None else int(p.povm.shape[0]), float(p.alpha), _p(self._intensity))

    def _state(self, n_steps, bufs):
        R = self.p.n_chains
        bufs = bufs or {}
        return _State(_p(self.x), _p(self.ll), _p(self.beta), _p(self.acc_win, c_int32_p),
                      _p(self.rho_cur), _p(self.s1), _p(self.s2), _p(self.n_stored, c_int64_p),
                      _p(bufs.get("n_accepted"), c_int64_p), _p(bufs.get("n_stage1"), c_int64_p),
                      _p(bufs.get("n_near"), c_int64_p), _p(bufs.get("tr_llprop")),
                      _p(bufs.get("tr_logu")), _p(bufs.get("tr_accept"), c_int8_p),
                      _p(bufs.get("rec")), _p(self.s_cur))

    def run(self, n_steps):
        p, R, D2 = self.p, self.p.n_chains, self.D * self.D
        T = max(p.trace_chains, 0)
        n_rec = n_steps // p.record_every if p.record_every > 0 else 0
        bufs = {
            "n_accepted": np.zeros(R, dtype=np.int64),
            "n_stage1": np.zeros(R, dtype=np.int64),
            "n_near": np.zeros(R, dtype=np.int64),
            "tr_llprop": np.zeros((max(T, 1), n_steps)),
            "tr_logu": np.zeros((max(T, 1), n_steps)),
            "tr_accept": np.zeros((max(T, 1), n_steps), dtype=np.int8),
            "rec": np.zeros((max(p.record_chains, 1), max(n_rec, 1), D2)),
        }
        lib().orc_run_chains(C.byref(self._desc(n_steps)), C.byref(self._state(n_steps, bufs)))
        self.step += n_steps
        self.last = {
            "n_accepted": bufs["n_accepted"], "n_stage1": bufs["n_stage1"],
            "n_near": bufs["n_near"],
            "trace_llprop": bufs["tr_llprop"][:T], "trace_logu": bufs["tr_logu"][:T],
            "trace_accept": bufs["tr_accept"][:T],
            "records": bufs["rec"][:p.record_chains, :n_rec],
        }
        return self.last

    def pool(self):
        """Eq. (BME2): pooled mean rho (complex D x D), pooled E[(Re a)^2],
        E[(Im a)^2] and the between-chain standard error of each element."""
        D2 = self.D * self.D
        mean_p = np.zeros(D2)
        second_p = np.zeros(D2)
        lib().orc_pool(self.Q, self.p.n_chains, _p(self.s1), _p(self.s2),
                       _p(self.n_stored, c_int64_p), _p(mean_p), _p(second_p))
        return {"mean": unpack(mean_p.reshape(self.D, self.D)),
                "mean_packed": mean_p.reshape(self.D, self.D),
                "second_packed": second_p.reshape(self.D, self.D),
                "chain_means_packed": (self.s1 / np.maximum(self.n_stored, 1)[:, None]).reshape(
                    -1, self.D, self.D),
                "n_samples": int(self.n_stored.sum())}
