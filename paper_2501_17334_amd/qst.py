"""Thin Python binding of the C ABI in include/qst.h (argument marshalling only).

Every computation runs in libqst.so's HIP kernels; this module converts
Python arguments to the C structs, passes torch device pointers and the
current HIP stream, and raises on any non-zero status.  If libqst.so is
missing it raises: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqst.so")

QST_OK, QST_ERR_INVALID, QST_ERR_NOMEM, QST_ERR_DEVICE, QST_ERR_STATE, QST_ERR_UNSUPPORTED = range(6)
FP64, FP32, BF16X3 = 0, 1, 2
PATH_AUTO, PATH_DENSE, PATH_KRON = 0, 1, 2

_PREC = {"fp64": FP64, "fp32": FP32, "bf16x3": BF16X3}
_PATH = {"auto": PATH_AUTO, "dense": PATH_DENSE, "kron": PATH_KRON}


class QstError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"qst status {status}: {msg}")
        self.status = status


class _ProblemDesc(C.Structure):
    _fields_ = [("n_qubits", C.c_int32), ("counts", C.POINTER(C.c_int64)),
                ("precision", C.c_int), ("path", C.c_int), ("device", C.c_int32), ("param", C.c_int),
                ("povm", C.POINTER(C.c_double)), ("n_povm", C.c_int32), ("alpha", C.c_double),
                ("intensity", C.POINTER(C.c_double))]


# parameterisation of rho(x): the Gaussian/gamma form (2D^2+D parameters) or
# the paper's Algorithm 1, the Bures draw (4D^2 parameters)
_PARAM = {"gamma": 0, "bures": 1, "dirichlet": 2}


class _Surrogate(C.Structure):
    _fields_ = [("h1", C.c_int32), ("h2", C.c_int32), ("W1", C.c_void_p), ("b1", C.c_void_p),
                ("W2", C.c_void_p), ("b2", C.c_void_p), ("w3", C.c_void_p), ("b3", C.c_float),
                ("out_scale", C.c_float), ("out_shift", C.c_float), ("model", C.c_void_p)]


class _RunDesc(C.Structure):
    _fields_ = [("n_chains", C.c_int64), ("n_steps", C.c_int64), ("thin", C.c_int32),
                ("burn_in", C.c_int64), ("beta0", C.c_double), ("adapt_every", C.c_int32),
                ("adapt_lo", C.c_double), ("adapt_hi", C.c_double), ("adapt_factor", C.c_double),
                ("adapt_until", C.c_int64), ("seed", C.c_uint64), ("resume", C.c_int32),
                ("surrogate", C.POINTER(_Surrogate)), ("trace_chains", C.c_int32),
                ("trace_llprop", C.c_void_p), ("trace_logu", C.c_void_p), ("trace_accept", C.c_void_p),
                ("record_every", C.c_int32), ("record_chains", C.c_int32), ("record_buf", C.c_void_p),
                ("pair_every", C.c_int32), ("pair_chains", C.c_int32), ("pair_x", C.c_void_p),
                ("pair_ll", C.c_void_p), ("stream", C.c_void_p), ("chain_offset", C.c_int64)]


class _RunStats(C.Structure):
    _fields_ = [("proposed", C.c_int64), ("accepted", C.c_int64), ("stage1_passed", C.c_int64),
                ("near_threshold", C.c_int64), ("nonfinite_chains", C.c_int64),
                ("beta_min", C.c_double), ("beta_max", C.c_double)]


_lib = None


def lib():
    """Load libqst.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} (run paper_2501_17334_amd/build.py)")
        # torch ships its own HIP runtime under the same soname; loading torch
        # first makes libqst.so bind to that one runtime, so torch's streams and
        # allocations are the library's too
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.qst_init_problem.argtypes = [C.POINTER(_ProblemDesc), C.POINTER(vp)]
        L.qst_run_chains.argtypes = [C.POINTER(vp), C.c_int32, C.POINTER(_RunDesc), C.POINTER(_RunStats)]
        L.qst_pool_moments.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                       C.POINTER(C.c_double), C.POINTER(C.c_int64)]
        L.qst_chain_state.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                      C.POINTER(C.c_double), C.POINTER(C.c_int64)]
        L.qst_chain_moments.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.qst_set_chain_state.argtypes = [vp, C.c_int64, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                          C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_int64)]
        L.qst_loglik.argtypes = [vp, vp, C.c_int64, vp, C.c_int, C.c_int, vp]
        L.qst_acf.argtypes = [vp, C.c_int64, C.c_int64, C.c_int32, C.c_int32, C.POINTER(C.c_double), vp]
        L.qst_set_launch_shape.argtypes = [C.c_int32, C.c_int32, C.c_int32]
        L.qst_get_launch_shape.argtypes = [C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.qst_get_batch_shape.argtypes = [C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.qst_set_auto_path.argtypes = [C.c_int32, C.c_int, C.c_int]
        L.qst_get_auto_path.argtypes = [C.c_int32, C.c_int, C.POINTER(C.c_int)]
        L.qst_list_launch_shapes.argtypes = [C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.c_int32,
                                             C.POINTER(C.c_int32)]
        L.qst_mlp_create.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.POINTER(vp)]
        L.qst_mlp_free.argtypes = [vp]
        L.qst_mlp_free.restype = None
        L.qst_mlp_num_params.argtypes = [vp]
        L.qst_mlp_num_params.restype = C.c_int64
        L.qst_mlp_set_params.argtypes = [vp, C.POINTER(C.c_float), C.c_int64, C.c_float, C.c_float]
        L.qst_mlp_get_params.argtypes = [vp, C.POINTER(C.c_float), C.c_int64]
        L.qst_mlp_gradients.argtypes = [vp, vp, vp, C.c_int64, C.POINTER(C.c_float), C.POINTER(C.c_float), vp]
        L.qst_mlp_train_step.argtypes = [vp, vp, vp, C.c_int64, C.c_float, C.POINTER(C.c_float), vp]
        L.qst_mlp_predict.argtypes = [vp, vp, C.c_int64, vp, vp]
        L.qst_mlp_surrogate.argtypes = [vp, C.POINTER(_Surrogate)]
        L.qst_mlp_targets.argtypes = [vp, C.c_int64, vp, C.POINTER(C.c_double), C.POINTER(C.c_double), vp]
        L.qst_gather_rows.argtypes = [vp, C.c_int32, vp, C.c_int64, vp, C.c_int64, vp, vp, vp]
        L.qst_free_problem.argtypes = [vp]
        L.qst_free_problem.restype = None
        L.qst_last_error.restype = C.c_char_p
        L.qst_version.restype = C.c_char_p
        for f in ("qst_init_problem", "qst_run_chains", "qst_pool_moments", "qst_chain_state", "qst_chain_moments",
                  "qst_set_chain_state", "qst_set_auto_path", "qst_get_auto_path",
                  "qst_loglik", "qst_acf", "qst_set_launch_shape", "qst_get_launch_shape", "qst_get_batch_shape",
                  "qst_list_launch_shapes", "qst_mlp_create", "qst_mlp_set_params", "qst_mlp_get_params",
                  "qst_mlp_gradients", "qst_mlp_train_step", "qst_mlp_predict", "qst_mlp_surrogate",
                  "qst_mlp_targets", "qst_gather_rows"):
            getattr(L, f).restype = C.c_int
        _lib = L
        _install_tuned_shapes()
    return _lib


def _install_tuned_shapes():
    """Apply the autotuner's saved launch shapes (tune_gfx950.json), if any."""
    import json
    path = os.path.join(_HERE, "tune_gfx950.json")
    if not os.path.exists(path):
        return
    with open(path) as f:
        table = json.load(f)
    for q, ent in table.items():
        if q.isdigit():
            _lib.qst_set_launch_shape(int(q), int(ent["team"]), int(ent["workgroup"]))
    for q, per in table.get("paths", {}).items():
        for prec, ent in per.items():
            _lib.qst_set_auto_path(int(q), _PREC[prec], _PATH[ent["path"]])


def _check(status):
    if status != QST_OK:
        raise QstError(status, lib().qst_last_error().decode())


def _dptr(t):
    """Device pointer of a torch tensor (or None)."""
    return None if t is None else C.c_void_p(t.data_ptr())


def _dev_tensor(t, dtypes, name):
    """A torch tensor the library reads or writes through a raw pointer: on
    a GPU, contiguous, of one of the given dtype names (the library checks
    the memory type and the extent of the allocation itself)."""
    import torch
    if t is None:
        return
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise QstError(QST_ERR_INVALID, f"{name} must be a GPU tensor")
    if not t.is_contiguous():
        raise QstError(QST_ERR_INVALID, f"{name} must be contiguous")
    if str(t.dtype).replace("torch.", "") not in dtypes:
        raise QstError(QST_ERR_INVALID, f"{name} must have dtype {' or '.join(dtypes)}, not {t.dtype}")


def _need(t, count, name):
    """The library writes `count` elements through t's pointer: refuse a
    shorter tensor (the library's own check only sees the end of the
    allocation, which for a torch tensor is the caching allocator's block)."""
    if t is not None and t.numel() < count:
        raise QstError(QST_ERR_INVALID, f"{name} holds {t.numel()} elements; the call writes {count}")


def _check_run_buffers(trace, record, pairs, cfg=None, D2=None, width=None):
    trace, record, pairs = trace or {}, record or {}, pairs or {}
    _dev_tensor(trace.get("llprop"), ("float64",), "trace llprop")
    _dev_tensor(trace.get("logu"), ("float64",), "trace logu")
    _dev_tensor(trace.get("accept"), ("int8", "uint8"), "trace accept")
    _dev_tensor(record.get("buf"), ("float64",), "record buf")
    _dev_tensor(pairs.get("x"), ("bfloat16", "int16", "uint16"), "pairs x")
    _dev_tensor(pairs.get("ll"), ("float64",), "pairs ll")
    if cfg is None:
        return
    R, T = cfg.n_chains, cfg.n_steps
    tc = min(trace.get("chains", 0), R)
    for k in ("llprop", "logu", "accept"):
        _need(trace.get(k), tc * T, f"trace {k}")
    if record.get("every", 0) > 0 and record.get("chains", 0) > 0:
        _need(record.get("buf"), min(record["chains"], R) * (T // record["every"]) * D2, "record buf")
    if pairs.get("every", 0) > 0 and pairs.get("chains", 0) > 0:
        slots, pc = T // pairs["every"], pairs["chains"]
        rows = (slots - 1) * pc + min(pc, R) if slots > 0 else 0
        _need(pairs.get("x"), rows * width, "pairs x")
        _need(pairs.get("ll"), rows, "pairs ll")


def _f64(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def current_stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


@dataclass
class RunConfig:
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
    resume: bool = False
    chain_offset: int = 0


class Problem:
    """A tomography problem on one GPU (qst_init_problem / qst_free_problem)."""

    def __init__(self, n_qubits, counts, precision="fp64", path="auto", device=0, param="gamma", povm=None,
                 alpha=0.5, intensity=None):
        """param: "gamma" (default), "bures" (Algorithm 1) or "dirichlet"
        (Dirichlet(alpha) weights); povm: optional [n, D, D] complex POVM
        elements in place of the Pauli settings (counts then has n entries;
        dense path, FP64 or FP32); intensity: optional Poisson intensities,
        one per count (count m ~ Poisson(intensity_m p_m))."""
        self.Q = int(n_qubits)
        self.D = 2 ** self.Q
        self.K = 3 ** self.Q
        self.param = param
        self.d = 4 * self.D * self.D if param == "bures" else 2 * self.D * self.D + self.D
        self.counts = np.ascontiguousarray(counts, dtype=np.int64).reshape(-1)
        self._povm = None
        n_povm = 0
        if povm is not None:
            povm = np.asarray(povm, dtype=complex)
            n_povm = povm.shape[0]
            if povm.shape != (n_povm, self.D, self.D) or self.counts.size != n_povm:
                raise ValueError("povm must be [n, D, D] with one count per element")
            self._povm = np.ascontiguousarray(np.stack([povm.real, povm.imag], axis=-1))
        elif self.counts.size != self.K * self.D:
            raise ValueError("counts must have 3^Q * 2^Q entries")
        self._intensity = None
        if intensity is not None:
            self._intensity = np.ascontiguousarray(intensity, dtype=np.float64).reshape(-1)
            if self._intensity.size != self.counts.size:
                raise ValueError("intensity must have one entry per count")
        desc = _ProblemDesc(self.Q, self.counts.ctypes.data_as(C.POINTER(C.c_int64)),
                            _PREC[precision], _PATH[path], device, _PARAM[param],
                            _f64(self._povm) if self._povm is not None else None, n_povm, float(alpha),
                            _f64(self._intensity) if self._intensity is not None else None)
        h = C.c_void_p()
        _check(lib().qst_init_problem(C.byref(desc), C.byref(h)))
        self._h = h
        self.n_chains = 0

    def close(self):
        if getattr(self, "_h", None):
            lib().qst_free_problem(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def pair_width(self):
        """Width of a surrogate input row: d rounded up to a multiple of 32."""
        return (self.d + 31) // 32 * 32

    def _run_desc(self, cfg: RunConfig, trace=None, record=None, stream=None, surrogate=None, pairs=None):
        trace = trace or {}
        record = record or {}
        pairs = pairs or {}
        self._sur = C.pointer(surrogate) if surrogate is not None else None
        return _RunDesc(cfg.n_chains, cfg.n_steps, cfg.thin, cfg.burn_in, cfg.beta0, cfg.adapt_every,
                        cfg.adapt_lo, cfg.adapt_hi, cfg.adapt_factor, cfg.adapt_until, cfg.seed,
                        1 if cfg.resume else 0, self._sur, trace.get("chains", 0),
                        _dptr(trace.get("llprop")), _dptr(trace.get("logu")),
                        _dptr(trace.get("accept")), record.get("every", 0), record.get("chains", 0),
                        _dptr(record.get("buf")), pairs.get("every", 0), pairs.get("chains", 0),
                        _dptr(pairs.get("x")), _dptr(pairs.get("ll")),
                        stream if stream is not None else current_stream(), cfg.chain_offset)

    def run(self, cfg: RunConfig, trace=None, record=None, stats=True, stream=None, surrogate=None, pairs=None):
        """qst_run_chains on this problem alone.  trace: dict(chains=k, llprop=,
        logu=, accept=) torch device tensors [k, n_steps]; record: dict(every=,
        chains=, buf=) torch device tensor [chains, n_steps // every, D, D];
        surrogate: an Mlp.surrogate() (delayed acceptance); pairs: dict(every=,
        chains=, x= bfloat16 [n_steps // every, chains, pair_width], ll= float64
        [n_steps // every, chains]): the proposal of step (s + 1) * every of
        chain c and its log L in row s * chains + c."""
        _check_run_buffers(trace, record, pairs, cfg, self.D * self.D, self.pair_width)
        rd = self._run_desc(cfg, trace, record, stream, surrogate, pairs)
        arr = (C.c_void_p * 1)(self._h)
        st = _RunStats()
        _check(lib().qst_run_chains(arr, 1, C.byref(rd), C.byref(st) if stats else None))
        self.n_chains = cfg.n_chains
        if stats:
            return {f: getattr(st, f) for f, _ in _RunStats._fields_}
        return None

    def pool(self):
        """qst_pool_moments: mean rho, second moments, standard errors."""
        D2 = self.D * self.D
        mean = np.zeros(2 * D2)
        second = np.zeros(2 * D2)
        se = np.zeros(2 * D2)
        n = C.c_int64()
        _check(lib().qst_pool_moments(self._h, _f64(mean), _f64(second), _f64(se), C.byref(n)))
        cplx = np.array([1.0, 1j])
        return {"mean": mean.reshape(self.D, self.D, 2) @ cplx,
                "second_re": second.reshape(self.D, self.D, 2)[..., 0],
                "second_im": second.reshape(self.D, self.D, 2)[..., 1],
                "se_re": se.reshape(self.D, self.D, 2)[..., 0],
                "se_im": se.reshape(self.D, self.D, 2)[..., 1],
                "n_samples": int(n.value)}

    def state(self):
        """qst_chain_state: (x [R, d], loglik [R], beta [R], n_stored [R])."""
        R = self.n_chains
        x = np.zeros((R, self.d))
        ll = np.zeros(R)
        beta = np.zeros(R)
        nst = np.zeros(R, dtype=np.int64)
        _check(lib().qst_chain_state(self._h, _f64(x), _f64(ll), _f64(beta),
                                     nst.ctypes.data_as(C.POINTER(C.c_int64))))
        return x, ll, beta, nst

    def set_state(self, x=None, beta=None, step=-1, s1=None, s2=None, n_stored=None):
        """qst_set_chain_state from host arrays (None keeps): x [R, d],
        beta [R], s1 / s2 [R, D, D] (as moments() returns them), n_stored [R];
        step >= 0 sets the steps already run.  The next run with resume=True
        evaluates a new x first."""
        R, D = self.n_chains, self.D

        def arr(a, shape, dtype=np.float64):
            if a is None:
                return None
            a = np.ascontiguousarray(a, dtype=dtype)
            if a.shape != shape:
                raise ValueError(f"expected shape {shape}, got {a.shape}")
            return a
        xa, ba = arr(x, (R, self.d)), arr(beta, (R,))
        s1a, s2a = arr(s1, (R, D, D)), arr(s2, (R, D, D))
        na = arr(n_stored, (R,), np.int64)
        f = lambda a: _f64(a) if a is not None else None
        _check(lib().qst_set_chain_state(self._h, int(step), f(xa), f(ba), f(s1a), f(s2a),
                                         na.ctypes.data_as(C.POINTER(C.c_int64)) if na is not None else None))

    def moments(self):
        """qst_chain_moments: per-chain sums (s1 [R, D, D], s2 [R, D, D]) of the
        packed rho of the stored samples."""
        R, D = self.n_chains, self.D
        s1 = np.zeros((R, D, D))
        s2 = np.zeros((R, D, D))
        _check(lib().qst_chain_moments(self._h, _f64(s1), _f64(s2)))
        return s1, s2

    def loglik(self, rho_dev, out_dev, path="auto", precision="fp64", stream=None):
        """qst_loglik on torch device tensors: rho [n, D, D] complex128 (or
        float64 [n, D, D, 2]), out float64 [n]."""
        _dev_tensor(rho_dev, ("complex128", "float64"), "rho")
        _dev_tensor(out_dev, ("float64",), "out")
        n = out_dev.numel()
        D2 = self.D * self.D
        _need(rho_dev, n * D2 * (1 if rho_dev.is_complex() else 2), "rho")
        _check(lib().qst_loglik(self._h, C.c_void_p(rho_dev.data_ptr()), n, C.c_void_p(out_dev.data_ptr()),
                                _PATH[path], _PREC[precision],
                                stream if stream is not None else current_stream()))


class Mlp:
    """The MLP surrogate (qst_mlp_*): parameters, training step, prediction."""

    def __init__(self, d_in, h1=512, h2=512, device=0):
        h = C.c_void_p()
        _check(lib().qst_mlp_create(d_in, h1, h2, device, C.byref(h)))
        self._h = h
        self.d, self.h1, self.h2 = d_in, h1, h2
        self.n_params = int(lib().qst_mlp_num_params(h))

    def close(self):
        if getattr(self, "_h", None):
            lib().qst_mlp_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, flat, out_scale=1.0, out_shift=0.0):
        a = np.ascontiguousarray(flat, dtype=np.float32)
        _check(lib().qst_mlp_set_params(self._h, a.ctypes.data_as(C.POINTER(C.c_float)), a.size,
                                        out_scale, out_shift))

    def get_params(self):
        a = np.zeros(self.n_params, dtype=np.float32)
        _check(lib().qst_mlp_get_params(self._h, a.ctypes.data_as(C.POINTER(C.c_float)), a.size))
        return a

    @staticmethod
    def _bf16(x):
        import torch
        return x.to(torch.bfloat16).contiguous()

    def gradients(self, x, y):
        """x: torch device tensor [n, d] (any float dtype; rounded to BF16), y [n]."""
        import torch
        xb = self._bf16(x)
        yf = y.to(torch.float32).contiguous()
        g = np.zeros(self.n_params, dtype=np.float32)
        loss = C.c_float()
        _check(lib().qst_mlp_gradients(self._h, C.c_void_p(xb.data_ptr()), C.c_void_p(yf.data_ptr()), xb.shape[0],
                                       g.ctypes.data_as(C.POINTER(C.c_float)), C.byref(loss), current_stream()))
        return g, loss.value

    def train_step(self, x_bf16, y_f32, lr, want_loss=False, rows=None, offset=0):
        """One Adam step on rows [offset, offset + rows) of device tensors
        x_bf16 [N, d] (bfloat16) and y_f32 [N] (pointer arithmetic only)."""
        _dev_tensor(x_bf16, ("bfloat16",), "x")
        _dev_tensor(y_f32, ("float32",), "y")
        n = x_bf16.shape[0] if rows is None else rows
        if offset < 0 or offset + n > x_bf16.shape[0] or offset + n > y_f32.numel():
            raise QstError(QST_ERR_INVALID, f"rows [{offset}, {offset + n}) exceed x ({x_bf16.shape[0]} rows) "
                                            f"or y ({y_f32.numel()} values)")
        xp = x_bf16.data_ptr() + offset * x_bf16.shape[1] * 2
        yp = y_f32.data_ptr() + offset * 4
        loss = C.c_float()
        _check(lib().qst_mlp_train_step(self._h, C.c_void_p(xp), C.c_void_p(yp), n, lr,
                                        C.byref(loss) if want_loss else None, current_stream()))
        return loss.value if want_loss else None

    def predict(self, x):
        import torch
        xb = self._bf16(x)
        out = torch.empty(xb.shape[0], dtype=torch.float32, device=xb.device)
        _check(lib().qst_mlp_predict(self._h, C.c_void_p(xb.data_ptr()), xb.shape[0], C.c_void_p(out.data_ptr()),
                                     current_stream()))
        return out

    def surrogate(self):
        s = _Surrogate()
        _check(lib().qst_mlp_surrogate(self._h, C.byref(s)))
        return s


def standardise_targets(ll_dev, y_dev, stream=None):
    """qst_mlp_targets: y = (ll - mean) / sd on the device; returns (mean, sd)."""
    _dev_tensor(ll_dev, ("float64",), "ll")
    _dev_tensor(y_dev, ("float32",), "y")
    _need(y_dev, ll_dev.numel(), "y")
    mean, sd = C.c_double(), C.c_double()
    _check(lib().qst_mlp_targets(C.c_void_p(ll_dev.data_ptr()), ll_dev.numel(), C.c_void_p(y_dev.data_ptr()),
                                 C.byref(mean), C.byref(sd), stream if stream is not None else current_stream()))
    return mean.value, sd.value


def gather_rows(x, y, idx, xo, yo, stream=None):
    """qst_gather_rows on torch device tensors (idx int64)."""
    for t, dt, name in ((x, ("bfloat16",), "x"), (y, ("float32",), "y"), (idx, ("int64",), "idx"),
                        (xo, ("bfloat16",), "xo"), (yo, ("float32",), "yo")):
        _dev_tensor(t, dt, name)
    n_rows, n = x.shape[0], idx.numel()
    _need(y, n_rows, "y")
    _need(xo, n * x.shape[1], "xo")
    _need(yo, n, "yo")
    _check(lib().qst_gather_rows(C.c_void_p(x.data_ptr()), x.shape[1], C.c_void_p(y.data_ptr()), n_rows,
                                 C.c_void_p(idx.data_ptr()), n, C.c_void_p(xo.data_ptr()),
                                 C.c_void_p(yo.data_ptr()), stream if stream is not None else current_stream()))


def set_launch_shape(n_qubits, team, workgroup):
    _check(lib().qst_set_launch_shape(n_qubits, team, workgroup))


def get_launch_shape(n_qubits):
    t, w = C.c_int32(), C.c_int32()
    _check(lib().qst_get_launch_shape(n_qubits, C.byref(t), C.byref(w)))
    return t.value, w.value


def get_batch_shape(n_qubits):
    """(team, workgroup) of n_qubits tiles inside an uneven batch."""
    t, w = C.c_int32(), C.c_int32()
    _check(lib().qst_get_batch_shape(n_qubits, C.byref(t), C.byref(w)))
    return t.value, w.value


def set_auto_path(n_qubits, precision, path):
    _check(lib().qst_set_auto_path(n_qubits, _PREC[precision], _PATH[path]))


def get_auto_path(n_qubits, precision):
    v = C.c_int()
    _check(lib().qst_get_auto_path(n_qubits, _PREC[precision], C.byref(v)))
    return {PATH_AUTO: "auto", PATH_DENSE: "dense", PATH_KRON: "kron"}[v.value]


def list_launch_shapes(n_qubits):
    n = C.c_int32()
    _check(lib().qst_list_launch_shapes(n_qubits, None, None, 0, C.byref(n)))
    T = (C.c_int32 * n.value)()
    W = (C.c_int32 * n.value)()
    _check(lib().qst_list_launch_shapes(n_qubits, T, W, n.value, C.byref(n)))
    return list(zip(T, W))


def run_batch(problems, configs, stats=True, stream=None, traces=None):
    """qst_run_chains on several problems at once (the uneven batch: one
    work-queue launch per qubit count and precision).
    traces: optional list (one entry per problem, None or a trace dict as in
    Problem.run)."""
    n = len(problems)
    traces = traces or [None] * n
    for p, c, t in zip(problems, configs, traces):
        _check_run_buffers(t, None, None, c, p.D * p.D, p.pair_width)
    rds = (_RunDesc * n)(*[p._run_desc(c, t, None, stream) for p, c, t in zip(problems, configs, traces)])
    hs = (C.c_void_p * n)(*[p._h for p in problems])
    st = (_RunStats * n)()
    _check(lib().qst_run_chains(hs, n, rds, st if stats else None))
    for p, c in zip(problems, configs):
        p.n_chains = c.n_chains
    if stats:
        return [{f: getattr(s, f) for f, _ in _RunStats._fields_} for s in st]
    return None


def acf(records_dev, l_max=200, stream=None):
    """qst_acf: pooled c[0..l_max] (Eq. (ACFrho)) of recorded packed samples,
    a torch device tensor [chains, N, D, D] float64."""
    _dev_tensor(records_dev, ("float64",), "records")
    C_, N, D, _ = records_dev.shape
    Q = int(D).bit_length() - 1
    out = np.zeros(l_max + 1)
    _check(lib().qst_acf(C.c_void_p(records_dev.data_ptr()), C_, N, Q, l_max, _f64(out),
                         stream if stream is not None else current_stream()))
    return out


def iact(c):
    """Eq. (IACT): tau = 1 + 2 sum_{l>=1} c[l]."""
    return 1.0 + 2.0 * float(np.sum(c[1:]))


def _run_desc(problem, cfg, trace, record, stream):
    return problem._run_desc(cfg, trace, record, stream)
