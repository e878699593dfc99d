"""The allocation-free pooling call qst_pool_moments_static, through the C
ABI, against qst_pool_moments on the same handles: two calls in a row, the
second on a smaller problem (fewer chains, fewer qubits), each bit for bit
equal to the allocating call; a problem too large for the static scratch is
refused before anything is queued."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_2501_17334_amd import qst, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _lib():
    L = qst.lib()
    L.qst_pool_moments_static.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    L.qst_pool_moments_static.restype = C.c_int
    return L


def _static_pool(P, stream):
    D2 = P.D * P.D
    out = torch.full((6 * D2,), float("nan"), dtype=torch.float64, device="cuda")
    n = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    st = _lib().qst_pool_moments_static(P._h, C.c_void_p(out.data_ptr()), C.c_void_p(n.data_ptr()),
                                        C.c_void_p(stream.cuda_stream))
    assert st == qst.QST_OK, qst.lib().qst_last_error().decode()
    return out, n


def _allocating_pool(P):
    D2 = P.D * P.D
    mean, second, se = np.zeros(2 * D2), np.zeros(2 * D2), np.zeros(2 * D2)
    n = C.c_int64()
    dp = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
    st = qst.lib().qst_pool_moments(P._h, dp(mean), dp(second), dp(se), C.byref(n))
    assert st == qst.QST_OK
    return np.concatenate([mean, second, se]), n.value


@pytest.mark.parametrize("first,second", [(("c3", 3000), ("c2", 700)), (("c5_0", 2048), ("c1", 64))])
def test_static_pool_equals_allocating_pool(first, second):
    stream = torch.cuda.Stream()
    for name, R in (first, second):
        prob = synth.make_problem(name)
        print(f"[no-alloc] {name}: Q={prob.n_qubits} R={R}", flush=True)
        P = qst.Problem(prob.n_qubits, prob.counts)
        with torch.cuda.stream(stream):
            P.run(qst.RunConfig(n_chains=R, n_steps=30, seed=prob.seed, beta0=0.02, adapt_every=10, burn_in=5),
                  stats=False)
            out, n = _static_pool(P, stream)
        want, n_want = _allocating_pool(P)
        stream.synchronize()
        torch.cuda.synchronize()
        assert int(n.cpu()[0]) == n_want == R * 25
        assert np.array_equal(out.cpu().numpy(), want), np.max(np.abs(out.cpu().numpy() - want))
        P.close()


def test_static_pool_refuses_what_does_not_fit():
    prob = synth.make_problem("c5_0")           # 6 qubits: 163,848 bytes of scratch per 256 chains
    P = qst.Problem(prob.n_qubits, prob.counts)
    P.run(qst.RunConfig(n_chains=26113 + 256, n_steps=0, seed=1, beta0=0.02), stats=False)
    out = torch.zeros(6 * 4096, dtype=torch.float64, device="cuda")
    n = torch.zeros(1, dtype=torch.int64, device="cuda")
    st = _lib().qst_pool_moments_static(P._h, C.c_void_p(out.data_ptr()), C.c_void_p(n.data_ptr()), None)
    assert st == qst.QST_ERR_INVALID and "scratch" in qst.lib().qst_last_error().decode()
    fresh = qst.Problem(1, synth.make_problem("c1").counts)
    st = _lib().qst_pool_moments_static(fresh._h, C.c_void_p(out.data_ptr()), C.c_void_p(n.data_ptr()), None)
    assert st == qst.QST_ERR_STATE
