"""The C ABI refuses caller buffers that are not device memory of the
handle's device or that end before what a call would write, and the binding
refuses host, strided and mistyped tensors.

Each library-level case also carries a second, independent error that the
library detects later (resume on a fresh handle, or an unknown precision),
so no kernel is launched whatever the buffer check decides; the test tells
the two apart by the message.
"""
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


class _RawPointer:
    """Stands in for a tensor in a run descriptor: only data_ptr() is read."""

    def __init__(self, addr):
        self.addr = addr

    def data_ptr(self):
        return self.addr


def _run_raw(P, cfg, trace=None, record=None):
    rd = P._run_desc(cfg, trace, record)
    arr = (C.c_void_p * 1)(P._h)
    status = qst.lib().qst_run_chains(arr, 1, C.byref(rd), None)
    return status, qst.lib().qst_last_error().decode()


def test_host_pointer_in_a_run_is_refused():
    prob = synth.make_problem("c2")
    P = qst.Problem(2, prob.counts)
    host = np.zeros(64 * 10)
    cfg = qst.RunConfig(n_chains=64, n_steps=10, seed=1, resume=True)   # fresh handle: resume is an error too
    status, msg = _run_raw(P, cfg, trace=dict(chains=64, llprop=_RawPointer(host.ctypes.data)))
    assert status == qst.QST_ERR_INVALID and "trace_llprop is not device memory" in msg, (status, msg)


def test_buffer_shorter_than_the_run_is_refused():
    prob = synth.make_problem("c3")
    P = qst.Problem(4, prob.counts)
    buf = torch.zeros((64, 16, 16, 16), dtype=torch.float64, device="cuda")
    # 64 chains x 10^7 records x 256 doubles: far beyond any allocation
    cfg = qst.RunConfig(n_chains=64, n_steps=10 ** 7, seed=1, resume=True)
    status, msg = _run_raw(P, cfg, record=dict(every=1, chains=64, buf=buf))
    assert status == qst.QST_ERR_INVALID and "record_buf is smaller than the call needs" in msg, (status, msg)


def test_loglik_host_pointers_are_refused():
    prob = synth.make_problem("c2")
    P = qst.Problem(2, prob.counts)
    host = np.zeros(16 * 2 * 4)
    out = torch.zeros(4, dtype=torch.float64, device="cuda")
    bad_precision = 7
    st = qst.lib().qst_loglik(P._h, C.c_void_p(host.ctypes.data), 4, C.c_void_p(out.data_ptr()), qst.PATH_KRON,
                              bad_precision, None)
    msg = qst.lib().qst_last_error().decode()
    assert st == qst.QST_ERR_INVALID and "rho is not device memory" in msg, (st, msg)
    rho = torch.zeros((4, 4, 4, 2), dtype=torch.float64, device="cuda")
    outh = np.zeros(4)
    st = qst.lib().qst_loglik(P._h, C.c_void_p(rho.data_ptr()), 4, C.c_void_p(outh.ctypes.data), qst.PATH_KRON,
                              bad_precision, None)
    msg = qst.lib().qst_last_error().decode()
    assert st == qst.QST_ERR_INVALID and "ll_out is not device memory" in msg, (st, msg)
    # the library still works afterwards
    rho[:, :, :, 0] = torch.eye(4, dtype=torch.float64) / 4
    P.loglik(rho, out)
    torch.cuda.synchronize()
    assert np.all(np.isfinite(out.cpu().numpy()))


def test_binding_refuses_bad_tensors():
    prob = synth.make_problem("c2")
    P = qst.Problem(2, prob.counts)
    cfg = qst.RunConfig(n_chains=8, n_steps=4, seed=1)
    cases = [dict(chains=8, llprop=torch.zeros((8, 4), dtype=torch.float64)),                       # host
             dict(chains=8, llprop=torch.zeros((4, 8), dtype=torch.float64, device="cuda").t()),    # strided
             dict(chains=8, llprop=torch.zeros((8, 4), dtype=torch.float32, device="cuda"))]        # dtype
    for tr in cases:
        with pytest.raises(qst.QstError) as e:
            P.run(cfg, trace=tr)
        assert e.value.status == qst.QST_ERR_INVALID
    rho = torch.zeros((2, 4, 4, 2), dtype=torch.float32, device="cuda")
    with pytest.raises(qst.QstError):
        P.loglik(rho, torch.zeros(2, dtype=torch.float64, device="cuda"))
    # a good run still goes through
    st = P.run(cfg)
    assert st["proposed"] == 8 * 4


def test_binding_refuses_a_tensor_one_row_short():
    """A tensor carved by torch's caching allocator lies inside a larger
    block, so the library's allocation-extent check cannot see that it is
    short; the binding compares the element count with what the call writes
    and raises before anything is queued."""
    prob = synth.make_problem("c2")
    P = qst.Problem(2, prob.counts)
    R, T = 16, 8
    cfg = qst.RunConfig(n_chains=R, n_steps=T, seed=1)
    short = dict(chains=R, llprop=torch.zeros((R - 1, T), dtype=torch.float64, device="cuda"))
    with pytest.raises(qst.QstError) as e:
        P.run(cfg, trace=short)
    assert e.value.status == qst.QST_ERR_INVALID and "trace llprop" in str(e.value)
    rec = dict(every=2, chains=4, buf=torch.zeros((4, T // 2 - 1, 4, 4), dtype=torch.float64, device="cuda"))
    with pytest.raises(qst.QstError) as e:
        P.run(cfg, record=rec)
    assert e.value.status == qst.QST_ERR_INVALID and "record buf" in str(e.value)
    rho = torch.zeros((2, 4, 4, 2), dtype=torch.float64, device="cuda")
    with pytest.raises(qst.QstError) as e:
        P.loglik(rho[:1], torch.zeros(2, dtype=torch.float64, device="cuda"))
    assert e.value.status == qst.QST_ERR_INVALID and "rho" in str(e.value)
    # nothing was launched: the handle has not run yet
    with pytest.raises(qst.QstError) as e:
        P.pool()
    assert e.value.status == qst.QST_ERR_STATE
    ok = dict(chains=R, llprop=torch.zeros((R, T), dtype=torch.float64, device="cuda"))
    assert P.run(cfg, trace=ok)["proposed"] == R * T


def test_gather_rows_checks_every_index():
    n_rows, width = 40, 32
    x = torch.arange(n_rows * width, device="cuda").to(torch.bfloat16).reshape(n_rows, width)
    y = torch.arange(n_rows, dtype=torch.float32, device="cuda")
    xo = torch.zeros((3, width), dtype=torch.bfloat16, device="cuda")
    yo = torch.zeros(3, dtype=torch.float32, device="cuda")
    for bad in ([0, n_rows, 1], [5, -1, 2]):
        idx = torch.tensor(bad, dtype=torch.int64, device="cuda")
        with pytest.raises(qst.QstError) as e:
            qst.gather_rows(x, y, idx, xo, yo)
        assert e.value.status == qst.QST_ERR_INVALID and "is not a row index" in str(e.value)
    assert float(yo.abs().sum()) == 0.0        # nothing was written
    idx = torch.tensor([n_rows - 1, 0, 7], dtype=torch.int64, device="cuda")
    qst.gather_rows(x, y, idx, xo, yo)
    torch.cuda.synchronize()
    assert yo.cpu().tolist() == [n_rows - 1, 0, 7]
    assert torch.equal(xo.cpu(), x[[n_rows - 1, 0, 7]].cpu())
