"""The C-ABI library loads and exports every function include/qst.h declares;
argument validation that happens before any device work."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2501_17334_amd import qst

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "qst.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qst_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    lib = ctypes.CDLL(qst.LIB_PATH)
    names = declared_functions()
    assert {"qst_init_problem", "qst_run_chains", "qst_pool_moments"} <= set(names)
    for n in names:
        assert hasattr(lib, n), n


def test_version_and_error_string():
    assert qst.lib().qst_version().startswith(b"qst-gfx950")
    assert isinstance(qst.lib().qst_last_error(), bytes)


@pytest.mark.parametrize("Q", [0, 7, -1])
def test_bad_qubit_count_is_invalid(Q):
    counts = np.zeros(max(1, 3 ** max(Q, 0) * 2 ** max(Q, 0)), dtype=np.int64)
    with pytest.raises(qst.QstError) as e:
        _init(Q, counts)
    assert e.value.status == qst.QST_ERR_INVALID


def _init(Q, counts):
    desc = qst._ProblemDesc(Q, counts.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), 0, 0, 0)
    h = ctypes.c_void_p()
    qst._check(qst.lib().qst_init_problem(ctypes.byref(desc), ctypes.byref(h)))


def test_null_arguments_are_invalid():
    h = ctypes.c_void_p()
    assert qst.lib().qst_init_problem(None, ctypes.byref(h)) == qst.QST_ERR_INVALID
    assert qst.lib().qst_pool_moments(None, None, None, None, None) == qst.QST_ERR_INVALID
    assert qst.lib().qst_run_chains(None, 0, None, None) == qst.QST_ERR_INVALID


def test_binding_refuses_host_and_strided_tensors():
    """Tensors handed to the library as raw pointers must be contiguous GPU
    tensors of the documented dtype; the binding refuses anything else before
    any library call."""
    import torch
    with pytest.raises(qst.QstError) as e:
        qst._dev_tensor(torch.zeros(4, dtype=torch.float64), ("float64",), "buf")
    assert e.value.status == qst.QST_ERR_INVALID and "GPU tensor" in str(e.value)
    with pytest.raises(qst.QstError):
        qst._dev_tensor(np.zeros(4), ("float64",), "buf")
    with pytest.raises(qst.QstError):
        qst._check_run_buffers(dict(chains=1, llprop=torch.zeros((1, 4), dtype=torch.float64)), None, None)
    qst._dev_tensor(None, ("float64",), "buf")          # absent buffers are allowed
    qst._check_run_buffers(None, None, None)


def test_batch_tiles_use_the_tuned_single_problem_teams():
    """Batch tiles run with a fixed team per qubit count (qst_get_batch_shape);
    a batch problem equals its solo run with that team, so the committed
    tuning table must choose the same team for single-problem launches, and
    the shape must be one the library compiles."""
    import json
    with open(os.path.join(ROOT, "paper_2501_17334_amd", "tune_gfx950.json")) as f:
        tuned = json.load(f)
    for Q in range(1, 7):
        team, wg = qst.get_batch_shape(Q)
        assert wg % team == 0 and wg in (256, 1024)
        assert tuned[str(Q)]["team"] == team, (Q, tuned[str(Q)]["team"], team)
        teams, wgs = (ctypes.c_int32 * 16)(), (ctypes.c_int32 * 16)()
        n = ctypes.c_int32()
        qst._check(qst.lib().qst_list_launch_shapes(Q, teams, wgs, 16, ctypes.byref(n)))
        assert team in list(teams)[:n.value]
    with pytest.raises(qst.QstError):
        qst.get_batch_shape(7)
