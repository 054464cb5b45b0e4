"""CPU-side checks of the C ABI: the library loads, exports every function the
header declares, and its host-only entry points behave (no GPU compute here)."""
import ctypes
import os
import re

import numpy as np
import pytest

import graphgen as gg
from conftest import ROOT, golden_rows

kh = pytest.importorskip("paper_2112_06154_amd.khcore")

HEADER = os.path.join(ROOT, "include", "khcore.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(kh_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = kh.lib()
    names = declared_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(L, name), name
    assert sorted(kh.EXPORTED) == names


def test_status_strings():
    for code in range(0, -9, -1):
        s = kh.status_str(code)
        assert s.startswith("KH_")


def test_buffer_size_table1():
    for name, n, printed in golden_rows("table1_M.txt"):
        assert kh.buffer_size(int(n), 0.5, 0.05) == int(printed), name
    assert kh.buffer_size(0, 0.5) == -1
    assert kh.buffer_size(10, 0.0) == -1
    assert kh.buffer_size(10, 0.5, 1.5) == -1


def test_validate_csr_accepts_canonical():
    for g in (gg.erdos_renyi(300, 900, seed=1), gg.star(20), gg.empty(5), gg.path(2)):
        assert kh.validate_csr(g.n, g.row_ptr, g.col) == kh.KH_OK


@pytest.mark.parametrize("case", ["asym", "loop", "dup", "unsorted", "range", "rowptr"])
def test_validate_csr_rejects(case):
    g = gg.erdos_renyi(50, 120, seed=2)
    rp = g.row_ptr.copy()
    col = g.col.copy()
    v = int(np.argmax(np.diff(rp)))  # a vertex with >= 2 neighbours
    a, b = rp[v], rp[v + 1]
    if case == "asym":
        # replace one neighbour of v by a vertex x that is not adjacent to v
        nbrs = set(col[a:b].tolist())
        x = next(x for x in range(g.n) if x != v and x not in nbrs)
        col[a] = x
        col[a:b] = np.sort(col[a:b])
    elif case == "loop":
        col[a] = v
        col[a:b] = np.sort(col[a:b])
    elif case == "dup":
        col[a + 1] = col[a]
    elif case == "unsorted":
        col[a], col[a + 1] = col[a + 1], col[a]
    elif case == "range":
        col[a] = g.n + 3
    elif case == "rowptr":
        rp[-1] -= 1
    assert kh.validate_csr(g.n, rp, col) == kh.KH_EGRAPH


def test_context_without_gpu_reports_device_error():
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present")
    except ImportError:
        pass
    h = ctypes.c_void_p()
    assert kh.lib().kh_context_create(0, 0, ctypes.byref(h)) == kh.KH_EDEVICE


def test_batch_and_serve_reject_missing_arguments():
    # host-side argument checks; no context or GPU is needed to reach them
    L = kh.lib()
    p = kh.make_params(2)
    res = kh.Result()
    t = ctypes.c_uint64()
    assert L.kh_core_batch(None, 1, None, ctypes.byref(p), None, None, None) == -1
    assert L.kh_core_batch(None, -1, None, ctypes.byref(p), None, None, None) == -1
    assert L.kh_serve_start(None, 1, 0, 0, 0) == -1
    assert L.kh_serve_submit(None, None, ctypes.byref(p), None, ctypes.byref(t)) == -1
    assert L.kh_serve_poll(None, 1, ctypes.byref(res)) == -1
    assert L.kh_serve_wait(None, 1, ctypes.byref(res)) == -1
    assert L.kh_serve_cancel(None, 1) == -1
    assert L.kh_serve_stop(None) == -1


def test_validate_csr_rejects_arc_counts_beyond_the_int32_headroom():
    # arc indices are int32 on the device with 2^24 of headroom for chunked ranges
    limit = 2**31 - 1 - 2**24
    L = kh.lib()
    rp = np.zeros(2, np.int32)
    col = np.zeros(1, np.int32)
    assert L.kh_validate_csr(1, limit + 1, rp.ctypes.data, col.ctypes.data) == kh.KH_EINVAL
    assert L.kh_validate_csr(1, 2**31 - 1, rp.ctypes.data, col.ctypes.data) == kh.KH_EINVAL
