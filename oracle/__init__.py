"""CPU oracle for (k,h)-core decomposition -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The GPU library never does, and this package never
imports the GPU library: the two share no code.

The arithmetic lives in ``khoracle.c`` (plain C, compiled with gcc into
``libkhoracle.so`` next to it); this module only marshals numpy arrays.
Definitions follow Tatti, arXiv 2112.06154: Sec. 2 (h-neighbourhoods,
(k,h)-cores, ExactCore), Sec. 3 (Eq. buffer, ranks, B[v,i]/k[v,i]),
Def. est in Sec. 4 (the estimator), Alg. 4 (Core) and Sec. 6 (h-density,
densest core level).  ``oracle.refined`` runs Alg. 4 on the refined
bookkeeping of Sec. 5 (Alg. 5 and 6) in plain Python, for small graphs.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "khoracle.c")
_LIB = os.path.join(_HERE, "libkhoracle.so")
# KH_ORACLE_LIB: an oracle library built elsewhere from the same source (the
# sanitizer test loads an ASan/UBSan build this way); used as given, not rebuilt
_LIB_OVERRIDE = os.environ.get("KH_ORACLE_LIB")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no OpenMP, no vectorisation flags)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fvisibility=hidden",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if _LIB_OVERRIDE:
            L = ctypes.CDLL(_LIB_OVERRIDE)
        else:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
            L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64, u64, u32, dbl, ci = ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_double, ctypes.c_int
        L.orc_splitmix64.argtypes = [u64]
        L.orc_splitmix64.restype = u64
        L.orc_rank.argtypes = [u64, u32, i64]
        L.orc_rank.restype = ci
        L.orc_ranks.argtypes = [i64, u64, u32, P]
        L.orc_ranks.restype = None
        L.orc_M_real.argtypes = [i64, dbl, dbl, ci]
        L.orc_M_real.restype = dbl
        L.orc_M.argtypes = [i64, dbl, dbl, ci]
        L.orc_M.restype = i64
        L.orc_delta.argtypes = [P, i64, i64]
        L.orc_delta.restype = i64
        L.orc_hdeg_all.argtypes = [i64, P, P, P, ci, P, P]
        L.orc_hdeg_all.restype = ci
        L.orc_hdeg_list.argtypes = [i64, P, P, P, ci, i64, P, P, P]
        L.orc_hdeg_list.restype = ci
        L.orc_est_all.argtypes = [i64, P, P, P, ci, P, i64, P]
        L.orc_est_all.restype = ci
        L.orc_exact_core.argtypes = [i64, P, P, ci, u64, ci, P, P, P]
        L.orc_exact_core.restype = ci
        L.orc_sampled_core.argtypes = [i64, P, P, ci, P, i64, u64, ci, P, P]
        L.orc_sampled_core.restype = ci
        L.orc_exact_core_sweep.argtypes = [i64, P, P, ci, P]
        L.orc_exact_core_sweep.restype = ci
        L.orc_sampled_lists.argtypes = [i64, P, P, P, ci, P, i64, P, P, P]
        L.orc_sampled_lists.restype = i64
        L.orc_dense.argtypes = [i64, P, P, P, ci, ci, P, i64, ci, dbl, P, P, P, P, P, P, P]
        L.orc_dense.restype = ci
        L.orc_bulk_order.argtypes = [i64, P, P, P, ci, ci, P, i64, P, P, P]
        L.orc_bulk_order.restype = i64
        L.orc_dense_suffix.argtypes = [i64, P, P, ci, ci, P, i64, i64, P, P, P]
        L.orc_dense_suffix.restype = ci
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _csr(g):
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.int32)
    col = np.ascontiguousarray(g.col, dtype=np.int32)
    if col.size == 0:
        col = np.zeros(1, np.int32)
    return rp, col


def _alive(g, alive):
    if alive is None:
        return np.ones(max(g.n, 1), np.uint8)
    a = np.ascontiguousarray(alive, dtype=np.uint8)
    return a if a.size else np.ones(1, np.uint8)


def splitmix64(x: int) -> int:
    return int(lib().orc_splitmix64(x & 0xFFFFFFFFFFFFFFFF))


def ranks(n: int, seed: int, stream: int = 0) -> np.ndarray:
    """Geometric(1/2) ranks r[v] (Sec. 3) from the counter-based stream."""
    r = np.zeros(max(n, 1), np.uint8)
    lib().orc_ranks(n, seed & 0xFFFFFFFFFFFFFFFF, stream, _p(r))
    return r[:n]


def M_real(n: int, eps: float, delta: float = 0.05, dense: bool = False) -> float:
    return float(lib().orc_M_real(n, eps, delta, int(dense)))


def M_int(n: int, eps: float, delta: float = 0.05, dense: bool = False) -> int:
    """floor(M) of Eq. (buffer); dense=True uses C = log(n^2/delta) (Alg. 7)."""
    return int(lib().orc_M(n, eps, delta, int(dense)))


def delta_est(x, M: int) -> int:
    """Def. est: Delta(x_1..x_d; M) for a rank list whose first entry is r[v]."""
    a = np.ascontiguousarray(x, dtype=np.int32)
    if a.size == 0:
        a = np.zeros(1, np.int32)
        return int(lib().orc_delta(_p(a), 0, M))
    return int(lib().orc_delta(_p(a), a.size, M))


def hdeg(g, h: int, alive=None, with_te: bool = False):
    """deg_h(v; X) for every alive v; -1 for dead vertices (Sec. 2)."""
    rp, col = _csr(g)
    out = np.zeros(max(g.n, 1), np.int64)
    te = ctypes.c_int64(0)
    if g.n:
        lib().orc_hdeg_all(g.n, _p(rp), _p(col), _p(_alive(g, alive)), h, _p(out), ctypes.byref(te))
    return (out[:g.n], te.value) if with_te else out[:g.n]


def hdeg_list(g, h: int, sources, alive=None, with_te: bool = False):
    rp, col = _csr(g)
    src = np.ascontiguousarray(sources, dtype=np.int32)
    out = np.zeros(max(src.size, 1), np.int64)
    te = ctypes.c_int64(0)
    if src.size:
        lib().orc_hdeg_list(g.n, _p(rp), _p(col), _p(_alive(g, alive)), h, src.size, _p(src), _p(out),
                            ctypes.byref(te))
    return (out[:src.size], te.value) if with_te else out[:src.size]


def estimate_all(g, h: int, r, M: int, alive=None) -> np.ndarray:
    """The estimate Delta((r[v], r[u] : u in N(v;h,X)\\{v}); M) per alive v."""
    rp, col = _csr(g)
    rr = np.ascontiguousarray(r, dtype=np.uint8)
    out = np.zeros(max(g.n, 1), np.int64)
    if g.n:
        lib().orc_est_all(g.n, _p(rp), _p(col), _p(_alive(g, alive)), h, _p(rr), M, _p(out))
    return out[:g.n]


def exact_core(g, h: int, tie_seed: int = 0, with_order: bool = False, with_te: bool = False,
               early_stop: bool = False):
    """ExactCore (Sec. 2): sequential min-peel on deg_h, running maximum.
    early_stop: the Sec. 5 heuristic (stop once c + 1 >= remaining)."""
    rp, col = _csr(g)
    core = np.zeros(max(g.n, 1), np.int64)
    order = np.zeros(max(g.n, 1), np.int32)
    te = ctypes.c_int64(0)
    if g.n:
        lib().orc_exact_core(g.n, _p(rp), _p(col), h, tie_seed, int(early_stop), _p(core), _p(order),
                             ctypes.byref(te))
    res = [core[:g.n]]
    if with_order:
        res.append(order[:g.n])
    if with_te:
        res.append(te.value)
    return res[0] if len(res) == 1 else tuple(res)


def exact_core_sweep(g, h: int) -> np.ndarray:
    rp, col = _csr(g)
    core = np.zeros(max(g.n, 1), np.int64)
    if g.n:
        lib().orc_exact_core_sweep(g.n, _p(rp), _p(col), h, _p(core))
    return core[:g.n]


def sampled_core(g, h: int, r, M: int, tie_seed: int = 0, with_order: bool = False, early_stop: bool = False):
    """Core (Alg. 4) through the closed form of its estimate.
    early_stop: the Sec. 5 heuristic (stop once c + 1 >= remaining)."""
    rp, col = _csr(g)
    rr = np.ascontiguousarray(r, dtype=np.uint8)
    if rr.size == 0:
        rr = np.zeros(1, np.uint8)
    core = np.zeros(max(g.n, 1), np.int64)
    order = np.zeros(max(g.n, 1), np.int32)
    if g.n:
        lib().orc_sampled_core(g.n, _p(rp), _p(col), h, _p(rr), M, tie_seed, int(early_stop), _p(core), _p(order))
    return (core[:g.n], order[:g.n]) if with_order else core[:g.n]


def sampled_lists(g, i: int, r, M: int, alive=None):
    """Closed form of (k[v,i], B[v,i]) for every alive v (Sec. 3).

    Returns (k int32[n], sizes int32[n], offsets int64[n+1], members int32[...])
    with each B[v,i] listed in ascending id order."""
    rp, col = _csr(g)
    rr = np.ascontiguousarray(r, dtype=np.uint8)
    if rr.size == 0:
        rr = np.zeros(1, np.uint8)
    a = _alive(g, alive)
    k = np.zeros(max(g.n, 1), np.int32)
    s = np.zeros(max(g.n, 1), np.int32)
    if g.n == 0:
        return k[:0], s[:0], np.zeros(1, np.int64), np.zeros(0, np.int32)
    total = lib().orc_sampled_lists(g.n, _p(rp), _p(col), _p(a), i, _p(rr), M, _p(k), _p(s), None)
    mem = np.zeros(max(total, 1), np.int32)
    lib().orc_sampled_lists(g.n, _p(rp), _p(col), _p(a), i, _p(rr), M, _p(k), _p(s), _p(mem))
    off = np.zeros(g.n + 1, np.int64)
    np.cumsum(s[:g.n], out=off[1:])
    return k[:g.n], s[:g.n], off, mem[:total]


def dense(g, core, h: int, mode: str = "exact", r=None, M: int = 0, prune: bool = False, eps: float = 0.5):
    """Densest core level (Sec. 6).  Returns dict with best K, |F_K|, R_K,
    density R_K/(2|F_K|) and the list of all candidates."""
    rp, col = _csr(g)
    c = np.ascontiguousarray(core, dtype=np.int64)
    if c.size == 0:
        return {"k": -1, "size": 0, "R": 0, "density": 0.0, "cands": []}
    rr = np.ascontiguousarray(r if r is not None else np.zeros(g.n, np.uint8), dtype=np.uint8)
    bk, bs, bR, nc = (ctypes.c_int64() for _ in range(4))
    ck = np.zeros(g.n + 1, np.int64)
    cs = np.zeros(g.n + 1, np.int64)
    cR = np.zeros(g.n + 1, np.int64)
    lib().orc_dense(g.n, _p(rp), _p(col), _p(c), h, 0 if mode == "exact" else 1, _p(rr), M, int(prune), eps,
                    ctypes.byref(bk), ctypes.byref(bs), ctypes.byref(bR), ctypes.byref(nc), _p(ck), _p(cs), _p(cR))
    cands = [(int(ck[i]), int(cs[i]), int(cR[i])) for i in range(nc.value)]
    return {"k": bk.value, "size": bs.value, "R": bR.value,
            "density": (bR.value / (2.0 * bs.value)) if bs.value else 0.0, "cands": cands}


def bulk_order(g, h: int, mode: str = "exact", r=None, M: int = 0, alive=None):
    """Deletion order of the bulk-round peel (rounds in sequence; inside a
    round by (f, level of Def. est, id)), with the core numbers and the round
    of every deletion.  Returns (order int32[count], core int64[n], round int64[n])."""
    rp, col = _csr(g)
    rr = np.ascontiguousarray(r if r is not None else np.zeros(max(g.n, 1), np.uint8), dtype=np.uint8)
    order = np.zeros(max(g.n, 1), np.int32)
    core = np.zeros(max(g.n, 1), np.int64)
    rnd = np.zeros(max(g.n, 1), np.int64)
    cnt = 0
    if g.n:
        cnt = lib().orc_bulk_order(g.n, _p(rp), _p(col), _p(_alive(g, alive)), h, 0 if mode == "exact" else 1,
                                   _p(rr), M, _p(order), _p(core), _p(rnd))
    return order[:cnt], core[:g.n], rnd[:g.n]


def dense_suffix(g, order, h: int, mode: str = "exact", r=None, M: int = 0):
    """Alg. 7 over every suffix of `order`: R[i] = sum of f over the suffix
    starting at i, measured inside it.  Returns dict with R (int64[count]),
    the best start index (ties: later), its size, R and density R/(2 size)."""
    rp, col = _csr(g)
    o = np.ascontiguousarray(order, dtype=np.int32)
    cnt = int(o.size)
    if cnt == 0:
        return {"R": np.zeros(0, np.int64), "best": -1, "size": 0, "best_R": 0, "density": 0.0}
    rr = np.ascontiguousarray(r if r is not None else np.zeros(max(g.n, 1), np.uint8), dtype=np.uint8)
    R = np.zeros(cnt, np.int64)
    bi = ctypes.c_int64(-1)
    lib().orc_dense_suffix(g.n, _p(rp), _p(col), h, 0 if mode == "exact" else 1, _p(rr), M, cnt, _p(o), _p(R),
                           ctypes.byref(bi))
    b = bi.value
    size = cnt - b
    return {"R": R, "best": b, "size": size, "best_R": int(R[b]), "density": R[b] / (2.0 * size)}
