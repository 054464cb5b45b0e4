"""ctypes binding of libkhcore.so (include/khcore.h).

Argument marshalling only: every step of the decomposition runs in the HIP
library.  torch provides device memory (tensors whose storage the library
reads or writes) and the current HIP stream.  If the shared library is
missing this module raises on first use; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libkhcore.so")

KH_OK = 0
KH_EINVAL = -1
KH_ENOMEM = -2
KH_EDEVICE = -3
KH_EGRAPH = -4
KH_EOVERFLOW = -5
KH_EBUSY = -6
KH_ENOTFOUND = -7
KH_ENOTIMPL = -8

KH_PTRS_HOST = 0
KH_PTRS_DEVICE_BORROW = 1
KH_CANONICALIZE = 2
KH_TRUST_CSR = 4

KH_WANT_DENSE = 1
KH_DENSE_PRUNE = 2
KH_EARLY_STOP = 4
KH_OUT_DEVICE = 8
KH_DENSE_FULL = 16
KH_LAZY_INIT = 32

EXPORTED = [
    "kh_status_str", "kh_buffer_size", "kh_validate_csr", "kh_context_create", "kh_context_destroy",
    "kh_graph_load_csr", "kh_graph_free", "kh_graph_n", "kh_graph_nnz", "kh_core", "kh_core_batch", "kh_hdeg",
    "kh_ranks", "kh_serve_start", "kh_serve_submit", "kh_serve_poll", "kh_serve_wait", "kh_serve_cancel",
    "kh_serve_stop",
    "kh_sampled_lists", "kh_dense", "kh_profile_enable", "kh_profile_read", "kh_hdeg_noalloc",
]

# size of the fixed device array of kh_hdeg_noalloc (KH_NOALLOC_SCRATCH_BYTES)
NOALLOC_SCRATCH_BYTES = 64 << 20


class Params(ctypes.Structure):
    _fields_ = [("h", ctypes.c_int32), ("epsilon", ctypes.c_double), ("delta", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("M_override", ctypes.c_int32), ("M_dense_override", ctypes.c_int32),
                ("flags", ctypes.c_uint32)]


class Result(ctypes.Structure):
    _fields_ = [("M_used", ctypes.c_int32), ("M_dense_used", ctypes.c_int32), ("rounds", ctypes.c_int32),
                ("max_core", ctypes.c_int32), ("dense_k", ctypes.c_int64), ("dense_size", ctypes.c_int64),
                ("dense_R", ctypes.c_int64), ("dense_density", ctypes.c_double),
                ("edges_traversed", ctypes.c_int64), ("arcs_scanned", ctypes.c_int64),
                ("list_elements", ctypes.c_int64), ("seconds", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class KhError(RuntimeError):
    def __init__(self, code, what=""):
        self.code = code
        super().__init__(f"{what}: {status_str(code)} ({code})" if what else f"{status_str(code)} ({code})")


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libkhcore.so is not built ({LIB_PATH}); run paper_2112_06154_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        P, i32, i64, u32, u64, dbl = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                                      ctypes.c_uint64, ctypes.c_double)
        L.kh_status_str.argtypes = [i32]
        L.kh_status_str.restype = ctypes.c_char_p
        L.kh_buffer_size.argtypes = [i64, dbl, dbl, i32]
        L.kh_buffer_size.restype = i64
        L.kh_validate_csr.argtypes = [i32, i64, P, P]
        L.kh_validate_csr.restype = i32
        L.kh_context_create.argtypes = [i32, u64, ctypes.POINTER(P)]
        L.kh_context_create.restype = i32
        L.kh_context_destroy.argtypes = [P]
        L.kh_context_destroy.restype = None
        L.kh_graph_load_csr.argtypes = [P, i32, i64, P, P, u32, P, ctypes.POINTER(P)]
        L.kh_graph_load_csr.restype = i32
        L.kh_graph_free.argtypes = [P]
        L.kh_graph_free.restype = None
        L.kh_graph_n.argtypes = [P]
        L.kh_graph_n.restype = i32
        L.kh_graph_nnz.argtypes = [P]
        L.kh_graph_nnz.restype = i64
        L.kh_core.argtypes = [P, ctypes.POINTER(Params), P, ctypes.POINTER(Result), P]
        L.kh_core.restype = i32
        L.kh_core_batch.argtypes = [P, i32, P, ctypes.POINTER(Params), P, P, P]
        L.kh_core_batch.restype = i32
        L.kh_serve_start.argtypes = [P, i32, u64, i32, i64]
        L.kh_serve_start.restype = i32
        L.kh_serve_submit.argtypes = [P, P, ctypes.POINTER(Params), P, ctypes.POINTER(u64)]
        L.kh_serve_submit.restype = i32
        L.kh_serve_poll.argtypes = [P, u64, ctypes.POINTER(Result)]
        L.kh_serve_poll.restype = i32
        L.kh_serve_wait.argtypes = [P, u64, ctypes.POINTER(Result)]
        L.kh_serve_wait.restype = i32
        L.kh_serve_cancel.argtypes = [P, u64]
        L.kh_serve_cancel.restype = i32
        L.kh_serve_stop.argtypes = [P]
        L.kh_serve_stop.restype = i32
        L.kh_hdeg.argtypes = [P, i32, P, u32, P, ctypes.POINTER(i64), P]
        L.kh_hdeg.restype = i32
        L.kh_hdeg_noalloc.argtypes = [P, i32, P, P, P, P]
        L.kh_hdeg_noalloc.restype = i32
        L.kh_ranks.argtypes = [P, i32, u64, u32, P, P]
        L.kh_ranks.restype = i32
        L.kh_sampled_lists.argtypes = [P, ctypes.POINTER(Params), P, i32, P, P, P, i64, P, P]
        L.kh_sampled_lists.restype = i32
        L.kh_dense.argtypes = [P, ctypes.POINTER(Params), P, ctypes.POINTER(Result), P]
        L.kh_dense.restype = i32
        L.kh_profile_enable.argtypes = [P, i32]
        L.kh_profile_enable.restype = i32
        L.kh_profile_read.argtypes = [P, i32, ctypes.POINTER(i64), ctypes.POINTER(dbl), ctypes.POINTER(i64),
                                      ctypes.POINTER(i64)]
        L.kh_profile_read.restype = i32
        _lib = L
    return _lib


def status_str(code: int) -> str:
    return lib().kh_status_str(code).decode()


def _check(code, what=""):
    if code != KH_OK:
        raise KhError(code, what)


def _ptr(a):
    """Address of a numpy array or torch tensor (None -> NULL)."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data_as(ctypes.c_void_p)
    return ctypes.c_void_p(a.data_ptr())


def _stream(stream=None):
    if stream is not None:
        return ctypes.c_void_p(stream)
    try:
        import torch
        if torch.cuda.is_available():
            return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    except ImportError:
        pass
    return None


def buffer_size(n: int, epsilon: float, delta: float = 0.05, dense: bool = False) -> int:
    """floor(M) of Eq. (buffer) (host only)."""
    return int(lib().kh_buffer_size(n, epsilon, delta, int(dense)))


def validate_csr(n: int, row_ptr, col) -> int:
    """kh_validate_csr on host arrays; returns the status code."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    cl = np.ascontiguousarray(col, dtype=np.int32)
    return int(lib().kh_validate_csr(n, int(cl.size), _ptr(rp), _ptr(cl) if cl.size else None))


class Context:
    def __init__(self, device: int = 0, hbm_budget: int = 0):
        h = ctypes.c_void_p()
        _check(lib().kh_context_create(device, hbm_budget, ctypes.byref(h)), "kh_context_create")
        self.handle = h
        self.device = device

    def close(self):
        if self.handle:
            lib().kh_context_destroy(self.handle)
            self.handle = None

    def profile(self, on: bool) -> None:
        """Start (resetting totals) or stop HIP-event timing of the instrumented kernels."""
        _check(lib().kh_profile_enable(self.handle, int(on)), "kh_profile_enable")

    def profile_read(self, kernel: int = 0) -> dict:
        """Totals for kernel 0 (h-degree pull), 1 (sample-list union) or 2 (R-mask BFS hop of the exact peel)."""
        la, by, ga = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        ms = ctypes.c_double()
        _check(lib().kh_profile_read(self.handle, kernel, ctypes.byref(la), ctypes.byref(ms), ctypes.byref(by),
                                     ctypes.byref(ga)), "kh_profile_read")
        return {"launches": la.value, "ms": ms.value, "alg_bytes": by.value, "gather_bytes": ga.value}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Graph:
    """A device-resident CSR graph.  `row_ptr`/`col` are numpy arrays (copied)
    or torch device tensors (borrowed: they are kept alive by this object)."""

    def __init__(self, ctx: Context, n: int, row_ptr, col, canonicalize: bool = False, trust: bool = False,
                 stream=None):
        self.ctx = ctx
        flags = 0
        if isinstance(row_ptr, np.ndarray) or isinstance(row_ptr, list):
            rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
            cl = np.ascontiguousarray(col, dtype=np.int32)
            self._keep = (rp, cl)
            flags |= KH_PTRS_HOST
            if canonicalize:
                flags |= KH_CANONICALIZE
        else:
            rp, cl = row_ptr, col
            self._keep = (rp, cl)
            flags |= KH_PTRS_DEVICE_BORROW
        if trust:
            flags |= KH_TRUST_CSR
        nnz = int(cl.size if isinstance(cl, np.ndarray) else cl.numel())
        h = ctypes.c_void_p()
        _check(lib().kh_graph_load_csr(ctx.handle, n, nnz, _ptr(rp), _ptr(cl) if nnz else None, flags,
                                       _stream(stream), ctypes.byref(h)), "kh_graph_load_csr")
        self.handle = h

    @staticmethod
    def from_gg(ctx: Context, g, **kw) -> "Graph":
        return Graph(ctx, g.n, g.row_ptr, g.col, **kw)

    @property
    def n(self) -> int:
        return int(lib().kh_graph_n(self.handle))

    @property
    def nnz(self) -> int:
        return int(lib().kh_graph_nnz(self.handle))

    def close(self):
        if getattr(self, "handle", None):
            lib().kh_graph_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_params(h: int, epsilon: float = 0.0, delta: float = 0.05, seed: int = 0, M_override: int = 0,
                M_dense_override: int = 0, dense: bool = False, prune: bool = False, early_stop: bool = False,
                out_device: bool = False, dense_full: bool = False, lazy_init: bool = False) -> Params:
    flags = (KH_WANT_DENSE if dense or dense_full else 0) | (KH_DENSE_PRUNE if prune else 0) | \
            (KH_EARLY_STOP if early_stop else 0) | (KH_OUT_DEVICE if out_device else 0) | \
            (KH_DENSE_FULL if dense_full else 0) | (KH_LAZY_INIT if lazy_init else 0)
    return Params(h, epsilon, delta, seed & 0xFFFFFFFFFFFFFFFF, M_override, M_dense_override, flags)


def core(graph: Graph, h: int, epsilon: float = 0.0, out=None, stream=None, **kw):
    """(k,h)-core numbers: ExactCore for epsilon <= 0, else Core (Alg. 4).

    Returns (core, result_dict).  `out` may be an int32 torch device tensor of
    n elements, in which case the numbers stay on the device."""
    p = make_params(h, epsilon, out_device=out is not None, **kw)
    res = Result()
    if out is None:
        out = np.zeros(max(graph.n, 1), np.int32)
    _check(lib().kh_core(graph.handle, ctypes.byref(p), _ptr(out), ctypes.byref(res), _stream(stream)), "kh_core")
    if isinstance(out, np.ndarray):
        out = out[:graph.n]
    return out, res.as_dict()


def core_batch(graphs, h: int, epsilon: float = 0.0, outs=None, stream=None, **kw):
    """kh_core over many graphs packed into disjoint unions (kh_core_batch).

    Returns (list of core arrays, list of result dicts).  `outs` may be a list
    of int32 torch device tensors (one per graph), in which case the numbers
    stay on the device."""
    graphs = list(graphs)
    count = len(graphs)
    if count == 0:
        return [], []
    p = make_params(h, epsilon, out_device=outs is not None, **kw)
    if outs is None:
        outs = [np.zeros(max(g.n, 1), np.int32) for g in graphs]
    handles = (ctypes.c_void_p * max(count, 1))(*[g.handle for g in graphs])
    optrs = (ctypes.c_void_p * max(count, 1))(*[_ptr(o) for o in outs])
    res = (Result * max(count, 1))()
    ctx = graphs[0].ctx.handle
    _check(lib().kh_core_batch(ctx, count, handles, ctypes.byref(p), optrs, res, _stream(stream)),
           "kh_core_batch")
    cores = [o[:g.n] if isinstance(o, np.ndarray) else o for o, g in zip(outs, graphs)]
    return cores, [res[i].as_dict() for i in range(count)]


class Server:
    """The context's serving loop (kh_serve_*): submit returns a ticket, poll
    returns None while the request is pending and (core, result) once done.
    Output arrays are kept alive here until collected."""

    def __init__(self, ctx: Context, workers: int = 0, hbm_budget: int = 0, queue_cap: int = 0,
                 batch_vertices: int = 0):
        self.ctx = ctx
        _check(lib().kh_serve_start(ctx.handle, workers, hbm_budget, queue_cap, batch_vertices), "kh_serve_start")
        self._pending = {}

    def submit(self, graph: Graph, h: int, epsilon: float = 0.0, out=None, **kw) -> int:
        p = make_params(h, epsilon, out_device=out is not None, **kw)
        if out is None:
            out = np.zeros(max(graph.n, 1), np.int32)
        t = ctypes.c_uint64()
        _check(lib().kh_serve_submit(self.ctx.handle, graph.handle, ctypes.byref(p), _ptr(out), ctypes.byref(t)),
               "kh_serve_submit")
        self._pending[t.value] = (out, graph)
        return t.value

    def _collect(self, ticket: int, wait: bool):
        res = Result()
        fn = lib().kh_serve_wait if wait else lib().kh_serve_poll
        # hold the output while the call runs: a concurrent stop() forgets it
        out, graph = self._pending.get(ticket, (None, None))
        code = fn(self.ctx.handle, ticket, ctypes.byref(res))
        if code == KH_EBUSY:
            return None
        self._pending.pop(ticket, None)
        _check(code, "kh_serve_wait" if wait else "kh_serve_poll")
        if isinstance(out, np.ndarray):
            out = out[:graph.n]
        return out, res.as_dict()

    def poll(self, ticket: int):
        return self._collect(ticket, False)

    def wait(self, ticket: int):
        return self._collect(ticket, True)

    def cancel(self, ticket: int) -> bool:
        """True if the request was still queued and is withdrawn; False if it
        already runs or has finished (collect it with poll / wait)."""
        code = lib().kh_serve_cancel(self.ctx.handle, ticket)
        if code == KH_EBUSY:
            return False
        _check(code, "kh_serve_cancel")
        self._pending.pop(ticket, None)
        return True

    def stop(self):
        _check(lib().kh_serve_stop(self.ctx.handle), "kh_serve_stop")
        self._pending.clear()


def hdeg(graph: Graph, h: int, alive=None, out=None, stream=None):
    """h-degrees of every vertex of X (alive: uint8 torch device tensor or None)."""
    te = ctypes.c_int64(0)
    flags = KH_OUT_DEVICE if out is not None else 0
    if out is None:
        out = np.zeros(max(graph.n, 1), np.int32)
    _check(lib().kh_hdeg(graph.handle, h, _ptr(alive), flags, _ptr(out), ctypes.byref(te), _stream(stream)),
           "kh_hdeg")
    if isinstance(out, np.ndarray):
        out = out[:graph.n]
    return out, te.value


def hdeg_noalloc(graph: Graph, h: int, deg_out, alive=None, te_out=None, stream=None) -> None:
    """kh_hdeg_noalloc: h-degrees into the int32 device tensor deg_out (n
    entries) and, if given, the edges-traversed count into the int64 device
    tensor te_out; enqueued on the stream, nothing allocated."""
    _check(lib().kh_hdeg_noalloc(graph.handle, h, _ptr(alive), _ptr(deg_out), _ptr(te_out), _stream(stream)),
           "kh_hdeg_noalloc")


def ranks(ctx: Context, n: int, seed: int, stream_id: int = 0, stream=None):
    """Geometric(1/2) ranks into a new uint8 torch device tensor."""
    import torch
    r = torch.empty(max(n, 1), dtype=torch.uint8, device=f"cuda:{ctx.device}")
    _check(lib().kh_ranks(ctx.handle, n, seed & 0xFFFFFFFFFFFFFFFF, stream_id, _ptr(r), _stream(stream)),
           "kh_ranks")
    return r[:n]


def sampled_lists(graph: Graph, h: int, level: int, epsilon: float = 0.5, alive=None, members: bool = True,
                  stream=None, **kw):
    """B[v,level], k[v,level] after initialisation, and Alg. 1's estimate.

    Returns (k int32[n], size int32[n], members list of int32 arrays or None, est int64[n])."""
    n = graph.n
    p = make_params(h, epsilon, **kw)
    k = np.zeros(max(n, 1), np.int32)
    sz = np.zeros(max(n, 1), np.int32)
    est = np.zeros(max(n, 1), np.int64)
    _check(lib().kh_sampled_lists(graph.handle, ctypes.byref(p), _ptr(alive), level, _ptr(k), _ptr(sz), None, 0,
                                  _ptr(est), _stream(stream)), "kh_sampled_lists")
    mem = None
    if members:
        total = int(sz[:n].sum())
        buf = np.zeros(max(total, 1), np.int32)
        _check(lib().kh_sampled_lists(graph.handle, ctypes.byref(p), _ptr(alive), level, _ptr(k), _ptr(sz),
                                      _ptr(buf), total, None, _stream(stream)), "kh_sampled_lists")
        off = np.concatenate([[0], np.cumsum(sz[:n].astype(np.int64))])
        mem = [buf[off[v]:off[v + 1]] for v in range(n)]
    return k[:n], sz[:n], mem, est[:n]


def dense(graph: Graph, core_in, h: int, epsilon: float = 0.0, stream=None, **kw):
    """Densest core level of a given core map (Sec. 6)."""
    p = make_params(h, epsilon, **kw)
    c = np.ascontiguousarray(core_in, dtype=np.int32)
    res = Result()
    _check(lib().kh_dense(graph.handle, ctypes.byref(p), _ptr(c), ctypes.byref(res), _stream(stream)), "kh_dense")
    return res.as_dict()
