"""Seeded synthetic graph generators.

This module produces the inputs that both the GPU library and the CPU oracle
read: simple undirected graphs in canonical int32 CSR form (both arc
directions stored, each adjacency sorted ascending, no self-loops, no
duplicate edges).  It holds none of the core-decomposition arithmetic; the
only randomness is a counter-based SplitMix64 stream (Steele, Lea and Flood,
"Fast splittable pseudorandom number generators", OOPSLA 2014) used to draw
edges and to relabel vertices.

Families (the shapes of the paper's workloads, Section 8, stand-ins for its
public datasets which are not available here):

* ``erdos_renyi(n, m, seed)``      -- exactly m distinct uniform pairs.
* ``chung_lu(n, m, gamma, seed)``  -- power-law expected degrees
  w_i ~ (i+1)^(-1/(gamma-1)), endpoints drawn i.i.d. proportional to w,
  loops and duplicates dropped, topped up to exactly m edges, ids permuted.
* ``barabasi_albert(n, k, seed)``  -- preferential attachment, k edges per
  new vertex, seed clique K_{k+1}, targets proportional to degree without
  repetition.
* ``sbm(n, seed)``                 -- the hierarchical stochastic block model of
  the paper's scaling experiment (Sec. 8): 10 equal blocks, every pair of
  vertices in blocks i < j joined with probability 1e-6 i^2, pairs inside a
  block with probability p_in.
* small deterministic shapes (path, cycle, star, clique, ...) for tests.
"""
from __future__ import annotations

import dataclasses
import math
import os

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _mix64(z: np.ndarray) -> np.ndarray:
    z = z.astype(np.uint64, copy=True)
    with np.errstate(over="ignore"):
        z ^= z >> np.uint64(30)
        z *= _M1
        z ^= z >> np.uint64(27)
        z *= _M2
        z ^= z >> np.uint64(31)
    return z


def splitmix_stream(key: int, start: int, count: int) -> np.ndarray:
    """Outputs start..start+count-1 of the SplitMix64 sequence whose state
    starts at ``key`` (output i is mix(key + (i+1) * golden))."""
    idx = np.arange(start + 1, start + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(key & 0xFFFFFFFFFFFFFFFF) + idx * _GOLDEN
    return _mix64(z)


def _key(seed: int, tag: int) -> int:
    """Derive an independent stream key from (seed, tag)."""
    v = np.array([(seed * 0x100000001B3 + tag) & 0xFFFFFFFFFFFFFFFF], dtype=np.uint64)
    return int(_mix64(v)[0])


def _uniform_below(x: np.ndarray, n: int) -> np.ndarray:
    """Map 64-bit words to [0, n) by a 32x32 multiply-high (n < 2^32)."""
    hi = (x >> np.uint64(32)).astype(np.uint64)
    with np.errstate(over="ignore"):
        return ((hi * np.uint64(n)) >> np.uint64(32)).astype(np.int64)


def _unit_double(x: np.ndarray) -> np.ndarray:
    return (x >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


@dataclasses.dataclass
class Graph:
    """Canonical CSR of a simple undirected graph."""
    n: int
    row_ptr: np.ndarray  # int32[n+1]
    col: np.ndarray      # int32[2m]
    name: str = ""

    @property
    def m(self) -> int:
        return int(self.col.shape[0]) // 2

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr.astype(np.int64))

    def edges(self) -> np.ndarray:
        """Each undirected edge once, as an (m, 2) int64 array with u < v."""
        src = np.repeat(np.arange(self.n, dtype=np.int64), self.degrees())
        dst = self.col.astype(np.int64)
        keep = src < dst
        return np.stack([src[keep], dst[keep]], axis=1)

    def save(self, path: str) -> None:
        np.savez(path, n=np.int64(self.n), row_ptr=self.row_ptr, col=self.col)

    @staticmethod
    def load(path: str) -> "Graph":
        z = np.load(path, allow_pickle=False)
        return Graph(int(z["n"]), z["row_ptr"].astype(np.int32), z["col"].astype(np.int32),
                     os.path.basename(path))


def from_edges(n: int, edges, name: str = "") -> Graph:
    """Canonical CSR from an undirected edge list; loops and duplicates are
    removed, both directions are stored and adjacencies are sorted."""
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    if e.size and (e.min() < 0 or e.max() >= n):
        raise ValueError("edge endpoint out of range")
    e = e[e[:, 0] != e[:, 1]]
    nn = np.int64(max(n, 1))
    lo = np.minimum(e[:, 0], e[:, 1])
    hi = np.maximum(e[:, 0], e[:, 1])
    keys = np.unique(lo * nn + hi)
    lo = keys // nn
    hi = keys % nn
    arc = np.concatenate([lo * nn + hi, hi * nn + lo])
    arc.sort()
    src = arc // nn
    dst = arc % nn
    deg = np.bincount(src, minlength=n) if n > 0 else np.zeros(0, np.int64)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(deg, out=row_ptr[1:])
    if row_ptr[-1] > np.iinfo(np.int32).max:
        raise ValueError("too many arcs for int32 CSR")
    return Graph(n, row_ptr.astype(np.int32), dst.astype(np.int32), name)


def relabel(g: Graph, perm: np.ndarray, name: str | None = None) -> Graph:
    """Rename vertex v to perm[v]."""
    e = g.edges()
    return from_edges(g.n, perm[e], g.name if name is None else name)


def random_permutation(n: int, seed: int) -> np.ndarray:
    keys = splitmix_stream(_key(seed, 0x5045524D), 0, n)
    return np.argsort(keys, kind="stable").astype(np.int64)


def _first_distinct_pairs(n: int, m: int, draw, name: str) -> np.ndarray:
    """Collect the first m distinct non-loop unordered pairs produced by
    ``draw(start, count) -> (u, v)`` in counter order."""
    if m > n * (n - 1) // 2:
        raise ValueError("m exceeds the number of vertex pairs")
    keys_all = np.zeros(0, dtype=np.int64)
    start = 0
    chunk = max(64, int(m * 1.15) + 64)
    while True:
        u, v = draw(start, chunk)
        start += chunk
        lo = np.minimum(u, v)
        hi = np.maximum(u, v)
        k = np.where(lo != hi, lo * np.int64(n) + hi, np.int64(-1))
        keys_all = np.concatenate([keys_all, k])
        uniq, first = np.unique(keys_all, return_index=True)
        good = uniq >= 0
        if good.sum() >= m:
            idx = np.sort(first[good])[:m]
            sel = keys_all[idx]
            return np.stack([sel // n, sel % n], axis=1)
        chunk = max(chunk, int((m - good.sum()) * 2) + 64)


def erdos_renyi(n: int, m: int, seed: int = 1, permute: bool = True) -> Graph:
    """G(n, m): exactly m distinct uniform vertex pairs."""
    key = _key(seed, 0x4552)

    def draw(start, count):
        x = splitmix_stream(key, 2 * start, 2 * count)
        return _uniform_below(x[0::2], n), _uniform_below(x[1::2], n)

    e = _first_distinct_pairs(n, m, draw, "er")
    if permute:
        e = random_permutation(n, seed)[e]
    return from_edges(n, e, f"er_n{n}_m{m}_s{seed}")


def chung_lu(n: int, m: int, gamma: float, seed: int = 1, permute: bool = True) -> Graph:
    """Chung-Lu power-law graph with exactly m edges (see module docstring)."""
    key = _key(seed, 0x434C)
    w = np.power(np.arange(1, n + 1, dtype=np.float64), -1.0 / (gamma - 1.0))
    w *= (2.0 * m) / w.sum()
    cdf = np.cumsum(w)
    cdf /= cdf[-1]

    def draw(start, count):
        x = splitmix_stream(key, 2 * start, 2 * count)
        a = np.searchsorted(cdf, _unit_double(x[0::2]), side="right")
        b = np.searchsorted(cdf, _unit_double(x[1::2]), side="right")
        return np.minimum(a, n - 1).astype(np.int64), np.minimum(b, n - 1).astype(np.int64)

    e = _first_distinct_pairs(n, m, draw, "cl")
    if permute:
        e = random_permutation(n, seed)[e]
    return from_edges(n, e, f"cl_n{n}_m{m}_g{gamma}_s{seed}")


_BA_LIB = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libggba.so")
_ba_lib = None


def build_native() -> str:
    """Compile the C preferential-attachment drawer (ba.c) in place."""
    import subprocess
    src = os.path.join(os.path.dirname(_BA_LIB), "ba.c")
    subprocess.run(["gcc", "-O2", "-shared", "-fPIC", "-o", _BA_LIB, src], check=True)
    return _BA_LIB


def _ba_native(n: int, k: int, key: int):
    """Edge pairs from ba.c (same stream and order as the Python loop below),
    or None when the library is not built."""
    global _ba_lib
    if _ba_lib is None:
        if not os.path.exists(_BA_LIB):
            return None
        import ctypes
        L = ctypes.CDLL(_BA_LIB)
        L.gg_ba_edges.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64, ctypes.c_void_p]
        L.gg_ba_edges.restype = ctypes.c_int64
        _ba_lib = L
    if k > 64:
        return None
    pairs = k * (k + 1) // 2 + k * (n - k - 1)
    out = np.empty(2 * pairs, dtype=np.int64)
    got = _ba_lib.gg_ba_edges(n, k, key & 0xFFFFFFFFFFFFFFFF, out.ctypes.data)
    if got != pairs:
        raise RuntimeError("gg_ba_edges failed")
    return out.reshape(-1, 2)


def barabasi_albert(n: int, k: int = 3, seed: int = 1, permute: bool = True) -> Graph:
    """Preferential attachment: start from the clique K_{k+1}; every new vertex
    links to k distinct existing vertices chosen proportionally to degree."""
    if n <= k + 1:
        return clique(n)
    key = _key(seed, 0x4241)
    e = _ba_native(n, k, key)
    if e is not None:
        if permute:
            e = random_permutation(n, seed)[e]
        return from_edges(n, e, f"ba_n{n}_k{k}_s{seed}")
    rnd = splitmix_stream(key, 0, 4 * k * n + 64)
    pos = 0
    ends = np.empty(2 * (k * (k + 1) // 2 + k * (n - k - 1)), dtype=np.int64)
    ne = 0
    edges = []
    for a in range(k + 1):
        for b in range(a + 1, k + 1):
            edges.append((a, b))
            ends[ne] = a
            ends[ne + 1] = b
            ne += 2
    for t in range(k + 1, n):
        chosen = []
        while len(chosen) < k:
            if pos >= rnd.shape[0]:
                rnd = np.concatenate([rnd, splitmix_stream(key, rnd.shape[0], 4 * k * n)])
            x = int(rnd[pos]) >> 32
            pos += 1
            c = int(ends[(x * ne) >> 32])
            if c not in chosen:
                chosen.append(c)
        for c in chosen:
            edges.append((c, t))
            ends[ne] = c
            ends[ne + 1] = t
            ne += 2
    e = np.asarray(edges, dtype=np.int64)
    if permute:
        e = random_permutation(n, seed)[e]
    return from_edges(n, e, f"ba_n{n}_k{k}_s{seed}")


def _bernoulli_positions(key: int, total: int, p: float) -> np.ndarray:
    """Indices in [0, total) each kept independently with probability p,
    by geometric skips: the gap before the next kept index is
    floor(log(1-U) / log(1-p)), which is Geometric(p) for U uniform on [0, 1)
    (Batagelj and Brandes, "Efficient generation of large random networks",
    Phys. Rev. E 71, 2005)."""
    if total <= 0 or p <= 0.0:
        return np.zeros(0, dtype=np.int64)
    if p >= 1.0:
        return np.arange(total, dtype=np.int64)
    lq = math.log1p(-p)
    out = []
    pos = -1
    start = 0
    while True:
        cnt = int(total * p * 1.1) + 64
        u = _unit_double(splitmix_stream(key, start, cnt))
        start += cnt
        gap = np.floor(np.log1p(-u) / lq).astype(np.int64)
        idx = pos + np.cumsum(gap + 1)
        keep = idx < total
        out.append(idx[keep])
        if not keep.all():
            return np.concatenate(out)
        pos = int(idx[-1])


def sbm(n: int, seed: int = 1, blocks: int = 10, p_in: float = 4e-4, p_scale: float = 1e-6,
        permute: bool = True) -> Graph:
    """Stochastic block model with hierarchical inter-block density.

    Vertices are split into ``blocks`` consecutive blocks C_1..C_B of equal
    size (the first n mod B blocks one larger).  A pair in C_i x C_j, i < j,
    is an edge with probability p_scale * i^2; a pair inside one block with
    probability p_in.  Every pair is drawn independently.  The inter-block
    rule is the paper's (Sec. 8); the intra-block probability is not given
    there, and the default 4e-4 makes the expected edge count run from
    about 2.8e3 at n = 1e4 to about 2.8e5 at n = 1e5, the range of edges
    that experiment plots."""
    sizes = np.full(blocks, n // blocks, dtype=np.int64)
    sizes[: n % blocks] += 1
    first = np.concatenate([[0], np.cumsum(sizes)])
    es = []
    for i in range(blocks):
        si = int(sizes[i])
        for j in range(i, blocks):
            sj = int(sizes[j])
            p = p_in if i == j else p_scale * (i + 1) ** 2
            idx = _bernoulli_positions(_key(seed, 0x53424D0000 + i * blocks + j), si * sj, min(p, 1.0))
            a = idx // sj
            b = idx % sj
            if i == j:
                keep = a < b          # each unordered pair once, as (a, b) with a < b
                a, b = a[keep], b[keep]
            es.append(np.stack([first[i] + a, first[j] + b], axis=1))
    e = np.concatenate(es) if es else np.zeros((0, 2), np.int64)
    if permute:
        e = random_permutation(n, seed)[e]
    return from_edges(n, e, f"sbm_n{n}_s{seed}")


# ---- small deterministic shapes ---------------------------------------------

def path(n: int) -> Graph:
    return from_edges(n, [(i, i + 1) for i in range(n - 1)], f"path{n}")


def cycle(n: int) -> Graph:
    return from_edges(n, [(i, (i + 1) % n) for i in range(n)] if n >= 3 else [], f"cycle{n}")


def star(leaves: int) -> Graph:
    return from_edges(leaves + 1, [(0, i) for i in range(1, leaves + 1)], f"star{leaves}")


def clique(n: int) -> Graph:
    return from_edges(n, [(a, b) for a in range(n) for b in range(a + 1, n)], f"clique{n}")


def empty(n: int) -> Graph:
    return from_edges(n, np.zeros((0, 2), np.int64), f"empty{n}")


def disjoint_union(*gs: Graph) -> Graph:
    off = 0
    es = []
    for g in gs:
        es.append(g.edges() + off)
        off += g.n
    return from_edges(off, np.concatenate(es) if es else np.zeros((0, 2), np.int64), "union")


def random_small(n: int, p: float, seed: int) -> Graph:
    """Each of the n(n-1)/2 pairs present independently with probability p
    (for tiny brute-force cases)."""
    pairs = [(a, b) for a in range(n) for b in range(a + 1, n)]
    if not pairs:
        return empty(n)
    u = _unit_double(splitmix_stream(_key(seed, 0x534D), 0, len(pairs)))
    return from_edges(n, [pr for pr, x in zip(pairs, u) if x < p], f"small{n}_{seed}")


def lognormal_sizes(count: int, median: float, sigma: float, lo: int, hi: int, seed: int) -> np.ndarray:
    """Vertex counts n ~ lognormal(ln median, sigma), clipped to [lo, hi]
    (Box-Muller on the SplitMix64 stream)."""
    x = _unit_double(splitmix_stream(_key(seed, 0x4C4E), 0, 2 * count))
    u1 = np.maximum(x[0::2], 1e-300)
    u2 = x[1::2]
    z = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * math.pi * u2)
    return np.clip(np.round(median * np.exp(sigma * z)), lo, hi).astype(np.int64)


def loguniform_sizes(count: int, lo: int, hi: int, seed: int) -> np.ndarray:
    x = _unit_double(splitmix_stream(_key(seed, 0x4C55), 0, count))
    return np.clip(np.round(np.exp(math.log(lo) + x * (math.log(hi) - math.log(lo)))), lo, hi).astype(np.int64)


# ---- the named workloads -----------------------------------------------------

def batch_workload(count: int = 4096, lo: int = 100, hi: int = 50_000, base_seed: int = 1) -> list:
    """Many graphs of uneven size: n log-uniform on [lo, hi]; the first half
    Erdos-Renyi with m = 3n (average degree 6), the second half
    Barabasi-Albert with 3 edges per new vertex; graph i uses seed
    base_seed + i."""
    sizes = loguniform_sizes(count, lo, hi, base_seed)
    out = []
    for i in range(count):
        n = int(sizes[i])
        if i < count // 2:
            out.append(erdos_renyi(n, 3 * n, base_seed + i))
        else:
            out.append(barabasi_albert(n, 3, base_seed + i))
    return out


def workload(name: str, seed: int = 1) -> Graph:
    """The single-graph synthetic workloads by name."""
    if name == "er2k":          # ER n=2000, m=8000 (average degree 8)
        return erdos_renyi(2000, 8000, seed)
    if name == "cl1m":          # Chung-Lu n=1e6, m=1e7, gamma=2.1
        return chung_lu(1_000_000, 10_000_000, 2.1, seed)
    if name == "cl4m":          # Chung-Lu n=4e6, m=6e7, gamma=2.3
        return chung_lu(4_000_000, 60_000_000, 2.3, seed)
    if name.startswith("sbm"):  # sbm<n>: the block model above at n vertices
        return sbm(int(name[3:]), seed)
    raise KeyError(name)
