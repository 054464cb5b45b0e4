"""The seeded input generators (shared by the oracle tests and the GPU tests):
canonical CSR, determinism, and the C preferential-attachment drawer giving
the same graph as the pure-Python loop."""
import os

import numpy as np
import pytest

import graphgen as gg


def canonical(g):
    rp, col = g.row_ptr, g.col
    assert rp[0] == 0 and rp[-1] == col.size
    for v in range(g.n):
        a = col[rp[v]:rp[v + 1]]
        assert np.all(np.diff(a) > 0)
        assert not np.any(a == v)
    src = np.repeat(np.arange(g.n), np.diff(rp))
    fwd = set(zip(src.tolist(), col.tolist()))
    assert all((b, a) in fwd for a, b in fwd)


@pytest.mark.parametrize("n,seed", [(5, 1), (60, 2), (2500, 9)])
def test_ba_native_equals_python_loop(n, seed, monkeypatch):
    if not os.path.exists(gg._BA_LIB):
        gg.build_native()
    a = gg.barabasi_albert(n, 3, seed)
    monkeypatch.setattr(gg, "_ba_native", lambda *args: None)
    b = gg.barabasi_albert(n, 3, seed)
    assert np.array_equal(a.row_ptr, b.row_ptr) and np.array_equal(a.col, b.col)
    canonical(a)
    # every vertex after the seed clique brings 3 edges
    assert a.col.size // 2 == 6 + 3 * (n - 4) if n > 4 else True


def test_batch_workload_shape():
    gs = gg.batch_workload(count=16, lo=100, hi=3000, base_seed=4)
    assert len(gs) == 16
    sizes = gg.loguniform_sizes(16, 100, 3000, 4)
    for i, g in enumerate(gs):
        assert g.n == sizes[i]
        canonical(g)
        if i < 8:
            assert g.col.size == 2 * 3 * g.n          # ER with m = 3n
        else:
            assert g.col.size == 2 * (6 + 3 * (g.n - 4))  # BA, 3 edges per new vertex
    again = gg.batch_workload(count=16, lo=100, hi=3000, base_seed=4)
    assert all(np.array_equal(x.col, y.col) for x, y in zip(gs, again))
