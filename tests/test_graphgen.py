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


def test_bernoulli_positions_are_independent_coin_flips():
    # each index kept with probability p, independently of the others
    total, p, trials = 12, 0.3, 6000
    hits = np.zeros((trials, total), dtype=np.float64)
    for t in range(trials):
        hits[t, gg._bernoulli_positions(gg._key(t, 77), total, p)] = 1.0
    freq = hits.mean(axis=0)
    sd = np.sqrt(p * (1 - p) / trials)
    assert np.all(np.abs(freq - p) < 5 * sd), freq
    corr = np.corrcoef(hits.T)[np.triu_indices(total, 1)]
    assert np.all(np.abs(corr) < 5 / np.sqrt(trials)), corr.max()
    assert gg._bernoulli_positions(5, 0, 0.5).size == 0
    assert gg._bernoulli_positions(5, 7, 0.0).size == 0
    assert gg._bernoulli_positions(5, 7, 1.0).tolist() == list(range(7))
    big = gg._bernoulli_positions(9, 2_000_000, 0.01)
    assert np.all(np.diff(big) > 0) and big[-1] < 2_000_000
    assert abs(big.size - 20_000) < 5 * np.sqrt(20_000 * 0.99)


def test_sbm_block_structure():
    n, blocks = 100_000, 10
    g = gg.sbm(n, seed=2, permute=False)
    canonical(g)
    s = n // blocks
    e = g.edges()
    bi, bj = e[:, 0] // s, e[:, 1] // s
    counts = np.zeros((blocks, blocks), np.int64)
    np.add.at(counts, (bi, bj), 1)
    for i in range(blocks):
        for j in range(blocks):
            if j < i:
                assert counts[i, j] == 0          # edges stored with u < v
                continue
            p = 4e-4 if i == j else 1e-6 * (i + 1) ** 2
            pairs = s * (s - 1) // 2 if i == j else s * s
            mu = pairs * p
            assert abs(counts[i, j] - mu) < 5 * np.sqrt(mu * (1 - p)) + 1, (i, j, counts[i, j], mu)
    # the range of edge counts of the paper's scaling experiment
    assert 275_000 < g.m < 290_000
    assert 2_500 < gg.sbm(10_000, seed=2).m < 3_100
    # seeded and permuted
    a, b = gg.workload("sbm20000", seed=3), gg.sbm(20_000, seed=3)
    assert np.array_equal(a.col, b.col) and np.array_equal(a.row_ptr, b.row_ptr)
    assert not np.array_equal(gg.sbm(20_000, seed=4).col, b.col)
    uneven = gg.sbm(1003, seed=1, p_in=0.05)
    canonical(uneven)
    assert uneven.n == 1003
