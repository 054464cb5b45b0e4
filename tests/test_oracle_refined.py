"""Pins of the refined bookkeeping of Sec. 5 (oracle/refined.py, Alg. 5 and 6).

After every single deletion of Alg. 4's loop, every alive vertex's B[v,i] and
k[v,i] must equal the closed form of Sec. 3 (the C oracle's sampled_lists, which
is itself pinned in test_oracle.py), the per-entry counts, m[v,i] and D[v,i]
must equal their definitions, and the core numbers must equal the C oracle's
Core.  The refined criterion must re-merge no more lists than the naive Update,
and strictly fewer on graphs where truncation is active."""
import numpy as np
import pytest

import graphgen as gg
import oracle
from oracle.refined import RefinedCore


def check_state(R, g, lists_cache):
    alive = np.array(R.alive, dtype=np.uint8)
    for i in range(1, R.h + 1):
        k, sz, off, mem = oracle.sampled_lists(g, i, R.r, R.M, alive)
        for v in range(R.n):
            if not R.alive[v]:
                continue
            want = set(mem[off[v]:off[v + 1]].tolist())
            assert set(R.B[v][i]) == want, (i, v)
            assert R.k[v][i] == int(k[v]), (i, v)
            nbrs = [w for w in R.adj[v] if R.alive[w]]
            # counts: one for v itself, one per alive neighbour listing the member
            for u, z in R.B[v][i].items():
                assert z == (u == v) + sum(1 for w in nbrs if u in R.B[w][i - 1]), (i, v, u)
            assert R.m[v][i] == sum(1 for w in nbrs if R.k[w][i - 1] == R.k[v][i]), (i, v)
            if R.m[v][i] == 0:
                want_d = {}
                for w in nbrs:
                    for u in R.B[w][i - 1]:
                        if R.r[u] == R.k[v][i] - 1:
                            want_d[u] = want_d.get(u, 0) + 1
                assert R.D[v][i] == want_d, (i, v)


GRAPHS = [
    ("er", lambda: gg.erdos_renyi(40, 110, seed=3)),
    ("cl", lambda: gg.chung_lu(60, 200, 2.1, seed=5)),
    ("ba", lambda: gg.barabasi_albert(50, 3, seed=7)),
]


@pytest.mark.parametrize("name,make", GRAPHS)
@pytest.mark.parametrize("h,M", [(2, 4), (2, 9), (3, 5)])
def test_refined_update_keeps_the_closed_form(name, make, h, M):
    g = make()
    r = oracle.ranks(g.n, 11)
    R = RefinedCore(g, h, r, M)
    check_state(R, g, None)
    core = R.core(after_delete=lambda S: check_state(S, g, None))
    assert np.array_equal(np.array(core, dtype=np.int64), oracle.sampled_core(g, h, r, M))


def test_refined_criterion_saves_merges():
    g = gg.chung_lu(120, 500, 2.1, seed=2)
    r = oracle.ranks(g.n, 4)
    saved = []
    for h, M in [(2, 6), (3, 6), (2, 20)]:
        R = RefinedCore(g, h, r, M)
        core = R.core()
        assert np.array_equal(np.array(core, dtype=np.int64), oracle.sampled_core(g, h, r, M))
        assert R.computes <= R.naive_computes
        saved.append(R.naive_computes - R.computes)
    assert max(saved) > 0


def test_refined_equals_exact_when_M_covers_the_graph():
    # M >= n: every list is the whole ball, the estimate is deg_h (Sec. 3)
    g = gg.erdos_renyi(30, 60, seed=9)
    R = RefinedCore(g, 2, oracle.ranks(g.n, 1), g.n + 1)
    core = R.core()
    assert np.array_equal(np.array(core, dtype=np.int64), oracle.exact_core(g, 2))
