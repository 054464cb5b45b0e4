"""GPU parity of the full EstDense (Alg. 7 over every suffix of the deletion
order, flag KH_DENSE_FULL) against the oracle's bulk-round order and suffix
sums, exact and sampled, with and without the pruning variant."""
import sys
from fractions import Fraction

import numpy as np
import pytest

import graphgen as gg
import oracle

torch = pytest.importorskip("torch")
kh = pytest.importorskip("paper_2112_06154_amd")

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = kh.Context(0)
    yield c
    c.close()


def oracle_full(g, h, mode, r0, M, r1, M2, prune, eps):
    order, core, _ = oracle.bulk_order(g, h, mode, r0, M)
    if prune:
        e = eps if mode == "sampled" else 0.0
        keep = core.astype(np.float64) * (1.0 + e) >= (1.0 - e) * float(core.max())
        order = order[keep[order]]
    res = oracle.dense_suffix(g, order, h, mode, r1, M2)
    return core, res["size"], res["best_R"], int(core[order[res["best"]]])


GRAPHS = [lambda: gg.erdos_renyi(1200, 4800, seed=21), lambda: gg.barabasi_albert(700, 3, seed=22),
          lambda: gg.chung_lu(900, 3600, 2.2, seed=23)]


@pytest.mark.parametrize("gi", range(3))
def test_dense_full_exact(ctx, gi):
    g = GRAPHS[gi]()
    G = kh.Graph.from_gg(ctx, g)
    for h in (2, 3):
        for prune in (False, True):
            say("dense full exact", g.name, h, prune)
            got, res = kh.core(G, h, dense_full=True, prune=prune)
            core, size, R, k = oracle_full(g, h, "exact", None, 0, None, 0, prune, 0.0)
            assert np.array_equal(got.astype(np.int64), core)
            assert (res["dense_size"], res["dense_R"], res["dense_k"]) == (size, R, k)
            # the core levels are suffixes: the full variant is at least as dense
            _, lvl = kh.core(G, h, dense=True, prune=prune)
            assert Fraction(R, size) >= Fraction(lvl["dense_R"], lvl["dense_size"])


@pytest.mark.parametrize("gi", range(3))
def test_dense_full_sampled(ctx, gi):
    g = GRAPHS[gi]()
    G = kh.Graph.from_gg(ctx, g)
    seed = 30 + gi
    r0, r1 = oracle.ranks(g.n, seed, 0), oracle.ranks(g.n, seed, 1)
    for h in (2, 3):
        for M, M2 in ((12, 20), (0, 0)):
            for prune in (False, True):
                Mi = M if M else oracle.M_int(g.n, 0.5)
                M2i = M2 if M2 else oracle.M_int(g.n, 0.5, dense=True)
                say("dense full sampled", g.name, h, Mi, M2i, prune)
                got, res = kh.core(G, h, epsilon=0.5, seed=seed, M_override=M, M_dense_override=M2,
                                   dense_full=True, prune=prune)
                core, size, R, k = oracle_full(g, h, "sampled", r0, Mi, r1, M2i, prune, 0.5)
                assert np.array_equal(got.astype(np.int64), core)
                assert res["M_dense_used"] == M2i
                assert (res["dense_size"], res["dense_R"], res["dense_k"]) == (size, R, k)


def test_dense_full_rejected_where_the_order_is_unknown(ctx):
    g = gg.erdos_renyi(200, 600, seed=5)
    G = kh.Graph.from_gg(ctx, g)
    with pytest.raises(kh.KhError) as e:
        kh.core_batch([G], 2, dense_full=True)
    assert e.value.code == kh.KH_ENOTIMPL
    with pytest.raises(kh.KhError) as e:
        kh.dense(G, np.zeros(g.n, np.int32), 2, dense_full=True)
    assert e.value.code == kh.KH_ENOTIMPL
    with pytest.raises(kh.KhError) as e:
        kh.core(G, 2, epsilon=0.5, dense_full=True, early_stop=True)
    assert e.value.code == kh.KH_ENOTIMPL
