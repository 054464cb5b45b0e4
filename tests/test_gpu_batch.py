"""GPU parity of kh_core_batch: every graph of a packed batch gets exactly the
core numbers (and densest core) it gets alone, and those of the oracle."""
import sys

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


def mixed_graphs():
    """Uneven small graphs of both batch families plus degenerate ones."""
    gs = gg.batch_workload(count=20, lo=20, hi=600, base_seed=7)
    gs += [gg.empty(1), gg.path(2), gg.star(300), gg.clique(25), gg.empty(6),
           gg.disjoint_union(gg.cycle(9), gg.path(5)), gg.chung_lu(700, 2500, 2.1, seed=3)]
    return gs


def load(ctx, gs):
    out = []
    for g in gs:
        if g.n == 0:
            out.append(kh.Graph(ctx, 0, np.zeros(1, np.int32), np.zeros(0, np.int32)))
        else:
            out.append(kh.Graph.from_gg(ctx, g))
    return out


def test_batch_exact_matches_oracle_and_single(ctx):
    gs = mixed_graphs()
    Gs = load(ctx, gs)
    for h in (1, 2, 3):
        say("batch exact", h, len(gs))
        cores, res = kh.core_batch(Gs, h)
        for g, G, c, r in zip(gs, Gs, cores, res):
            want = oracle.exact_core(g, h)
            assert np.array_equal(c.astype(np.int64), want), g.name
            assert r["max_core"] == int(want.max())
            single, _ = kh.core(G, h)
            assert np.array_equal(c, single)


def test_batch_with_empty_graphs(ctx):
    gs = [gg.path(7), None, gg.star(12), None]
    Gs = []
    for g in gs:
        Gs.append(kh.Graph(ctx, 0, np.zeros(1, np.int32), np.zeros(0, np.int32)) if g is None
                  else kh.Graph.from_gg(ctx, g))
    say("batch with n = 0 members")
    cores, res = kh.core_batch(Gs, 2)
    assert cores[1].size == 0 and cores[3].size == 0
    assert np.array_equal(cores[0].astype(np.int64), oracle.exact_core(gs[0], 2))
    assert np.array_equal(cores[2].astype(np.int64), oracle.exact_core(gs[2], 2))
    assert kh.core_batch([], 2) == ([], [])


def test_batch_sampled_matches_oracle(ctx):
    gs = mixed_graphs()
    Gs = load(ctx, gs)
    for h in (2, 3):
        for M in (0, 6):
            seed = 77
            say("batch sampled", h, M)
            cores, res = kh.core_batch(Gs, h, epsilon=0.5, seed=seed, M_override=M)
            for g, c, r in zip(gs, cores, res):
                Mi = M if M else oracle.M_int(g.n, 0.5)
                want = oracle.sampled_core(g, h, oracle.ranks(g.n, seed), Mi)
                assert r["M_used"] == Mi
                assert np.array_equal(c.astype(np.int64), want), g.name


def test_batch_device_outputs_and_chunks(ctx, monkeypatch):
    gs = mixed_graphs()
    Gs = load(ctx, gs)
    want_e = [oracle.exact_core(g, 2) for g in gs]
    want_s = [oracle.sampled_core(g, 2, oracle.ranks(g.n, 5), 9) for g in gs]
    for chunk in (None, "700", "1"):
        if chunk:
            monkeypatch.setenv("KH_BATCH_MAX_VERTICES", chunk)
        else:
            monkeypatch.delenv("KH_BATCH_MAX_VERTICES", raising=False)
        say("batch device outputs, union size limit", chunk)
        outs = [torch.full((max(g.n, 1),), -7, dtype=torch.int32, device="cuda:0") for g in gs]
        kh.core_batch(Gs, 2, outs=outs)
        for g, o, w in zip(gs, outs, want_e):
            assert np.array_equal(o.cpu().numpy()[:g.n].astype(np.int64), w)
        cores, _ = kh.core_batch(Gs, 2, epsilon=0.5, seed=5, M_override=9)
        for c, w in zip(cores, want_s):
            assert np.array_equal(c.astype(np.int64), w)
    monkeypatch.delenv("KH_BATCH_MAX_VERTICES", raising=False)


def test_batch_dense_matches_single(ctx):
    gs = mixed_graphs()[:8]
    Gs = load(ctx, gs)
    for h in (2, 3):
        for eps in (0.0, 0.5):
            say("batch dense", h, eps)
            kw = dict(seed=11, M_override=12, M_dense_override=20) if eps > 0 else {}
            cores, res = kh.core_batch(Gs, h, epsilon=eps, dense=True, **kw)
            for G, c, r in zip(Gs, cores, res):
                c1, r1 = kh.core(G, h, epsilon=eps, dense=True, **kw)
                assert np.array_equal(c, c1)
                for f in ("dense_k", "dense_size", "dense_R", "M_used", "M_dense_used", "max_core"):
                    assert r[f] == r1[f], f


def test_batch_workload_slice_matches_single(ctx):
    # graphs of the 4,096-graph batch workload itself (both families, large
    # and small n), batched against their single-graph results
    full = gg.loguniform_sizes(4096, 100, 50_000, 1)
    idx = [0, 1, 2, 3, 2048, 2049, 2050, 2051]
    gs = [gg.erdos_renyi(int(full[i]), 3 * int(full[i]), 1 + i) if i < 2048
          else gg.barabasi_albert(int(full[i]), 3, 1 + i) for i in idx]
    Gs = load(ctx, gs)
    for h in (2, 3):
        say("batch workload slice", h, [g.n for g in gs])
        cores, _ = kh.core_batch(Gs, h)
        for g, G, c in zip(gs, Gs, cores):
            single, _ = kh.core(G, h)
            assert np.array_equal(c, single)
            if g.n <= 1500:
                assert np.array_equal(c.astype(np.int64), oracle.exact_core(g, h))


def test_batch_rejects_early_stop(ctx):
    G = kh.Graph.from_gg(ctx, gg.path(5))
    with pytest.raises(kh.KhError) as e:
        kh.core_batch([G], 2, epsilon=0.5, early_stop=True)
    assert e.value.code == -8


def test_batch_many_tiny_graphs(ctx):
    # hundreds of graphs of 1..12 vertices: one 64-vertex tile holds many graphs
    rng = np.random.default_rng(5)
    gs = [gg.random_small(int(rng.integers(1, 13)), float(rng.uniform(0.1, 0.7)), seed=i) for i in range(300)]
    Gs = load(ctx, gs)
    for h in (1, 2, 3):
        say("batch tiny graphs", h)
        cores, _ = kh.core_batch(Gs, h)
        for g, c in zip(gs, cores):
            assert np.array_equal(c.astype(np.int64), oracle.exact_core(g, h)), g.name
        cs, _ = kh.core_batch(Gs, h, epsilon=0.5, seed=3, M_override=3)
        for g, c in zip(gs, cs):
            assert np.array_equal(c.astype(np.int64), oracle.sampled_core(g, h, oracle.ranks(g.n, 3), 3)), g.name
