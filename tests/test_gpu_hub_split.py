"""GPU parity of split hub merges, through the C ABI.

During the sampled peel a hub of a level's worklist with more than KH_HUB_SLICE
arcs (8192 by default) is merged in slices: each slice's neighbour lists are
merged in parallel into a partial list, and the hub then merges its slices'
partial lists (the truncated union of Alg. 2 / Prop. dyn is associative above
the largest slice level).  The tests force small slices so that graphs the
oracle can check take that path, and compare with the oracle and with the
unsplit merge on larger graphs.
"""
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


def hub_graph(n, m, hub_degree, seed):
    """Erdos-Renyi G(n, m) plus one hub (vertex n) adjacent to hub_degree of its vertices."""
    base = gg.erdos_renyi(n, m, seed=seed)
    rng = np.random.default_rng(seed)
    nb = rng.choice(n, hub_degree, replace=False)
    edges = [tuple(int(x) for x in e) for e in base.edges()] + [(n, int(v)) for v in nb]
    return gg.from_edges(n + 1, edges)


@pytest.mark.parametrize("slice_arcs", [128, 300, 1024])
@pytest.mark.parametrize("h,M", [(2, 40), (2, 0), (3, 40)])
def test_split_hub_sampled_core_matches_oracle(ctx, monkeypatch, slice_arcs, h, M):
    monkeypatch.setenv("KH_HUB_SLICE", str(slice_arcs))
    g = hub_graph(1200, 2400, 1100, seed=3)
    assert int(np.diff(g.row_ptr).max()) > max(1024, slice_arcs)
    G = kh.Graph.from_gg(ctx, g)
    Mi = M if M else oracle.M_int(g.n, 0.5)
    say("split hub sampled core", slice_arcs, h, Mi)
    got, res = kh.core(G, h, epsilon=0.5, seed=5, M_override=M)
    want = oracle.sampled_core(g, h, oracle.ranks(g.n, 5), Mi)
    assert res["M_used"] == Mi
    assert np.array_equal(got.astype(np.int64), want)


def _run(G, h, **kw):
    core, res = kh.core(G, h, epsilon=0.5, seed=11, **kw)
    keys = ("M_used", "rounds", "max_core", "dense_k", "dense_size", "dense_density", "list_elements")
    return core, {k: res[k] for k in keys if k in res}


@pytest.mark.parametrize("h", [2, 3])
@pytest.mark.parametrize("lazy", [False, True])
def test_split_equals_whole_hub_merges(ctx, monkeypatch, h, lazy):
    # several hubs above 1024 arcs (max degree ~1,700), split into 256-arc slices
    g = gg.chung_lu(5000, 25000, 2.1, seed=1)
    G = kh.Graph.from_gg(ctx, g)
    say("split vs whole", h, lazy)
    monkeypatch.setenv("KH_HUB_SLICE", "0")
    c0, r0 = _run(G, h, dense=True, prune=True, lazy_init=lazy)
    monkeypatch.setenv("KH_HUB_SLICE", "256")
    c1, r1 = _run(G, h, dense=True, prune=True, lazy_init=lazy)
    assert np.array_equal(c0, c1)
    for k in ("M_used", "rounds", "max_core", "dense_k", "dense_size", "dense_density"):
        assert r0[k] == r1[k], k


def test_split_on_larger_power_law_graph(ctx, monkeypatch):
    # max degree above 8192: the default slice size splits the largest hubs
    g = gg.chung_lu(60000, 600000, 2.1, seed=4)
    assert int(np.diff(g.row_ptr).max()) > 2 * 8192
    G = kh.Graph.from_gg(ctx, g)
    for h in (2, 3):
        say("split on chung_lu(60000)", h)
        monkeypatch.setenv("KH_HUB_SLICE", "0")
        c0, r0 = _run(G, h, dense=True, prune=True)
        monkeypatch.delenv("KH_HUB_SLICE")
        c1, r1 = _run(G, h, dense=True, prune=True)
        assert np.array_equal(c0, c1)
        for k in ("M_used", "rounds", "max_core", "dense_k", "dense_size", "dense_density"):
            assert r0[k] == r1[k], k
