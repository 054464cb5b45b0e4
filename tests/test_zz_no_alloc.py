"""kh_hdeg_noalloc (the entry point for callers that cannot allocate) against
kh_hdeg through the C ABI: identical h-degrees and edges-traversed counts on
two calls in a row that share the fixed device array, the second on a smaller
graph, and the size limit rejected on the host before anything runs."""
import sys

import numpy as np
import pytest

import graphgen as gg

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


def run_noalloc(G, n, h, alive=None):
    deg = torch.full((max(n, 1),), -7, dtype=torch.int32, device="cuda")
    te = torch.zeros(1, dtype=torch.int64, device="cuda")
    kh.hdeg_noalloc(G, h, deg, alive=alive, te_out=te)
    torch.cuda.synchronize()
    return deg[:n].cpu().numpy(), int(te.item())


def test_noalloc_matches_kh_hdeg_on_consecutive_calls(ctx):
    # the first graph is large enough that the bit planes narrow to fit the array
    big = gg.chung_lu(150_000, 750_000, 2.2, seed=11)
    small = gg.erdos_renyi(3000, 9000, seed=12)
    Gb = kh.Graph.from_gg(ctx, big)
    Gs = kh.Graph.from_gg(ctx, small)
    rng = np.random.default_rng(13)
    alive_np = (rng.random(big.n) < 0.8).astype(np.uint8)
    alive = torch.from_numpy(alive_np).cuda()
    for rep in range(2):
        for G, g, h, al in ((Gb, big, 2, alive), (Gs, small, 3, None), (Gs, small, 1, None)):
            say("noalloc", rep, g.name, h, al is not None)
            got, te = run_noalloc(G, g.n, h, al)
            want, te_want = kh.hdeg(G, h, al)
            assert np.array_equal(got, want)
            assert te == te_want
    # edge cases: one vertex, isolated vertices, a hub split into many pieces
    for g in (gg.empty(1), gg.empty(40), gg.disjoint_union(gg.star(5000), gg.path(300), gg.empty(3))):
        G = kh.Graph.from_gg(ctx, g)
        for h in (1, 2, 3):
            say("noalloc edge", g.name, h)
            got, te = run_noalloc(G, g.n, h)
            want, te_want = kh.hdeg(G, h)
            assert np.array_equal(got, want) and te == te_want


def test_noalloc_rejects_graphs_beyond_the_array(ctx):
    g = gg.empty(1_000_000)  # about 110 bytes per vertex even at one word per vertex
    G = kh.Graph.from_gg(ctx, g)
    deg = torch.zeros(g.n, dtype=torch.int32, device="cuda")
    with pytest.raises(kh.KhError) as e:
        kh.hdeg_noalloc(G, 2, deg)
    assert e.value.code == kh.KH_ENOMEM
    with pytest.raises(kh.KhError) as e:
        kh.hdeg_noalloc(G, 0, deg)
    assert e.value.code == kh.KH_EINVAL
