"""GPU tests of the serving loop (kh_serve_*): every request's result is the
same alone and in a mix of concurrent requests, and the ticket protocol and
admission behave as declared."""
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


def pool(count=10, seed=3):
    """Chung-Lu graphs (gamma 2.2, average degree 10) of uneven size."""
    sizes = gg.lognormal_sizes(count, 800, 1.0, 60, 6000, seed)
    return [gg.chung_lu(int(n), 5 * int(n), 2.2, seed=seed + i) for i, n in enumerate(sizes)]


def requests(gs, count, seed):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        gi = int(rng.integers(len(gs)))
        h = int(rng.integers(2, 4))
        eps = 0.5 if rng.random() < 0.5 else 0.0
        out.append((gi, h, eps))
    return out


def kwargs(eps):
    return dict(seed=9) if eps > 0 else {}


def test_serve_alone_equals_mix(ctx):
    gs = pool()
    Gs = [kh.Graph.from_gg(ctx, g) for g in gs]
    reqs = requests(gs, 48, 1)
    alone = {}
    for gi, h, eps in set(reqs):
        say("alone", gi, h, eps)
        alone[(gi, h, eps)] = kh.core(Gs[gi], h, epsilon=eps, **kwargs(eps))[0]
    srv = kh.Server(ctx, workers=4)
    try:
        say("mix", len(reqs))
        tickets = [srv.submit(Gs[gi], h, epsilon=eps, **kwargs(eps)) for gi, h, eps in reqs]
        for t, key in zip(tickets, reqs):
            core, res = srv.wait(t)
            assert np.array_equal(core, alone[key]), key
            assert res["max_core"] == int(alone[key].max())
            assert res["seconds"] > 0
        # and against the oracle for the smallest graphs
        small = sorted(range(len(gs)), key=lambda i: gs[i].n)[:3]
        for gi in small:
            for h in (2, 3):
                t1 = srv.submit(Gs[gi], h)
                t2 = srv.submit(Gs[gi], h, epsilon=0.5, seed=9)
                assert np.array_equal(srv.wait(t1)[0].astype(np.int64), oracle.exact_core(gs[gi], h))
                M = oracle.M_int(gs[gi].n, 0.5)
                want = oracle.sampled_core(gs[gi], h, oracle.ranks(gs[gi].n, 9), M)
                assert np.array_equal(srv.wait(t2)[0].astype(np.int64), want)
    finally:
        srv.stop()


def test_serve_ticket_protocol(ctx):
    g = gg.erdos_renyi(300, 900, seed=2)
    G = kh.Graph.from_gg(ctx, g)
    srv = kh.Server(ctx, workers=2)
    try:
        with pytest.raises(kh.KhError) as e:
            srv.poll(123456789)
        assert e.value.code == kh.khcore.KH_ENOTFOUND
        t = srv.submit(G, 2)
        got = None
        while got is None:
            got = srv.poll(t)
        assert np.array_equal(got[0].astype(np.int64), oracle.exact_core(g, 2))
        with pytest.raises(kh.KhError) as e:
            srv.poll(t)  # retired
        assert e.value.code == kh.khcore.KH_ENOTFOUND
        with pytest.raises(kh.KhError) as e:
            srv.submit(G, 0)
        assert e.value.code == -1
        # withdrawing: unknown tickets are not found; a queued request may be
        # withdrawn, a running or finished one must be collected
        with pytest.raises(kh.KhError) as e:
            srv.cancel(987654321)
        assert e.value.code == kh.khcore.KH_ENOTFOUND
        big = gg.barabasi_albert(20000, 3, seed=5)
        GB = kh.Graph.from_gg(ctx, big)
        t1 = srv.submit(GB, 3)
        t2 = srv.submit(GB, 3)
        t3 = srv.submit(G, 2, epsilon=0.5, seed=1)
        for t in (t2, t3):
            if srv.cancel(t):
                with pytest.raises(kh.KhError) as e:
                    srv.poll(t)
                assert e.value.code == kh.khcore.KH_ENOTFOUND
            else:
                assert srv.wait(t)[0].size > 0
        srv.wait(t1)
        # a second start on a serving context is refused
        with pytest.raises(kh.KhError) as e:
            kh.Server(ctx)
        assert e.value.code == kh.khcore.KH_EBUSY
    finally:
        srv.stop()


def test_serve_tiny_budget_runs_one_at_a_time(ctx):
    gs = pool(6, seed=11)
    Gs = [kh.Graph.from_gg(ctx, g) for g in gs]
    srv = kh.Server(ctx, workers=3, hbm_budget=1, batch_vertices=1)
    try:
        say("tiny budget")
        ts = [srv.submit(G, 2) for G in Gs] + [srv.submit(G, 3, epsilon=0.5, seed=4) for G in Gs]
        for i, t in enumerate(ts):
            core, _ = srv.wait(t)
            G = Gs[i % len(Gs)]
            want = kh.core(G, 2)[0] if i < len(Gs) else kh.core(G, 3, epsilon=0.5, seed=4)[0]
            assert np.array_equal(core, want)
    finally:
        srv.stop()


def test_serve_device_outputs(ctx):
    gs = pool(5, seed=21)
    Gs = [kh.Graph.from_gg(ctx, g) for g in gs]
    srv = kh.Server(ctx)
    try:
        outs = [torch.full((g.n,), -1, dtype=torch.int32, device="cuda:0") for g in gs]
        ts = [srv.submit(G, 2, out=o) for G, o in zip(Gs, outs)]
        for t, G, o in zip(ts, Gs, outs):
            srv.wait(t)
            assert np.array_equal(o.cpu().numpy(), kh.core(G, 2)[0])
    finally:
        srv.stop()


def test_concurrent_calls_on_one_context(ctx):
    # plain kh_core calls from several host threads on one context (no server)
    import threading
    gs = pool(6, seed=31)
    Gs = [kh.Graph.from_gg(ctx, g) for g in gs]
    want = [oracle.exact_core(g, 2) if g.n <= 3000 else kh.core(G, 2)[0].astype(np.int64) for g, G in zip(gs, Gs)]
    got = [None] * len(gs)
    errors = []

    def run(i):
        try:
            for _ in range(3):
                c, _ = kh.core(Gs[i], 2)
                got[i] = c.astype(np.int64)
        except Exception as e:  # noqa: BLE001
            errors.append(e)

    say("concurrent kh_core threads")
    threads = [threading.Thread(target=run, args=(i,)) for i in range(len(gs))]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not errors
    for g, w, c in zip(gs, want, got):
        assert np.array_equal(c, w), g.name


def test_stop_while_callers_wait(ctx):
    # kh_serve_stop finishes the queued requests; a kh_serve_wait blocked
    # meanwhile returns its result or, if the stop dropped it first,
    # KH_ENOTFOUND -- never a crash.  A new loop can start afterwards.
    import threading
    gs = pool(4, seed=5)
    Gs = [kh.Graph.from_gg(ctx, g) for g in gs]
    want = {gi: kh.core(Gs[gi], 2)[0] for gi in range(4)}
    S = kh.Server(ctx, workers=1)
    tickets = [(S.submit(Gs[i % 4], 2), i % 4) for i in range(12)]
    got = {}

    def waiter(t, gi):
        try:
            got[t] = ("ok", S.wait(t)[0], gi)
        except kh.KhError as e:
            got[t] = ("err", e.code, gi)

    ths = [threading.Thread(target=waiter, args=tg) for tg in tickets[-4:]]
    for th in ths:
        th.start()
    say("stop while waiting")
    S.stop()
    for th in ths:
        th.join(timeout=60)
        assert not th.is_alive()
    assert len(got) == 4
    for kind, val, gi in got.values():
        if kind == "ok":
            assert np.array_equal(val, want[gi])
        else:
            assert val == kh.khcore.KH_ENOTFOUND
    S2 = kh.Server(ctx, workers=2)
    t = S2.submit(Gs[1], 2)
    assert np.array_equal(S2.wait(t)[0], want[1])
    S2.stop()
