"""Pins of the CPU oracle against what the paper and mathematics fix.

Each test ties an oracle function to something other than itself: values the
paper prints (Table 1), published generator vectors, hand-derived worked
examples of Def. est, a graph library (networkx), brute force over all
vertex subsets of tiny graphs, closed forms, and the paper's propositions.
"""
import math
from fractions import Fraction

import networkx as nx
import numpy as np
import pytest

import brute
import graphgen as gg
import oracle
from conftest import golden_rows


def to_nx(g, alive=None):
    G = nx.Graph()
    nodes = range(g.n) if alive is None else [v for v in range(g.n) if alive[v]]
    G.add_nodes_from(nodes)
    e = g.edges()
    for u, v in e:
        if alive is None or (alive[u] and alive[v]):
            G.add_edge(int(u), int(v))
    return G


# ---- Eq. (buffer), Table 1 --------------------------------------------------

def test_M_reproduces_table1():
    rows = golden_rows("table1_M.txt")
    assert len(rows) == 8
    for name, n, printed in rows:
        assert oracle.M_int(int(n), 0.5, 0.05) == int(printed), name


def test_M_dense_is_M_of_half_n_squared():
    # Alg. 7 sets C = log(n^2/delta); Eq. (buffer) for Alg. 4 has C = log(2N/delta).
    # So the dense M of n equals the Table-1-pinned M of N = n^2/2 (even n): a
    # wrong constant in either C (e.g. log(2n^2/delta)) breaks the identity.
    for n in (2, 10, 1000, 12008, 1_000_000, 4_000_000):
        for eps in (0.25, 0.5, 0.9):
            assert oracle.M_real(n, eps, 0.05, dense=True) == oracle.M_real(n * n // 2, eps, 0.05, dense=False)
            assert oracle.M_int(n, eps, 0.05, dense=True) == oracle.M_int(n * n // 2, eps, 0.05, dense=False)


def test_M_dense_uses_log_n2_over_delta():
    # Alg. 7 sets C = log(n^2/delta); check against the formula's pieces.
    n, eps, delta = 10 ** 6, 0.5, 0.05
    C = math.log(n * n / delta)
    expect = 1 + 4 * (2 + eps) / eps ** 2 * (C + math.log(8))
    assert abs(oracle.M_real(n, eps, delta, dense=True) - expect) < 1e-9
    assert oracle.M_int(n, eps, delta, dense=True) == math.floor(expect)
    assert oracle.M_int(n, eps, delta, dense=True) > oracle.M_int(n, eps, delta)


# ---- ranks -------------------------------------------------------------------

def test_splitmix64_published_vectors():
    golden = 0x9E3779B97F4A7C15
    for idx, hexv in golden_rows("splitmix64_vectors.txt"):
        i = int(idx)
        assert oracle.splitmix64((i * golden) & 0xFFFFFFFFFFFFFFFF) == int(hexv, 16)


def test_rank_distribution_geometric_half():
    # Sec. 3: r ~ geo(1/2), P(r >= k) = 2^-k.  Chi-square over 1e6 vertices.
    n = 1_000_000
    r = oracle.ranks(n, seed=12345, stream=0).astype(np.int64)
    counts = np.bincount(r, minlength=64)
    chi2 = 0.0
    dof = 0
    for k in range(0, 14):
        e = n * 2.0 ** -(k + 1)
        chi2 += (counts[k] - e) ** 2 / e
        dof += 1
    tail_e = n * 2.0 ** -14
    chi2 += (counts[14:].sum() - tail_e) ** 2 / tail_e
    assert chi2 < 45.0, chi2  # dof 14; p ~ 5e-5
    # streams are different draws
    r1 = oracle.ranks(n, seed=12345, stream=1).astype(np.int64)
    assert (r1 != r).mean() > 0.4


# ---- Def. est ------------------------------------------------------------------

def test_delta_worked_examples():
    for row in golden_rows("delta_examples.txt"):
        M, d = int(row[0]), int(row[1])
        x = [int(t) for t in row[2:2 + d]]
        assert oracle.delta_est(x, M) == int(row[2 + d]), row
        assert brute.delta_def(x, M) == int(row[2 + d]), row


def test_delta_exact_when_few():
    # If S_0 = d <= M then k = 0 and Delta = d - 1 whatever the ranks.
    rng = np.random.default_rng(1)
    for _ in range(200):
        d = int(rng.integers(1, 30))
        x = rng.integers(0, 10, d)
        assert oracle.delta_est(x, 30) == d - 1


def test_delta_monotone_prop():
    # Prop. monotone: Delta of a prefix keeping x_1 is at most Delta of all.
    rng = np.random.default_rng(2)
    for _ in range(3000):
        d = int(rng.integers(1, 40))
        x = rng.geometric(0.5, d) - 1
        M = int(rng.integers(1, 8))
        full = oracle.delta_est(x, M)
        for dp in range(1, d + 1):
            assert oracle.delta_est(x[:dp], M) <= full
        # and any subset that keeps x_1 (order of the rest does not matter)
        keep = rng.random(d) < 0.5
        keep[0] = True
        assert oracle.delta_est(x[keep], M) <= full


def test_delta_accuracy_prop_approx():
    # Prop. approx: |Delta - (d-1)| <= eps (d-1) w.p. 1 - e^-C for eps <= 1/2.
    eps = 0.5
    C = math.log(2 * 1000 / 0.05)
    M = math.floor(1 + 4 * (2 + eps) / eps ** 2 * (C + math.log(8)))
    rng = np.random.default_rng(3)
    for d in (M // 2, M + 1, 2 * M, 10 * M, 100 * M):
        for _ in range(40):
            x = rng.geometric(0.5, d) - 1
            est = oracle.delta_est(x, M)
            assert abs(est - (d - 1)) <= eps * (d - 1) + 1e-9, (d, est)


# ---- h-degree ----------------------------------------------------------------

@pytest.mark.parametrize("seed", range(6))
def test_hdeg_matches_networkx(seed):
    g = gg.erdos_renyi(60, 110, seed=seed) if seed % 2 else gg.barabasi_albert(60, 2, seed=seed)
    rng = np.random.default_rng(seed)
    alive = (rng.random(g.n) < 0.8).astype(np.uint8)
    G = to_nx(g, alive)
    for h in (1, 2, 3, 4):
        deg = oracle.hdeg(g, h, alive)
        for v in range(g.n):
            if alive[v]:
                expect = len(nx.single_source_shortest_path_length(G, v, cutoff=h)) - 1
                assert deg[v] == expect
            else:
                assert deg[v] == -1


def test_hdeg_list_equals_hdeg_all_on_permuted_sources():
    # the per-source entry point returns, in the order given, the values of the
    # all-vertex pass (itself pinned to networkx above), dead sources as -1
    g = gg.chung_lu(500, 2500, 2.2, seed=3)
    rng = np.random.default_rng(5)
    alive = (rng.random(g.n) < 0.9).astype(np.uint8)
    for h in (1, 2, 3):
        full, te_full = oracle.hdeg(g, h, alive, with_te=True)
        src = rng.permutation(g.n)[:137].astype(np.int32)
        got, te = oracle.hdeg_list(g, h, src, alive, with_te=True)
        assert np.array_equal(got, full[src])
        # all sources in any order: same values and the same edges-traversed total
        perm = rng.permutation(g.n).astype(np.int32)
        got_all, te_all = oracle.hdeg_list(g, h, perm, alive, with_te=True)
        assert np.array_equal(got_all, full[perm])
        assert te_all == te_full


def test_edges_traversed_count():
    # TE of one source = sum of alive degrees over vertices within h-1 hops.
    g = gg.erdos_renyi(80, 200, seed=4)
    G = to_nx(g)
    for h in (1, 2, 3):
        _, te = oracle.hdeg(g, h, with_te=True)
        expect = 0
        for s in range(g.n):
            for u, d in nx.single_source_shortest_path_length(G, s, cutoff=h - 1).items():
                expect += G.degree(u)
        assert te == expect


# ---- ExactCore -----------------------------------------------------------------

@pytest.mark.parametrize("seed", range(5))
def test_exact_h1_is_classic_kcore(seed):
    g = gg.chung_lu(400, 1500, 2.3, seed=seed)
    expect = nx.core_number(to_nx(g))
    got = oracle.exact_core(g, 1)
    assert all(got[v] == expect[v] for v in range(g.n))


@pytest.mark.parametrize("seed", range(12))
def test_exact_core_bruteforce(seed):
    n = 7 + seed % 4
    g = gg.random_small(n, 0.35, seed)
    adj = brute.adjacency(g)
    for h in (2, 3):
        expect = brute.core_by_subsets(adj, n, lambda u, X: brute.f_exact(adj, u, h, X))
        assert list(oracle.exact_core(g, h)) == expect


def test_exact_closed_forms():
    for h in (1, 2, 3, 4):
        for n in (1, 2, 3, 5, 8):
            assert list(oracle.exact_core(gg.path(n), h)) == [min(h, n - 1)] * n
            assert list(oracle.exact_core(gg.clique(n), h)) == [n - 1] * n
        for n in (3, 4, 7, 10):
            assert list(oracle.exact_core(gg.cycle(n), h)) == [min(2 * h, n - 1)] * n
        for s in (1, 2, 5, 9):
            expect = (1 if h == 1 else s)
            assert list(oracle.exact_core(gg.star(s), h)) == [expect] * (s + 1)
    # disjoint union: per component
    g = gg.disjoint_union(gg.path(4), gg.clique(5), gg.cycle(6), gg.empty(2))
    assert list(oracle.exact_core(g, 2)) == [2] * 4 + [4] * 5 + [4] * 6 + [0, 0]
    # h >= n-1: component size minus one
    g = gg.disjoint_union(gg.erdos_renyi(9, 12, seed=3), gg.path(3))
    comps = list(nx.connected_components(to_nx(g)))
    c = oracle.exact_core(g, g.n)
    for comp in comps:
        for v in comp:
            assert c[v] == len(comp) - 1


def test_not_kcore_of_power_graph():
    # (k,2)-cores are measured inside the induced subgraph, so they are not the
    # k-cores of G^2.  On this 7-vertex graph every (k,2)-core number is 4.
    g = gg.from_edges(7, [(0, 2), (0, 6), (1, 3), (1, 5), (2, 5), (3, 4), (3, 5), (3, 6), (4, 5)])
    assert list(oracle.exact_core(g, 2)) == [4] * 7
    G2 = nx.power(to_nx(g), 2)
    assert list(nx.core_number(G2)[v] for v in range(7)) == [4, 5, 5, 5, 5, 5, 5]


@pytest.mark.parametrize("seed", range(3))
def test_two_exact_oracles_agree(seed):
    g = gg.barabasi_albert(120, 2, seed=seed)
    for h in (2, 3):
        assert np.array_equal(oracle.exact_core(g, h), oracle.exact_core_sweep(g, h))


def test_tie_break_does_not_matter():
    g = gg.erdos_renyi(150, 400, seed=9)
    r = oracle.ranks(g.n, 7)
    for h in (2, 3):
        base = oracle.exact_core(g, h)
        sbase = oracle.sampled_core(g, h, r, 5)
        for ts in (11, 12, 13):
            assert np.array_equal(oracle.exact_core(g, h, tie_seed=ts), base)
            assert np.array_equal(oracle.sampled_core(g, h, r, 5, tie_seed=ts), sbase)


def test_cores_nested_and_valid():
    # Every v with core >= K has at least K vertices within distance h inside
    # F_K = {core >= K}; F_K are nested by construction.
    g = gg.chung_lu(300, 1200, 2.2, seed=5)
    for h in (2, 3):
        c = oracle.exact_core(g, h)
        for K in np.unique(c):
            F = (c >= K).astype(np.uint8)
            d = oracle.hdeg(g, h, F)
            assert d[F == 1].min() >= K
            # maximality: peeling G[F_K] cannot keep any vertex of core < K
        # the core number is attained: v's own level set has v with deg >= c(v)


# ---- Core (sampled) -------------------------------------------------------------

@pytest.mark.parametrize("seed", range(12))
def test_sampled_core_bruteforce(seed):
    n = 7 + seed % 4
    g = gg.random_small(n, 0.45, seed + 100)
    adj = brute.adjacency(g)
    r = oracle.ranks(n, seed)
    for h in (2, 3):
        for M in (1, 2, 3):
            expect = brute.core_by_subsets(adj, n, lambda u, X: brute.f_est(adj, u, h, X, r, M))
            assert list(oracle.sampled_core(g, h, r, M)) == expect, (h, M)


def test_sampled_equals_exact_when_M_ge_n():
    for seed in range(4):
        g = gg.erdos_renyi(200, 700, seed=seed)
        r = oracle.ranks(g.n, seed)
        for h in (2, 3):
            assert np.array_equal(oracle.sampled_core(g, h, r, g.n), oracle.exact_core(g, h))


def test_min_core_M_agrees():
    # If |N(v;h,X)| <= M the estimate is exact, else both values are >= M, so
    # min(c', M) = min(c, M) for every seed (second claim of Prop. yield).
    g = gg.barabasi_albert(250, 3, seed=2)
    for h in (2, 3):
        c = oracle.exact_core(g, h)
        for M in (5, 20, 60):
            for seed in range(3):
                cp = oracle.sampled_core(g, h, oracle.ranks(g.n, seed), M)
                assert np.array_equal(np.minimum(cp, M), np.minimum(c, M))


def test_sampled_estimate_is_approx():
    # With the paper's M the estimate of each h-degree is within eps.
    g = gg.barabasi_albert(3000, 3, seed=8)
    eps = 0.5
    M = oracle.M_int(g.n, eps)
    d = oracle.hdeg(g, 3)
    est = oracle.estimate_all(g, 3, oracle.ranks(g.n, 1), M)
    assert (d > M).sum() > 100  # sampling is exercised
    assert np.all(np.abs(est - d) <= eps * d + 1e-9)


def test_estimate_guarantee_over_200_seeds():
    # Prop. approx with the union bound behind C = log(2n/delta) (Eq. buffer):
    # with the paper's M, the probability over the ranks that any vertex's
    # estimate misses deg_h by more than eps is at most delta.
    g = gg.barabasi_albert(3000, 3, seed=8)
    eps, delta = 0.5, 0.05
    M = oracle.M_int(g.n, eps, delta)
    d = oracle.hdeg(g, 3).astype(np.float64)
    assert (d > M).sum() > 1000  # most estimates are sampled
    bad = 0
    worst = 0.0
    for seed in range(200):
        est = oracle.estimate_all(g, 3, oracle.ranks(g.n, seed), M).astype(np.float64)
        rel = np.max(np.abs(est - d) / np.maximum(d, 1.0))
        worst = max(worst, rel)
        bad += rel > eps
    assert bad <= delta * 200, (bad, worst)


@pytest.mark.parametrize("seed", range(6))
def test_sampled_lists_match_compute_recursion(seed):
    # Closed form of B[v,i], k[v,i] (Sec. 3) equals the Compute recursion of
    # Prop. dyn / Alg. 2 run from level 0, also on a reduced vertex set.
    g = gg.erdos_renyi(40, 90, seed=seed) if seed % 2 else gg.barabasi_albert(40, 2, seed=seed)
    adj = brute.adjacency(g)
    r = oracle.ranks(g.n, seed + 5)
    rng = np.random.default_rng(seed)
    alive = (rng.random(g.n) < 0.85).astype(np.uint8)
    X = {v for v in range(g.n) if alive[v]}
    for M in (2, 4, 8):
        kd, Bd = brute.compute_lists_dp(adj, g.n, 4, r, M, X)
        for i in (1, 2, 3, 4):
            k, s, off, mem = oracle.sampled_lists(g, i, r, M, alive)
            for v in range(g.n):
                if not alive[v]:
                    assert k[v] == -1 and s[v] == 0
                    continue
                assert k[v] == kd[i][v]
                assert set(mem[off[v]:off[v + 1]].tolist()) == Bd[i][v]


def test_estimate_from_lists_is_alg1():
    # Alg. 1 applied to the closed-form lists equals Delta of the ball (the
    # remark after Def. est).
    g = gg.barabasi_albert(300, 3, seed=4)
    r = oracle.ranks(g.n, 3)
    for h in (2, 3):
        for M in (3, 10, 40):
            k, s, off, mem = oracle.sampled_lists(g, h, r, M)
            est = oracle.estimate_all(g, h, r, M)
            for v in range(g.n):
                members = mem[off[v]:off[v + 1]]
                d = (len(members) - (1 if v in set(members.tolist()) else 0)) * 2 ** int(k[v])
                if k[v] > 0:
                    d = max(d, M * 2 ** (int(k[v]) - 1))
                assert d == est[v]


# ---- densest core level ----------------------------------------------------------

def test_dense_exact_counts_h_pairs():
    g = gg.barabasi_albert(60, 2, seed=1)
    adj = brute.adjacency(g)
    for h in (2, 3):
        c = oracle.exact_core(g, h)
        res = oracle.dense(g, c, h, "exact")
        best = None
        for K, size, R in res["cands"]:
            F = {v for v in range(g.n) if c[v] >= K}
            assert size == len(F)
            assert R == 2 * brute.h_pairs(adj, h, F)
            if best is None or R * best[1] >= best[2] * size:
                best = (K, size, R)
        assert (res["k"], res["size"], res["R"]) == best
        assert [k for k, _, _ in res["cands"]] == sorted(set(c.tolist()))


def test_dense_sampled_equals_exact_when_M_ge_n():
    g = gg.erdos_renyi(120, 500, seed=2)
    c = oracle.exact_core(g, 2)
    a = oracle.dense(g, c, 2, "exact")
    b = oracle.dense(g, c, 2, "sampled", oracle.ranks(g.n, 5, 1), g.n)
    assert (a["k"], a["size"], a["R"]) == (b["k"], b["size"], b["R"])


def test_dense_prune_keeps_top_levels():
    # end of Sec. 6: the pruning variant drops exactly the levels K below
    # gamma k' (gamma = (1-eps)/(1+eps), k' = max core) and keeps every other
    # candidate unchanged (each candidate's sum is measured inside F_K alone)
    for eps in (0.25, 0.5):
        for seed, h in ((3, 2), (4, 3), (5, 2)):
            g = gg.disjoint_union(gg.clique(25), gg.erdos_renyi(150, 300, seed=seed),
                                  gg.barabasi_albert(80, 3, seed=seed))
            c = oracle.exact_core(g, h)
            kmax = int(c.max())
            full = oracle.dense(g, c, h, "exact")
            pr = oracle.dense(g, c, h, "exact", prune=True, eps=eps)
            keep = [t for t in full["cands"] if t[0] * (1 + eps) >= (1 - eps) * kmax]
            assert pr["cands"] == keep
            assert len(keep) < len(full["cands"])  # pruning removes levels here
            best = max(keep, key=lambda t: (Fraction(t[2], t[1]), t[0]))
            assert (pr["k"], pr["size"], pr["R"]) == best


# ---- early stop (Sec. 5 heuristic) -------------------------------------------------

def test_early_stop_worked_example():
    g = gg.from_edges(5, [(0, 1), (1, 2), (1, 3), (1, 4), (2, 3), (2, 4), (3, 4)])
    r = np.array([3, 2, 5, 5, 5], np.uint8)
    for row in golden_rows("early_stop_example.txt"):
        mode, es, want = row[0], bool(int(row[1])), [int(x) for x in row[2:]]
        if mode == "sampled":
            got = oracle.sampled_core(g, 1, r, 1, early_stop=es)
        else:
            got = oracle.exact_core(g, 1, early_stop=es)
        assert list(got) == want, (mode, es)


def early_stop_closed_form(core):
    """Derived from the peel: vertices leave in non-decreasing core order, the
    test c + 1 >= |X| is weakest at the end of each level's deletions, where
    |X| = #{core > c}; so the first level c with c + 1 >= #{core > c} stops the
    peel and every vertex gets min(core, c)."""
    core = np.asarray(core)
    for c in np.unique(core):
        if c + 1 >= int((core > c).sum()):
            return np.minimum(core, c)
    return core


@pytest.mark.parametrize("seed", range(4))
def test_early_stop_closed_form_and_exact_safety(seed):
    g = gg.chung_lu(60, 200, 2.2, seed=seed) if seed % 2 else gg.erdos_renyi(40, 120, seed=seed)
    r = oracle.ranks(g.n, seed)
    changed = 0
    for h in (2, 3):
        # exact: deg_h <= |X| - 1, so stopping never changes a core number
        c = oracle.exact_core(g, h)
        assert np.array_equal(oracle.exact_core(g, h, early_stop=True), c)
        assert np.array_equal(early_stop_closed_form(c), c)
        for M in (1, 2, 3, 5):
            cp = oracle.sampled_core(g, h, r, M)
            es = oracle.sampled_core(g, h, r, M, early_stop=True)
            assert np.array_equal(es, early_stop_closed_form(cp)), (h, M)
            changed += int((es != cp).any())
            # tie-breaks still do not matter
            assert np.array_equal(oracle.sampled_core(g, h, r, M, tie_seed=77, early_stop=True), es)
    if seed in (2, 3):
        assert changed > 0  # the heuristic does change sampled outputs here


# ---- full EstDense (Alg. 7 over every suffix of the deletion order) --------------------

def _round_starts(rnd):
    return sorted(set(rnd.tolist()))


@pytest.mark.parametrize("mode", ["exact", "sampled"])
def test_bulk_order_is_the_bulk_peel(mode):
    # rounds of the bulk peel, checked from their plain definition with the
    # (separately pinned) h-degree and estimate: at the start of round j with
    # alive set X_j, c_j = max(c_{j-1}, min f), R_j = {f <= c_j}, listed by
    # (f, level, id); the order's core numbers equal the sequential peel's.
    g = gg.chung_lu(250, 1000, 2.2, seed=7)
    h, M = 2, 6
    r = oracle.ranks(g.n, 3)
    order, core, rnd = oracle.bulk_order(g, h, mode, r, M)
    assert sorted(order.tolist()) == list(range(g.n))
    want = oracle.exact_core(g, h) if mode == "exact" else oracle.sampled_core(g, h, r, M)
    assert np.array_equal(core, want)
    assert np.all(np.diff(rnd[order]) >= 0)
    c = -1
    for j in _round_starts(rnd):
        X = (rnd >= j).astype(np.uint8)
        f = oracle.hdeg(g, h, X) if mode == "exact" else oracle.estimate_all(g, h, r, M, X)
        c = max(c, int(f[X == 1].min()))
        R = [v for v in order if rnd[v] == j]
        assert set(R) == {v for v in range(g.n) if X[v] and f[v] <= c}
        if mode == "exact":
            lev = {v: 0 for v in R}
        else:
            k, _, _, _ = oracle.sampled_lists(g, h, r, M, X)
            lev = {v: int(k[v]) for v in R}
        assert R == sorted(R, key=lambda v: (int(f[v]), lev[v], v))
        assert all(core[v] == c for v in R)
    # every core level set is a suffix
    pos = np.empty(g.n, np.int64)
    pos[order] = np.arange(g.n)
    for K in np.unique(core):
        F = np.nonzero(core >= K)[0]
        assert pos[F].min() == g.n - F.size


def test_dense_suffix_exact_counts_h_pairs():
    # R of every suffix = 2 |E_h(S)| by brute-force pair counting (Sec. 6 identity)
    g = gg.barabasi_albert(40, 2, seed=1)
    adj = brute.adjacency(g)
    for h in (2, 3):
        order, _, _ = oracle.bulk_order(g, h)
        res = oracle.dense_suffix(g, order, h)
        for i in range(g.n):
            S = set(order[i:].tolist())
            assert res["R"][i] == 2 * brute.h_pairs(adj, h, S)
        best = max(range(g.n), key=lambda i: (Fraction(int(res["R"][i]), g.n - i), i))
        assert res["best"] == best and res["size"] == g.n - best


def test_dense_suffix_sampled_sums_the_estimate():
    # R of every suffix = sum of Def. est over it (estimate_all, pinned above);
    # M >= n reduces it to the exact count; suffixes include every core level,
    # so the best suffix is at least as dense as the best core level
    g = gg.chung_lu(150, 600, 2.2, seed=2)
    h = 2
    r0, r1 = oracle.ranks(g.n, 4, 0), oracle.ranks(g.n, 4, 1)
    order, core, _ = oracle.bulk_order(g, h, "sampled", r0, 5)
    res = oracle.dense_suffix(g, order, h, "sampled", r1, 7)
    for i in (0, 1, 17, 60, 149):
        S = np.zeros(g.n, np.uint8)
        S[order[i:]] = 1
        assert res["R"][i] == int(oracle.estimate_all(g, h, r1, 7, S)[S == 1].sum())
    ex = oracle.dense_suffix(g, order, h, "exact")
    big = oracle.dense_suffix(g, order, h, "sampled", r1, g.n)
    assert np.array_equal(ex["R"], big["R"])
    lvl = oracle.dense(g, core, h, "sampled", r1, 7)
    assert Fraction(res["best_R"], res["size"]) >= Fraction(lvl["R"], lvl["size"])
