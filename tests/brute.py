"""Independent brute-force references used to pin the oracle (tiny inputs).

Written directly from the definitions of Tatti, arXiv 2112.06154, Sec. 2-4,
in plain Python and sharing no code with the oracle or the GPU library.
"""
from __future__ import annotations

import itertools
from collections import deque


def adjacency(g):
    rp = g.row_ptr
    return [list(int(x) for x in g.col[rp[v]:rp[v + 1]]) for v in range(g.n)]


def ball(adj, v, h, X):
    """N(v; h, X): vertices reachable from v by a path of at most h edges
    that stays inside the vertex set X (Sec. 2)."""
    dist = {v: 0}
    q = deque([v])
    while q:
        u = q.popleft()
        if dist[u] == h:
            continue
        for w in adj[u]:
            if w in X and w not in dist:
                dist[w] = dist[u] + 1
                q.append(w)
    return set(dist)


def delta_def(x, M):
    """Def. est, written out with explicit sets."""
    k = 0
    while sum(1 for t in x if t >= k) > M:
        k += 1
    T = sum(1 for j, t in enumerate(x) if j >= 1 and t >= k)
    est = T * 2 ** k
    if k > 0:
        est = max(est, M * 2 ** (k - 1))
    return est


def f_exact(adj, v, h, X):
    return len(ball(adj, v, h, X)) - 1


def f_est(adj, v, h, X, r, M):
    b = ball(adj, v, h, X)
    return delta_def([int(r[v])] + [int(r[u]) for u in b if u != v], M)


def core_by_subsets(adj, n, fn):
    """c(v) = max{k : exists X containing v with fn(u, X) >= k for all u in X}
    by enumerating every non-empty vertex subset (Sec. 2 definition)."""
    best = [0] * n
    for mask in range(1, 1 << n):
        X = frozenset(i for i in range(n) if mask >> i & 1)
        mu = min(fn(u, X) for u in X)
        for u in X:
            if mu > best[u]:
                best[u] = mu
    return best


def compute_lists_dp(adj, n, h, r, M, X):
    """The Compute recursion of Sec. 3 (Prop. dyn / Alg. 2) from B[.,0] = {v},
    k[.,0] = 0: T = {v} united with B[w,i-1] over alive neighbours w, sorted by
    rank descending; k = max(max_w k[w,i-1], r[t_{M+1}] + 1 if |T| > M);
    B = {u in T : r[u] >= k}.  Returns per level dicts k[i][v], B[i][v]."""
    r = [int(t) for t in r]
    k = [{v: 0 for v in X}]
    B = [{v: {v} for v in X}]
    for i in range(1, h + 1):
        ki, Bi = {}, {}
        for v in X:
            T = {v}
            kk = 0
            for w in adj[v]:
                if w in X:
                    T |= B[i - 1][w]
                    kk = max(kk, k[i - 1][w])
            ts = sorted(T, key=lambda u: -r[u])
            if len(ts) > M:
                kk = max(kk, r[ts[M]] + 1)
            ki[v] = kk
            Bi[v] = {u for u in T if r[u] >= kk}
        k.append(ki)
        B.append(Bi)
    return k, B


def h_pairs(adj, h, X):
    """|E_h(X)|: unordered pairs of distinct nodes of X joined by an h-path in X."""
    cnt = 0
    for v in X:
        cnt += len(ball(adj, v, h, X)) - 1
    return cnt // 2


def all_subsets(n):
    for size in range(1, n + 1):
        for c in itertools.combinations(range(n), size):
            yield frozenset(c)
