"""The refined bookkeeping of Sec. 5 (Alg. 5 and Alg. 6) -- TEST INFRASTRUCTURE ONLY.

Plain Python for small graphs: only the tests may use it.  It keeps, for every
alive vertex v and level i = 1..h,

- B[v,i] as a map u -> z, where z counts the alive neighbours w with u in
  B[w,i-1], plus one for v itself (the entry v starts with in Compute);
- k[v,i];
- m[v,i], the alive neighbours w with k[w,i-1] = k[v,i];
- D[v,i] (kept only while m[v,i] = 0), the members of rank k[v,i] - 1 of the
  neighbours' lists, with the same kind of counts.

Deleting a vertex u (Update) runs level by level.  At level i every vertex v
whose level i-1 list lost members Y (all of it when v = u) or whose level
k[v,i-1] dropped lowers the counts of Y in B[w,i] and D[w,i] of its alive
neighbours w, removing members whose count reaches zero, and lowers m[w,i] if
v left w's level; a touched w is re-merged from scratch (Compute) only when
|B[w,i]| + |D[w,i]| <= M and m[w,i] = 0, the only case in which its level can
drop and new members enter.  Otherwise the deletions alone keep B[w,i]
current.  The paper shows the result equals the naive Update (Alg. 3), i.e.
the closed form of Sec. 3; the tests check exactly that after every deletion,
and count how many re-merges the refined criterion saves against re-merging
every touched list.
"""
from __future__ import annotations


class RefinedCore:
    """Alg. 4 (Core) on top of the refined Compute/Update of Sec. 5."""

    def __init__(self, g, h: int, r, M: int):
        self.n = int(g.n)
        self.h = int(h)
        self.M = int(M)
        self.r = [int(x) for x in r[: self.n]]
        rp, col = g.row_ptr, g.col
        self.adj = [[int(w) for w in col[rp[v]:rp[v + 1]]] for v in range(self.n)]
        self.alive = [True] * self.n
        n, H = self.n, self.h
        self.B = [[None] * (H + 1) for _ in range(n)]
        self.k = [[0] * (H + 1) for _ in range(n)]
        self.m = [[0] * (H + 1) for _ in range(n)]
        self.D = [[None] * (H + 1) for _ in range(n)]
        for v in range(n):
            self.B[v][0] = {v: 1}  # B[v,0] = {v}, k[v,0] = 0
            self.D[v][0] = {}
        self.computes = 0       # re-merges done by the refined criterion
        self.naive_computes = 0  # re-merges the naive Update would do (every touched list)
        self.count_updates = 0  # counter decrements of Delete
        for i in range(1, H + 1):
            for v in range(n):
                self.compute(v, i)
        self.computes = 0

    # ---- Alg. 5: Compute(v, i) from scratch ------------------------------------------------
    def compute(self, v: int, i: int) -> None:
        self.computes += 1
        r, M = self.r, self.M
        nbrs = [w for w in self.adj[v] if self.alive[w]]
        k = max((self.k[w][i - 1] for w in nbrs), default=0)
        T = {v: 1}
        for w in nbrs:
            for u in self.B[w][i - 1]:
                if r[u] >= k:
                    T[u] = T.get(u, 0) + 1
            if len(T) > M:
                # the (M+1)-th highest rank sets the level; lower ranks leave
                kth = sorted((r[u] for u in T), reverse=True)[M]
                k = max(k, kth + 1)
                T = {u: z for u, z in T.items() if r[u] >= k}
        # v entered T before the level was known: it stays only if its rank
        # reaches the level (B[v,i] = {u in T : r[u] >= k[v,i]}, as in Alg. 2);
        # every merged entry already does
        self.B[v][i] = {u: z for u, z in T.items() if r[u] >= k}
        self.k[v][i] = k
        self.m[v][i] = sum(1 for w in nbrs if self.k[w][i - 1] == k)
        D = {}
        if self.m[v][i] == 0:
            for w in nbrs:
                for u in self.B[w][i - 1]:
                    if r[u] == k - 1:
                        D[u] = D.get(u, 0) + 1
        self.D[v][i] = D

    # ---- Alg. 1: the estimate from B[v,h] ----------------------------------------------------
    def estimate(self, v: int) -> int:
        k = self.k[v][self.h]
        t = len(self.B[v][self.h]) - (1 if self.r[v] >= k else 0)
        d = t << k
        if k > 0:
            d = max(d, self.M << (k - 1))
        return d

    # ---- Alg. 6: Update(u), deleting u ----------------------------------------------------------
    def delete(self, u: int) -> None:
        self.alive[u] = False
        # per vertex of the level below: (members removed from its list, its old
        # level if that level changed or the vertex left, or None)
        changes = {u: (set(self.B[u][0]), self.k[u][0])}
        for i in range(1, self.h + 1):
            touched = {}
            for v, (Y, oldk) in changes.items():
                for w in self.adj[v]:
                    if not self.alive[w]:
                        continue
                    Z = touched.setdefault(w, set())
                    Bw, Dw = self.B[w][i], self.D[w][i]
                    for y in Y:
                        if y in Bw:
                            self.count_updates += 1
                            Bw[y] -= 1
                            if Bw[y] == 0:
                                del Bw[y]
                                Z.add(y)
                        if y in Dw:
                            Dw[y] -= 1
                            if Dw[y] == 0:
                                del Dw[y]
                    if oldk is not None and oldk == self.k[w][i]:
                        self.m[w][i] -= 1
            nxt = {}
            for w, Z in touched.items():
                self.naive_computes += 1
                kold = self.k[w][i]
                if len(self.B[w][i]) + len(self.D[w][i]) <= self.M and self.m[w][i] == 0:
                    before = set(self.B[w][i])
                    self.compute(w, i)
                    Z |= before - set(self.B[w][i])
                if Z or self.k[w][i] != kold:
                    nxt[w] = (Z, kold if self.k[w][i] != kold else None)
            # u's own level-i list leaves the neighbourhoods of level i + 1
            nxt[u] = (set(self.B[u][i]), self.k[u][i])
            changes = nxt

    # ---- Alg. 4 ------------------------------------------------------------------------------------
    def core(self, after_delete=None):
        """Delete an argmin of (d, k[v,h], id) one vertex at a time, recording
        the running maximum; after_delete(self) is called after every deletion."""
        n = self.n
        core = [0] * n
        c = 0
        for _ in range(n):
            best = None
            for v in range(n):
                if self.alive[v]:
                    key = (self.estimate(v), self.k[v][self.h], v)
                    if best is None or key < best:
                        best = key
            d, _, v = best
            c = max(c, d)
            core[v] = c
            self.delete(v)
            if after_delete is not None:
                after_delete(self)
        return core
