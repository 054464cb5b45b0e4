/*
 * khoracle.c -- CPU oracle for distance-generalized (k,h)-core decomposition.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it.  It shares
 * no code, header, table or helper with the GPU library.
 *
 * Everything follows Tatti, "Fast computation of distance-generalized cores
 * using sampling" (arXiv 2112.06154):
 *
 *   h-neighbourhood N(v;h,X), deg_h(v;X) = |N(v;h,X)| - 1   (Sec. 2)
 *   (k,h)-core, core number c(v), ExactCore min-peeling      (Sec. 2)
 *   buffer size M, Eq. (buffer); C = log(2n/delta)          (Sec. 3)
 *   ranks r[v] ~ geometric(1/2), P(r >= k) = 2^-k            (Sec. 3, Alg. 4)
 *   B[v,i], k[v,i] (the sampled i-neighbourhood)             (Sec. 3)
 *   estimator Delta(X;M), Def. est; equal to Alg. 1 output   (Sec. 4)
 *   Core = min-peel on the estimate, running maximum         (Alg. 4)
 *   h-density |E_h(X)|/|X|, identity 2|E_h(X)| = sum deg_h   (Sec. 6)
 *   core-level densest-subgraph candidates, pruning by gamma (Sec. 6, Alg. 7)
 *
 * Readings where the paper leaves a choice (all listed with reasons in the
 * design notes of the repository):
 *   - log is the natural logarithm, and M is used as the integer floor(M);
 *   - ranks come from a counter-based SplitMix64 stream (see orc_rank);
 *   - N(v;h,X) is measured inside the current induced subgraph G[X];
 *   - an h-path has at most h edges;
 *   - the sampled core is computed from the closed form of the estimate
 *     (Def. est applied to the ranks of N(v;h,X) with r[v] first), which the
 *     paper shows equals Algorithm 1 on the maintained lists (Prop. dyn and
 *     the remark after Def. est).  The list machinery itself is NOT here.
 *
 * Parity of every function here is pinned by CPU tests against values the
 * paper prints (Table 1's M column), closed forms, a graph library, brute
 * force on tiny graphs and the paper's propositions.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_API __attribute__((visibility("default")))

/* ------------------------------------------------------------------------ */
/* Random ranks (Sec. 3: r[v] = geo(1/2), ties allowed).                     */
/* SplitMix64 mixing function, Steele, Lea and Flood (OOPSLA 2014):          */
/*   z = x + 0x9E3779B97F4A7C15;                                             */
/*   z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9;                               */
/*   z = (z ^ (z >> 27)) * 0x94D049BB133111EB;                               */
/*   return z ^ (z >> 31).                                                   */
/* ------------------------------------------------------------------------ */
ORC_API uint64_t orc_splitmix64(uint64_t x)
{
    uint64_t z = x + 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Coin-flip word j of vertex v in stream s:
 *   w_j(v) = sm(sm(sm(seed) ^ v) ^ (s * 2^32 + j)).
 * The rank is the number of leading successes of that coin sequence, where
 * bit b of w_j is flip 64 j + b and a zero bit is a success.  Hence
 * P(r >= k) = 2^-k.  Capped at 255. */
ORC_API int orc_rank(uint64_t seed, uint32_t stream, int64_t v)
{
    uint64_t base = orc_splitmix64(orc_splitmix64(seed) ^ (uint64_t)v);
    int r = 0;
    for (uint32_t j = 0; j < 4; j++) {
        uint64_t w = orc_splitmix64(base ^ (((uint64_t)stream << 32) | j));
        if (w != 0) {
            int t = 0;
            while (((w >> t) & 1ULL) == 0) t++;
            r += t;
            return r > 255 ? 255 : r;
        }
        r += 64;
    }
    return 255;
}

ORC_API void orc_ranks(int64_t n, uint64_t seed, uint32_t stream, uint8_t *r_out)
{
    for (int64_t v = 0; v < n; v++) r_out[v] = (uint8_t)orc_rank(seed, stream, v);
}

/* ------------------------------------------------------------------------ */
/* Eq. (buffer): C = log(2n/delta), M = 1 + 4(2+eps)/eps^2 (C + log 8).      */
/* For the dense-subgraph pass (Alg. 7) C = log(n^2/delta).                  */
/* ------------------------------------------------------------------------ */
ORC_API double orc_M_real(int64_t n, double eps, double delta, int dense)
{
    double C = dense ? log((double)n * (double)n / delta) : log(2.0 * (double)n / delta);
    return 1.0 + 4.0 * (2.0 + eps) / (eps * eps) * (C + log(8.0));
}

ORC_API int64_t orc_M(int64_t n, double eps, double delta, int dense)
{
    return (int64_t)floor(orc_M_real(n, eps, delta, dense));
}

/* ------------------------------------------------------------------------ */
/* Def. est: Delta(x_1..x_d; M).                                             */
/*   S_i = #{j : x_j >= i},  T_i = #{j >= 2 : x_j >= i},                     */
/*   k   = smallest integer k >= 0 with S_k <= M,                            */
/*   Delta = T_k 2^k, and if k > 0, max(T_k 2^k, M 2^(k-1)).                 */
/* ------------------------------------------------------------------------ */
ORC_API int64_t orc_delta(const int32_t *x, int64_t d, int64_t M)
{
    int64_t k = 0;
    for (;;) {
        int64_t S = 0;
        for (int64_t j = 0; j < d; j++)
            if (x[j] >= k) S++;
        if (S <= M) break;
        k++;
    }
    int64_t T = 0;
    for (int64_t j = 1; j < d; j++)
        if (x[j] >= k) T++;
    int64_t est = T << k;
    if (k > 0) {
        int64_t floor_term = M << (k - 1);
        if (floor_term > est) est = floor_term;
    }
    return est;
}

/* ------------------------------------------------------------------------ */
/* Breadth-first search inside G[X], X = {u : alive[u] != 0}, to depth h.    */
/* Writes the vertices of N(src;h,X) into ball[] (src first) and returns    */
/* their count.  mark[] must be all-zero on entry and is all-zero on exit.  */
/* When te != NULL, adds the number of arcs inspected from vertices at      */
/* distance <= h-1 whose other end is alive (the edges-traversed count).    */
/* ------------------------------------------------------------------------ */
static int64_t ball_of(int64_t src, int h, const int32_t *rp, const int32_t *col,
                       const uint8_t *alive, uint8_t *mark, int32_t *ball, int64_t *te)
{
    int64_t head = 0, tail = 0;
    ball[tail++] = (int32_t)src;
    mark[src] = 1;
    for (int depth = 0; depth < h; depth++) {
        int64_t level_end = tail;
        while (head < level_end) {
            int32_t u = ball[head++];
            for (int32_t p = rp[u]; p < rp[u + 1]; p++) {
                int32_t w = col[p];
                if (!alive[w]) continue;
                if (te) (*te)++;
                if (!mark[w]) {
                    mark[w] = 1;
                    ball[tail++] = w;
                }
            }
        }
        if (head == tail) break;
    }
    for (int64_t i = 0; i < tail; i++) mark[ball[i]] = 0;
    return tail;
}

typedef struct {
    int64_t n;
    const int32_t *rp, *col;
    uint8_t *mark;
    int32_t *ball;
    int32_t *xr; /* rank list scratch */
} orc_ws;

static int ws_init(orc_ws *ws, int64_t n, const int32_t *rp, const int32_t *col)
{
    ws->n = n;
    ws->rp = rp;
    ws->col = col;
    ws->mark = (uint8_t *)calloc((size_t)(n > 0 ? n : 1), 1);
    ws->ball = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    ws->xr = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    return ws->mark && ws->ball && ws->xr ? 0 : -1;
}

static void ws_free(orc_ws *ws)
{
    free(ws->mark);
    free(ws->ball);
    free(ws->xr);
}

/* The vertex function f(v; X) the peel works with:
 *   mode 0 (exact):   deg_h(v;X) = |N(v;h,X)| - 1                     (Sec. 2)
 *   mode 1 (sampled): Delta((r[v], r[u] : u in N(v;h,X) \ {v}); M)   (Def. est) */
static int64_t vertex_fn(orc_ws *ws, int64_t v, int h, const uint8_t *alive, int mode,
                         const uint8_t *r, int64_t M, int64_t *te)
{
    int64_t cnt = ball_of(v, h, ws->rp, ws->col, alive, ws->mark, ws->ball, te);
    if (mode == 0) return cnt - 1;
    for (int64_t i = 0; i < cnt; i++) ws->xr[i] = r[ws->ball[i]];
    return orc_delta(ws->xr, cnt, M);
}

/* deg_h(v;X) for every alive v (dead vertices get -1). Returns 0 on success. */
ORC_API int orc_hdeg_all(int64_t n, const int32_t *rp, const int32_t *col, const uint8_t *alive,
                         int h, int64_t *deg_out, int64_t *te_out)
{
    orc_ws ws;
    if (ws_init(&ws, n, rp, col)) return -1;
    int64_t te = 0;
    for (int64_t v = 0; v < n; v++)
        deg_out[v] = alive[v] ? vertex_fn(&ws, v, h, alive, 0, NULL, 0, &te) : -1;
    if (te_out) *te_out = te;
    ws_free(&ws);
    return 0;
}

/* deg_h for a list of sources only (for sampled checks on large graphs). */
ORC_API int orc_hdeg_list(int64_t n, const int32_t *rp, const int32_t *col, const uint8_t *alive,
                          int h, int64_t count, const int32_t *src, int64_t *deg_out, int64_t *te_out)
{
    orc_ws ws;
    if (ws_init(&ws, n, rp, col)) return -1;
    int64_t te = 0;
    for (int64_t i = 0; i < count; i++)
        deg_out[i] = alive[src[i]] ? vertex_fn(&ws, src[i], h, alive, 0, NULL, 0, &te) : -1;
    if (te_out) *te_out = te;
    ws_free(&ws);
    return 0;
}

/* Estimate Delta for every alive v (dead vertices get -1). */
ORC_API int orc_est_all(int64_t n, const int32_t *rp, const int32_t *col, const uint8_t *alive,
                        int h, const uint8_t *r, int64_t M, int64_t *est_out)
{
    orc_ws ws;
    if (ws_init(&ws, n, rp, col)) return -1;
    for (int64_t v = 0; v < n; v++)
        est_out[v] = alive[v] ? vertex_fn(&ws, v, h, alive, 1, r, M, NULL) : -1;
    ws_free(&ws);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Peeling (ExactCore, Sec. 2; Core, Alg. 4).                                */
/* Repeatedly delete an alive vertex u minimising f(u;X); the running        */
/* maximum c of the deleted values is u's core number.  Ties are broken by   */
/* the smallest id, or by a seeded random key when tie_seed != 0 (the        */
/* result does not depend on it; a test checks that).  After deleting u only */
/* the vertices of N(u;h,X) -- measured before the deletion -- can change,   */
/* so only those are recomputed.  order_out (nullable) receives the deletion */
/* order and fval_out (nullable) the value f(u;X) at deletion.               */
/* ------------------------------------------------------------------------ */
/* Early stop (Sec. 5, second heuristic; Sec. 8 states the test as "current  */
/* core value plus one equals the number of remaining nodes"): right after a */
/* deletion, if c + 1 >= |X| for the remaining set X, every remaining vertex */
/* receives c and the peel ends.  For deg_h this changes nothing (every      */
/* remaining vertex has deg_h <= |X| - 1 <= c and would leave next at c);    */
/* for the estimate it may, since Delta can exceed |X| - 1.                  */
static int peel(int64_t n, const int32_t *rp, const int32_t *col, const uint8_t *alive_in, int h,
                int mode, const uint8_t *r, int64_t M, uint64_t tie_seed, int early_stop, int64_t *core_out,
                int32_t *order_out, int64_t *fval_out, int64_t *te_out)
{
    orc_ws ws;
    if (ws_init(&ws, n, rp, col)) return -1;
    uint8_t *alive = (uint8_t *)malloc((size_t)(n > 0 ? n : 1));
    int64_t *f = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    uint64_t *tie = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(n > 0 ? n : 1));
    int32_t *aff = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!alive || !f || !tie || !aff) return -1;
    int64_t te = 0, remaining = 0;
    for (int64_t v = 0; v < n; v++) {
        alive[v] = alive_in ? alive_in[v] : 1;
        remaining += alive[v] ? 1 : 0;
        tie[v] = tie_seed ? orc_splitmix64(tie_seed ^ (uint64_t)v) : (uint64_t)v;
        core_out[v] = -1;
    }
    for (int64_t v = 0; v < n; v++)
        f[v] = alive[v] ? vertex_fn(&ws, v, h, alive, mode, r, M, &te) : 0;
    int64_t c = 0, step = 0;
    while (remaining > 0) {
        int64_t u = -1;
        for (int64_t v = 0; v < n; v++) {
            if (!alive[v]) continue;
            if (u < 0 || f[v] < f[u] || (f[v] == f[u] && tie[v] < tie[u])) u = v;
        }
        if (f[u] > c) c = f[u];
        core_out[u] = c;
        if (order_out) order_out[step] = (int32_t)u;
        if (fval_out) fval_out[step] = f[u];
        step++;
        int64_t na = ball_of(u, h, rp, col, alive, ws.mark, aff, NULL);
        alive[u] = 0;
        remaining--;
        if (early_stop && remaining > 0 && c + 1 >= remaining) {
            for (int64_t v = 0; v < n; v++) {
                if (!alive[v]) continue;
                core_out[v] = c;
                if (order_out) order_out[step] = (int32_t)v;
                if (fval_out) fval_out[step] = f[v];
                step++;
                alive[v] = 0;
            }
            remaining = 0;
            break;
        }
        for (int64_t i = 1; i < na; i++)
            f[aff[i]] = vertex_fn(&ws, aff[i], h, alive, mode, r, M, &te);
    }
    if (te_out) *te_out = te;
    free(alive);
    free(f);
    free(tie);
    free(aff);
    ws_free(&ws);
    return 0;
}

ORC_API int orc_exact_core(int64_t n, const int32_t *rp, const int32_t *col, int h, uint64_t tie_seed,
                           int early_stop, int64_t *core_out, int32_t *order_out, int64_t *te_out)
{
    return peel(n, rp, col, NULL, h, 0, NULL, 0, tie_seed, early_stop, core_out, order_out, NULL, te_out);
}

ORC_API int orc_sampled_core(int64_t n, const int32_t *rp, const int32_t *col, int h, const uint8_t *r,
                             int64_t M, uint64_t tie_seed, int early_stop, int64_t *core_out, int32_t *order_out)
{
    return peel(n, rp, col, NULL, h, 1, r, M, tie_seed, early_stop, core_out, order_out, NULL, NULL);
}

/* Second exact oracle (test-only cross-check): level sweep.  For k = 0,1,...
 * repeatedly delete every alive vertex with deg_h < k, recomputing all
 * degrees from scratch after each sweep; vertices deleted while sweeping
 * level k have core number k-1. */
ORC_API int orc_exact_core_sweep(int64_t n, const int32_t *rp, const int32_t *col, int h, int64_t *core_out)
{
    orc_ws ws;
    if (ws_init(&ws, n, rp, col)) return -1;
    uint8_t *alive = (uint8_t *)malloc((size_t)(n > 0 ? n : 1));
    uint8_t *kill = (uint8_t *)malloc((size_t)(n > 0 ? n : 1));
    int64_t remaining = n;
    for (int64_t v = 0; v < n; v++) alive[v] = 1;
    for (int64_t k = 0; remaining > 0; k++) {
        for (;;) {
            int64_t nk = 0;
            for (int64_t v = 0; v < n; v++) {
                kill[v] = 0;
                if (alive[v] && vertex_fn(&ws, v, h, alive, 0, NULL, 0, NULL) < k) {
                    kill[v] = 1;
                    nk++;
                }
            }
            if (nk == 0) break;
            for (int64_t v = 0; v < n; v++)
                if (kill[v]) {
                    alive[v] = 0;
                    core_out[v] = k - 1;
                    remaining--;
                }
        }
    }
    free(alive);
    free(kill);
    ws_free(&ws);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Closed form of the sampled lists (Sec. 3 definition of B and k, with     */
/* Prop. dyn showing the Compute recursion reaches it): for alive v,         */
/*   k[v,i] = smallest k >= 0 with |{u in N(v;i,X) : r[u] >= k}| <= M,       */
/*   B[v,i] = {u in N(v;i,X) : r[u] >= k[v,i]}.                              */
/* Output: k_out[v], size_out[v] and the members of B[v,i] concatenated in   */
/* vertex order (ids ascending within a vertex) into members_out, which must */
/* hold sum of size_out entries (call with members_out == NULL to size it).  */
/* Dead vertices get k = -1, size 0.  Returns the total member count.        */
/* ------------------------------------------------------------------------ */
static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

ORC_API int64_t orc_sampled_lists(int64_t n, const int32_t *rp, const int32_t *col, const uint8_t *alive,
                                  int i, const uint8_t *r, int64_t M, int32_t *k_out, int32_t *size_out,
                                  int32_t *members_out)
{
    orc_ws ws;
    if (ws_init(&ws, n, rp, col)) return -1;
    int64_t total = 0;
    for (int64_t v = 0; v < n; v++) {
        if (!alive[v]) {
            k_out[v] = -1;
            size_out[v] = 0;
            continue;
        }
        int64_t cnt = ball_of(v, i, rp, col, alive, ws.mark, ws.ball, NULL);
        int64_t k = 0;
        for (;;) {
            int64_t S = 0;
            for (int64_t j = 0; j < cnt; j++)
                if (r[ws.ball[j]] >= k) S++;
            if (S <= M) break;
            k++;
        }
        int64_t s = 0;
        for (int64_t j = 0; j < cnt; j++)
            if (r[ws.ball[j]] >= k) ws.xr[s++] = ws.ball[j];
        qsort(ws.xr, (size_t)s, sizeof(int32_t), cmp_i32);
        if (members_out) memcpy(members_out + total, ws.xr, sizeof(int32_t) * (size_t)s);
        k_out[v] = (int32_t)k;
        size_out[v] = (int32_t)s;
        total += s;
    }
    ws_free(&ws);
    return total;
}

/* ------------------------------------------------------------------------ */
/* Densest subgraph among the core levels (Sec. 6).                          */
/* For every distinct core value K (ascending) let F_K = {v : core[v] >= K}  */
/* and R_K = sum over v in F_K of f(v;F_K), with f = deg_h (mode 0) or the   */
/* estimate with the given ranks and M (mode 1).  By the identity            */
/* 2|E_h(X)| = sum_v deg_h(v;X), R_K/(2|F_K|) is the (estimated) h-density.  */
/* The best K maximises R_K/|F_K| (ties: the larger K).  With prune != 0     */
/* only K with K(1+eps) >= (1-eps) max(core) are candidates (the pruning     */
/* variant at the end of Sec. 6).  Returns 0, and the winner through         */
/* best_k/best_size/best_R; all candidates through cand_* when non-NULL      */
/* (in ascending K order, count in *ncand).                                  */
/* ------------------------------------------------------------------------ */
ORC_API int orc_dense(int64_t n, const int32_t *rp, const int32_t *col, const int64_t *core, int h, int mode,
                      const uint8_t *r, int64_t M, int prune, double eps, int64_t *best_k, int64_t *best_size,
                      int64_t *best_R, int64_t *ncand, int64_t *cand_k, int64_t *cand_size, int64_t *cand_R)
{
    orc_ws ws;
    if (ws_init(&ws, n, rp, col)) return -1;
    uint8_t *alive = (uint8_t *)malloc((size_t)(n > 0 ? n : 1));
    int64_t maxc = -1;
    for (int64_t v = 0; v < n; v++)
        if (core[v] > maxc) maxc = core[v];
    *best_k = -1;
    *best_size = 0;
    *best_R = 0;
    int64_t nc = 0;
    int64_t K = -1;
    for (;;) {
        /* next distinct core value above K */
        int64_t next = -1;
        for (int64_t v = 0; v < n; v++)
            if (core[v] > K && (next < 0 || core[v] < next)) next = core[v];
        if (next < 0) break;
        K = next;
        if (prune && (double)K * (1.0 + eps) < (1.0 - eps) * (double)maxc) continue;
        int64_t size = 0, R = 0;
        for (int64_t v = 0; v < n; v++) {
            alive[v] = core[v] >= K;
            size += alive[v];
        }
        for (int64_t v = 0; v < n; v++)
            if (alive[v]) R += vertex_fn(&ws, v, h, alive, mode, r, M, NULL);
        if (cand_k) {
            cand_k[nc] = K;
            cand_size[nc] = size;
            cand_R[nc] = R;
        }
        nc++;
        /* R/size >= best_R/best_size, exact in 128-bit integers */
        if (*best_k < 0 ||
            (__int128)R * (__int128)(*best_size) >= (__int128)(*best_R) * (__int128)size) {
            *best_k = K;
            *best_size = size;
            *best_R = R;
        }
    }
    if (ncand) *ncand = nc;
    free(alive);
    ws_free(&ws);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Full EstDense (Alg. 7): every suffix of a deletion order as a candidate.  */
/*                                                                           */
/* The order is the one the library's bulk-round peel deletes in (the order  */
/* Alg. 7 takes from Core).  Round j of the peel: c = max(c, min f over X);  */
/* R_j = {v in X : f(v;X) <= c}, listed by (f(v;X), lev(v;X), id) ascending, */
/* where lev is the level k of Def. est for the estimate (the paper's tie    */
/* key k[v,h] of Alg. 4) and 0 for deg_h; then X <- X \ R_j.  Every core set */
/* {c >= K} is a suffix of this order, which is all that Prop. dense's proof */
/* uses of the order.                                                        */
/* ------------------------------------------------------------------------ */
static int64_t est_level(const int32_t *x, int64_t d, int64_t M)
{
    int64_t k = 0;
    for (;;) {
        int64_t S = 0;
        for (int64_t j = 0; j < d; j++)
            if (x[j] >= k) S++;
        if (S <= M) return k;
        k++;
    }
}

/* f(v;X) as vertex_fn, and lev(v;X) into *lev. */
static int64_t vertex_fn_lev(orc_ws *ws, int64_t v, int h, const uint8_t *alive, int mode, const uint8_t *r,
                             int64_t M, int64_t *lev)
{
    int64_t cnt = ball_of(v, h, ws->rp, ws->col, alive, ws->mark, ws->ball, NULL);
    if (mode == 0) {
        *lev = 0;
        return cnt - 1;
    }
    for (int64_t i = 0; i < cnt; i++) ws->xr[i] = r[ws->ball[i]];
    *lev = est_level(ws->xr, cnt, M);
    return orc_delta(ws->xr, cnt, M);
}

typedef struct {
    int64_t f, lev;
    int32_t id;
} orc_okey;

static int cmp_okey(const void *a, const void *b)
{
    const orc_okey *x = (const orc_okey *)a, *y = (const orc_okey *)b;
    if (x->f != y->f) return x->f < y->f ? -1 : 1;
    if (x->lev != y->lev) return x->lev < y->lev ? -1 : 1;
    return (x->id > y->id) - (x->id < y->id);
}

/* Bulk-round deletion order of X = alive_in (NULL: V).  order_out[count]
 * receives the order, core_out[n] the core numbers (-1 outside X) and
 * round_out[n] (nullable) the round of each deletion.  Returns the count. */
ORC_API int64_t orc_bulk_order(int64_t n, const int32_t *rp, const int32_t *col, const uint8_t *alive_in, int h,
                               int mode, const uint8_t *r, int64_t M, int32_t *order_out, int64_t *core_out,
                               int64_t *round_out)
{
    orc_ws ws;
    if (ws_init(&ws, n, rp, col)) return -1;
    size_t nn = (size_t)(n > 0 ? n : 1);
    uint8_t *alive = (uint8_t *)malloc(nn);
    uint8_t *aff = (uint8_t *)calloc(nn, 1);
    int64_t *f = (int64_t *)malloc(sizeof(int64_t) * nn);
    int64_t *lev = (int64_t *)malloc(sizeof(int64_t) * nn);
    orc_okey *R = (orc_okey *)malloc(sizeof(orc_okey) * nn);
    int32_t *ball = (int32_t *)malloc(sizeof(int32_t) * nn);
    if (!alive || !aff || !f || !lev || !R || !ball) return -1;
    int64_t remaining = 0;
    for (int64_t v = 0; v < n; v++) {
        alive[v] = alive_in ? (alive_in[v] != 0) : 1;
        remaining += alive[v];
        core_out[v] = -1;
        if (round_out) round_out[v] = -1;
    }
    for (int64_t v = 0; v < n; v++)
        if (alive[v]) f[v] = vertex_fn_lev(&ws, v, h, alive, mode, r, M, &lev[v]);
    int64_t c = -1, pos = 0, round = 0;
    while (remaining > 0) {
        int64_t mn = -1;
        for (int64_t v = 0; v < n; v++)
            if (alive[v] && (mn < 0 || f[v] < mn)) mn = f[v];
        if (mn > c) c = mn;
        int64_t nr = 0;
        for (int64_t v = 0; v < n; v++)
            if (alive[v] && f[v] <= c) {
                R[nr].f = f[v];
                R[nr].lev = lev[v];
                R[nr].id = (int32_t)v;
                nr++;
            }
        qsort(R, (size_t)nr, sizeof(orc_okey), cmp_okey);
        /* the vertices whose f can change: the h-balls of R, measured in X */
        for (int64_t i = 0; i < nr; i++) {
            int64_t nb = ball_of(R[i].id, h, rp, col, alive, ws.mark, ball, NULL);
            for (int64_t j = 0; j < nb; j++) aff[ball[j]] = 1;
        }
        for (int64_t i = 0; i < nr; i++) {
            int32_t u = R[i].id;
            order_out[pos++] = u;
            core_out[u] = c;
            if (round_out) round_out[u] = round;
            alive[u] = 0;
        }
        remaining -= nr;
        for (int64_t v = 0; v < n; v++)
            if (aff[v]) {
                aff[v] = 0;
                if (alive[v]) f[v] = vertex_fn_lev(&ws, v, h, alive, mode, r, M, &lev[v]);
            }
        round++;
    }
    free(alive);
    free(aff);
    free(f);
    free(lev);
    free(R);
    free(ball);
    ws_free(&ws);
    return pos;
}

/* Alg. 7's loop over a given order v_1..v_count of the vertex set S_1 (the
 * vertices listed; every other vertex is absent throughout).  For the suffix
 * S_i = {v_i, ..., v_count}: R_out[i-1] = sum over v in S_i of f(v; S_i), with
 * f = deg_h (mode 0; then R_i = 2|E_h(S_i)|) or the estimate with ranks r and
 * buffer M (mode 1; Alg. 7 uses fresh ranks and M from C = log(n^2/delta)).
 * R is kept up to date as Alg. 7 does: deleting v_i changes f only inside its
 * h-ball, measured before the deletion.  The best suffix maximises
 * R_i / |S_i| (ties: the later suffix, i.e. the smaller set); its start
 * index (0-based) goes to *best_i.  Returns 0. */
ORC_API int orc_dense_suffix(int64_t n, const int32_t *rp, const int32_t *col, int h, int mode, const uint8_t *r,
                             int64_t M, int64_t count, const int32_t *order, int64_t *R_out, int64_t *best_i)
{
    orc_ws ws;
    if (ws_init(&ws, n, rp, col)) return -1;
    size_t nn = (size_t)(n > 0 ? n : 1);
    uint8_t *alive = (uint8_t *)calloc(nn, 1);
    int64_t *f = (int64_t *)malloc(sizeof(int64_t) * nn);
    int32_t *ball = (int32_t *)malloc(sizeof(int32_t) * nn);
    if (!alive || !f || !ball) return -1;
    for (int64_t i = 0; i < count; i++) alive[order[i]] = 1;
    int64_t R = 0;
    for (int64_t i = 0; i < count; i++) {
        int32_t v = order[i];
        f[v] = vertex_fn(&ws, v, h, alive, mode, r, M, NULL);
        R += f[v];
    }
    *best_i = -1;
    for (int64_t i = 0; i < count; i++) {
        R_out[i] = R;
        int64_t size = count - i;
        if (*best_i < 0 ||
            (__int128)R * (__int128)(count - *best_i) >= (__int128)R_out[*best_i] * (__int128)size)
            *best_i = i;
        int32_t u = order[i];
        int64_t nb = ball_of(u, h, rp, col, alive, ws.mark, ball, NULL);
        R -= f[u];
        alive[u] = 0;
        for (int64_t j = 1; j < nb; j++) {
            int32_t a = ball[j];
            R -= f[a];
            f[a] = vertex_fn(&ws, a, h, alive, mode, r, M, NULL);
            R += f[a];
        }
    }
    free(alive);
    free(f);
    free(ball);
    ws_free(&ws);
    return 0;
}
