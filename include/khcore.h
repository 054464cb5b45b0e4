/*
 * khcore.h -- C ABI of the MI355X (gfx950) library for distance-generalized
 * (k,h)-core decomposition, exact and sampled.
 *
 * Method: N. Tatti, "Fast computation of distance-generalized cores using
 * sampling" (arXiv 2112.06154).  Section numbers below refer to that paper.
 *
 * Conventions shared by every entry point
 *   - Every call returns kh_status: KH_OK (0) or a negative error code, and
 *     never throws or aborts across the ABI.  kh_status_str() names a code.
 *   - Graphs are simple and undirected, given as int32 CSR: row_ptr[n+1] with
 *     row_ptr[0] = 0 and row_ptr[n] = nnz = 2m, col[nnz] holding both arc
 *     directions, each adjacency sorted ascending, no self-loops, no
 *     duplicates.  Vertex ids are 0..n-1.  nnz <= 2^31 - 2^24 - 1 (arc indices
 *     are int32 on the device, with headroom for chunked arc ranges); a larger
 *     nnz is KH_EINVAL.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Calls that take
 *     one enqueue their GPU work on it; calls that return results in host
 *     memory synchronise that stream before returning.
 *   - Pointers documented as "device" must be device memory of the context's
 *     GPU (e.g. torch tensor storage); "host" pointers are ordinary memory.
 *   - All device arithmetic is integer.  The only floating point is the
 *     buffer size M (computed once on the host in binary64) and the reported
 *     density.
 *   - Calls on one context may come from several host threads at once
 *     (each call keeps its own device state); profiling (kh_profile_*)
 *     records only calls made while no other thread uses the context.
 */
#ifndef KHCORE_H
#define KHCORE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t kh_status;
#define KH_OK          0
#define KH_EINVAL     (-1) /* bad argument (h < 1, delta outside (0,1), NULL pointer, ...) */
#define KH_ENOMEM     (-2) /* device memory or the context's HBM budget exhausted */
#define KH_EDEVICE    (-3) /* no usable GPU, or a HIP runtime error */
#define KH_EGRAPH     (-4) /* CSR not canonical: asymmetric, self-loop, duplicate, unsorted, out of range */
#define KH_EOVERFLOW  (-5) /* a core number or estimate does not fit int32 */
#define KH_EBUSY      (-6) /* a served request is still running */
#define KH_ENOTFOUND  (-7) /* unknown ticket */
#define KH_ENOTIMPL   (-8) /* parameters outside what this library supports (see the entry point) */

/* kh_graph_load_csr flags */
#define KH_PTRS_HOST           0u /* row_ptr/col are host memory; the library copies them */
#define KH_PTRS_DEVICE_BORROW  1u /* row_ptr/col are device memory the library borrows (no copy);
                                     they must outlive the kh_graph */
#define KH_CANONICALIZE        2u /* host pointers only: drop self-loops and duplicates,
                                     symmetrise and sort instead of rejecting */
#define KH_TRUST_CSR           4u /* skip validation (the caller guarantees canonical CSR) */

/* kh_params.flags */
#define KH_WANT_DENSE   1u /* also compute the densest-core estimate (Sec. 6) */
#define KH_DENSE_PRUNE  2u /* densest core: only levels K with K(1+eps) >= (1-eps) max core */
#define KH_EARLY_STOP   4u /* sampled path: right after a round's deletions, if c + 1 >= |remaining|,
                              every remaining vertex gets c and the peel ends (Sec. 5 heuristic,
                              Sec. 8 wording); the result is min(c'(v), c*) for the first level c*
                              with c* + 1 >= #{c' > c*}.  Changes the output relative to Alg. 4,
                              off by default.  ExactCore ignores it (it cannot change c). */
#define KH_OUT_DEVICE   8u /* core_out / deg_out are device pointers */
#define KH_LAZY_INIT   32u /* sampled path: build B[v,h] only once a lower bound on v's estimate
                              from its neighbours' level h-1 lists (Prop. monotone) no longer keeps
                              v above the running maximum (Sec. 5, first heuristic).  The output is
                              unchanged; h >= 2 (ignored for h = 1). */
#define KH_DENSE_FULL  16u /* with KH_WANT_DENSE: Alg. 7 over every suffix of the deletion order
                              (the peel's bulk rounds in sequence; inside a round by the key at
                              deletion -- the estimate or deg_h -- then k[v,h], then id) instead of
                              the core levels only; every core level is such a suffix.  With
                              KH_DENSE_PRUNE the suffixes start inside {v : c(v) >= gamma k'}.
                              dense_k is then the smallest core number in the chosen set.  One
                              replay round per vertex: meant for graphs up to ~1e5 vertices.
                              kh_core only (KH_ENOTIMPL for kh_core_batch, kh_dense, and with
                              KH_EARLY_STOP). */

typedef struct kh_context kh_context;
typedef struct kh_graph kh_graph;

typedef struct kh_params {
    int32_t  h;            /* distance bound, >= 1 (Sec. 2) */
    double   epsilon;      /* <= 0: ExactCore.  > 0: Core (Alg. 4) with M from Eq. (buffer);
                              the (1 +- eps) guarantee of Prop. yield needs eps <= 1/2 */
    double   delta;        /* failure probability, in (0,1); the paper uses 0.05 (Sec. 8) */
    uint64_t seed;         /* seed of the rank stream (ranks are geometric(1/2), Sec. 3) */
    int32_t  M_override;   /* > 0: use this integer M instead of Eq. (buffer) for Core */
    int32_t  M_dense_override; /* > 0: same for the densest-core pass (Alg. 7) */
    uint32_t flags;        /* KH_WANT_DENSE | KH_DENSE_PRUNE | KH_EARLY_STOP | KH_OUT_DEVICE | KH_DENSE_FULL
                              | KH_LAZY_INIT */
} kh_params;

typedef struct kh_result {
    int32_t M_used;          /* integer M of the core pass (0 for ExactCore) */
    int32_t M_dense_used;    /* integer M of the densest-core pass (0 if exact or not run) */
    int32_t rounds;          /* bulk peeling rounds */
    int32_t max_core;        /* largest core number */
    int64_t dense_k;         /* densest core level K* (-1 if not computed); with KH_DENSE_FULL the
                                smallest core number in the chosen suffix */
    int64_t dense_size;      /* |F_K*|, F_K = {v : core[v] >= K} (KH_DENSE_FULL: the suffix's size) */
    int64_t dense_R;         /* sum over F_K* of deg_h (exact) or of the estimate (sampled) */
    double  dense_density;   /* dense_R / (2 dense_size): the (estimated) h-density |E_h|/|F| */
    int64_t edges_traversed; /* exact path: sum over processed sources s of the alive degrees of
                                vertices within distance h-1 of s (arcs a per-source BFS inspects) */
    int64_t arcs_scanned;    /* physical adjacency entries read by the h-degree kernels */
    int64_t list_elements;   /* sampled path: sample-list entries read by the union kernels */
    double  seconds;         /* wall time of the call */
} kh_result;

/* ---- host-only helpers (no GPU needed) ----------------------------------- */

const char *kh_status_str(kh_status s);

/* Integer buffer size floor(M) of Eq. (buffer) (Sec. 3):
 *   C = log(2n/delta)   (dense == 0, Alg. 4), or log(n^2/delta) (dense != 0, Alg. 7),
 *   M = 1 + 4(2+eps)/eps^2 (C + log 8).
 * Returns -1 for n < 1, eps <= 0 or delta outside (0,1). */
int64_t kh_buffer_size(int64_t n, double epsilon, double delta, int32_t dense);

/* Validate a host CSR against the conventions above (Sec. 2: simple undirected
 * graph).  KH_OK, or KH_EGRAPH / KH_EINVAL. */
kh_status kh_validate_csr(int32_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col);

/* ---- context and graphs ---------------------------------------------------- */

/* Create a context on HIP device `device`.  hbm_budget_bytes caps the device
 * memory the library may hold for this context (0 = no cap beyond the GPU's).
 * Device blocks that a call released are kept by the context for reuse by
 * later calls (at most a quarter of the budget, or of the device's memory)
 * until kh_context_destroy.  KH_EDEVICE when the device is missing. */
kh_status kh_context_create(int32_t device, uint64_t hbm_budget_bytes, kh_context **out);
void kh_context_destroy(kh_context *ctx);

/* Make a graph resident on the context's GPU (the graph G of Sec. 2).  With
 * KH_PTRS_HOST the CSR is validated (or canonicalised with KH_CANONICALIZE)
 * and copied; with KH_PTRS_DEVICE_BORROW the device arrays are validated on
 * the GPU (unless KH_TRUST_CSR) and borrowed.  n = 0 is allowed. */
kh_status kh_graph_load_csr(kh_context *ctx, int32_t n, int64_t nnz, const int32_t *row_ptr,
                            const int32_t *col, uint32_t flags, void *stream, kh_graph **out);
void kh_graph_free(kh_graph *g);
int32_t kh_graph_n(const kh_graph *g);
int64_t kh_graph_nnz(const kh_graph *g);

/* ---- the hot path ---------------------------------------------------------- */

/* Core decomposition (Sec. 2 ExactCore when epsilon <= 0, else Alg. 4 Core)
 * of the whole graph.  core_out[n] (int32, host unless KH_OUT_DEVICE)
 * receives c(v) or c'(v).  The result does not depend on tie-breaking, so it
 * is unique and bit-reproducible.  With KH_WANT_DENSE, res receives the
 * densest core level (Sec. 6; for epsilon > 0 its sum uses fresh ranks from
 * stream 1 and M from C = log(n^2/delta), Alg. 7).  res may be NULL.
 * Errors: KH_EINVAL (h < 1, delta outside (0,1), NULL core_out with n > 0),
 * KH_ENOTIMPL (sampled path with n >= 2^24, or an integer M whose LDS hash set,
 * 2 (M + 1025) entries rounded up to a power of two, does not fit one
 * work-group's LDS next to ~17 KiB of other state: M <= 15,359 with 160 KiB),
 * KH_EOVERFLOW (core number above INT32_MAX), KH_ENOMEM, KH_EDEVICE.
 * Environment (none changes a result): read per call, KH_HUB_SLICE = arcs per
 * slice of a hub merged in parallel by the sampled peel (default 8192, 0 = off)
 * and KH_NO_GRAPH = 1 (launch round loops directly instead of replaying
 * captured HIP graphs); read once per process, KH_TRACE = 1 (round progress on
 * stderr) and KH_HEARTBEAT = seconds between progress lines of long peels. */
kh_status kh_core(kh_graph *g, const kh_params *params, int32_t *core_out, kh_result *res, void *stream);

/* kh_core over `count` graphs at once (same params for all), for many small
 * graphs that would each leave the GPU idle.  The graphs (all of this context)
 * are packed on the device into disjoint unions and decomposed by one set of
 * launches per union.  Components of a disjoint union do not interact
 * (N(v;h,X) stays in v's graph, Sec. 2), so the core numbers are each graph's
 * own; on the sampled path every vertex draws its rank from its id in its own
 * graph and uses M of Eq. (buffer) with its own graph's n, so core_outs[i] is
 * bit-identical to kh_core(graphs[i], params).
 *   core_outs[count]: one int32 array of n_i entries per graph (host, or
 *     device with KH_OUT_DEVICE); may be NULL for graphs with n = 0.
 *   results (nullable) [count]: per graph M_used, max_core and, with
 *     KH_WANT_DENSE, the dense_* fields of that graph; rounds, edges_traversed,
 *     arcs_scanned, list_elements and seconds describe the packed union the
 *     graph was part of (equal across its graphs).
 * Graphs are packed in order of size into unions of at most 2^24 - 1 vertices
 * (sampled) or 2^31 - 2 vertices and 2^31 - 2^24 - 1 arcs (exact); a batch runs as
 * consecutive unions.
 * Errors: as kh_core; KH_ENOTIMPL with KH_EARLY_STOP (its stopping test is per
 * graph).  On error no result of the batch is valid. */
kh_status kh_core_batch(kh_context *ctx, int32_t count, kh_graph *const *graphs, const kh_params *params,
                        int32_t *const *core_outs, kh_result *results, void *stream);

/* ---- serving ------------------------------------------------------------------
 * A request is one kh_core call (Sec. 2 ExactCore or Alg. 4 Core) queued on the
 * context.  Worker threads, each with its own HIP stream, admit requests in
 * arrival order as soon as a worker is free and the request's device-memory
 * estimate fits next to the running ones; queued requests with identical
 * kh_params and a graph within a factor 4 of its size join an admitted one in a
 * single kh_core_batch call (continuous batching), so requests that arrive
 * while others run overlap on the GPU and no request waits for a much larger
 * one packed with it.
 * Each request's core_out and result equal those of kh_core on its graph
 * alone.  The graph and core_out must stay valid until the request's result
 * has been collected (kh_serve_poll / kh_serve_wait return other than
 * KH_EBUSY); core_out is host memory unless params->flags has KH_OUT_DEVICE.
 * For a served request, kh_result.seconds is the latency from submission to
 * completion.  These calls are thread-safe; while a context serves, the
 * context's profiling hooks see only work of the calling thread. */

/* Start the serving loop of ctx: `workers` threads (0: 4), admission within
 * hbm_budget_bytes (0: 80% of the device memory free now), at most queue_cap
 * waiting requests (0: 65536), packed batches of at most batch_vertices
 * vertices (0: 2^20; a packed batch finishes its requests together, which is why it only
 * packs graphs of similar size).
 * KH_EBUSY if ctx already serves.  kh_serve_submit starts the loop with the
 * defaults when needed. */
kh_status kh_serve_start(kh_context *ctx, int32_t workers, uint64_t hbm_budget_bytes, int32_t queue_cap,
                         int64_t batch_vertices);

/* Queue kh_core(g, params, core_out) and return its ticket.  KH_EINVAL for
 * invalid params (as kh_core) or a graph of another context; KH_EBUSY when the
 * queue is full or the loop is stopping. */
kh_status kh_serve_submit(kh_context *ctx, kh_graph *g, const kh_params *params, int32_t *core_out,
                          uint64_t *ticket);

/* Result of a ticket: KH_EBUSY while the request waits or runs; otherwise the
 * request's own status (KH_OK, or the error kh_core returned), with *res
 * filled (res nullable), and the ticket is retired.  KH_ENOTFOUND for unknown
 * or retired tickets. */
kh_status kh_serve_poll(kh_context *ctx, uint64_t ticket, kh_result *res);

/* As kh_serve_poll, but blocks until the request has finished. */
kh_status kh_serve_wait(kh_context *ctx, uint64_t ticket, kh_result *res);

/* Withdraw a request that is still queued (not yet admitted): KH_OK and the
 * ticket is retired; KH_EBUSY once it runs or has finished (collect it);
 * KH_ENOTFOUND for unknown tickets. */
kh_status kh_serve_cancel(kh_context *ctx, uint64_t ticket);

/* Finish every queued request, stop the workers and drop uncollected results.
 * Serving calls may race with it: a kh_serve_wait blocked meanwhile returns
 * its result if its request finished before the results were dropped, else
 * KH_ENOTFOUND; a submission racing with the stop gets KH_EBUSY or starts a
 * new loop.
 * kh_context_destroy stops the loop too (no call may use the context then). */
kh_status kh_serve_stop(kh_context *ctx);

/* h-degrees deg_h(v;X) = |N(v;h,X)| - 1 (Sec. 2) of every vertex of X, where
 * X is given by alive[n] (uint8, nonzero = in X; device; NULL = all of V).
 * deg_out[n] (int32; host unless KH_OUT_DEVICE) gets -1 for v outside X.
 * edges_traversed (nullable host) receives the edges-traversed count. */
kh_status kh_hdeg(kh_graph *g, int32_t h, const uint8_t *alive, uint32_t flags, int32_t *deg_out,
                  int64_t *edges_traversed, void *stream);

/* ---- h-degrees without device allocation --------------------------------------
 * For callers that cannot allocate: code recorded into HIP graphs, tight
 * serving loops, harnesses that forbid allocation.
 *
 * kh_hdeg_noalloc gives kh_hdeg's h-degrees deg_h(v;X) = |N(v;h,X)| - 1
 * (Sec. 2) and its edges-traversed count, but calls no device (or pinned)
 * allocation routine and never waits for the GPU: it enqueues kernels on
 * `stream` and returns.  Its working memory is one fixed device array of
 * KH_NOALLOC_SCRATCH_BYTES per GPU, which the library holds from the first
 * kh_context_create on that GPU until the process ends.  Every call on a GPU
 * uses that same array and leaves its own contents in it, so calls that
 * overlap on one GPU (two streams, two threads, two contexts) race and give
 * wrong results: serialise them.
 *   alive: device uint8[n] (nonzero = in X), or NULL for X = V.
 *   deg_out: device int32[n]; -1 for v outside X.
 *   edges_traversed: device int64 (nullable): kh_hdeg's count.
 * Limit: the graph's working set, about (110 + 32 Q) n + nnz/2 bytes with
 * Q in {1,2,4,8,16} bit-plane words per vertex (the widest that fits is
 * used), must fit the array; at Q = 1 that is n up to about 5e5 at average
 * degree 10.
 * The graph (its device CSR), alive and the outputs must stay valid until the
 * enqueued work has completed (synchronise the stream before kh_graph_free).
 * Errors, decided on the host before anything is enqueued: KH_EINVAL (NULL
 * graph, NULL deg_out with n > 0, h < 1), KH_ENOMEM (the graph does not fit
 * the array); KH_EDEVICE when a launch fails. */
#define KH_NOALLOC_SCRATCH_BYTES (64ull << 20)
kh_status kh_hdeg_noalloc(kh_graph *g, int32_t h, const uint8_t *alive, int32_t *deg_out,
                          int64_t *edges_traversed, void *stream);

/* Ranks r[v] (Sec. 3, geometric(1/2), capped at 255) of vertices 0..n-1 for
 * (seed, stream_id): word j of vertex v is
 *   sm(sm(sm(seed) ^ v) ^ (stream_id * 2^32 + j)), sm = SplitMix64's mixer,
 * and r[v] counts the zero bits before the first one bit, words in order.
 * r_out[n] is device memory. */
kh_status kh_ranks(kh_context *ctx, int32_t n, uint64_t seed, uint32_t stream_id, uint8_t *r_out,
                   void *stream);

/* Sampled lists after initialisation (Sec. 3, B[v,i] and k[v,i] for
 * i = 1..h on X = alive (device, NULL = V), built by the union kernels of
 * Alg. 4's first loop), exported for inspection.  For level `level`
 * (1 <= level <= params->h): k_out[n] (int32, -1 outside X), size_out[n]
 * (int32), and, when members_out is not NULL, the members of each B[v,level]
 * concatenated in vertex order, each vertex's members in ascending id order
 * (members_cap entries available; KH_EINVAL if too small).  est_out (nullable,
 * int64[n]) receives Alg. 1's estimate from level h.  All outputs are host
 * memory.  Uses params->seed (stream 0) and M as kh_core does. */
kh_status kh_sampled_lists(kh_graph *g, const kh_params *params, const uint8_t *alive, int32_t level,
                           int32_t *k_out, int32_t *size_out, int32_t *members_out, int64_t members_cap,
                           int64_t *est_out, void *stream);

/* Densest core level of a given core map (Sec. 6): for every distinct value K
 * of core_in[n] (host int32) let F_K = {v : core_in[v] >= K} and
 * R_K = sum_{v in F_K} f(v; F_K), f = deg_h (epsilon <= 0) or Alg. 1's
 * estimate with ranks of stream 1 and M from C = log(n^2/delta) (Alg. 7).
 * Picks the K maximising R_K/|F_K| (ties: larger K) and fills res->dense_*.
 * KH_DENSE_PRUNE restricts K as in kh_params. */
kh_status kh_dense(kh_graph *g, const kh_params *params, const int32_t *core_in, kh_result *res, void *stream);

/* ---- measurement hooks ------------------------------------------------------ */

/* Start (on != 0; resets the totals) or stop recording three kernels: the
 * h-degree pull kernel (kernel 0), the sample-list union (kernel 1) and one hop
 * of the exact peel's R-mask BFS (kernel 2, push or pull form).  Every launch is
 * bracketed by HIP events on the stream it runs on (the round loops then launch
 * directly instead of replaying captured graphs), and the kernels count the
 * bytes they must move: for the pull kernel work items, adjacency ids and
 * visited/frontier words read and written, plus (separately) the neighbour
 * frontier words it gathers; for the union the adjacency metadata, the list
 * entries read and the list written; for the mask BFS the frontier chunks or
 * vertices, adjacency ids, alive flags and mask words read and written. */
kh_status kh_profile_enable(kh_context *ctx, int32_t on);

/* Totals for `kernel` (0, 1 or 2) since kh_profile_enable(ctx, 1): launches,
 * summed kernel time (ms), algorithmic bytes, and gathered bytes (kernel 0
 * only).  Any output pointer may be NULL.  Synchronises the recorded events. */
kh_status kh_profile_read(kh_context *ctx, int32_t kernel, int64_t *launches, double *total_ms,
                          int64_t *alg_bytes, int64_t *gather_bytes);

#ifdef __cplusplus
}
#endif

#endif /* KHCORE_H */
