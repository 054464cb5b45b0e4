// Internal declarations shared by the kernels (*.hip) and the host
// orchestration (kh_host.cpp).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/khcore.h"
#include "kh_csr.hpp"

namespace kh {

// ---- sizes --------------------------------------------------------------------

// Arcs per work item of the h-degree pull kernel; vertices with more arcs are
// split across several items whose partial ORs meet in an accumulator plane.
constexpr int kPullChunk = 128;
// Arcs per chunk of the frontier-expansion kernels.
constexpr int kExpandChunk = 256;
// A hop of the R-mask BFS pulls (every alive vertex scans its neighbours) once
// its frontier's arcs exceed 1 / kRbfsPullRatio of all arcs; below that it
// pushes.  A packed union of many graphs uses kRbfsPullRatioUnion: its
// frontiers are spread over many components, and a pull scans every vertex
// of the union.
constexpr int kRbfsPullRatio = 32;
constexpr int kRbfsPullRatioUnion = 4;
// In a pulled hop a thread scans a vertex of at most kRbfsLight arcs; the arcs
// of a larger one are scanned by its whole wave.
constexpr int kRbfsLight = 32;
// A BFS hop sweeps every work item once the previous frontier's adjacency
// exceeds 1 / kSweepRatio of all arcs; below that it pulls only the alive
// neighbours of the frontier.
constexpr int kSweepRatio = 16;
// Sampled lists store 32-bit keys ((255 - rank) << 24 | id): ascending key
// order is rank descending, id ascending.  Needs n < 2^24.
constexpr int32_t kMaxSampledN = (1 << 24) - 1;
constexpr uint32_t kEmptyKey = 0xFFFFFFFFu;
// Threads of a union work-group and the largest hash table (entries) that fits
// the LDS budget of one work-group.
constexpr int kUnionThreads = 256;
// one-wave blocks of the union kernel for vertices of at most kUnionSmall
// neighbours (most vertices of a power-law graph): a smaller hash table, so more
// of them are in flight per CU, and no block-wide barriers across waves
constexpr int kUnionSmall = 64;
// block size of the union kernel for hubs (more than kHubDegree neighbours)
constexpr int kUnionHubThreads = 1024;
// Vertices with more neighbours than this order their arcs by list head rank in the union.
constexpr int kHubDegree = 1024;
// Largest hub slice (kMaxArcs, in kh_csr.hpp, leaves room for it).
constexpr int64_t kMaxHubSlice = (int64_t)1 << 23;
// Arcs per slice of a hub merged in parallel (more arcs: split; see HubSplit).
constexpr int kHubSlice = 8192;

// Per-run device state for the bulk peeling rounds (one instance in device memory).
struct RoundState {
    long long c;             // running maximum (core value of this round), starts at -1
    long long min_key;       // reduction: min key over alive vertices
    long long sum_val;       // reduction: sum of values over alive vertices
    int alive_count;         // reduction: alive vertices at round start
    int rcount;              // |R| of this round
    int rounds;              // rounds that removed at least one vertex
    int ncand;               // densest-core candidates recorded so far
    int stop;                // early-stop decision of this round
    int qcount;              // expansion chunk-queue fill
    int front_lo, front_hi;  // current frontier range inside the affected list
    int aff_fill;            // affected-list fill
    int wl_count;            // union worklist fill
    int changed_count[2];    // vertices whose (k, B) changed (ping-pong by level parity)
    int rc_count;            // worklist vertices that must be re-merged / recomputed
    int hub_count;           // the hubs among them (sampled peel: merged by wider blocks)
    int pad_hub;
    int blocks_done;         // last-block detection of the lazy exact peel's final kernel
    int mode;                // device-driven exact peel: 0 commit, 1 recompute, 2 done
    int ms_ns;               // sources of the current device-driven h-degree batch
    long long hi;            // recompute every inexact vertex whose bound is <= hi
    int hist[48];            // inexact vertices by bound - c: [0] <= 0, [b] in [2^(b-1), 2^b)
    int fcount[2];           // R-mask BFS frontier fills (ping-pong by hop parity)
    int epoch;               // device-side mark epoch (advanced by the round / level resets)
    int fepoch;              // device-side frontier-mark epoch (advanced per mask-BFS hop)
    int overflow;            // an estimate exceeded the representable range
    long long min_inexact;   // lazy exact peel: smallest bound of an inexact alive vertex
    int stall;               // lazy exact peel: a commit sequence waits for exact recomputations
    int pull_ratio;          // lazy exact peel: a mask-BFS hop pulls once its frontier holds > 1/pull_ratio of the arcs (0: never)
    unsigned long long te;     // edges traversed (exact h-degree work)
    unsigned long long arcs;   // adjacency entries read by the h-degree kernels
    unsigned long long elems;  // sample-list entries read by the union kernels
    unsigned long long pull_bytes;   // algorithmic bytes of the pull kernel (without neighbour gathers)
    unsigned long long pull_gather;  // bytes of neighbour frontier words gathered by the pull kernel
    unsigned long long union_bytes;  // algorithmic bytes of the level >= 2 union kernel
    unsigned long long rbfs_bytes;   // algorithmic bytes of the R-mask BFS hops (push and pull)
    long long hop_arcs;              // arcs of the current R-mask BFS frontier (push/pull choice)
    long long next_arcs;             // arcs of the frontier the current hop builds
    long long hop_log[4];            // trace: frontier arcs of mask-BFS hops 1..3 of the last round
    int unit_count;                  // sampled peel: work items of the hub launch (whole hubs and slices)
    int slot_count;                  // sampled peel: partial-list slots taken by hub slices
    int giant_count;                 // sampled peel: hubs split into slices
    int small_count;                 // sampled peel: worklist vertices merged by one-wave blocks
};

// Optional HIP-event timing of every launch of a kernel, on the stream it is
// launched on (slot 0: h-degree pull, slot 1: sample-list union).
struct PullTimer {
    hipEvent_t* ev = nullptr;  // pairs: ev[2i] before, ev[2i+1] after launch i
    int cap = 0;
    int used = 0;
};

// ---- kernels: graph, ranks, bookkeeping (kh_graph.hip) -------------------------------

// lid (nullable): rank of vertex v is drawn for id lid[v] (the vertex's id in its own graph).
void launch_ranks(uint8_t* r, int32_t n, uint64_t seed, uint32_t stream_id, hipStream_t s,
                  const int32_t* lid = nullptr);
// Pack graphs into one disjoint union: col[a_off[g] + j] = cols[g][j] + v_off[g].
void launch_pack_col(int32_t count, const int64_t* a_off, const int32_t* v_off, const uint64_t* col_ptrs,
                     int64_t nnz, int32_t* col, hipStream_t s);
// Scatter a packed int32 vector back to per-graph device arrays (graphs with
// n = 0 must be left out of the tables: v_off is strictly increasing).
void launch_unpack_i32(int32_t count, const int32_t* v_off, const uint64_t* dst_ptrs, int32_t total,
                       const int32_t* src, hipStream_t s);
void launch_validate(const int32_t* rp, const int32_t* col, int32_t n, int64_t nnz, int* err, hipStream_t s);
void launch_fill_i32(int32_t* p, int32_t v, int64_t count, hipStream_t s);
void launch_fill_i64(int64_t* p, int64_t v, int64_t count, hipStream_t s);
void launch_alive_from(const uint8_t* src, uint8_t* alive, int32_t n, hipStream_t s);
void launch_alive_degree(const int32_t* rp, const int32_t* col, const uint8_t* alive, int32_t* adeg, int32_t n,
                         hipStream_t s);
void launch_compact_alive(const uint8_t* alive, int32_t n, int32_t* out, int* count, hipStream_t s);
void launch_round_reset(RoundState* st, hipStream_t s, int gate = 0);
// inexact (nullable): also st->min_inexact = min key over alive v with inexact[v] == 0
// ("not exact": for the lazy top level, the vertices not yet active).
void launch_reduce(const int64_t* key, const int64_t* val, const uint8_t* alive, int32_t n, RoundState* st,
                   hipStream_t s, int gate = 0, const uint8_t* exact = nullptr);
void launch_round_begin(RoundState* st, int64_t* cand_k, int64_t* cand_size, int64_t* cand_sum, int early_stop,
                        hipStream_t s);
// rnd (nullable): rnd[v] = the round's epoch for every vertex taken (its deletion round).
void launch_select(const int64_t* key, uint8_t* alive, int32_t n, RoundState* st, int64_t* core, int32_t* rlist,
                   int32_t* mark, int32_t epoch, int kill, hipStream_t s, int32_t* rnd = nullptr);
void launch_kill_list(const int32_t* list, const int* count, uint8_t* alive, hipStream_t s);
// Chunk queue over the adjacency of list[*lo .. *hi) (lo/hi may be NULL: 0 and count).
// arcs (nullable): adds the listed vertices' degrees.  pull_st (nullable): does
// nothing when that round state's mask-BFS hop pulls (see launch_rbfs_hop).
// grid (0: 128 blocks): blocks of the launch.
void launch_enqueue(const int32_t* list, const int* lo, const int* hi, const int32_t* rp, int32_t* qv, int32_t* qb,
                    int* qcount, hipStream_t s, long long* arcs = nullptr, const RoundState* pull_st = nullptr,
                    int64_t nnz = -1, int grid = 0);
// mode 0: mark alive unmarked neighbours with `epoch` and append them to out[*out_count++]
// mode 1: decrement adeg of alive neighbours
void launch_expand(const int32_t* qv, const int32_t* qb, const int* qcount, const int32_t* rp, const int32_t* col,
                   const uint8_t* alive, int32_t* mark, int32_t epoch, int mode, int32_t* out, int* out_count,
                   int32_t* adeg, hipStream_t s);
// front_lo = front_hi; front_hi = aff_fill; qcount = 0
void launch_next_frontier(RoundState* st, hipStream_t s);
// qcount = 0, wl_count = 0, changed_count[level & 1] = 0
void launch_level_reset(RoundState* st, int level, hipStream_t s);
void launch_set_int(int* p, int v, hipStream_t s);
void launch_scan_i64(const int64_t* in, int64_t* out, int32_t n, int64_t* partials, hipStream_t s);
void launch_core_to_i32(const int64_t* core, int32_t* out, int32_t n, int* overflow, hipStream_t s);
// anchor[v] = alive neighbour of largest alive degree (smallest id on ties), -1 if none;
// list == NULL: all vertices; only_dead: refresh only anchors that were deleted.
void launch_anchor(const int32_t* list, const int* count, int32_t n, const int32_t* rp, const int32_t* col,
                   const uint8_t* alive, const int32_t* adeg, int32_t* anchor, int only_dead, hipStream_t s);
// deg[v] = a lower bound of deg_h(v;X) (alive degrees along the anchor chain), exact[v] = (h == 1).
void launch_lower_bound(const int32_t* list, const int* count, int32_t n, int h, const uint8_t* alive,
                        const int32_t* adeg, const int32_t* anchor, int64_t* deg, uint8_t* exact, hipStream_t s);
void launch_record_fill(RoundState* st, int* hopfill, int t, hipStream_t s);
// device-driven exact peel steps
void launch_bound_hist(const uint8_t* alive, const int64_t* deg, const uint8_t* exact, int32_t n, RoundState* st,
                       hipStream_t s, const int32_t* seg = nullptr, int* shist = nullptr, int gate = 0);
void launch_decide(RoundState* st, int cap, hipStream_t s);
// The recompute sequence ends by lifting the stall and resetting the round state.
// One sweep for the commit sequence: min key, alive count and the smallest
// bound of an inexact vertex.
void launch_reduce_hist(const int64_t* deg, const uint8_t* alive, const uint8_t* exact, int32_t n, RoundState* st,
                        hipStream_t s);
void launch_unstall(RoundState* st, hipStream_t s);
// The commit decision and the round begin folded into the selection: commit
// when no inexact bound is at or below c' = max(c, min key) (then c = c',
// rounds += 1, R = {key <= c}), else stall; mode 2 once nothing is alive.
void launch_select_commit(const int64_t* key, uint8_t* alive, int32_t n, RoundState* st, int64_t* core,
                          int32_t* rlist, int32_t* mark, hipStream_t s, int32_t* rnd = nullptr);
// For the listed R (rlist, *rcount): mode 0 sets R's mask bits (bit j for
// rlist[j]) in rmask and gain and R's bits in the frontier bitmap fbits, mode 1
// removes R from the alive set; both then queue R's adjacency in chunks for the
// next expansion (*qcount must be 0).
void launch_enqueue_r(const int32_t* rlist, const int* rcount, const int32_t* rp, int32_t* qv, int32_t* qb, int* qcount,
                      int mode, uint64_t* rmask, uint64_t* gain, uint32_t* fbits, uint8_t* alive, hipStream_t s,
                      long long* arcs = nullptr);
// arr[list[i]] = 0 and fbits[list[i] / 32] = 0 for i < *count, then end mask-BFS
// hop t: hopfill[t] = aff_fill, qcount = 0, hop_arcs = next_arcs (next_arcs =
// 0), and for t < h a new frontier epoch and fcount[(t+1)&1] = 0.
void launch_clear_hop_end(const int32_t* list, const int* count, uint64_t* arr, uint32_t* fbits, RoundState* st,
                          int* hopfill, int t, int h, hipStream_t s, int grid = 0);
// arr_k[list_k[i]] = 0 for three (list, count, array) triples at once; with
// st != NULL the last block then resets the round state for the next round
// (unless the sequence is stalled).
void launch_clear_u64_lists3(const int32_t* l0, const int* c0, uint64_t* a0, const int32_t* l1, const int* c1,
                             uint64_t* a1, const int32_t* l2, const int* c2, uint64_t* a2, hipStream_t s,
                             RoundState* st = nullptr, int grid = 0);
// Picks the inexact alive vertices with deg <= st->hi as the next sources (at
// most cap).  seg (nullable): segment (graph) of every vertex of a packed union;
// then each source also gets a bit position sbit[slot] that is unique within its
// segment, at most qbits per segment (gcnt: per-segment counters, all-zero
// before; the scatter of the batch zeroes them again).
void launch_pick(const uint8_t* alive, const int64_t* deg, const uint8_t* exact, int32_t n, RoundState* st,
                 int32_t* out, int cap, hipStream_t s, const int32_t* seg = nullptr, int* gcnt = nullptr,
                 int32_t* sbit = nullptr, int qbits = 0, const long long* shi = nullptr);
// Per-segment thresholds shi[seg] (packed unions) from per-segment histograms.
void launch_decide_seg(RoundState* st, int nseg, int* shist, long long* shi, int cap, hipStream_t s);
// R-mask BFS: after h hops rmask[v] holds bit (j mod 64) for every deleted r_j within
// distance h of v in G[X]; first-visited vertices are appended to alist in hop order.
// One hop, in push form (the frontier's chunks queued by launch_enqueue_r /
// launch_enqueue) or, when the frontier's arcs exceed 1/kRbfsPullRatio of all
// nnz arcs, in pull form (every alive vertex ORs the frontier masks of its
// neighbours), decided inside the one kernel.  The frontier is gain_cur (bits
// passed on, zero elsewhere) and the bitmap fbits_cur of the same vertices;
// the next frontier goes to gain_next, fnext and fbits_next (nullable: the last
// hop's frontier is not needed as a bitmap).  timer (nullable) brackets it.
void launch_rbfs_hop(const int32_t* qv, const int32_t* qb, const int* qcount, int32_t n, const int32_t* rp,
                     const int32_t* col, const uint8_t* alive, const uint64_t* gain_cur, const uint32_t* fbits_cur,
                     uint64_t* rmask, uint64_t* gain_next, uint32_t* fbits_next, int32_t* mark, int32_t* fmark,
                     int32_t* fnext, int* fnext_count, int32_t* alist, int* aff_fill, RoundState* st, int64_t nnz,
                     hipStream_t s, PullTimer* timer = nullptr, int grid = 0);
// exact decrement for vertices at distance exactly h (deg -= |R within h|), bound otherwise
void launch_decay_masked(const int32_t* alist, RoundState* st, const int* hopfill, int h, const uint8_t* alive,
                         const int32_t* adeg, const int32_t* anchor, const uint64_t* rmask, int64_t* deg,
                         uint8_t* exact, hipStream_t s);

// ---- kernels: bit-parallel multi-source bounded BFS (kh_msbfs.hip) ---------------------

// Per-batch control block of the bit-parallel BFS (device memory, reset by the
// batch's first kernel).  Lists are double-buffered by hop parity.
struct MsCtl {
    int fl_count[2];        // frontier list length (vertices with new bits at the hop)
    long long fdeg[2];      // sum of the degrees of the frontier list
    int cv_count[2];        // candidate vertices of the hop
    int ci_count[2];        // candidate work items of the hop
    int fc_count[2];        // 64-arc chunks of the frontier's vertices with more than 64 arcs
    int tl_count;           // visited tiles (64 consecutive vertices holding a nonzero vis word)
    int dense;              // 1 once a hop has swept the whole graph (sticky for the batch)
    int dense_at;           // first dense hop (0: none)
    int pad;
};
// All-zero between batches: the last kernel of a batch zeroes it.

struct MsPlanes {
    int Q;                // 64-bit words per vertex (sources per batch = 64 Q)
    uint64_t* vis;        // n*Q, visited sets; kept all-zero between batches
    uint64_t* frA;        // n*Q, frontier (ping)
    uint64_t* frB;        // n*Q, frontier (pong)
    uint64_t* acc;        // n*Q, OR accumulator for split / pushed vertices; kept all-zero
    uint32_t* bmA;        // ceil(n/32), bit per vertex: frontier word nonzero (ping); kept all-zero
    uint32_t* bmB;        // (pong)
    uint32_t* bmT;        // touched-by-push bitmap; kept all-zero
    uint32_t* bmC;        // candidate bitmap; kept all-zero
    int32_t* touched;     // n, vertices touched by the push hop
    int* touched_count;   // device counter
    int32_t* flA;         // n, frontier list (hop parity 0)
    int32_t* flB;         // n, frontier list (hop parity 1)
    int2* fcA;            // n + nnz/64: (vertex, first arc) chunks of large frontier vertices (parity 0)
    int2* fcB;            // (parity 1)
    int32_t* tl;          // ceil(n/64), visited tile list
    uint32_t* bmTile;     // bit per tile: listed in tl; kept all-zero
    int32_t* cvA;         // n, candidate vertices (parity 0)
    int32_t* cvB;         // n, (parity 1)
    int32_t* ciA;         // nitems, candidate work items (parity 0)
    int32_t* ciB;         // nitems, (parity 1)
    MsCtl* ctl;
    uint32_t* cnt;        // 64 Q per-source counters (per segment when seg != NULL); kept all-zero
    // Segmented batches (a packed union of graphs): sources of different graphs
    // never meet, so each graph uses the 64 Q bit positions on its own.
    const int32_t* seg;   // nullable: segment of every vertex
    const int32_t* sbit;  // nullable: bit position of source j (else j)
    int* gcnt;            // per-segment pick counters (reset by the scatter)
    int ns_cap;           // most sources of one batch (64 Q, or n when segmented)
    uint8_t* exact_out;   // nullable: exact_out[source] = 1 (its h-degree is now exact)
    uint64_t* valid;      // Q words: bits of the batch's sources
    PullTimer* timer;     // nullable
};

struct MsItems {
    int32_t nitems;
    int32_t* u;       // item vertex
    int32_t* beg;     // first arc
    int32_t* end;     // one past last arc
    uint8_t* split;   // 1 if the vertex has several items
    int32_t nsplit;
    int32_t* split_list;  // vertices with several items
    int32_t* vitem;   // n: first item of each vertex (its items are consecutive)
    int64_t nnz;      // arcs of the graph
};

// One batch of ns <= 64 Q sources: deg[src[j]] = |N(src[j]; h, X)| - 1.  With
// ns_dev != NULL the batch size is min(*ns_dev, 64 Q), read on the device (0: no-op).
void ms_batch(const MsPlanes& P, const MsItems& I, int32_t n, const int32_t* rp, const int32_t* col,
              const uint8_t* alive, const int32_t* adeg, const int32_t* src, int ns, const int* ns_dev, int h,
              int64_t* deg, RoundState* st, hipStream_t s);

// ---- kernels: sampled lists (kh_union.hip) ---------------------------------------------

// Device arrays of one level i of the sampled lists.
struct LevelView {
    const int64_t* off;  // n+1 list offsets (capacity bounds)
    uint32_t* keys;      // list entries
    int32_t* size;       // |B[v,i]|
    uint8_t* k;          // k[v,i]
    int32_t* m;          // alive neighbours w with k[w,i-1] == k[v,i]
    uint8_t* cut;        // 1 if k[v,i] was set by the M threshold (k > max_w k[w,i-1])
    int16_t* lost;       // for vertices changed this round: highest rank that left B[v,i] (-1: none)
    uint8_t* kold;       // for vertices changed this round: k[v,i] before the change
    uint32_t* meta;      // packed |B[v,i]| (bits 0-15) | k[v,i] (16-23) | rank of the first entry (24-31)
};

// Mv (nullable): per-vertex M, for batches of graphs of different sizes.
void launch_cap_level1(const int32_t* rp, int32_t n, int32_t M, const int32_t* Mv, int64_t* cap, hipStream_t s);
void launch_cap_next(const int32_t* rp, const int32_t* col, int32_t n, int32_t M, const int32_t* Mv,
                     const int64_t* cap_prev, int64_t* cap, hipStream_t s);
// Level 1 (neighbour lists are singletons).  worklist == NULL: all vertices (initialisation).
void launch_union1(const int32_t* worklist, const int* wl_count, int32_t n, const int32_t* rp, const int32_t* col,
                   const uint8_t* alive, const uint8_t* rank, int32_t M, const int32_t* Mv, LevelView cur,
                   int32_t* changed, int* changed_count, RoundState* st, hipStream_t s);
// Hubs of a level's worklist with more than `slice` arcs are split: their
// slices of at most `slice` arcs are merged in parallel like vertices of their
// own, each into a partial list (its entries of rank >= its own level), and the
// hub then merges its slices' partial lists.  Unions are associative under the
// truncation (the level of a union is at least every part's level, and above
// that level every part's list is complete), so the result is the hub's list.
struct HubSplit {
    int32_t slice = 0;          // arcs per slice (0: no split)
    int4* unit = nullptr;       // hub-launch work items: (vertex, first arc, end arc, slot or -1)
    int32_t unit_cap = 0;
    int4* giant = nullptr;      // split hubs: (vertex, first slot, slices, 0)
    uint32_t* pkeys = nullptr;  // partial lists: slot q at pkeys + q * pcap, grouped by rank
    int32_t pcap = 0;           // >= M
    int32_t* pmeta = nullptr;   // per slot: size, level, largest neighbour level, head rank
    int32_t* phk = nullptr;     // per slot: the slice's alive neighbours by level (256 counts)
    int32_t slot_cap = 0;
};
// Level i >= 2.  hubs (nullable): vertices of the worklist with more than
// kHubDegree arcs, merged by wider blocks (split per `split` when it is on).
void launch_union(const int32_t* worklist, const int* wl_count, int32_t n, const int32_t* rp, const int32_t* col,
                  const uint8_t* alive, const uint8_t* rank, int32_t M, const int32_t* Mv, int hash_log2,
                  LevelView prev, LevelView cur, int32_t* cursor, int32_t* order, int32_t* changed,
                  int* changed_count, RoundState* st, hipStream_t s, PullTimer* timer = nullptr,
                  const int32_t* hubs = nullptr, const int* hub_count = nullptr, const HubSplit* split = nullptr,
                  const int32_t* smalls = nullptr, const int* small_count = nullptr, int hash_log2_small = 0);
// Propagate the deletions and changes of level i-1 over the arcs of the queued
// vertices: mark + append alive neighbours, fold the highest lost rank into
// lostmax[], and keep m[.,i] current.
void launch_expand_lists(const int32_t* qv, const int32_t* qb, const int* qcount, const int32_t* rp,
                         const int32_t* col, const uint8_t* alive, const uint8_t* rank, int32_t* mark, int32_t epoch,
                         int level, LevelView prev, LevelView cur, int32_t* lostmax, int32_t* out, int* out_count,
                         RoundState* st, hipStream_t s);
// Keep only the worklist vertices whose list can change.
// hubs (nullable): vertices with more than kHubDegree neighbours that need a
// re-merge go to this list instead of rc; smalls (nullable): those with at most
// kUnionSmall neighbours go to smalls.
// active (nullable): vertices with active[v] == 0 (not yet initialised at this
// level) are never re-merged.
void launch_classify(const int32_t* wl, const int* wl_count, LevelView cur, int32_t* lostmax, int32_t* rc,
                     int* rc_count, hipStream_t s, const int32_t* rp = nullptr, int32_t* hubs = nullptr,
                     int* hub_count = nullptr, const uint8_t* active = nullptr, int32_t* smalls = nullptr,
                     int* small_count = nullptr);
// Lazy initialisation of level h (Sec. 5): d[v] = a lower bound on the estimate
// from the level h-1 lists of v's alive neighbours (prev), for the inactive
// vertices of the list (NULL: all); resets their lostmax.
void launch_lazy_lb(const int32_t* list, const int* count, int32_t n, const int32_t* rp, const int32_t* col,
                    const uint8_t* alive, const uint8_t* active, const uint8_t* rank, int32_t M, const int32_t* Mv,
                    LevelView prev, int64_t* d, int32_t* lostmax, hipStream_t s);
// stall = (some inactive bound <= c' = max(c, min d)), hi = 2 c' + 64, rc_count = 0
void launch_lazy_decide(RoundState* st, hipStream_t s);
// When stalled: out[rc_count++] = every alive inactive v with d[v] <= hi, now active.
void launch_lazy_pick(const uint8_t* alive, uint8_t* active, const int64_t* d, int32_t n, RoundState* st,
                      int32_t* out, hipStream_t s);
// Alg. 1 estimate from level h.  worklist == NULL: all vertices.
void launch_estimate(const int32_t* worklist, const int* wl_count, int32_t n, const uint8_t* alive,
                     const uint8_t* rank, const int32_t* size, const uint8_t* kk, int32_t M, const int32_t* Mv,
                     int64_t* d, RoundState* st, hipStream_t s);

// ---- deletion order of the bulk-round peel (kh_order.hip) ------------------------------
// Working arrays of deletion_order: n entries each, plus temp_bytes of sort storage.
struct OrderScratch {
    uint32_t* lkey;
    uint32_t* lkey_out;
    int32_t* ids;
    int32_t* ids_out;
    uint64_t* mkey;
    uint64_t* mkey_out;
    void* temp;
    size_t temp_bytes;
};
size_t order_temp_bytes(int32_t n);
// order[i] = i-th deleted vertex by (rnd[v], key[v], lev[v] (nullable: 0), v);
// pos[order[i]] = i.  *bad |= 1 if some rnd < 0 or key outside [0, 2^32).
hipError_t deletion_order(int32_t n, const int32_t* rnd, const int64_t* key, const uint8_t* lev, OrderScratch w,
                          int32_t* order, int64_t* pos, int* bad, hipStream_t s);

// ---- h-degrees in a fixed device array (kh_noalloc.hip) --------------------------------
// Size of the array (per GPU, held until the process ends) and the most GPUs
// the library tracks it for.
constexpr size_t kNoallocScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;
// Address of the array on `device` (which must be current); looked up once per device.
hipError_t noalloc_scratch_init(int device, void** out);
// Bytes the layout needs for a graph with nitems pull work items (nsplit split
// vertices) at Q words per vertex.
int64_t noalloc_hdeg_bytes(int32_t n, int64_t nnz, int64_t nitems, int64_t nsplit, int Q);
// deg_out[v] = deg_h(v;X) (device int32), te_out (device, nullable) = edges
// traversed; enqueued on s, no allocation, no host wait.  KH_ENOMEM when the
// graph does not fit the array.
kh_status noalloc_hdeg(void* scratch_ptr, int32_t n, int64_t nnz, const int32_t* rp, const int32_t* col,
                       int64_t nitems, int64_t nsplit, int h, const uint8_t* alive_in, int32_t* deg_out,
                       int64_t* te_out, hipStream_t s);

// ---- serving (kh_serve.cpp) and its hooks into the engines (kh_host.cpp) -------------
// A serving thread runs requests with its own pinned round-state mirror, and
// without the context's profiling slots.
void worker_thread_begin(RoundState* pinned);
void worker_thread_end();
// Stops the context's serving loop, if any (kh_context_destroy calls it).
void serve_shutdown(kh_context* ctx);
kh_context* graph_context(const kh_graph* g);
int context_device(const kh_context* ctx);

}  // namespace kh
