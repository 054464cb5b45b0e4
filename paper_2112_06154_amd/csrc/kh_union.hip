// Sampled i-neighbourhoods B[v,i], k[v,i] and the estimate (Sec. 3, Alg. 1,
// Prop. dyn) on gfx950.
//
// For an alive v and level i >= 1 the lists satisfy (Prop. dyn)
//     T        = {v} united with B[w,i-1] over alive neighbours w,
//     k[v,i]   = max(max_w k[w,i-1], smallest k with |{u in T : r[u] >= k}| <= M),
//     B[v,i]   = {u in T : r[u] >= k[v,i]},
// which equals N(v;i,X) cut at the smallest level keeping at most M members.
//
// Lists hold 32-bit keys (255 - r) << 24 | id grouped by rank, highest rank first
// (the order inside a rank group is free).  The union is computed top-down by
// rank: a work-group walks every neighbour list with a cursor, inserting the
// members of rank L into an LDS hash set, level after level, and stops at the
// first level where the distinct count exceeds M.  Only list entries of rank
// >= k[v,i] - 1 are ever read, which is what keeps the work near the paper's
// O(M deg v) per Compute call even for hubs.
#include <climits>
#include <mutex>

#include "kh_common.hpp"
#include "kh_internal.hpp"

namespace kh {

// Neighbour walks issue the loads of several arcs per thread before using any
// of them, so that a block walking a hub keeps many random reads in flight.
constexpr int kScanUnroll = 8;
constexpr int kWideUnroll = 4;


__device__ __forceinline__ uint32_t* keys_at(const LevelView& L, int32_t v) { return L.keys + L.off[v]; }

// Packed per-list header: one 4-byte read instead of three scattered ones.
__device__ __forceinline__ uint32_t pack_meta(int size, int k, int head_rank) {
    return (uint32_t)size | ((uint32_t)k << 16) | ((uint32_t)(head_rank & 255) << 24);
}
__device__ __forceinline__ int meta_size(uint32_t m) { return (int)(m & 0xFFFFu); }
__device__ __forceinline__ int meta_k(uint32_t m) { return (int)((m >> 16) & 0xFFu); }
__device__ __forceinline__ int meta_head(uint32_t m) { return (int)(m >> 24); }

__global__ void k_cap_level1(const int32_t* __restrict__ rp, int32_t n, int32_t M, const int32_t* __restrict__ Mv,
                             int64_t* __restrict__ cap) {
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        const int64_t Mx = Mv ? Mv[v] : M;
        const int64_t c = 1 + (int64_t)(rp[v + 1] - rp[v]);
        cap[v] = c < Mx ? c : Mx;
    }
}
void launch_cap_level1(const int32_t* rp, int32_t n, int32_t M, const int32_t* Mv, int64_t* cap, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_cap_level1, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, rp, n, M, Mv, cap);
}

// cap_i(v) = min(M, 1 + sum_w cap_{i-1}(w)) bounds |B[v,i]| for every X.
__global__ void k_cap_next(const int32_t* __restrict__ rp, const int32_t* __restrict__ col, int32_t n, int32_t M0,
                           const int32_t* __restrict__ Mv, const int64_t* __restrict__ cap_prev,
                           int64_t* __restrict__ cap) {
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int nwaves = (gridDim.x * blockDim.x) >> 6;
    const int l = lane_id();
    for (int32_t v = wave; v < n; v += nwaves) {
        const long long M = Mv ? Mv[v] : M0;
        long long sum = 0;
        for (int32_t p = rp[v] + l; p < rp[v + 1]; p += 64) {
            sum += cap_prev[col[p]];
            if (sum > M) sum = M + 1;  // saturate: only min(M, .) matters
        }
        sum = wave_sum_ll(sum);
        if (l == 0) {
            const long long c = 1 + sum;
            cap[v] = c < M ? c : M;
        }
    }
}
void launch_cap_next(const int32_t* rp, const int32_t* col, int32_t n, int32_t M, const int32_t* Mv,
                     const int64_t* cap_prev, int64_t* cap, hipStream_t s) {
    if (n > 0)
        hipLaunchKernelGGL(k_cap_next, dim3(grid_for((int64_t)n * 64, 256, 16384)), dim3(256), 0, s, rp, col, n, M,
                           Mv, cap_prev, cap);
}

// ---- level 1: T = {v} + alive neighbours (all distinct) -------------------------------------
// Besides B[v,1] and k[v,1] this writes m[v,1] (alive neighbours with
// k[w,0] = 0 = k[v,1]), the cut flag (k[v,1] > 0), and for a changed list the
// highest rank that left it (a member leaves exactly when it was deleted).
__global__ __launch_bounds__(256) void k_union1(const int32_t* __restrict__ worklist, const int* wl_count, int32_t n,
                                                const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                const uint8_t* __restrict__ alive, const uint8_t* __restrict__ rank,
                                                int32_t M0, const int32_t* __restrict__ Mv, LevelView cur,
                                                int32_t* __restrict__ changed, int* changed_count, RoundState* st) {
    __shared__ int hist[256];
    __shared__ int s_k, s_size, s_nb, s_ok, s_os, s_lost, s_head;
    const int tid = threadIdx.x;
    const int total = worklist ? *wl_count : n;
    unsigned long long elems = 0;
    for (int wi = blockIdx.x; wi < total; wi += gridDim.x) {
        const int32_t v = worklist ? worklist[wi] : wi;
        if (!alive[v]) continue;
        const int M = Mv ? Mv[v] : M0;
        const int32_t b = rp[v], e = rp[v + 1];
        hist[tid] = 0;
        if (tid == 0) {
            s_ok = cur.k[v];
            s_os = cur.size[v];
            s_lost = -1;
        }
        __syncthreads();
        for (int32_t p0 = b + tid; p0 < e; p0 += (int32_t)blockDim.x * kScanUnroll) {
            int32_t w[kScanUnroll];
            int rw[kScanUnroll];
#pragma unroll
            for (int u = 0; u < kScanUnroll; ++u) {
                const int32_t p = p0 + u * (int32_t)blockDim.x;
                w[u] = p < e ? col[p] : -1;
            }
#pragma unroll
            for (int u = 0; u < kScanUnroll; ++u) rw[u] = (w[u] >= 0 && alive[w[u]]) ? rank[w[u]] : -1;
#pragma unroll
            for (int u = 0; u < kScanUnroll; ++u)
                if (rw[u] >= 0) atomicAdd(&hist[rw[u]], 1);
        }
        elems += (unsigned long long)((e - b + (int)blockDim.x - 1 - tid) / (int)blockDim.x);
        if (tid == 0) atomicAdd(&hist[rank[v]], 1);
        __syncthreads();
        if (tid == 0) {
            // k = smallest level whose suffix count is <= M
            int run = 0, k = 0, all = 0;
            for (int L = 0; L < 256; ++L) all += hist[L];
            for (int L = 255; L >= 0; --L) {
                if (run + hist[L] > M) {
                    k = L + 1;
                    break;
                }
                run += hist[L];
            }
            run = 0;
            int hr = 0;
            for (int L = 255; L >= k; --L) {
                const int c = hist[L];
                if (c > 0 && run == 0) hr = L;  // highest nonempty rank group
                hist[L] = run;                  // becomes the write cursor of rank group L
                run += c;
            }
            s_k = k;
            s_size = run;
            s_nb = all - 1;
            s_head = hr;
        }
        __syncthreads();
        const int k = s_k;
        const bool chg = changed && (s_ok != k || s_os != s_size);
        uint32_t* out = keys_at(cur, v);
        if (chg) {
            int lm = -1;
            for (int t = tid; t < s_os; t += blockDim.x) {
                const uint32_t key = out[t];
                if (!alive[key & 0xFFFFFFu]) lm = max(lm, key_rank(key));
            }
            lm = wave_max_i(lm);
            if (lane_id() == 0 && lm >= 0) atomicMax(&s_lost, lm);
            __syncthreads();
        }
        for (int32_t p0 = b + tid; p0 < e; p0 += (int32_t)blockDim.x * kScanUnroll) {
            int32_t w[kScanUnroll];
            int rw[kScanUnroll];
#pragma unroll
            for (int u = 0; u < kScanUnroll; ++u) {
                const int32_t p = p0 + u * (int32_t)blockDim.x;
                w[u] = p < e ? col[p] : -1;
            }
#pragma unroll
            for (int u = 0; u < kScanUnroll; ++u) rw[u] = (w[u] >= 0 && alive[w[u]]) ? rank[w[u]] : -1;
#pragma unroll
            for (int u = 0; u < kScanUnroll; ++u)
                if (rw[u] >= k) out[atomicAdd(&hist[rw[u]], 1)] = sample_key(rw[u], w[u]);
        }
        if (tid == 0) {
            const int rv = rank[v];
            if (rv >= k) out[atomicAdd(&hist[rv], 1)] = sample_key(rv, v);
            cur.size[v] = s_size;
            cur.k[v] = (uint8_t)k;
            cur.meta[v] = pack_meta(s_size, k, s_head);
            cur.m[v] = k == 0 ? s_nb : 0;
            cur.cut[v] = k > 0 ? 1 : 0;
            if (chg) {
                cur.lost[v] = (int16_t)s_lost;
                cur.kold[v] = (uint8_t)s_ok;
                changed[atomicAdd(changed_count, 1)] = v;
            }
        }
        __syncthreads();
    }
    elems = (unsigned long long)wave_sum_ll((long long)elems);
    if (lane_id() == 0 && elems) atomicAdd(&st->elems, elems);
}

void launch_union1(const int32_t* worklist, const int* wl_count, int32_t n, const int32_t* rp, const int32_t* col,
                   const uint8_t* alive, const uint8_t* rank, int32_t M, const int32_t* Mv, LevelView cur,
                   int32_t* changed, int* changed_count, RoundState* st, hipStream_t s) {
    if (n <= 0) return;
    const int grid = worklist ? 4096 : grid_for(n, 1, 16384);
    hipLaunchKernelGGL(k_union1, dim3(grid), dim3(256), 0, s, worklist, wl_count, n, rp, col, alive, rank, M, Mv, cur,
                       changed, changed_count, st);
}

// ---- levels i >= 2 ----------------------------------------------------------------------
struct HashSet {
    uint32_t* tab;
    uint32_t mask;
    int shift;
    int* count;
    int* hist;
    int M;
};

__device__ __forceinline__ uint32_t hs_slot(const HashSet& H, uint32_t key) { return (key * 2654435761u) >> H.shift; }

__device__ __forceinline__ void hs_insert(const HashSet& H, uint32_t key) {
    uint32_t h = hs_slot(H, key);
    for (;;) {
        const uint32_t old = atomicCAS(&H.tab[h], kEmptyKey, key);
        if (old == kEmptyKey) {
            atomicAdd(H.count, 1);
            atomicAdd(&H.hist[key_rank(key)], 1);
            return;
        }
        if (old == key) return;
        h = (h + 1u) & H.mask;
    }
}

__device__ __forceinline__ bool hs_contains(const HashSet& H, uint32_t key) {
    uint32_t h = hs_slot(H, key);
    for (;;) {
        const uint32_t x = H.tab[h];
        if (x == key) return true;
        if (x == kEmptyKey) return false;
        h = (h + 1u) & H.mask;
    }
}

// Block-wide exclusive scan of one int per thread (blockDim.x == BS).
template <int BS>
__device__ __forceinline__ int block_excl_scan_i(int v, int* sh, int* total) {
    const int l = lane_id();
    const int w = threadIdx.x >> 6;
    const int x = wave_incl_scan(v);
    if (l == 63) sh[w] = x;
    __syncthreads();
    int off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < BS / 64; ++i) {
        if (i < w) off += sh[i];
        tot += sh[i];
    }
    __syncthreads();
    *total = tot;
    return off + x - v;
}

// One flattened pass: insert every list entry of rank >= lo that sits at or
// after the arc's cursor, i.e. the next run of entries of rank >= lo (lists are
// grouped by rank, highest first, and every entry before the cursor has a
// higher rank than any pass still to come).  Each thread owns one arc per
// chunk; a block scan lays the runs end to end and all threads then insert
// entries of any run.
struct ArcState {  // one arc of the current vertex, kept in registers across passes
    int64_t off;
    int size;
    int cur;
};

__device__ __forceinline__ int arc_run(const uint32_t* __restrict__ lst, ArcState& a, int lo,
                                       unsigned long long& bytes) {
    if (a.cur >= a.size) return 0;
    bytes += 4;
    if (key_rank(lst[a.cur]) < lo) return 0;
    int end;
    bytes += 4;
    if (key_rank(lst[a.size - 1]) >= lo) {
        end = a.size;
    } else {
        // first entry of rank < lo (ranks never increase along a list)
        int x = a.cur + 1, z = a.size - 1;
        while (x < z) {
            const int mid = (x + z) >> 1;
            if (key_rank(lst[mid]) >= lo) x = mid + 1; else z = mid;
            bytes += 4;
        }
        end = x;
    }
    const int len = end - a.cur;
    a.cur = end;
    return len;
}

template <int BS>
__device__ __forceinline__ void insert_runs(int len, long long seg, const LevelView& prev, const HashSet& H, int M,
                                            int* s_offs, long long* s_seg, int* s_scan,
                                            unsigned long long& elems, unsigned long long& bytes) {
    const int tid = threadIdx.x;
    s_seg[tid] = seg;
    int tot;
    const int off = block_excl_scan_i<BS>(len, s_scan, &tot);
    s_offs[tid] = off;
    __syncthreads();
    for (int j = tid; j < tot; j += BS) {
        // the run holding entry j: last a with offs[a] <= j
        int a = 0, z = BS - 1;
        while (a < z) {
            const int mid = (a + z + 1) >> 1;
            if (s_offs[mid] <= j) a = mid; else z = mid - 1;
        }
        const uint32_t key = prev.keys[s_seg[a] + (j - s_offs[a])];
        if (*(volatile int*)H.count <= M) hs_insert(H, key);
    }
    if (tid == 0) {
        elems += (unsigned long long)tot;
        bytes += 4ull * (unsigned long long)tot;
    }
    __syncthreads();
}

// Vertices with more than kUnionThreads neighbours: arcs in chunks, cursors in
// global scratch (hubs visit only the arcs whose list head reaches lo).
template <int BS>
__device__ void union_pass_wide(int lo, int32_t b, int32_t span, bool hub, const int32_t* __restrict__ order,
                                const int32_t* __restrict__ col, const uint8_t* __restrict__ alive,
                                const LevelView& prev, int32_t* __restrict__ cursor, const HashSet& H, int M,
                                int* s_offs, long long* s_seg, int* s_scan, unsigned long long& elems,
                                unsigned long long& bytes) {
    const int tid = threadIdx.x;
    for (int32_t c0 = 0; c0 < span; c0 += BS * kWideUnroll) {
        int32_t p[kWideUnroll], w[kWideUnroll];
        ArcState a[kWideUnroll];
#pragma unroll
        for (int u = 0; u < kWideUnroll; ++u) {
            const int32_t i = c0 + u * BS + tid;
            p[u] = i < span ? (hub ? order[b + i] : b + i) : -1;
        }
#pragma unroll
        for (int u = 0; u < kWideUnroll; ++u) w[u] = p[u] >= 0 ? col[p[u]] : -1;
#pragma unroll
        for (int u = 0; u < kWideUnroll; ++u) {
            a[u].size = 0;
            a[u].cur = 0;
            a[u].off = 0;
            if (w[u] >= 0 && alive[w[u]]) {
                a[u].size = meta_size(prev.meta[w[u]]);
                a[u].cur = cursor[p[u]];
            }
        }
#pragma unroll
        for (int u = 0; u < kWideUnroll; ++u)
            if (a[u].cur < a[u].size) a[u].off = prev.off[w[u]];
        int len[kWideUnroll];
        long long seg[kWideUnroll];
#pragma unroll
        for (int u = 0; u < kWideUnroll; ++u) {
            len[u] = 0;
            seg[u] = 0;
            if (w[u] < 0) continue;
            bytes += hub ? 9 : 5;
            if (!alive[w[u]]) continue;
            bytes += 8;
            if (a[u].cur >= a[u].size) continue;
            bytes += 8;
            const int start = a[u].cur;
            len[u] = arc_run(prev.keys + a[u].off, a[u], lo, bytes);
            if (len[u]) {
                seg[u] = a[u].off + start;
                cursor[p[u]] = a[u].cur;
                bytes += 4;
            }
        }
#pragma unroll
        for (int u = 0; u < kWideUnroll; ++u)
            insert_runs<BS>(len[u], seg[u], prev, H, M, s_offs, s_seg, s_scan, elems, bytes);
    }
}

// Besides B[v,i] and k[v,i] this writes m[v,i] (alive neighbours whose
// k[w,i-1] equals the new k[v,i]), the cut flag (k[v,i] above every
// neighbour's level, i.e. fixed by the M threshold), and for a changed list the
// highest rank among its members that are not in the new list.
//
// On a recomputation (changed != NULL) the old k[v,i] bounds the new one from
// above and the old list held every member of rank >= old k, at most M of
// them; removing vertices only shrinks N(v;i).  So all entries of rank >= old k
// are inserted in one pass, and the level-by-level search only runs below it.
template <int BS>
__global__ __launch_bounds__(BS) void k_union(const int32_t* __restrict__ worklist, const int* wl_count, int32_t n,
                                               const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                                               const uint8_t* __restrict__ alive, const uint8_t* __restrict__ rank,
                                               int32_t M0, const int32_t* __restrict__ Mv, int hash_log2,
                                               LevelView prev, LevelView cur, int32_t* __restrict__ cursor,
                                               int32_t* __restrict__ order, int32_t* __restrict__ changed,
                                               int* changed_count, RoundState* st, HubSplit sp) {
    extern __shared__ uint32_t tab[];
    __shared__ int hist[256];
    __shared__ int hk[256];
    __shared__ int hh[256];    // hubs: neighbours by head rank, then scatter cursors
    __shared__ int hcum[257];  // hubs: neighbours whose list head rank is >= L
    __shared__ int s_offs[BS], s_scan[BS / 64];
    __shared__ long long s_seg[BS];
    __shared__ int s_kmax, s_htop, s_count, s_k, s_size, s_ok, s_os, s_lost, s_head;
    const int tid = threadIdx.x;
    const int bs = blockDim.x;
    const int hcap = 1 << hash_log2;
    HashSet H{tab, (uint32_t)(hcap - 1), 32 - hash_log2, &s_count, hist, M0};
    // work items: vertices (worklist, or all), or with sp.unit the hub launch's
    // units -- a whole hub, or one slice of a split hub whose result goes to a
    // partial-list slot instead of B[v,i]
    const int total = sp.unit ? *wl_count : (worklist ? *wl_count : n);
    unsigned long long elems = 0, bytes = 0;
    for (int wi = blockIdx.x; wi < total; wi += gridDim.x) {
        int32_t v, b, e;
        int slot = -1;
        if (sp.unit) {
            const int4 u = sp.unit[wi];
            v = u.x;
            b = u.y;
            e = u.z;
            slot = u.w;
        } else {
            v = worklist ? worklist[wi] : wi;
            b = rp[v];
            e = rp[v + 1];
        }
        if (!alive[v]) continue;
        const int M = Mv ? Mv[v] : M0;
        H.M = M;
        const int32_t deg = e - b;
        if (tid == 0) bytes += 8 + 6;  // rp[v], rank/alive/old state of v
        // small vertices: thread tid owns arc b + tid for the whole computation;
        // hubs: order the arcs by the head rank of the neighbour's list so that a
        // pass at rank >= L only visits the neighbours whose list reaches rank L
        const bool small = deg <= BS;
        const bool hub = deg > kHubDegree;
        for (int t = tid; t < hcap; t += bs) tab[t] = kEmptyKey;
        if (tid < 256) {
            hist[tid] = 0;
            hk[tid] = 0;
            hh[tid] = 0;
        }
        if (tid == 0) {
            s_kmax = 0;
            s_htop = rank[v];
            s_count = 0;
            s_ok = cur.k[v];
            s_os = cur.size[v];
            s_lost = -1;
        }
        __syncthreads();
        int kmax_l = 0, htop_l = -1;
        ArcState mine{0, 0, 0};
        for (int32_t p0 = b + tid; p0 < e; p0 += bs * kScanUnroll) {
            int32_t w[kScanUnroll];
            uint32_t mt[kScanUnroll];
            bool al[kScanUnroll];
#pragma unroll
            for (int u = 0; u < kScanUnroll; ++u) {
                const int32_t p = p0 + u * bs;
                w[u] = p < e ? col[p] : -1;
            }
#pragma unroll
            for (int u = 0; u < kScanUnroll; ++u) al[u] = w[u] >= 0 && alive[w[u]];
#pragma unroll
            for (int u = 0; u < kScanUnroll; ++u) mt[u] = al[u] ? prev.meta[w[u]] : 0u;
#pragma unroll
            for (int u = 0; u < kScanUnroll; ++u) {
                const int32_t p = p0 + u * bs;
                if (w[u] < 0) continue;
                bytes += 5;
                if (!small) cursor[p] = 0;
                if (!al[u]) continue;
                bytes += 4;
                const int kw = meta_k(mt[u]);
                const int sz = meta_size(mt[u]);
                atomicAdd(&hk[kw], 1);
                kmax_l = kw > kmax_l ? kw : kmax_l;
                if (sz > 0) {
                    const int hr = meta_head(mt[u]);
                    htop_l = hr > htop_l ? hr : htop_l;
                    if (hub) atomicAdd(&hh[hr], 1);
                    if (small) {
                        mine.size = sz;
                        mine.off = prev.off[w[u]];
                        bytes += 8;
                    }
                }
            }
        }
        kmax_l = wave_max_i(kmax_l);
        htop_l = wave_max_i(htop_l);
        if (lane_id() == 0) {
            atomicMax(&s_kmax, kmax_l);
            atomicMax(&s_htop, htop_l);
        }
        __syncthreads();
        if (hub) {
            if (tid == 0) {
                int run = 0;
                hcum[256] = 0;
                for (int r = 255; r >= 0; --r) {
                    const int c = hh[r];
                    hh[r] = run;  // scatter cursor of head rank r
                    run += c;
                    hcum[r] = run;
                }
            }
            __syncthreads();
            for (int32_t p0 = b + tid; p0 < e; p0 += bs * kScanUnroll) {
                int32_t w[kScanUnroll];
                uint32_t mt[kScanUnroll];
#pragma unroll
                for (int u = 0; u < kScanUnroll; ++u) {
                    const int32_t p = p0 + u * bs;
                    w[u] = p < e ? col[p] : -1;
                }
#pragma unroll
                for (int u = 0; u < kScanUnroll; ++u) mt[u] = (w[u] >= 0 && alive[w[u]]) ? prev.meta[w[u]] : 0u;
#pragma unroll
                for (int u = 0; u < kScanUnroll; ++u)
                    if (meta_size(mt[u]) > 0) order[b + atomicAdd(&hh[meta_head(mt[u])], 1)] = p0 + u * bs;
            }
            bytes += tid == 0 ? 9ull * (unsigned long long)deg : 0ull;
            __syncthreads();
        }
        const int kmax = s_kmax;
        const int htop = s_htop;
        const int rv = rank[v];
        int k = kmax;
        // first pass: every rank >= lo0 at once (the old level on a recomputation)
        const int lo0 = (changed && s_ok >= kmax && s_ok <= htop) ? s_ok : htop + 1;
        if (lo0 <= htop) {
            if (tid == 0 && rv >= lo0) hs_insert(H, sample_key(rv, v));
            if (small) {
                const int start = mine.cur;
                const int len = arc_run(prev.keys + mine.off, mine, lo0, bytes);
                insert_runs<BS>(len, mine.off + start, prev, H, M, s_offs, s_seg, s_scan, elems, bytes);
            } else {
                union_pass_wide<BS>(lo0, b, hub ? hcum[lo0] : deg, hub, order, col, alive, prev, cursor, H, M, s_offs,
                                s_seg, s_scan, elems, bytes);
            }
        }
        // then one rank at a time down to kmax, stopping once more than M are in
        for (int L = min(lo0 - 1, htop); L >= kmax; --L) {
            if (tid == 0 && rv == L && *(volatile int*)&s_count <= M) hs_insert(H, sample_key(L, v));
            if (small) {
                const int start = mine.cur;
                const int len = arc_run(prev.keys + mine.off, mine, L, bytes);
                insert_runs<BS>(len, mine.off + start, prev, H, M, s_offs, s_seg, s_scan, elems, bytes);
            } else {
                union_pass_wide<BS>(L, b, hub ? hcum[L] : deg, hub, order, col, alive, prev, cursor, H, M, s_offs,
                                s_seg, s_scan, elems, bytes);
            }
            const int over = s_count > M;
            __syncthreads();
            if (over) {
                k = L + 1;
                break;
            }
        }
        if (tid == 0) {
            // no key ranks above htop (it bounds r[v] and every list head)
            int run = 0, hr = 0;
            for (int L = htop; L >= k; --L) {
                const int c = hist[L];
                if (c > 0 && run == 0) hr = L;
                hist[L] = run;
                run += c;
            }
            s_k = k;
            s_size = run;
            s_head = hr;
        }
        __syncthreads();
        if (slot >= 0) {
            // a slice: its partial list (entries of rank >= its level, grouped by
            // rank), its level, largest neighbour level, head and level histogram
            uint32_t* pout = sp.pkeys + (size_t)slot * sp.pcap;
            for (int t = tid; t < hcap; t += bs) {
                const uint32_t key = tab[t];
                if (key != kEmptyKey) {
                    const int rk = key_rank(key);
                    if (rk >= k) pout[atomicAdd(&hist[rk], 1)] = key;
                }
            }
            for (int t = tid; t < 256; t += bs) sp.phk[(size_t)slot * 256 + t] = hk[t];
            if (tid == 0) {
                bytes += 4ull * (unsigned long long)s_size + 1040;
                sp.pmeta[4 * slot + 0] = s_size;
                sp.pmeta[4 * slot + 1] = s_k;
                sp.pmeta[4 * slot + 2] = kmax;
                sp.pmeta[4 * slot + 3] = s_size > 0 ? s_head : -1;
            }
            __syncthreads();
            continue;
        }
        const bool chg = changed && (s_ok != s_k || s_os != s_size);
        uint32_t* out = keys_at(cur, v);
        if (chg) {
            // members of the old list that are not in the new one (the old list is
            // still in place: every old member has rank >= old k >= new k, so it is
            // in the table exactly when it is still in the list)
            int lm = -1;
            for (int t = tid; t < s_os; t += bs) {
                const uint32_t key = out[t];
                if (!hs_contains(H, key)) lm = max(lm, key_rank(key));
            }
            if (tid == 0) bytes += 4ull * (unsigned long long)s_os;
            lm = wave_max_i(lm);
            if (lane_id() == 0 && lm >= 0) atomicMax(&s_lost, lm);
            __syncthreads();
        }
        for (int t = tid; t < hcap; t += bs) {
            const uint32_t key = tab[t];
            if (key != kEmptyKey) {
                const int rk = key_rank(key);
                if (rk >= k) out[atomicAdd(&hist[rk], 1)] = key;
            }
        }
        if (tid == 0) {
            bytes += 4ull * (unsigned long long)s_size + 17;
            cur.size[v] = s_size;
            cur.k[v] = (uint8_t)s_k;
            cur.meta[v] = pack_meta(s_size, s_k, s_head);
            cur.m[v] = hk[s_k];
            cur.cut[v] = s_k > kmax ? 1 : 0;
            if (chg) {
                cur.lost[v] = (int16_t)s_lost;
                cur.kold[v] = (uint8_t)s_ok;
                changed[atomicAdd(changed_count, 1)] = v;
            }
        }
        __syncthreads();
    }
    elems = (unsigned long long)wave_sum_ll((long long)elems);
    bytes = (unsigned long long)wave_sum_ll((long long)bytes);
    if (lane_id() == 0) {
        if (elems) atomicAdd(&st->elems, elems);
        if (bytes) atomicAdd(&st->union_bytes, bytes);
    }
}

// Work items of the hub launch: every hub of the list whole, or (more than
// sp.slice arcs) as slices of at least sp.slice arcs, at most kMergeThreads of
// them, each with a partial-list slot; a split hub is also listed for the merge.
constexpr int kMergeThreads = 256;

__global__ void k_hub_units(const int32_t* __restrict__ hubs, const int* hub_count, const int32_t* __restrict__ rp,
                            HubSplit sp, RoundState* st) {
    const int total = *hub_count;
    const int stride = gridDim.x * blockDim.x;
    for (int base = blockIdx.x * blockDim.x; base < total; base += stride) {
        const int i = base + threadIdx.x;
        int32_t v = 0, b = 0, e = 0, sl = 1;
        int ns = 0;
        if (i < total) {
            v = hubs[i];
            b = rp[v];
            e = rp[v + 1];
            const int32_t deg = e - b;
            sl = max(sp.slice, (deg + kMergeThreads - 1) / kMergeThreads);
            ns = (deg + sl - 1) / sl;
        }
        // slots (split hubs), then work items, one atomic per wave each
        const int nslot = ns > 1 ? ns : 0;
        const int si = wave_incl_scan(nslot);
        int sb = 0;
        if (lane_id() == 63 && si > 0) sb = atomicAdd(&st->slot_count, si);
        sb = __shfl(sb, 63);
        int q0 = sb + si - nslot;
        // the slots are sized for every split the hubs of a graph can need; a
        // hub that found none left is merged whole
        const bool split = nslot > 0 && q0 + nslot <= sp.slot_cap;
        const int nunit = i < total ? (split ? ns : 1) : 0;
        const int ui = wave_incl_scan(nunit);
        int ub = 0;
        if (lane_id() == 63 && ui > 0) ub = atomicAdd(&st->unit_count, ui);
        ub = __shfl(ub, 63);
        const int u0 = ub + ui - nunit;
        if (i < total) {
            if (split) {
                for (int j = 0; j < ns; ++j) sp.unit[u0 + j] = make_int4(v, b + j * sl, min(e, b + (j + 1) * sl), q0 + j);
            } else {
                sp.unit[u0] = make_int4(v, b, e, -1);
            }
        }
        const int gs = wave_append_slot(split, &st->giant_count);
        if (split) sp.giant[gs] = make_int4(v, q0, ns, 0);
    }
}

// The merge of a split hub: its slices' partial lists stand for the neighbours'
// lists.  Above F, the largest level of a slice, every partial list holds all of
// its slice's entries, and the hub's level is at least F (each slice's entries
// are a subset of the hub's, and the neighbour levels bound both), so the walk
// from the top stops at F.  m counts the neighbours at the final level from the
// slices' histograms; the cut flag compares with the largest neighbour level.
template <int BS>
__global__ __launch_bounds__(BS) void k_union_merge(const int* giant_count, const uint8_t* __restrict__ alive,
                                                     const uint8_t* __restrict__ rank, int32_t M0,
                                                     const int32_t* __restrict__ Mv, int hash_log2, LevelView cur,
                                                     int32_t* __restrict__ changed, int* changed_count,
                                                     RoundState* st, HubSplit sp) {
    extern __shared__ uint32_t tab[];
    __shared__ int hist[256];
    __shared__ int s_offs[BS], s_scan[BS / 64];
    __shared__ long long s_seg[BS];
    __shared__ int s_kmax, s_floor, s_htop, s_count, s_k, s_size, s_ok, s_os, s_lost, s_head, s_m;
    const int tid = threadIdx.x;
    const int bs = blockDim.x;
    const int hcap = 1 << hash_log2;
    HashSet H{tab, (uint32_t)(hcap - 1), 32 - hash_log2, &s_count, hist, M0};
    LevelView pv{};
    pv.keys = sp.pkeys;
    const int total = *giant_count;
    unsigned long long elems = 0, bytes = 0;
    for (int gi = blockIdx.x; gi < total; gi += gridDim.x) {
        const int4 G = sp.giant[gi];
        const int32_t v = G.x;
        if (!alive[v]) continue;
        const int M = Mv ? Mv[v] : M0;
        H.M = M;
        const int ns = G.z;
        for (int t = tid; t < hcap; t += bs) tab[t] = kEmptyKey;
        if (tid < 256) hist[tid] = 0;
        if (tid == 0) {
            s_kmax = 0;
            s_floor = 0;
            s_htop = rank[v];
            s_count = 0;
            s_m = 0;
            s_ok = cur.k[v];
            s_os = cur.size[v];
            s_lost = -1;
            bytes += 16 + 6;  // work item, rank/alive/old state of v
        }
        __syncthreads();
        ArcState mine{0, 0, 0};
        int kmax_l = 0, floor_l = 0, htop_l = -1;
        if (tid < ns) {
            const int q = G.y + tid;
            mine.size = sp.pmeta[4 * q + 0];
            mine.off = (int64_t)q * sp.pcap;
            floor_l = sp.pmeta[4 * q + 1];
            kmax_l = sp.pmeta[4 * q + 2];
            if (mine.size > 0) htop_l = sp.pmeta[4 * q + 3];
            bytes += 16;
        }
        kmax_l = wave_max_i(kmax_l);
        floor_l = wave_max_i(floor_l);
        htop_l = wave_max_i(htop_l);
        if (lane_id() == 0) {
            atomicMax(&s_kmax, kmax_l);
            atomicMax(&s_floor, floor_l);
            atomicMax(&s_htop, htop_l);
        }
        __syncthreads();
        const int kmax = s_kmax;
        const int F = s_floor;
        const int htop = s_htop;
        const int rv = rank[v];
        int k = F;
        const int lo0 = (changed && s_ok >= F && s_ok <= htop) ? s_ok : htop + 1;
        if (lo0 <= htop) {
            if (tid == 0 && rv >= lo0) hs_insert(H, sample_key(rv, v));
            const int start = mine.cur;
            const int len = arc_run(sp.pkeys + mine.off, mine, lo0, bytes);
            insert_runs<BS>(len, mine.off + start, pv, H, M, s_offs, s_seg, s_scan, elems, bytes);
        }
        for (int L = min(lo0 - 1, htop); L >= F; --L) {
            if (tid == 0 && rv == L && *(volatile int*)&s_count <= M) hs_insert(H, sample_key(L, v));
            const int start = mine.cur;
            const int len = arc_run(sp.pkeys + mine.off, mine, L, bytes);
            insert_runs<BS>(len, mine.off + start, pv, H, M, s_offs, s_seg, s_scan, elems, bytes);
            const int over = s_count > M;
            __syncthreads();
            if (over) {
                k = L + 1;
                break;
            }
        }
        if (tid == 0) {
            // no key ranks above htop (it bounds r[v] and every list head)
            int run = 0, hr = 0;
            for (int L = htop; L >= k; --L) {
                const int c = hist[L];
                if (c > 0 && run == 0) hr = L;
                hist[L] = run;
                run += c;
            }
            s_k = k;
            s_size = run;
            s_head = hr;
        }
        __syncthreads();
        // m: alive neighbours at the final level, summed over the slices
        int mc = tid < ns ? sp.phk[(size_t)(G.y + tid) * 256 + s_k] : 0;
        mc = wave_sum_i(mc);
        if (lane_id() == 0 && mc) atomicAdd(&s_m, mc);
        const bool chg = changed && (s_ok != s_k || s_os != s_size);
        uint32_t* out = keys_at(cur, v);
        if (chg) {
            int lm = -1;
            for (int t = tid; t < s_os; t += bs) {
                const uint32_t key = out[t];
                if (!hs_contains(H, key)) lm = max(lm, key_rank(key));
            }
            if (tid == 0) bytes += 4ull * (unsigned long long)s_os;
            lm = wave_max_i(lm);
            if (lane_id() == 0 && lm >= 0) atomicMax(&s_lost, lm);
        }
        __syncthreads();
        for (int t = tid; t < hcap; t += bs) {
            const uint32_t key = tab[t];
            if (key != kEmptyKey) {
                const int rk = key_rank(key);
                if (rk >= k) out[atomicAdd(&hist[rk], 1)] = key;
            }
        }
        if (tid == 0) {
            bytes += 4ull * (unsigned long long)s_size + 4ull * ns + 17;
            cur.size[v] = s_size;
            cur.k[v] = (uint8_t)s_k;
            cur.meta[v] = pack_meta(s_size, s_k, s_head);
            cur.m[v] = s_m;
            cur.cut[v] = s_k > kmax ? 1 : 0;
            if (chg) {
                cur.lost[v] = (int16_t)s_lost;
                cur.kold[v] = (uint8_t)s_ok;
                changed[atomicAdd(changed_count, 1)] = v;
            }
        }
        __syncthreads();
    }
    elems = (unsigned long long)wave_sum_ll((long long)elems);
    bytes = (unsigned long long)wave_sum_ll((long long)bytes);
    if (lane_id() == 0) {
        if (elems) atomicAdd(&st->elems, elems);
        if (bytes) atomicAdd(&st->union_bytes, bytes);
    }
}

void launch_union(const int32_t* worklist, const int* wl_count, int32_t n, const int32_t* rp, const int32_t* col,
                  const uint8_t* alive, const uint8_t* rank, int32_t M, const int32_t* Mv, int hash_log2,
                  LevelView prev, LevelView cur, int32_t* cursor, int32_t* order, int32_t* changed,
                  int* changed_count, RoundState* st, hipStream_t s, PullTimer* timer, const int32_t* hubs,
                  const int* hub_count, const HubSplit* split, const int32_t* smalls, const int* small_count,
                  int hash_log2_small) {
    if (n <= 0) return;
    const int grid = worklist ? 4096 : grid_for(n, 1, 16384);
    const size_t lds = sizeof(uint32_t) << hash_log2;
    // The dynamic-LDS limit of both union kernels is raised (never lowered),
    // per device, under a lock: contexts on several threads launch with
    // different hash sizes.
    static std::mutex lds_lock;
    static size_t lds_set[kMaxDevices] = {};
    int dev = 0;
    (void)hipGetDevice(&dev);
    if (lds > 65536 && dev >= 0 && dev < kMaxDevices) {
        std::lock_guard<std::mutex> g(lds_lock);
        if (lds > lds_set[dev]) {
            (void)hipFuncSetAttribute((const void*)k_union<kUnionThreads>,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            (void)hipFuncSetAttribute((const void*)k_union<kUnionHubThreads>,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            (void)hipFuncSetAttribute((const void*)k_union_merge<kMergeThreads>,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            (void)hipFuncSetAttribute((const void*)k_union<kUnionSmall>,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            lds_set[dev] = lds;
        }
    }
    const bool timed = timer && timer->used < timer->cap;
    if (timed) (void)hipEventRecord(timer->ev[2 * timer->used], s);
    const HubSplit none{};
    // vertices of at most kUnionSmall neighbours: one wave each, a hash table
    // sized for that block width
    if (smalls)
        hipLaunchKernelGGL(k_union<kUnionSmall>, dim3(8192), dim3(kUnionSmall), sizeof(uint32_t) << hash_log2_small, s,
                           smalls, small_count, n, rp, col, alive, rank, M, Mv, hash_log2_small, prev, cur, cursor,
                           order, changed, changed_count, st, none);
    hipLaunchKernelGGL(k_union<kUnionThreads>, dim3(grid), dim3(kUnionThreads), lds, s, worklist, wl_count, n, rp, col,
                       alive, rank, M, Mv, hash_log2, prev, cur, cursor, order, changed, changed_count, st, none);
    // hubs of the worklist: wider blocks for their neighbour walks; split into
    // slices merged in parallel, then merged per hub, when splitting is on
    if (hubs && split && split->slice > 0) {
        hipLaunchKernelGGL(k_hub_units, dim3(8), dim3(256), 0, s, hubs, hub_count, rp, *split, st);
        hipLaunchKernelGGL(k_union<kUnionHubThreads>, dim3(512), dim3(kUnionHubThreads), lds, s, hubs,
                           &st->unit_count, n, rp, col, alive, rank, M, Mv, hash_log2, prev, cur, cursor, order,
                           changed, changed_count, st, *split);
        hipLaunchKernelGGL(k_union_merge<kMergeThreads>, dim3(256), dim3(kMergeThreads), lds, s, &st->giant_count,
                           alive, rank, M, Mv, hash_log2, cur, changed, changed_count, st, *split);
    } else if (hubs) {
        hipLaunchKernelGGL(k_union<kUnionHubThreads>, dim3(512), dim3(kUnionHubThreads), lds, s, hubs, hub_count, n,
                           rp, col, alive, rank, M, Mv, hash_log2, prev, cur, cursor, order, changed, changed_count,
                           st, none);
    }
    if (timed) {
        (void)hipEventRecord(timer->ev[2 * timer->used + 1], s);
        timer->used += 1;
    }
}

// ---- propagation of deletions and changes to the next level ---------------------------------
// For an arc w -> v with v alive and w deleted or changed at level i-1:
//   * every member B[w,i-1] lost (all of it when w was deleted) may leave
//     B[v,i]; the highest such rank goes into lostmax[v];
//   * if k[w,i-1] was equal to k[v,i] and w was deleted or its level dropped,
//     m[v,i] loses one (the paper's m counter, Sec. 5).
__global__ void k_expand_lists(const int32_t* __restrict__ qv, const int32_t* __restrict__ qb, const int* qcount,
                               const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                               const uint8_t* __restrict__ alive, const uint8_t* __restrict__ rank,
                               int32_t* __restrict__ mark, int32_t epoch, int level, LevelView prev, LevelView cur,
                               int32_t* __restrict__ lostmax, int32_t* __restrict__ out, int* out_count,
                               RoundState* st) {
    if (epoch < 0) epoch = st->epoch;
    const int nq = *qcount;
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int nwaves = (gridDim.x * blockDim.x) >> 6;
    const int l = lane_id();
    for (int q = wave; q < nq; q += nwaves) {
        const int32_t w = qv[q];
        const int32_t b = qb[q];
        const int32_t e = min(b + kExpandChunk, rp[w + 1]);
        const bool removed = !alive[w];
        int lw, kw_old, kw_new;
        if (level == 1) {
            lw = rank[w];  // B[w,0] = {w}; only deleted vertices reach level 1
            kw_old = kw_new = 0;
        } else if (removed) {
            const uint32_t mt = prev.meta[w];
            lw = meta_size(mt) > 0 ? meta_head(mt) : -1;
            kw_old = kw_new = meta_k(mt);
        } else {
            lw = prev.lost[w];
            kw_old = prev.kold[w];
            kw_new = prev.k[w];
        }
        const bool dec_any = removed || kw_new < kw_old;
        for (int32_t p0 = b; p0 < e; p0 += 64) {
            const int32_t p = p0 + l;
            bool want = false;
            int32_t v = 0;
            if (p < e) {
                v = col[p];
                if (alive[v]) {
                    if (lw >= 0 && lostmax[v] < lw) atomicMax(&lostmax[v], lw);
                    if (dec_any && cur.k[v] == kw_old) atomicSub(&cur.m[v], 1);
                    if (mark[v] != epoch) want = atomicExch(&mark[v], epoch) != epoch;
                }
            }
            const int slot = wave_append_slot(want, out_count);
            if (want) out[slot] = v;
        }
    }
}
void launch_expand_lists(const int32_t* qv, const int32_t* qb, const int* qcount, const int32_t* rp,
                         const int32_t* col, const uint8_t* alive, const uint8_t* rank, int32_t* mark, int32_t epoch,
                         int level, LevelView prev, LevelView cur, int32_t* lostmax, int32_t* out, int* out_count,
                         RoundState* st, hipStream_t s) {
    hipLaunchKernelGGL(k_expand_lists, dim3(2048), dim3(256), 0, s, qv, qb, qcount, rp, col, alive, rank, mark, epoch,
                       level, prev, cur, lostmax, out, out_count, st);
}

// A list can only change when (cut) a member of rank >= k-1 left some input
// list -- otherwise |N(v;i)| at ranks >= k-1 still exceeds M, k stays and no
// member left; or (not cut, m > 0) a member of rank >= k left -- k cannot drop
// while a neighbour sits at level k; or (not cut, m = 0) always.
__global__ void k_classify(const int32_t* __restrict__ wl, const int* wl_count, LevelView cur,
                           int32_t* __restrict__ lostmax, int32_t* __restrict__ rc, int* rc_count,
                           const int32_t* __restrict__ rp, int32_t* __restrict__ hubs, int* hub_count,
                           const uint8_t* __restrict__ active, int32_t* __restrict__ smalls, int* small_count) {
    const int total = *wl_count;
    const int stride = gridDim.x * blockDim.x;
    for (int base = blockIdx.x * blockDim.x; base < total; base += stride) {
        const int i = base + threadIdx.x;
        bool need = false;
        int32_t v = 0;
        if (i < total) {
            v = wl[i];
            if (!active || active[v]) {
                // (inactive vertices of a lazily initialised level get a new bound instead)
                const int k = cur.k[v];
                const int L = lostmax[v];
                lostmax[v] = -1;
                if (cur.cut[v]) need = L >= k - 1;
                else if (cur.m[v] > 0) need = L >= k;
                else need = true;
            }
        }
        const int32_t deg = need && (hubs || smalls) ? rp[v + 1] - rp[v] : 0;
        const bool hub = need && hubs && deg > kHubDegree;
        const bool sm = need && smalls && deg <= kUnionSmall;
        const bool mid = need && !hub && !sm;
        const int slot = wave_append_slot(mid, rc_count);
        if (mid) rc[slot] = v;
        const int hs = wave_append_slot(hub, hub_count);
        if (hub) hubs[hs] = v;
        const int ss = wave_append_slot(sm, small_count);
        if (sm) smalls[ss] = v;
    }
}
void launch_classify(const int32_t* wl, const int* wl_count, LevelView cur, int32_t* lostmax, int32_t* rc,
                     int* rc_count, hipStream_t s, const int32_t* rp, int32_t* hubs, int* hub_count,
                     const uint8_t* active, int32_t* smalls, int* small_count) {
    hipLaunchKernelGGL(k_classify, dim3(1024), dim3(256), 0, s, wl, wl_count, cur, lostmax, rc, rc_count, rp, hubs,
                       hub_count, active, smalls, small_count);
}

// ---- lazy initialisation of the top level (Sec. 5, first heuristic) ---------------------
// For alive v and an alive neighbour w, Y = N(w; h-1, X) lies inside N(v; h, X)
// and contains v, so by Prop. monotone the estimate of the rank list
// (r[v], ranks of Y \ {v}) is at most d(v).  Its level is k[w,h-1] (the
// smallest k with |Y_{r>=k}| <= M, the closed form of the level) and its count
// at that level is |B[w,h-1]| - [r[v] >= k[w,h-1]].  The largest such value over
// the alive neighbours is a lower bound on d(v) that needs no list of v's own:
// B[v,h] is built only once that bound no longer keeps v above the running
// maximum.  Written to d[v] for the inactive vertices of the list (all
// vertices when list == NULL); lostmax[v] is reset for them.
__global__ void k_lazy_lb(const int32_t* __restrict__ list, const int* count, int32_t n,
                          const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                          const uint8_t* __restrict__ alive, const uint8_t* __restrict__ active,
                          const uint8_t* __restrict__ rank, int32_t M0, const int32_t* __restrict__ Mv,
                          LevelView prev, int64_t* __restrict__ d, int32_t* __restrict__ lostmax) {
    const int total = list ? *count : n;
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int nwaves = (gridDim.x * blockDim.x) >> 6;
    const int l = lane_id();
    for (int i = wave; i < total; i += nwaves) {
        const int32_t v = list ? list[i] : i;
        if (!alive[v] || active[v]) continue;
        const long long M = Mv ? Mv[v] : M0;
        const int rv = rank[v];
        long long lb = 0;
        for (int32_t p = rp[v] + l; p < rp[v + 1]; p += 64) {
            const int32_t w = col[p];
            if (!alive[w]) continue;
            const uint32_t mt = prev.meta[w];
            const int k = (int)((mt >> 16) & 0xFFu);
            const long long T = (long long)(mt & 0xFFFFu) - (rv >= k ? 1 : 0);
            // levels this high only make the bound smaller than it could be: still a bound
            const int kk = k < 40 ? k : 40;
            long long e = T << kk;
            if (kk > 0) {
                const long long fl = M << (kk - 1);
                e = fl > e ? fl : e;
            }
            lb = e > lb ? e : lb;
        }
        for (int o = 32; o > 0; o >>= 1) {
            const long long t = __shfl_xor(lb, o);
            lb = t > lb ? t : lb;
        }
        if (l == 0) {
            d[v] = lb;
            lostmax[v] = -1;
        }
    }
}
void launch_lazy_lb(const int32_t* list, const int* count, int32_t n, const int32_t* rp, const int32_t* col,
                    const uint8_t* alive, const uint8_t* active, const uint8_t* rank, int32_t M, const int32_t* Mv,
                    LevelView prev, int64_t* d, int32_t* lostmax, hipStream_t s) {
    if (n <= 0) return;
    const int grid = list ? 1024 : grid_for((int64_t)n * 64, 256, 16384);
    hipLaunchKernelGGL(k_lazy_lb, dim3(grid), dim3(256), 0, s, list, count, n, rp, col, alive, active, rank, M, Mv,
                       prev, d, lostmax);
}

// Activation round: when some inactive bound is at or below c' = max(c, min d),
// the round stalls (no deletion) and every inactive vertex with bound <= 2 c' + 64
// becomes active; its top-level list is then built from scratch.  (Activating
// early only costs list upkeep; the slack keeps the number of stalled rounds
// near the number of doublings of c instead of one per distinct bound.)
__global__ void k_lazy_decide(RoundState* st) {
    if (st->alive_count == 0) {
        st->stall = 0;
        return;
    }
    const long long c = st->min_key > st->c ? st->min_key : st->c;
    st->stall = st->min_inexact <= c ? 1 : 0;
    st->hi = c > (1ll << 60) ? c : 2 * c + 64;
    st->rc_count = 0;
}
void launch_lazy_decide(RoundState* st, hipStream_t s) { hipLaunchKernelGGL(k_lazy_decide, dim3(1), dim3(1), 0, s, st); }

__global__ void k_lazy_pick(const uint8_t* __restrict__ alive, uint8_t* __restrict__ active,
                            const int64_t* __restrict__ d, int32_t n, RoundState* st, int32_t* __restrict__ out) {
    if (!st->stall) return;
    const long long hi = st->hi;
    const int32_t stride = gridDim.x * blockDim.x;
    for (int32_t base = blockIdx.x * blockDim.x; base < n; base += stride) {
        const int32_t v = base + threadIdx.x;
        const bool take = v < n && alive[v] && !active[v] && d[v] <= hi;
        const int slot = wave_append_slot(take, &st->rc_count);
        if (take) {
            out[slot] = v;
            active[v] = 1;
        }
    }
}
void launch_lazy_pick(const uint8_t* alive, uint8_t* active, const int64_t* d, int32_t n, RoundState* st,
                      int32_t* out, hipStream_t s) {
    if (n > 0)
        hipLaunchKernelGGL(k_lazy_pick, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, alive, active, d, n, st, out);
}

// ---- Alg. 1: d = |B[v,h] \ {v}| 2^k, and max(d, M 2^(k-1)) when k > 0 ---------------------------
__global__ void k_estimate(const int32_t* __restrict__ worklist, const int* wl_count, int32_t n,
                           const uint8_t* __restrict__ alive, const uint8_t* __restrict__ rank,
                           const int32_t* __restrict__ size, const uint8_t* __restrict__ kk, int32_t M0,
                           const int32_t* __restrict__ Mv, int64_t* __restrict__ d, RoundState* st) {
    const int total = worklist ? *wl_count : n;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
        const int32_t v = worklist ? worklist[i] : i;
        if (!alive[v]) continue;
        const int k = kk[v];
        const long long M = Mv ? Mv[v] : M0;
        const long long T = (long long)size[v] - (rank[v] >= k ? 1 : 0);
        long long est;
        if (k >= 62 || (T > 0 && T > (LLONG_MAX >> k))) {
            atomicOr(&st->overflow, 1);
            est = LLONG_MAX;
        } else {
            est = T << k;
            if (k > 0) {
                const long long fl = M << (k - 1);
                est = fl > est ? fl : est;
            }
        }
        d[v] = est;
    }
}
void launch_estimate(const int32_t* worklist, const int* wl_count, int32_t n, const uint8_t* alive,
                     const uint8_t* rank, const int32_t* size, const uint8_t* kk, int32_t M, const int32_t* Mv,
                     int64_t* d, RoundState* st, hipStream_t s) {
    if (n <= 0) return;
    const int grid = worklist ? 1024 : grid_for(n, 256, 8192);
    hipLaunchKernelGGL(k_estimate, dim3(grid), dim3(256), 0, s, worklist, wl_count, n, alive, rank, size, kk, M, Mv,
                       d, st);
}

}  // namespace kh
