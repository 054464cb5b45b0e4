// Graph residency, ranks and the bulk-peeling bookkeeping kernels (gfx950, wave64).
//
// Peeling follows the paper's deletion loop (ExactCore, Sec. 2; Core, Alg. 4):
// the running maximum c of the minimum key is the core number.  Deleting every
// vertex whose key is <= c in one round gives the same numbers as deleting one
// minimum at a time, because the key of a vertex only depends on the vertex and
// the remaining set and never grows when vertices are removed (for the exact
// degree by inclusion of neighbourhoods, for the estimate by Prop. monotone).
#include <climits>

#include "kh_common.hpp"
#include "kh_internal.hpp"

namespace kh {

// ---- ranks (Sec. 3: r[v] ~ geometric(1/2), ties allowed) -----------------------------
// SplitMix64's mixer (Steele, Lea, Flood, OOPSLA 2014); the rank counts the zero
// bits before the first one bit of the word stream w_j = sm(sm(sm(seed)^v) ^ (sid<<32 | j)).
__device__ __forceinline__ uint64_t sm64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ void k_ranks(uint8_t* __restrict__ r, int32_t n, uint64_t seed, uint32_t sid,
                        const int32_t* __restrict__ lid) {
    const uint64_t s0 = sm64(seed);
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        const int64_t id = lid ? lid[v] : v;
        const uint64_t base = sm64(s0 ^ (uint64_t)id);
        int rank = 0;
        int j = 0;
        for (; j < 4; ++j) {
            const uint64_t w = sm64(base ^ (((uint64_t)sid << 32) | (uint64_t)j));
            if (w != 0ull) {
                rank += __builtin_ctzll(w);
                break;
            }
            rank += 64;
        }
        r[v] = (uint8_t)(rank > 255 ? 255 : rank);
    }
}

void launch_ranks(uint8_t* r, int32_t n, uint64_t seed, uint32_t sid, hipStream_t s, const int32_t* lid) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_ranks, dim3(grid_for(n, 256, 16384)), dim3(256), 0, s, r, n, seed, sid, lid);
}

// ---- packing many graphs into one disjoint union ------------------------------------------
__global__ void k_pack_col(int32_t count, const int64_t* __restrict__ a_off, const int32_t* __restrict__ v_off,
                           const uint64_t* __restrict__ col_ptrs, int64_t nnz, int32_t* __restrict__ col) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nnz; i += (int64_t)gridDim.x * blockDim.x) {
        // graph of arc i: last g with a_off[g] <= i
        int lo = 0, hi = count - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (a_off[mid] <= i) lo = mid; else hi = mid - 1;
        }
        const int32_t* src = reinterpret_cast<const int32_t*>(col_ptrs[lo]);
        col[i] = src[i - a_off[lo]] + v_off[lo];
    }
}
void launch_pack_col(int32_t count, const int64_t* a_off, const int32_t* v_off, const uint64_t* col_ptrs,
                     int64_t nnz, int32_t* col, hipStream_t s) {
    if (nnz > 0 && count > 0)
        hipLaunchKernelGGL(k_pack_col, dim3(grid_for(nnz, 256, 16384)), dim3(256), 0, s, count, a_off, v_off,
                           col_ptrs, nnz, col);
}

// dst_ptrs[g][i - v_off[g]] = src[i] for the vertices i of graph g
__global__ void k_unpack_i32(int32_t count, const int32_t* __restrict__ v_off, const uint64_t* __restrict__ dst_ptrs,
                             int32_t total, const int32_t* __restrict__ src) {
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
        int lo = 0, hi = count - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (v_off[mid] <= i) lo = mid; else hi = mid - 1;
        }
        reinterpret_cast<int32_t*>(dst_ptrs[lo])[i - v_off[lo]] = src[i];
    }
}
void launch_unpack_i32(int32_t count, const int32_t* v_off, const uint64_t* dst_ptrs, int32_t total,
                       const int32_t* src, hipStream_t s) {
    if (total > 0 && count > 0)
        hipLaunchKernelGGL(k_unpack_i32, dim3(grid_for(total, 256, 16384)), dim3(256), 0, s, count, v_off, dst_ptrs,
                           total, src);
}

// ---- CSR validation on the device (simple undirected graph, Sec. 2) ---------------------
// err bits: 1 row_ptr, 2 id out of range, 4 self-loop, 8 unsorted/duplicate, 16 asymmetric.
__global__ void k_validate(const int32_t* __restrict__ rp, const int32_t* __restrict__ col, int32_t n, int64_t nnz,
                           int* err) {
    const int lanes = 64;
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) / lanes;
    const int nwaves = gridDim.x * blockDim.x / lanes;
    const int l = lane_id();
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (rp[0] != 0 || (int64_t)rp[n] != nnz) atomicOr(err, 1);
    }
    for (int32_t v = wave; v < n; v += nwaves) {
        const int32_t a = rp[v], b = rp[v + 1];
        if (a > b || a < 0 || (int64_t)b > nnz) {
            if (l == 0) atomicOr(err, 1);
            continue;
        }
        int e = 0;
        for (int32_t p = a + l; p < b; p += lanes) {
            const int32_t w = col[p];
            if (w < 0 || w >= n) {
                e |= 2;
                continue;
            }
            if (w == v) e |= 4;
            if (p > a && col[p - 1] >= w) e |= 8;
            // symmetric: v must appear in the adjacency of w
            int32_t lo = rp[w], hi = rp[w + 1];
            if (lo < 0 || hi > nnz || lo > hi) {
                e |= 1;
                continue;
            }
            while (lo < hi) {
                const int32_t mid = lo + ((hi - lo) >> 1);
                if (col[mid] < v) lo = mid + 1; else hi = mid;
            }
            if (lo >= rp[w + 1] || col[lo] != v) e |= 16;
        }
        for (int o = 32; o > 0; o >>= 1) e |= __shfl_xor(e, o);
        if (l == 0 && e) atomicOr(err, e);
    }
}

void launch_validate(const int32_t* rp, const int32_t* col, int32_t n, int64_t nnz, int* err, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_validate, dim3(grid_for((int64_t)n * 64, 256, 16384)), dim3(256), 0, s, rp, col, n, nnz,
                       err);
}

// ---- fills (used instead of memset so the sequences can be graph-captured) ----------------
template <typename T>
__global__ void k_fill(T* __restrict__ p, T v, int64_t count) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
void launch_fill_i32(int32_t* p, int32_t v, int64_t count, hipStream_t s) {
    if (count > 0) hipLaunchKernelGGL(k_fill<int32_t>, dim3(grid_for(count, 256, 8192)), dim3(256), 0, s, p, v, count);
}
void launch_fill_i64(int64_t* p, int64_t v, int64_t count, hipStream_t s) {
    if (count > 0) hipLaunchKernelGGL(k_fill<int64_t>, dim3(grid_for(count, 256, 8192)), dim3(256), 0, s, p, v, count);
}

__global__ void k_alive_from(const uint8_t* __restrict__ src, uint8_t* __restrict__ alive, int32_t n) {
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
        alive[v] = src ? (src[v] != 0) : 1;
}
void launch_alive_from(const uint8_t* src, uint8_t* alive, int32_t n, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_alive_from, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, src, alive, n);
}

// Alive degree |A(v) ∩ X| (one wave per vertex).
__global__ void k_alive_degree(const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                               const uint8_t* __restrict__ alive, int32_t* __restrict__ adeg, int32_t n) {
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int nwaves = (gridDim.x * blockDim.x) >> 6;
    const int l = lane_id();
    for (int32_t v = wave; v < n; v += nwaves) {
        int c = 0;
        if (alive[v]) {
            for (int32_t p = rp[v] + l; p < rp[v + 1]; p += 64) c += alive[col[p]] ? 1 : 0;
            c = wave_sum_i(c);
        }
        if (l == 0) adeg[v] = c;
    }
}
void launch_alive_degree(const int32_t* rp, const int32_t* col, const uint8_t* alive, int32_t* adeg, int32_t n,
                         hipStream_t s) {
    if (n > 0)
        hipLaunchKernelGGL(k_alive_degree, dim3(grid_for((int64_t)n * 64, 256, 16384)), dim3(256), 0, s, rp, col,
                           alive, adeg, n);
}

__global__ void k_compact_alive(const uint8_t* __restrict__ alive, int32_t n, int32_t* __restrict__ out, int* count) {
    const int32_t stride = gridDim.x * blockDim.x;
    // every lane of a wave runs the same trip count so the ballot is wave-wide
    for (int32_t base = blockIdx.x * blockDim.x; base < n; base += stride) {
        const int32_t v = base + threadIdx.x;
        const bool want = v < n && alive[v];
        const int slot = wave_append_slot(want, count);
        if (want) out[slot] = v;
    }
}
void launch_compact_alive(const uint8_t* alive, int32_t n, int32_t* out, int* count, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_compact_alive, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, alive, n, out, count);
}

// ---- round bookkeeping ------------------------------------------------------------------
__device__ void round_reset_fields(RoundState* st) {
    st->min_key = LLONG_MAX;
    st->min_inexact = LLONG_MAX;
    st->sum_val = 0;
    st->alive_count = 0;
    st->rcount = 0;
    st->stop = 0;
    st->qcount = 0;
    st->front_lo = 0;
    st->front_hi = 0;
    st->aff_fill = 0;
    st->wl_count = 0;
    st->changed_count[0] = 0;
    st->changed_count[1] = 0;
    st->rc_count = 0;
    st->ms_ns = 0;
    for (int b = 0; b < 48; ++b) st->hist[b] = 0;
    st->fcount[0] = 0;
    st->fcount[1] = 0;
    st->hop_arcs = 0;
    st->next_arcs = 0;
    st->epoch += 1;
    st->fepoch += 1;  // frontier marks of the mask BFS's first hop
}
__global__ void k_round_reset(RoundState* st, int gate) {
    if (gate && st->stall) return;
    round_reset_fields(st);
}
void launch_round_reset(RoundState* st, hipStream_t s, int gate) {
    hipLaunchKernelGGL(k_round_reset, dim3(1), dim3(1), 0, s, st, gate);
}

// min of key, sum of val and count over alive vertices (one atomic triple per block).
__global__ __launch_bounds__(512) void k_reduce(const int64_t* __restrict__ key, const int64_t* __restrict__ val,
                                                const uint8_t* __restrict__ alive, int32_t n, RoundState* st,
                                                int gate, const uint8_t* __restrict__ exact) {
    if (gate && st->stall) return;
    __shared__ long long smin[8], ssum[8], sinx[8];
    __shared__ int scnt[8];
    long long mn = LLONG_MAX, sm = 0, mi = LLONG_MAX;
    int cnt = 0;
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        if (alive[v]) {
            const long long k = key[v];
            mn = k < mn ? k : mn;
            sm += val ? val[v] : 0;
            ++cnt;
            if (exact && !exact[v]) mi = k < mi ? k : mi;
        }
    }
    mn = wave_min_ll(mn);
    sm = wave_sum_ll(sm);
    mi = wave_min_ll(mi);
    cnt = wave_sum_i(cnt);
    const int w = threadIdx.x >> 6;
    if (lane_id() == 0) {
        smin[w] = mn;
        ssum[w] = sm;
        sinx[w] = mi;
        scnt[w] = cnt;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < (int)(blockDim.x >> 6); ++i) {
            mn = smin[i] < mn ? smin[i] : mn;
            mi = sinx[i] < mi ? sinx[i] : mi;
            sm += ssum[i];
            cnt += scnt[i];
        }
        if (cnt > 0) {
            atomicMin(&st->min_key, mn);
            if (sm) atomicAdd((unsigned long long*)&st->sum_val, (unsigned long long)sm);
            atomicAdd(&st->alive_count, cnt);
            if (mi != LLONG_MAX) atomicMin(&st->min_inexact, mi);
        }
    }
}
void launch_reduce(const int64_t* key, const int64_t* val, const uint8_t* alive, int32_t n, RoundState* st,
                   hipStream_t s, int gate, const uint8_t* exact) {
    if (n > 0)
        hipLaunchKernelGGL(k_reduce, dim3(grid_for(n, 512, 256)), dim3(512), 0, s, key, val, alive, n, st, gate,
                           exact);
}

// c = max(c, min key).  When c rises to K, the alive set is exactly
// F_K = {v : core(v) >= K} and sum_val is the sum of the values over it: that
// is recorded as a densest-core candidate (Sec. 6).
//
// Early stop (Sec. 5 heuristic, in the Sec. 8 form c + 1 = |remaining|): tested
// right after a round's deletions, with that round's c.  When c + 1 >= |X| the
// round takes every remaining vertex at c.  Deleting in bulk gives the same
// numbers as testing after every single deletion: vertices leave in
// non-decreasing core order and the test is weakest at the end of a level.
__global__ void k_round_begin(RoundState* st, int64_t* cand_k, int64_t* cand_size, int64_t* cand_sum, int early_stop) {
    if (st->alive_count == 0 || st->stall) return;
    long long c = st->c;
    if (early_stop && st->rounds > 0 && c + 1 >= (long long)st->alive_count) {
        st->stop = 1;
        st->rounds += 1;
        return;
    }
    if (st->min_key > c) {
        c = st->min_key;
        if (cand_k) {
            const int i = st->ncand;
            cand_k[i] = c;
            cand_size[i] = st->alive_count;
            cand_sum[i] = st->sum_val;
        }
        st->ncand += 1;
    }
    st->c = c;
    st->rounds += 1;
}
void launch_round_begin(RoundState* st, int64_t* cand_k, int64_t* cand_size, int64_t* cand_sum, int early_stop,
                        hipStream_t s) {
    hipLaunchKernelGGL(k_round_begin, dim3(1), dim3(1), 0, s, st, cand_k, cand_size, cand_sum, early_stop);
}

// R = {alive v : key[v] <= c} (all alive when the early stop fired): core = c.
__global__ void k_select(const int64_t* __restrict__ key, uint8_t* __restrict__ alive, int32_t n, RoundState* st,
                         int64_t* __restrict__ core, int32_t* __restrict__ rlist, int32_t* __restrict__ mark,
                         int32_t epoch, int kill, int32_t* __restrict__ rnd) {
    if (st->stall) return;  // a lazy activation takes this round's place
    const long long c = st->c;
    const int stop = st->stop;
    const int32_t round_id = st->epoch;
    const int32_t stride = gridDim.x * blockDim.x;
    for (int32_t base = blockIdx.x * blockDim.x; base < n; base += stride) {
        const int32_t v = base + threadIdx.x;
        bool take = false;
        if (v < n && alive[v]) take = stop || key[v] <= c;
        const int slot = wave_append_slot(take, &st->rcount);
        if (take) {
            core[v] = c;
            rlist[slot] = v;
            if (mark) mark[v] = epoch;
            if (kill) alive[v] = 0;
            if (rnd) rnd[v] = round_id;
        }
    }
}
void launch_select(const int64_t* key, uint8_t* alive, int32_t n, RoundState* st, int64_t* core, int32_t* rlist,
                   int32_t* mark, int32_t epoch, int kill, hipStream_t s, int32_t* rnd) {
    if (n > 0)
        hipLaunchKernelGGL(k_select, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, key, alive, n, st, core, rlist,
                           mark, epoch, kill, rnd);
}

__global__ void k_kill_list(const int32_t* __restrict__ list, const int* count, uint8_t* __restrict__ alive) {
    const int cnt = *count;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += gridDim.x * blockDim.x) alive[list[i]] = 0;
}
void launch_kill_list(const int32_t* list, const int* count, uint8_t* alive, hipStream_t s) {
    hipLaunchKernelGGL(k_kill_list, dim3(1024), dim3(256), 0, s, list, count, alive);
}

// ---- load-balanced frontier expansion ------------------------------------------------------
// The adjacency of each listed vertex is cut into chunks of kExpandChunk arcs so
// that hubs are spread over many waves.
__global__ void k_enqueue(const int32_t* __restrict__ list, const int* lo_p, const int* hi_p,
                          const int32_t* __restrict__ rp, int32_t* __restrict__ qv, int32_t* __restrict__ qb,
                          int* qcount, long long* arcs, const RoundState* pull_st, int64_t nnz) {
    // a mask-BFS hop that pulls needs no chunk queue
    if (pull_st && nnz > 0 && pull_st->hop_arcs * (long long)pull_st->pull_ratio > nnz) return;
    const int lo = lo_p ? *lo_p : 0;
    const int hi = *hi_p;
    const int stride = gridDim.x * blockDim.x;
    for (int base = lo + blockIdx.x * blockDim.x; base < hi; base += stride) {
        const int i = base + threadIdx.x;
        int v = 0, nch = 0, d = 0;
        if (i < hi) {
            v = list[i];
            d = rp[v + 1] - rp[v];
            nch = (d + kExpandChunk - 1) / kExpandChunk;
        }
        if (arcs) {
            const long long ws = wave_sum_ll((long long)d);
            if (lane_id() == 0 && ws) atomicAdd((unsigned long long*)arcs, (unsigned long long)ws);
        }
        const int incl = wave_incl_scan(nch);
        const int total = __shfl(incl, 63);
        int wbase = 0;
        if (lane_id() == 63 && total > 0) wbase = atomicAdd(qcount, total);
        wbase = __shfl(wbase, 63);
        const int first = wbase + incl - nch;
        for (int c = 0; c < nch; ++c) {
            qv[first + c] = v;
            qb[first + c] = rp[v] + c * kExpandChunk;
        }
    }
}
void launch_enqueue(const int32_t* list, const int* lo, const int* hi, const int32_t* rp, int32_t* qv, int32_t* qb,
                    int* qcount, hipStream_t s, long long* arcs, const RoundState* pull_st, int64_t nnz, int grid) {
    hipLaunchKernelGGL(k_enqueue, dim3(grid > 0 ? grid : 128), dim3(256), 0, s, list, lo, hi, rp, qv, qb, qcount, arcs,
                       pull_st, nnz);
}

__global__ void k_enqueue_r(const int32_t* __restrict__ rlist, const int* rcount, const int32_t* __restrict__ rp,
                            int32_t* __restrict__ qv, int32_t* __restrict__ qb, int* qcount, int mode,
                            uint64_t* __restrict__ rmask, uint64_t* __restrict__ gain, uint32_t* __restrict__ fbits,
                            uint8_t* __restrict__ alive, long long* arcs) {
    const int hi = *rcount;
    const int stride = gridDim.x * blockDim.x;
    for (int base = blockIdx.x * blockDim.x; base < hi; base += stride) {
        const int i = base + threadIdx.x;
        int v = 0, nch = 0, d = 0;
        if (i < hi) {
            v = rlist[i];
            if (mode == 0) {
                const unsigned long long b = 1ull << (i & 63);
                atomicOr((unsigned long long*)&rmask[v], b);
                atomicOr((unsigned long long*)&gain[v], b);
                atomicOr(&fbits[v >> 5], 1u << (v & 31));
            } else {
                alive[v] = 0;
            }
            d = rp[v + 1] - rp[v];
            nch = (d + kExpandChunk - 1) / kExpandChunk;
        }
        if (arcs) {
            const long long ws = wave_sum_ll((long long)d);
            if (lane_id() == 0 && ws) atomicAdd((unsigned long long*)arcs, (unsigned long long)ws);
        }
        const int incl = wave_incl_scan(nch);
        const int total = __shfl(incl, 63);
        int wbase = 0;
        if (lane_id() == 63 && total > 0) wbase = atomicAdd(qcount, total);
        wbase = __shfl(wbase, 63);
        const int first = wbase + incl - nch;
        for (int c = 0; c < nch; ++c) {
            qv[first + c] = v;
            qb[first + c] = rp[v] + c * kExpandChunk;
        }
    }
}
void launch_enqueue_r(const int32_t* rlist, const int* rcount, const int32_t* rp, int32_t* qv, int32_t* qb, int* qcount,
                      int mode, uint64_t* rmask, uint64_t* gain, uint32_t* fbits, uint8_t* alive, hipStream_t s,
                      long long* arcs) {
    hipLaunchKernelGGL(k_enqueue_r, dim3(256), dim3(256), 0, s, rlist, rcount, rp, qv, qb, qcount, mode, rmask, gain,
                       fbits, alive, arcs);
}

__global__ void k_expand(const int32_t* __restrict__ qv, const int32_t* __restrict__ qb, const int* qcount,
                         const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                         const uint8_t* __restrict__ alive, int32_t* __restrict__ mark, int32_t epoch, int mode,
                         int32_t* __restrict__ out, int* out_count, int32_t* __restrict__ adeg) {
    const int nq = *qcount;
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int nwaves = (gridDim.x * blockDim.x) >> 6;
    const int l = lane_id();
    for (int q = wave; q < nq; q += nwaves) {
        const int32_t v = qv[q];
        const int32_t b = qb[q];
        const int32_t e = min(b + kExpandChunk, rp[v + 1]);
        for (int32_t p0 = b; p0 < e; p0 += 64) {
            const int32_t p = p0 + l;
            bool want = false;
            int32_t w = 0;
            if (p < e) {
                w = col[p];
                if (alive[w]) {
                    if (mode == 0) {
                        if (mark[w] != epoch) want = atomicExch(&mark[w], epoch) != epoch;
                    } else {
                        atomicSub(&adeg[w], 1);
                    }
                }
            }
            if (mode == 0) {
                const int slot = wave_append_slot(want, out_count);
                if (want) out[slot] = w;
            }
        }
    }
}
void launch_expand(const int32_t* qv, const int32_t* qb, const int* qcount, const int32_t* rp, const int32_t* col,
                   const uint8_t* alive, int32_t* mark, int32_t epoch, int mode, int32_t* out, int* out_count,
                   int32_t* adeg, hipStream_t s) {
    hipLaunchKernelGGL(k_expand, dim3(2048), dim3(256), 0, s, qv, qb, qcount, rp, col, alive, mark, epoch, mode, out,
                       out_count, adeg);
}

__global__ void k_next_frontier(RoundState* st) {
    st->front_lo = st->front_hi;
    st->front_hi = st->aff_fill;
    st->qcount = 0;
}
void launch_next_frontier(RoundState* st, hipStream_t s) {
    hipLaunchKernelGGL(k_next_frontier, dim3(1), dim3(1), 0, s, st);
}

__global__ void k_level_reset(RoundState* st, int level) {
    st->epoch += 1;
    st->qcount = 0;
    st->wl_count = 0;
    st->rc_count = 0;
    st->hub_count = 0;
    st->unit_count = 0;
    st->slot_count = 0;
    st->giant_count = 0;
    st->small_count = 0;
    st->changed_count[level & 1] = 0;
}
void launch_level_reset(RoundState* st, int level, hipStream_t s) {
    hipLaunchKernelGGL(k_level_reset, dim3(1), dim3(1), 0, s, st, level);
}

__global__ void k_set_int(int* p, int v) { *p = v; }
void launch_set_int(int* p, int v, hipStream_t s) { hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, s, p, v); }

// ---- exclusive scan of int64 values: out[0] = 0, out[i+1] = sum in[0..i] -------------------
constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

__device__ long long block_excl_scan(long long v, long long* sh, long long* total) {
    // sh holds kScanThreads/64 partial sums
    const int l = lane_id();
    const int w = threadIdx.x >> 6;
    long long x = v;
    for (int o = 1; o < 64; o <<= 1) {
        long long t = __shfl_up(x, o);
        if (l >= o) x += t;
    }
    if (l == 63) sh[w] = x;
    __syncthreads();
    long long off = 0, tot = 0;
    for (int i = 0; i < kScanThreads / 64; ++i) {
        if (i < w) off += sh[i];
        tot += sh[i];
    }
    __syncthreads();
    *total = tot;
    return off + x - v;
}

__global__ void k_scan_partials(const int64_t* __restrict__ in, int32_t n, int64_t* __restrict__ partials) {
    __shared__ long long sh[kScanThreads / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    long long s = 0;
    for (int i = 0; i < kScanItems; ++i)
        if (base + i < n) s += in[base + i];
    long long tot;
    block_excl_scan(s, sh, &tot);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}
__global__ void k_scan_top(int64_t* __restrict__ partials, int32_t nb) {
    __shared__ long long sh[kScanThreads / 64];
    long long carry = 0;
    for (int32_t b0 = 0; b0 < nb; b0 += kScanThreads) {
        const int32_t i = b0 + threadIdx.x;
        const long long v = i < nb ? partials[i] : 0;
        long long tot;
        const long long ex = block_excl_scan(v, sh, &tot);
        if (i < nb) partials[i] = carry + ex;
        carry += tot;
    }
}
__global__ void k_scan_final(const int64_t* __restrict__ in, int64_t* __restrict__ out, int32_t n,
                             const int64_t* __restrict__ partials) {
    __shared__ long long sh[kScanThreads / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    long long loc[kScanItems];
    long long s = 0;
    for (int i = 0; i < kScanItems; ++i) {
        loc[i] = base + i < n ? in[base + i] : 0;
        s += loc[i];
    }
    long long tot;
    long long ex = block_excl_scan(s, sh, &tot) + partials[blockIdx.x];
    for (int i = 0; i < kScanItems; ++i) {
        if (base + i < n) out[base + i] = ex;
        ex += loc[i];
        if (base + i == n - 1) out[n] = ex;
    }
}
void launch_scan_i64(const int64_t* in, int64_t* out, int32_t n, int64_t* partials, hipStream_t s) {
    if (n <= 0) {
        launch_fill_i64(out, 0, 1, s);
        return;
    }
    const int nb = (int)((n + kScanTile - 1) / kScanTile);
    hipLaunchKernelGGL(k_scan_partials, dim3(nb), dim3(kScanThreads), 0, s, in, n, partials);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanThreads), 0, s, partials, nb);
    hipLaunchKernelGGL(k_scan_final, dim3(nb), dim3(kScanThreads), 0, s, in, out, n, partials);
}

__global__ void k_core_to_i32(const int64_t* __restrict__ core, int32_t* __restrict__ out, int32_t n, int* overflow) {
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        const int64_t c = core[v];
        if (c > INT_MAX || c < INT_MIN) {
            atomicOr(overflow, 1);
            out[v] = INT_MAX;
        } else {
            out[v] = (int32_t)c;
        }
    }
}
void launch_core_to_i32(const int64_t* core, int32_t* out, int32_t n, int* overflow, hipStream_t s) {
    if (n > 0)
        hipLaunchKernelGGL(k_core_to_i32, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, core, out, n, overflow);
}

// ---- lower bounds for the lazy exact peel ---------------------------------------------------
// For h >= 2 and any alive x within distance h-1 of v in G[X],
// N(x;1,X) is contained in N(v;h,X), so |A(x) ∩ X| <= deg_h(v;X).  The anchor
// chain v, anchor(v), anchor(anchor(v)), ... walks alive edges, so every vertex
// on its first h-1 steps qualifies.
__global__ void k_anchor(const int32_t* __restrict__ list, const int* count, int32_t n, const int32_t* __restrict__ rp,
                         const int32_t* __restrict__ col, const uint8_t* __restrict__ alive,
                         const int32_t* __restrict__ adeg, int32_t* __restrict__ anchor, int only_dead) {
    const int total = list ? *count : n;
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int nwaves = (gridDim.x * blockDim.x) >> 6;
    const int l = lane_id();
    // a wave takes 64 entries (one per lane), and then walks the arcs of those
    // whose anchor must be found again, all lanes on one vertex at a time
    for (int base = wave * 64; base < total; base += nwaves * 64) {
        const int i = base + l;
        int32_t v = -1;
        bool need = false;
        if (i < total) {
            v = list ? list[i] : i;
            if (alive[v]) {
                need = true;
                if (only_dead) {
                    const int32_t a = anchor[v];
                    need = !(a >= 0 && alive[a]);
                }
            }
        }
        unsigned long long todo = __ballot(need);
        while (todo) {
            const int src = __ffsll((long long)todo) - 1;
            todo &= todo - 1ull;
            const int32_t u = __shfl(v, src);
            long long best = -1;
            for (int32_t p = rp[u] + l; p < rp[u + 1]; p += 64) {
                const int32_t w = col[p];
                if (alive[w]) {
                    const long long key = ((long long)adeg[w] << 32) | (long long)(0x7FFFFFFF - w);
                    best = key > best ? key : best;
                }
            }
            for (int o = 32; o > 0; o >>= 1) {
                const long long t = __shfl_xor(best, o);
                best = t > best ? t : best;
            }
            if (l == 0) anchor[u] = best < 0 ? -1 : (int32_t)(0x7FFFFFFF - (int32_t)(best & 0x7FFFFFFF));
        }
    }
}
void launch_anchor(const int32_t* list, const int* count, int32_t n, const int32_t* rp, const int32_t* col,
                   const uint8_t* alive, const int32_t* adeg, int32_t* anchor, int only_dead, hipStream_t s) {
    if (n <= 0) return;
    const int grid = list ? 2048 : grid_for((int64_t)n * 64, 256, 16384);
    hipLaunchKernelGGL(k_anchor, dim3(grid), dim3(256), 0, s, list, count, n, rp, col, alive, adeg, anchor,
                       only_dead);
}

__global__ void k_lower_bound(const int32_t* __restrict__ list, const int* count, int32_t n, int h,
                              const uint8_t* __restrict__ alive, const int32_t* __restrict__ adeg,
                              const int32_t* __restrict__ anchor, int64_t* __restrict__ deg,
                              uint8_t* __restrict__ exact) {
    const int total = list ? *count : n;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
        const int32_t v = list ? list[i] : i;
        if (!alive[v]) continue;
        long long lb = adeg[v];
        int32_t x = v;
        for (int t = 1; t < h; ++t) {
            x = anchor[x];
            if (x < 0 || !alive[x]) break;
            const long long a = adeg[x];
            lb = a > lb ? a : lb;
        }
        deg[v] = lb;
        exact[v] = h == 1 ? 1 : 0;
    }
}
void launch_lower_bound(const int32_t* list, const int* count, int32_t n, int h, const uint8_t* alive,
                        const int32_t* adeg, const int32_t* anchor, int64_t* deg, uint8_t* exact, hipStream_t s) {
    if (n <= 0) return;
    const int grid = list ? 1024 : grid_for(n, 256, 8192);
    hipLaunchKernelGGL(k_lower_bound, dim3(grid), dim3(256), 0, s, list, count, n, h, alive, adeg, anchor, deg,
                       exact);
}



__global__ void k_record_fill(RoundState* st, int* hopfill, int t) { hopfill[t] = st->aff_fill; }
void launch_record_fill(RoundState* st, int* hopfill, int t, hipStream_t s) {
    hipLaunchKernelGGL(k_record_fill, dim3(1), dim3(1), 0, s, st, hopfill, t);
}


// ---- device-driven rounds of the lazy exact peel -------------------------------------------
__device__ __forceinline__ long long cur_level(const RoundState* st) {
    return st->min_key > st->c ? st->min_key : st->c;
}

// hist[b] = inexact alive vertices with bound - c' in bucket b (c' = max(c, min)).
// shist (nullable, packed unions): the same per segment, shist[seg * 48 + b].
__global__ void k_bound_hist(const uint8_t* __restrict__ alive, const int64_t* __restrict__ deg,
                             const uint8_t* __restrict__ exact, int32_t n, RoundState* st,
                             const int32_t* __restrict__ seg, int* __restrict__ shist, int gate) {
    if (gate && st->stall) return;
    __shared__ int h[48];
    __shared__ int hs[48];  // segment histogram of the block's first vertex of the step
    if (threadIdx.x < 48) h[threadIdx.x] = 0;
    __syncthreads();
    if (st->alive_count > 0) {
        const long long c = cur_level(st);
        for (int32_t base = blockIdx.x * blockDim.x; base < n; base += gridDim.x * blockDim.x) {
            const int32_t v = base + threadIdx.x;
            int b = -1;
            if (v < n && alive[v] && !exact[v]) {
                const long long d = deg[v] - c;
                b = d <= 0 ? 0 : min(47, 64 - __clzll((unsigned long long)d));
                atomicAdd(&h[b], 1);
            }
            if (shist) {
                // the block's vertices mostly share one segment: count those in LDS
                if (threadIdx.x < 48) hs[threadIdx.x] = 0;
                __syncthreads();
                const int32_t g0 = seg[base];
                if (b >= 0) {
                    const int32_t g = seg[v];
                    if (g == g0) atomicAdd(&hs[b], 1);
                    else atomicAdd(&shist[(size_t)g * 48 + b], 1);
                }
                __syncthreads();
                if (threadIdx.x < 48 && hs[threadIdx.x]) atomicAdd(&shist[(size_t)g0 * 48 + threadIdx.x], hs[threadIdx.x]);
            }
        }
    }
    __syncthreads();
    if (threadIdx.x < 48 && h[threadIdx.x]) atomicAdd(&st->hist[threadIdx.x], h[threadIdx.x]);
}
void launch_bound_hist(const uint8_t* alive, const int64_t* deg, const uint8_t* exact, int32_t n, RoundState* st,
                       hipStream_t s, const int32_t* seg, int* shist, int gate) {
    if (n > 0)
        hipLaunchKernelGGL(k_bound_hist, dim3(grid_for(n, 256, 256)), dim3(256), 0, s, alive, deg, exact, n, st, seg,
                           shist, gate);
}

// Per segment of a packed union: the bound threshold of its next sources, chosen
// as k_decide does for one graph (whole buckets, up to cap sources, at least
// every one at or below c'); segments with nothing at or below c' take no
// sources.  Zeroes the segment histograms for the next iteration.
__global__ void k_decide_seg(RoundState* st, int nseg, int* __restrict__ shist, long long* __restrict__ shi, int cap) {
    const bool rec = st->mode == 1;
    const long long c = cur_level(st);
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < nseg; g += gridDim.x * blockDim.x) {
        int* hg = shist + (size_t)g * 48;
        if (rec) {
            long long hi = LLONG_MIN;
            if (hg[0] > 0) {
                int acc = hg[0], B = 0;
                for (int b = 1; b < 48; ++b) {
                    if (acc + hg[b] > cap) break;
                    acc += hg[b];
                    B = b;
                }
                hi = B == 0 ? c : c + ((1ll << B) - 1);
            }
            shi[g] = hi;
        }
        for (int b = 0; b < 48; ++b)
            if (hg[b]) hg[b] = 0;
    }
}
void launch_decide_seg(RoundState* st, int nseg, int* shist, long long* shi, int cap, hipStream_t s) {
    hipLaunchKernelGGL(k_decide_seg, dim3(grid_for(nseg, 256, 1024)), dim3(256), 0, s, st, nseg, shist, shi, cap);
}

// Commit the round when no inexact vertex is at or below c'; otherwise recompute
// the cap inexact vertices with the smallest bounds (whole buckets).
__device__ __forceinline__ void decide_round(RoundState* st, int cap) {
    if (st->alive_count == 0) {
        st->mode = 2;
        return;
    }
    const long long c = cur_level(st);
    if (st->hist[0] == 0) {
        st->mode = 0;
        return;
    }
    st->mode = 1;
    int acc = st->hist[0], B = 0;
    for (int b = 1; b < 48; ++b) {
        if (acc + st->hist[b] > cap) break;
        acc += st->hist[b];
        B = b;
    }
    st->hi = B == 0 ? c : c + ((1ll << B) - 1);
}
__global__ void k_decide(RoundState* st, int cap) { decide_round(st, cap); }
void launch_decide(RoundState* st, int cap, hipStream_t s) {
    hipLaunchKernelGGL(k_decide, dim3(1), dim3(1), 0, s, st, cap);
}

__global__ __launch_bounds__(256) void k_reduce_hist(const int64_t* __restrict__ deg,
                                                     const uint8_t* __restrict__ alive,
                                                     const uint8_t* __restrict__ exact, int32_t n, RoundState* st) {
    if (st->stall) return;
    __shared__ long long smin[4], smi[4];
    __shared__ int scnt[4];
    long long mn = LLONG_MAX, mi = LLONG_MAX;
    int cnt = 0;
    // four consecutive vertices per thread, all loads issued together
    const int32_t groups = (n + 3) >> 2;
    for (int32_t g = blockIdx.x * blockDim.x + threadIdx.x; g < groups; g += gridDim.x * blockDim.x) {
        const int32_t v0 = g << 2;
        uint8_t a[4], x[4];
        long long k[4];
        if (v0 + 3 < n) {
            const uchar4 a4 = reinterpret_cast<const uchar4*>(alive)[g];
            const uchar4 x4 = reinterpret_cast<const uchar4*>(exact)[g];
            const longlong2 k01 = reinterpret_cast<const longlong2*>(deg)[2 * g];
            const longlong2 k23 = reinterpret_cast<const longlong2*>(deg)[2 * g + 1];
            a[0] = a4.x; a[1] = a4.y; a[2] = a4.z; a[3] = a4.w;
            x[0] = x4.x; x[1] = x4.y; x[2] = x4.z; x[3] = x4.w;
            k[0] = k01.x; k[1] = k01.y; k[2] = k23.x; k[3] = k23.y;
        } else {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const bool in = v0 + u < n;
                a[u] = in ? alive[v0 + u] : 0;
                x[u] = in ? exact[v0 + u] : 1;
                k[u] = in ? deg[v0 + u] : 0;
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (!a[u]) continue;
            mn = k[u] < mn ? k[u] : mn;
            ++cnt;
            if (!x[u]) mi = k[u] < mi ? k[u] : mi;
        }
    }
    mn = wave_min_ll(mn);
    mi = wave_min_ll(mi);
    cnt = wave_sum_i(cnt);
    const int w = threadIdx.x >> 6;
    if (lane_id() == 0) {
        smin[w] = mn;
        smi[w] = mi;
        scnt[w] = cnt;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < (int)(blockDim.x >> 6); ++i) {
            mn = smin[i] < mn ? smin[i] : mn;
            mi = smi[i] < mi ? smi[i] : mi;
            cnt += scnt[i];
        }
        if (cnt > 0) {
            atomicMin(&st->min_key, mn);
            atomicAdd(&st->alive_count, cnt);
            if (mi != LLONG_MAX) atomicMin(&st->min_inexact, mi);
        }
    }
}
void launch_reduce_hist(const int64_t* deg, const uint8_t* alive, const uint8_t* exact, int32_t n, RoundState* st,
                        hipStream_t s) {
    if (n > 0)
        // one block per CU: each block adds three values into one cache line of
        // the round state, and those atomics queue up behind each other
        hipLaunchKernelGGL(k_reduce_hist, dim3(grid_for((n + 3) / 4, 256, 256)), dim3(256), 0, s, deg, alive, exact,
                           n, st);
}
__global__ void k_unstall(RoundState* st) {
    st->stall = 0;
    round_reset_fields(st);
}
void launch_unstall(RoundState* st, hipStream_t s) { hipLaunchKernelGGL(k_unstall, dim3(1), dim3(1), 0, s, st); }

__global__ void k_pick(const uint8_t* __restrict__ alive, const int64_t* __restrict__ deg,
                       const uint8_t* __restrict__ exact, int32_t n, RoundState* st, int32_t* __restrict__ out,
                       int cap, const int32_t* __restrict__ seg, int* __restrict__ gcnt, int32_t* __restrict__ sbit,
                       int qbits, const long long* __restrict__ shi) {
    if (st->mode != 1) return;
    const long long hi0 = st->hi;
    const int32_t stride = gridDim.x * blockDim.x;
    for (int32_t base = blockIdx.x * blockDim.x; base < n; base += stride) {
        if (*(volatile int*)&st->rc_count >= cap) break;
        const int32_t v = base + threadIdx.x;
        bool want = v < n && alive[v] && !exact[v];
        if (want) want = deg[v] <= (shi ? shi[seg[v]] : hi0);
        int b = 0;
        if (want && seg) {
            // a bit position of its own graph; the rest waits for a later batch
            b = atomicAdd(&gcnt[seg[v]], 1);
            want = b < qbits;
        }
        const int slot = wave_append_slot(want, &st->rc_count);
        if (want && slot < cap) {
            out[slot] = v;
            if (sbit) sbit[slot] = b;
        }
    }
}
__global__ void k_pick_finish(RoundState* st, int cap) {
    if (st->mode == 1) st->ms_ns = st->rc_count < cap ? st->rc_count : cap;
}
void launch_pick(const uint8_t* alive, const int64_t* deg, const uint8_t* exact, int32_t n, RoundState* st,
                 int32_t* out, int cap, hipStream_t s, const int32_t* seg, int* gcnt, int32_t* sbit, int qbits,
                 const long long* shi) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_pick, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, alive, deg, exact, n, st, out, cap, seg,
                       gcnt, sbit, qbits, shi);
    hipLaunchKernelGGL(k_pick_finish, dim3(1), dim3(1), 0, s, st, cap);
}




__global__ void k_select_commit(const int64_t* __restrict__ key, uint8_t* __restrict__ alive, int32_t n,
                                RoundState* st, int64_t* __restrict__ core, int32_t* __restrict__ rlist,
                                int32_t* __restrict__ mark, int32_t* __restrict__ rnd) {
    if (st->stall) return;
    // every block takes the same decision from the sweep's reductions; block 0 records it
    const long long c = cur_level(st);
    const int mode = st->alive_count == 0 ? 2 : (st->min_inexact > c ? 0 : 1);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->mode = mode;
        if (mode == 1) st->stall = 1;
        if (mode == 0) {
            st->c = c;
            st->rounds += 1;
        }
    }
    if (mode != 0) return;
    const int32_t epoch = st->epoch;
    const int32_t stride = gridDim.x * blockDim.x;
    for (int32_t base = blockIdx.x * blockDim.x; base < n; base += stride) {
        const int32_t v = base + threadIdx.x;
        const bool take = v < n && alive[v] && key[v] <= c;
        const int slot = wave_append_slot(take, &st->rcount);
        if (take) {
            core[v] = c;
            rlist[slot] = v;
            mark[v] = epoch;
            if (rnd) rnd[v] = epoch;
        }
    }
}
void launch_select_commit(const int64_t* key, uint8_t* alive, int32_t n, RoundState* st, int64_t* core,
                          int32_t* rlist, int32_t* mark, hipStream_t s, int32_t* rnd) {
    if (n > 0)
        hipLaunchKernelGGL(k_select_commit, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, key, alive, n, st, core,
                           rlist, mark, rnd);
}

// ---- R-mask BFS of the lazy exact peel ---------------------------------------------------------
// For v at distance exactly h from R, every vertex that leaves N(v;h,X) when R is
// deleted is itself in R (a path that needed R reaches it after h steps), so
// deg_h(v; X \ R) = deg_h(v; X) - |R ∩ N(v;h,X)|: an exact update.  The mask BFS
// gives |R ∩ N(v;h,X)| as a popcount when |R| <= 64 (R's bits are set by
// launch_enqueue_r).
__device__ __forceinline__ bool rbfs_pulls(const RoundState* st, int64_t nnz) {
    return nnz > 0 && st->hop_arcs * (long long)st->pull_ratio > nnz;
}

// Algorithmic bytes of a block of the mask BFS and the arcs of the vertices it
// put on the next frontier: one atomic per block and counter.
__device__ __forceinline__ void rbfs_count(unsigned long long bytes, long long next_arcs, RoundState* st) {
    __shared__ unsigned long long red[2][16];
    bytes = (unsigned long long)wave_sum_ll((long long)bytes);
    next_arcs = wave_sum_ll(next_arcs);
    if (lane_id() == 0) {
        red[0][threadIdx.x >> 6] = bytes;
        red[1][threadIdx.x >> 6] = (unsigned long long)next_arcs;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        unsigned long long t = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[threadIdx.x][w];
        if (t) atomicAdd(threadIdx.x == 0 ? &st->rbfs_bytes : (unsigned long long*)&st->next_arcs, t);
    }
}

// One hop of the mask BFS, in either form, chosen on the device (rbfs_pulls).
// The frontier is held twice: gain (the bits each frontier vertex passes on,
// zero elsewhere) and a one-bit-per-vertex bitmap fbits (n/8 bytes, resident in
// L2), so that a neighbour off the frontier costs a bit test, not an 8-byte
// gather.  fbits_next is null at the last hop, whose frontier is never read.
// Push: a wave per 256-arc chunk of the frontier; every new bit of an alive
// neighbour is or-ed into its mask with an atomic, and a vertex that gains one
// joins the next frontier (fmark dedups) and, the first time in the round, the
// affected list (mark).  Pull: vertex w gets new =
// (OR over alive neighbours u of gain_cur[u]) & ~rmask[w] -- the union of what
// the frontier would push to it (gain_cur is zero off the frontier and on
// deleted vertices, which never carry bits); the scan of w's arcs stops once w
// holds every bit of R (full), which for the one- and two-vertex deletions of a
// long peel is usually at the first frontier neighbour.  A thread owns a vertex
// of at most kRbfsLight arcs and scans four arcs per step; the arcs of a larger
// vertex are scanned by its whole wave, 64 at a time.
__device__ __forceinline__ bool fbit(const uint32_t* __restrict__ fbits, int32_t x) {
    return (fbits[x >> 5] >> (x & 31)) & 1u;
}

// The hop's two output lists (next frontier, affected) are gathered per block in
// LDS and copied out with one global atomic per flush: a device-wide counter
// hit once per wave step serialises (about 6 ns per atomic, so the 20,000
// appends of a 600,000-arc hop cost more than the hop's own work).
constexpr int kRbfsBuf = 2048;

__device__ __forceinline__ void lds_append(bool want, int32_t v, int32_t* buf, int* n) {
    const unsigned long long m = __ballot(want);
    if (m == 0ull) return;
    const int leader = __ffsll((long long)m) - 1;
    int base = 0;
    if (lane_id() == leader) base = atomicAdd(n, __popcll(m));
    base = __shfl(base, leader);
    if (want) buf[base + __popcll(m & ((1ull << lane_id()) - 1ull))] = v;
}

// Block-uniform (every thread calls it after a barrier): copies the buffered
// entries to out[*count ...] and empties the buffer.
__device__ __forceinline__ void lds_flush(int32_t* buf, int* n, int* gbase, int32_t* __restrict__ out, int* count) {
    const int cnt = *n;
    if (cnt == 0) return;
    if (threadIdx.x == 0) *gbase = atomicAdd(count, cnt);
    __syncthreads();
    const int base = *gbase;
    for (int i = threadIdx.x; i < cnt; i += blockDim.x) out[base + i] = buf[i];
    __syncthreads();
    if (threadIdx.x == 0) *n = 0;
    __syncthreads();
}

__global__ __launch_bounds__(256) void k_rbfs_hop(const int32_t* __restrict__ qv, const int32_t* __restrict__ qb,
                                                  const int* qcount, int32_t n, const int32_t* __restrict__ rp,
                                                  const int32_t* __restrict__ col,
                                                  const uint8_t* __restrict__ alive,
                                                  const uint64_t* __restrict__ gain_cur,
                                                  const uint32_t* __restrict__ fbits_cur,
                                                  uint64_t* __restrict__ rmask, uint64_t* __restrict__ gain_next,
                                                  uint32_t* __restrict__ fbits_next,
                                                  int32_t* __restrict__ mark, int32_t* __restrict__ fmark,
                                                  int32_t* __restrict__ fnext, int* fnext_count,
                                                  int32_t* __restrict__ alist, int* aff_fill, RoundState* st,
                                                  int64_t nnz) {
    const int32_t epoch = st->epoch;
    const int l = lane_id();
    unsigned long long bytes = 0;
    long long next_arcs = 0;
    __shared__ int32_t s_f[kRbfsBuf], s_a[kRbfsBuf];
    __shared__ int s_nf, s_na, s_gb;
    if (threadIdx.x == 0) {
        s_nf = 0;
        s_na = 0;
    }
    __syncthreads();
    // after each block-wide step: flush a buffer that could not take another
    // step's worth of entries
    auto maybe_flush = [&]() {
        __syncthreads();
        const bool ff = s_nf > kRbfsBuf - 256, fa = s_na > kRbfsBuf - 256;
        __syncthreads();
        if (ff) lds_flush(s_f, &s_nf, &s_gb, fnext, fnext_count);
        if (fa) lds_flush(s_a, &s_na, &s_gb, alist, aff_fill);
    };
    if (!rbfs_pulls(st, nnz)) {
        const int32_t fepoch = st->fepoch;
        const int nq = *qcount;
        const int wpb = blockDim.x >> 6;
        const int wib = threadIdx.x >> 6;
        // the block takes wpb chunks at a time (one per wave), so that every
        // thread runs the same number of steps
        for (int qg = blockIdx.x * wpb; qg < nq; qg += gridDim.x * wpb) {
            const int q = qg + wib;
            int32_t b = 0, e = 0;
            uint64_t g = 0ull;
            if (q < nq) {
                const int32_t u = qv[q];
                b = qb[q];
                e = min(b + kExpandChunk, rp[u + 1]);
                g = gain_cur[u];
                if (l == 0) bytes += 20;  // chunk (u, b), rp[u + 1], gain[u]
            }
            for (int step = 0; step < kExpandChunk; step += 64) {
                const int32_t p = b + step + l;
                bool want_f = false, want_a = false;
                int32_t w = 0;
                if (p < e && g) {
                    w = col[p];
                    bytes += 5;  // id, alive
                    if (alive[w]) {
                        bytes += 8;  // rmask
                        const uint64_t nb = g & ~rmask[w];
                        if (nb) {
                            const uint64_t old = atomicOr((unsigned long long*)&rmask[w], (unsigned long long)nb);
                            const uint64_t nw = nb & ~old;
                            if (nw) {
                                bytes += 16;  // rmask, gain written
                                atomicOr((unsigned long long*)&gain_next[w], (unsigned long long)nw);
                                if (fmark[w] != fepoch) want_f = atomicExch(&fmark[w], fepoch) != fepoch;
                                if (mark[w] != epoch) want_a = atomicExch(&mark[w], epoch) != epoch;
                            }
                        }
                    }
                }
                if (want_f) {
                    next_arcs += rp[w + 1] - rp[w];
                    if (fbits_next) atomicOr(&fbits_next[w >> 5], 1u << (w & 31));
                }
                lds_append(want_f, w, s_f, &s_nf);
                lds_append(want_a, w, s_a, &s_na);
                bytes += (want_f ? 12 : 0) + (want_a ? 4 : 0);
                maybe_flush();
            }
        }
    } else {
        const int rc = st->rcount;
        const uint64_t full = rc >= 64 ? ~0ull : ((1ull << rc) - 1ull);
        // one deleted vertex: any frontier neighbour carries its only bit
        const bool one = rc == 1;
        const int32_t stride = gridDim.x * blockDim.x;
        for (int32_t base = blockIdx.x * blockDim.x; base < n; base += stride) {
            const int32_t w = base + threadIdx.x;
            bool heavy = false;
            uint64_t have = 0ull, acc = 0ull;
            int32_t b = 0, e = 0;
            if (w < n) {
                bytes += 1;
                if (alive[w]) {
                    have = rmask[w];
                    bytes += 8;
                    if (have != full) {
                        b = rp[w];
                        e = rp[w + 1];
                        bytes += 8;
                        if (e - b > kRbfsLight) {
                            heavy = true;
                        } else {
                            int32_t p = b;
                            while (p < e) {
                                int32_t x[4];
                                bool f[4];
#pragma unroll
                                for (int k = 0; k < 4; ++k) x[k] = p + k < e ? col[p + k] : -1;
#pragma unroll
                                for (int k = 0; k < 4; ++k) f[k] = x[k] >= 0 && fbit(fbits_cur, x[k]);
                                if (f[0] | f[1] | f[2] | f[3]) {
                                    if (one) {
                                        acc = full;
                                    } else {
#pragma unroll
                                        for (int k = 0; k < 4; ++k)
                                            if (f[k]) {
                                                acc |= gain_cur[x[k]];
                                                bytes += 8;
                                            }
                                    }
                                }
                                p = min(p + 4, e);
                                if ((acc | have) == full) break;
                            }
                            bytes += 8ull * (unsigned long long)(p - b);  // ids and frontier bit words
                        }
                    }
                }
            }
            // the wave scans its heavy vertices together, 64 arcs per step
            unsigned long long hm = __ballot(heavy);
            while (hm) {
                const int src = __ffsll((long long)hm) - 1;
                hm &= hm - 1ull;
                const int32_t hb = __shfl(b, src), he = __shfl(e, src);
                const uint64_t hhave = __shfl(have, src);
                uint64_t hacc = 0ull;
                int32_t p0 = hb;
                for (; p0 < he; p0 += 64) {
                    const int32_t p = p0 + l;
                    int32_t x = 0;
                    bool f = false;
                    if (p < he) {
                        x = col[p];
                        f = fbit(fbits_cur, x);
                    }
                    const unsigned long long hits = __ballot(f);
                    if (!hits) continue;
                    if (one) {
                        hacc = full;
                    } else {
                        uint64_t gv = f ? gain_cur[x] : 0ull;
                        if (f) bytes += 8;
#pragma unroll
                        for (int o = 32; o >= 1; o >>= 1) gv |= __shfl_xor(gv, o);
                        hacc |= gv;
                    }
                    if ((hacc | hhave) == full) {
                        p0 += 64;
                        break;
                    }
                }
                if (l == 0) bytes += 8ull * (unsigned long long)(min(p0, he) - hb);
                if (l == src) acc = hacc;
            }
            bool front = false, first = false;
            const uint64_t nw = acc & ~have;
            if (nw) {
                rmask[w] = have | nw;
                gain_next[w] = nw;
                front = true;
                next_arcs += e - b;
                first = mark[w] != epoch;
                if (first) mark[w] = epoch;
                bytes += 20;
            }
            // the wave's 64 vertices are two whole words of the next bitmap
            if (fbits_next) {
                const unsigned long long fm = __ballot(front);
                const int32_t w0 = base + (threadIdx.x & ~63);
                if (l == 0 && w0 < n) fbits_next[w0 >> 5] = (uint32_t)fm;
                if (l == 32 && w0 + 32 < n) fbits_next[(w0 >> 5) + 1] = (uint32_t)(fm >> 32);
            }
            lds_append(front, w, s_f, &s_nf);
            lds_append(first, w, s_a, &s_na);
            bytes += (front ? 4 : 0) + (first ? 4 : 0);
            maybe_flush();
        }
    }
    __syncthreads();
    lds_flush(s_f, &s_nf, &s_gb, fnext, fnext_count);
    lds_flush(s_a, &s_na, &s_gb, alist, aff_fill);
    rbfs_count(bytes, next_arcs, st);
}

void launch_rbfs_hop(const int32_t* qv, const int32_t* qb, const int* qcount, int32_t n, const int32_t* rp,
                     const int32_t* col, const uint8_t* alive, const uint64_t* gain_cur, const uint32_t* fbits_cur,
                     uint64_t* rmask, uint64_t* gain_next, uint32_t* fbits_next, int32_t* mark, int32_t* fmark,
                     int32_t* fnext, int* fnext_count, int32_t* alist, int* aff_fill, RoundState* st, int64_t nnz,
                     hipStream_t s, PullTimer* timer, int grid) {
    const bool timed = timer && timer->used < timer->cap;
    if (timed) (void)hipEventRecord(timer->ev[2 * timer->used], s);
    hipLaunchKernelGGL(k_rbfs_hop, dim3(grid > 0 ? grid : 512), dim3(256), 0, s, qv, qb, qcount, n, rp, col, alive,
                       gain_cur, fbits_cur, rmask, gain_next, fbits_next, mark, fmark, fnext, fnext_count, alist,
                       aff_fill, st, nnz);
    if (timed) {
        (void)hipEventRecord(timer->ev[2 * timer->used + 1], s);
        timer->used += 1;
    }
}

// Zero arr[list[i]] and the list's bitmap words for the previous frontier,
// then (last block) end hop t:
// record the affected count reached (hopfill[t]), reset the chunk queue, take
// the next frontier's arcs and clear its list fill.  Every block has read the
// list's count before it is counted, and the end of the hop touches nothing the
// blocks write.
__global__ void k_clear_hop_end(const int32_t* __restrict__ list, const int* count, uint64_t* __restrict__ arr,
                                uint32_t* __restrict__ fbits, RoundState* st, int* hopfill, int t, int h) {
    const int cnt = *count;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += gridDim.x * blockDim.x) {
        const int32_t v = list[i];
        arr[v] = 0ull;
        fbits[v >> 5] = 0u;
    }
    __shared__ int s_last;
    __syncthreads();
    if (threadIdx.x == 0) s_last = atomicAdd(&st->blocks_done, 1) == (int)gridDim.x - 1;
    __syncthreads();
    if (s_last && threadIdx.x == 0) {
        st->blocks_done = 0;
        hopfill[t] = st->aff_fill;
        if (t < 4) st->hop_log[t] = st->hop_arcs;
        st->qcount = 0;
        st->hop_arcs = st->next_arcs;
        st->next_arcs = 0;
        if (t < h) {
            st->fepoch += 1;
            st->fcount[(t + 1) & 1] = 0;
        }
    }
}
void launch_clear_hop_end(const int32_t* list, const int* count, uint64_t* arr, uint32_t* fbits, RoundState* st,
                          int* hopfill, int t, int h, hipStream_t s, int grid) {
    hipLaunchKernelGGL(k_clear_hop_end, dim3(grid > 0 ? grid : 128), dim3(256), 0, s, list, count, arr, fbits, st,
                       hopfill, t, h);
}


__global__ void k_clear_u64_lists3(const int32_t* __restrict__ l0, const int* c0, uint64_t* __restrict__ a0,
                                   const int32_t* __restrict__ l1, const int* c1, uint64_t* __restrict__ a1,
                                   const int32_t* __restrict__ l2, const int* c2, uint64_t* __restrict__ a2,
                                   RoundState* st) {
    const int tid = blockIdx.x * blockDim.x + threadIdx.x, nth = gridDim.x * blockDim.x;
    const int n0 = *c0, n1 = *c1, n2 = *c2;
    for (int i = tid; i < n0; i += nth) a0[l0[i]] = 0ull;
    for (int i = tid; i < n1; i += nth) a1[l1[i]] = 0ull;
    for (int i = tid; i < n2; i += nth) a2[l2[i]] = 0ull;
    if (!st) return;
    // the last block to finish resets the round state for the next round:
    // every block has consumed the counts it read before it is counted, and
    // the reset touches nothing the blocks write, so no fence is needed (a
    // device-scope fence per block would write back L2 on every XCD)
    __shared__ int s_last;
    __syncthreads();
    if (threadIdx.x == 0) s_last = atomicAdd(&st->blocks_done, 1) == (int)gridDim.x - 1;
    __syncthreads();
    if (s_last && threadIdx.x == 0) {
        st->blocks_done = 0;
        if (!st->stall) round_reset_fields(st);
    }
}
void launch_clear_u64_lists3(const int32_t* l0, const int* c0, uint64_t* a0, const int32_t* l1, const int* c1,
                             uint64_t* a1, const int32_t* l2, const int* c2, uint64_t* a2, hipStream_t s,
                             RoundState* st, int grid) {
    hipLaunchKernelGGL(k_clear_u64_lists3, dim3(grid > 0 ? grid : 128), dim3(256), 0, s, l0, c0, a0, l1, c1, a1, l2,
                       c2, a2, st);
}


__global__ void k_decay_masked(const int32_t* __restrict__ alist, RoundState* st, const int* __restrict__ hopfill,
                               int h, const uint8_t* __restrict__ alive, const int32_t* __restrict__ adeg,
                               const int32_t* __restrict__ anchor, const uint64_t* __restrict__ rmask,
                               int64_t* __restrict__ deg, uint8_t* __restrict__ exact) {
    const int total = st->aff_fill;
    const int rc = st->rcount;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
        const int32_t v = alist[i];
        if (!alive[v]) continue;
        if (h == 1) {
            deg[v] = adeg[v];
            exact[v] = 1;
            continue;
        }
        int t = 1;
        while (t < h && i >= hopfill[t]) ++t;
        if (t == h && rc <= 64) {
            // exact values stay exact, bounds stay bounds
            deg[v] -= (int64_t)__popcll(rmask[v]);
            continue;
        }
        const long long lost = (long long)rc + (h - t >= 1 ? (long long)hopfill[h - t] : 0ll);
        long long lb = deg[v] - lost;
        long long ab = adeg[v];
        int32_t x = v;
        for (int q = 1; q < h; ++q) {
            x = anchor[x];
            if (x < 0 || !alive[x]) break;
            const long long a = adeg[x];
            ab = a > ab ? a : ab;
        }
        deg[v] = lb > ab ? lb : ab;
        exact[v] = 0;
    }
}
void launch_decay_masked(const int32_t* alist, RoundState* st, const int* hopfill, int h, const uint8_t* alive,
                         const int32_t* adeg, const int32_t* anchor, const uint64_t* rmask, int64_t* deg,
                         uint8_t* exact, hipStream_t s) {
    hipLaunchKernelGGL(k_decay_masked, dim3(1024), dim3(256), 0, s, alist, st, hopfill, h, alive, adeg, anchor, rmask,
                       deg, exact);
}

}  // namespace kh
