// Bit-parallel multi-source bounded BFS: h-degrees deg_h(s;X) = |N(s;h,X)| - 1
// (Sec. 2) for a batch of up to 64 Q sources at once (gfx950, wave64).
//
// Every vertex u carries Q 64-bit words per plane; bit j of word (j / 64) stands
// for source s_j.  vis[u] is the set of sources whose ball already contains u,
// fr[u] the sources that reached u at the previous hop.  One hop is
//     new[u] = (OR over alive neighbours w of fr[w]) & ~vis[u],  vis[u] |= new[u],
// and deg(s_j) = (number of u with bit j of vis[u]) - 1 after h hops.
//
// Layout: a vertex's Q words are contiguous (Q = 16 gives one 128-byte line), and
// a group of Q lanes owns one vertex, lane j owning word j, so every neighbour
// gather is one coalesced line.  Work items are (vertex, arc range) pieces of at
// most kPullChunk arcs sorted by length, so hubs are spread over many groups; the
// pieces of a split vertex meet in an accumulator plane.  A one-bit-per-vertex
// frontier bitmap lets a gather be skipped when the neighbour's word is empty, so
// stale frontier words never need clearing.  Hop 1 pushes from the sources
// instead of sweeping the whole graph.
//
// Work is proportional to what the batch reaches: each later hop first lists
// the alive neighbours of the previous frontier (candidates) and pulls only
// their work items; frontier, candidate and visited lists let every clear and
// the final count touch only listed vertices.  Once a frontier's adjacency
// exceeds 1/kSweepRatio of all arcs the hop (and the rest of the batch) sweeps
// every work item instead, and the clears and the count sweep too.
#include "kh_common.hpp"
#include "kh_internal.hpp"

namespace kh {

// Neighbour frontier words a group of the pull kernel gathers at once.
constexpr int kGatherDepth = 4;

// First visit of a vertex in its 64-vertex tile: the tile joins the visited list.
__device__ __forceinline__ bool tile_first(int32_t u, uint32_t* __restrict__ bmTile) {
    const int32_t t = u >> 6;
    const uint32_t b = 1u << (t & 31);
    return !(bmTile[t >> 5] & b) && !(atomicOr(&bmTile[t >> 5], b) & b);
}

// A frontier vertex with more than 64 arcs also lists its 64-arc chunks, so that
// the candidate expansion spreads it over many waves.
__device__ __forceinline__ void frontier_chunks(int32_t u, const int32_t* __restrict__ rp, int* count,
                                                int2* __restrict__ fc) {
    const int32_t b = rp[u], d = rp[u + 1] - b;
    if (d <= 64) return;
    const int nc = (d + 63) >> 6;
    const int base = atomicAdd(count, nc);
    for (int k = 0; k < nc; ++k) fc[base + k] = make_int2(u, b + 64 * k);
}

template <int Q>
__global__ void k_ms_init(const int32_t* __restrict__ src, int ns, const int* ns_dev, int ns_cap,
                          const int32_t* __restrict__ sbit, const int32_t* __restrict__ seg,
                          uint64_t* __restrict__ vis, const int32_t* __restrict__ adeg, uint64_t* __restrict__ valid,
                          RoundState* st, MsCtl* ctl, int32_t* __restrict__ tl, uint32_t* __restrict__ bmTile,
                          uint8_t* __restrict__ exact_out) {
    if (ns_dev) ns = min(*ns_dev, ns_cap);
    unsigned long long te = 0;
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < ns; j += gridDim.x * blockDim.x) {
        const int32_t s = src[j];
        if (exact_out) exact_out[s] = 1;
        const int bj = sbit ? sbit[j] : j;
        vis[(size_t)s * Q + (bj >> 6)] = 1ull << (bj & 63);
        te += (unsigned long long)adeg[s];
        const int slot = wave_append_slot(tile_first(s, bmTile), &ctl->tl_count);
        if (slot >= 0) tl[slot] = s >> 6;
    }
    if (blockIdx.x == 0 && threadIdx.x < Q) {
        // segmented batches use every bit position in some graph
        const int c = seg ? 64 * Q : ns - 64 * (int)threadIdx.x;
        valid[threadIdx.x] = c >= 64 ? ~0ull : (c <= 0 ? 0ull : ((1ull << c) - 1ull));
    }
    te = (unsigned long long)wave_sum_ll((long long)te);
    if (lane_id() == 0 && te) atomicAdd(&st->te, te);
}

// Hop 1: push the sources' bits to their alive neighbours.
template <int Q>
__global__ void k_ms_push(const int32_t* __restrict__ src, int ns, const int* ns_dev, int ns_cap,
                          const int32_t* __restrict__ sbit, const int32_t* __restrict__ rp,
                          const int32_t* __restrict__ col, const uint8_t* __restrict__ alive,
                          uint64_t* __restrict__ acc, uint32_t* __restrict__ bmT, int32_t* __restrict__ touched,
                          int* tcount, RoundState* st) {
    if (ns_dev) ns = min(*ns_dev, ns_cap);
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int nwaves = (gridDim.x * blockDim.x) >> 6;
    const int l = lane_id();
    unsigned long long arcs = 0;
    for (int j = wave; j < ns; j += nwaves) {
        const int32_t s = src[j];
        const int bj = sbit ? sbit[j] : j;
        const uint64_t bit = 1ull << (bj & 63);
        const int word = bj >> 6;
        const int32_t b = rp[s], e = rp[s + 1];
        arcs += (unsigned long long)(e - b);
        for (int32_t p0 = b; p0 < e; p0 += 64) {
            const int32_t p = p0 + l;
            bool want = false;
            int32_t w = 0;
            if (p < e) {
                w = col[p];
                if (alive[w]) {
                    atomicOr((unsigned long long*)&acc[(size_t)w * Q + word], (unsigned long long)bit);
                    const uint32_t wb = 1u << (w & 31);
                    if (!(bmT[w >> 5] & wb)) want = !(atomicOr(&bmT[w >> 5], wb) & wb);
                }
            }
            const int slot = wave_append_slot(want, tcount);
            if (want) touched[slot] = w;
        }
    }
    if (l == 0 && arcs) atomicAdd(&st->arcs, arcs);
}

// new = acc & ~vis for listed vertices (the pushed ones, or the split ones after a
// pull).  Unless the batch went dense, vertices with new bits join the frontier
// list of the hop and first visits put their tile on the visited list.  bm_clear
// (nullable) is a bitmap whose bits are exactly the listed vertices: cleared here.
template <int Q>
__global__ void k_ms_finalize(const int32_t* __restrict__ list, const int* count_p, int count_i,
                              uint64_t* __restrict__ acc, uint64_t* __restrict__ vis, uint64_t* __restrict__ fr_next,
                              uint32_t* __restrict__ bm_next, const uint64_t* __restrict__ valid, int last,
                              const int32_t* __restrict__ adeg, RoundState* st, MsCtl* ctl,
                              int32_t* __restrict__ fl_out, int2* __restrict__ fc_out, int slot,
                              int32_t* __restrict__ tl, uint32_t* __restrict__ bmTile, const int32_t* __restrict__ rp,
                              uint32_t* __restrict__ bm_clear) {
    const int cnt = count_p ? *count_p : count_i;
    const bool lists = ctl->dense == 0;
    const int l = lane_id();
    const int j = l % Q;
    const int gbase = l - j;
    const unsigned long long gmask = (Q == 64 ? ~0ull : ((1ull << Q) - 1ull)) << gbase;
    const int gpb = blockDim.x / Q;
    const int ngroups = gridDim.x * gpb;
    const uint64_t vm = valid[j];
    unsigned long long te = 0;
    long long fdeg = 0;
    for (int idx = blockIdx.x * gpb + threadIdx.x / Q; idx < cnt; idx += ngroups) {
        const int32_t u = list[idx];
        if (bm_clear && j == 0) bm_clear[u >> 5] = 0u;
        const size_t at = (size_t)u * Q + j;
        const uint64_t a = acc[at];
        if (a) acc[at] = 0ull;
        const uint64_t vw = vis[at];
        const uint64_t nw = a & ~vw & vm;
        const bool any = (__ballot(nw != 0ull) & gmask) != 0ull;
        bool fresh = false, front = false;
        if (any) {
            fresh = (__ballot(vw != 0ull) & gmask) == 0ull;
            if (nw) vis[at] = vw | nw;
            if (!last) {
                fr_next[at] = nw;
                if (j == 0) atomicOr(&bm_next[u >> 5], 1u << (u & 31));
                te += (unsigned long long)__popcll(nw) * (unsigned long long)adeg[u];
                front = true;
            }
        }
        if (lists) {
            const int sf = wave_append_slot(j == 0 && front, &ctl->fl_count[slot]);
            if (sf >= 0) {
                fl_out[sf] = u;
                fdeg += rp[u + 1] - rp[u];
                frontier_chunks(u, rp, &ctl->fc_count[slot], fc_out);
            }
            const int sv = wave_append_slot(j == 0 && fresh && tile_first(u, bmTile), &ctl->tl_count);
            if (sv >= 0) tl[sv] = u >> 6;
        }
    }
    te = (unsigned long long)wave_sum_ll((long long)te);
    fdeg = wave_sum_ll(fdeg);
    if (l == 0) {
        if (te) atomicAdd(&st->te, te);
        if (fdeg) atomicAdd((unsigned long long*)&ctl->fdeg[slot], (unsigned long long)fdeg);
    }
}

// Candidates of hop t: the alive neighbours of the frontier of hop t - 1, each
// listed once (bmC), with all of its work items.  Decides the hop's mode: a
// frontier whose adjacency exceeds 1/kSweepRatio of the arcs makes the batch
// dense from this hop on.  Also resets the counters that hop t and hop t + 1
// will fill (their previous readers have finished).
__device__ __forceinline__ void expand_arc(bool has, int32_t w, const int32_t* __restrict__ rp,
                                           const uint8_t* __restrict__ alive, uint32_t* __restrict__ bmC,
                                           int32_t* __restrict__ cv, int32_t* __restrict__ ci,
                                           const int32_t* __restrict__ vitem, int* cv_count, int* ci_count) {
    const int l = lane_id();
    bool want = false;
    if (has && alive[w]) {
        const uint32_t wb = 1u << (w & 31);
        if (!(bmC[w >> 5] & wb)) want = !(atomicOr(&bmC[w >> 5], wb) & wb);
    }
    const int sc = wave_append_slot(want, cv_count);
    if (sc >= 0) cv[sc] = w;
    int ni = 0;
    if (want) {
        const int32_t dw = rp[w + 1] - rp[w];
        ni = dw > kPullChunk ? (dw + kPullChunk - 1) / kPullChunk : 1;
    }
    const int incl_i = wave_incl_scan(ni);
    const int tot_i = __shfl(incl_i, 63);
    if (tot_i) {
        int cbase = 0;
        if (l == 0) cbase = atomicAdd(ci_count, tot_i);
        cbase = __shfl(cbase, 0);
        const int32_t first = want ? vitem[w] : 0;
        for (int k2 = 0; k2 < ni; ++k2) ci[cbase + incl_i - ni + k2] = first + k2;
    }
}

__global__ void k_ms_expand(const int32_t* __restrict__ fl, const int2* __restrict__ fc, MsCtl* ctl, int t,
                            int64_t nnz,
                            const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                            const uint8_t* __restrict__ alive, uint32_t* __restrict__ bmC, int32_t* __restrict__ cv,
                            int32_t* __restrict__ ci, const int32_t* __restrict__ vitem, const int* ns_dev) {
    const int cur = t & 1, prev = cur ^ 1;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctl->fl_count[cur] = 0;
        ctl->fc_count[cur] = 0;
        ctl->fdeg[cur] = 0;
        ctl->cv_count[prev] = 0;
        ctl->ci_count[prev] = 0;
    }
    if (ns_dev && *ns_dev == 0) return;
    const bool was_dense = ctl->dense != 0;
    if (was_dense || ctl->fdeg[prev] * kSweepRatio > nnz) {
        if (!was_dense && blockIdx.x == 0 && threadIdx.x == 0) {
            ctl->dense = 1;
            ctl->dense_at = t;
        }
        return;
    }
    const int nf = ctl->fl_count[prev];
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int nwaves = (gridDim.x * blockDim.x) >> 6;
    const int l = lane_id();
    // a wave takes 64 frontier vertices (one per lane) and walks the arcs of
    // those with at most 64 together, 64 at a time: lane l's arc belongs to the
    // last vertex k whose first flattened index excl_k is <= its index
    for (int base = wave * 64; base < nf; base += nwaves * 64) {
        const int i = base + l;
        int32_t b = 0, d = 0;
        if (i < nf) {
            const int32_t u = fl[i];
            b = rp[u];
            d = rp[u + 1] - b;
            if (d > 64) d = 0;  // walked by chunks below
        }
        const int incl = wave_incl_scan(d);
        const int total = __shfl(incl, 63);
        const int excl = incl - d;
        for (int off = 0; off < total; off += 64) {
            const int idx = min(off + l, total - 1);
            int k = 0;
#pragma unroll
            for (int step = 32; step >= 1; step >>= 1) {
                const int e = __shfl(excl, k + step);
                if (e <= idx) k += step;
            }
            const int32_t bk = __shfl(b, k);
            const int ek = __shfl(excl, k);
            const bool has = off + l < total;
            const int32_t w = has ? col[bk + (idx - ek)] : 0;
            expand_arc(has, w, rp, alive, bmC, cv, ci, vitem, &ctl->cv_count[cur], &ctl->ci_count[cur]);
        }
    }
    // larger frontier vertices: one 64-arc chunk per wave step
    const int nc = ctl->fc_count[prev];
    for (int c = wave; c < nc; c += nwaves) {
        const int2 ch = fc[c];
        const int32_t e = rp[ch.x + 1];
        const int32_t p = ch.y + l;
        const bool has = p < e;
        const int32_t w = has ? col[p] : 0;
        expand_arc(has, w, rp, alive, bmC, cv, ci, vitem, &ctl->cv_count[cur], &ctl->ci_count[cur]);
    }
}

// After hop t: clear the frontier bitmap of hop t - 1 and the candidate bitmap of
// hop t (by their lists; the frontier bitmap by a sweep when hop t - 1 was dense).
__global__ void k_ms_clear(const MsCtl* ctl, int t, const int32_t* __restrict__ fl, uint32_t* __restrict__ bm_cur,
                           int64_t bmwords, const int32_t* __restrict__ cv, uint32_t* __restrict__ bmC,
                           const int* ns_dev) {
    if (ns_dev && *ns_dev == 0) return;
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    const int nth = gridDim.x * blockDim.x;
    // hop k ran sparse unless dense_at is set and <= k
    const int dat = ctl->dense_at;
    const int dfrom = dat ? dat : 0x7fffffff;
    if (dfrom > t - 1) {
        const int nf = ctl->fl_count[(t - 1) & 1];
        for (int i = tid; i < nf; i += nth) bm_cur[fl[i] >> 5] = 0u;
    } else {
        for (int64_t w = tid; w < bmwords; w += nth) bm_cur[w] = 0u;
    }
    if (dfrom > t) {
        const int nc = ctl->cv_count[t & 1];
        for (int i = tid; i < nc; i += nth) bmC[cv[i] >> 5] = 0u;
    }
}

// Hops 2..h: pull the neighbours' frontier words.
template <int Q>
__global__ __launch_bounds__(256) void k_ms_pull(int32_t nitems, const int32_t* __restrict__ item_u,
                                                 const int32_t* __restrict__ item_beg,
                                                 const int32_t* __restrict__ item_end,
                                                 const uint8_t* __restrict__ item_split,
                                                 const int32_t* __restrict__ col, const uint8_t* __restrict__ alive,
                                                 uint64_t* __restrict__ vis, const uint64_t* __restrict__ fr_cur,
                                                 const uint32_t* __restrict__ bm_cur, uint64_t* __restrict__ fr_next,
                                                 uint32_t* __restrict__ bm_next, uint64_t* __restrict__ acc,
                                                 const uint64_t* __restrict__ valid, int last,
                                                 const int32_t* __restrict__ adeg, RoundState* st,
                                                 const int* ns_dev, const int32_t* __restrict__ citems, MsCtl* ctl,
                                                 int t, int32_t* __restrict__ fl_out, int2* __restrict__ fc_out,
                                                 int32_t* __restrict__ tl, uint32_t* __restrict__ bmTile,
                                                 const int32_t* __restrict__ rp) {
    if (ns_dev && *ns_dev == 0) return;
    const bool sparse = ctl->dense == 0;
    const int slot = t & 1;
    const int count = sparse ? ctl->ci_count[slot] : nitems;
    const int l = lane_id();
    const int j = l % Q;
    const int gbase = l - j;
    const unsigned long long gmask = (Q == 64 ? ~0ull : ((1ull << Q) - 1ull)) << gbase;
    const int gpb = blockDim.x / Q;
    const int ngroups = gridDim.x * gpb;
    const uint64_t vm = valid[j];
    unsigned long long te = 0, arcs = 0, bytes = 0, gath = 0;
    long long fdeg = 0;
    for (int k = blockIdx.x * gpb + threadIdx.x / Q; k < count; k += ngroups) {
        const int it = sparse ? citems[k] : k;
        const int32_t u = item_u[it];
        if (j == 0) bytes += sparse ? 18 : 14;  // (candidate index,) item (u, beg, end, split) and alive[u]
        if (!alive[u]) continue;
        if (j == 0) bytes += 8 * Q;  // vis[u]
        const size_t at = (size_t)u * Q + j;
        const uint64_t vw = vis[at];
        const bool full = (vw & vm) == vm;
        if ((__ballot(full) & gmask) == gmask) continue;
        const int32_t b = item_beg[it], e = item_end[it];
        uint64_t a = 0ull;
        int32_t p = b;
        if (Q >= 4) {
            // Q adjacency ids per chunk (lane j reads arc base + j), their frontier
            // bits tested in parallel, then the group gathers word j of every
            // frontier neighbour, four loads in flight at a time
            for (; p < e; p += Q) {
                const int32_t pj = p + j;
                int32_t w = 0;
                bool f = false;
                if (pj < e) {
                    w = col[pj];
                    f = (bm_cur[w >> 5] >> (w & 31)) & 1u;
                }
                unsigned long long fm = (__ballot(f) & gmask) >> gbase;
                if (j == 0) gath += (unsigned long long)__popcll(fm) * 8 * Q;
                while (fm) {
                    int32_t ws[kGatherDepth];
#pragma unroll
                    for (int u = 0; u < kGatherDepth; ++u) {
                        ws[u] = -1;
                        if (fm) {
                            const int k = __ffsll((long long)fm) - 1;
                            fm &= fm - 1ull;
                            ws[u] = __shfl(w, gbase + k);
                        }
                    }
                    uint64_t x[kGatherDepth];
#pragma unroll
                    for (int u = 0; u < kGatherDepth; ++u) x[u] = ws[u] >= 0 ? fr_cur[(size_t)ws[u] * Q + j] : 0ull;
#pragma unroll
                    for (int u = 0; u < kGatherDepth; ++u) a |= x[u];
                }
                const bool full = ((a | vw) & vm) == vm;
                if ((__ballot(full) & gmask) == gmask) {
                    p = min(p + Q, e);
                    break;
                }
            }
            if (p > e) p = e;
        } else {
            // narrow groups: four independent arcs per step
            while (p < e) {
                int32_t w[4];
                bool f[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    w[u] = p + u < e ? col[p + u] : -1;
                    f[u] = w[u] >= 0 && ((bm_cur[w[u] >> 5] >> (w[u] & 31)) & 1u);
                }
                uint64_t x[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) x[u] = f[u] ? fr_cur[(size_t)w[u] * Q + j] : 0ull;
                a |= x[0] | x[1] | x[2] | x[3];
                if (j == 0) gath += (unsigned long long)(f[0] + f[1] + f[2] + f[3]) * 8 * Q;
                p = min(p + 4, e);
                if (((p - b) & 15) == 0) {
                    const bool full = ((a | vw) & vm) == vm;
                    if ((__ballot(full) & gmask) == gmask) break;
                }
            }
        }
        if (item_split[it]) {
            const uint64_t nw = a & ~vw & vm;
            if (nw) atomicOr((unsigned long long*)&acc[at], (unsigned long long)nw);
            if ((__ballot(nw != 0ull) & gmask) != 0ull && j == 0) bytes += 8 * Q;
        } else {
            const uint64_t nw = a & ~vw & vm;
            const bool any = (__ballot(nw != 0ull) & gmask) != 0ull;
            bool fresh = false, front = false;
            if (any) {
                fresh = (__ballot(vw != 0ull) & gmask) == 0ull;
                if (nw) vis[at] = vw | nw;
                if (j == 0) bytes += (last ? 8 : 16) * Q;  // vis (+ next frontier) write
                if (!last) {
                    fr_next[at] = nw;
                    if (j == 0) atomicOr(&bm_next[u >> 5], 1u << (u & 31));
                    te += (unsigned long long)__popcll(nw) * (unsigned long long)adeg[u];
                    front = true;
                }
            }
            if (sparse) {
                const int sf = wave_append_slot(j == 0 && front, &ctl->fl_count[slot]);
                if (sf >= 0) {
                    fl_out[sf] = u;
                    fdeg += rp[u + 1] - rp[u];
                    frontier_chunks(u, rp, &ctl->fc_count[slot], fc_out);
                }
                const int sv = wave_append_slot(j == 0 && fresh && tile_first(u, bmTile), &ctl->tl_count);
                if (sv >= 0) tl[sv] = u >> 6;
            }
        }
    }
    // Counters: one atomic per block and counter.  They all sit in one cache
    // line, so atomics from every wave of a dense sweep queue up behind each
    // other and cost more than the sweep itself on small graphs.
    __shared__ unsigned long long red[5][256 / 64];
    const int wv = threadIdx.x >> 6;
    fdeg = wave_sum_ll(fdeg);
    te = (unsigned long long)wave_sum_ll((long long)te);
    arcs = (unsigned long long)wave_sum_ll((long long)arcs);
    bytes = (unsigned long long)wave_sum_ll((long long)bytes);
    gath = (unsigned long long)wave_sum_ll((long long)gath);
    if (l == 0) {
        red[0][wv] = (unsigned long long)fdeg;
        red[1][wv] = te;
        red[2][wv] = arcs;
        red[3][wv] = bytes;
        red[4][wv] = gath;
    }
    __syncthreads();
    if (threadIdx.x < 5) {
        unsigned long long v = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) v += red[threadIdx.x][w];
        if (v) {
            unsigned long long* dst[5] = {(unsigned long long*)&ctl->fdeg[slot], &st->te, &st->arcs,
                                          &st->pull_bytes, &st->pull_gather};
            atomicAdd(dst[threadIdx.x], v);
        }
    }
}

// Column popcounts of vis: cnt[j] += #{u : bit j of vis[u]}; vis is cleared on the way.
// A wave takes 64 vertices (lane = vertex) and, per word, transposes the 64x64
// bit matrix across lanes with six shuffle-and-mask steps, after which lane b
// holds bit b of all 64 vertices and one popcount counts it.
__device__ __forceinline__ uint64_t transpose64(uint64_t x, int l) {
    const uint64_t masks[6] = {0x00000000FFFFFFFFull, 0x0000FFFF0000FFFFull, 0x00FF00FF00FF00FFull,
                               0x0F0F0F0F0F0F0F0Full, 0x3333333333333333ull, 0x5555555555555555ull};
#pragma unroll
    for (int t = 0; t < 6; ++t) {
        const int sft = 32 >> t;
        const uint64_t m = masks[t];
        const uint64_t y = __shfl_xor(x, sft);
        if (l & sft) x = (x & ~m) | ((y >> sft) & m);
        else x = (x & m) | ((y & m) << sft);
    }
    return x;
}

// Column popcounts over the visited tiles (all tiles once the batch went dense),
// per segment: lanes of a tile that belong to different segments are counted in
// turns.  vis and the tile bitmap are cleared on the way.
template <int Q>
__global__ void k_ms_count(int32_t n, uint64_t* __restrict__ vis, uint32_t* __restrict__ cnt, const int* ns_dev,
                           const MsCtl* ctl, const int32_t* __restrict__ tl, uint32_t* __restrict__ bmTile,
                           const int32_t* __restrict__ seg) {
    if (ns_dev && *ns_dev == 0) return;
    const bool list = ctl->dense == 0;
    const int32_t ntiles_all = (n + 63) >> 6;
    const int32_t m = list ? ctl->tl_count : ntiles_all;
    if (!list) {
        // the tile bitmap only holds tiles of the sparse hops: sweep it
        const int32_t words = (ntiles_all + 31) >> 5;
        for (int32_t w = blockIdx.x * blockDim.x + threadIdx.x; w < words; w += gridDim.x * blockDim.x)
            bmTile[w] = 0u;
    }
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int nwaves = (gridDim.x * blockDim.x) >> 6;
    const int l = lane_id();
    uint32_t c[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) c[q] = 0;
    int gacc = -1;
    for (int32_t t = wave; t < m; t += nwaves) {
        const int32_t tile = list ? tl[t] : t;
        if (list && l == 0) bmTile[tile >> 5] = 0u;  // every bit of the word is a listed tile
        const int32_t u = (tile << 6) + l;
        uint64_t w[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) w[q] = 0ull;
        int g = -1;
        if (u < n) {
#pragma unroll
            for (int q = 0; q < Q; ++q) w[q] = vis[(size_t)u * Q + q];
#pragma unroll
            for (int q = 0; q < Q; ++q)
                if (w[q]) vis[(size_t)u * Q + q] = 0ull;
            g = seg ? seg[u] : 0;
        }
        unsigned long long rest = __ballot(u < n);
        while (rest) {
            const int g0 = __shfl(g, __ffsll((long long)rest) - 1);
            const bool in = g == g0;
            rest &= ~__ballot(in);
            if (g0 != gacc) {
                if (gacc >= 0) {
#pragma unroll
                    for (int q = 0; q < Q; ++q)
                        if (c[q]) atomicAdd(&cnt[(size_t)gacc * (64 * Q) + q * 64 + l], c[q]);
                }
#pragma unroll
                for (int q = 0; q < Q; ++q) c[q] = 0;
                gacc = g0;
            }
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const uint64_t x = in ? w[q] : 0ull;
                if (__ballot(x != 0ull) == 0ull) continue;
                c[q] += (uint32_t)__popcll(transpose64(x, l));
            }
        }
    }
    if (gacc >= 0) {
#pragma unroll
        for (int q = 0; q < Q; ++q)
            if (c[q]) atomicAdd(&cnt[(size_t)gacc * (64 * Q) + q * 64 + l], c[q]);
    }
}

// deg = count - 1 for every source; zeroes the counters it read, the per-segment
// pick counters and the batch's control block.
__global__ void k_ms_scatter(const int32_t* __restrict__ src, int ns, const int* ns_dev, int ns_cap, int Q,
                             const int32_t* __restrict__ sbit, const int32_t* __restrict__ seg, int* __restrict__ gcnt,
                             uint32_t* __restrict__ cnt, int64_t* __restrict__ deg, MsCtl* ctl, int* tcount) {
    if (ns_dev) ns = min(*ns_dev, ns_cap);
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < ns; j += gridDim.x * blockDim.x) {
        const int32_t s = src[j];
        const int bj = sbit ? sbit[j] : j;
        const int g = seg ? seg[s] : 0;
        const size_t at = (size_t)g * (64 * Q) + bj;
        deg[s] = (int64_t)cnt[at] - 1;
        cnt[at] = 0u;
        if (gcnt) gcnt[g] = 0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        for (int b = 0; b < 2; ++b) {
            ctl->fl_count[b] = 0;
            ctl->fdeg[b] = 0;
            ctl->cv_count[b] = 0;
            ctl->ci_count[b] = 0;
            ctl->fc_count[b] = 0;
        }
        ctl->tl_count = 0;
        ctl->dense = 0;
        ctl->dense_at = 0;
        *tcount = 0;
    }
}

template <int Q>
static void ms_batch_q(const MsPlanes& P, const MsItems& I, int32_t n, const int32_t* rp, const int32_t* col,
                       const uint8_t* alive, const int32_t* adeg, const int32_t* src, int ns, const int* ns_dev, int h,
                       int64_t* deg, RoundState* st, hipStream_t s) {
    const int64_t bmwords = ((int64_t)n + 31) / 32;
    const int ns_cap = P.seg ? P.ns_cap : 64 * Q;
    const int nsg = ns_dev ? ns_cap : ns;  // grid sizing
    int32_t* fl[2] = {P.flA, P.flB};
    int32_t* cv[2] = {P.cvA, P.cvB};
    int32_t* ci[2] = {P.ciA, P.ciB};
    int2* fc[2] = {P.fcA, P.fcB};
    hipLaunchKernelGGL(k_ms_init<Q>, dim3(grid_for(nsg, 256, 64)), dim3(256), 0, s, src, ns, ns_dev, ns_cap, P.sbit,
                       P.seg, P.vis, adeg, P.valid, st, P.ctl, P.tl, P.bmTile, P.exact_out);
    // hop 1: push
    hipLaunchKernelGGL(k_ms_push<Q>, dim3(grid_for((int64_t)nsg * 64, 256, 4096)), dim3(256), 0, s, src, ns, ns_dev,
                       ns_cap, P.sbit, rp, col, alive, P.acc, P.bmT, P.touched, P.touched_count, st);
    uint64_t* fr_cur = P.frA;
    uint32_t* bm_cur = P.bmA;
    uint64_t* fr_nxt = P.frB;
    uint32_t* bm_nxt = P.bmB;
    const int fin_grid = grid_for((int64_t)n * Q, 256, 8192);
    hipLaunchKernelGGL(k_ms_finalize<Q>, dim3(fin_grid), dim3(256), 0, s, P.touched, P.touched_count, 0, P.acc,
                       P.vis, fr_nxt, bm_nxt, P.valid, h == 1 ? 1 : 0, adeg, st, P.ctl, fl[1], fc[1], 1, P.tl,
                       P.bmTile, rp, P.bmT);
    const int exp_grid = grid_for((int64_t)n, 256, 2048);
    const int clr_grid = grid_for(bmwords, 256, 1024);
    for (int t = 2; t <= h; ++t) {
        std::swap(fr_cur, fr_nxt);
        std::swap(bm_cur, bm_nxt);
        const int last = t == h ? 1 : 0;
        hipLaunchKernelGGL(k_ms_expand, dim3(exp_grid), dim3(256), 0, s, fl[(t - 1) & 1], fc[(t - 1) & 1], P.ctl, t,
                           I.nnz, rp, col, alive, P.bmC, cv[t & 1], ci[t & 1], I.vitem, ns_dev);
        const int pull_grid = grid_for((int64_t)I.nitems * Q, 256, 2048);
        PullTimer* T = P.timer;
        const bool timed = T && T->used < T->cap;
        if (timed) (void)hipEventRecord(T->ev[2 * T->used], s);
        hipLaunchKernelGGL(k_ms_pull<Q>, dim3(pull_grid), dim3(256), 0, s, I.nitems, I.u, I.beg, I.end, I.split, col,
                           alive, P.vis, fr_cur, bm_cur, fr_nxt, bm_nxt, P.acc, P.valid, last, adeg, st, ns_dev,
                           ci[t & 1], P.ctl, t, fl[t & 1], fc[t & 1], P.tl, P.bmTile, rp);
        if (timed) {
            (void)hipEventRecord(T->ev[2 * T->used + 1], s);
            T->used += 1;
        }
        if (I.nsplit > 0)
            hipLaunchKernelGGL(k_ms_finalize<Q>, dim3(grid_for((int64_t)I.nsplit * Q, 256, 4096)), dim3(256), 0, s,
                               I.split_list, (const int*)nullptr, I.nsplit, P.acc, P.vis, fr_nxt, bm_nxt, P.valid,
                               last, adeg, st, P.ctl, fl[t & 1], fc[t & 1], t & 1, P.tl, P.bmTile, rp,
                               (uint32_t*)nullptr);
        hipLaunchKernelGGL(k_ms_clear, dim3(clr_grid), dim3(256), 0, s, P.ctl, t, fl[(t - 1) & 1], bm_cur, bmwords,
                           cv[t & 1], P.bmC, ns_dev);
    }
    hipLaunchKernelGGL(k_ms_count<Q>, dim3(grid_for((int64_t)n, 256, 4096)), dim3(256), 0, s, n, P.vis, P.cnt, ns_dev,
                       P.ctl, P.tl, P.bmTile, P.seg);
    hipLaunchKernelGGL(k_ms_scatter, dim3(grid_for(nsg, 256, 64)), dim3(256), 0, s, src, ns, ns_dev, ns_cap, Q, P.sbit,
                       P.seg, P.gcnt, P.cnt, deg, P.ctl, P.touched_count);
}

void ms_batch(const MsPlanes& P, const MsItems& I, int32_t n, const int32_t* rp, const int32_t* col,
              const uint8_t* alive, const int32_t* adeg, const int32_t* src, int ns, const int* ns_dev, int h,
              int64_t* deg, RoundState* st, hipStream_t s) {
    if ((!ns_dev && ns <= 0) || n <= 0) return;
    switch (P.Q) {
        case 1: ms_batch_q<1>(P, I, n, rp, col, alive, adeg, src, ns, ns_dev, h, deg, st, s); break;
        case 2: ms_batch_q<2>(P, I, n, rp, col, alive, adeg, src, ns, ns_dev, h, deg, st, s); break;
        case 4: ms_batch_q<4>(P, I, n, rp, col, alive, adeg, src, ns, ns_dev, h, deg, st, s); break;
        case 8: ms_batch_q<8>(P, I, n, rp, col, alive, adeg, src, ns, ns_dev, h, deg, st, s); break;
        default: ms_batch_q<16>(P, I, n, rp, col, alive, adeg, src, ns, ns_dev, h, deg, st, s); break;
    }
}

}  // namespace kh
