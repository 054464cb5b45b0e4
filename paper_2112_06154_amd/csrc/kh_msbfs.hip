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
#include "kh_common.hpp"
#include "kh_internal.hpp"

namespace kh {

template <int Q>
__global__ void k_ms_init(const int32_t* __restrict__ src, int ns, const int* ns_dev, uint64_t* __restrict__ vis,
                          const int32_t* __restrict__ adeg, uint64_t* __restrict__ valid, RoundState* st) {
    if (ns_dev) ns = min(*ns_dev, 64 * Q);
    unsigned long long te = 0;
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < ns; j += gridDim.x * blockDim.x) {
        const int32_t s = src[j];
        vis[(size_t)s * Q + (j >> 6)] = 1ull << (j & 63);
        te += (unsigned long long)adeg[s];
    }
    if (blockIdx.x == 0 && threadIdx.x < Q) {
        const int c = ns - 64 * (int)threadIdx.x;
        valid[threadIdx.x] = c >= 64 ? ~0ull : (c <= 0 ? 0ull : ((1ull << c) - 1ull));
    }
    te = (unsigned long long)wave_sum_ll((long long)te);
    if (lane_id() == 0 && te) atomicAdd(&st->te, te);
}

// Hop 1: push the sources' bits to their alive neighbours.
template <int Q>
__global__ void k_ms_push(const int32_t* __restrict__ src, int ns, const int* ns_dev, const int32_t* __restrict__ rp,
                          const int32_t* __restrict__ col, const uint8_t* __restrict__ alive,
                          uint64_t* __restrict__ acc, uint32_t* __restrict__ bmT, int32_t* __restrict__ touched,
                          int* tcount, RoundState* st) {
    if (ns_dev) ns = min(*ns_dev, 64 * Q);
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int nwaves = (gridDim.x * blockDim.x) >> 6;
    const int l = lane_id();
    unsigned long long arcs = 0;
    for (int j = wave; j < ns; j += nwaves) {
        const int32_t s = src[j];
        const uint64_t bit = 1ull << (j & 63);
        const int word = j >> 6;
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

// new = acc & ~vis for listed vertices (the pushed ones, or the split ones after a pull).
template <int Q>
__global__ void k_ms_finalize(const int32_t* __restrict__ list, const int* count_p, int count_i,
                              uint64_t* __restrict__ acc, uint64_t* __restrict__ vis, uint64_t* __restrict__ fr_next,
                              uint32_t* __restrict__ bm_next, const uint64_t* __restrict__ valid, int last,
                              const int32_t* __restrict__ adeg, RoundState* st) {
    const int cnt = count_p ? *count_p : count_i;
    const int l = lane_id();
    const int j = l % Q;
    const int gbase = l - j;
    const unsigned long long gmask = (Q == 64 ? ~0ull : ((1ull << Q) - 1ull)) << gbase;
    const int gpb = blockDim.x / Q;
    const int ngroups = gridDim.x * gpb;
    const uint64_t vm = valid[j];
    unsigned long long te = 0;
    for (int idx = blockIdx.x * gpb + threadIdx.x / Q; idx < cnt; idx += ngroups) {
        const int32_t u = list[idx];
        const size_t at = (size_t)u * Q + j;
        const uint64_t a = acc[at];
        if (a) acc[at] = 0ull;
        const uint64_t vw = vis[at];
        const uint64_t nw = a & ~vw & vm;
        const bool any = (__ballot(nw != 0ull) & gmask) != 0ull;
        if (any) {
            if (nw) vis[at] = vw | nw;
            if (!last) {
                fr_next[at] = nw;
                if (j == 0) atomicOr(&bm_next[u >> 5], 1u << (u & 31));
                te += (unsigned long long)__popcll(nw) * (unsigned long long)adeg[u];
            }
        }
    }
    te = (unsigned long long)wave_sum_ll((long long)te);
    if (l == 0 && te) atomicAdd(&st->te, te);
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
                                                 const int* ns_dev) {
    if (ns_dev && *ns_dev == 0) return;
    const int l = lane_id();
    const int j = l % Q;
    const int gbase = l - j;
    const unsigned long long gmask = (Q == 64 ? ~0ull : ((1ull << Q) - 1ull)) << gbase;
    const int gpb = blockDim.x / Q;
    const int ngroups = gridDim.x * gpb;
    const uint64_t vm = valid[j];
    unsigned long long te = 0, arcs = 0, bytes = 0, gath = 0;
    for (int it = blockIdx.x * gpb + threadIdx.x / Q; it < nitems; it += ngroups) {
        const int32_t u = item_u[it];
        if (j == 0) bytes += 14;  // item (u, beg, end, split) and alive[u]
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
                    int32_t ws[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        ws[u] = -1;
                        if (fm) {
                            const int k = __ffsll((long long)fm) - 1;
                            fm &= fm - 1ull;
                            ws[u] = __shfl(w, gbase + k);
                        }
                    }
                    uint64_t x[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) x[u] = ws[u] >= 0 ? fr_cur[(size_t)ws[u] * Q + j] : 0ull;
                    a |= x[0] | x[1] | x[2] | x[3];
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
            if (any) {
                if (nw) vis[at] = vw | nw;
                if (j == 0) bytes += (last ? 8 : 16) * Q;  // vis (+ next frontier) write
                if (!last) {
                    fr_next[at] = nw;
                    if (j == 0) atomicOr(&bm_next[u >> 5], 1u << (u & 31));
                    te += (unsigned long long)__popcll(nw) * (unsigned long long)adeg[u];
                }
            }
        }
    }
    te = (unsigned long long)wave_sum_ll((long long)te);
    arcs = (unsigned long long)wave_sum_ll((long long)arcs);
    bytes = (unsigned long long)wave_sum_ll((long long)bytes);
    gath = (unsigned long long)wave_sum_ll((long long)gath);
    if (l == 0) {
        if (te) atomicAdd(&st->te, te);
        if (arcs) atomicAdd(&st->arcs, arcs);
        if (bytes) atomicAdd(&st->pull_bytes, bytes);
        if (gath) atomicAdd(&st->pull_gather, gath);
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

template <int Q>
__global__ void k_ms_count(int32_t n, uint64_t* __restrict__ vis, uint32_t* __restrict__ cnt, const int* ns_dev) {
    if (ns_dev && *ns_dev == 0) return;
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int nwaves = (gridDim.x * blockDim.x) >> 6;
    const int l = lane_id();
    uint32_t c[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) c[q] = 0;
    const int32_t ntiles = (n + 63) >> 6;
    for (int32_t t = wave; t < ntiles; t += nwaves) {
        const int32_t u = (t << 6) + l;
        uint64_t w[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) w[q] = 0ull;
        if (u < n) {
#pragma unroll
            for (int q = 0; q < Q; ++q) w[q] = vis[(size_t)u * Q + q];
#pragma unroll
            for (int q = 0; q < Q; ++q)
                if (w[q]) vis[(size_t)u * Q + q] = 0ull;
        }
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            if (__ballot(w[q] != 0ull) == 0ull) continue;
            c[q] += (uint32_t)__popcll(transpose64(w[q], l));
        }
    }
#pragma unroll
    for (int q = 0; q < Q; ++q)
        if (c[q]) atomicAdd(&cnt[q * 64 + l], c[q]);
}

__global__ void k_ms_scatter(const int32_t* __restrict__ src, int ns, const int* ns_dev, int qmax,
                             uint32_t* __restrict__ cnt, int64_t* __restrict__ deg) {
    if (ns_dev) ns = min(*ns_dev, 64 * qmax);
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < ns; j += gridDim.x * blockDim.x) {
        deg[src[j]] = (int64_t)cnt[j] - 1;
        cnt[j] = 0u;
    }
}

template <int Q>
static void ms_batch_q(const MsPlanes& P, const MsItems& I, int32_t n, const int32_t* rp, const int32_t* col,
                       const uint8_t* alive, const int32_t* adeg, const int32_t* src, int ns, const int* ns_dev, int h,
                       int64_t* deg, RoundState* st, hipStream_t s) {
    const int64_t bmwords = ((int64_t)n + 31) / 32;
    const int nsg = ns_dev ? 64 * Q : ns;  // grid sizing
    hipLaunchKernelGGL(k_ms_init<Q>, dim3(grid_for(nsg, 256, 64)), dim3(256), 0, s, src, ns, ns_dev, P.vis, adeg,
                       P.valid, st);
    // hop 1: push
    launch_fill_u32(P.bmT, 0u, bmwords, s);
    launch_set_int(P.touched_count, 0, s);
    hipLaunchKernelGGL(k_ms_push<Q>, dim3(grid_for((int64_t)nsg * 64, 256, 4096)), dim3(256), 0, s, src, ns, ns_dev,
                       rp, col, alive, P.acc, P.bmT, P.touched, P.touched_count, st);
    uint64_t* fr_cur = P.frA;
    uint32_t* bm_cur = P.bmA;
    uint64_t* fr_nxt = P.frB;
    uint32_t* bm_nxt = P.bmB;
    launch_fill_u32(bm_nxt, 0u, bmwords, s);
    const int fin_grid = grid_for((int64_t)n * Q, 256, 8192);
    hipLaunchKernelGGL(k_ms_finalize<Q>, dim3(fin_grid), dim3(256), 0, s, P.touched, P.touched_count, 0, P.acc,
                       P.vis, fr_nxt, bm_nxt, P.valid, h == 1 ? 1 : 0, adeg, st);
    for (int t = 2; t <= h; ++t) {
        std::swap(fr_cur, fr_nxt);
        std::swap(bm_cur, bm_nxt);
        const int last = t == h ? 1 : 0;
        if (!last) launch_fill_u32(bm_nxt, 0u, bmwords, s);
        const int pull_grid = grid_for((int64_t)I.nitems * Q, 256, 16384);
        PullTimer* T = P.timer;
        const bool timed = T && T->used < T->cap;
        if (timed) (void)hipEventRecord(T->ev[2 * T->used], s);
        hipLaunchKernelGGL(k_ms_pull<Q>, dim3(pull_grid), dim3(256), 0, s, I.nitems, I.u, I.beg, I.end, I.split, col,
                           alive, P.vis, fr_cur, bm_cur, fr_nxt, bm_nxt, P.acc, P.valid, last, adeg, st, ns_dev);
        if (timed) {
            (void)hipEventRecord(T->ev[2 * T->used + 1], s);
            T->used += 1;
        }
        if (I.nsplit > 0)
            hipLaunchKernelGGL(k_ms_finalize<Q>, dim3(grid_for((int64_t)I.nsplit * Q, 256, 4096)), dim3(256), 0, s,
                               I.split_list, (const int*)nullptr, I.nsplit, P.acc, P.vis, fr_nxt, bm_nxt, P.valid,
                               last, adeg, st);
    }
    hipLaunchKernelGGL(k_ms_count<Q>, dim3(grid_for((int64_t)n, 256, 4096)), dim3(256), 0, s, n, P.vis, P.cnt, ns_dev);
    hipLaunchKernelGGL(k_ms_scatter, dim3(grid_for(nsg, 256, 64)), dim3(256), 0, s, src, ns, ns_dev, Q, P.cnt, deg);
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
