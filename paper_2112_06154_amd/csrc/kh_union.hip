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

#include "kh_common.hpp"
#include "kh_internal.hpp"

namespace kh {

__global__ void k_cap_level1(const int32_t* __restrict__ rp, int32_t n, int32_t M, int64_t* __restrict__ cap) {
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        const int64_t c = 1 + (int64_t)(rp[v + 1] - rp[v]);
        cap[v] = c < M ? c : M;
    }
}
void launch_cap_level1(const int32_t* rp, int32_t n, int32_t M, int64_t* cap, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_cap_level1, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, rp, n, M, cap);
}

// cap_i(v) = min(M, 1 + sum_w cap_{i-1}(w)) bounds |B[v,i]| for every X.
__global__ void k_cap_next(const int32_t* __restrict__ rp, const int32_t* __restrict__ col, int32_t n, int32_t M,
                           const int64_t* __restrict__ cap_prev, int64_t* __restrict__ cap) {
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int nwaves = (gridDim.x * blockDim.x) >> 6;
    const int l = lane_id();
    for (int32_t v = wave; v < n; v += nwaves) {
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
void launch_cap_next(const int32_t* rp, const int32_t* col, int32_t n, int32_t M, const int64_t* cap_prev,
                     int64_t* cap, hipStream_t s) {
    if (n > 0)
        hipLaunchKernelGGL(k_cap_next, dim3(grid_for((int64_t)n * 64, 256, 16384)), dim3(256), 0, s, rp, col, n, M,
                           cap_prev, cap);
}

// ---- level 1: T = {v} + alive neighbours (all distinct) -------------------------------------
__global__ __launch_bounds__(256) void k_union1(const int32_t* __restrict__ worklist, const int* wl_count, int32_t n,
                                                const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                const uint8_t* __restrict__ alive, const uint8_t* __restrict__ rank,
                                                int32_t M, const int64_t* __restrict__ off, uint32_t* __restrict__ keys,
                                                int32_t* __restrict__ size, uint8_t* __restrict__ kk,
                                                int32_t* __restrict__ changed, int* changed_count, RoundState* st) {
    __shared__ int hist[256];
    __shared__ int s_k, s_size;
    const int tid = threadIdx.x;
    const int total = worklist ? *wl_count : n;
    unsigned long long elems = 0;
    for (int wi = blockIdx.x; wi < total; wi += gridDim.x) {
        const int32_t v = worklist ? worklist[wi] : wi;
        if (!alive[v]) continue;
        const int32_t b = rp[v], e = rp[v + 1];
        hist[tid] = 0;
        __syncthreads();
        for (int32_t p = b + tid; p < e; p += blockDim.x) {
            const int32_t w = col[p];
            if (alive[w]) atomicAdd(&hist[rank[w]], 1);
        }
        elems += (unsigned long long)((e - b + (int)blockDim.x - 1 - tid) / (int)blockDim.x);
        if (tid == 0) atomicAdd(&hist[rank[v]], 1);
        __syncthreads();
        if (tid == 0) {
            // k = smallest level whose suffix count is <= M
            int run = 0, k = 0;
            for (int L = 255; L >= 0; --L) {
                if (run + hist[L] > M) {
                    k = L + 1;
                    break;
                }
                run += hist[L];
            }
            run = 0;
            for (int L = 255; L >= k; --L) {
                const int c = hist[L];
                hist[L] = run;  // becomes the write cursor of rank group L
                run += c;
            }
            s_k = k;
            s_size = run;
        }
        __syncthreads();
        const int k = s_k;
        uint32_t* out = keys + off[v];
        for (int32_t p = b + tid; p < e; p += blockDim.x) {
            const int32_t w = col[p];
            if (alive[w]) {
                const int rw = rank[w];
                if (rw >= k) out[atomicAdd(&hist[rw], 1)] = sample_key(rw, w);
            }
        }
        if (tid == 0) {
            const int rv = rank[v];
            if (rv >= k) out[atomicAdd(&hist[rv], 1)] = sample_key(rv, v);
            const int ok = kk[v], os = size[v];
            size[v] = s_size;
            kk[v] = (uint8_t)k;
            if (changed && (ok != k || os != s_size)) changed[atomicAdd(changed_count, 1)] = v;
        }
        __syncthreads();
    }
    elems = (unsigned long long)wave_sum_ll((long long)elems);
    if (lane_id() == 0 && elems) atomicAdd(&st->elems, elems);
}

void launch_union1(const int32_t* worklist, const int* wl_count, int32_t n, const int32_t* rp, const int32_t* col,
                   const uint8_t* alive, const uint8_t* rank, int32_t M, const int64_t* off, uint32_t* keys,
                   int32_t* size, uint8_t* kk, int32_t* changed, int* changed_count, RoundState* st, hipStream_t s) {
    if (n <= 0) return;
    const int grid = worklist ? 4096 : grid_for(n, 1, 16384);
    hipLaunchKernelGGL(k_union1, dim3(grid), dim3(256), 0, s, worklist, wl_count, n, rp, col, alive, rank, M, off, keys,
                       size, kk, changed, changed_count, st);
}

// ---- levels i >= 2 ----------------------------------------------------------------------
struct HashSet {
    uint32_t* tab;
    uint32_t mask;
    int shift;
    int* count;
    int* hist;
    int* over;
    int M;
};

__device__ __forceinline__ void hs_insert(const HashSet& H, uint32_t key) {
    uint32_t h = (key * 2654435761u) >> H.shift;
    for (;;) {
        const uint32_t old = atomicCAS(&H.tab[h], kEmptyKey, key);
        if (old == kEmptyKey) {
            const int c = atomicAdd(H.count, 1) + 1;
            atomicAdd(&H.hist[key_rank(key)], 1);
            if (c > H.M) *(volatile int*)H.over = 1;
            return;
        }
        if (old == key) return;
        h = (h + 1u) & H.mask;
    }
}

__global__ __launch_bounds__(256) void k_union(const int32_t* __restrict__ worklist, const int* wl_count, int32_t n,
                                               const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                                               const uint8_t* __restrict__ alive, const uint8_t* __restrict__ rank,
                                               int32_t M, int hash_log2, const int64_t* __restrict__ off_prev,
                                               const uint32_t* __restrict__ keys_prev,
                                               const int32_t* __restrict__ size_prev,
                                               const uint8_t* __restrict__ k_prev, const int64_t* __restrict__ off,
                                               uint32_t* __restrict__ keys, int32_t* __restrict__ size,
                                               uint8_t* __restrict__ kk, int32_t* __restrict__ cursor,
                                               int32_t* __restrict__ changed, int* changed_count, RoundState* st) {
    extern __shared__ uint32_t tab[];
    __shared__ int hist[256];
    __shared__ int s_kmax, s_htop, s_count, s_over, s_k, s_size;
    const int tid = threadIdx.x;
    const int bs = blockDim.x;
    const int hcap = 1 << hash_log2;
    HashSet H{tab, (uint32_t)(hcap - 1), 32 - hash_log2, &s_count, hist, &s_over, M};
    const int total = worklist ? *wl_count : n;
    unsigned long long elems = 0;
    for (int wi = blockIdx.x; wi < total; wi += gridDim.x) {
        const int32_t v = worklist ? worklist[wi] : wi;
        if (!alive[v]) continue;
        const int32_t b = rp[v], e = rp[v + 1];
        for (int t = tid; t < hcap; t += bs) tab[t] = kEmptyKey;
        hist[tid] = 0;
        if (tid == 0) {
            s_kmax = 0;
            s_htop = rank[v];
            s_count = 0;
            s_over = 0;
        }
        __syncthreads();
        int kmax_l = 0, htop_l = -1;
        for (int32_t p = b + tid; p < e; p += bs) {
            const int32_t w = col[p];
            cursor[p] = 0;
            if (alive[w]) {
                const int kw = k_prev[w];
                kmax_l = kw > kmax_l ? kw : kmax_l;
                if (size_prev[w] > 0) {
                    const int hr = key_rank(keys_prev[off_prev[w]]);
                    htop_l = hr > htop_l ? hr : htop_l;
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
        const int kmax = s_kmax;
        int k = kmax;
        for (int L = s_htop; L >= kmax; --L) {
            for (int32_t p = b + tid; p < e; p += bs) {
                const int32_t w = col[p];
                if (!alive[w]) continue;
                int c = cursor[p];
                const int sz = size_prev[w];
                if (c >= sz) continue;
                const uint32_t* lst = keys_prev + off_prev[w];
                const int c0 = c;
                while (c < sz) {
                    const uint32_t key = lst[c];
                    if (key_rank(key) != L) break;
                    ++c;
                    // once more than M distinct keys are in, rank L is cut anyway; each
                    // thread inserts at most one key after that, so the table stays half empty
                    if (*(volatile int*)&s_count <= M) hs_insert(H, key);
                }
                elems += (unsigned long long)(c - c0 + 1);
                if (c != c0) cursor[p] = c;
            }
            if (tid == 0 && rank[v] == L && *(volatile int*)&s_count <= M) hs_insert(H, sample_key(L, v));
            __syncthreads();
            const int over = s_over;
            __syncthreads();
            if (over) {
                k = L + 1;
                break;
            }
        }
        if (tid == 0) {
            int run = 0;
            for (int L = 255; L >= k; --L) {
                const int c = hist[L];
                hist[L] = run;
                run += c;
            }
            s_k = k;
            s_size = run;
        }
        __syncthreads();
        uint32_t* out = keys + off[v];
        for (int t = tid; t < hcap; t += bs) {
            const uint32_t key = tab[t];
            if (key != kEmptyKey) {
                const int rk = key_rank(key);
                if (rk >= k) out[atomicAdd(&hist[rk], 1)] = key;
            }
        }
        if (tid == 0) {
            const int ok = kk[v], os = size[v];
            size[v] = s_size;
            kk[v] = (uint8_t)s_k;
            if (changed && (ok != s_k || os != s_size)) changed[atomicAdd(changed_count, 1)] = v;
        }
        __syncthreads();
    }
    elems = (unsigned long long)wave_sum_ll((long long)elems);
    if (lane_id() == 0 && elems) atomicAdd(&st->elems, elems);
}

void launch_union(const int32_t* worklist, const int* wl_count, int32_t n, const int32_t* rp, const int32_t* col,
                  const uint8_t* alive, const uint8_t* rank, int32_t M, int hash_log2, const int64_t* off_prev,
                  const uint32_t* keys_prev, const int32_t* size_prev, const uint8_t* k_prev, const int64_t* off,
                  uint32_t* keys, int32_t* size, uint8_t* kk, int32_t* cursor, int32_t* changed, int* changed_count,
                  RoundState* st, hipStream_t s) {
    if (n <= 0) return;
    const int grid = worklist ? 4096 : grid_for(n, 1, 16384);
    const size_t lds = sizeof(uint32_t) << hash_log2;
    static size_t lds_set = 65536;
    if (lds > lds_set) {
        (void)hipFuncSetAttribute((const void*)k_union, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        lds_set = lds;
    }
    hipLaunchKernelGGL(k_union, dim3(grid), dim3(kUnionThreads), lds, s, worklist, wl_count, n, rp, col, alive, rank,
                       M, hash_log2, off_prev, keys_prev, size_prev, k_prev, off, keys, size, kk, cursor, changed,
                       changed_count, st);
}

// ---- Alg. 1: d = |B[v,h] \ {v}| 2^k, and max(d, M 2^(k-1)) when k > 0 ---------------------------
__global__ void k_estimate(const int32_t* __restrict__ worklist, const int* wl_count, int32_t n,
                           const uint8_t* __restrict__ alive, const uint8_t* __restrict__ rank,
                           const int32_t* __restrict__ size, const uint8_t* __restrict__ kk, int32_t M,
                           int64_t* __restrict__ d, RoundState* st) {
    const int total = worklist ? *wl_count : n;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
        const int32_t v = worklist ? worklist[i] : i;
        if (!alive[v]) continue;
        const int k = kk[v];
        const long long T = (long long)size[v] - (rank[v] >= k ? 1 : 0);
        long long est;
        if (k >= 62 || (T > 0 && T > (LLONG_MAX >> k))) {
            atomicOr(&st->overflow, 1);
            est = LLONG_MAX;
        } else {
            est = T << k;
            if (k > 0) {
                const long long fl = (long long)M << (k - 1);
                est = fl > est ? fl : est;
            }
        }
        d[v] = est;
    }
}
void launch_estimate(const int32_t* worklist, const int* wl_count, int32_t n, const uint8_t* alive,
                     const uint8_t* rank, const int32_t* size, const uint8_t* kk, int32_t M, int64_t* d,
                     RoundState* st, hipStream_t s) {
    if (n <= 0) return;
    const int grid = worklist ? 1024 : grid_for(n, 256, 8192);
    hipLaunchKernelGGL(k_estimate, dim3(grid), dim3(256), 0, s, worklist, wl_count, n, alive, rank, size, kk, M, d,
                       st);
}

}  // namespace kh
