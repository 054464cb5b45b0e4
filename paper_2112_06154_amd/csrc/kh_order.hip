// Deletion order of the bulk-round peel, for Alg. 7's suffix candidates.
//
// The peel deletes R_1, R_2, ... in rounds; inside a round the order is by the
// key at deletion (the estimate d, or deg_h for ExactCore), then by k[v,h] (the
// tie key Alg. 4 names), then by id.  Every core set {c >= K} is a suffix of
// this order.  The order is a lexicographic sort of (round, key, level, id),
// done as two stable radix sorts: first by level (ids enter in ascending
// order), then by (round << 32 | key).
#include <hipcub/hipcub.hpp>

#include "kh_common.hpp"
#include "kh_internal.hpp"

namespace kh {

namespace {

__global__ void k_order_init(int32_t n, const uint8_t* __restrict__ lev, uint32_t* __restrict__ lkey,
                             int32_t* __restrict__ ids) {
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        lkey[v] = lev ? lev[v] : 0u;
        ids[v] = v;
    }
}

__global__ void k_order_major(int32_t n, const int32_t* __restrict__ ids, const int32_t* __restrict__ rnd,
                              const int64_t* __restrict__ key, uint64_t* __restrict__ mkey, int* bad) {
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int32_t v = ids[i];
        const long long r = rnd[v];
        const long long k = key[v];
        if (r < 0 || k < 0 || k > 0xFFFFFFFFll) atomicOr(bad, 1);
        mkey[i] = ((unsigned long long)(r < 0 ? 0 : r) << 32) | (unsigned long long)(k < 0 ? 0 : (k & 0xFFFFFFFFll));
    }
}

__global__ void k_order_pos(int32_t n, const int32_t* __restrict__ order, int64_t* __restrict__ pos) {
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) pos[order[i]] = i;
}

}  // namespace

size_t order_temp_bytes(int32_t n) {
    size_t a = 0, b = 0;
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, a, (const uint32_t*)nullptr, (uint32_t*)nullptr,
                                             (const int32_t*)nullptr, (int32_t*)nullptr, n, 0, 8);
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, b, (const uint64_t*)nullptr, (uint64_t*)nullptr,
                                             (const int32_t*)nullptr, (int32_t*)nullptr, n, 0, 64);
    return a > b ? a : b;
}

hipError_t deletion_order(int32_t n, const int32_t* rnd, const int64_t* key, const uint8_t* lev, OrderScratch w,
                          int32_t* order, int64_t* pos, int* bad, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int grid = grid_for(n, 256, 8192);
    hipLaunchKernelGGL(k_order_init, dim3(grid), dim3(256), 0, s, n, lev, w.lkey, w.ids);
    size_t tb = w.temp_bytes;
    hipError_t e = hipcub::DeviceRadixSort::SortPairs(w.temp, tb, w.lkey, w.lkey_out, w.ids, w.ids_out, n, 0, 8, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_order_major, dim3(grid), dim3(256), 0, s, n, w.ids_out, rnd, key, w.mkey, bad);
    tb = w.temp_bytes;
    e = hipcub::DeviceRadixSort::SortPairs(w.temp, tb, w.mkey, w.mkey_out, w.ids_out, order, n, 0, 64, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_order_pos, dim3(grid), dim3(256), 0, s, n, order, pos);
    return hipGetLastError();
}

}  // namespace kh
