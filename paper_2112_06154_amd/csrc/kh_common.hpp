// Device helpers shared by the gfx950 kernels (wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace kh {

constexpr int kWave = 64;

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Wave-aggregated append: every lane with `want` gets a distinct slot of
// out[*count ...]; one atomic per wave.
__device__ __forceinline__ int wave_append_slot(bool want, int* count) {
    unsigned long long m = __ballot(want);
    if (m == 0ull) return -1;
    int leader = __ffsll((long long)m) - 1;
    int base = 0;
    if (lane_id() == leader) base = atomicAdd(count, __popcll(m));
    base = __shfl(base, leader);
    if (!want) return -1;
    unsigned long long below = m & ((1ull << lane_id()) - 1ull);
    return base + __popcll(below);
}

__device__ __forceinline__ long long wave_sum_ll(long long v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ __forceinline__ long long wave_min_ll(long long v) {
    for (int o = 32; o > 0; o >>= 1) {
        long long t = __shfl_xor(v, o);
        v = t < v ? t : v;
    }
    return v;
}
__device__ __forceinline__ int wave_sum_i(int v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ __forceinline__ int wave_max_i(int v) {
    for (int o = 32; o > 0; o >>= 1) {
        int t = __shfl_xor(v, o);
        v = t > v ? t : v;
    }
    return v;
}
// Inclusive prefix sum across the wave.
__device__ __forceinline__ int wave_incl_scan(int v) {
    const int l = lane_id();
    for (int o = 1; o < 64; o <<= 1) {
        int t = __shfl_up(v, o);
        if (l >= o) v += t;
    }
    return v;
}

__device__ __forceinline__ uint32_t sample_key(int rank, int32_t v) {
    return ((uint32_t)(255 - rank) << 24) | (uint32_t)v;
}
__device__ __forceinline__ int key_rank(uint32_t key) { return 255 - (int)(key >> 24); }

inline int grid_for(long long items, int per_block, int cap = 65535 * 4) {
    long long g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

}  // namespace kh
