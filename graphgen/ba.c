/* Preferential-attachment edge drawing for graphgen.barabasi_albert, in C
 * because the per-vertex rejection loop is slow in Python.  It draws from the
 * same SplitMix64 stream, in the same order, as the Python loop it replaces,
 * so both give the same edge list.  Input generation only: no part of the
 * core decomposition lives here. */
#include <stdint.h>

static uint64_t mix64(uint64_t z) {
    z ^= z >> 30;
    z *= 0xBF58476D1CE4E5B9ull;
    z ^= z >> 27;
    z *= 0x94D049BB133111EBull;
    z ^= z >> 31;
    return z;
}

/* edges: room for 2 * (k (k+1) / 2 + k (n - k - 1)) int64, written as
 * (a, b) pairs: the clique K_{k+1} first, then for t = k+1 .. n-1 the k
 * distinct targets c of t as (c, t), in draw order.  Returns the pair count,
 * or -1 for k > 64 or n <= k + 1. */
int64_t gg_ba_edges(int64_t n, int32_t k, uint64_t key, int64_t *edges) {
    if (k < 1 || k > 64 || n <= k + 1) return -1;
    const uint64_t golden = 0x9E3779B97F4A7C15ull;
    int64_t *ends = edges; /* every endpoint written so far, in order */
    int64_t ne = 0, pos = 0;
    for (int64_t a = 0; a <= k; ++a)
        for (int64_t b = a + 1; b <= k; ++b) {
            ends[ne++] = a;
            ends[ne++] = b;
        }
    int64_t chosen[64];
    for (int64_t t = k + 1; t < n; ++t) {
        int nc = 0;
        while (nc < k) {
            const uint64_t x = mix64(key + (uint64_t)(pos + 1) * golden) >> 32;
            ++pos;
            const int64_t c = ends[(int64_t)(((unsigned __int128)x * (uint64_t)ne) >> 32)];
            int dup = 0;
            for (int j = 0; j < nc; ++j) dup |= chosen[j] == c;
            if (!dup) chosen[nc++] = c;
        }
        for (int j = 0; j < nc; ++j) {
            ends[ne++] = chosen[j];
            ends[ne++] = t;
        }
    }
    return ne / 2;
}
