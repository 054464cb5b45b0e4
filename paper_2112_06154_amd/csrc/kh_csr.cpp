// Host-only helpers of the C ABI: status names, Eq. (buffer) (Sec. 3), and the
// CSR checks of the graph conventions (Sec. 2: simple undirected graphs).  No
// HIP here: the same source builds into the library and, with host
// sanitizers, into the sanitizer test driver.
#include "kh_csr.hpp"

#include <algorithm>
#include <cmath>
#include <utility>

using namespace kh;

extern "C" const char* kh_status_str(kh_status s) {
    switch (s) {
        case KH_OK: return "KH_OK";
        case KH_EINVAL: return "KH_EINVAL: invalid argument";
        case KH_ENOMEM: return "KH_ENOMEM: out of device memory or HBM budget";
        case KH_EDEVICE: return "KH_EDEVICE: GPU unavailable or HIP error";
        case KH_EGRAPH: return "KH_EGRAPH: CSR is not a canonical simple undirected graph";
        case KH_EOVERFLOW: return "KH_EOVERFLOW: value does not fit int32";
        case KH_EBUSY: return "KH_EBUSY: request still running";
        case KH_ENOTFOUND: return "KH_ENOTFOUND: unknown ticket";
        case KH_ENOTIMPL: return "KH_ENOTIMPL: parameters outside what this library supports";
        default: return "unknown kh_status";
    }
}

// Eq. (buffer), Sec. 3: C = log(2n/delta) (Alg. 4) or log(n^2/delta) (Alg. 7).
extern "C" int64_t kh_buffer_size(int64_t n, double epsilon, double delta, int32_t dense) {
    if (n < 1 || !(epsilon > 0.0) || !(delta > 0.0 && delta < 1.0)) return -1;
    const double C = dense ? std::log((double)n * (double)n / delta) : std::log(2.0 * (double)n / delta);
    const double M = 1.0 + 4.0 * (2.0 + epsilon) / (epsilon * epsilon) * (C + std::log(8.0));
    if (!(M < 9.0e18)) return INT64_MAX;
    return (int64_t)std::floor(M);
}

extern "C" kh_status kh_validate_csr(int32_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col) {
    if (n < 0 || nnz < 0 || nnz > kMaxArcs) return KH_EINVAL;
    if (!row_ptr || (nnz > 0 && !col)) return KH_EINVAL;
    if (row_ptr[0] != 0 || (int64_t)row_ptr[n] != nnz) return KH_EGRAPH;
    for (int32_t v = 0; v < n; ++v) {
        const int32_t a = row_ptr[v], b = row_ptr[v + 1];
        if (a > b || a < 0 || (int64_t)b > nnz) return KH_EGRAPH;
        for (int32_t p = a; p < b; ++p) {
            const int32_t w = col[p];
            if (w < 0 || w >= n || w == v) return KH_EGRAPH;
            if (p > a && col[p - 1] >= w) return KH_EGRAPH;
        }
    }
    for (int32_t v = 0; v < n; ++v) {
        for (int32_t p = row_ptr[v]; p < row_ptr[v + 1]; ++p) {
            const int32_t w = col[p];
            const int32_t* lo = col + row_ptr[w];
            const int32_t* hi = col + row_ptr[w + 1];
            const int32_t* it = std::lower_bound(lo, hi, v);
            if (it == hi || *it != v) return KH_EGRAPH;
        }
    }
    return KH_OK;
}

namespace kh {

kh_status canonicalize_csr(int32_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col,
                           std::vector<int32_t>& rp, std::vector<int32_t>& cl) {
    if (n < 0 || nnz < 0 || nnz > kMaxArcs) return KH_EINVAL;
    if (!row_ptr || (nnz > 0 && !col)) return KH_EINVAL;
    // row_ptr must be a CSR of nnz arcs before any col entry is read
    if (row_ptr[0] != 0 || (int64_t)row_ptr[n] != nnz) return KH_EGRAPH;
    for (int32_t v = 0; v < n; ++v)
        if (row_ptr[v] > row_ptr[v + 1]) return KH_EGRAPH;
    std::vector<std::pair<int32_t, int32_t>> arcs;
    arcs.reserve((size_t)nnz * 2);
    for (int32_t v = 0; v < n; ++v) {
        for (int32_t p = row_ptr[v]; p < row_ptr[v + 1]; ++p) {
            const int32_t w = col[p];
            if (w < 0 || w >= n) return KH_EGRAPH;
            if (w == v) continue;
            arcs.emplace_back(v, w);
            arcs.emplace_back(w, v);
        }
    }
    std::sort(arcs.begin(), arcs.end());
    arcs.erase(std::unique(arcs.begin(), arcs.end()), arcs.end());
    if ((int64_t)arcs.size() > kMaxArcs) return KH_EINVAL;
    rp.assign((size_t)n + 1, 0);
    cl.resize(arcs.size());
    for (size_t i = 0; i < arcs.size(); ++i) {
        rp[(size_t)arcs[i].first + 1]++;
        cl[i] = arcs[i].second;
    }
    for (int32_t v = 0; v < n; ++v) rp[(size_t)v + 1] += rp[(size_t)v];
    return KH_OK;
}

}  // namespace kh
