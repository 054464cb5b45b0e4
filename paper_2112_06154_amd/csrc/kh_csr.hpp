// Host-only CSR helpers of the C ABI (no HIP): status names, Eq. (buffer), CSR
// validation and canonicalisation.  Kept apart from the GPU engine so that the
// same source also builds with host sanitizers.
#pragma once

#include <climits>
#include <cstdint>
#include <vector>

#include "../../include/khcore.h"

namespace kh {

// Arc indices are int32 in the kernels, which step through arc ranges in
// chunks (at most a hub slice, 2^23 arcs) that may end past the last arc:
// graphs and packed unions hold at most this many arcs so none overflows.
constexpr int64_t kMaxArcs = (int64_t)INT32_MAX - ((int64_t)1 << 24);

// The canonical simple undirected graph of an arbitrary CSR (Sec. 2): loops
// dropped, both directions of every arc, duplicates merged, adjacency sorted.
// KH_EGRAPH when row_ptr is not a CSR of n vertices and nnz arcs or an id is
// out of range, KH_EINVAL when the result would exceed kMaxArcs arcs.
kh_status canonicalize_csr(int32_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col,
                           std::vector<int32_t>& rp, std::vector<int32_t>& cl);

}  // namespace kh
