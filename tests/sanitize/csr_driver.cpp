// Drives the library's host-only CSR helpers (paper_2112_06154_amd/csrc/kh_csr.cpp)
// over valid, malformed and hostile inputs.  Built by tests/test_sanitizers.py
// with AddressSanitizer and UndefinedBehaviorSanitizer; exits non-zero on the
// first wrong answer (the sanitizers abort on any memory or UB error).
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <random>
#include <set>
#include <utility>
#include <vector>

#include "../../paper_2112_06154_amd/csrc/kh_csr.hpp"

namespace {

int failures = 0;

void expect(bool ok, const char* what, int i) {
    if (!ok) {
        std::fprintf(stderr, "FAIL %s (case %d)\n", what, i);
        ++failures;
    }
}

// reference: the canonical simple graph of a list of arcs
void reference(int32_t n, const std::vector<std::pair<int32_t, int32_t>>& arcs, std::vector<int32_t>& rp,
               std::vector<int32_t>& col) {
    std::set<std::pair<int32_t, int32_t>> s;
    for (auto [u, v] : arcs)
        if (u != v) {
            s.insert({u, v});
            s.insert({v, u});
        }
    rp.assign((size_t)n + 1, 0);
    col.clear();
    for (auto [u, v] : s) {
        rp[(size_t)u + 1]++;
        col.push_back(v);
    }
    for (int32_t v = 0; v < n; ++v) rp[(size_t)v + 1] += rp[(size_t)v];
}

void csr_of(int32_t n, const std::vector<std::pair<int32_t, int32_t>>& arcs, std::vector<int32_t>& rp,
            std::vector<int32_t>& col) {
    // arcs as given (any order inside a row), rows by source
    std::vector<std::vector<int32_t>> adj((size_t)n);
    for (auto [u, v] : arcs) adj[(size_t)u].push_back(v);
    rp.assign((size_t)n + 1, 0);
    col.clear();
    for (int32_t v = 0; v < n; ++v) {
        for (int32_t w : adj[(size_t)v]) col.push_back(w);
        rp[(size_t)v + 1] = (int32_t)col.size();
    }
}

}  // namespace

int main() {
    std::mt19937_64 rng(12345);
    // 1. random multigraphs: canonicalisation equals the reference and validates;
    //    the reference itself validates, and a copy with one defect does not
    for (int i = 0; i < 400; ++i) {
        const int32_t n = 1 + (int32_t)(rng() % 40);
        const int m = (int)(rng() % 120);
        std::vector<std::pair<int32_t, int32_t>> arcs;
        for (int e = 0; e < m; ++e) arcs.push_back({(int32_t)(rng() % n), (int32_t)(rng() % n)});
        std::vector<int32_t> rp, col, crp, ccol, want_rp, want_col;
        csr_of(n, arcs, rp, col);
        const kh_status c = kh::canonicalize_csr(n, (int64_t)col.size(), rp.data(), col.data(), crp, ccol);
        expect(c == KH_OK, "canonicalize ok", i);
        reference(n, arcs, want_rp, want_col);
        expect(crp == want_rp && ccol == want_col, "canonical form", i);
        expect(kh_validate_csr(n, (int64_t)want_col.size(), want_rp.data(), want_col.empty() ? nullptr : want_col.data()) ==
                   KH_OK,
               "canonical validates", i);
        if (!want_col.empty()) {
            std::vector<int32_t> bad = want_col;
            const size_t k = rng() % bad.size();
            bad[k] = (int32_t)(rng() % 3 == 0 ? n : (rng() % 2 ? -1 : bad[k] ^ 1));
            if (bad[k] != want_col[k])
                expect(kh_validate_csr(n, (int64_t)bad.size(), want_rp.data(), bad.data()) != KH_OK, "defect found",
                       i);
        }
    }
    // 2. hostile row pointers: every helper must refuse them without reading
    //    outside the arrays (the sanitizers check the second part)
    {
        const int32_t col[5] = {1, 0, 2, 1, 0};
        const std::vector<std::vector<int32_t>> rps = {
            {0, 100, 5},     // runs past nnz before a later row comes back
            {0, 3, 2, 5},    // not monotone
            {-4, 1, 5},      // negative start
            {0, 2, 6},       // ends past nnz
            {1, 2, 5},       // does not start at 0
            {0, INT32_MAX, 5},
        };
        int i = 1000;
        for (const auto& rp : rps) {
            const int32_t n = (int32_t)rp.size() - 1;
            std::vector<int32_t> crp, ccol;
            expect(kh_validate_csr(n, 5, rp.data(), col) != KH_OK, "validate refuses hostile row_ptr", i);
            expect(kh::canonicalize_csr(n, 5, rp.data(), col, crp, ccol) != KH_OK, "canonicalize refuses hostile row_ptr",
                   i);
            ++i;
        }
        std::vector<int32_t> crp, ccol;
        const int32_t rp0[1] = {0};
        expect(kh_validate_csr(0, 0, rp0, nullptr) == KH_OK, "empty graph", 2000);
        expect(kh::canonicalize_csr(0, 0, rp0, nullptr, crp, ccol) == KH_OK && crp.size() == 1, "empty canonical",
               2001);
        expect(kh_validate_csr(-1, 0, rp0, nullptr) == KH_EINVAL, "negative n", 2002);
        expect(kh_validate_csr(1, 1, nullptr, col) == KH_EINVAL, "null row_ptr", 2003);
        expect(kh_validate_csr(2, 2, rp0, nullptr) == KH_EINVAL, "null col", 2004);
        expect(kh_validate_csr(1, kh::kMaxArcs + 1, rp0, col) == KH_EINVAL, "too many arcs", 2005);
        expect(kh::canonicalize_csr(1, kh::kMaxArcs + 1, rp0, col, crp, ccol) == KH_EINVAL, "too many arcs (canon)",
               2006);
    }
    // 3. Eq. (buffer) and status names at the edges of their domains
    expect(kh_buffer_size(0, 0.5, 0.05, 0) == -1, "M for n = 0", 3000);
    expect(kh_buffer_size(10, 0.0, 0.05, 0) == -1, "M for eps = 0", 3001);
    expect(kh_buffer_size(10, 0.5, 1.0, 0) == -1, "M for delta = 1", 3002);
    expect(kh_buffer_size(12008, 0.5, 0.05, 0) == 607, "M of Table 1 (n = 12008)", 3003);
    expect(kh_buffer_size(INT64_MAX, 1e-9, 1e-300, 1) > 0, "M saturates", 3004);
    for (int s = -20; s <= 5; ++s) expect(kh_status_str(s) != nullptr, "status name", 3100 + s);
    if (failures) return 1;
    std::printf("csr helpers ok\n");
    return 0;
}
