// Host side of the C ABI declared in include/khcore.h: validation, residency,
// the buffer size M, and the bulk peeling round loops that drive the kernels.
//
// Exact path (ExactCore, Sec. 2), one round:
//   c <- max(c, min deg);  R = {alive v : deg[v] <= c};  core[R] = c;
//   A = alive vertices within distance h of R in G[X] (1-bit BFS from R);
//   X <- X \ R;  deg[A] <- h-degrees recomputed by the bit-parallel BFS.
// Only vertices within distance h of a deleted vertex can change degree.
//
// Sampled path (Core, Alg. 4 with Update of Alg. 3), one round:
//   c <- max(c, min d);  R = {alive v : d[v] <= c};  core'[R] = c;  X <- X \ R;
//   for i = 1..h: recompute B[v,i] for the alive neighbours of R and of the
//   vertices whose (k, B) changed at level i-1;  at i = h refresh d.
// Deleting all of R at once gives the same numbers as Alg. 4's one-at-a-time
// deletion: both keys only depend on (v, X) and never increase as X shrinks
// (Prop. monotone for the estimate), so the running-maximum peel is the
// maximal-core characterisation for every deletion order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <map>
#include <mutex>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <exception>
#include <new>
#include <stdexcept>
#include <vector>

#include "../../include/khcore.h"
#include "kh_internal.hpp"

using namespace kh;

// ---------------------------------------------------------------------------------------------
// errors and device memory
// ---------------------------------------------------------------------------------------------
namespace {

struct KhError {
    kh_status code;
};

[[noreturn]] void fail(kh_status s) { throw KhError{s}; }

void hip_ok(hipError_t e) {
    if (e == hipErrorOutOfMemory) {
        (void)hipGetLastError();
        fail(KH_ENOMEM);
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        fail(KH_EDEVICE);
    }
}

}  // namespace

struct kh_context {
    int device = 0;
    uint64_t budget = 0;
    std::atomic<uint64_t> used{0};
    size_t lds_per_block = 65536;
    int num_cu = 0;
    RoundState* host_state = nullptr;  // pinned mirror of the device round state (fallback)
    void* noalloc_scratch = nullptr;   // this device's fixed working array of kh_hdeg_noalloc
    // pinned mirrors leased by concurrent calls (StateLease)
    std::mutex pool_lock;
    std::vector<RoundState*> pool;
    // pull-kernel timing (kh_profile_enable / kh_profile_read)
    bool prof_on = false;
    PullTimer timer[3];  // 0: h-degree pull, 1: sample-list union, 2: R-mask BFS hop
    long long prof_launches[3] = {0, 0, 0};
    double prof_ms[3] = {0.0, 0.0, 0.0};
    unsigned long long prof_bytes[3] = {0, 0, 0}, prof_gather = 0;
    // idle device blocks kept for reuse, by size: hipFree waits for the whole
    // device, which would serialise calls running on several streams (served
    // requests), and most calls allocate the same sizes again
    std::mutex cache_lock;
    std::multimap<size_t, void*> cache;
    uint64_t cached = 0;      // bytes held in `cache`
    uint64_t cache_cap = 0;   // most bytes `cache` may hold
};

namespace {

// Threads of the serving loop run requests concurrently on one context: each
// has its own pinned mirror of the device round state, and profiling (whose
// event slots the context shares) stays with the owner thread.
thread_local RoundState* tl_state = nullptr;
thread_local bool tl_worker = false;

RoundState* hstate(kh_context* ctx) { return tl_state ? tl_state : ctx->host_state; }
bool prof_active(const kh_context* ctx) { return ctx->prof_on && !tl_worker; }

// Every entry point that runs an engine leases a pinned round-state mirror of
// its own for the calling thread, so that calls from several threads on one
// context never share one (serving threads bring their own).
struct StateLease {
    kh_context* ctx = nullptr;
    RoundState* mine = nullptr;
    explicit StateLease(kh_context* c) : ctx(c) {
        if (tl_state) return;
        {
            std::lock_guard<std::mutex> lk(ctx->pool_lock);
            if (!ctx->pool.empty()) {
                mine = ctx->pool.back();
                ctx->pool.pop_back();
            }
        }
        if (!mine) {
            void* q = nullptr;
            if (hipHostMalloc(&q, sizeof(RoundState), hipHostMallocDefault) != hipSuccess) {
                (void)hipGetLastError();
                throw KhError{KH_ENOMEM};
            }
            mine = static_cast<RoundState*>(q);
        }
        tl_state = mine;
    }
    ~StateLease() {
        if (!mine) return;
        tl_state = nullptr;
        std::lock_guard<std::mutex> lk(ctx->pool_lock);
        ctx->pool.push_back(mine);
    }
    StateLease(const StateLease&) = delete;
    StateLease& operator=(const StateLease&) = delete;
};

// Device blocks come in size classes (powers of two up to 1 MiB, then whole
// MiB) so that a block released by one call fits the next call's request.
size_t block_bytes(size_t bytes) {
    if (bytes <= ((size_t)1 << 20)) {
        size_t b = 256;
        while (b < bytes) b <<= 1;
        return b;
    }
    return (bytes + ((size_t)1 << 20) - 1) & ~(((size_t)1 << 20) - 1);
}

// Give every cached block back to the device (waits for the device).
void cache_flush(kh_context* ctx) {
    std::lock_guard<std::mutex> lk(ctx->cache_lock);
    for (auto& kv : ctx->cache) (void)hipFree(kv.second);
    ctx->cache.clear();
    ctx->cached = 0;
}

// A device block of exactly `bytes` (a size class): a cached one, else hipMalloc.
// Blocks only enter the cache when the call that used them has synchronised its
// streams (every entry point does before its buffers are released), so a block
// taken from the cache is idle.
void* device_take(kh_context* ctx, size_t bytes) {
    {
        std::lock_guard<std::mutex> lk(ctx->cache_lock);
        auto it = ctx->cache.find(bytes);
        if (it != ctx->cache.end()) {
            void* p = it->second;
            ctx->cache.erase(it);
            ctx->cached -= bytes;
            return p;
        }
    }
    if (ctx->budget && ctx->used.load() + ctx->cached + bytes > ctx->budget) cache_flush(ctx);
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, bytes);
    if (e == hipErrorOutOfMemory) {
        (void)hipGetLastError();
        cache_flush(ctx);
        e = hipMalloc(&q, bytes);
    }
    hip_ok(e);
    return q;
}

void device_give(kh_context* ctx, void* p, size_t bytes) {
    if (std::uncaught_exceptions() > 0) {
        // a call that failed may still have kernels in flight: hipFree waits for them
        (void)hipFree(p);
        return;
    }
    {
        std::lock_guard<std::mutex> lk(ctx->cache_lock);
        if (ctx->cached + bytes <= ctx->cache_cap) {
            ctx->cache.emplace(bytes, p);
            ctx->cached += bytes;
            return;
        }
    }
    (void)hipFree(p);
}

template <typename T>
struct Buf {
    kh_context* ctx = nullptr;
    T* p = nullptr;
    size_t count = 0;
    Buf() = default;
    Buf(const Buf&) = delete;
    Buf& operator=(const Buf&) = delete;
    Buf(Buf&& o) noexcept : ctx(o.ctx), p(o.p), count(o.count) {
        o.p = nullptr;
        o.count = 0;
    }
    Buf& operator=(Buf&& o) noexcept {
        if (this != &o) {
            release();
            ctx = o.ctx;
            p = o.p;
            count = o.count;
            o.p = nullptr;
            o.count = 0;
        }
        return *this;
    }
    ~Buf() { release(); }
    void alloc(kh_context* c, size_t n) {
        release();
        ctx = c;
        const size_t bytes = block_bytes(std::max<size_t>(n, 1) * sizeof(T));
        const uint64_t before = ctx->used.fetch_add(bytes);
        if (ctx->budget && before + bytes > ctx->budget) {
            ctx->used.fetch_sub(bytes);
            fail(KH_ENOMEM);
        }
        try {
            p = static_cast<T*>(device_take(ctx, bytes));
        } catch (...) {
            ctx->used.fetch_sub(bytes);
            throw;
        }
        count = n;
    }
    void release() {
        if (p) {
            const size_t bytes = block_bytes(std::max<size_t>(count, 1) * sizeof(T));
            device_give(ctx, p, bytes);
            ctx->used -= bytes;
            p = nullptr;
            count = 0;
        }
    }
};

int ceil_log2(long long x) {
    int l = 0;
    while ((1ll << l) < x) ++l;
    return l;
}

}  // namespace

struct kh_graph {
    kh_context* ctx = nullptr;
    int32_t n = 0;
    int64_t nnz = 0;
    Buf<int32_t> rp_own, col_own;
    const int32_t* rp = nullptr;
    const int32_t* col = nullptr;
    std::vector<int32_t> h_rp;
    // work items of the h-degree pull kernel (built on first use, under the lock:
    // served requests on one graph may run on several threads)
    std::mutex items_lock;
    bool items_built = false;
    Buf<int32_t> it_u, it_beg, it_end, split_list, vitem;
    // packed unions of several graphs: segment (graph) of every vertex
    Buf<int32_t> seg_own;
    const int32_t* seg = nullptr;
    int32_t nseg = 1;
    Buf<uint8_t> it_split;
    MsItems items{};
};

// ---------------------------------------------------------------------------------------------
// host helpers
// ---------------------------------------------------------------------------------------------
// ---------------------------------------------------------------------------------------------
// context and graphs
// ---------------------------------------------------------------------------------------------
extern "C" kh_status kh_context_create(int32_t device, uint64_t hbm_budget_bytes, kh_context** out) {
    if (!out) return KH_EINVAL;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0 || device < 0 || device >= count) {
        (void)hipGetLastError();
        return KH_EDEVICE;
    }
    if (hipSetDevice(device) != hipSuccess) return KH_EDEVICE;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return KH_EDEVICE;
    auto* ctx = new (std::nothrow) kh_context();
    if (!ctx) return KH_ENOMEM;
    ctx->device = device;
    ctx->budget = hbm_budget_bytes;
    ctx->lds_per_block = prop.sharedMemPerBlock;
    ctx->num_cu = prop.multiProcessorCount;
    // idle blocks kept for reuse: at most a quarter of the budget (or of the device)
    ctx->cache_cap = (hbm_budget_bytes ? hbm_budget_bytes : (uint64_t)prop.totalGlobalMem) / 4;
    void* hs = nullptr;
    if (hipHostMalloc(&hs, sizeof(RoundState), hipHostMallocDefault) != hipSuccess) {
        delete ctx;
        return KH_EDEVICE;
    }
    ctx->host_state = static_cast<RoundState*>(hs);
    // the fixed array of kh_hdeg_noalloc: its address on this device, looked up once
    if (kh::noalloc_scratch_init(device, &ctx->noalloc_scratch) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipHostFree(hs);
        delete ctx;
        return KH_EDEVICE;
    }
    *out = ctx;
    return KH_OK;
}

namespace kh {
void worker_thread_begin(RoundState* pinned) {
    tl_state = pinned;
    tl_worker = true;
}
void worker_thread_end() {
    tl_state = nullptr;
    tl_worker = false;
}
kh_context* graph_context(const kh_graph* g);
}  // namespace kh

extern "C" void kh_context_destroy(kh_context* ctx) {
    if (!ctx) return;
    kh::serve_shutdown(ctx);
    cache_flush(ctx);
    if (ctx->host_state) (void)hipHostFree(ctx->host_state);
    for (RoundState* p : ctx->pool) (void)hipHostFree(p);
    for (auto& T : ctx->timer) {
        if (T.ev) {
            for (int i = 0; i < 2 * T.cap; ++i) (void)hipEventDestroy(T.ev[i]);
            delete[] T.ev;
        }
    }
    delete ctx;
}

namespace {

// Fold the recorded launches into the context totals.
void prof_collect(kh_context* ctx) {
    for (int k = 0; k < 3; ++k) {
        PullTimer& T = ctx->timer[k];
        for (int i = 0; i < T.used; ++i) {
            float ms = 0.f;
            hip_ok(hipEventSynchronize(T.ev[2 * i + 1]));
            hip_ok(hipEventElapsedTime(&ms, T.ev[2 * i], T.ev[2 * i + 1]));
            ctx->prof_ms[k] += ms;
            ctx->prof_launches[k] += 1;
        }
        T.used = 0;
    }
}

void prof_add_counters(kh_context* ctx, const RoundState& hs) {
    if (!prof_active(ctx)) return;
    prof_collect(ctx);
    ctx->prof_bytes[0] += hs.pull_bytes;
    ctx->prof_gather += hs.pull_gather;
    ctx->prof_bytes[1] += hs.union_bytes;
    ctx->prof_bytes[2] += hs.rbfs_bytes;
}

}  // namespace

extern "C" kh_status kh_profile_enable(kh_context* ctx, int32_t on) {
    if (!ctx) return KH_EINVAL;
    try {
        hip_ok(hipSetDevice(ctx->device));
        for (auto& T : ctx->timer) {
            if (on && !T.ev) {
                const int cap = 8192;
                T.ev = new hipEvent_t[2 * cap];
                for (int i = 0; i < 2 * cap; ++i) hip_ok(hipEventCreate(&T.ev[i]));
                T.cap = cap;
            }
        }
        if (ctx->prof_on) prof_collect(ctx);
        ctx->prof_on = on != 0;
        if (on) {
            for (int k = 0; k < 3; ++k) {
                ctx->timer[k].used = 0;
                ctx->prof_launches[k] = 0;
                ctx->prof_ms[k] = 0.0;
                ctx->prof_bytes[k] = 0;
            }
            ctx->prof_gather = 0;
        }
    } catch (const KhError& e) {
        return e.code;
    }
    return KH_OK;
}

extern "C" kh_status kh_profile_read(kh_context* ctx, int32_t kernel, int64_t* launches, double* total_ms,
                                     int64_t* alg_bytes, int64_t* gather_bytes) {
    if (!ctx || kernel < 0 || kernel > 2) return KH_EINVAL;
    try {
        if (ctx->prof_on) prof_collect(ctx);
    } catch (const KhError& e) {
        return e.code;
    }
    if (launches) *launches = ctx->prof_launches[kernel];
    if (total_ms) *total_ms = ctx->prof_ms[kernel];
    if (alg_bytes) *alg_bytes = (int64_t)ctx->prof_bytes[kernel];
    if (gather_bytes) *gather_bytes = kernel == 0 ? (int64_t)ctx->prof_gather : 0;
    return KH_OK;
}


extern "C" kh_status kh_graph_load_csr(kh_context* ctx, int32_t n, int64_t nnz, const int32_t* row_ptr,
                                       const int32_t* col, uint32_t flags, void* stream, kh_graph** out) {
    if (!ctx || !out || n < 0 || nnz < 0 || nnz > kMaxArcs) return KH_EINVAL;
    *out = nullptr;
    if (!row_ptr || (nnz > 0 && !col)) return KH_EINVAL;
    const bool borrow = (flags & KH_PTRS_DEVICE_BORROW) != 0;
    if (borrow && (flags & KH_CANONICALIZE)) return KH_EINVAL;
    auto s = static_cast<hipStream_t>(stream);
    kh_graph* g = new (std::nothrow) kh_graph();
    if (!g) return KH_ENOMEM;
    try {
        hip_ok(hipSetDevice(ctx->device));
        g->ctx = ctx;
        g->n = n;
        if (!borrow) {
            std::vector<int32_t> crp, ccol;
            const int32_t* hrp = row_ptr;
            const int32_t* hcol = col;
            if (flags & KH_CANONICALIZE) {
                const kh_status c = canonicalize_csr(n, nnz, row_ptr, col, crp, ccol);
                if (c != KH_OK) fail(c);
                hrp = crp.data();
                hcol = ccol.data();
                nnz = (int64_t)ccol.size();
            } else if (!(flags & KH_TRUST_CSR)) {
                const kh_status v = kh_validate_csr(n, nnz, row_ptr, col);
                if (v != KH_OK) fail(v);
            }
            g->nnz = nnz;
            g->h_rp.assign(hrp, hrp + (size_t)n + 1);
            g->rp_own.alloc(ctx, (size_t)n + 1);
            g->col_own.alloc(ctx, (size_t)std::max<int64_t>(nnz, 1));
            hip_ok(hipMemcpyAsync(g->rp_own.p, hrp, sizeof(int32_t) * ((size_t)n + 1), hipMemcpyHostToDevice, s));
            if (nnz > 0)
                hip_ok(hipMemcpyAsync(g->col_own.p, hcol, sizeof(int32_t) * (size_t)nnz, hipMemcpyHostToDevice, s));
            hip_ok(hipStreamSynchronize(s));
            g->rp = g->rp_own.p;
            g->col = g->col_own.p;
        } else {
            g->nnz = nnz;
            g->rp = row_ptr;
            g->col = col;
            g->h_rp.resize((size_t)n + 1);
            hip_ok(hipMemcpyAsync(g->h_rp.data(), row_ptr, sizeof(int32_t) * ((size_t)n + 1), hipMemcpyDeviceToHost,
                                  s));
            hip_ok(hipStreamSynchronize(s));
            if (!(flags & KH_TRUST_CSR) && n > 0) {
                if (g->h_rp[0] != 0 || (int64_t)g->h_rp[n] != nnz) fail(KH_EGRAPH);
                Buf<int> err;
                err.alloc(ctx, 1);
                launch_set_int(err.p, 0, s);
                launch_validate(row_ptr, col, n, nnz, err.p, s);
                int herr = 0;
                hip_ok(hipMemcpyAsync(&herr, err.p, sizeof(int), hipMemcpyDeviceToHost, s));
                hip_ok(hipStreamSynchronize(s));
                if (herr) fail(KH_EGRAPH);
            }
        }
    } catch (const KhError& e) {
        delete g;
        return e.code;
    } catch (const std::bad_alloc&) {
        delete g;
        return KH_ENOMEM;
    }
    *out = g;
    return KH_OK;
}

extern "C" void kh_graph_free(kh_graph* g) { delete g; }
kh_context* kh::graph_context(const kh_graph* g) { return g ? g->ctx : nullptr; }
int kh::context_device(const kh_context* ctx) { return ctx->device; }
extern "C" int32_t kh_graph_n(const kh_graph* g) { return g ? g->n : -1; }
extern "C" int64_t kh_graph_nnz(const kh_graph* g) { return g ? g->nnz : -1; }

// ---------------------------------------------------------------------------------------------
// engines
// ---------------------------------------------------------------------------------------------
namespace {

using Clock = std::chrono::steady_clock;

// Opt-in progress trace on stderr (KH_TRACE=1): one line per traced round.
bool trace_on() {
    static const bool on = [] {
        const char* e = std::getenv("KH_TRACE");
        return e && e[0] && e[0] != '0';
    }();
    return on;
}

// Opt-in heartbeat on stderr (KH_HEARTBEAT=<seconds>): a line at most every
// that many seconds from the long round loops, so that a caller watching the
// output can tell a long peel from a stuck one.
double heartbeat_every() {
    static const double s = [] {
        const char* e = std::getenv("KH_HEARTBEAT");
        return e && e[0] ? std::atof(e) : 0.0;
    }();
    return s;
}

struct Heartbeat {
    Clock::time_point t0 = Clock::now(), last = Clock::now();
    void tick(const char* what, const RoundState& hs) {
        const double every = heartbeat_every();
        if (every <= 0.0) return;
        const auto now = Clock::now();
        if (std::chrono::duration<double>(now - last).count() < every) return;
        last = now;
        std::fprintf(stderr, "[kh] %s: round %d, c %lld, %d alive, %.1fs\n", what, hs.rounds, hs.c, hs.alive_count,
                     std::chrono::duration<double>(now - t0).count());
    }
};

void check_params(const kh_graph* g, const kh_params* P) {
    if (!g || !P) fail(KH_EINVAL);
    if (P->h < 1) fail(KH_EINVAL);
    if (!(P->delta > 0.0 && P->delta < 1.0)) fail(KH_EINVAL);
    if (std::isnan(P->epsilon)) fail(KH_EINVAL);
}

// Work items of the pull kernel: (vertex, arc range) pieces of at most
// kPullChunk arcs; split pieces first, then whole vertices by decreasing degree,
// so that the groups of a wave see items of similar length.
void build_items(kh_graph* g, hipStream_t s) {
    std::lock_guard<std::mutex> lock(g->items_lock);
    if (g->items_built) return;
    const int32_t n = g->n;
    const std::vector<int32_t>& rp = g->h_rp;
    std::vector<int32_t> iu, ib, ie, sl, vit((size_t)std::max(n, 1), -1);
    std::vector<uint8_t> isp;
    int32_t maxd = 0;
    for (int32_t v = 0; v < n; ++v) maxd = std::max(maxd, rp[v + 1] - rp[v]);
    for (int32_t v = 0; v < n; ++v) {
        const int32_t d = rp[v + 1] - rp[v];
        if (d > kPullChunk) {
            sl.push_back(v);
            vit[v] = (int32_t)iu.size();
            for (int32_t b = rp[v]; b < rp[v + 1]; b += kPullChunk) {
                iu.push_back(v);
                ib.push_back(b);
                ie.push_back(std::min(b + kPullChunk, rp[v + 1]));
                isp.push_back(1);
            }
        }
    }
    // counting sort of whole vertices by degree, descending
    std::vector<int32_t> cnt((size_t)kPullChunk + 2, 0);
    for (int32_t v = 0; v < n; ++v) {
        const int32_t d = rp[v + 1] - rp[v];
        if (d >= 1 && d <= kPullChunk) cnt[(size_t)d]++;
    }
    std::vector<int32_t> start((size_t)kPullChunk + 2, 0);
    int32_t acc = 0;
    for (int32_t d = kPullChunk; d >= 1; --d) {
        start[(size_t)d] = acc;
        acc += cnt[(size_t)d];
    }
    const size_t base = iu.size();
    iu.resize(base + (size_t)acc);
    ib.resize(base + (size_t)acc);
    ie.resize(base + (size_t)acc);
    isp.resize(base + (size_t)acc, 0);
    for (int32_t v = 0; v < n; ++v) {
        const int32_t d = rp[v + 1] - rp[v];
        if (d >= 1 && d <= kPullChunk) {
            const size_t at = base + (size_t)start[(size_t)d]++;
            vit[v] = (int32_t)at;
            iu[at] = v;
            ib[at] = rp[v];
            ie[at] = rp[v + 1];
        }
    }
    kh_context* ctx = g->ctx;
    const size_t ni = iu.size();
    g->it_u.alloc(ctx, ni);
    g->it_beg.alloc(ctx, ni);
    g->it_end.alloc(ctx, ni);
    g->it_split.alloc(ctx, ni);
    g->split_list.alloc(ctx, sl.size());
    g->vitem.alloc(ctx, vit.size());
    hip_ok(hipMemcpyAsync(g->vitem.p, vit.data(), vit.size() * 4, hipMemcpyHostToDevice, s));
    if (ni) {
        hip_ok(hipMemcpyAsync(g->it_u.p, iu.data(), ni * 4, hipMemcpyHostToDevice, s));
        hip_ok(hipMemcpyAsync(g->it_beg.p, ib.data(), ni * 4, hipMemcpyHostToDevice, s));
        hip_ok(hipMemcpyAsync(g->it_end.p, ie.data(), ni * 4, hipMemcpyHostToDevice, s));
        hip_ok(hipMemcpyAsync(g->it_split.p, isp.data(), ni, hipMemcpyHostToDevice, s));
    }
    if (!sl.empty()) hip_ok(hipMemcpyAsync(g->split_list.p, sl.data(), sl.size() * 4, hipMemcpyHostToDevice, s));
    hip_ok(hipStreamSynchronize(s));
    g->items.nitems = (int32_t)ni;
    g->items.u = g->it_u.p;
    g->items.beg = g->it_beg.p;
    g->items.end = g->it_end.p;
    g->items.split = g->it_split.p;
    g->items.nsplit = (int32_t)sl.size();
    g->items.split_list = g->split_list.p;
    g->items.vitem = g->vitem.p;
    g->items.nnz = g->nnz;
    g->items_built = true;
}

// Bitset width per vertex (in 64-bit words): sources per batch = 64 Q.
int pick_q(int64_t sources) {
    int q = 1;
    while (q < 16 && 64ll * q < sources) q <<= 1;
    return q;
}

struct Planes {
    Buf<uint64_t> vis, frA, frB, acc, valid;
    Buf<uint32_t> bmA, bmB, bmT, bmC, bmTile, cnt;
    Buf<int32_t> touched, flA, flB, tl, cvA, cvB, ciA, ciB, sbit;
    Buf<int> tcount, gcnt;
    Buf<int2> fcA, fcB;
    Buf<MsCtl> ctl;
    int qmax = 0;
    const int32_t* seg = nullptr;
    int32_t ns_cap = 0;
    // nitems: work items of the graph (build_items first).  seg/nseg: segments
    // of a packed union (seg == NULL: one graph).
    void alloc(kh_context* ctx, int32_t n, int64_t nnz, int qmax_, int32_t nitems, const int32_t* seg_ = nullptr,
               int32_t nseg = 1) {
        qmax = qmax_;
        seg = seg_;
        const size_t nn = (size_t)std::max(n, 1);
        const size_t words = nn * qmax;
        const size_t bm = (nn + 31) / 32;
        const size_t ntiles = (nn + 63) / 64;
        vis.alloc(ctx, words);
        frA.alloc(ctx, words);
        frB.alloc(ctx, words);
        acc.alloc(ctx, words);
        valid.alloc(ctx, 16);
        bmA.alloc(ctx, bm);
        bmB.alloc(ctx, bm);
        bmT.alloc(ctx, bm);
        bmC.alloc(ctx, bm);
        bmTile.alloc(ctx, (ntiles + 31) / 32);
        cnt.alloc(ctx, (size_t)64 * std::max(qmax, 16) * (seg ? (size_t)std::max(nseg, 1) : 1));
        touched.alloc(ctx, nn);
        flA.alloc(ctx, nn);
        flB.alloc(ctx, nn);
        fcA.alloc(ctx, nn + (size_t)(nnz / 64) + 1);
        fcB.alloc(ctx, nn + (size_t)(nnz / 64) + 1);
        tl.alloc(ctx, ntiles);
        if (seg) {
            sbit.alloc(ctx, nn);
            gcnt.alloc(ctx, (size_t)std::max(nseg, 1));
            ns_cap = (int32_t)nn;
        }
        cvA.alloc(ctx, nn);
        cvB.alloc(ctx, nn);
        ciA.alloc(ctx, (size_t)std::max(nitems, 1));
        ciB.alloc(ctx, (size_t)std::max(nitems, 1));
        tcount.alloc(ctx, 1);
        ctl.alloc(ctx, 1);
    }
    // the planes, bitmaps, counters and control block start all-zero; every
    // batch leaves them so
    void clear(hipStream_t s) {
        hip_ok(hipMemsetAsync(vis.p, 0, vis.count * 8, s));
        hip_ok(hipMemsetAsync(acc.p, 0, acc.count * 8, s));
        hip_ok(hipMemsetAsync(cnt.p, 0, cnt.count * 4, s));
        for (Buf<uint32_t>* b : {&bmA, &bmB, &bmT, &bmC, &bmTile}) hip_ok(hipMemsetAsync(b->p, 0, b->count * 4, s));
        hip_ok(hipMemsetAsync(tcount.p, 0, sizeof(int), s));
        hip_ok(hipMemsetAsync(ctl.p, 0, sizeof(MsCtl), s));
        if (gcnt.p) hip_ok(hipMemsetAsync(gcnt.p, 0, gcnt.count * sizeof(int), s));
    }
    PullTimer* timer = nullptr;
    MsPlanes view(int q) const {
        MsPlanes P;
        P.Q = q;
        P.timer = timer;
        P.vis = vis.p;
        P.frA = frA.p;
        P.frB = frB.p;
        P.acc = acc.p;
        P.bmA = bmA.p;
        P.bmB = bmB.p;
        P.bmT = bmT.p;
        P.bmC = bmC.p;
        P.touched = touched.p;
        P.touched_count = tcount.p;
        P.flA = flA.p;
        P.flB = flB.p;
        P.fcA = fcA.p;
        P.fcB = fcB.p;
        P.tl = tl.p;
        P.bmTile = bmTile.p;
        P.seg = seg;
        P.sbit = seg ? sbit.p : nullptr;
        P.gcnt = seg ? gcnt.p : nullptr;
        P.ns_cap = seg ? ns_cap : 64 * q;
        P.exact_out = nullptr;
        P.cvA = cvA.p;
        P.cvB = cvB.p;
        P.ciA = ciA.p;
        P.ciB = ciB.p;
        P.ctl = ctl.p;
        P.cnt = cnt.p;
        P.valid = valid.p;
        return P;
    }
};

// h-degrees of every vertex in `src[0..count)` (device list, host count).
void hdeg_sources(kh_graph* g, Planes& PL, const uint8_t* alive, const int32_t* adeg, const int32_t* src, int64_t count,
                  int h, int64_t* deg, RoundState* st, hipStream_t s) {
    int64_t done = 0;
    kh_context* ctx = g->ctx;
    PL.timer = prof_active(ctx) ? &ctx->timer[0] : nullptr;
    while (done < count) {
        if (PL.timer && PL.timer->used + 8 >= PL.timer->cap) prof_collect(ctx);
        const int64_t rest = count - done;
        const int q = std::min(PL.qmax, pick_q(rest));
        const int ns = (int)std::min<int64_t>(rest, 64ll * q);
        MsPlanes P = PL.view(q);
        P.seg = nullptr;  // host-chosen batches number their sources 0..ns-1
        P.sbit = nullptr;
        P.gcnt = nullptr;
        P.ns_cap = 64 * q;
        ms_batch(P, g->items, g->n, g->rp, g->col, alive, adeg, src + done, ns, nullptr, h, deg, st, s);
        done += ns;
    }
}

void read_state(kh_context* ctx, RoundState* dst_dev, hipStream_t s) {
    hip_ok(hipGetLastError());
    hip_ok(hipMemcpyAsync(hstate(ctx), dst_dev, sizeof(RoundState), hipMemcpyDeviceToHost, s));
    hip_ok(hipStreamSynchronize(s));
}

void init_state(RoundState* st, hipStream_t s) {
    RoundState z;
    std::memset(&z, 0, sizeof(z));
    z.c = -1;
    hip_ok(hipMemcpyAsync(st, &z, sizeof(z), hipMemcpyHostToDevice, s));
    hip_ok(hipStreamSynchronize(s));
}

struct Candidates {
    std::vector<int64_t> k, size, sum;
};

bool graphs_off() {
    const char* e = std::getenv("KH_NO_GRAPH");
    return e && e[0] && e[0] != '0';
}

// Replays a fixed sequence of kernel launches (recorded once by stream capture)
// on a private stream that is ordered after the caller's stream.  The sequences
// hold kernels only (clears are fill kernels), and every launch reads its
// round-dependent values from device memory, so each replay is the same work as
// issuing the launches directly.
struct Replay {
    hipStream_t gs = nullptr;
    std::vector<hipGraph_t> graphs;
    std::vector<hipGraphExec_t> execs;
    bool direct = false;
    ~Replay() {
        for (auto e : execs) (void)hipGraphExecDestroy(e);
        for (auto g : graphs) (void)hipGraphDestroy(g);
        if (gs) (void)hipStreamDestroy(gs);
    }
    // The stream, ordered after the caller's, and the first sequence (index 0).
    template <typename F>
    hipStream_t prepare(hipStream_t caller, bool use_graph, F&& record) {
        hip_ok(hipStreamCreate(&gs));
        hipEvent_t ev;
        hip_ok(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        hip_ok(hipEventRecord(ev, caller));
        hip_ok(hipStreamWaitEvent(gs, ev, 0));
        hip_ok(hipEventDestroy(ev));
        direct = !use_graph;
        add(record);
        return gs;
    }
    // Another sequence on the same stream (next index).
    template <typename F>
    int add(F&& record) {
        if (!direct) {
            hipGraph_t g = nullptr;
            hipGraphExec_t e = nullptr;
            hip_ok(hipStreamBeginCapture(gs, hipStreamCaptureModeThreadLocal));
            record(gs);
            hip_ok(hipStreamEndCapture(gs, &g));
            graphs.push_back(g);
            hip_ok(hipGraphInstantiate(&e, g, nullptr, nullptr, 0));
            execs.push_back(e);
            return (int)execs.size() - 1;
        }
        return 0;
    }
    template <typename F>
    void run(F&& record, int index = 0) {
        if (direct) record(gs);
        else hip_ok(hipGraphLaunch(execs[(size_t)index], gs));
    }
};

void pick_dense(const Candidates& C, bool prune, double eps, int64_t maxcore, kh_result* res) {
    int64_t bk = -1, bs = 0, bR = 0;
    const double e = eps > 0.0 ? std::min(eps, 0.999999) : 0.0;
    for (size_t i = 0; i < C.k.size(); ++i) {
        const int64_t K = C.k[i];
        if (prune && (double)K * (1.0 + e) < (1.0 - e) * (double)maxcore) continue;
        const int64_t S = C.size[i], R = C.sum[i];
        if (bk < 0 || (__int128)R * (__int128)bs >= (__int128)bR * (__int128)S) {
            bk = K;
            bs = S;
            bR = R;
        }
    }
    res->dense_k = bk;
    res->dense_size = bs;
    res->dense_R = bR;
    res->dense_density = bs > 0 ? (double)bR / (2.0 * (double)bs) : 0.0;
}

Candidates read_candidates(const RoundState& hs, const Buf<int64_t>& ck, const Buf<int64_t>& cs,
                           const Buf<int64_t>& cr, hipStream_t s) {
    Candidates C;
    const size_t nc = (size_t)hs.ncand;
    C.k.resize(nc);
    C.size.resize(nc);
    C.sum.resize(nc);
    if (nc) {
        hip_ok(hipMemcpyAsync(C.k.data(), ck.p, nc * 8, hipMemcpyDeviceToHost, s));
        hip_ok(hipMemcpyAsync(C.size.data(), cs.p, nc * 8, hipMemcpyDeviceToHost, s));
        hip_ok(hipMemcpyAsync(C.sum.data(), cr.p, nc * 8, hipMemcpyDeviceToHost, s));
        hip_ok(hipStreamSynchronize(s));
    }
    return C;
}

// ----- exact engine ---------------------------------------------------------------------------
// key == nullptr: ExactCore peel (key = deg).  Otherwise a replay whose rounds
// delete by the given key (a core map), used for the densest-core sums.
struct ExactRun {
    kh_graph* g;
    int h;
    hipStream_t s;
    Buf<uint8_t> alive, exact;
    Buf<int32_t> adeg, mark, rlist, alist, qv, qb, srcl, anchor, hopfill, fmark, flA, flB;
    Buf<uint64_t> rmask, gainA, gainB;
    Buf<uint32_t> fbA, fbB;
    Buf<int64_t> deg, core, ck, cs, cr;
    Buf<RoundState> st;
    Planes PL;
    Candidates cands;
    RoundState fin{};
    long long recomputed = 0;  // exact h-degree evaluations
    int32_t* rnd_out = nullptr;  // nullable: deletion round (epoch) of every vertex

    void alloc(int32_t n) {
        kh_context* ctx = g->ctx;
        alive.alloc(ctx, n);
        adeg.alloc(ctx, n);
        mark.alloc(ctx, n);
        rlist.alloc(ctx, n);
        alist.alloc(ctx, n);
        srcl.alloc(ctx, n);
        const size_t qcap = (size_t)n + (size_t)(g->nnz / kExpandChunk) + 2;
        qv.alloc(ctx, qcap);
        qb.alloc(ctx, qcap);
        deg.alloc(ctx, n);
        core.alloc(ctx, n);
        ck.alloc(ctx, (size_t)n + 1);
        cs.alloc(ctx, (size_t)n + 1);
        cr.alloc(ctx, (size_t)n + 1);
        st.alloc(ctx, 1);
        PL.alloc(ctx, n, g->nnz, pick_q(n), g->items.nitems, g->seg, g->nseg);
        PL.clear(s);
        init_state(st.p, s);
    }

    // Deleting R: core[R] = c, then mark the alive vertices within distance h
    // of R in G[X] (R still alive) into alist, then remove R and update the
    // alive degrees.
    void delete_round(int32_t epoch, const int64_t* key) {
        launch_select(key, alive.p, g->n, st.p, core.p, rlist.p, mark.p, epoch, 0, s);
        delete_round_tail(epoch);
    }

    void delete_round_tail(int32_t epoch) {
        launch_enqueue(rlist.p, nullptr, &st.p->rcount, g->rp, qv.p, qb.p, &st.p->qcount, s);
        launch_expand(qv.p, qb.p, &st.p->qcount, g->rp, g->col, alive.p, mark.p, epoch, 0, alist.p, &st.p->aff_fill,
                      nullptr, s);
        if (hopfill.p) launch_record_fill(st.p, hopfill.p, 1, s);
        for (int t = 2; t <= h; ++t) {
            launch_next_frontier(st.p, s);
            launch_enqueue(alist.p, &st.p->front_lo, &st.p->front_hi, g->rp, qv.p, qb.p, &st.p->qcount, s);
            launch_expand(qv.p, qb.p, &st.p->qcount, g->rp, g->col, alive.p, mark.p, epoch, 0, alist.p,
                          &st.p->aff_fill, nullptr, s);
            if (hopfill.p) launch_record_fill(st.p, hopfill.p, t, s);
        }
        launch_kill_list(rlist.p, &st.p->rcount, alive.p, s);
        launch_set_int(&st.p->qcount, 0, s);
        launch_enqueue(rlist.p, nullptr, &st.p->rcount, g->rp, qv.p, qb.p, &st.p->qcount, s);
        launch_expand(qv.p, qb.p, &st.p->qcount, g->rp, g->col, alive.p, mark.p, epoch, 1, nullptr, nullptr, adeg.p,
                      s);
    }

    // Deletion tail of the lazy peel: mask BFS from R over h hops (R still alive),
    // remove R, update alive degrees.  Leaves alist/hopfill/rmask for the decay step.
    // The deletion of the commit sequence: mask BFS from R (|R| <= 64 gives the
    // exact decrement of the vertices at distance exactly h), R leaves X, the
    // alive degrees drop.  Every list count it reads is zero when no round was
    // committed.
    // Launch widths of the per-round kernels: small grids keep the per-round
    // cost of a single graph low; a large packed union's frontiers and lists
    // need the wider ones.
    bool wide() const { return g->n >= (1 << 22); }
    int hop_grid() const { return wide() ? 2048 : 512; }
    int list_grid() const { return wide() ? 512 : 128; }

    void delete_round_masked() {
        // R's mask bits and the chunks of hop 1 (the round reset zeroed qcount)
        launch_enqueue_r(rlist.p, &st.p->rcount, g->rp, qv.p, qb.p, &st.p->qcount, 0, rmask.p, gainA.p, fbA.p, nullptr,
                         s, &st.p->hop_arcs);
        int32_t* fl[2] = {flA.p, flB.p};
        uint64_t* gain[2] = {gainA.p, gainB.p};
        uint32_t* fb[2] = {fbA.p, fbB.p};
        PullTimer* rt = prof_active(g->ctx) ? &g->ctx->timer[2] : nullptr;
        for (int t = 1; t <= h; ++t) {
            const int32_t* src = t == 1 ? rlist.p : fl[(t - 1) & 1];
            const int* srcn = t == 1 ? &st.p->rcount : &st.p->fcount[(t - 1) & 1];
            if (t > 1)
                launch_enqueue(src, nullptr, srcn, g->rp, qv.p, qb.p, &st.p->qcount, s, nullptr, st.p, g->nnz,
                               list_grid());
            // push from the frontier's chunks, or pull into every alive vertex
            // when the frontier holds more than 1/pull_ratio of the arcs
            launch_rbfs_hop(qv.p, qb.p, &st.p->qcount, g->n, g->rp, g->col, alive.p, gain[(t - 1) & 1],
                            fb[(t - 1) & 1], rmask.p, gain[t & 1], t < h ? fb[t & 1] : nullptr, mark.p, fmark.p,
                            fl[t & 1], &st.p->fcount[t & 1], alist.p, &st.p->aff_fill, st.p, g->nnz, s, rt,
                            hop_grid());
            launch_clear_hop_end(src, srcn, gain[(t - 1) & 1], fb[(t - 1) & 1], st.p, hopfill.p, t, h, s,
                                 list_grid());
        }
        // R leaves X and its chunks are queued (hop_end of hop h zeroed qcount);
        // the alive degrees drop
        launch_enqueue_r(rlist.p, &st.p->rcount, g->rp, qv.p, qb.p, &st.p->qcount, 1, nullptr, nullptr, nullptr,
                         alive.p, s);
        launch_expand(qv.p, qb.p, &st.p->qcount, g->rp, g->col, alive.p, mark.p, 0, 1, nullptr, nullptr, adeg.p, s);
    }

    void trace_round(const RoundState& hs, const char* what, Clock::time_point t0) {
        if (trace_on() && (hs.rounds < 8 || (hs.rounds & 63) == 0))
            std::fprintf(stderr,
                         "[kh exact] %s round %d c %lld alive %d removed %d affected %d hop arcs %lld %lld %lld "
                         "recomputed %lld t %.3fs\n",
                         what, hs.rounds, hs.c, hs.alive_count, hs.rcount, hs.aff_fill, hs.hop_log[1], hs.hop_log[2],
                         hs.hop_log[3], recomputed, std::chrono::duration<double>(Clock::now() - t0).count());
    }

    // ExactCore with lazy degrees: deg[v] is either exact (exact[v] = 1) or a
    // lower bound.  A round only commits c = max(c, min deg) when no inexact
    // vertex has deg <= c; the inexact ones at or below c are recomputed first.
    // So every deleted vertex has its exact h-degree <= c, and every survivor's
    // exact h-degree is above c: the same rounds as the eager peel.
    void run_lazy() {
        kh_context* ctx = g->ctx;
        const int32_t n = g->n;
        const auto t0 = Clock::now();
        build_items(g, s);
        alloc(n);
        exact.alloc(ctx, n);
        anchor.alloc(ctx, n);
        hopfill.alloc(ctx, (size_t)h + 2);
        fmark.alloc(ctx, n);
        flA.alloc(ctx, n);
        flB.alloc(ctx, n);
        rmask.alloc(ctx, n);
        gainA.alloc(ctx, n);
        gainB.alloc(ctx, n);
        fbA.alloc(ctx, ((size_t)n >> 5) + 1);
        fbB.alloc(ctx, ((size_t)n >> 5) + 1);
        launch_fill_i32(fmark.p, 0, n, s);
        hip_ok(hipMemsetAsync(fbA.p, 0, fbA.count * sizeof(uint32_t), s));
        hip_ok(hipMemsetAsync(fbB.p, 0, fbB.count * sizeof(uint32_t), s));
        hip_ok(hipMemsetAsync(rmask.p, 0, 8 * (size_t)n, s));
        hip_ok(hipMemsetAsync(gainA.p, 0, 8 * (size_t)n, s));
        hip_ok(hipMemsetAsync(gainB.p, 0, 8 * (size_t)n, s));
        launch_alive_from(nullptr, alive.p, n, s);
        launch_alive_degree(g->rp, g->col, alive.p, adeg.p, n, s);
        launch_fill_i32(mark.p, 0, n, s);
        launch_fill_i64(core.p, -1, n, s);
        launch_anchor(nullptr, nullptr, n, g->rp, g->col, alive.p, adeg.p, anchor.p, 0, s);
        launch_lower_bound(nullptr, nullptr, n, h, alive.p, adeg.p, anchor.p, deg.p, exact.p, s);
        launch_round_reset(st.p, s, 0);
        launch_set_int(&st.p->pull_ratio, g->seg ? kRbfsPullRatioUnion : kRbfsPullRatio, s);
        long long iters = 0;
        // one batch takes up to 64 Q sources, per graph of a packed union
        const int qbits = 64 * PL.qmax;
        const int cap = g->seg ? n : qbits;
        Buf<int> shist;
        Buf<long long> shi;
        if (g->seg) {
            shist.alloc(ctx, (size_t)48 * g->nseg);
            shi.alloc(ctx, (size_t)g->nseg);
            hip_ok(hipMemsetAsync(shist.p, 0, shist.count * sizeof(int), s));
        }
        // Two fixed kernel sequences, replayed on one stream.  The commit
        // sequence (iterated) counts the inexact vertices by (bound - c') and
        // commits the round when none is at or below c'; otherwise it stalls
        // and its remaining kernels do nothing.  The recompute sequence then
        // recomputes the smallest bounds (up to 64 Q sources, per graph of a
        // packed union) and lifts the stall.  Every kernel reads its decision
        // from device memory, so the host only checks every few iterations.
        const hipStream_t caller = s;
        Replay rp;
        int32_t* fl[2] = {flA.p, flB.p};
        uint64_t* gain[2] = {gainA.p, gainB.p};
        auto commit_body = [&](hipStream_t q, int iters_per) {
            const hipStream_t keep = s;
            s = q;
            // the round state is reset by the previous round's last kernel (or
            // by the recompute sequence, or before the first replay)
            for (int r = 0; r < iters_per; ++r) {
                launch_reduce_hist(deg.p, alive.p, exact.p, n, st.p, s);
                launch_select_commit(deg.p, alive.p, n, st.p, core.p, rlist.p, mark.p, s, rnd_out);
                delete_round_masked();
                launch_anchor(alist.p, &st.p->aff_fill, n, g->rp, g->col, alive.p, adeg.p, anchor.p, 1, s);
                launch_decay_masked(alist.p, st.p, hopfill.p, h, alive.p, adeg.p, anchor.p, rmask.p, deg.p, exact.p,
                                    s);
                launch_clear_u64_lists3(fl[h & 1], &st.p->fcount[h & 1], gain[h & 1], alist.p, &st.p->aff_fill,
                                        rmask.p, rlist.p, &st.p->rcount, rmask.p, s, st.p, list_grid());
            }
            s = keep;
        };
        const int long_iters = 32, short_iters = 2;
        auto record_long = [&](hipStream_t q) { commit_body(q, long_iters); };
        auto record_short = [&](hipStream_t q) { commit_body(q, short_iters); };
        // Recomputation: count the inexact bounds left by the stalled sweep
        // (per graph too in a packed union), choose and pick the sources.
        auto record_pick = [&](hipStream_t q) {
            launch_bound_hist(alive.p, deg.p, exact.p, n, st.p, q, g->seg, g->seg ? shist.p : nullptr, 0);
            launch_decide(st.p, qbits, q);
            if (g->seg) launch_decide_seg(st.p, g->nseg, shist.p, shi.p, qbits, q);
            launch_pick(alive.p, deg.p, exact.p, n, st.p, srcl.p, cap, q, g->seg, PL.gcnt.p, PL.sbit.p, qbits,
                        g->seg ? shi.p : nullptr);
        };
        // then the bit-parallel BFS of the picked sources with Q words per
        // vertex, and lift the stall
        auto record_bfs = [&](hipStream_t q, int qq) {
            MsPlanes P = PL.view(qq);
            P.exact_out = exact.p;
            ms_batch(P, g->items, n, g->rp, g->col, alive.p, adeg.p, srcl.p, 0, &st.p->rc_count, h, deg.p, st.p, q);
            launch_unstall(st.p, q);
        };
        auto record_recompute = [&](hipStream_t q) {
            record_pick(q);
            record_bfs(q, PL.qmax);
        };
        const bool use_graph = !graphs_off() && !prof_active(ctx);
        PL.timer = prof_active(ctx) ? &ctx->timer[0] : nullptr;
        const hipStream_t q = rp.prepare(caller, use_graph, record_long);
        const int i_short = rp.add(record_short);
        // Commit sequences of several lengths: once a sequence stalls, its
        // remaining iterations only launch kernels that return at once, so the
        // host replays the length closest to the rounds it expects before the
        // next stall (a running average of the rounds between stalls).  Small
        // graphs keep the two lengths (capture costs more than it saves there).
        std::vector<std::pair<int, int>> seqs = {{short_iters, i_short}, {long_iters, 0}};
        if (n >= 100000) {
            // (launched directly when not captured: any length then costs nothing up front)
            for (int L : {4, 8, 16}) seqs.push_back({L, rp.add([&, L](hipStream_t qs) { commit_body(qs, L); })});
            std::sort(seqs.begin(), seqs.end());
        }
        auto pick_len = [&](double want) -> std::pair<int, int> {
            for (const auto& sq : seqs)
                if ((double)sq.first >= want) return sq;
            return seqs.back();
        };
        double ema_run = long_iters;  // rounds between stalls
        long long rounds_prev = 0, since_stall = 0;
        // One graph: the host reads how many sources were picked and replays the
        // BFS captured for the narrowest bit planes that hold them (a batch of
        // 40 sources does not need 16 words per vertex).  A packed union keeps
        // the full width: its sources carry per-graph bit positions.
        const bool adaptive = g->seg == nullptr;
        int i_rec = -1, i_pick = -1;
        std::vector<int> i_bfs(5, -1);
        if (adaptive) {
            i_pick = rp.add(record_pick);
            for (int lq = 0; (1 << lq) <= PL.qmax; ++lq)
                i_bfs[(size_t)lq] = rp.add([&, lq](hipStream_t qs) { record_bfs(qs, 1 << lq); });
        } else {
            i_rec = rp.add(record_recompute);
        }
        bool stalled = false;
        Heartbeat hb;
        for (;;) {
            if (stalled) {
                if (adaptive) {
                    rp.run(record_pick, i_pick);
                    read_state(ctx, st.p, q);
                    const int picked = std::min(hstate(ctx)->rc_count, qbits);
                    const int qq = std::min(PL.qmax, pick_q(std::max(picked, 1)));
                    int lq = 0;
                    while ((1 << lq) < qq) ++lq;
                    rp.run([&](hipStream_t qs) { record_bfs(qs, qq); }, i_bfs[(size_t)lq]);
                } else {
                    rp.run(record_recompute, i_rec);
                }
                rp.run(record_short, i_short);
                iters += short_iters + 1;
            } else {
                const auto sq = pick_len(ema_run - (double)since_stall);
                rp.run([&](hipStream_t qs) { commit_body(qs, sq.first); }, sq.second);
                iters += sq.first;
            }
            if (prof_active(ctx)) prof_collect(ctx);
            read_state(ctx, st.p, q);
            const RoundState hs = *hstate(ctx);
            if (hs.mode == 2) break;
            stalled = hs.stall != 0;
            since_stall += hs.rounds - rounds_prev;
            rounds_prev = hs.rounds;
            if (stalled) {
                ema_run = 0.75 * ema_run + 0.25 * (double)since_stall;
                since_stall = 0;
            }
            if (iters > 8ll * n + 4096) fail(KH_EDEVICE);
            if (hs.fepoch > (1 << 30)) {
                // frontier marks are compared for equality only: restart their epochs
                launch_fill_i32(fmark.p, 0, n, q);
                launch_set_int(&st.p->fepoch, 0, q);
            }
            trace_round(hs, "lazy", t0);
            hb.tick("ExactCore", hs);
        }
        hip_ok(hipStreamSynchronize(q));
        fin = *hstate(ctx);
        prof_add_counters(ctx, fin);
    }

    // Replay deleting by a given core map (key); every round records
    // sum deg_h over the alive set = 2 |E_h(F_K)| (Sec. 6).
    void run_replay(const uint8_t* alive_in, const int64_t* key) {
        kh_context* ctx = g->ctx;
        const int32_t n = g->n;
        const auto t0 = Clock::now();
        build_items(g, s);
        alloc(n);
        launch_alive_from(alive_in, alive.p, n, s);
        launch_alive_degree(g->rp, g->col, alive.p, adeg.p, n, s);
        launch_fill_i32(mark.p, 0, n, s);
        launch_fill_i64(deg.p, 0, n, s);
        launch_fill_i64(core.p, -1, n, s);
        launch_round_reset(st.p, s);
        launch_compact_alive(alive.p, n, srcl.p, &st.p->aff_fill, s);
        read_state(ctx, st.p, s);
        hdeg_sources(g, PL, alive.p, adeg.p, srcl.p, hstate(ctx)->aff_fill, h, deg.p, st.p, s);
        int32_t epoch = 0;
        for (;;) {
            ++epoch;
            launch_round_reset(st.p, s);
            launch_reduce(key, deg.p, alive.p, n, st.p, s);
            launch_round_begin(st.p, ck.p, cs.p, cr.p, 0, s);
            delete_round(epoch, key);
            read_state(ctx, st.p, s);
            const RoundState hs = *hstate(ctx);
            if (hs.alive_count == 0) break;
            if (hs.rounds > n + 1) fail(KH_EDEVICE);
            trace_round(hs, "replay", t0);
            if (hs.aff_fill > 0) hdeg_sources(g, PL, alive.p, adeg.p, alist.p, hs.aff_fill, h, deg.p, st.p, s);
        }
        fin = *hstate(ctx);
        prof_add_counters(ctx, fin);
        cands = read_candidates(fin, ck, cs, cr, s);
    }
};

// ----- sampled engine ---------------------------------------------------------------------------
struct Lists {
    int h = 0;
    int32_t M = 0;
    int hash_log2 = 9;
    std::vector<Buf<int64_t>> cap, off;
    std::vector<Buf<uint32_t>> keys;
    std::vector<Buf<int32_t>> size, m;
    std::vector<Buf<uint8_t>> kk, cut, kold;
    std::vector<Buf<uint32_t>> meta;
    std::vector<Buf<int16_t>> lost;
    std::vector<int64_t> total;
    LevelView view(int i) const {
        LevelView L{};
        if (i < 1 || i > h) return L;
        L.off = off[i].p;
        L.keys = keys[i].p;
        L.size = size[i].p;
        L.k = kk[i].p;
        L.m = m[i].p;
        L.cut = cut[i].p;
        L.lost = lost[i].p;
        L.kold = kold[i].p;
        L.meta = meta[i].p;
        return L;
    }
};

// The union kernel's LDS hash set may exceed M by one entry per thread of the
// block (every thread can pass the "count <= M" test before any insert lands)
// plus the vertex itself; twice that bound keeps the load factor <= 1/2, so
// every probe sequence ends.  The widest block (hubs) sets the size.
int hash_log2_for(int32_t M) { return std::max(9, ceil_log2(2ll * ((long long)M + 1 + kUnionHubThreads))); }
// the same bound for the one-wave blocks of small vertices
int hash_log2_small_for(int32_t M) { return std::max(7, ceil_log2(2ll * ((long long)M + 1 + kUnionSmall))); }

int32_t max_sampled_M(const kh_context* ctx) {
    // dynamic LDS of the union kernel: 4 << hash_log2 bytes, plus ~17 KiB
    // static for the widest block
    int l = 9;
    while (l < 20 && ((size_t)4 << (l + 1)) + 20480 <= ctx->lds_per_block) ++l;
    return (int32_t)((1ll << (l - 1)) - 1 - kUnionHubThreads);
}

struct SampledRun {
    kh_graph* g;
    int h;
    int32_t M;
    uint64_t seed;
    uint32_t stream_id;
    bool early_stop = false;
    // lazy initialisation of level h (Sec. 5 heuristic): B[v,h] is built only once
    // the lower bound from the neighbours' level h-1 lists no longer keeps v above c
    bool lazy = false;
    int32_t* rnd_out = nullptr;  // nullable: deletion round (epoch) of every vertex
    hipStream_t s;
    // packed batches: per-vertex M (nullable; M is then the largest) and the
    // vertex's id inside its own graph, from which its rank is drawn
    const int32_t* Mv = nullptr;
    const int32_t* lid = nullptr;
    Buf<uint8_t> alive, rank, active;
    Buf<int32_t> mark, rlist, wl, rc, hubs, smalls, lostmax, chA, chB, qv, qb, cursor, order;
    Buf<int64_t> d, core, ck, cs, cr, partials;
    Buf<RoundState> st;
    Lists L;
    Candidates cands;
    RoundState fin{};
    // hubs split into slices merged in parallel (HubSplit); slice size from
    // KH_HUB_SLICE (arcs; 0 turns splitting off)
    HubSplit split;
    Buf<int4> units, giants;
    Buf<uint32_t> pkeys;
    Buf<int32_t> pmeta, phk;

    void alloc_split() {
        kh_context* ctx = g->ctx;
        int64_t sl = kHubSlice;
        if (const char* e = std::getenv("KH_HUB_SLICE")) sl = std::atoll(e);
        if (sl <= 0 || h < 2 || g->nnz <= 2 * (int64_t)sl) return;
        // (one slice's arc range must not overflow int32 past the last arc)
        sl = std::min<int64_t>(sl, kMaxHubSlice);
        // a split hub has more than sl arcs and at most deg / sl + 1 slices
        const int64_t slots = 2 * (g->nnz / sl) + 1;
        const int64_t ucap = g->nnz / (kHubDegree + 1) + 1 + slots;
        units.alloc(ctx, (size_t)ucap);
        giants.alloc(ctx, (size_t)(g->nnz / sl + 1));
        pkeys.alloc(ctx, (size_t)slots * (size_t)M);
        pmeta.alloc(ctx, (size_t)slots * 4);
        phk.alloc(ctx, (size_t)slots * 256);
        split.slice = (int32_t)sl;
        split.unit = units.p;
        split.unit_cap = (int32_t)ucap;
        split.giant = giants.p;
        split.pkeys = pkeys.p;
        split.pcap = M;
        split.pmeta = pmeta.p;
        split.phk = phk.p;
        split.slot_cap = (int32_t)slots;
    }

    void alloc_common() {
        kh_context* ctx = g->ctx;
        const int32_t n = g->n;
        alive.alloc(ctx, n);
        rank.alloc(ctx, n);
        mark.alloc(ctx, n);
        rlist.alloc(ctx, n);
        wl.alloc(ctx, n);
        rc.alloc(ctx, n);
        hubs.alloc(ctx, n);
        smalls.alloc(ctx, n);
        lostmax.alloc(ctx, n);
        chA.alloc(ctx, n);
        chB.alloc(ctx, n);
        const size_t qcap = (size_t)n + (size_t)(g->nnz / kExpandChunk) + 2;
        qv.alloc(ctx, qcap);
        qb.alloc(ctx, qcap);
        cursor.alloc(ctx, (size_t)std::max<int64_t>(g->nnz, 1));
        order.alloc(ctx, (size_t)std::max<int64_t>(g->nnz, 1));
        d.alloc(ctx, n);
        core.alloc(ctx, n);
        ck.alloc(ctx, (size_t)n + 1);
        cs.alloc(ctx, (size_t)n + 1);
        cr.alloc(ctx, (size_t)n + 1);
        partials.alloc(ctx, (size_t)n / 2048 + 2);
        st.alloc(ctx, 1);
        alloc_split();
    }

    void build_lists() {
        kh_context* ctx = g->ctx;
        const int32_t n = g->n;
        L.h = h;
        L.M = M;
        L.hash_log2 = hash_log2_for(M);
        L.cap.resize(h + 1);
        L.off.resize(h + 1);
        L.keys.resize(h + 1);
        L.size.resize(h + 1);
        L.kk.resize(h + 1);
        L.m.resize(h + 1);
        L.cut.resize(h + 1);
        L.kold.resize(h + 1);
        L.lost.resize(h + 1);
        L.meta.resize(h + 1);
        L.total.assign(h + 1, 0);
        for (int i = 1; i <= h; ++i) {
            L.cap[i].alloc(ctx, n);
            L.off[i].alloc(ctx, (size_t)n + 1);
            if (i == 1)
                launch_cap_level1(g->rp, n, M, Mv, L.cap[i].p, s);
            else
                launch_cap_next(g->rp, g->col, n, M, Mv, L.cap[i - 1].p, L.cap[i].p, s);
            launch_scan_i64(L.cap[i].p, L.off[i].p, n, partials.p, s);
            int64_t tot = 0;
            hip_ok(hipMemcpyAsync(&tot, L.off[i].p + n, 8, hipMemcpyDeviceToHost, s));
            hip_ok(hipStreamSynchronize(s));
            L.total[i] = tot;
            L.keys[i].alloc(ctx, (size_t)std::max<int64_t>(tot, 1));
            L.size[i].alloc(ctx, n);
            L.kk[i].alloc(ctx, n);
            L.m[i].alloc(ctx, n);
            L.cut[i].alloc(ctx, n);
            L.kold[i].alloc(ctx, n);
            L.lost[i].alloc(ctx, n);
            L.meta[i].alloc(ctx, n);
        }
        for (int i = 1; i < h; ++i) L.cap[i].release();
        if (h >= 1) L.cap[h].release();
    }

    void init_lists() {
        const int32_t n = g->n;
        launch_union1(nullptr, nullptr, n, g->rp, g->col, alive.p, rank.p, M, Mv, L.view(1), nullptr, nullptr, st.p,
                      s);
        kh_context* ctx = g->ctx;
        PullTimer* utimer = prof_active(ctx) ? &ctx->timer[1] : nullptr;
        for (int i = 2; i <= (lazy ? h - 1 : h); ++i) {
            if (utimer && utimer->used + 2 >= utimer->cap) prof_collect(ctx);
            launch_union(nullptr, nullptr, n, g->rp, g->col, alive.p, rank.p, M, Mv, L.hash_log2, L.view(i - 1),
                         L.view(i), cursor.p, order.p, nullptr, nullptr, st.p, s, utimer);
        }
        if (lazy) {
            // every vertex starts inactive at level h, its estimate replaced by the bound
            active.alloc(g->ctx, n);
            hip_ok(hipMemsetAsync(active.p, 0, (size_t)n, s));
            launch_lazy_lb(nullptr, nullptr, n, g->rp, g->col, alive.p, active.p, rank.p, M, Mv, L.view(h - 1), d.p,
                           lostmax.p, s);
        } else {
            launch_estimate(nullptr, nullptr, n, alive.p, rank.p, L.size[h].p, L.kk[h].p, M, Mv, d.p, st.p, s);
        }
    }

    void setup(const uint8_t* alive_in) {
        lazy = lazy && h >= 2;
        alloc_common();
        init_state(st.p, s);
        launch_alive_from(alive_in, alive.p, g->n, s);
        launch_ranks(rank.p, g->n, seed, stream_id, s, lid);
        launch_fill_i32(mark.p, 0, g->n, s);
        launch_fill_i64(core.p, -1, g->n, s);
        launch_fill_i64(d.p, 0, g->n, s);
        launch_fill_i32(lostmax.p, -1, g->n, s);
        build_lists();
        init_lists();
    }

    // Alg. 4's deletion loop in bulk rounds.  key == nullptr: delete by the
    // estimate d (Core).  Otherwise delete by the given core map (the replay of
    // Alg. 7) and record sum d at every level.
    void peel(const int64_t* key_ext) {
        kh_context* ctx = g->ctx;
        const int32_t n = g->n;
        const int64_t* key = key_ext ? key_ext : d.p;
        int32_t* changed[2] = {chA.p, chB.p};
        const int batch = 8;
        const auto t_start = Clock::now();
        PullTimer* utimer = prof_active(ctx) ? &ctx->timer[1] : nullptr;
        const hipStream_t caller = s;
        Replay rp;
        const bool lz = lazy && key_ext == nullptr;
        auto record = [&](hipStream_t q) {
            for (int r = 0; r < batch; ++r) {
                launch_round_reset(st.p, q);
                launch_reduce(key, d.p, alive.p, n, st.p, q, 0, lz ? active.p : nullptr);
                if (lz) {
                    // when an inactive bound is at or below c' = max(c, min d), this
                    // iteration activates every such vertex instead of deleting:
                    // its level-h list is built from scratch, then its estimate
                    launch_lazy_decide(st.p, q);
                    launch_lazy_pick(alive.p, active.p, d.p, n, st.p, rc.p, q);
                    launch_union(rc.p, &st.p->rc_count, n, g->rp, g->col, alive.p, rank.p, M, Mv, L.hash_log2,
                                 L.view(h - 1), L.view(h), cursor.p, order.p, nullptr, nullptr, st.p, q, utimer);
                    launch_estimate(rc.p, &st.p->rc_count, n, alive.p, rank.p, L.size[h].p, L.kk[h].p, M, Mv, d.p,
                                    st.p, q);
                }
                launch_round_begin(st.p, ck.p, cs.p, cr.p, early_stop ? 1 : 0, q);
                launch_select(key, alive.p, n, st.p, core.p, rlist.p, nullptr, 0, 1, q, rnd_out);
                for (int i = 1; i <= h; ++i) {
                    launch_level_reset(st.p, i, q);
                    launch_enqueue(rlist.p, nullptr, &st.p->rcount, g->rp, qv.p, qb.p, &st.p->qcount, q);
                    if (i > 1)
                        launch_enqueue(changed[(i - 1) & 1], nullptr, &st.p->changed_count[(i - 1) & 1], g->rp, qv.p,
                                       qb.p, &st.p->qcount, q);
                    launch_expand_lists(qv.p, qb.p, &st.p->qcount, g->rp, g->col, alive.p, rank.p, mark.p, -1, i,
                                        L.view(i - 1), L.view(i), lostmax.p, wl.p, &st.p->wl_count, st.p, q);
                    // inactive vertices of a lazy level h get a new bound from the level h-1 lists
                    const bool lzh = lz && i == h;
                    if (lzh)
                        launch_lazy_lb(wl.p, &st.p->wl_count, n, g->rp, g->col, alive.p, active.p, rank.p, M, Mv,
                                       L.view(h - 1), d.p, lostmax.p, q);
                    // levels >= 2: hubs are merged by the wide-block variant of the union kernel
                    launch_classify(wl.p, &st.p->wl_count, L.view(i), lostmax.p, rc.p, &st.p->rc_count, q, g->rp,
                                    i > 1 ? hubs.p : nullptr, &st.p->hub_count, lzh ? active.p : nullptr,
                                    i > 1 ? smalls.p : nullptr, &st.p->small_count);
                    if (i == 1)
                        launch_union1(rc.p, &st.p->rc_count, n, g->rp, g->col, alive.p, rank.p, M, Mv, L.view(1),
                                      changed[1], &st.p->changed_count[1], st.p, q);
                    else
                        launch_union(rc.p, &st.p->rc_count, n, g->rp, g->col, alive.p, rank.p, M, Mv, L.hash_log2,
                                     L.view(i - 1), L.view(i), cursor.p, order.p, changed[i & 1],
                                     &st.p->changed_count[i & 1], st.p, q, utimer, hubs.p, &st.p->hub_count,
                                     &split, smalls.p, &st.p->small_count, hash_log2_small_for(M));
                }
                launch_estimate(changed[h & 1], &st.p->changed_count[h & 1], n, alive.p, rank.p, L.size[h].p,
                                L.kk[h].p, M, Mv, d.p, st.p, q);
            }
        };
        const hipStream_t q = rp.prepare(caller, !graphs_off() && !prof_active(ctx), record);
        long long iters = 0;
        Heartbeat hb;
        for (;;) {
            rp.run(record);
            iters += batch;
            if (prof_active(ctx)) prof_collect(ctx);
            read_state(ctx, st.p, q);
            if (hstate(ctx)->alive_count == 0) break;
            // every round deletes at least the minimum vertex, every lazy
            // activation activates at least one vertex
            if (hstate(ctx)->rounds > n + 1 || iters > 2ll * n + 64) fail(KH_EDEVICE);
            hb.tick(key_ext ? "replay" : "Core", *hstate(ctx));
            if (trace_on() && ((hstate(ctx)->rounds & 255) < batch))
                std::fprintf(stderr, "[kh sampled] round %d c %lld alive %d removed %d worklist %d merged %d t %.3fs\n",
                             hstate(ctx)->rounds, hstate(ctx)->c, hstate(ctx)->alive_count,
                             hstate(ctx)->rcount, hstate(ctx)->wl_count, hstate(ctx)->rc_count,
                             std::chrono::duration<double>(Clock::now() - t_start).count());
        }
        hip_ok(hipStreamSynchronize(q));
        fin = *hstate(ctx);
        prof_add_counters(ctx, fin);
        cands = read_candidates(fin, ck, cs, cr, s);
    }
};

void finish_core(kh_context* ctx, const int64_t* core64, int32_t n, int32_t* core_out, bool out_dev, hipStream_t s,
                 int32_t* max_core) {
    Buf<int32_t> tmp;
    Buf<int> ovf;
    ovf.alloc(ctx, 1);
    launch_set_int(ovf.p, 0, s);
    int32_t* dst = core_out;
    if (!out_dev) {
        tmp.alloc(ctx, n);
        dst = tmp.p;
    }
    launch_core_to_i32(core64, dst, n, ovf.p, s);
    int hovf = 0;
    hip_ok(hipMemcpyAsync(&hovf, ovf.p, sizeof(int), hipMemcpyDeviceToHost, s));
    if (!out_dev) hip_ok(hipMemcpyAsync(core_out, tmp.p, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost, s));
    hip_ok(hipStreamSynchronize(s));
    if (hovf) fail(KH_EOVERFLOW);
    if (max_core) {
        int32_t m = 0;
        if (!out_dev) {
            for (int32_t v = 0; v < n; ++v) m = std::max(m, core_out[v]);
        } else {
            std::vector<int32_t> h(n);
            hip_ok(hipMemcpyAsync(h.data(), core_out, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost, s));
            hip_ok(hipStreamSynchronize(s));
            for (int32_t v = 0; v < n; ++v) m = std::max(m, h[v]);
        }
        *max_core = m;
    }
}

int32_t resolve_M(const kh_graph* g, const kh_params* P, bool dense) {
    const int32_t ov = dense ? P->M_dense_override : P->M_override;
    int64_t M = ov > 0 ? ov : kh_buffer_size(std::max<int64_t>(g->n, 1), P->epsilon, P->delta, dense ? 1 : 0);
    if (M < 1) fail(KH_EINVAL);
    if (M > max_sampled_M(g->ctx)) fail(KH_ENOTIMPL);
    return (int32_t)M;
}

int effective_h(const kh_graph* g, int h) {
    // N(v;h,X) is the whole component once h >= |X| - 1
    const int64_t cap = std::max<int64_t>((int64_t)g->n - 1, 1);
    return (int)std::min<int64_t>(h, cap);
}

// Densest core level of a core map given on the device (Sec. 6 / Alg. 7).
void dense_sampled(kh_graph* g, const kh_params* P, const int64_t* core_dev, int64_t maxcore, kh_result* res,
                   hipStream_t s) {
    const int h = effective_h(g, P->h);
    const bool prune = (P->flags & KH_DENSE_PRUNE) != 0;
    SampledRun R;
    R.g = g;
    R.h = h;
    R.M = resolve_M(g, P, true);
    R.seed = P->seed;
    R.stream_id = 1;
    R.s = s;
    Buf<uint8_t> start;
    const uint8_t* alive_in = nullptr;
    if (prune) {
        // only levels K with K (1 + eps) >= (1 - eps) max core take part
        std::vector<int64_t> hc((size_t)g->n);
        hip_ok(hipMemcpyAsync(hc.data(), core_dev, 8 * (size_t)g->n, hipMemcpyDeviceToHost, s));
        hip_ok(hipStreamSynchronize(s));
        const double e = std::min(std::max(P->epsilon, 0.0), 0.999999);
        std::vector<uint8_t> a((size_t)g->n);
        for (int32_t v = 0; v < g->n; ++v) a[v] = (double)hc[v] * (1.0 + e) >= (1.0 - e) * (double)maxcore;
        start.alloc(g->ctx, g->n);
        hip_ok(hipMemcpyAsync(start.p, a.data(), (size_t)g->n, hipMemcpyHostToDevice, s));
        alive_in = start.p;
    }
    R.setup(alive_in);
    R.peel(core_dev);
    pick_dense(R.cands, prune, P->epsilon, maxcore, res);
    res->M_dense_used = R.M;
    res->list_elements += (int64_t)R.fin.elems;
}

void dense_exact(kh_graph* g, const kh_params* P, const int64_t* core_dev, int64_t maxcore, kh_result* res,
                 hipStream_t s) {
    const bool prune = (P->flags & KH_DENSE_PRUNE) != 0;
    ExactRun E;
    E.g = g;
    E.h = effective_h(g, P->h);
    E.s = s;
    Buf<uint8_t> start;
    const uint8_t* alive_in = nullptr;
    if (prune) {
        // exact map: only the innermost level K = max core is a candidate
        std::vector<int64_t> hc((size_t)g->n);
        hip_ok(hipMemcpyAsync(hc.data(), core_dev, 8 * (size_t)g->n, hipMemcpyDeviceToHost, s));
        hip_ok(hipStreamSynchronize(s));
        std::vector<uint8_t> a((size_t)g->n);
        for (int32_t v = 0; v < g->n; ++v) a[v] = hc[v] >= maxcore;
        start.alloc(g->ctx, g->n);
        hip_ok(hipMemcpyAsync(start.p, a.data(), (size_t)g->n, hipMemcpyHostToDevice, s));
        alive_in = start.p;
    }
    E.run_replay(alive_in, core_dev);
    pick_dense(E.cands, prune, 0.0, maxcore, res);
    res->edges_traversed += (int64_t)E.fin.te;
    res->arcs_scanned += (int64_t)E.fin.arcs;
}

// Start set of the pruning variant (end of Sec. 6): {v : core(v) (1 + eps) >=
// (1 - eps) max core}, eps = 0 for an exact map (only the innermost core).
void prune_mask(kh_graph* g, const int64_t* core_dev, int64_t maxcore, double eps, Buf<uint8_t>& start,
                hipStream_t s) {
    std::vector<int64_t> hc((size_t)g->n);
    hip_ok(hipMemcpyAsync(hc.data(), core_dev, 8 * (size_t)g->n, hipMemcpyDeviceToHost, s));
    hip_ok(hipStreamSynchronize(s));
    const double e = std::min(std::max(eps, 0.0), 0.999999);
    std::vector<uint8_t> a((size_t)g->n);
    for (int32_t v = 0; v < g->n; ++v) a[v] = (double)hc[v] * (1.0 + e) >= (1.0 - e) * (double)maxcore;
    start.alloc(g->ctx, g->n);
    hip_ok(hipMemcpyAsync(start.p, a.data(), (size_t)g->n, hipMemcpyHostToDevice, s));
    hip_ok(hipStreamSynchronize(s));
}

// Alg. 7 over every suffix of the peel's deletion order (flag KH_DENSE_FULL).
// The order: rounds in sequence, inside a round by the key at deletion (key_dev:
// the estimate, or deg_h), then by k[v,h] (lev_dev, nullable for ExactCore),
// then by id.  The replay deletes one vertex per round in that order (key =
// position), recording sum f over the remaining suffix before each deletion,
// with fresh ranks and M from C = log(n^2/delta) on the sampled path.
void dense_full(kh_graph* g, const kh_params* P, const int64_t* core_dev, const int64_t* key_dev,
                const uint8_t* lev_dev, const int32_t* rnd_dev, int64_t maxcore, bool sampled, kh_result* res,
                hipStream_t s) {
    kh_context* ctx = g->ctx;
    const int32_t n = g->n;
    Buf<int32_t> order;
    Buf<int64_t> pos;
    order.alloc(ctx, n);
    pos.alloc(ctx, n);
    {
        Buf<uint32_t> lk, lk2;
        Buf<int32_t> ids, ids2;
        Buf<uint64_t> mk, mk2;
        Buf<unsigned char> temp;
        Buf<int> bad;
        lk.alloc(ctx, n);
        lk2.alloc(ctx, n);
        ids.alloc(ctx, n);
        ids2.alloc(ctx, n);
        mk.alloc(ctx, n);
        mk2.alloc(ctx, n);
        OrderScratch w{lk.p, lk2.p, ids.p, ids2.p, mk.p, mk2.p, nullptr, order_temp_bytes(n)};
        temp.alloc(ctx, w.temp_bytes);
        w.temp = temp.p;
        bad.alloc(ctx, 1);
        launch_set_int(bad.p, 0, s);
        hip_ok(deletion_order(n, rnd_dev, key_dev, lev_dev, w, order.p, pos.p, bad.p, s));
        int hbad = 0;
        hip_ok(hipMemcpyAsync(&hbad, bad.p, sizeof(int), hipMemcpyDeviceToHost, s));
        hip_ok(hipStreamSynchronize(s));
        if (hbad) fail(KH_EOVERFLOW);
    }
    const bool prune = (P->flags & KH_DENSE_PRUNE) != 0;
    Buf<uint8_t> start;
    if (prune) prune_mask(g, core_dev, maxcore, sampled ? P->epsilon : 0.0, start, s);
    const uint8_t* alive_in = prune ? start.p : nullptr;
    Candidates C;
    if (sampled) {
        SampledRun R;
        R.g = g;
        R.h = effective_h(g, P->h);
        R.M = resolve_M(g, P, true);
        R.seed = P->seed;
        R.stream_id = 1;
        R.s = s;
        R.setup(alive_in);
        R.peel(pos.p);
        C = R.cands;
        res->M_dense_used = R.M;
        res->list_elements += (int64_t)R.fin.elems;
    } else {
        ExactRun E;
        E.g = g;
        E.h = effective_h(g, P->h);
        E.s = s;
        E.run_replay(alive_in, pos.p);
        C = E.cands;
        res->edges_traversed += (int64_t)E.fin.te;
        res->arcs_scanned += (int64_t)E.fin.arcs;
    }
    // candidates are positions; ties go to the later suffix (the smaller set)
    pick_dense(C, false, 0.0, 0, res);
    if (res->dense_k >= 0) {
        // report the smallest core number in the chosen suffix: that of its first vertex
        int32_t v = 0;
        int64_t c = 0;
        hip_ok(hipMemcpyAsync(&v, order.p + res->dense_k, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        hip_ok(hipStreamSynchronize(s));
        hip_ok(hipMemcpyAsync(&c, core_dev + v, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        hip_ok(hipStreamSynchronize(s));
        res->dense_k = c;
    }
}

void clear_result(kh_result* r) {
    std::memset(r, 0, sizeof(*r));
    r->dense_k = -1;
}

}  // namespace

// ---------------------------------------------------------------------------------------------
// the hot path
// ---------------------------------------------------------------------------------------------
extern "C" kh_status kh_core(kh_graph* g, const kh_params* P, int32_t* core_out, kh_result* res, void* stream) {
    const auto t0 = Clock::now();
    kh_result local;
    kh_result* R = res ? res : &local;
    clear_result(R);
    try {
        check_params(g, P);
        if (g->n > 0 && !core_out) fail(KH_EINVAL);
        hip_ok(hipSetDevice(g->ctx->device));
        StateLease lease(g->ctx);
        auto s = static_cast<hipStream_t>(stream);
        const bool out_dev = (P->flags & KH_OUT_DEVICE) != 0;
        const bool want_dense = (P->flags & KH_WANT_DENSE) != 0;
        if (g->n == 0) {
            R->seconds = std::chrono::duration<double>(Clock::now() - t0).count();
            return KH_OK;
        }
        const int h = effective_h(g, P->h);
        const bool full_dense = want_dense && (P->flags & KH_DENSE_FULL);
        Buf<int32_t> rnd;
        if (full_dense) {
            if (P->epsilon > 0.0 && (P->flags & KH_EARLY_STOP)) fail(KH_ENOTIMPL);
            rnd.alloc(g->ctx, g->n);
            launch_fill_i32(rnd.p, -1, g->n, s);
        }
        if (P->epsilon <= 0.0) {
            ExactRun E;
            E.g = g;
            E.h = h;
            E.s = s;
            E.rnd_out = rnd.p;
            E.run_lazy();
            finish_core(g->ctx, E.core.p, g->n, core_out, out_dev, s, &R->max_core);
            R->rounds = E.fin.rounds;
            R->edges_traversed = (int64_t)E.fin.te;
            R->arcs_scanned = (int64_t)E.fin.arcs;
            if (full_dense) dense_full(g, P, E.core.p, E.deg.p, nullptr, rnd.p, R->max_core, false, R, s);
            else if (want_dense) dense_exact(g, P, E.core.p, R->max_core, R, s);
        } else {
            if (g->n > kMaxSampledN) fail(KH_ENOTIMPL);
            SampledRun S;
            S.g = g;
            S.h = h;
            S.M = resolve_M(g, P, false);
            S.seed = P->seed;
            S.stream_id = 0;
            S.early_stop = (P->flags & KH_EARLY_STOP) != 0;
            S.lazy = (P->flags & KH_LAZY_INIT) != 0;
            S.rnd_out = rnd.p;
            S.s = s;
            S.setup(nullptr);
            S.peel(nullptr);
            if (S.fin.overflow) fail(KH_EOVERFLOW);
            finish_core(g->ctx, S.core.p, g->n, core_out, out_dev, s, &R->max_core);
            R->M_used = S.M;
            R->rounds = S.fin.rounds;
            R->list_elements = (int64_t)S.fin.elems;
            if (want_dense) {
                // free the core pass's lists before the dense pass allocates its own
                for (auto& k : S.L.keys) k.release();
                if (full_dense)
                    dense_full(g, P, S.core.p, S.d.p, S.L.kk[(size_t)h].p, rnd.p, R->max_core, true, R, s);
                else
                    dense_sampled(g, P, S.core.p, R->max_core, R, s);
            }
        }
    } catch (const KhError& e) {
        return e.code;
    } catch (const std::bad_alloc&) {
        return KH_ENOMEM;
    }
    R->seconds = std::chrono::duration<double>(Clock::now() - t0).count();
    return KH_OK;
}

// ---------------------------------------------------------------------------------------------
// batches: many graphs packed into one disjoint union
// ---------------------------------------------------------------------------------------------
// Components of a disjoint union never interact: N(v;h,X) stays inside v's
// graph, so every h-degree, sample list and estimate of the union equals the
// one of the graph alone, and the running-maximum peel of the union yields
// each graph's own core numbers (Sec. 2's characterisation as the largest k
// with a witness set containing v; a witness restricted to v's graph is still
// one).  For the sampled path each vertex draws its rank from its id inside
// its own graph and uses its own graph's M (Eq. (buffer) with that graph's n),
// so the numbers are those of kh_core on the graph alone.
namespace {

struct Packed {
    kh_graph G;
    std::vector<int32_t> v_off;  // first vertex of each graph (count + 1 entries)
    std::vector<int64_t> a_off;  // first arc of each graph
    Buf<int32_t> lid, Mv;
};

void pack(kh_context* ctx, kh_graph* const* gs, int32_t count, Packed& P, bool sampled, const int32_t* Ms,
          hipStream_t s) {
    P.v_off.assign((size_t)count + 1, 0);
    P.a_off.assign((size_t)count + 1, 0);
    for (int32_t i = 0; i < count; ++i) {
        P.v_off[i + 1] = P.v_off[i] + gs[i]->n;
        P.a_off[i + 1] = P.a_off[i] + gs[i]->nnz;
    }
    const int32_t n = P.v_off[count];
    const int64_t nnz = P.a_off[count];
    kh_graph& G = P.G;
    G.ctx = ctx;
    G.n = n;
    G.nnz = nnz;
    G.h_rp.resize((size_t)n + 1);
    for (int32_t i = 0; i < count; ++i) {
        const int32_t* r = gs[i]->h_rp.data();
        const int32_t a = (int32_t)P.a_off[i];
        int32_t* dst = G.h_rp.data() + P.v_off[i];
        for (int32_t v = 0; v < gs[i]->n; ++v) dst[v] = a + r[v];
    }
    G.h_rp[n] = (int32_t)nnz;
    G.rp_own.alloc(ctx, (size_t)n + 1);
    G.col_own.alloc(ctx, (size_t)std::max<int64_t>(nnz, 1));
    hip_ok(hipMemcpyAsync(G.rp_own.p, G.h_rp.data(), 4 * ((size_t)n + 1), hipMemcpyHostToDevice, s));
    std::vector<uint64_t> cp((size_t)count);
    for (int32_t i = 0; i < count; ++i) cp[i] = reinterpret_cast<uint64_t>(gs[i]->col);
    Buf<int64_t> d_aoff;
    Buf<int32_t> d_voff;
    Buf<uint64_t> d_cp;
    d_aoff.alloc(ctx, (size_t)count + 1);
    d_voff.alloc(ctx, (size_t)count + 1);
    d_cp.alloc(ctx, (size_t)count);
    hip_ok(hipMemcpyAsync(d_aoff.p, P.a_off.data(), 8 * ((size_t)count + 1), hipMemcpyHostToDevice, s));
    hip_ok(hipMemcpyAsync(d_voff.p, P.v_off.data(), 4 * ((size_t)count + 1), hipMemcpyHostToDevice, s));
    hip_ok(hipMemcpyAsync(d_cp.p, cp.data(), 8 * (size_t)count, hipMemcpyHostToDevice, s));
    launch_pack_col(count, d_aoff.p, d_voff.p, d_cp.p, nnz, G.col_own.p, s);
    if (sampled) {
        std::vector<int32_t> hl((size_t)n), hm((size_t)n);
        for (int32_t i = 0; i < count; ++i)
            for (int32_t v = 0; v < gs[i]->n; ++v) {
                hl[(size_t)P.v_off[i] + v] = v;
                hm[(size_t)P.v_off[i] + v] = Ms[i];
            }
        P.lid.alloc(ctx, n);
        P.Mv.alloc(ctx, n);
        hip_ok(hipMemcpyAsync(P.lid.p, hl.data(), 4 * (size_t)n, hipMemcpyHostToDevice, s));
        hip_ok(hipMemcpyAsync(P.Mv.p, hm.data(), 4 * (size_t)n, hipMemcpyHostToDevice, s));
    }
    std::vector<int32_t> hseg((size_t)std::max(n, 1), 0);
    for (int32_t i = 0; i < count; ++i)
        std::fill(hseg.begin() + P.v_off[i], hseg.begin() + P.v_off[i + 1], i);
    G.seg_own.alloc(ctx, hseg.size());
    hip_ok(hipMemcpyAsync(G.seg_own.p, hseg.data(), 4 * hseg.size(), hipMemcpyHostToDevice, s));
    G.seg = G.seg_own.p;
    G.nseg = count;
    hip_ok(hipStreamSynchronize(s));  // the host tables above go out of scope
    G.rp = G.rp_own.p;
    G.col = G.col_own.p;
}

// One packed run over gs[0..count) (all with n > 0).
void batch_chunk(kh_context* ctx, kh_graph* const* gs, int32_t count, const kh_params* P, int32_t* const* outs,
                 kh_result* results, hipStream_t s) {
    const auto t0 = Clock::now();
    const bool sampled = P->epsilon > 0.0;
    const bool out_dev = (P->flags & KH_OUT_DEVICE) != 0;
    std::vector<int32_t> Ms((size_t)count, 0);
    int32_t Mmax = 0;
    if (sampled)
        for (int32_t i = 0; i < count; ++i) {
            Ms[i] = resolve_M(gs[i], P, false);
            Mmax = std::max(Mmax, Ms[i]);
        }
    Packed PK;
    pack(ctx, gs, count, PK, sampled, Ms.data(), s);
    kh_graph* g = &PK.G;
    const int32_t n = g->n;
    const int h = effective_h(g, P->h);
    ExactRun E;
    SampledRun S;
    const int64_t* core64 = nullptr;
    RoundState fin{};
    if (!sampled) {
        E.g = g;
        E.h = h;
        E.s = s;
        E.run_lazy();
        core64 = E.core.p;
        fin = E.fin;
    } else {
        S.g = g;
        S.h = h;
        S.M = Mmax;
        S.Mv = PK.Mv.p;
        S.lid = PK.lid.p;
        S.seed = P->seed;
        S.stream_id = 0;
        S.lazy = (P->flags & KH_LAZY_INIT) != 0;
        S.s = s;
        S.setup(nullptr);
        S.peel(nullptr);
        if (S.fin.overflow) fail(KH_EOVERFLOW);
        core64 = S.core.p;
        fin = S.fin;
        for (auto& k : S.L.keys) k.release();
    }
    Buf<int32_t> c32;
    c32.alloc(ctx, n);
    finish_core(ctx, core64, n, c32.p, true, s, nullptr);
    std::vector<int32_t> hc((size_t)n);
    hip_ok(hipMemcpyAsync(hc.data(), c32.p, 4 * (size_t)n, hipMemcpyDeviceToHost, s));
    if (out_dev) {
        std::vector<uint64_t> dp((size_t)count);
        for (int32_t i = 0; i < count; ++i) dp[i] = reinterpret_cast<uint64_t>(outs[i]);
        Buf<int32_t> d_voff;
        Buf<uint64_t> d_dp;
        d_voff.alloc(ctx, (size_t)count + 1);
        d_dp.alloc(ctx, (size_t)count);
        hip_ok(hipMemcpyAsync(d_voff.p, PK.v_off.data(), 4 * ((size_t)count + 1), hipMemcpyHostToDevice, s));
        hip_ok(hipMemcpyAsync(d_dp.p, dp.data(), 8 * (size_t)count, hipMemcpyHostToDevice, s));
        launch_unpack_i32(count, d_voff.p, d_dp.p, n, c32.p, s);
        hip_ok(hipStreamSynchronize(s));
    } else {
        hip_ok(hipStreamSynchronize(s));
        for (int32_t i = 0; i < count; ++i)
            std::memcpy(outs[i], hc.data() + PK.v_off[i], 4 * (size_t)gs[i]->n);
    }
    const double secs = std::chrono::duration<double>(Clock::now() - t0).count();
    for (int32_t i = 0; i < count; ++i) {
        if (!results) break;
        kh_result* R = &results[i];
        int32_t m = 0;
        for (int32_t v = PK.v_off[i]; v < PK.v_off[i + 1]; ++v) m = std::max(m, hc[v]);
        R->max_core = m;
        R->M_used = Ms[i];
        R->rounds = fin.rounds;
        R->edges_traversed = (int64_t)fin.te;
        R->arcs_scanned = (int64_t)fin.arcs;
        R->list_elements = (int64_t)fin.elems;
        R->seconds = secs;
    }
    prof_add_counters(ctx, fin);
    if (results && (P->flags & KH_WANT_DENSE)) {
        // the densest core is a per-graph quantity: one pass per graph over its
        // slice of the packed core map
        for (int32_t i = 0; i < count; ++i) {
            const int64_t* slice = core64 + PK.v_off[i];
            if (sampled) dense_sampled(gs[i], P, slice, results[i].max_core, &results[i], s);
            else dense_exact(gs[i], P, slice, results[i].max_core, &results[i], s);
        }
    }
}

}  // namespace

extern "C" kh_status kh_core_batch(kh_context* ctx, int32_t count, kh_graph* const* graphs, const kh_params* P,
                                   int32_t* const* core_outs, kh_result* results, void* stream) {
    try {
        if (!ctx || count < 0 || (count > 0 && (!graphs || !core_outs))) fail(KH_EINVAL);
        if (count == 0) return KH_OK;
        if ((P->flags & KH_WANT_DENSE) && (P->flags & KH_DENSE_FULL)) fail(KH_ENOTIMPL);
        for (int32_t i = 0; i < count; ++i) {
            check_params(graphs[i], P);
            if (graphs[i]->ctx != ctx) fail(KH_EINVAL);
            if (graphs[i]->n > 0 && !core_outs[i]) fail(KH_EINVAL);
            if (results) clear_result(&results[i]);
        }
        if (P->flags & KH_EARLY_STOP) fail(KH_ENOTIMPL);
        hip_ok(hipSetDevice(ctx->device));
        StateLease lease(ctx);
        auto s = static_cast<hipStream_t>(stream);
        const bool sampled = P->epsilon > 0.0;
        // chunks of consecutive non-empty graphs: packed ids and arc offsets stay
        // in int32, sampled keys hold 24-bit ids
        int64_t vmax = sampled ? (int64_t)kMaxSampledN : (int64_t)INT32_MAX - 1;
        // KH_BATCH_MAX_VERTICES (tests): smaller unions
        if (const char* e = std::getenv("KH_BATCH_MAX_VERTICES")) {
            const long long x = std::atoll(e);
            if (x > 0) vmax = std::min<int64_t>(vmax, x);
        }
        std::vector<kh_graph*> cg;
        std::vector<int32_t*> co;
        std::vector<int32_t> ci;
        int64_t vn = 0, an = 0;
        auto flush = [&]() {
            if (cg.empty()) return;
            std::vector<kh_result> rs(cg.size());
            for (auto& r : rs) clear_result(&r);
            batch_chunk(ctx, cg.data(), (int32_t)cg.size(), P, co.data(), results ? rs.data() : nullptr, s);
            if (results)
                for (size_t j = 0; j < cg.size(); ++j) results[ci[j]] = rs[j];
            cg.clear();
            co.clear();
            ci.clear();
            vn = an = 0;
        };
        // Graphs are packed in order of size.  Unions are not split further by
        // size: a union's rounds follow the distinct core values of all its
        // graphs, and separate unions of similar graphs repeat most of those
        // rounds one after the other (measured slower at h = 3 on the
        // 4,096-graph workload than one union per size cap).
        std::vector<int32_t> idx;
        for (int32_t i = 0; i < count; ++i) {
            if (graphs[i]->n == 0) continue;
            if (sampled && graphs[i]->n > kMaxSampledN) fail(KH_ENOTIMPL);
            idx.push_back(i);
        }
        std::stable_sort(idx.begin(), idx.end(), [&](int32_t a, int32_t b) { return graphs[a]->n < graphs[b]->n; });
        for (int32_t i : idx) {
            kh_graph* g = graphs[i];
            if (vn + g->n > vmax || an + g->nnz > kMaxArcs) flush();
            cg.push_back(g);
            co.push_back(core_outs[i]);
            ci.push_back(i);
            vn += g->n;
            an += g->nnz;
        }
        flush();
    } catch (const KhError& e) {
        return e.code;
    } catch (const std::bad_alloc&) {
        return KH_ENOMEM;
    }
    return KH_OK;
}

extern "C" kh_status kh_hdeg(kh_graph* g, int32_t h, const uint8_t* alive_in, uint32_t flags, int32_t* deg_out,
                             int64_t* edges_traversed, void* stream) {
    try {
        if (!g || h < 1) fail(KH_EINVAL);
        if (g->n > 0 && !deg_out) fail(KH_EINVAL);
        if (g->n == 0) return KH_OK;
        hip_ok(hipSetDevice(g->ctx->device));
        StateLease lease(g->ctx);
        auto s = static_cast<hipStream_t>(stream);
        kh_context* ctx = g->ctx;
        const int32_t n = g->n;
        const int he = effective_h(g, h);
        build_items(g, s);
        Buf<uint8_t> alive;
        Buf<int32_t> adeg, srcl;
        Buf<int64_t> deg, core;
        Buf<RoundState> st;
        Planes PL;
        alive.alloc(ctx, n);
        adeg.alloc(ctx, n);
        srcl.alloc(ctx, n);
        deg.alloc(ctx, n);
        st.alloc(ctx, 1);
        PL.alloc(ctx, n, g->nnz, pick_q(n), g->items.nitems);
        PL.clear(s);
        init_state(st.p, s);
        launch_alive_from(alive_in, alive.p, n, s);
        launch_alive_degree(g->rp, g->col, alive.p, adeg.p, n, s);
        launch_fill_i64(deg.p, -1, n, s);
        launch_round_reset(st.p, s);
        launch_compact_alive(alive.p, n, srcl.p, &st.p->aff_fill, s);
        read_state(ctx, st.p, s);
        hdeg_sources(g, PL, alive.p, adeg.p, srcl.p, hstate(ctx)->aff_fill, he, deg.p, st.p, s);
        finish_core(ctx, deg.p, n, deg_out, (flags & KH_OUT_DEVICE) != 0, s, nullptr);
        read_state(ctx, st.p, s);
        if (edges_traversed) *edges_traversed = (int64_t)hstate(ctx)->te;
        prof_add_counters(ctx, *hstate(ctx));
    } catch (const KhError& e) {
        return e.code;
    } catch (const std::bad_alloc&) {
        return KH_ENOMEM;
    }
    return KH_OK;
}

// No device allocation, no host wait: the working memory is the context's
// device's fixed array (kh_noalloc.hip); the pull kernel's work-item counts come
// from the host copy of row_ptr.
extern "C" kh_status kh_hdeg_noalloc(kh_graph* g, int32_t h, const uint8_t* alive, int32_t* deg_out,
                                     int64_t* edges_traversed, void* stream) {
    if (!g || h < 1) return KH_EINVAL;
    if (g->n > 0 && !deg_out) return KH_EINVAL;
    kh_context* ctx = g->ctx;
    if (!ctx->noalloc_scratch) return KH_EDEVICE;
    if (hipSetDevice(ctx->device) != hipSuccess) {
        (void)hipGetLastError();
        return KH_EDEVICE;
    }
    int64_t nitems = 0, nsplit = 0;
    for (int32_t v = 0; v < g->n; ++v) {
        const int32_t d = g->h_rp[(size_t)v + 1] - g->h_rp[(size_t)v];
        if (d > kPullChunk) {
            nitems += (d + kPullChunk - 1) / kPullChunk;
            ++nsplit;
        } else if (d > 0) {
            ++nitems;
        }
    }
    return noalloc_hdeg(ctx->noalloc_scratch, g->n, g->nnz, g->rp, g->col, nitems, nsplit, effective_h(g, h), alive,
                        deg_out, edges_traversed, static_cast<hipStream_t>(stream));
}

extern "C" kh_status kh_ranks(kh_context* ctx, int32_t n, uint64_t seed, uint32_t stream_id, uint8_t* r_out,
                              void* stream) {
    if (!ctx || n < 0 || (n > 0 && !r_out)) return KH_EINVAL;
    try {
        hip_ok(hipSetDevice(ctx->device));
        auto s = static_cast<hipStream_t>(stream);
        launch_ranks(r_out, n, seed, stream_id, s);
        hip_ok(hipGetLastError());
    } catch (const KhError& e) {
        return e.code;
    }
    return KH_OK;
}

extern "C" kh_status kh_sampled_lists(kh_graph* g, const kh_params* P, const uint8_t* alive_in, int32_t level,
                                      int32_t* k_out, int32_t* size_out, int32_t* members_out, int64_t members_cap,
                                      int64_t* est_out, void* stream) {
    try {
        check_params(g, P);
        if (!(P->epsilon > 0.0) && P->M_override <= 0) fail(KH_EINVAL);
        if (level < 1 || level > P->h) fail(KH_EINVAL);
        if (g->n > 0 && (!k_out || !size_out)) fail(KH_EINVAL);
        if (g->n == 0) return KH_OK;
        if (g->n > kMaxSampledN) fail(KH_ENOTIMPL);
        hip_ok(hipSetDevice(g->ctx->device));
        StateLease lease(g->ctx);
        auto s = static_cast<hipStream_t>(stream);
        const int32_t n = g->n;
        SampledRun S;
        S.g = g;
        S.h = P->h;
        S.M = resolve_M(g, P, false);
        S.seed = P->seed;
        S.stream_id = 0;
        S.s = s;
        S.setup(alive_in);
        std::vector<uint8_t> ha((size_t)n), hk((size_t)n);
        std::vector<int32_t> hs((size_t)n);
        std::vector<int64_t> ho((size_t)n + 1);
        hip_ok(hipMemcpyAsync(ha.data(), S.alive.p, (size_t)n, hipMemcpyDeviceToHost, s));
        hip_ok(hipMemcpyAsync(hk.data(), S.L.kk[level].p, (size_t)n, hipMemcpyDeviceToHost, s));
        hip_ok(hipMemcpyAsync(hs.data(), S.L.size[level].p, 4 * (size_t)n, hipMemcpyDeviceToHost, s));
        hip_ok(hipMemcpyAsync(ho.data(), S.L.off[level].p, 8 * ((size_t)n + 1), hipMemcpyDeviceToHost, s));
        std::vector<uint32_t> hkeys((size_t)std::max<int64_t>(S.L.total[level], 1));
        hip_ok(hipMemcpyAsync(hkeys.data(), S.L.keys[level].p, 4 * (size_t)S.L.total[level], hipMemcpyDeviceToHost, s));
        if (est_out) hip_ok(hipMemcpyAsync(est_out, S.d.p, 8 * (size_t)n, hipMemcpyDeviceToHost, s));
        hip_ok(hipStreamSynchronize(s));
        int64_t total = 0;
        for (int32_t v = 0; v < n; ++v) {
            if (!ha[v]) {
                k_out[v] = -1;
                size_out[v] = 0;
                if (est_out) est_out[v] = -1;
                continue;
            }
            k_out[v] = hk[v];
            size_out[v] = hs[v];
            if (members_out) {
                if (total + hs[v] > members_cap) fail(KH_EINVAL);
                int32_t* dst = members_out + total;
                for (int32_t i = 0; i < hs[v]; ++i) dst[i] = (int32_t)(hkeys[(size_t)ho[v] + i] & 0xFFFFFFu);
                std::sort(dst, dst + hs[v]);
            }
            total += hs[v];
        }
    } catch (const KhError& e) {
        return e.code;
    } catch (const std::bad_alloc&) {
        return KH_ENOMEM;
    }
    return KH_OK;
}

extern "C" kh_status kh_dense(kh_graph* g, const kh_params* P, const int32_t* core_in, kh_result* res, void* stream) {
    try {
        check_params(g, P);
        if (!res || (g->n > 0 && !core_in)) fail(KH_EINVAL);
        clear_result(res);
        if (P->flags & KH_DENSE_FULL) fail(KH_ENOTIMPL);  // the order comes from the peel itself
        if (g->n == 0) return KH_OK;
        hip_ok(hipSetDevice(g->ctx->device));
        StateLease lease(g->ctx);
        auto s = static_cast<hipStream_t>(stream);
        const int32_t n = g->n;
        std::vector<int64_t> hc((size_t)n);
        int64_t maxcore = 0;
        for (int32_t v = 0; v < n; ++v) {
            if (core_in[v] < 0) fail(KH_EINVAL);
            hc[v] = core_in[v];
            maxcore = std::max<int64_t>(maxcore, hc[v]);
        }
        Buf<int64_t> cd;
        cd.alloc(g->ctx, n);
        hip_ok(hipMemcpyAsync(cd.p, hc.data(), 8 * (size_t)n, hipMemcpyHostToDevice, s));
        if (P->epsilon <= 0.0) {
            dense_exact(g, P, cd.p, maxcore, res, s);
        } else {
            if (n > kMaxSampledN) fail(KH_ENOTIMPL);
            dense_sampled(g, P, cd.p, maxcore, res, s);
        }
    } catch (const KhError& e) {
        return e.code;
    } catch (const std::bad_alloc&) {
        return KH_ENOMEM;
    }
    return KH_OK;
}
