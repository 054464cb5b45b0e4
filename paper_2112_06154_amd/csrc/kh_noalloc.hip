// h-degrees without device allocation: kh_hdeg_noalloc keeps every piece of
// its working memory in one fixed device array per GPU (`scratch` below), for
// callers that cannot allocate (code recorded into HIP graphs, tight serving
// loops, harnesses that forbid allocation).  The computation is kh_hdeg's:
// deg_h(v;X) = |N(v;h,X)| - 1 (Sec. 2) by the bit-parallel multi-source BFS of
// kh_msbfs.hip, batches of 64 Q sources.
//
// The pull kernel's work items, which kh_hdeg builds on the host once per
// graph, are built here on the device in the scratch array at every call:
// every vertex's arcs cut into pieces of at most kPullChunk arcs, in vertex
// order (kh_hdeg sorts them by length, which only changes the speed).  Batch
// sizes are read on the device, so the call never waits for the GPU: it only
// enqueues kernels on the caller's stream.
#include <algorithm>
#include <cstddef>
#include <mutex>

#include "kh_common.hpp"
#include "kh_internal.hpp"

namespace kh {

// The fixed working array.  In host code its name is only a stand-in: every
// host-side use goes through the address hipGetSymbolAddress returned for the
// current device (noalloc_scratch_init).
static_assert(kNoallocScratchBytes == KH_NOALLOC_SCRATCH_BYTES, "the array size is part of the C ABI");
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

namespace {
std::mutex g_scratch_lock;
void* g_scratch_addr[kMaxDevices] = {};
}  // namespace

hipError_t noalloc_scratch_init(int device, void** out) {
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_lock);
    if (!g_scratch_addr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_addr[device] = p;
    }
    *out = g_scratch_addr[device];
    return hipSuccess;
}

namespace {

__global__ void k_items_count(const int32_t* __restrict__ rp, int32_t n, int64_t* __restrict__ cnt) {
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        const int32_t d = rp[v + 1] - rp[v];
        cnt[v] = d <= 0 ? 0 : (d > kPullChunk ? (d + kPullChunk - 1) / kPullChunk : 1);
    }
}

// Items of vertex v occupy off[v] .. off[v+1]-1; vitem[v] = off[v] (-1 without arcs).
__global__ void k_items_fill(const int32_t* __restrict__ rp, int32_t n, const int64_t* __restrict__ off,
                             int32_t* __restrict__ iu, int32_t* __restrict__ ib, int32_t* __restrict__ ie,
                             uint8_t* __restrict__ isp, int32_t* __restrict__ vitem, int32_t* __restrict__ split_list,
                             int* split_count) {
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        const int32_t b = rp[v], e = rp[v + 1];
        const int32_t first = (int32_t)off[v];
        vitem[v] = e > b ? first : -1;
        const bool split = e - b > kPullChunk;
        int32_t k = first;
        for (int32_t p = b; p < e; p += kPullChunk, ++k) {
            iu[k] = v;
            ib[k] = p;
            ie[k] = min(p + kPullChunk, e);
            isp[k] = split ? 1 : 0;
        }
        if (split) split_list[atomicAdd(split_count, 1)] = v;
    }
}

__global__ void k_state_zero(RoundState* st) {
    uint32_t* w = reinterpret_cast<uint32_t*>(st);
    for (int i = threadIdx.x; i < (int)(sizeof(RoundState) / 4); i += blockDim.x) w[i] = 0u;
    __syncthreads();
    if (threadIdx.x == 0) st->c = -1;
}

// Sources of batch b: alive list entries b*cap .. ; their count, read by the batch's kernels.
__global__ void k_batch_count(const RoundState* st, int64_t b, int cap, int* out) {
    const long long rest = (long long)st->aff_fill - b * (long long)cap;
    *out = (int)(rest <= 0 ? 0 : (rest > cap ? cap : rest));
}

__global__ void k_te_out(const RoundState* st, int64_t* out) { *out = (int64_t)st->te; }

inline size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }

// Carves consecutive 256-byte aligned regions out of the array starting at
// `base` (base 0 only measures the layout).
struct Carver {
    uintptr_t base;
    size_t used = 0;
    template <typename T>
    T* take(size_t count) {
        T* p = reinterpret_cast<T*>(base + used);
        used += up256(std::max<size_t>(count, 1) * sizeof(T));
        return p;
    }
};

struct Layout {
    uint8_t* alive;
    int32_t *adeg, *srcl, *bcount, *ovf;
    int64_t *deg, *cnt_items, *off_items, *partials;
    RoundState* st;
    MsPlanes P;
    MsItems I;
    int* split_count;
    size_t bytes;
};

Layout carve(uintptr_t base, int32_t n, int64_t nnz, int64_t nitems, int64_t nsplit, int Q) {
    Carver c{base};
    Layout L{};
    const size_t nn = (size_t)std::max(n, 1);
    const size_t bm = (nn + 31) / 32;
    const size_t ntiles = (nn + 63) / 64;
    L.st = c.take<RoundState>(1);
    L.bcount = c.take<int32_t>(1);
    L.ovf = c.take<int32_t>(1);
    L.split_count = c.take<int>(1);
    L.alive = c.take<uint8_t>(nn);
    L.adeg = c.take<int32_t>(nn);
    L.srcl = c.take<int32_t>(nn);
    L.deg = c.take<int64_t>(nn);
    L.cnt_items = c.take<int64_t>(nn);
    L.off_items = c.take<int64_t>(nn + 1);
    L.partials = c.take<int64_t>(nn / 2048 + 2);
    MsPlanes& P = L.P;
    P.Q = Q;
    P.vis = c.take<uint64_t>(nn * Q);
    P.frA = c.take<uint64_t>(nn * Q);
    P.frB = c.take<uint64_t>(nn * Q);
    P.acc = c.take<uint64_t>(nn * Q);
    P.valid = c.take<uint64_t>(16);
    P.bmA = c.take<uint32_t>(bm);
    P.bmB = c.take<uint32_t>(bm);
    P.bmT = c.take<uint32_t>(bm);
    P.bmC = c.take<uint32_t>(bm);
    P.bmTile = c.take<uint32_t>((ntiles + 31) / 32);
    P.cnt = c.take<uint32_t>((size_t)64 * 16);
    P.touched = c.take<int32_t>(nn);
    P.touched_count = c.take<int>(1);
    P.flA = c.take<int32_t>(nn);
    P.flB = c.take<int32_t>(nn);
    P.fcA = c.take<int2>(nn + (size_t)(nnz / 64) + 1);
    P.fcB = c.take<int2>(nn + (size_t)(nnz / 64) + 1);
    P.tl = c.take<int32_t>(ntiles);
    P.cvA = c.take<int32_t>(nn);
    P.cvB = c.take<int32_t>(nn);
    P.ciA = c.take<int32_t>((size_t)nitems);
    P.ciB = c.take<int32_t>((size_t)nitems);
    P.ctl = c.take<MsCtl>(1);
    P.seg = nullptr;
    P.sbit = nullptr;
    P.gcnt = nullptr;
    P.ns_cap = 64 * Q;
    P.exact_out = nullptr;
    P.timer = nullptr;
    MsItems& I = L.I;
    I.nitems = (int32_t)nitems;
    I.nsplit = (int32_t)nsplit;
    I.nnz = nnz;
    I.u = c.take<int32_t>((size_t)nitems);
    I.beg = c.take<int32_t>((size_t)nitems);
    I.end = c.take<int32_t>((size_t)nitems);
    I.split = c.take<uint8_t>((size_t)nitems);
    I.vitem = c.take<int32_t>(nn);
    I.split_list = c.take<int32_t>((size_t)nsplit);
    L.bytes = c.used;
    return L;
}

}  // namespace

int64_t noalloc_hdeg_bytes(int32_t n, int64_t nnz, int64_t nitems, int64_t nsplit, int Q) {
    return (int64_t)carve(0, n, nnz, nitems, nsplit, Q).bytes;
}

kh_status noalloc_hdeg(void* scratch_ptr, int32_t n, int64_t nnz, const int32_t* rp, const int32_t* col,
                       int64_t nitems, int64_t nsplit, int h, const uint8_t* alive_in, int32_t* deg_out,
                       int64_t* te_out, hipStream_t s) {
    // the widest bit planes that fit (sources per batch = 64 Q)
    int Q = 1;
    while (Q < 16 && 64ll * Q < (long long)n) Q <<= 1;
    while (Q > 1 && noalloc_hdeg_bytes(n, nnz, nitems, nsplit, Q) > (int64_t)kNoallocScratchBytes) Q >>= 1;
    if (noalloc_hdeg_bytes(n, nnz, nitems, nsplit, Q) > (int64_t)kNoallocScratchBytes) return KH_ENOMEM;
    const Layout L = carve(reinterpret_cast<uintptr_t>(scratch_ptr), n, nnz, nitems, nsplit, Q);
    // the array keeps the previous call's contents: clear everything this call uses
    launch_fill_i32(reinterpret_cast<int32_t*>(scratch_ptr), 0, (int64_t)(L.bytes / 4), s);
    hipLaunchKernelGGL(k_state_zero, dim3(1), dim3(256), 0, s, L.st);
    launch_alive_from(alive_in, L.alive, n, s);
    launch_alive_degree(rp, col, L.alive, L.adeg, n, s);
    launch_fill_i64(L.deg, -1, n, s);
    launch_compact_alive(L.alive, n, L.srcl, &L.st->aff_fill, s);
    hipLaunchKernelGGL(k_items_count, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, rp, n, L.cnt_items);
    launch_scan_i64(L.cnt_items, L.off_items, n, L.partials, s);
    hipLaunchKernelGGL(k_items_fill, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, rp, n, L.off_items, L.I.u,
                       L.I.beg, L.I.end, L.I.split, L.I.vitem, L.I.split_list, L.split_count);
    const int cap = 64 * Q;
    const int64_t batches = ((int64_t)n + cap - 1) / cap;
    for (int64_t b = 0; b < batches; ++b) {
        hipLaunchKernelGGL(k_batch_count, dim3(1), dim3(1), 0, s, L.st, b, cap, L.bcount);
        ms_batch(L.P, L.I, n, rp, col, L.alive, L.adeg, L.srcl + b * cap, 0, L.bcount, h, L.deg, L.st, s);
    }
    launch_core_to_i32(L.deg, deg_out, n, L.ovf, s);
    if (te_out) hipLaunchKernelGGL(k_te_out, dim3(1), dim3(1), 0, s, L.st, te_out);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? KH_OK : KH_EDEVICE;
}

}  // namespace kh
