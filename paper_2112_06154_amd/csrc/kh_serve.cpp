// Serving loop of a context (kh_serve_* in include/khcore.h): requests
// (graph, params) wait in a FIFO queue; worker threads, each with its own HIP
// stream, admit them as they and device memory become free, and run them on the
// GPU concurrently.  Queued requests with identical parameters that fit join the
// admitted one in a single packed batch (kh_core_batch), so requests that
// arrive while others run are batched continuously.  Every request gets the
// numbers kh_core gives it alone: a batch packs disjoint graphs, whose cores do
// not interact.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/khcore.h"
#include "kh_internal.hpp"

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
    uint64_t id = 0;
    kh_graph* g = nullptr;
    kh_params p{};
    int32_t* out = nullptr;
    int64_t n = 0, nnz = 0;
    uint64_t est = 0;  // device bytes reserved while it runs
    bool done = false;
    kh_status status = KH_EBUSY;
    kh_result res{};
    Clock::time_point t_submit;
};

struct Server {
    kh_context* ctx = nullptr;
    int device = 0;
    std::mutex m;
    std::condition_variable cv_work, cv_done;
    std::deque<Request*> queue;
    std::unordered_map<uint64_t, Request*> table;
    std::vector<std::thread> threads;
    uint64_t budget = 0, reserved = 0;
    int running = 0;
    bool stopping = false;
    int queue_cap = 65536;
    int64_t batch_vertices = 1 << 20;
    uint64_t next_id = 1;
};

// A server lives while the map or any call in progress holds it, so a call
// that races with kh_serve_stop never touches freed memory.  The map itself is
// never destroyed: a server still running at process exit must not be torn
// down (with its joinable threads) by a static destructor.
std::mutex g_lock;
std::unordered_map<kh_context*, std::shared_ptr<Server>>& g_servers =
    *new std::unordered_map<kh_context*, std::shared_ptr<Server>>();

std::shared_ptr<Server> find_server(kh_context* ctx) {
    std::lock_guard<std::mutex> lk(g_lock);
    auto it = g_servers.find(ctx);
    return it == g_servers.end() ? nullptr : it->second;
}

// Upper bound of the device memory one request allocates (the engines' arrays:
// bit planes of 16 words per vertex, peel state, work items; for the sampled
// path h levels of at most min(M, n) keys per vertex).
uint64_t estimate_bytes(const Request& r) {
    const double n = (double)r.n, nnz = (double)r.nnz;
    const int h = std::max(r.p.h, 1);
    double b = 1200.0 * n + 24.0 * nnz + (double)(1 << 20);
    if (r.p.epsilon > 0.0) {
        int64_t M = r.p.M_override > 0 ? r.p.M_override
                                        : kh_buffer_size(std::max<int64_t>(r.n, 1), r.p.epsilon, r.p.delta, 0);
        if (r.p.flags & KH_WANT_DENSE) {
            const int64_t Md = r.p.M_dense_override > 0
                                   ? r.p.M_dense_override
                                   : kh_buffer_size(std::max<int64_t>(r.n, 1), r.p.epsilon, r.p.delta, 1);
            M = std::max(M, Md);
        }
        const double Mm = (double)std::min<int64_t>(std::max<int64_t>(M, 1), std::max<int64_t>(r.n, 1));
        b = 400.0 * n + 24.0 * nnz + 4.0 * n * Mm * h + 64.0 * n * h + (double)(1 << 20);
    } else if (r.p.flags & KH_WANT_DENSE) {
        b *= 2.0;
    }
    return (uint64_t)b;
}

bool same_params(const kh_params& a, const kh_params& b) {
    return a.h == b.h && a.epsilon == b.epsilon && a.delta == b.delta && a.seed == b.seed &&
           a.M_override == b.M_override && a.M_dense_override == b.M_dense_override && a.flags == b.flags;
}

bool admissible(const Server* S) {
    if (S->queue.empty()) return false;
    const Request* r = S->queue.front();
    return S->running == 0 || S->reserved + r->est <= S->budget;
}

void finish(Server* S, Request* r, kh_status st, const kh_result* res) {
    r->status = st;
    if (res) r->res = *res;
    // for a served request, seconds is the latency from submission to completion
    r->res.seconds = std::chrono::duration<double>(Clock::now() - r->t_submit).count();
    r->done = true;
}

void run_batch(Server* S, std::vector<Request*>& batch, hipStream_t stream) {
    if (batch.size() == 1) {
        Request* r = batch[0];
        kh_result res;
        std::memset(&res, 0, sizeof(res));
        const kh_status st = kh_core(r->g, &r->p, r->out, &res, stream);
        std::lock_guard<std::mutex> lk(S->m);
        finish(S, r, st, &res);
        return;
    }
    std::vector<kh_graph*> gs;
    std::vector<int32_t*> outs;
    for (Request* r : batch) {
        gs.push_back(r->g);
        outs.push_back(r->out);
    }
    std::vector<kh_result> res(batch.size());
    const kh_status st =
        kh_core_batch(S->ctx, (int32_t)batch.size(), gs.data(), &batch[0]->p, outs.data(), res.data(), stream);
    if (st == KH_OK) {
        std::lock_guard<std::mutex> lk(S->m);
        for (size_t i = 0; i < batch.size(); ++i) finish(S, batch[i], KH_OK, &res[i]);
        return;
    }
    // a failed batch (e.g. out of memory) runs its requests one by one
    for (Request* r : batch) {
        kh_result one;
        std::memset(&one, 0, sizeof(one));
        const kh_status s1 = kh_core(r->g, &r->p, r->out, &one, stream);
        std::lock_guard<std::mutex> lk(S->m);
        finish(S, r, s1, &one);
    }
}

void worker(Server* S) {
    hipStream_t stream = nullptr;
    kh::RoundState* pinned = nullptr;
    bool ok = hipSetDevice(S->device) == hipSuccess && hipStreamCreate(&stream) == hipSuccess;
    void* hp = nullptr;
    ok = ok && hipHostMalloc(&hp, sizeof(kh::RoundState), hipHostMallocDefault) == hipSuccess;
    pinned = static_cast<kh::RoundState*>(hp);
    if (ok) kh::worker_thread_begin(pinned);
    for (;;) {
        std::vector<Request*> batch;
        uint64_t est = 0;
        {
            std::unique_lock<std::mutex> lk(S->m);
            S->cv_work.wait(lk, [&] { return (S->stopping && S->queue.empty()) || admissible(S); });
            if (S->queue.empty()) break;
            Request* head = S->queue.front();
            S->queue.pop_front();
            batch.push_back(head);
            est = head->est;
            int64_t vn = head->n;
            if (!(head->p.flags & KH_EARLY_STOP) && !(head->p.flags & KH_DENSE_FULL)) {
                for (auto it = S->queue.begin(); it != S->queue.end();) {
                    Request* r = *it;
                    // a packed batch finishes with its largest graph, so only
                    // graphs within a factor 4 of the head's size join it: a
                    // small request never waits for a large one
                    const bool similar = 4 * r->n >= head->n && r->n <= 4 * head->n;
                    if (similar && same_params(r->p, head->p) && vn + r->n <= S->batch_vertices &&
                        S->reserved + est + r->est <= S->budget) {
                        batch.push_back(r);
                        est += r->est;
                        vn += r->n;
                        it = S->queue.erase(it);
                    } else {
                        ++it;
                    }
                }
            }
            S->reserved += est;
            S->running += 1;
        }
        if (ok) {
            run_batch(S, batch, stream);
        } else {
            std::lock_guard<std::mutex> lk(S->m);
            for (Request* r : batch) finish(S, r, KH_EDEVICE, nullptr);
        }
        {
            std::lock_guard<std::mutex> lk(S->m);
            S->reserved -= est;
            S->running -= 1;
        }
        S->cv_done.notify_all();
        S->cv_work.notify_all();
    }
    if (ok) kh::worker_thread_end();
    if (pinned) (void)hipHostFree(pinned);
    if (stream) (void)hipStreamDestroy(stream);
}

void stop(Server* S);

kh_status start(kh_context* ctx, int32_t workers, uint64_t budget, int32_t queue_cap, int64_t batch_vertices,
                 std::shared_ptr<Server>* out) {
    if (!ctx || workers < 0 || queue_cap < 0 || batch_vertices < 0) return KH_EINVAL;
    std::lock_guard<std::mutex> lk(g_lock);
    if (g_servers.count(ctx)) return KH_EBUSY;
    const int dev = kh::context_device(ctx);
    if (hipSetDevice(dev) != hipSuccess) return KH_EDEVICE;
    auto S = std::make_shared<Server>();
    S->ctx = ctx;
    S->device = dev;
    if (budget == 0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) return KH_EDEVICE;
        budget = (uint64_t)(0.8 * (double)fr);
    }
    S->budget = budget;
    if (queue_cap > 0) S->queue_cap = queue_cap;
    if (batch_vertices > 0) S->batch_vertices = batch_vertices;
    const int w = workers > 0 ? workers : 4;
    try {
        for (int i = 0; i < w; ++i) S->threads.emplace_back(worker, S.get());
    } catch (...) {
        {
            std::lock_guard<std::mutex> l2(S->m);
            S->stopping = true;
        }
        S->cv_work.notify_all();
        for (auto& t : S->threads) t.join();
        return KH_ENOMEM;
    }
    try {
        g_servers[ctx] = S;
    } catch (...) {
        stop(S.get());
        return KH_ENOMEM;
    }
    *out = S;
    return KH_OK;
}

// The workers finish every queued request before they exit; results nobody
// collected are dropped, and a kh_serve_wait still blocked on one of them
// wakes up to KH_ENOTFOUND.
void stop(Server* S) {
    {
        std::lock_guard<std::mutex> lk(S->m);
        S->stopping = true;
    }
    S->cv_work.notify_all();
    for (auto& t : S->threads) t.join();
    S->threads.clear();
    {
        std::lock_guard<std::mutex> lk(S->m);
        for (auto& kv : S->table) delete kv.second;
        S->table.clear();
    }
    S->cv_done.notify_all();
}

}  // namespace

void kh::serve_shutdown(kh_context* ctx) {
    std::shared_ptr<Server> S;
    {
        std::lock_guard<std::mutex> lk(g_lock);
        auto it = g_servers.find(ctx);
        if (it == g_servers.end()) return;
        S = it->second;
        g_servers.erase(it);
    }
    stop(S.get());
}

extern "C" kh_status kh_serve_start(kh_context* ctx, int32_t workers, uint64_t hbm_budget_bytes, int32_t queue_cap,
                                    int64_t batch_vertices) {
    std::shared_ptr<Server> S;
    try {
        return start(ctx, workers, hbm_budget_bytes, queue_cap, batch_vertices, &S);
    } catch (...) {
        return KH_ENOMEM;
    }
}

extern "C" kh_status kh_serve_submit(kh_context* ctx, kh_graph* g, const kh_params* params, int32_t* core_out,
                                     uint64_t* ticket) {
    if (!ctx || !g || !params || !ticket) return KH_EINVAL;
    if (kh::graph_context(g) != ctx) return KH_EINVAL;
    if (params->h < 1 || !(params->delta > 0.0 && params->delta < 1.0) || std::isnan(params->epsilon))
        return KH_EINVAL;
    const int32_t n = kh_graph_n(g);
    if (n > 0 && !core_out) return KH_EINVAL;
    try {
        std::shared_ptr<Server> S = find_server(ctx);
        if (!S) {
            const kh_status st = start(ctx, 0, 0, 0, 0, &S);
            if (st == KH_EBUSY) S = find_server(ctx);  // started meanwhile by another thread
            else if (st != KH_OK) return st;
            if (!S) return KH_EDEVICE;
        }
        std::unique_ptr<Request> r(new Request());
        r->g = g;
        r->p = *params;
        r->out = core_out;
        r->n = n;
        r->nnz = kh_graph_nnz(g);
        r->est = estimate_bytes(*r);
        r->t_submit = Clock::now();
        {
            std::lock_guard<std::mutex> lk(S->m);
            if (S->stopping || (int)S->queue.size() >= S->queue_cap) return KH_EBUSY;
            const uint64_t id = S->next_id;
            S->table[id] = r.get();
            try {
                S->queue.push_back(r.get());
            } catch (...) {
                S->table.erase(id);
                throw;
            }
            S->next_id += 1;
            r->id = id;
            *ticket = id;
            r.release();  // owned by the table from here on
        }
        S->cv_work.notify_one();
        return KH_OK;
    } catch (...) {
        return KH_ENOMEM;
    }
}

namespace {
kh_status collect(Server* S, uint64_t ticket, kh_result* res, bool wait) {
    std::unique_lock<std::mutex> lk(S->m);
    auto it = S->table.find(ticket);
    if (it == S->table.end()) return KH_ENOTFOUND;
    if (!it->second->done) {
        if (!wait) return KH_EBUSY;
        // look the ticket up again after every wake-up: another caller may have
        // collected it, or a stop dropped it, while this one slept
        S->cv_done.wait(lk, [&] {
            auto jt = S->table.find(ticket);
            return jt == S->table.end() || jt->second->done;
        });
        it = S->table.find(ticket);
        if (it == S->table.end()) return KH_ENOTFOUND;
    }
    Request* r = it->second;
    const kh_status st = r->status;
    if (res) *res = r->res;
    S->table.erase(ticket);
    delete r;
    return st;
}
}  // namespace

extern "C" kh_status kh_serve_poll(kh_context* ctx, uint64_t ticket, kh_result* res) {
    if (!ctx) return KH_EINVAL;
    std::shared_ptr<Server> S = find_server(ctx);
    if (!S) return KH_ENOTFOUND;
    return collect(S.get(), ticket, res, false);
}

extern "C" kh_status kh_serve_wait(kh_context* ctx, uint64_t ticket, kh_result* res) {
    if (!ctx) return KH_EINVAL;
    std::shared_ptr<Server> S = find_server(ctx);
    if (!S) return KH_ENOTFOUND;
    return collect(S.get(), ticket, res, true);
}

extern "C" kh_status kh_serve_cancel(kh_context* ctx, uint64_t ticket) {
    if (!ctx) return KH_EINVAL;
    std::shared_ptr<Server> S = find_server(ctx);
    if (!S) return KH_ENOTFOUND;
    std::lock_guard<std::mutex> lk(S->m);
    auto it = S->table.find(ticket);
    if (it == S->table.end()) return KH_ENOTFOUND;
    Request* r = it->second;
    auto q = std::find(S->queue.begin(), S->queue.end(), r);
    if (q == S->queue.end()) return KH_EBUSY;  // running or finished: collect it instead
    S->queue.erase(q);
    S->table.erase(it);
    delete r;
    return KH_OK;
}

extern "C" kh_status kh_serve_stop(kh_context* ctx) {
    if (!ctx) return KH_EINVAL;
    kh::serve_shutdown(ctx);
    return KH_OK;
}
