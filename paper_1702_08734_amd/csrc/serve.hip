// Serving loop for a resident IVFADC index: requests of any size (host
// query rows) are queued, packed in arrival order into batches bounded by a
// row limit and a device-memory budget for the search workspace, and each
// batch runs on one of several HIP streams (pinned staging, upload, search,
// download), so that one batch's transfers and kernels overlap the next
// batch's.  Each stream has its own search workspace, so a batch makes no
// allocator calls (per-search allocations through the stream-ordered
// allocator cost the launching thread more than the GPU time of a small
// batch).  A completion thread copies each request's rows back to the
// caller's buffers and records its latency (submission to completion).
//
// Every query's result is independent of the batch it shares: the search
// kernels treat queries independently (per-query coarse selection, per
// (query, list) scans, per-query merges), so a request gives the same D, I as
// a search of that request alone.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "common.hpp"

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
    uint64_t ticket = 0;
    const float* xq = nullptr;
    int64_t nq = 0;
    float* D = nullptr;
    int64_t* I = nullptr;
    Clock::time_point t_submit, t_done;
    bool done = false;
    mk_status status = MK_OK;
    std::string error;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t ready = nullptr;
    float* h_q = nullptr;    // pinned staging of the batch's queries
    float* h_D = nullptr;    // pinned results
    int64_t* h_I = nullptr;
    float* d_q = nullptr;
    float* d_D = nullptr;
    int64_t* d_I = nullptr;
    unsigned char* d_ws = nullptr;  // the search scratch of this slot's batches
    size_t ws_bytes = 0;
    std::vector<std::shared_ptr<Request>> reqs;
    int64_t rows = 0;
    mk_status status = MK_OK;
    std::string error;
    bool busy = false;
};

}  // namespace

struct mk_server {
    mk_ivfpq* ix = nullptr;
    mk_server_config cfg{};
    int32_t d = 0;
    std::vector<Slot> slots;
    std::mutex mu;
    std::condition_variable cv_work, cv_done, cv_slot;
    std::deque<std::shared_ptr<Request>> queue;
    std::unordered_map<uint64_t, std::shared_ptr<Request>> live;
    std::deque<int> inflight;  // slot indices in launch order
    uint64_t next_ticket = 1;
    bool stop = false;
    int64_t batches = 0, rows = 0;
    std::thread worker, completer;
    int device = 0;
};

namespace mk {
namespace {

// Launch one batch on its slot (worker thread, lock not held).
void launch_batch(mk_server* sv, Slot& sl) {
    const int32_t d = sv->d;
    const int32_t k = sv->cfg.k;
    int64_t off = 0;
    for (auto& r : sl.reqs) {
        std::memcpy(sl.h_q + off * d, r->xq, sizeof(float) * (size_t)r->nq * d);
        off += r->nq;
    }
    sl.rows = off;
    sl.status = MK_OK;
    hipError_t e = hipMemcpyAsync(sl.d_q, sl.h_q, sizeof(float) * (size_t)off * d,
                                  hipMemcpyHostToDevice, sl.stream);
    if (e != hipSuccess) sl.status = MK_ERR_DEVICE;
    if (sl.status == MK_OK) {
        const mk_server_config& c = sv->cfg;
        // the search's scratch is carved from the slot's workspace, which the
        // slot's previous batch no longer uses (it has completed before the
        // slot was handed out again)
        mk::Arena arena;
        arena.base = sl.d_ws;
        arena.size = sl.ws_bytes;
        mk::ArenaScope scope(&arena);
        if (c.net)
            sl.status = mk_ivfpq_search_learned(sv->ix, c.net, c.delta, sl.d_q, off, k, c.cap, c.R,
                                                c.xb, c.nb, sl.d_D, sl.d_I, nullptr, sl.stream);
        else if (c.R > 0)
            sl.status = mk_ivfpq_search_rerank(sv->ix, sl.d_q, off, k, c.nprobe, c.R, c.xb, c.nb,
                                               sl.d_D, sl.d_I, sl.stream);
        else
            sl.status = mk_ivfpq_search(sv->ix, sl.d_q, off, k, c.nprobe, sl.d_D, sl.d_I,
                                        sl.stream);
    }
    if (sl.status == MK_OK) {
        e = hipMemcpyAsync(sl.h_D, sl.d_D, sizeof(float) * (size_t)off * k,
                           hipMemcpyDeviceToHost, sl.stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(sl.h_I, sl.d_I, sizeof(int64_t) * (size_t)off * k,
                               hipMemcpyDeviceToHost, sl.stream);
        if (e != hipSuccess) sl.status = MK_ERR_DEVICE;
    }
    if (hipEventRecord(sl.ready, sl.stream) != hipSuccess && sl.status == MK_OK)
        sl.status = MK_ERR_DEVICE;
    sl.error = sl.status == MK_OK ? std::string() : std::string(mk_last_error());
}

void worker_main(mk_server* sv) {
    (void)hipSetDevice(sv->device);
    const int64_t budget = sv->cfg.workspace_budget;
    for (;;) {
        std::unique_lock<std::mutex> lk(sv->mu);
        sv->cv_work.wait(lk, [&] { return sv->stop || !sv->queue.empty(); });
        if (sv->queue.empty()) break;  // stopping and drained
        // a free slot (batches complete in launch order)
        int si = -1;
        sv->cv_slot.wait(lk, [&] {
            for (size_t i = 0; i < sv->slots.size(); ++i)
                if (!sv->slots[i].busy) { si = (int)i; return true; }
            return false;
        });
        Slot& sl = sv->slots[si];
        sl.reqs.clear();
        int64_t rows = 0;
        while (!sv->queue.empty()) {
            const auto& r = sv->queue.front();
            const int64_t nr = rows + r->nq;
            if (nr > sv->cfg.max_batch) break;
            if (rows > 0 && budget > 0) {
                size_t ws = 0;
                mk_ivfpq_search_workspace_bytes(sv->ix, nr, sv->cfg.k,
                                                sv->cfg.net ? sv->cfg.cap : sv->cfg.nprobe,
                                                sv->cfg.R, &ws);
                if ((int64_t)ws > budget) break;
            }
            rows = nr;
            sl.reqs.push_back(r);
            sv->queue.pop_front();
        }
        sl.busy = true;
        lk.unlock();
        launch_batch(sv, sl);
        lk.lock();
        sv->inflight.push_back(si);
        sv->batches += 1;
        sv->rows += rows;
        lk.unlock();
        sv->cv_done.notify_all();
    }
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->inflight.push_back(-1);  // tells the completion thread to finish
    sv->cv_done.notify_all();
}

void completer_main(mk_server* sv) {
    (void)hipSetDevice(sv->device);
    for (;;) {
        int si;
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            sv->cv_done.wait(lk, [&] { return !sv->inflight.empty(); });
            si = sv->inflight.front();
            sv->inflight.pop_front();
        }
        if (si < 0) break;
        Slot& sl = sv->slots[si];
        mk_status st = sl.status;
        if (hipEventSynchronize(sl.ready) != hipSuccess && st == MK_OK) st = MK_ERR_DEVICE;
        const int32_t k = sv->cfg.k;
        int64_t off = 0;
        const auto now = Clock::now();
        for (auto& r : sl.reqs) {
            if (st == MK_OK) {
                std::memcpy(r->D, sl.h_D + off * k, sizeof(float) * (size_t)r->nq * k);
                std::memcpy(r->I, sl.h_I + off * k, sizeof(int64_t) * (size_t)r->nq * k);
            }
            off += r->nq;
        }
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            for (auto& r : sl.reqs) {
                r->status = st;
                r->error = sl.error;
                r->t_done = now;
                r->done = true;
            }
            sl.reqs.clear();
            sl.busy = false;
        }
        sv->cv_done.notify_all();
        sv->cv_slot.notify_all();
    }
}

void release(mk_server* sv) {
    for (Slot& sl : sv->slots) {
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
        if (sl.ready) (void)hipEventDestroy(sl.ready);
        for (void* p : {(void*)sl.h_q, (void*)sl.h_D, (void*)sl.h_I})
            if (p) (void)hipHostFree(p);
        for (void* p : {(void*)sl.d_q, (void*)sl.d_D, (void*)sl.d_I, (void*)sl.d_ws})
            if (p) (void)hipFree(p);
    }
    sv->slots.clear();
}

}  // namespace
}  // namespace mk

// ---------------------------------------------------------------- C ABI
extern "C" mk_status mk_server_create(mk_ivfpq* ix, const mk_server_config* cfg,
                                      mk_server** out) {
    MK_REQUIRE(out, MK_ERR_INVALID_ARG, "null output pointer");
    *out = nullptr;
    MK_REQUIRE(ix && cfg, MK_ERR_INVALID_ARG, "null index or configuration");
    MK_REQUIRE(cfg->k >= 1 && cfg->max_batch >= 1 && cfg->nstreams >= 1 && cfg->nstreams <= 8,
               MK_ERR_INVALID_ARG, "need k >= 1, max_batch >= 1, 1 <= nstreams <= 8");
    MK_REQUIRE(cfg->net || cfg->nprobe >= 1, MK_ERR_INVALID_ARG, "need nprobe >= 1");
    MK_REQUIRE(!cfg->net || cfg->cap >= 1, MK_ERR_INVALID_ARG,
               "a learned probe count needs cap >= 1");
    MK_REQUIRE(cfg->R <= 0 || (cfg->xb && cfg->R >= cfg->k), MK_ERR_INVALID_ARG,
               "a re-rank needs xb and R >= k");
    const int32_t d = mk_ivfpq_dim(ix);
    auto sv = std::make_unique<mk_server>();
    sv->ix = ix;
    sv->cfg = *cfg;
    sv->d = d;
    MK_HIP(hipGetDevice(&sv->device));
    sv->slots.resize(cfg->nstreams);
    const size_t B = (size_t)cfg->max_batch;
    // per-slot search workspace: the estimate for a full batch (at most the
    // per-batch budget, when one is set) plus a margin for what it leaves
    // out; scratch that does not fit is allocated per search as usual
    size_t ws = 0;
    {
        mk_status st = mk_ivfpq_search_workspace_bytes(ix, cfg->max_batch, cfg->k,
                                                       cfg->net ? cfg->cap : cfg->nprobe, cfg->R,
                                                       &ws);
        if (st != MK_OK) return st;
    }
    if (cfg->workspace_budget > 0 && ws > (size_t)cfg->workspace_budget)
        ws = (size_t)cfg->workspace_budget;
    ws += ws / 4 + ((size_t)64 << 20);
    hipError_t e = hipSuccess;
    for (Slot& sl : sv->slots) {
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.ready, hipEventDisableTiming);
        if (e == hipSuccess) e = hipHostMalloc((void**)&sl.h_q, sizeof(float) * B * d, 0);
        if (e == hipSuccess) e = hipHostMalloc((void**)&sl.h_D, sizeof(float) * B * cfg->k, 0);
        if (e == hipSuccess) e = hipHostMalloc((void**)&sl.h_I, sizeof(int64_t) * B * cfg->k, 0);
        if (e == hipSuccess) e = hipMalloc(&sl.d_q, sizeof(float) * B * d);
        if (e == hipSuccess) e = hipMalloc(&sl.d_D, sizeof(float) * B * cfg->k);
        if (e == hipSuccess) e = hipMalloc(&sl.d_I, sizeof(int64_t) * B * cfg->k);
        if (e == hipSuccess) {
            // without room for the workspace the slot allocates per search
            const hipError_t ew = hipMalloc(&sl.d_ws, ws);
            if (ew == hipSuccess) {
                sl.ws_bytes = ws;
            } else if (ew == hipErrorOutOfMemory) {
                (void)hipGetLastError();
                sl.d_ws = nullptr;
            } else {
                e = ew;
            }
        }
    }
    if (e != hipSuccess) {
        mk::release(sv.get());
        mk::set_error(std::string("mk_server_create: ") + hipGetErrorString(e));
        return e == hipErrorOutOfMemory ? MK_ERR_OOM : MK_ERR_DEVICE;
    }
    mk_server* p = sv.release();
    p->worker = std::thread(mk::worker_main, p);
    p->completer = std::thread(mk::completer_main, p);
    *out = p;
    return MK_OK;
}

extern "C" mk_status mk_server_submit(mk_server* sv, const float* xq, int64_t nq, float* D,
                                      int64_t* I, uint64_t* ticket) {
    MK_REQUIRE(sv && ticket, MK_ERR_INVALID_ARG, "null server or ticket");
    MK_REQUIRE(nq >= 1 && nq <= sv->cfg.max_batch, MK_ERR_INVALID_ARG,
               "need 1 <= nq <= max_batch");
    MK_REQUIRE(xq && D && I, MK_ERR_INVALID_ARG, "null pointer");
    auto r = std::make_shared<Request>();
    r->xq = xq;
    r->nq = nq;
    r->D = D;
    r->I = I;
    r->t_submit = Clock::now();
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        MK_REQUIRE(!sv->stop, MK_ERR_STATE, "server is stopping");
        r->ticket = sv->next_ticket++;
        sv->live[r->ticket] = r;
        sv->queue.push_back(r);
    }
    sv->cv_work.notify_one();
    *ticket = r->ticket;
    return MK_OK;
}

extern "C" mk_status mk_server_wait(mk_server* sv, uint64_t ticket, double* latency_s) {
    MK_REQUIRE(sv, MK_ERR_INVALID_ARG, "null server");
    std::shared_ptr<Request> r;
    {
        std::unique_lock<std::mutex> lk(sv->mu);
        auto it = sv->live.find(ticket);
        MK_REQUIRE(it != sv->live.end(), MK_ERR_INVALID_ARG, "unknown or already collected ticket");
        r = it->second;
        sv->cv_done.wait(lk, [&] { return r->done; });
        // submissions may have rehashed the map while the lock was released
        // inside wait(): erase by key, not through the old iterator
        sv->live.erase(ticket);
    }
    if (latency_s)
        *latency_s = std::chrono::duration<double>(r->t_done - r->t_submit).count();
    if (r->status != MK_OK) mk::set_error("mk_server_wait: the request's batch failed: " + r->error);
    return r->status;
}

extern "C" mk_status mk_server_stats(mk_server* sv, int64_t* batches, int64_t* rows) {
    MK_REQUIRE(sv, MK_ERR_INVALID_ARG, "null server");
    std::lock_guard<std::mutex> lk(sv->mu);
    if (batches) *batches = sv->batches;
    if (rows) *rows = sv->rows;
    return MK_OK;
}

extern "C" void mk_server_destroy(mk_server* sv) {
    if (!sv) return;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
    }
    sv->cv_work.notify_all();
    if (sv->worker.joinable()) sv->worker.join();
    if (sv->completer.joinable()) sv->completer.join();
    mk::release(sv);
    delete sv;
}
