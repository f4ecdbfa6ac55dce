// serve.cpp -- batched CG entry point and the continuous-batching solve server.
//
// spx_cg_batch: a fixed set of independent CSR systems, one persistent
// launch, one work-group per system (batch_cg.hip).
//
// Server: requests (host CSR + right-hand side) are queued FIFO; a worker
// thread admits them while a slot is free and the HBM pool (one allocation of
// hbm_budget_bytes made at creation, carved first-fit) can hold the matrix and
// its Krylov vectors, looking past a request that does not fit at most
// kBackfill places. Admitted requests are copied to the device on a copy
// stream while the current tick runs. A tick is one captured hipGraph (reset
// the work counter, run the persistent batched-CG kernel over the slot table)
// that advances every active slot by its iteration budget; between ticks the
// worker reads the slot table back, copies the solutions of finished slots to
// the callers' buffers, frees their memory and slots, and admits more. The
// per-slot budget keeps a tick around tick_us of work so that new requests
// join within a few milliseconds (continuous batching). Matrices and Krylov
// state stay resident in HBM between ticks.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "batch_cg.hpp"
#include "common.hpp"

using namespace spx;
using Clock = std::chrono::steady_clock;

namespace {

constexpr int kBackfill = 8;

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Device bytes of one system: CSR arrays + b, x, r, p, q.
size_t system_bytes(int64_t n, int64_t nnz)
{
    return align256((size_t)(n + 1) * 4) + align256((size_t)nnz * 4) + align256((size_t)nnz * 8) +
           5 * align256((size_t)n * 8);
}

struct Pool {
    size_t cap = 0;
    std::map<size_t, size_t> free_;  // offset -> size, coalesced
    size_t in_use = 0, peak = 0;
    void init(size_t c)
    {
        cap = c;
        free_.clear();
        free_[0] = c;
    }
    bool alloc(size_t bytes, size_t *off)
    {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t noff = it->first + bytes;
                free_.erase(it);
                if (rest) free_[noff] = rest;
                in_use += bytes;
                peak = std::max(peak, in_use);
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        in_use -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

struct Pending {
    uint64_t ticket;
    spx_request req;
    Clock::time_point t_submit;
    size_t bytes;
};

struct Active {
    uint64_t ticket = 0;
    size_t off = 0, bytes = 0;
    double *x_dev = nullptr;
    double *x_out = nullptr;
    int64_t n = 0, nnz = 0;
    Clock::time_point t_submit;
    bool cancel = false;
    bool live = false;
    bool staged = false;  // descriptor waiting in spx_server::staged
};

struct Result {
    bool done = false;
    spx_status status = SPX_PENDING;
    spx_solve_info info{};
};

spx_status slot_status_to_spx(int32_t s)
{
    switch (s) {
    case kSlotConverged: return SPX_OK;
    case kSlotBreakdown: return SPX_ERR_BREAKDOWN;
    case kSlotNonfinite: return SPX_ERR_NONFINITE;
    case kSlotMaxit: return SPX_ERR_NOT_CONVERGED;
    default: return SPX_ERR_NOT_CONVERGED;
    }
}

}  // namespace

struct spx_server {
    spx_server_config cfg{};
    int device = 0;
    hipStream_t s_compute = nullptr, s_copy = nullptr;
    char *pool_base = nullptr;
    Pool pool;
    BatchSlot *slots_dev = nullptr;
    BatchSlot *slots_host = nullptr;  // pinned mirror
    std::vector<BatchSlot> staged;    // descriptors of slots admitted since the last table upload
    int32_t *counter = nullptr;
    hipGraphExec_t tick = nullptr;
    std::vector<Active> active;
    std::deque<Pending> queue;
    std::unordered_map<uint64_t, Result> results;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::thread worker;
    std::atomic<bool> stop{false};
    uint64_t next_ticket = 1;
    spx_server_stats stats{};
    std::string fatal;
};

namespace {

// Budget of CG iterations for one tick: about tick_us of one work-group's
// streaming time (iteration bytes / an assumed 25 GB/s per work-group).
int32_t budget_for(const spx_server &S, int64_t n, int64_t nnz, int32_t remaining)
{
    if (S.cfg.iters_per_tick > 0) return std::min(S.cfg.iters_per_tick, std::max(remaining, 1));
    const double bytes = (double)nnz * 12.0 + (double)n * 76.0;
    const double us_per_iter = bytes / 25e3;  // 25 GB/s = 25e3 bytes per microsecond
    const double tick_us = S.cfg.tick_us > 0 ? S.cfg.tick_us : 2000.0;
    int64_t b = (int64_t)(tick_us / std::max(us_per_iter, 0.01));
    b = std::max<int64_t>(1, std::min<int64_t>(b, remaining));
    return (int32_t)b;
}

void finish_ticket(spx_server &S, uint64_t ticket, spx_status st, const spx_solve_info &info)
{
    std::lock_guard<std::mutex> lk(S.mu);
    Result &r = S.results[ticket];
    r.done = true;
    r.status = st;
    r.info = info;
    S.stats.completed += 1;
    S.cv_done.notify_all();
}

// Admit queued requests into free slots and pool memory (copies on s_copy).
// Returns the number admitted.
int admit(spx_server &S)
{
    std::vector<std::pair<int, Pending>> take;
    {
        std::lock_guard<std::mutex> lk(S.mu);
        int scanned = 0;
        for (auto it = S.queue.begin(); it != S.queue.end() && scanned < kBackfill;) {
            int free_slot = -1;
            for (int i = 0; i < (int)S.active.size(); ++i)
                if (!S.active[i].live) {
                    bool claimed = false;
                    for (auto &t : take) claimed |= (t.first == i);
                    if (!claimed) {
                        free_slot = i;
                        break;
                    }
                }
            if (free_slot < 0) break;
            size_t off = 0;
            if (S.pool.alloc(it->bytes, &off)) {
                Pending p = *it;
                p.bytes = it->bytes;
                S.active[free_slot].off = off;  // reserve
                S.active[free_slot].bytes = it->bytes;
                take.emplace_back(free_slot, p);
                it = S.queue.erase(it);
            } else {
                ++it;
                ++scanned;
            }
        }
        S.stats.queued = (int64_t)S.queue.size();
    }
    for (auto &tp : take) {
        const int si = tp.first;
        const Pending &p = tp.second;
        Active &a = S.active[si];
        const int64_t n = p.req.n, nnz = p.req.nnz;
        char *base = S.pool_base + a.off;
        size_t o = 0;
        auto carve = [&](size_t b) {
            char *q = base + o;
            o += align256(b);
            return q;
        };
        int32_t *rp = reinterpret_cast<int32_t *>(carve((size_t)(n + 1) * 4));
        int32_t *ci = reinterpret_cast<int32_t *>(carve((size_t)nnz * 4));
        double *va = reinterpret_cast<double *>(carve((size_t)nnz * 8));
        double *b = reinterpret_cast<double *>(carve((size_t)n * 8));
        double *x = reinterpret_cast<double *>(carve((size_t)n * 8));
        double *r = reinterpret_cast<double *>(carve((size_t)n * 8));
        double *pp = reinterpret_cast<double *>(carve((size_t)n * 8));
        double *q = reinterpret_cast<double *>(carve((size_t)n * 8));
        (void)hipMemcpyAsync(rp, p.req.rowptr, (size_t)(n + 1) * 4, hipMemcpyHostToDevice, S.s_copy);
        if (nnz > 0) {
            (void)hipMemcpyAsync(ci, p.req.colidx, (size_t)nnz * 4, hipMemcpyHostToDevice, S.s_copy);
            (void)hipMemcpyAsync(va, p.req.vals, (size_t)nnz * 8, hipMemcpyHostToDevice, S.s_copy);
        }
        (void)hipMemcpyAsync(b, p.req.b, (size_t)n * 8, hipMemcpyHostToDevice, S.s_copy);
        (void)hipMemsetAsync(x, 0, (size_t)n * 8, S.s_copy);
        BatchSlot &d = S.staged[si];
        std::memset(&d, 0, sizeof(d));
        d.rowptr = rp;
        d.col = ci;
        d.val = va;
        d.b = b;
        d.x = x;
        d.r = r;
        d.p = pp;
        d.q = q;
        d.n = (int32_t)n;
        d.sub = batch_sub_for(n, nnz);
        d.status = kSlotRunning;
        d.started = 0;
        d.tol2 = p.req.tol * p.req.tol;
        d.maxit = p.req.maxit > 0 ? p.req.maxit : 100000;
        d.budget = 0;  // set before the tick
        a.ticket = p.ticket;
        a.x_dev = x;
        a.x_out = p.req.x_out;
        a.n = n;
        a.nnz = nnz;
        a.t_submit = p.t_submit;
        a.cancel = false;
        a.live = true;
        a.staged = true;
    }
    return (int)take.size();
}

// Move the descriptors of newly admitted slots into the table mirror (only
// when no read-back of the table is in flight).
void apply_staged(spx_server &S)
{
    for (int i = 0; i < (int)S.active.size(); ++i)
        if (S.active[i].staged) {
            S.slots_host[i] = S.staged[i];
            S.active[i].staged = false;
        }
}

void retire(spx_server &S)
{
    for (int i = 0; i < (int)S.active.size(); ++i) {
        Active &a = S.active[i];
        if (!a.live) continue;
        BatchSlot &d = S.slots_host[i];
        if (d.status == kSlotRunning && !a.cancel) continue;
        spx_solve_info info{};
        spx_status st = a.cancel ? SPX_CANCELLED : slot_status_to_spx(d.status);
        if (!a.cancel && a.x_out) (void)hipMemcpy(a.x_out, a.x_dev, (size_t)a.n * 8, hipMemcpyDeviceToHost);
        info.status = st;
        info.iters = d.iters;
        info.spmv_count = d.spmv;
        info.relres_recursive = d.bb > 0 ? sqrt(d.rr / d.bb) : 0.0;
        info.relres_true = d.relres_true;
        info.device_ms = std::chrono::duration<double, std::milli>(Clock::now() - a.t_submit).count();
        {
            std::lock_guard<std::mutex> lk(S.mu);
            S.pool.release(a.off, a.bytes);
        }
        d.status = kSlotEmpty;
        a.live = false;
        finish_ticket(S, a.ticket, st, info);
    }
}

void worker_main(spx_server *Sp)
{
    spx_server &S = *Sp;
    (void)hipSetDevice(S.device);
    while (!S.stop.load()) {
        int admitted = admit(S);
        bool any = false;
        for (auto &a : S.active) any |= a.live;
        if (!any) {
            std::unique_lock<std::mutex> lk(S.mu);
            if (S.queue.empty() && !S.stop.load()) S.cv_work.wait_for(lk, std::chrono::milliseconds(1));
            continue;
        }
        (void)admitted;
        if (hipStreamSynchronize(S.s_copy) != hipSuccess) {
            S.fatal = "admission copy failed";
            break;
        }
        apply_staged(S);
        for (int i = 0; i < (int)S.active.size(); ++i) {
            if (!S.active[i].live) continue;
            BatchSlot &d = S.slots_host[i];
            if (S.active[i].cancel) {
                d.budget = 0;
                continue;
            }
            d.budget = budget_for(S, S.active[i].n, S.active[i].nnz, std::max(1, d.maxit - d.iters));
        }
        const size_t tb = sizeof(BatchSlot) * S.active.size();
        hipError_t e = hipMemcpyAsync(S.slots_dev, S.slots_host, tb, hipMemcpyHostToDevice, S.s_compute);
        if (e == hipSuccess) e = hipGraphLaunch(S.tick, S.s_compute);
        if (e == hipSuccess) e = hipMemcpyAsync(S.slots_host, S.slots_dev, tb, hipMemcpyDeviceToHost, S.s_compute);
        // admit more while the tick runs (descriptors stay staged until the
        // read-back of the table has landed)
        admit(S);
        if (e == hipSuccess) e = hipStreamSynchronize(S.s_compute);
        if (e != hipSuccess) {
            S.fatal = hipGetErrorString(e);
            break;
        }
        if (hipStreamSynchronize(S.s_copy) != hipSuccess) {
            S.fatal = "admission copy failed";
            break;
        }
        apply_staged(S);
        {
            std::lock_guard<std::mutex> lk(S.mu);
            S.stats.ticks += 1;
        }
        retire(S);
    }
    // fail whatever is left
    std::lock_guard<std::mutex> lk(S.mu);
    for (auto &p : S.queue) {
        Result &r = S.results[p.ticket];
        r.done = true;
        r.status = SPX_CANCELLED;
    }
    S.queue.clear();
    S.cv_done.notify_all();
}

}  // namespace

extern "C" spx_status spx_server_create(const spx_server_config *cfg, spx_server **out)
{
    clear_error();
    SPX_REQUIRE(cfg && out, SPX_ERR_ARG, "spx_server_create: null argument");
    SPX_REQUIRE(cfg->max_slots >= 1 && cfg->max_slots <= 65536, SPX_ERR_ARG, "spx_server_create: bad max_slots");
    SPX_REQUIRE(cfg->hbm_budget_bytes >= 4096, SPX_ERR_ARG, "spx_server_create: budget too small");
    auto *S = new spx_server();
    S->cfg = *cfg;
    S->device = cfg->device;
    auto fail = [&](const char *what, hipError_t e) {
        set_error("spx_server_create: %s: %s", what, hipGetErrorString(e));
        if (S->tick) (void)hipGraphExecDestroy(S->tick);
        if (S->pool_base) (void)hipFree(S->pool_base);
        if (S->slots_dev) (void)hipFree(S->slots_dev);
        if (S->counter) (void)hipFree(S->counter);
        if (S->slots_host) (void)hipHostFree(S->slots_host);
        if (S->s_compute) (void)hipStreamDestroy(S->s_compute);
        if (S->s_copy) (void)hipStreamDestroy(S->s_copy);
        delete S;
        return e == hipErrorOutOfMemory ? SPX_ERR_NOMEM : SPX_ERR_HIP;
    };
    hipError_t e;
    if ((e = hipSetDevice(S->device)) != hipSuccess) return fail("hipSetDevice", e);
    if ((e = hipStreamCreateWithFlags(&S->s_compute, hipStreamNonBlocking)) != hipSuccess) return fail("stream", e);
    if ((e = hipStreamCreateWithFlags(&S->s_copy, hipStreamNonBlocking)) != hipSuccess) return fail("stream", e);
    if ((e = hipMalloc(reinterpret_cast<void **>(&S->pool_base), cfg->hbm_budget_bytes)) != hipSuccess)
        return fail("pool", e);
    S->pool.init(cfg->hbm_budget_bytes);
    const size_t tb = sizeof(BatchSlot) * (size_t)cfg->max_slots;
    if ((e = hipMalloc(reinterpret_cast<void **>(&S->slots_dev), tb)) != hipSuccess) return fail("slots", e);
    if ((e = hipHostMalloc(reinterpret_cast<void **>(&S->slots_host), tb, hipHostMallocDefault)) != hipSuccess)
        return fail("pinned slots", e);
    std::memset(S->slots_host, 0, tb);
    for (int i = 0; i < cfg->max_slots; ++i) S->slots_host[i].status = kSlotEmpty;
    if ((e = hipMalloc(reinterpret_cast<void **>(&S->counter), sizeof(int32_t))) != hipSuccess)
        return fail("counter", e);
    // the tick: reset the counter, then the persistent batched kernel
    hipGraph_t g = nullptr;
    if ((e = hipStreamBeginCapture(S->s_compute, hipStreamCaptureModeThreadLocal)) != hipSuccess)
        return fail("capture", e);
    spx_status s1 = batch_reset_launch(S->counter, S->s_compute);
    spx_status s2 = batch_cg_launch(S->slots_dev, cfg->max_slots, S->counter, batch_resident_groups(), S->s_compute);
    e = hipStreamEndCapture(S->s_compute, &g);
    if (s1 != SPX_OK || s2 != SPX_OK || e != hipSuccess) return fail("capture", e != hipSuccess ? e : hipErrorUnknown);
    e = hipGraphInstantiate(&S->tick, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail("instantiate", e);
    S->active.resize(cfg->max_slots);
    S->staged.resize(cfg->max_slots);
    S->stats.pool_bytes_total = cfg->hbm_budget_bytes;
    S->worker = std::thread(worker_main, S);
    *out = S;
    return SPX_OK;
}

extern "C" spx_status spx_serve_submit(spx_server *S, const spx_request *req, uint64_t *ticket)
{
    clear_error();
    SPX_REQUIRE(S && req && ticket, SPX_ERR_ARG, "spx_serve_submit: null argument");
    SPX_REQUIRE(req->n >= 1 && req->nnz >= 0 && req->rowptr && req->b && (req->nnz == 0 || (req->colidx && req->vals)),
                SPX_ERR_ARG, "spx_serve_submit: bad request");
    SPX_REQUIRE(req->solver == SPX_SOLVER_CG, SPX_ERR_ARG, "spx_serve_submit: only CG is served");
    SPX_REQUIRE(req->tol >= 0.0, SPX_ERR_ARG, "spx_serve_submit: negative tolerance");
    const size_t bytes = system_bytes(req->n, req->nnz);
    std::lock_guard<std::mutex> lk(S->mu);
    SPX_REQUIRE(S->fatal.empty(), SPX_ERR_HIP, "spx_serve_submit: server failed: %s", S->fatal.c_str());
    if (bytes > S->cfg.hbm_budget_bytes) {
        S->stats.rejected += 1;
        set_error("spx_serve_submit: request needs %zu bytes, budget is %zu", bytes, S->cfg.hbm_budget_bytes);
        return SPX_ERR_BUDGET;
    }
    const uint64_t t = S->next_ticket++;
    S->queue.push_back(Pending{t, *req, Clock::now(), bytes});
    S->results[t] = Result{};
    S->stats.submitted += 1;
    S->stats.queued = (int64_t)S->queue.size();
    S->cv_work.notify_one();
    *ticket = t;
    return SPX_OK;
}

extern "C" spx_status spx_serve_poll(spx_server *S, uint64_t ticket, spx_solve_info *info)
{
    SPX_REQUIRE(S, SPX_ERR_ARG, "spx_serve_poll: null server");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->results.find(ticket);
    SPX_REQUIRE(it != S->results.end(), SPX_ERR_ARG, "spx_serve_poll: unknown ticket %llu",
                (unsigned long long)ticket);
    if (!it->second.done) return SPX_PENDING;
    if (info) *info = it->second.info;
    return it->second.status;
}

extern "C" spx_status spx_serve_wait(spx_server *S, uint64_t ticket, double timeout_s, spx_solve_info *info)
{
    SPX_REQUIRE(S, SPX_ERR_ARG, "spx_serve_wait: null server");
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->results.find(ticket);
    SPX_REQUIRE(it != S->results.end(), SPX_ERR_ARG, "spx_serve_wait: unknown ticket %llu",
                (unsigned long long)ticket);
    const auto until = Clock::now() + std::chrono::duration<double>(timeout_s < 0 ? 1e9 : timeout_s);
    while (!S->results[ticket].done) {
        if (S->cv_done.wait_until(lk, until) == std::cv_status::timeout && !S->results[ticket].done)
            return SPX_PENDING;
    }
    const Result &r = S->results[ticket];
    if (info) *info = r.info;
    return r.status;
}

extern "C" spx_status spx_serve_cancel(spx_server *S, uint64_t ticket)
{
    SPX_REQUIRE(S, SPX_ERR_ARG, "spx_serve_cancel: null server");
    std::lock_guard<std::mutex> lk(S->mu);
    for (auto it = S->queue.begin(); it != S->queue.end(); ++it) {
        if (it->ticket == ticket) {
            S->queue.erase(it);
            Result &r = S->results[ticket];
            r.done = true;
            r.status = SPX_CANCELLED;
            r.info.status = SPX_CANCELLED;
            S->stats.completed += 1;
            S->cv_done.notify_all();
            return SPX_OK;
        }
    }
    for (auto &a : S->active)
        if (a.live && a.ticket == ticket) {
            a.cancel = true;  // retired at the end of the next tick
            return SPX_OK;
        }
    auto it = S->results.find(ticket);
    SPX_REQUIRE(it != S->results.end(), SPX_ERR_ARG, "spx_serve_cancel: unknown ticket");
    return SPX_OK;  // already finished
}

extern "C" spx_status spx_server_get_stats(spx_server *S, spx_server_stats *out)
{
    SPX_REQUIRE(S && out, SPX_ERR_ARG, "spx_server_get_stats: null argument");
    std::lock_guard<std::mutex> lk(S->mu);
    spx_server_stats st = S->stats;
    st.queued = (int64_t)S->queue.size();
    st.active = 0;
    for (auto &a : S->active) st.active += a.live ? 1 : 0;
    st.pool_bytes_in_use = S->pool.in_use;
    st.pool_bytes_peak = S->pool.peak;
    *out = st;
    return SPX_OK;
}

extern "C" spx_status spx_server_destroy(spx_server *S)
{
    if (!S) return SPX_OK;
    S->stop.store(true);
    S->cv_work.notify_all();
    if (S->worker.joinable()) S->worker.join();
    (void)hipStreamSynchronize(S->s_compute);
    (void)hipStreamSynchronize(S->s_copy);
    if (S->tick) (void)hipGraphExecDestroy(S->tick);
    (void)hipFree(S->pool_base);
    (void)hipFree(S->slots_dev);
    (void)hipFree(S->counter);
    (void)hipHostFree(S->slots_host);
    (void)hipStreamDestroy(S->s_compute);
    (void)hipStreamDestroy(S->s_copy);
    delete S;
    return SPX_OK;
}

// ------------------------------------------------------------------ spx_cg_batch
static size_t batch_ws_bytes(const spx_batch_system *sys, int32_t count)
{
    size_t b = align256(sizeof(BatchSlot) * (size_t)count) + 256;
    for (int32_t i = 0; i < count; ++i) b += 3 * align256((size_t)sys[i].n * 8);
    return b;
}

extern "C" spx_status spx_cg_batch_workspace(const spx_batch_system *sys, int32_t count, size_t *bytes)
{
    clear_error();
    SPX_REQUIRE(sys && bytes && count >= 0, SPX_ERR_ARG, "spx_cg_batch_workspace: bad argument");
    *bytes = batch_ws_bytes(sys, count);
    return SPX_OK;
}

extern "C" spx_status spx_cg_batch(spx_batch_system *sys, int32_t count, void *ws, size_t ws_bytes,
                                   hipStream_t stream)
{
    clear_error();
    SPX_REQUIRE(sys && count >= 0, SPX_ERR_ARG, "spx_cg_batch: bad argument");
    if (count == 0) return SPX_OK;
    SPX_REQUIRE(ws && ws_bytes >= batch_ws_bytes(sys, count), SPX_ERR_ARG, "spx_cg_batch: workspace too small");
    for (int32_t i = 0; i < count; ++i)
        SPX_REQUIRE(sys[i].n >= 1 && sys[i].rowptr && sys[i].b && sys[i].x && (sys[i].nnz == 0 || (sys[i].colidx && sys[i].vals)),
                    SPX_ERR_ARG, "spx_cg_batch: bad system %d", i);
    char *base = static_cast<char *>(ws);
    BatchSlot *slots_dev = reinterpret_cast<BatchSlot *>(base);
    size_t off = align256(sizeof(BatchSlot) * (size_t)count);
    int32_t *counter = reinterpret_cast<int32_t *>(base + off);
    off += 256;
    std::vector<BatchSlot> host((size_t)count);
    for (int32_t i = 0; i < count; ++i) {
        BatchSlot &d = host[i];
        std::memset(&d, 0, sizeof(d));
        const size_t vb = align256((size_t)sys[i].n * 8);
        d.rowptr = sys[i].rowptr;
        d.col = sys[i].colidx;
        d.val = sys[i].vals;
        d.b = sys[i].b;
        d.x = sys[i].x;
        d.r = reinterpret_cast<double *>(base + off);
        d.p = reinterpret_cast<double *>(base + off + vb);
        d.q = reinterpret_cast<double *>(base + off + 2 * vb);
        off += 3 * vb;
        d.n = sys[i].n;
        d.sub = batch_sub_for(sys[i].n, sys[i].nnz);
        d.status = kSlotRunning;
        d.tol2 = sys[i].tol * sys[i].tol;
        d.maxit = sys[i].maxit > 0 ? sys[i].maxit : 100000;
        d.budget = d.maxit;
        SPX_HIP(hipMemsetAsync(sys[i].x, 0, (size_t)sys[i].n * 8, stream));
    }
    SPX_HIP(hipMemcpyAsync(slots_dev, host.data(), sizeof(BatchSlot) * (size_t)count, hipMemcpyHostToDevice, stream));
    SPX_CHECK(batch_reset_launch(counter, stream));
    SPX_CHECK(batch_cg_launch(slots_dev, count, counter, batch_resident_groups(), stream));
    SPX_HIP(hipMemcpyAsync(host.data(), slots_dev, sizeof(BatchSlot) * (size_t)count, hipMemcpyDeviceToHost, stream));
    SPX_HIP(hipStreamSynchronize(stream));
    spx_status first = SPX_OK;
    for (int32_t i = 0; i < count; ++i) {
        const BatchSlot &d = host[i];
        sys[i].status = d.status == kSlotConverged ? SPX_OK : slot_status_to_spx(d.status);
        sys[i].iters = d.iters;
        sys[i].spmv_count = d.spmv;
        sys[i].relres_true = d.relres_true;
        if (first == SPX_OK && sys[i].status != SPX_OK) first = (spx_status)sys[i].status;
    }
    if (first != SPX_OK) set_error("spx_cg_batch: at least one system did not converge");
    return first;
}
