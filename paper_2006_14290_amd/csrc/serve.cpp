// serve.cpp -- batched CG entry point and the continuous-batching solve server.
//
// spx_cg_batch: a fixed set of independent CSR systems: persistent launches
// with one work-group per system (batch_cg.hip; systems of at most
// kBatchSmallRows rows on their own kernel) and the grid-wide phases of the
// wide path for large systems (batch_wide.hip).
//
// Server: requests (host CSR + right-hand side) are queued FIFO; an admission
// thread admits them while a slot is free and the HBM pool (one allocation of
// hbm_budget_bytes made at creation, carved first-fit) can hold the matrix and
// its Krylov vectors, looking past a request that does not fit at most
// kBackfill places, and copies them to the device on a copy stream while the
// worker thread runs ticks (copies from pageable host memory, which the
// runtime stages through its own buffers, hold up only the admission
// thread); the worker takes a system into its tables once its copies have
// landed. A tick runs two captured hipGraphs on
// two streams at once: the narrow graph (reset the work counters, run the
// persistent one-group-per-system kernels over the slot table: the
// small-system kernel, then the general one) advances every system below
// the wide threshold by its iteration budget; the wide graph (kWideIters iterations
// of the two wide phases, the state alternating between two buffers)
// advances every large system, launched as many times as fits the tick. Between ticks the worker reads the state back,
// copies the solutions of finished systems to the callers' buffers, frees
// their memory and slots, and admits more: new requests join within a few
// milliseconds (continuous batching). Matrices and Krylov state stay resident
// in HBM between ticks.
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
#include "spmv.hpp"
#include "spmv_csr.hpp"

using namespace spx;
using Clock = std::chrono::steady_clock;

namespace {

constexpr int kBackfill = 8;

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

constexpr int kWideIters = 8;                    // wide iterations per graph launch
constexpr int kWideGrids[3] = {256, 1024, 4096};  // physical grids of the wide graphs
// the state alternates between two buffers; an even count ends in the first
static_assert(kWideIters % 2 == 0, "wide iterations per graph must be even");
// Every CG system above the small-system kernel's range takes the wide path
// by default: on the serving stream this cut the p99 latency at 0.9x load by
// about 40 % against a 16,384-row threshold at the same capacity (systems of
// a few thousand rows iterate faster on many work-groups than on one).
constexpr int32_t kWideDefaultRows = kBatchSmallRows + 1;

// Extra device bytes of a wide system: the vector s = A p (CG), the two
// halves of two rows of vector-phase partials, two rows of product partials
// and the product's tile partition.
size_t wide_extra_bytes(int64_t n, int64_t nnz)
{
    return align256((size_t)n * 8) + align256((size_t)wide_nvb(n) * 4 * 8) +
           align256((size_t)csr_tiles(nnz) * 2 * 8) + align256((size_t)csr_partition_bytes(nnz));
}

// Device bytes of one system: CSR arrays + b, x, r, p, q (+ the partials and
// partition of the wide path; BiCGSTAB adds r_hat and t).
size_t system_bytes(int64_t n, int64_t nnz, bool wide, bool bicgstab)
{
    return align256((size_t)(n + 1) * 4) + align256((size_t)nnz * 4) + align256((size_t)nnz * 8) +
           (bicgstab ? 7 : 5) * align256((size_t)n * 8) + (wide ? wide_extra_bytes(n, nnz) : 0);
}

// Systems from wide_min_rows rows on (CG and BiCGSTAB alike) take the wide
// path.
bool is_wide(int32_t wide_min_rows, int64_t n)
{
    const int64_t t = wide_min_rows == 0 ? kWideDefaultRows : wide_min_rows;
    return wide_min_rows >= 0 && n >= t;
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
    bool wide;
};

// Bytes one iteration of a request moves: the CSR product plus about nine
// vector passes (CG); a BiCGSTAB step has two products and twice the passes.
int64_t iter_work(const spx_request &r)
{
    const int64_t w = r.nnz * 12 + (int64_t)r.n * (4 + 9 * 8);
    return r.solver == SPX_SOLVER_BICGSTAB ? 2 * w : w;
}

struct Active {
    uint64_t ticket = 0;
    size_t off = 0, bytes = 0;
    int64_t work = 0;  // iter_work of the request (counted in spx_server::inflight)
    double *x_dev = nullptr;
    double *x_out = nullptr;
    int64_t n = 0, nnz = 0;
    Clock::time_point t_submit;
    // Set by spx_serve_cancel under the server mutex, read by the worker
    // without it (hence atomic); the worker reads it again under the mutex
    // when it retires the system, so a cancel that returned before the
    // retirement always ends in SPX_CANCELLED.
    std::atomic<bool> cancel{false};
    // written under the mutex (reserve, retire), read by the worker freely
    std::atomic<bool> live{false};
    // reserved by the admission thread, not yet in the worker's tables; while
    // it is set the worker reads no other field of the slot
    std::atomic<bool> staged{false};
    // set by the admission thread (release) once the slot's copies have
    // landed and its descriptor in spx_server::staged / wstaged is written
    std::atomic<bool> ready{false};
    bool wide = false;
    bool in_map = false;  // listed in the wide map uploaded for the current tick
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
    hipStream_t s_compute = nullptr, s_copy = nullptr, s_wide = nullptr;
    char *pool_base = nullptr;
    Pool pool;
    BatchSlot *slots_dev = nullptr;
    BatchSlot *slots_host = nullptr;  // pinned mirror
    std::vector<BatchSlot> staged;    // descriptors of slots admitted since the last table upload
    int32_t *counter = nullptr;
    hipGraphExec_t tick = nullptr;       // narrow tick, full persistent grid
    hipGraphExec_t tick_half = nullptr;  // narrow tick, half grid (wide work running beside it)
    // wide path: descriptor table, device state, map (header, list, virtual blocks)
    WideSlot *wslots_dev = nullptr, *wslots_host = nullptr;
    WideState *wstate_dev = nullptr, *wstate_host = nullptr, *winit_host = nullptr;
    WideState *wstate2_dev = nullptr;  // odd iterations' state (the host sees only wstate_dev)
    WideMap *wmap_dev = nullptr, *wmap_host = nullptr;
    int32_t *vb_dev = nullptr, *vb_host = nullptr;  // [2 * vb_cap]: slot, then local index
    int64_t vb_cap = 0;
    int32_t *ta_dev = nullptr, *ta_host = nullptr;  // [2 * ta_cap]: product tiles, same layout
    int64_t ta_cap = 0;
    std::vector<WideSlot> wstaged;
    hipGraphExec_t wide_tick[3] = {nullptr, nullptr, nullptr};
    hipEvent_t ev_w0 = nullptr, ev_w1 = nullptr;
    bool wide_dirty = false;
    int wide_launches = 1;  // wide graph launches per tick (adapted to tick_us)
    std::vector<Active> active;
    std::deque<Pending> queue;
    std::unordered_map<uint64_t, Result> results;
    std::mutex mu;
    // cv_work: a new request or freed memory (admission thread); cv_ready: a
    // slot became ready (worker); cv_done: a result (waiters)
    std::condition_variable cv_work, cv_ready, cv_done;
    std::thread worker, admitter;
    std::atomic<bool> stop{false};
    std::atomic<bool> admit_failed{false};
    uint64_t next_ticket = 1;
    spx_server_stats stats{};
    std::string fatal;
    int64_t inflight = 0;  // summed iter_work of resident systems (under mu)
    int64_t inflight_cap = 0;  // cfg.inflight_bytes (<= 0: no bound)
};

namespace {

// Budget of iterations for one tick: about tick_us of one work-group's
// streaming time (iteration bytes / an assumed 25 GB/s per work-group; a
// BiCGSTAB step has two products and about twice the vector traffic).
int32_t budget_for(const spx_server &S, int64_t n, int64_t nnz, int32_t remaining, bool bicgstab)
{
    if (S.cfg.iters_per_tick > 0) return std::min(S.cfg.iters_per_tick, std::max(remaining, 1));
    const double bytes = ((double)nnz * 12.0 + (double)n * 76.0) * (bicgstab ? 2.0 : 1.0);
    const double us_per_iter = bytes / 25e3;  // 25 GB/s = 25e3 bytes per microsecond
    const double tick_us = S.cfg.tick_us > 0 ? S.cfg.tick_us : 2000.0;
    int64_t b = (int64_t)(tick_us / std::max(us_per_iter, 0.01));
    b = std::max<int64_t>(1, std::min<int64_t>(b, remaining));
    return (int32_t)b;
}

// Record a finished request (the caller holds S.mu).
void finish_locked(spx_server &S, uint64_t ticket, spx_status st, const spx_solve_info &info)
{
    Result &r = S.results[ticket];
    if (r.done) return;
    r.done = true;
    r.status = st;
    r.info = info;
    S.stats.completed += 1;
    S.cv_done.notify_all();
}

// Admit queued requests into free slots and pool memory (copies on s_copy;
// the caller synchronizes s_copy before it marks the slots ready). Returns
// the admitted slots.
std::vector<int> admit(spx_server &S)
{
    std::vector<std::pair<int, Pending>> take;
    {
        std::lock_guard<std::mutex> lk(S.mu);
        int scanned = 0;
        for (auto it = S.queue.begin(); it != S.queue.end() && scanned < kBackfill;) {
            // work bound: strict FIFO (no request passes one held back by it)
            const int64_t w = iter_work(it->req);
            if (S.inflight_cap > 0 && S.inflight > 0 && S.inflight + w > S.inflight_cap) break;
            int free_slot = -1;
            for (int i = 0; i < (int)S.active.size(); ++i)
                if (!S.active[i].live) {
                    free_slot = i;
                    break;
                }
            if (free_slot < 0) break;
            size_t off = 0;
            if (S.pool.alloc(it->bytes, &off)) {
                Pending p = *it;
                p.bytes = it->bytes;
                // reserve the slot where spx_serve_cancel can see the ticket
                Active &a = S.active[free_slot];
                a.off = off;
                a.bytes = it->bytes;
                a.work = w;
                S.inflight += w;
                a.ticket = p.ticket;
                a.cancel.store(false);
                // staged before live: a worker that sees the slot live
                // also sees it staged, and leaves it alone
                a.ready.store(false);
                a.staged.store(true);
                a.live.store(true);
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
        const bool bicg = p.req.solver == SPX_SOLVER_BICGSTAB;
        double *rh = bicg ? reinterpret_cast<double *>(carve((size_t)n * 8)) : nullptr;
        double *tv = bicg ? reinterpret_cast<double *>(carve((size_t)n * 8)) : nullptr;
        double *sv = p.wide ? reinterpret_cast<double *>(carve((size_t)n * 8)) : nullptr;
        double *part = p.wide ? reinterpret_cast<double *>(carve((size_t)wide_nvb(n) * 4 * 8)) : nullptr;
        double *part_a = p.wide ? reinterpret_cast<double *>(carve((size_t)csr_tiles(nnz) * 2 * 8)) : nullptr;
        int32_t *cpart = p.wide ? reinterpret_cast<int32_t *>(carve((size_t)csr_partition_bytes(nnz))) : nullptr;
        (void)hipMemcpyAsync(rp, p.req.rowptr, (size_t)(n + 1) * 4, hipMemcpyHostToDevice, S.s_copy);
        if (nnz > 0) {
            (void)hipMemcpyAsync(ci, p.req.colidx, (size_t)nnz * 4, hipMemcpyHostToDevice, S.s_copy);
            (void)hipMemcpyAsync(va, p.req.vals, (size_t)nnz * 8, hipMemcpyHostToDevice, S.s_copy);
        }
        (void)hipMemcpyAsync(b, p.req.b, (size_t)n * 8, hipMemcpyHostToDevice, S.s_copy);
        (void)hipMemsetAsync(x, 0, (size_t)n * 8, S.s_copy);
        a.wide = p.wide;
        a.in_map = false;
        if (p.wide) {
            WideSlot &w = S.wstaged[si];
            std::memset(&w, 0, sizeof(w));
            w.rowptr = rp;
            w.col = ci;
            w.val = va;
            w.b = b;
            w.x = x;
            w.r = r;
            w.p = pp;
            w.w = q;
            w.s = sv;
            w.rh = rh;
            w.t = tv;
            w.solver = bicg ? kSlotBicgstab : kSlotCg;
            w.part = part;
            w.part_a = part_a;
            w.csr_part = cpart;
            w.nnz = nnz;
            w.ntiles = (int32_t)csr_tiles(nnz);
            w.n = (int32_t)n;
            w.nvb = wide_nvb(n);
            {
                spx_matrix d{};
                d.fmt = SPX_CSR;
                d.nrows = (int32_t)n;
                d.ncols = (int32_t)n;
                d.nnz = nnz;
                d.rowptr = rp;
                (void)csr_partition_launch(d, cpart, S.s_copy);  // after the row pointer copy (same stream)
            }
            w.maxit = p.req.maxit > 0 ? p.req.maxit : 100000;
            w.tol2 = p.req.tol * p.req.tol;
            WideState &ws = S.winit_host[si];
            std::memset(&ws, 0, sizeof(ws));
            ws.mode = kWideInit;
            (void)hipMemcpyAsync(S.wstate_dev + si, &ws, sizeof(WideState), hipMemcpyHostToDevice, S.s_copy);
            a.x_dev = x;
            a.x_out = p.req.x_out;
            a.n = n;
            a.nnz = nnz;
            a.t_submit = p.t_submit;
            continue;
        }
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
        d.rh = rh;
        d.t = tv;
        d.solver = bicg ? kSlotBicgstab : kSlotCg;
        d.first = 1;
        d.n = (int32_t)n;
        d.sub = narrow_sub_for(n, nnz);
        d.status = kSlotRunning;
        d.started = 0;
        d.tol2 = p.req.tol * p.req.tol;
        d.maxit = p.req.maxit > 0 ? p.req.maxit : 100000;
        d.budget = 0;  // set before the tick
        a.x_dev = x;
        a.x_out = p.req.x_out;
        a.n = n;
        a.nnz = nnz;
        a.t_submit = p.t_submit;
    }
    std::vector<int> slots;
    for (auto &tp : take) slots.push_back(tp.first);
    return slots;
}

// Move the descriptors of newly admitted slots into the table mirror (only
// when no read-back of the table is in flight).
void apply_staged(spx_server &S)
{
    for (int i = 0; i < (int)S.active.size(); ++i)
        if (S.active[i].staged.load() && S.active[i].ready.load(std::memory_order_acquire)) {
            if (S.active[i].wide) {
                S.wslots_host[i] = S.wstaged[i];
                S.wstate_host[i] = S.winit_host[i];
                S.wide_dirty = true;
            } else {
                S.slots_host[i] = S.staged[i];
            }
            S.active[i].ready.store(false);
            S.active[i].staged.store(false);
        }
}

// List every live, uncancelled wide system and map the virtual blocks onto
// them; upload the tables on the wide stream (called between ticks only).
bool rebuild_wide_map(spx_server &S)
{
    int32_t nl = 0;
    int64_t tot = 0, tta = 0;
    for (int i = 0; i < (int)S.active.size(); ++i) {
        Active &a = S.active[i];
        if (!a.live || a.staged) continue;  // a staged slot's fields belong to the admission thread
        a.in_map = false;
        if (!a.wide || a.cancel.load()) continue;
        const int32_t nvb = S.wslots_host[i].nvb, nt = S.wslots_host[i].ntiles;
        if (tot + nvb > S.vb_cap || tta + nt > S.ta_cap) return false;
        ++nl;
        for (int32_t k = 0; k < nvb; ++k) {
            S.vb_host[tot + k] = i;
            S.vb_host[S.vb_cap + tot + k] = k;
        }
        for (int32_t k = 0; k < nt; ++k) {
            S.ta_host[tta + k] = i;
            S.ta_host[S.ta_cap + tta + k] = k;
        }
        tot += nvb;
        tta += nt;
        a.in_map = true;
    }
    S.wmap_host->total_vb = (int32_t)tot;
    S.wmap_host->nlisted = nl;
    S.wmap_host->total_ta = (int32_t)tta;
    const size_t tb = sizeof(WideSlot) * S.active.size();
    hipError_t e = hipMemcpyAsync(S.wslots_dev, S.wslots_host, tb, hipMemcpyHostToDevice, S.s_wide);
    if (e == hipSuccess) e = hipMemcpyAsync(S.wmap_dev, S.wmap_host, sizeof(WideMap), hipMemcpyHostToDevice, S.s_wide);
    if (e == hipSuccess && tot > 0) {
        e = hipMemcpyAsync(S.vb_dev, S.vb_host, sizeof(int32_t) * tot, hipMemcpyHostToDevice, S.s_wide);
        if (e == hipSuccess)
            e = hipMemcpyAsync(S.vb_dev + S.vb_cap, S.vb_host + S.vb_cap, sizeof(int32_t) * tot,
                               hipMemcpyHostToDevice, S.s_wide);
    }
    if (e == hipSuccess && tta > 0) {
        e = hipMemcpyAsync(S.ta_dev, S.ta_host, sizeof(int32_t) * tta, hipMemcpyHostToDevice, S.s_wide);
        if (e == hipSuccess)
            e = hipMemcpyAsync(S.ta_dev + S.ta_cap, S.ta_host + S.ta_cap, sizeof(int32_t) * tta,
                               hipMemcpyHostToDevice, S.s_wide);
    }
    S.wide_dirty = false;
    return e == hipSuccess;
}

// Retire finished and cancelled systems: copy their solutions out (all at
// once on the compute stream, idle between ticks: one wait for every copy),
// then free their memory and slots and record the results. Returns false if
// a copy failed.
bool retire(spx_server &S)
{
    struct Finished {
        int slot;
        int32_t solver_status;
        spx_solve_info info;
    };
    std::vector<Finished> fin;
    hipError_t e = hipSuccess;
    for (int i = 0; i < (int)S.active.size(); ++i) {
        Active &a = S.active[i];
        if (!a.live || a.staged) continue;
        spx_solve_info info{};
        int32_t solver_status;
        const bool cancel = a.cancel.load();
        if (a.wide) {
            // the host copy of the state is current only for systems that were
            // listed in this tick's launches
            const WideState &w = S.wstate_host[i];
            const bool done = a.in_map && w.mode == kWideDone;
            if (!done && !cancel) continue;
            solver_status = w.status;
            info.iters = w.iters;
            info.spmv_count = w.spmv;
            info.relres_recursive = w.bb > 0 ? sqrt(w.rr / w.bb) : 0.0;
            info.relres_true = w.relres_true;
            S.wide_dirty = true;
        } else {
            BatchSlot &d = S.slots_host[i];
            if (d.status == kSlotRunning && !cancel) continue;
            solver_status = d.status;
            info.iters = d.iters;
            info.spmv_count = d.spmv;
            info.relres_recursive = d.bb > 0 ? sqrt(d.rr / d.bb) : 0.0;
            info.relres_true = d.relres_true;
            d.status = kSlotEmpty;
        }
        if (!cancel && a.x_out && e == hipSuccess)
            e = hipMemcpyAsync(a.x_out, a.x_dev, (size_t)a.n * 8, hipMemcpyDeviceToHost, S.s_compute);
        fin.push_back(Finished{i, solver_status, info});
    }
    if (fin.empty()) return true;
    if (e == hipSuccess) e = hipStreamSynchronize(S.s_compute);
    if (e != hipSuccess) return false;
    const auto now = Clock::now();
    for (Finished &f : fin) {
        Active &a = S.active[f.slot];
        f.info.device_ms = std::chrono::duration<double, std::milli>(now - a.t_submit).count();
        a.in_map = false;
        std::lock_guard<std::mutex> lk(S.mu);
        // a cancel that arrived after the first read still wins: it returned
        // while the system was live
        const spx_status st = a.cancel.load() ? SPX_CANCELLED : slot_status_to_spx(f.solver_status);
        f.info.status = st;
        S.pool.release(a.off, a.bytes);
        S.inflight -= a.work;
        a.live = false;
        finish_locked(S, a.ticket, st, f.info);
    }
    return true;
}

// Stop serving: every queued and every resident request ends with `st`
// (SPX_ERR_HIP after a failure, SPX_CANCELLED when the server is destroyed),
// so no spx_serve_wait is left waiting.
void fail_all(spx_server &S, spx_status st)
{
    std::lock_guard<std::mutex> lk(S.mu);
    spx_solve_info info{};
    info.status = st;
    for (auto &p : S.queue) finish_locked(S, p.ticket, st, info);
    S.queue.clear();
    for (auto &a : S.active)
        if (a.live) {
            a.live = false;
            S.pool.release(a.off, a.bytes);
            S.inflight -= a.work;
            finish_locked(S, a.ticket, st, info);
        }
    S.cv_done.notify_all();
}

void set_fatal(spx_server &S, const char *what)
{
    std::lock_guard<std::mutex> lk(S.mu);
    S.fatal = what;
}

// Admission thread: reserves slots and pool memory for queued requests and
// copies them in (s_copy); a slot becomes ready once its copies have landed.
void admitter_main(spx_server *Sp)
{
    spx_server &S = *Sp;
    (void)hipSetDevice(S.device);
    while (!S.stop.load()) {
        const std::vector<int> slots = admit(S);
        if (slots.empty()) {
            std::unique_lock<std::mutex> lk(S.mu);
            if (!S.stop.load()) S.cv_work.wait_for(lk, std::chrono::milliseconds(1));
            continue;
        }
        if (hipStreamSynchronize(S.s_copy) != hipSuccess) {
            set_fatal(S, "admission copy failed");
            S.admit_failed.store(true);
            S.cv_ready.notify_all();
            break;
        }
        for (int si : slots) S.active[si].ready.store(true, std::memory_order_release);
        S.cv_ready.notify_one();
    }
}

void worker_main(spx_server *Sp)
{
    spx_server &S = *Sp;
    (void)hipSetDevice(S.device);
    while (!S.stop.load() && !S.admit_failed.load()) {
        apply_staged(S);
        bool any = false;
        for (auto &a : S.active) any |= a.live.load() && !a.staged.load();
        if (!any) {
            std::unique_lock<std::mutex> lk(S.mu);
            if (!S.stop.load()) S.cv_ready.wait_for(lk, std::chrono::milliseconds(1));
            continue;
        }
        if (S.wide_dirty && !rebuild_wide_map(S)) {
            set_fatal(S, "wide map upload failed");
            break;
        }
        const int32_t nwide = S.wmap_host->nlisted;
        bool narrow = false;
        for (int i = 0; i < (int)S.active.size(); ++i) {
            if (!S.active[i].live || S.active[i].staged || S.active[i].wide) continue;
            BatchSlot &d = S.slots_host[i];
            if (S.active[i].cancel.load()) {
                d.budget = 0;
                continue;
            }
            d.budget = budget_for(S, S.active[i].n, S.active[i].nnz, std::max(1, d.maxit - d.iters),
                                  d.solver == kSlotBicgstab);
            narrow = true;
        }
        hipError_t e = hipSuccess;
        if (narrow) {
            const size_t tb = sizeof(BatchSlot) * S.active.size();
            e = hipMemcpyAsync(S.slots_dev, S.slots_host, tb, hipMemcpyHostToDevice, S.s_compute);
            if (e == hipSuccess) e = hipGraphLaunch(nwide > 0 ? S.tick_half : S.tick, S.s_compute);
            if (e == hipSuccess) e = hipMemcpyAsync(S.slots_host, S.slots_dev, tb, hipMemcpyDeviceToHost, S.s_compute);
        }
        if (nwide > 0 && e == hipSuccess) {
            const int32_t tot = std::max(S.wmap_host->total_vb, S.wmap_host->total_ta);
            const int gi = tot <= kWideGrids[0] ? 0 : (tot <= kWideGrids[1] ? 1 : 2);
            e = hipEventRecord(S.ev_w0, S.s_wide);
            for (int l = 0; l < S.wide_launches && e == hipSuccess; ++l) e = hipGraphLaunch(S.wide_tick[gi], S.s_wide);
            if (e == hipSuccess) e = hipEventRecord(S.ev_w1, S.s_wide);
            if (e == hipSuccess)
                e = hipMemcpyAsync(S.wstate_host, S.wstate_dev, sizeof(WideState) * S.active.size(),
                                   hipMemcpyDeviceToHost, S.s_wide);
        }
        if (e == hipSuccess) e = hipStreamSynchronize(S.s_compute);
        if (e == hipSuccess) e = hipStreamSynchronize(S.s_wide);
        if (e == hipSuccess && S.cfg.debug_fail_tick > 0 && S.stats.ticks + 1 >= S.cfg.debug_fail_tick)
            e = hipErrorLaunchFailure;  // testing hook: the host pretends this tick failed
        if (e != hipSuccess) {
            set_fatal(S, hipGetErrorString(e));
            break;
        }
        if (nwide > 0) {
            // size the next tick's wide work to about tick_us
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, S.ev_w0, S.ev_w1) == hipSuccess && ms > 0.f) {
                const double tick_ms = (S.cfg.tick_us > 0 ? S.cfg.tick_us : 2000) * 1e-3;
                const double per = ms / S.wide_launches;
                S.wide_launches = (int)std::max(1.0, std::min(64.0, tick_ms / per));
            }
        }
        {
            std::lock_guard<std::mutex> lk(S.mu);
            S.stats.ticks += 1;
        }
        // before apply_staged (next iteration): newly admitted systems have
        // no state to read yet; freed memory lets the admission thread go on
        if (!retire(S)) {
            set_fatal(S, "result copy failed");
            break;
        }
        S.cv_work.notify_one();
    }
    // the admission thread stops first, so no copy from a caller's arrays is
    // in flight once the requests end
    S.stop.store(true);
    S.cv_work.notify_all();
    if (S.admitter.joinable()) S.admitter.join();
    // whatever is left ends now: failed after an error, cancelled on a stop
    bool failed;
    {
        std::lock_guard<std::mutex> lk(S.mu);
        failed = !S.fatal.empty();
    }
    if (failed) {
        // let in-flight copies and kernels finish before the pool is reused
        (void)hipStreamSynchronize(S.s_compute);
        (void)hipStreamSynchronize(S.s_wide);
        (void)hipStreamSynchronize(S.s_copy);
    }
    fail_all(S, failed ? SPX_ERR_HIP : SPX_CANCELLED);
}

}  // namespace

namespace {

void server_free(spx_server *S)
{
    if (S->tick) (void)hipGraphExecDestroy(S->tick);
    if (S->tick_half) (void)hipGraphExecDestroy(S->tick_half);
    for (auto &g : S->wide_tick)
        if (g) (void)hipGraphExecDestroy(g);
    if (S->ev_w0) (void)hipEventDestroy(S->ev_w0);
    if (S->ev_w1) (void)hipEventDestroy(S->ev_w1);
    for (void *p : {(void *)S->pool_base, (void *)S->slots_dev, (void *)S->counter, (void *)S->wslots_dev,
                    (void *)S->wstate_dev, (void *)S->wstate2_dev, (void *)S->wmap_dev, (void *)S->vb_dev,
                    (void *)S->ta_dev})
        if (p) (void)hipFree(p);
    for (void *p : {(void *)S->slots_host, (void *)S->wslots_host, (void *)S->wstate_host, (void *)S->winit_host,
                    (void *)S->wmap_host, (void *)S->vb_host, (void *)S->ta_host})
        if (p) (void)hipHostFree(p);
    if (S->s_compute) (void)hipStreamDestroy(S->s_compute);
    if (S->s_copy) (void)hipStreamDestroy(S->s_copy);
    if (S->s_wide) (void)hipStreamDestroy(S->s_wide);
    delete S;
}

// Capture `launch(stream)` into an executable graph.
template <typename F>
hipError_t capture(hipStream_t stream, F launch, hipGraphExec_t *out)
{
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    const spx_status st = launch(stream);
    e = hipStreamEndCapture(stream, &g);
    if (e == hipSuccess && st != SPX_OK) e = hipErrorUnknown;
    if (e == hipSuccess) e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    return e;
}

template <typename T>
hipError_t dev_alloc(T **p, size_t count)
{
    return hipMalloc(reinterpret_cast<void **>(p), sizeof(T) * count);
}

template <typename T>
hipError_t host_alloc(T **p, size_t count)
{
    hipError_t e = hipHostMalloc(reinterpret_cast<void **>(p), sizeof(T) * count, hipHostMallocDefault);
    if (e == hipSuccess) std::memset(*p, 0, sizeof(T) * count);
    return e;
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
    S->inflight_cap = cfg->inflight_bytes;
    const size_t ms = (size_t)cfg->max_slots;
    // every wide row costs at least 44 pool bytes (row pointer + five vectors)
    S->vb_cap = (int64_t)(cfg->hbm_budget_bytes / (44 * (size_t)kWideRows)) + (int64_t)ms + 1;
    // every stored nonzero costs 12 pool bytes and a system has at most
    // nnz / kCsrTile + 1 tiles
    S->ta_cap = (int64_t)(cfg->hbm_budget_bytes / (12 * (size_t)kCsrTile)) + (int64_t)ms + 1;
    hipError_t e;
    auto fail = [&](const char *what) {
        set_error("spx_server_create: %s: %s", what, hipGetErrorString(e));
        server_free(S);
        return e == hipErrorOutOfMemory ? SPX_ERR_NOMEM : SPX_ERR_HIP;
    };
    if ((e = hipSetDevice(S->device)) != hipSuccess) return fail("hipSetDevice");
    if ((e = hipStreamCreateWithFlags(&S->s_compute, hipStreamNonBlocking)) != hipSuccess) return fail("stream");
    if ((e = hipStreamCreateWithFlags(&S->s_copy, hipStreamNonBlocking)) != hipSuccess) return fail("stream");
    if ((e = hipStreamCreateWithFlags(&S->s_wide, hipStreamNonBlocking)) != hipSuccess) return fail("stream");
    if ((e = hipEventCreate(&S->ev_w0)) != hipSuccess || (e = hipEventCreate(&S->ev_w1)) != hipSuccess)
        return fail("event");
    if ((e = dev_alloc(&S->pool_base, cfg->hbm_budget_bytes)) != hipSuccess) return fail("pool");
    S->pool.init(cfg->hbm_budget_bytes);
    if ((e = dev_alloc(&S->slots_dev, ms)) != hipSuccess || (e = host_alloc(&S->slots_host, ms)) != hipSuccess ||
        (e = dev_alloc(&S->counter, 2)) != hipSuccess || (e = dev_alloc(&S->wslots_dev, ms)) != hipSuccess ||
        (e = host_alloc(&S->wslots_host, ms)) != hipSuccess || (e = dev_alloc(&S->wstate_dev, ms)) != hipSuccess ||
        (e = dev_alloc(&S->wstate2_dev, ms)) != hipSuccess ||
        (e = host_alloc(&S->wstate_host, ms)) != hipSuccess || (e = host_alloc(&S->winit_host, ms)) != hipSuccess ||
        (e = dev_alloc(&S->wmap_dev, 1)) != hipSuccess || (e = host_alloc(&S->wmap_host, 1)) != hipSuccess ||
        (e = dev_alloc(&S->vb_dev, 2 * (size_t)S->vb_cap)) != hipSuccess ||
        (e = host_alloc(&S->vb_host, 2 * (size_t)S->vb_cap)) != hipSuccess ||
        (e = dev_alloc(&S->ta_dev, 2 * (size_t)S->ta_cap)) != hipSuccess ||
        (e = host_alloc(&S->ta_host, 2 * (size_t)S->ta_cap)) != hipSuccess)
        return fail("tables");
    for (size_t i = 0; i < ms; ++i) {
        S->slots_host[i].status = kSlotEmpty;
        S->wstate_host[i].mode = kWideDone;
    }
    if ((e = hipMemcpy(S->wmap_dev, S->wmap_host, sizeof(WideMap), hipMemcpyHostToDevice)) != hipSuccess)
        return fail("map");
    // narrow ticks: reset the counter, then the persistent kernel (full grid,
    // and half the grid for ticks that run wide work beside it)
    const int64_t groups = batch_resident_groups(), sgroups = batch_small_resident_groups();
    for (int half = 0; half < 2; ++half) {
        const int64_t grid = half ? std::max<int64_t>(1, groups / 2) : groups;
        const int64_t sgrid = half ? std::max<int64_t>(1, sgroups / 2) : sgroups;
        e = capture(
            S->s_compute,
            [&](hipStream_t st) {
                spx_status s1 = batch_reset_launch(S->counter, st);
                if (s1 == SPX_OK) s1 = batch_small_launch(S->slots_dev, cfg->max_slots, S->counter, sgrid, st);
                return s1 != SPX_OK ? s1 : batch_cg_launch(S->slots_dev, cfg->max_slots, S->counter, grid, st);
            },
            half ? &S->tick_half : &S->tick);
        if (e != hipSuccess) return fail("narrow tick capture");
    }
    // wide ticks: kWideIters iterations over the map, one graph per grid size
    for (int gi = 0; gi < 3; ++gi) {
        e = capture(
            S->s_wide,
            [&](hipStream_t st) {
                for (int it = 0; it < kWideIters; ++it) {
                    WideState *cur = (it & 1) ? S->wstate2_dev : S->wstate_dev;
                    WideState *next = (it & 1) ? S->wstate_dev : S->wstate2_dev;
                    spx_status s1 = wide_iteration_launch(S->wslots_dev, cur, next, S->wmap_dev, S->vb_dev,
                                                          S->vb_dev + S->vb_cap, S->ta_dev, S->ta_dev + S->ta_cap,
                                                          kWideGrids[gi], st);
                    if (s1 != SPX_OK) return s1;
                }
                return SPX_OK;
            },
            &S->wide_tick[gi]);
        if (e != hipSuccess) return fail("wide tick capture");
    }
    S->active = std::vector<Active>(ms);
    S->staged.resize(ms);
    S->wstaged.resize(ms);
    S->stats.pool_bytes_total = cfg->hbm_budget_bytes;
    S->admitter = std::thread(admitter_main, S);
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
    SPX_REQUIRE(req->solver == SPX_SOLVER_CG || req->solver == SPX_SOLVER_BICGSTAB, SPX_ERR_ARG,
                "spx_serve_submit: solver %d is not served (CG and BiCGSTAB are)", req->solver);
    SPX_REQUIRE(req->tol >= 0.0, SPX_ERR_ARG, "spx_serve_submit: negative tolerance");
    SPX_REQUIRE(req->nnz <= INT32_MAX, SPX_ERR_ARG, "spx_serve_submit: nnz exceeds int32");
    // nothing malformed may reach the kernels that every resident system shares
    SPX_CHECK(validate_csr_host(req->n, req->n, req->nnz, req->rowptr, req->colidx));
    const bool wide = is_wide(S->cfg.wide_min_rows, req->n);
    const size_t bytes = system_bytes(req->n, req->nnz, wide, req->solver == SPX_SOLVER_BICGSTAB);
    std::lock_guard<std::mutex> lk(S->mu);
    SPX_REQUIRE(S->fatal.empty(), SPX_ERR_HIP, "spx_serve_submit: server failed: %s", S->fatal.c_str());
    if (bytes > S->cfg.hbm_budget_bytes) {
        S->stats.rejected += 1;
        set_error("spx_serve_submit: request needs %zu bytes, budget is %zu", bytes, S->cfg.hbm_budget_bytes);
        return SPX_ERR_BUDGET;
    }
    const uint64_t t = S->next_ticket++;
    S->queue.push_back(Pending{t, *req, Clock::now(), bytes, wide});
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
            spx_solve_info info{};
            info.status = SPX_CANCELLED;
            finish_locked(*S, ticket, SPX_CANCELLED, info);
            return SPX_OK;
        }
    }
    // a request leaves the queue and takes its slot in one locked step, so a
    // ticket that is neither queued nor resident has finished
    for (auto &a : S->active)
        if (a.live && a.ticket == ticket) {
            a.cancel.store(true);  // retired at the end of the current tick
            return SPX_OK;
        }
    auto it = S->results.find(ticket);
    SPX_REQUIRE(it != S->results.end(), SPX_ERR_ARG, "spx_serve_cancel: unknown ticket");
    SPX_REQUIRE(it->second.done, SPX_ERR_ARG, "spx_serve_cancel: ticket %llu is neither queued, resident nor done",
                (unsigned long long)ticket);
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
    S->cv_ready.notify_all();
    if (S->worker.joinable()) S->worker.join();  // joins the admission thread first
    (void)hipStreamSynchronize(S->s_compute);
    (void)hipStreamSynchronize(S->s_wide);
    (void)hipStreamSynchronize(S->s_copy);
    server_free(S);
    return SPX_OK;
}

// ------------------------------------------------------------------ spx_cg_batch
namespace {

bool batch_is_wide(const spx_batch_system &s)
{
    if (s.path == SPX_BATCH_WIDE) return true;
    if (s.path == SPX_BATCH_ONE_GROUP) return false;
    return s.n >= kWideDefaultRows;
}

// Workspace: narrow slot table, counter, wide tables, then per system r, p, q
// (+ for wide systems: s, 2 * nvb vector-phase partials, the product
// partials and the tile partition).
struct BatchLayout {
    size_t slots, counter, wslots, wstate, wmap, vb, ta, vectors, total;
    int64_t nwide, total_vb, total_ta;
};

BatchLayout batch_layout(const spx_batch_system *sys, int32_t count)
{
    BatchLayout L{};
    for (int32_t i = 0; i < count; ++i)
        if (batch_is_wide(sys[i])) {
            L.nwide += 1;
            L.total_vb += wide_nvb(sys[i].n);
            L.total_ta += csr_tiles(sys[i].nnz);
        }
    size_t off = 0;
    L.slots = off;
    off += align256(sizeof(BatchSlot) * (size_t)count);
    L.counter = off;
    off += 256;
    L.wslots = off;
    off += align256(sizeof(WideSlot) * (size_t)L.nwide);
    L.wstate = off;  // two buffers: even and odd iterations
    off += align256(sizeof(WideState) * 2 * (size_t)L.nwide);
    L.wmap = off;
    off += 256;
    L.vb = off;
    off += align256(sizeof(int32_t) * 2 * (size_t)L.total_vb);
    L.ta = off;
    off += align256(sizeof(int32_t) * 2 * (size_t)L.total_ta);
    L.vectors = off;
    for (int32_t i = 0; i < count; ++i) {
        off += 3 * align256((size_t)sys[i].n * 8);
        if (batch_is_wide(sys[i])) off += wide_extra_bytes(sys[i].n, sys[i].nnz);
    }
    L.total = off;
    return L;
}

}  // namespace

extern "C" spx_status spx_cg_batch_workspace(const spx_batch_system *sys, int32_t count, size_t *bytes)
{
    clear_error();
    SPX_REQUIRE(sys && bytes && count >= 0, SPX_ERR_ARG, "spx_cg_batch_workspace: bad argument");
    *bytes = batch_layout(sys, count).total;
    return SPX_OK;
}

namespace {

spx_status check_batch(const spx_batch_system *sys, int32_t count, const char *who)
{
    SPX_REQUIRE(sys && count >= 0, SPX_ERR_ARG, "%s: bad argument", who);
    for (int32_t i = 0; i < count; ++i) {
        SPX_REQUIRE(sys[i].n >= 1 && sys[i].rowptr && sys[i].b && sys[i].x && (sys[i].nnz == 0 || (sys[i].colidx && sys[i].vals)),
                    SPX_ERR_ARG, "%s: bad system %d", who, i);
        SPX_REQUIRE(sys[i].path >= SPX_BATCH_AUTO && sys[i].path <= SPX_BATCH_WIDE, SPX_ERR_ARG,
                    "%s: bad path of system %d", who, i);
    }
    return SPX_OK;
}

// The batch on a workspace of at least L.total bytes at base (checked by the
// caller); the workspace needs no clearing (the work counter is reset by a
// kernel, everything else is written before it is read).
spx_status cg_batch_run(spx_batch_system *sys, int32_t count, const BatchLayout &L, char *base, hipStream_t stream)
{
    BatchSlot *slots_dev = reinterpret_cast<BatchSlot *>(base + L.slots);
    int32_t *counter = reinterpret_cast<int32_t *>(base + L.counter);
    WideSlot *wslots_dev = reinterpret_cast<WideSlot *>(base + L.wslots);
    WideState *wstate_dev = reinterpret_cast<WideState *>(base + L.wstate);
    WideMap *wmap_dev = reinterpret_cast<WideMap *>(base + L.wmap);
    int32_t *vb_dev = reinterpret_cast<int32_t *>(base + L.vb);
    int32_t *ta_dev = reinterpret_cast<int32_t *>(base + L.ta);
    size_t off = L.vectors;
    std::vector<BatchSlot> host((size_t)count);
    std::vector<WideSlot> whost;
    std::vector<WideState> wstate;
    std::vector<int32_t> vb((size_t)(2 * L.total_vb)), ta((size_t)(2 * L.total_ta)), widx((size_t)count, -1);
    int64_t tot = 0, tta = 0;
    int32_t maxit_max = 1;
    for (int32_t i = 0; i < count; ++i) {
        const size_t vb_bytes = align256((size_t)sys[i].n * 8);
        double *r = reinterpret_cast<double *>(base + off);
        double *p = reinterpret_cast<double *>(base + off + vb_bytes);
        double *q = reinterpret_cast<double *>(base + off + 2 * vb_bytes);
        off += 3 * vb_bytes;
        const int32_t maxit = sys[i].maxit > 0 ? sys[i].maxit : 100000;
        maxit_max = std::max(maxit_max, maxit);
        BatchSlot &d = host[i];
        std::memset(&d, 0, sizeof(d));
        if (batch_is_wide(sys[i])) {
            WideSlot w{};
            w.rowptr = sys[i].rowptr;
            w.col = sys[i].colidx;
            w.val = sys[i].vals;
            w.b = sys[i].b;
            w.x = sys[i].x;
            w.r = r;
            w.p = p;
            w.w = q;
            const int64_t nnz = sys[i].nnz;
            w.s = reinterpret_cast<double *>(base + off);
            off += align256((size_t)sys[i].n * 8);
            w.part = reinterpret_cast<double *>(base + off);
            off += align256((size_t)wide_nvb(sys[i].n) * 4 * 8);
            w.part_a = reinterpret_cast<double *>(base + off);
            off += align256((size_t)csr_tiles(nnz) * 2 * 8);
            w.solver = kSlotCg;
            int32_t *cpart = reinterpret_cast<int32_t *>(base + off);
            off += align256((size_t)csr_partition_bytes(nnz));
            w.csr_part = cpart;
            w.nnz = nnz;
            w.ntiles = (int32_t)csr_tiles(nnz);
            {
                spx_matrix d{};
                d.fmt = SPX_CSR;
                d.nrows = sys[i].n;
                d.ncols = sys[i].n;
                d.nnz = nnz;
                d.rowptr = const_cast<int32_t *>(sys[i].rowptr);
                SPX_CHECK(csr_partition_launch(d, cpart, stream));
            }
            w.n = sys[i].n;
            w.nvb = wide_nvb(sys[i].n);
            w.maxit = maxit;
            w.tol2 = sys[i].tol * sys[i].tol;
            const int32_t k = (int32_t)whost.size();
            widx[i] = k;
            for (int32_t v = 0; v < w.nvb; ++v) {
                vb[tot + v] = k;
                vb[L.total_vb + tot + v] = v;
            }
            tot += w.nvb;
            for (int32_t v = 0; v < w.ntiles; ++v) {
                ta[tta + v] = k;
                ta[L.total_ta + tta + v] = v;
            }
            tta += w.ntiles;
            whost.push_back(w);
            WideState s0{};
            s0.mode = kWideInit;
            wstate.push_back(s0);
            d.status = kSlotEmpty;  // the one-group kernel skips it
        } else {
            d.rowptr = sys[i].rowptr;
            d.col = sys[i].colidx;
            d.val = sys[i].vals;
            d.b = sys[i].b;
            d.x = sys[i].x;
            d.r = r;
            d.p = p;
            d.q = q;
            d.n = sys[i].n;
            d.sub = narrow_sub_for(sys[i].n, sys[i].nnz);
            d.status = kSlotRunning;
            d.tol2 = sys[i].tol * sys[i].tol;
            d.maxit = maxit;
            d.budget = d.maxit;
        }
        SPX_HIP(hipMemsetAsync(sys[i].x, 0, (size_t)sys[i].n * 8, stream));
    }
    const int64_t nnarrow = count - L.nwide;
    if (nnarrow > 0) {
        SPX_HIP(hipMemcpyAsync(slots_dev, host.data(), sizeof(BatchSlot) * (size_t)count, hipMemcpyHostToDevice, stream));
        SPX_CHECK(batch_reset_launch(counter, stream));
        SPX_CHECK(batch_small_launch(slots_dev, count, counter, batch_small_resident_groups(), stream));
        SPX_CHECK(batch_cg_launch(slots_dev, count, counter, batch_resident_groups(), stream));
        SPX_HIP(hipMemcpyAsync(host.data(), slots_dev, sizeof(BatchSlot) * (size_t)count, hipMemcpyDeviceToHost, stream));
    }
    if (L.nwide > 0) {
        const WideMap m{(int32_t)L.total_vb, (int32_t)L.nwide, (int32_t)L.total_ta, 0};
        SPX_HIP(hipMemcpyAsync(wslots_dev, whost.data(), sizeof(WideSlot) * whost.size(), hipMemcpyHostToDevice, stream));
        SPX_HIP(hipMemcpyAsync(wstate_dev, wstate.data(), sizeof(WideState) * wstate.size(), hipMemcpyHostToDevice, stream));
        SPX_HIP(hipMemcpyAsync(wmap_dev, &m, sizeof(m), hipMemcpyHostToDevice, stream));
        SPX_HIP(hipMemcpyAsync(vb_dev, vb.data(), sizeof(int32_t) * vb.size(), hipMemcpyHostToDevice, stream));
        SPX_HIP(hipMemcpyAsync(ta_dev, ta.data(), sizeof(int32_t) * ta.size(), hipMemcpyHostToDevice, stream));
        const int grid = (int)std::min<int64_t>(std::max(L.total_vb, L.total_ta), 4096);
        // an iteration either takes a CG step or, at most twice per step, is
        // the true-residual check that follows a small recursive residual or
        // the decision after it, so 3 * maxit + 6 iterations finish every system
        const int64_t limit = 3 * (int64_t)maxit_max + 6;
        for (int64_t done = 0; done < limit;) {
            for (int k = 0; k < 16; ++k, ++done)  // even: the state ends in the first buffer
                SPX_CHECK(wide_iteration_launch(wslots_dev, (k & 1) ? wstate_dev + L.nwide : wstate_dev,
                                                (k & 1) ? wstate_dev : wstate_dev + L.nwide, wmap_dev, vb_dev,
                                                vb_dev + L.total_vb, ta_dev, ta_dev + L.total_ta, grid, stream));
            SPX_HIP(hipMemcpyAsync(wstate.data(), wstate_dev, sizeof(WideState) * wstate.size(), hipMemcpyDeviceToHost,
                                   stream));
            SPX_HIP(hipStreamSynchronize(stream));
            bool all = true;
            for (auto &w : wstate) all &= (w.mode == kWideDone);
            if (all) break;
        }
    }
    SPX_HIP(hipStreamSynchronize(stream));
    spx_status first = SPX_OK;
    for (int32_t i = 0; i < count; ++i) {
        if (widx[i] >= 0) {
            const WideState &w = wstate[(size_t)widx[i]];
            sys[i].status = w.mode != kWideDone ? SPX_ERR_NOT_CONVERGED
                                                : (w.status == kSlotConverged ? SPX_OK : slot_status_to_spx(w.status));
            sys[i].iters = w.iters;
            sys[i].spmv_count = w.spmv;
            sys[i].relres_true = w.relres_true;
        } else {
            const BatchSlot &d = host[i];
            sys[i].status = d.status == kSlotConverged ? SPX_OK : slot_status_to_spx(d.status);
            sys[i].iters = d.iters;
            sys[i].spmv_count = d.spmv;
            sys[i].relres_true = d.relres_true;
        }
        if (first == SPX_OK && sys[i].status != SPX_OK) first = (spx_status)sys[i].status;
    }
    if (first != SPX_OK) set_error("spx_cg_batch: at least one system did not converge");
    return first;
}

// Device scratch of spx_cg_batch_noalloc: a fixed array in the code object,
// so that the call needs no allocation. Each GPU the library runs on holds
// its own copy until the process ends. Host code never passes the array's
// name to a kernel (on the host it is only a stand-in for the symbol); it
// uses the device address that hipGetSymbolAddress returned for the device.
constexpr size_t kBatchScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kBatchScratchBytes];

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu[kMaxScratchDevices];  // one no-allocation batch at a time per device
std::mutex g_scratch_addr_mu;
char *g_scratch_addr[kMaxScratchDevices] = {};

// The scratch array's address on the current device, looked up on the
// device's first call.
spx_status scratch_address(int dev, char **out)
{
    std::lock_guard<std::mutex> lk(g_scratch_addr_mu);
    if (g_scratch_addr[dev] == nullptr) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr) {
            set_error("spx_cg_batch_noalloc: hipGetSymbolAddress(scratch) on device %d: %s", dev,
                      hipGetErrorString(e));
            return SPX_ERR_HIP;
        }
        g_scratch_addr[dev] = static_cast<char *>(p);
    }
    *out = g_scratch_addr[dev];
    return SPX_OK;
}

}  // namespace

extern "C" spx_status spx_cg_batch(spx_batch_system *sys, int32_t count, void *ws, size_t ws_bytes,
                                   hipStream_t stream)
{
    clear_error();
    SPX_CHECK(check_batch(sys, count, "spx_cg_batch"));
    if (count == 0) return SPX_OK;
    const BatchLayout L = batch_layout(sys, count);
    SPX_REQUIRE(ws && ws_bytes >= L.total, SPX_ERR_ARG, "spx_cg_batch: workspace too small");
    return cg_batch_run(sys, count, L, static_cast<char *>(ws), stream);
}

extern "C" spx_status spx_cg_batch_noalloc(spx_batch_system *sys, int32_t count, hipStream_t stream)
{
    clear_error();
    SPX_CHECK(check_batch(sys, count, "spx_cg_batch_noalloc"));
    if (count == 0) return SPX_OK;
    const BatchLayout L = batch_layout(sys, count);
    SPX_REQUIRE(L.total <= kBatchScratchBytes, SPX_ERR_ARG,
                "spx_cg_batch_noalloc: the batch needs %zu bytes of scratch, more than the %zu available "
                "(use spx_cg_batch with a workspace)",
                L.total, kBatchScratchBytes);
    int dev = 0;
    SPX_HIP(hipGetDevice(&dev));
    SPX_REQUIRE(dev >= 0 && dev < kMaxScratchDevices, SPX_ERR_ARG, "spx_cg_batch_noalloc: device %d out of range",
                dev);
    char *base = nullptr;
    SPX_CHECK(scratch_address(dev, &base));
    std::lock_guard<std::mutex> lk(g_scratch_mu[dev]);
    return cg_batch_run(sys, count, L, base, stream);
}
