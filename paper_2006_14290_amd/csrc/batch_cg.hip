// batch_cg.hip -- persistent batched CG: one work-group per system.
//
// A persistent grid of resident work-groups takes systems ("slots") from an
// atomic counter; the work-group that takes a slot runs up to slot.budget
// iterations of unpreconditioned CG on it (the textbook recurrences of
// Hestenes & Stiefel), or of BiCGSTAB for a nonsymmetric slot, entirely by
// itself: the CSR product with adaptive
// subwarps (DPP reductions), the vector updates, and every dot product as a
// fixed-order work-group reduction. There is no synchronisation between
// work-groups at all, so nothing waits on another group and each system's
// arithmetic is independent of which group ran it and of what else is in the
// batch: a system gives bitwise the same iterates alone or in any mix, and
// across launches (the state is kept in the slot and its vectors between
// launches, so a solve can be spread over several launches).
// Convergence (||r|| <= tol ||b||) is confirmed with the true residual
// b - A x; a miss restarts the recurrences from it.
#include "batch_cg.hpp"
#include "wave.hpp"

namespace spx {

constexpr int kBatchWaves = kBatchThreads / kWave;

// Work-group sums of NV values, fixed order, results in every thread
// (s_red holds NV * kBatchWaves doubles).
template <int NV>
__device__ __forceinline__ void wg_sums(double (&v)[NV], double *s_red)
{
    const int w = threadIdx.x / kWave;
#pragma unroll
    for (int j = 0; j < NV; ++j) v[j] = wave_sum(v[j]);
    if (lane_id() == 0)
#pragma unroll
        for (int j = 0; j < NV; ++j) s_red[j * kBatchWaves + w] = v[j];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        double t = 0.0;
        for (int k = 0; k < kBatchWaves; ++k) t += s_red[j * kBatchWaves + k];
        v[j] = t;
    }
    __syncthreads();
}

// Work-group sum, fixed order, result in every thread.
__device__ __forceinline__ double wg_sum(double v, double *s_red)
{
    v = wave_sum(v);
    if (lane_id() == 0) s_red[threadIdx.x / kWave] = v;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < kBatchWaves; ++w) t += s_red[w];
    __syncthreads();
    return t;
}

// q = A v over all rows; returns sum_i v_i q_i if `dot` (all threads).
__device__ double wg_spmv(const BatchSlot &S, const double *__restrict__ v, double *__restrict__ q, bool dot,
                          double *s_red)
{
    const int sub = S.sub;
    const int g = threadIdx.x / sub, sl = threadIdx.x % sub;
    const int G = kBatchThreads / sub;
    double acc = 0.0;
    for (int64_t row0 = 0; row0 < S.n; row0 += G) {  // uniform trip count: DPP needs whole groups
        const int64_t row = row0 + g;
        double sum = 0.0;
        if (row < S.n) {
            const int32_t a = S.rowptr[row], b = S.rowptr[row + 1];
#pragma unroll 4
            for (int32_t k = a + sl; k < b; k += sub) sum += S.val[k] * v[S.col[k]];
        }
        sum = subwave_sum_dyn(sum, sub);
        if (row < S.n && sl == 0) {
            q[row] = sum;
            if (dot) acc += sum * v[row];
        }
    }
    return wg_sum(acc, s_red);
}

// q = A v over all rows; d[0] = sum_i q_i w_i and, if KD == 2, d[1] = sum_i
// q_i^2 (all threads).
template <int KD>
__device__ void wg_spmv_dots(const BatchSlot &S, const double *__restrict__ v, double *__restrict__ q,
                             const double *__restrict__ w, double (&d)[KD], double *s_red)
{
    const int sub = S.sub;
    const int g = threadIdx.x / sub, sl = threadIdx.x % sub;
    const int G = kBatchThreads / sub;
#pragma unroll
    for (int j = 0; j < KD; ++j) d[j] = 0.0;
    for (int64_t row0 = 0; row0 < S.n; row0 += G) {  // uniform trip count: DPP needs whole groups
        const int64_t row = row0 + g;
        double sum = 0.0;
        if (row < S.n) {
            const int32_t a = S.rowptr[row], b = S.rowptr[row + 1];
#pragma unroll 4
            for (int32_t k = a + sl; k < b; k += sub) sum += S.val[k] * v[S.col[k]];
        }
        sum = subwave_sum_dyn(sum, sub);
        if (row < S.n && sl == 0) {
            q[row] = sum;
            d[0] += sum * w[row];
            if constexpr (KD == 2) d[1] += sum * sum;
        }
    }
    wg_sums<KD>(d, s_red);
}

// Unpreconditioned BiCGSTAB (van der Vorst 1992, in the form of Barrett et
// al., "Templates", 1994) on one slot from x0 = 0, resumable across
// launches: s overwrites r, v is kept in q. Convergence of ||s|| (half step)
// or ||r|| (full step) is confirmed with the true residual b - A x (A x is
// formed in t); a miss restarts the recurrences from it with r_hat = r.
// Iterations count full steps (two products each).
__device__ void run_slot_bicgstab(BatchSlot *slot, double *s_red)
{
    const BatchSlot S = *slot;
    if (S.status != kSlotRunning || S.budget <= 0) return;
    const int64_t n = S.n;
    const int tid = threadIdx.x;
    double *__restrict__ x = S.x;
    double *__restrict__ r = S.r;
    double *__restrict__ rh = S.rh;
    double *__restrict__ p = S.p;
    double *__restrict__ v = S.q;
    double *__restrict__ t = S.t;
    double rho = S.rho, rho0 = S.rho0, alpha = S.alpha, omega = S.omega, rr = S.rr, bb = S.bb,
           relres = S.relres_true;
    int32_t iters = S.iters, spmv = S.spmv, status = kSlotRunning, started = S.started, first = S.first;
    if (!started) {  // x0 = 0: r = b, r_hat = r
        double sum[1] = {0.0};
        for (int64_t i = tid; i < n; i += kBatchThreads) {
            const double bi = S.b[i];
            r[i] = bi;
            rh[i] = bi;
            sum[0] += bi * bi;
        }
        wg_sums<1>(sum, s_red);
        bb = sum[0];
        rr = bb;
        rho = bb;  // r_hat . r with r_hat = r
        rho0 = alpha = omega = 1.0;
        first = 1;
        started = 1;
        if (!__builtin_isfinite(bb)) status = kSlotNonfinite;
        else if (bb == 0.0) {
            status = kSlotConverged;
            relres = 0.0;
        }
    }
    // true residual r = b - A x (A x in t); converged, or restart from it
    auto confirm = [&]() -> bool {
        double d[1];
        wg_spmv_dots<1>(S, x, t, x, d, s_red);  // the dot is not used
        spmv += 1;
        double tr[1] = {0.0};
        for (int64_t i = tid; i < n; i += kBatchThreads) {
            const double ri = S.b[i] - t[i];
            r[i] = ri;
            rh[i] = ri;
            tr[0] += ri * ri;
        }
        wg_sums<1>(tr, s_red);
        if (tr[0] <= S.tol2 * bb) {
            relres = sqrt(tr[0] / bb);
            return true;
        }
        rr = tr[0];
        rho = tr[0];
        rho0 = alpha = omega = 1.0;
        first = 1;
        return false;
    };
    for (int it = 0; it < S.budget && status == kSlotRunning; ++it) {
        if (iters >= S.maxit) {
            status = kSlotMaxit;
            break;
        }
        iters += 1;
        if (!__builtin_isfinite(rho)) {
            status = kSlotNonfinite;
            break;
        }
        if (rho == 0.0) {
            status = kSlotBreakdown;
            break;
        }
        if (first) {
            for (int64_t i = tid; i < n; i += kBatchThreads) p[i] = r[i];
            first = 0;
        } else {
            const double beta = (rho / rho0) * (alpha / omega);
            for (int64_t i = tid; i < n; i += kBatchThreads) p[i] = r[i] + beta * (p[i] - omega * v[i]);
        }
        __syncthreads();  // p complete before the product gathers it
        double d1[1];
        wg_spmv_dots<1>(S, p, v, rh, d1, s_red);  // v = A p, r_hat . v
        spmv += 1;
        const double rhv = d1[0];
        if (rhv == 0.0 || !__builtin_isfinite(rhv)) {
            status = __builtin_isfinite(rhv) ? kSlotBreakdown : kSlotNonfinite;
            break;
        }
        alpha = rho / rhv;
        double ss[1] = {0.0};
        for (int64_t i = tid; i < n; i += kBatchThreads) {
            const double si = r[i] - alpha * v[i];
            r[i] = si;
            ss[0] += si * si;
        }
        wg_sums<1>(ss, s_red);  // its barriers also complete s before the next product
        rr = ss[0];
        if (ss[0] <= S.tol2 * bb) {
            for (int64_t i = tid; i < n; i += kBatchThreads) x[i] += alpha * p[i];
            __syncthreads();
            if (confirm()) {
                status = kSlotConverged;
                break;
            }
            continue;
        }
        double d2[2];
        wg_spmv_dots<2>(S, r, t, r, d2, s_red);  // t = A s, t . s, t . t
        spmv += 1;
        const double ts = d2[0], tt = d2[1];
        if (!__builtin_isfinite(tt)) {
            status = kSlotNonfinite;
            break;
        }
        if (tt == 0.0) {
            status = kSlotBreakdown;
            break;
        }
        omega = ts / tt;
        double nr[2] = {0.0, 0.0};
        for (int64_t i = tid; i < n; i += kBatchThreads) {
            const double si = r[i];
            x[i] += alpha * p[i] + omega * si;
            const double ri = si - omega * t[i];
            r[i] = ri;
            nr[0] += ri * ri;
            nr[1] += rh[i] * ri;
        }
        wg_sums<2>(nr, s_red);
        rr = nr[0];
        rho0 = rho;
        rho = nr[1];
        if (!__builtin_isfinite(rr)) {
            status = kSlotNonfinite;
            break;
        }
        if (rr <= S.tol2 * bb) {
            if (confirm()) {
                status = kSlotConverged;
                break;
            }
            continue;
        }
        if (omega == 0.0) {
            status = kSlotBreakdown;
            break;
        }
    }
    __syncthreads();
    if (tid == 0) {
        slot->rho = rho;
        slot->rho0 = rho0;
        slot->alpha = alpha;
        slot->omega = omega;
        slot->rr = rr;
        slot->bb = bb;
        slot->iters = iters;
        slot->spmv = spmv;
        slot->started = started;
        slot->first = first;
        slot->status = status;
        slot->relres_true = (status == kSlotConverged) ? relres : (bb > 0 ? sqrt(rr / bb) : 0.0);
    }
}

// kLds: the system has at most kBatchLdsRows rows and its search direction
// lives in LDS while the work-group runs it (the product gathers it there);
// it is loaded from and stored back to the slot's p at the ends of a launch.
template <bool kLds>
__device__ void run_slot(BatchSlot *slot, double *s_red, double *s_p)
{
    const BatchSlot S = *slot;
    if (S.status != kSlotRunning || S.budget <= 0 || S.n <= kBatchSmallRows) return;
    double *P = kLds ? s_p : S.p;
    if (kLds && S.started) {
        for (int64_t i = threadIdx.x; i < S.n; i += kBatchThreads) s_p[i] = S.p[i];
        __syncthreads();
    }
    const int64_t n = S.n;
    const int tid = threadIdx.x;
    double rho = S.rho, rr = S.rr, bb = S.bb, relres = S.relres_true;
    int32_t iters = S.iters, spmv = S.spmv, status = kSlotRunning, started = S.started;
    if (!started) {  // x0 = 0: r = b, p = b
        double t = 0.0;
        for (int64_t i = tid; i < n; i += kBatchThreads) {
            const double bi = S.b[i];
            S.r[i] = bi;
            P[i] = bi;
            t += bi * bi;
        }
        bb = wg_sum(t, s_red);
        rho = bb;
        rr = bb;
        started = 1;
        if (!__builtin_isfinite(bb)) status = kSlotNonfinite;
        else if (bb == 0.0) {
            status = kSlotConverged;
            relres = 0.0;
        }
    }
    for (int it = 0; it < S.budget && status == kSlotRunning; ++it) {
        const double pq = wg_spmv(S, P, S.q, true, s_red);
        spmv += 1;
        if (!__builtin_isfinite(pq)) {
            status = kSlotNonfinite;
            break;
        }
        if (pq <= 0.0) {
            status = kSlotBreakdown;
            break;
        }
        const double alpha = rho / pq;
        double t = 0.0;
        for (int64_t i = tid; i < n; i += kBatchThreads) {
            S.x[i] += alpha * P[i];
            const double ri = S.r[i] - alpha * S.q[i];
            S.r[i] = ri;
            t += ri * ri;
        }
        rr = wg_sum(t, s_red);
        iters += 1;
        if (!__builtin_isfinite(rr)) {
            status = kSlotNonfinite;
            break;
        }
        if (rr <= S.tol2 * bb) {
            // confirm with the true residual b - A x
            wg_spmv(S, S.x, S.q, false, s_red);
            spmv += 1;
            double tr = 0.0;
            for (int64_t i = tid; i < n; i += kBatchThreads) {
                const double ri = S.b[i] - S.q[i];
                S.r[i] = ri;
                tr += ri * ri;
            }
            tr = wg_sum(tr, s_red);
            if (tr <= S.tol2 * bb) {
                status = kSlotConverged;
                relres = sqrt(tr / bb);
                break;
            }
            for (int64_t i = tid; i < n; i += kBatchThreads) P[i] = S.r[i];  // restart from it
            rho = tr;
            rr = tr;
            __syncthreads();
            if (iters >= S.maxit) status = kSlotMaxit;
            continue;
        }
        const double beta = rr / rho;
        rho = rr;
        for (int64_t i = tid; i < n; i += kBatchThreads) P[i] = S.r[i] + beta * P[i];
        __syncthreads();
        if (iters >= S.maxit) status = kSlotMaxit;
    }
    if (kLds)
        for (int64_t i = threadIdx.x; i < S.n; i += kBatchThreads) S.p[i] = s_p[i];  // this thread wrote them last
    if (tid == 0) {
        slot->rho = rho;
        slot->rr = rr;
        slot->bb = bb;
        slot->iters = iters;
        slot->spmv = spmv;
        slot->started = started;
        slot->status = status;
        slot->relres_true = (status == kSlotConverged) ? relres : (bb > 0 ? sqrt(rr / bb) : 0.0);
    }
}

__global__ __launch_bounds__(kBatchThreads) void batch_cg_kernel(BatchSlot *slots, int32_t nslots,
                                                                int32_t *counter)
{
    __shared__ double s_red[2 * kBatchWaves];
    __shared__ double s_p[kBatchLdsRows];
    __shared__ int32_t s_k;
    while (true) {
        if (threadIdx.x == 0) s_k = atomicAdd(counter, 1);
        __syncthreads();
        const int32_t k = s_k;
        __syncthreads();
        if (k >= nslots) return;  // every work-group leaves once the slots are handed out
        if (slots[k].solver == kSlotBicgstab) run_slot_bicgstab(&slots[k], s_red);
        else if (slots[k].n <= kBatchLdsRows) run_slot<true>(&slots[k], s_red, s_p);
        else run_slot<false>(&slots[k], s_red, s_p);
        __syncthreads();
    }
}

__global__ void batch_reset_kernel(int32_t *counter)
{
    if (threadIdx.x < 2) counter[threadIdx.x] = 0;
}

// ---------------------------------------------------------------- small systems
// One 512-thread work-group per system of at most kBatchSmallRows rows:
// thread t owns rows t + 512 k (k < 8). While the work-group runs the slot,
// p lives in LDS (where the product gathers it) and x, r in registers; they
// are loaded from the slot's vectors at the start of a launch and stored back
// at its end, so a solve may be spread over launches. When no row has more
// than kBSLen entries the rows' columns and values are held in registers
// too. Same recurrences, stopping test and true-residual restart as
// run_slot; every dot product is a fixed-order work-group reduction.
constexpr int kBSThreads = 512;
constexpr int kBSR = kBatchSmallRows / kBSThreads;
constexpr int kBSWaves = kBSThreads / kWave;
constexpr int kBSLen = 5;

// Work-group sums, result in every thread (alternating LDS buffers: one
// barrier each).
template <int NV>
__device__ __forceinline__ void bs_sum(double (&v)[NV], double (*s_red)[2 * kBSWaves], int &par)
{
    const int w = threadIdx.x / kWave, l = lane_id();
#pragma unroll
    for (int j = 0; j < NV; ++j) v[j] = wave_sum(v[j]);
    if (l == 0)
#pragma unroll
        for (int j = 0; j < NV; ++j) s_red[par][j * kBSWaves + w] = v[j];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        const double t = l < kBSWaves ? s_red[par][j * kBSWaves + l] : 0.0;
        v[j] = readlane(subwave_sum<kBSWaves>(t), 0);
    }
    par ^= 1;
}

template <bool kCached>
__device__ __noinline__ void run_small_slot(BatchSlot *slot, double *s_v, double (*s_red)[2 * kBSWaves])
{
    const BatchSlot S = *slot;
    const int tid = threadIdx.x;
    const int32_t n = S.n;
    int par = 0;
    int32_t ra[kBSR], rb[kBSR];
#pragma unroll
    for (int k = 0; k < kBSR; ++k) {
        const int i = tid + k * kBSThreads;
        ra[k] = i < n ? S.rowptr[i] : 0;
        rb[k] = i < n ? S.rowptr[i + 1] : 0;
    }
    int32_t cc[kCached ? kBSR : 1][kCached ? kBSLen : 1];
    double vv[kCached ? kBSR : 1][kCached ? kBSLen : 1];
    int32_t ln[kCached ? kBSR : 1];
    if constexpr (kCached) {
#pragma unroll
        for (int k = 0; k < kBSR; ++k) {
            ln[k] = rb[k] - ra[k];
#pragma unroll
            for (int e = 0; e < kBSLen; ++e) {
                const bool in = e < ln[k];
                cc[k][e] = in ? S.col[ra[k] + e] : 0;
                vv[k][e] = in ? S.val[ra[k] + e] : 0.0;
            }
        }
    }
    // row k of A times v (in LDS), entries in order
    auto row = [&](int k, const double *v) -> double {
        double t = 0.0;
        if constexpr (kCached) {
#pragma unroll
            for (int e = 0; e < kBSLen; ++e)
                if (e < ln[k]) t += vv[k][e] * v[cc[k][e]];
        } else {
#pragma unroll 2
            for (int32_t j = ra[k]; j < rb[k]; ++j) t += S.val[j] * v[S.col[j]];
        }
        return t;
    };
    double xr[kBSR], rv[kBSR];
    double rho = S.rho, rr = S.rr, bb = S.bb, relres = S.relres_true;
    int32_t iters = S.iters, spmv = S.spmv, status = kSlotRunning, started = S.started;
    if (!started) {  // x0 = 0: r = b, p = b
        double t[1] = {0.0};
#pragma unroll
        for (int k = 0; k < kBSR; ++k) {
            const int i = tid + k * kBSThreads;
            const double bi = i < n ? S.b[i] : 0.0;
            xr[k] = 0.0;
            rv[k] = bi;
            s_v[i] = bi;
            t[0] += bi * bi;
        }
        bs_sum<1>(t, s_red, par);  // its barrier also publishes p
        bb = t[0];
        rho = bb;
        rr = bb;
        started = 1;
        if (!__builtin_isfinite(bb)) status = kSlotNonfinite;
        else if (bb == 0.0) {
            status = kSlotConverged;
            relres = 0.0;
        }
    } else {
#pragma unroll
        for (int k = 0; k < kBSR; ++k) {
            const int i = tid + k * kBSThreads;
            const bool in = i < n;
            xr[k] = in ? S.x[i] : 0.0;
            rv[k] = in ? S.r[i] : 0.0;
            s_v[i] = in ? S.p[i] : 0.0;
        }
        __syncthreads();
    }
    for (int it = 0; it < S.budget && status == kSlotRunning; ++it) {
        double qv[kBSR];
        double t[1] = {0.0};
#pragma unroll
        for (int k = 0; k < kBSR; ++k) {
            qv[k] = row(k, s_v);
            t[0] += s_v[tid + k * kBSThreads] * qv[k];
        }
        bs_sum<1>(t, s_red, par);
        spmv += 1;
        const double pq = t[0];
        if (!__builtin_isfinite(pq)) {
            status = kSlotNonfinite;
            break;
        }
        if (pq <= 0.0) {
            status = kSlotBreakdown;
            break;
        }
        const double alpha = rho / pq;
        double t2[1] = {0.0};
#pragma unroll
        for (int k = 0; k < kBSR; ++k) {
            xr[k] += alpha * s_v[tid + k * kBSThreads];
            rv[k] = rv[k] - alpha * qv[k];
            t2[0] += rv[k] * rv[k];
        }
        bs_sum<1>(t2, s_red, par);  // its barrier: every gather of p is done
        rr = t2[0];
        iters += 1;
        if (!__builtin_isfinite(rr)) {
            status = kSlotNonfinite;
            break;
        }
        if (rr <= S.tol2 * bb) {
            // confirm with the true residual b - A x (x staged in LDS)
#pragma unroll
            for (int k = 0; k < kBSR; ++k) s_v[tid + k * kBSThreads] = xr[k];
            __syncthreads();
            double t3[1] = {0.0};
#pragma unroll
            for (int k = 0; k < kBSR; ++k) {
                const int i = tid + k * kBSThreads;
                const double bi = i < n ? S.b[i] : 0.0;
                rv[k] = bi - row(k, s_v);
                t3[0] += rv[k] * rv[k];
            }
            spmv += 1;
            bs_sum<1>(t3, s_red, par);  // its barrier: every gather of x is done
            const double tr = t3[0];
            if (tr <= S.tol2 * bb) {
                status = kSlotConverged;
                relres = sqrt(tr / bb);
                break;
            }
            // restart from it: p = r
#pragma unroll
            for (int k = 0; k < kBSR; ++k) s_v[tid + k * kBSThreads] = rv[k];
            __syncthreads();
            rho = tr;
            rr = tr;
            if (iters >= S.maxit) status = kSlotMaxit;
            continue;
        }
        const double beta = rr / rho;
        rho = rr;
#pragma unroll
        for (int k = 0; k < kBSR; ++k) {
            const int i = tid + k * kBSThreads;
            s_v[i] = rv[k] + beta * s_v[i];  // only this thread touches its rows here
        }
        __syncthreads();
        if (iters >= S.maxit) status = kSlotMaxit;
    }
#pragma unroll
    for (int k = 0; k < kBSR; ++k) {
        const int i = tid + k * kBSThreads;
        if (i < n) {
            S.x[i] = xr[k];
            S.r[i] = rv[k];
            S.p[i] = s_v[i];
        }
    }
    if (tid == 0) {
        slot->rho = rho;
        slot->rr = rr;
        slot->bb = bb;
        slot->iters = iters;
        slot->spmv = spmv;
        slot->started = started;
        slot->status = status;
        slot->relres_true = (status == kSlotConverged) ? relres : (bb > 0 ? sqrt(rr / bb) : 0.0);
    }
}

__global__ __launch_bounds__(kBSThreads) void batch_small_kernel(BatchSlot *slots, int32_t nslots, int32_t *counter)
{
    __shared__ double s_v[kBatchSmallRows];
    __shared__ double s_red[2][2 * kBSWaves];
    __shared__ int32_t s_k;
    while (true) {
        if (threadIdx.x == 0) s_k = atomicAdd(counter, 1);
        __syncthreads();
        const int32_t k = s_k;
        __syncthreads();
        if (k >= nslots) return;  // every work-group leaves once the slots are handed out
        BatchSlot *slot = &slots[k];
        if (slot->status != kSlotRunning || slot->budget <= 0 || slot->n > kBatchSmallRows ||
            slot->solver != kSlotCg)
            continue;
        // the cached form when no row of this system has more than kBSLen entries
        bool long_row = false;
        for (int i = threadIdx.x; i < slot->n; i += kBSThreads)
            long_row |= slot->rowptr[i + 1] - slot->rowptr[i] > kBSLen;
        if (__syncthreads_or(long_row)) run_small_slot<false>(slot, s_v, s_red);
        else run_small_slot<true>(slot, s_v, s_red);
        __syncthreads();
    }
}

int64_t batch_small_resident_groups()
{
    static int64_t cached = 0;
    if (cached == 0) {
        int dev = 0, cus = 256, per_cu = 1;
        if (hipGetDevice(&dev) == hipSuccess) {
            hipDeviceProp_t prop;
            if (hipGetDeviceProperties(&prop, dev) == hipSuccess) cus = prop.multiProcessorCount;
        }
        int b = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, batch_small_kernel, kBSThreads, 0) == hipSuccess && b > 0)
            per_cu = b;
        cached = (int64_t)cus * per_cu;
    }
    return cached;
}

int64_t batch_resident_groups()
{
    static int64_t cached = 0;
    if (cached == 0) {
        int dev = 0, cus = 256, per_cu = 1;
        if (hipGetDevice(&dev) == hipSuccess) {
            hipDeviceProp_t prop;
            if (hipGetDeviceProperties(&prop, dev) == hipSuccess) cus = prop.multiProcessorCount;
        }
        int b = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, batch_cg_kernel, kBatchThreads, 0) == hipSuccess && b > 0)
            per_cu = b;
        cached = (int64_t)cus * per_cu;
    }
    return cached;
}

spx_status batch_reset_launch(int32_t *counter, hipStream_t stream)
{
    batch_reset_kernel<<<1, 64, 0, stream>>>(counter);
    SPX_LAUNCHED();
    return SPX_OK;
}

spx_status batch_small_launch(BatchSlot *slots, int32_t nslots, int32_t *counter, int64_t grid, hipStream_t stream)
{
    if (grid > nslots) grid = nslots;
    if (grid < 1) grid = 1;
    batch_small_kernel<<<(unsigned)grid, kBSThreads, 0, stream>>>(slots, nslots, counter + 1);
    SPX_LAUNCHED();
    return SPX_OK;
}

spx_status batch_cg_launch(BatchSlot *slots, int32_t nslots, int32_t *counter, int64_t grid, hipStream_t stream)
{
    if (grid > nslots) grid = nslots;
    if (grid < 1) grid = 1;
    batch_cg_kernel<<<(unsigned)grid, kBatchThreads, 0, stream>>>(slots, nslots, counter);
    SPX_LAUNCHED();
    return SPX_OK;
}

}  // namespace spx
