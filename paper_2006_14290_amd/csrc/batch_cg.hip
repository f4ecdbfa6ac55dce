// batch_cg.hip -- persistent batched CG: one work-group per system.
//
// A persistent grid of resident work-groups takes systems ("slots") from an
// atomic counter; the work-group that takes a slot runs up to slot.budget
// iterations of unpreconditioned CG on it (the textbook recurrences of
// Hestenes & Stiefel) entirely by itself: the CSR product with adaptive
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

__device__ void run_slot(BatchSlot *slot, double *s_red)
{
    const BatchSlot S = *slot;
    if (S.status != kSlotRunning || S.budget <= 0) return;
    const int64_t n = S.n;
    const int tid = threadIdx.x;
    double rho = S.rho, rr = S.rr, bb = S.bb, relres = S.relres_true;
    int32_t iters = S.iters, spmv = S.spmv, status = kSlotRunning, started = S.started;
    if (!started) {  // x0 = 0: r = b, p = b
        double t = 0.0;
        for (int64_t i = tid; i < n; i += kBatchThreads) {
            const double bi = S.b[i];
            S.r[i] = bi;
            S.p[i] = bi;
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
        const double pq = wg_spmv(S, S.p, S.q, true, s_red);
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
            S.x[i] += alpha * S.p[i];
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
            for (int64_t i = tid; i < n; i += kBatchThreads) S.p[i] = S.r[i];  // restart from it
            rho = tr;
            rr = tr;
            __syncthreads();
            if (iters >= S.maxit) status = kSlotMaxit;
            continue;
        }
        const double beta = rr / rho;
        rho = rr;
        for (int64_t i = tid; i < n; i += kBatchThreads) S.p[i] = S.r[i] + beta * S.p[i];
        __syncthreads();
        if (iters >= S.maxit) status = kSlotMaxit;
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

__global__ __launch_bounds__(kBatchThreads) void batch_cg_kernel(BatchSlot *slots, int32_t nslots,
                                                                int32_t *counter)
{
    __shared__ double s_red[kBatchWaves];
    __shared__ int32_t s_k;
    while (true) {
        if (threadIdx.x == 0) s_k = atomicAdd(counter, 1);
        __syncthreads();
        const int32_t k = s_k;
        __syncthreads();
        if (k >= nslots) return;  // every work-group leaves once the slots are handed out
        run_slot(&slots[k], s_red);
        __syncthreads();
    }
}

__global__ void batch_reset_kernel(int32_t *counter)
{
    if (threadIdx.x == 0) *counter = 0;
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

spx_status batch_cg_launch(BatchSlot *slots, int32_t nslots, int32_t *counter, int64_t grid, hipStream_t stream)
{
    if (grid > nslots) grid = nslots;
    if (grid < 1) grid = 1;
    batch_cg_kernel<<<(unsigned)grid, kBatchThreads, 0, stream>>>(slots, nslots, counter);
    SPX_LAUNCHED();
    return SPX_OK;
}

}  // namespace spx
