// batch_wide.hip -- CG on many large systems at once, several work-groups per
// system, no synchronisation between work-groups inside a launch.
//
// Unpreconditioned CG (Hestenes & Stiefel), x0 = 0, one iteration as three
// grid-wide phases over every listed system (a launch boundary is the only
// global synchronisation):
//   A  q = A p (or q = A x in the true-residual mode), partial sums of p.q:
//      the load-balanced CSR tile kernel over every listed system's tiles;
//   B  alpha = rho / p.q from the partials; x += alpha p, r -= alpha q,
//      partial sums of r.r (true-residual mode: r = b - q; init: r = b);
//   C  beta = r.r / rho from the partials; p = r + beta p (or p = r on a
//      restart or at init) -- skipped once r.r passes the tolerance; the
//      first block of each system also commits its scalar state (rho,
//      iteration count, mode, status) into the other of two state buffers.
// Every work-group that needs a sum forms it from the same partials in the
// same order, so all of them take the same decisions. A system's virtual
// blocks, partials and summation order depend only on its own size; its
// arithmetic is therefore independent of the other systems in the launch.
#include "batch_cg.hpp"
#include "spmv_csr.hpp"
#include "spmv_csr_tile.hpp"
#include "wave.hpp"

namespace spx {

constexpr int kWideWaves = kWideThreads / kWave;

// Work-group sum in a fixed order (result in every thread).
__device__ __forceinline__ double wide_wg_sum(double v, double *s_red)
{
    v = wave_sum(v);
    __syncthreads();  // s_red may still be read by a previous call
    if (lane_id() == 0) s_red[threadIdx.x / kWave] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kWideWaves; ++w) t += s_red[w];
    return t;
}

// Sum of part[0..cnt): thread t takes t, t + 256, ... in order (eight
// strides' loads in flight), then the fixed work-group reduction.
__device__ __forceinline__ double wide_part_sum(const double *part, int32_t cnt, double *s_red)
{
    double t = 0.0;
#pragma unroll 8
    for (int32_t i = threadIdx.x; i < cnt; i += kWideThreads) t += part[i];
    return wide_wg_sum(t, s_red);
}

// Product phase: one work-group per virtual tile (system, tile). The tile
// kernel runs with its p.q epilogue in both modes (the true-residual mode
// multiplies x and ignores the partial).
__global__ __launch_bounds__(kCsrThreads) void wide_a_kernel(const WideSlot *__restrict__ slots,
                                                             const WideState *__restrict__ st,
                                                             const WideMap *__restrict__ map,
                                                             const int32_t *__restrict__ ta_slot,
                                                             const int32_t *__restrict__ ta_local)
{
    const int32_t total = map->total_ta;
    for (int32_t v = blockIdx.x; v < total; v += gridDim.x) {
        const int32_t s = ta_slot[v], k = ta_local[v];
        const int32_t mode = st[s].mode;
        if (mode != kWideRun && mode != kWideCheck) continue;
        const WideSlot S = slots[s];
        const double *src = mode == kWideRun ? S.p : S.x;
        csr_tile<double, double, 1, kCsrThreads, kCsrTile, 1, kCsrLateGather>(
            k, S.n, S.nnz, S.ntiles, S.rowptr, S.col, S.val, src, S.q, 1.0, 0.0, src, S.part_a, S.csr_part);
    }
}

__global__ __launch_bounds__(kWideThreads) void wide_b_kernel(const WideSlot *__restrict__ slots,
                                                              const WideState *__restrict__ st,
                                                              const WideMap *__restrict__ map,
                                                              const int32_t *__restrict__ vb_slot,
                                                              const int32_t *__restrict__ vb_local)
{
    __shared__ double s_red[kWideWaves];
    const int32_t total = map->total_vb;
    for (int32_t v = blockIdx.x; v < total; v += gridDim.x) {
        const int32_t s = vb_slot[v], lv = vb_local[v];
        const int32_t mode = st[s].mode;
        if (mode == kWideDone) continue;
        const WideSlot S = slots[s];
        const int32_t r0 = lv * kWideRows, r1 = min(S.n, r0 + kWideRows);
        double t = 0.0;
        if (mode == kWideRun) {
            const double pq = wide_part_sum(S.part_a, S.ntiles, s_red);
            if (!(pq > 0.0) || !__builtin_isfinite(pq)) continue;  // the commit phase records the breakdown
            const double alpha = st[s].rho / pq;
            for (int32_t i = r0 + threadIdx.x; i < r1; i += kWideThreads) {
                S.x[i] += alpha * S.p[i];
                const double ri = S.r[i] - alpha * S.q[i];
                S.r[i] = ri;
                t += ri * ri;
            }
        } else if (mode == kWideCheck) {
            for (int32_t i = r0 + threadIdx.x; i < r1; i += kWideThreads) {
                const double ri = S.b[i] - S.q[i];
                S.r[i] = ri;
                t += ri * ri;
            }
        } else {  // init: x = 0 was written at admission
            for (int32_t i = r0 + threadIdx.x; i < r1; i += kWideThreads) {
                const double bi = S.b[i];
                S.r[i] = bi;
                t += bi * bi;
            }
        }
        t = wide_wg_sum(t, s_red);
        if (threadIdx.x == 0) S.part[lv] = t;
    }
}

// Scalar state update of one system from the two partial sums of this
// iteration (s1: p.q, s2: r.r or the true residual or b.b).
__device__ void commit(WideState &W, const WideSlot &S, double s1, double s2)
{
    if (W.mode == kWideRun) {
        W.spmv += 1;
        if (!__builtin_isfinite(s1)) {
            W.status = kSlotNonfinite;
            W.mode = kWideDone;
        } else if (!(s1 > 0.0)) {
            W.status = kSlotBreakdown;
            W.mode = kWideDone;
        } else {
            W.iters += 1;
            W.rr = s2;
            if (!__builtin_isfinite(s2)) {
                W.status = kSlotNonfinite;
                W.mode = kWideDone;
            } else if (s2 <= S.tol2 * W.bb) {
                W.mode = kWideCheck;
            } else {
                W.rho = s2;
                if (W.iters >= S.maxit) {
                    W.status = kSlotMaxit;
                    W.mode = kWideDone;
                }
            }
        }
    } else if (W.mode == kWideCheck) {
        W.spmv += 1;
        W.rr = s2;
        if (s2 <= S.tol2 * W.bb) {
            W.status = kSlotConverged;
            W.relres_true = sqrt(s2 / W.bb);
            W.mode = kWideDone;
        } else if (!__builtin_isfinite(s2)) {
            W.status = kSlotNonfinite;
            W.mode = kWideDone;
        } else {
            W.rho = s2;
            W.mode = kWideRun;
            if (W.iters >= S.maxit) {
                W.status = kSlotMaxit;
                W.mode = kWideDone;
            }
        }
    } else {  // init
        W.bb = s2;
        W.rho = s2;
        W.rr = s2;
        if (!__builtin_isfinite(s2)) {
            W.status = kSlotNonfinite;
            W.mode = kWideDone;
        } else if (s2 == 0.0) {
            W.status = kSlotConverged;
            W.relres_true = 0.0;
            W.mode = kWideDone;
        } else {
            W.mode = kWideRun;
        }
    }
    if (W.mode == kWideDone && W.status != kSlotConverged) W.relres_true = W.bb > 0 ? sqrt(W.rr / W.bb) : 0.0;
}

// Direction phase and commit. The first virtual block of every system also
// forms the two sums of the iteration (the same partials in the same order
// as every other block) and writes the system's updated state to st_next,
// while all blocks read this iteration's state from st (the two buffers
// alternate from one iteration to the next).
__global__ __launch_bounds__(kWideThreads) void wide_c_kernel(const WideSlot *__restrict__ slots,
                                                              const WideState *__restrict__ st,
                                                              WideState *__restrict__ st_next,
                                                              const WideMap *__restrict__ map,
                                                              const int32_t *__restrict__ vb_slot,
                                                              const int32_t *__restrict__ vb_local)
{
    __shared__ double s_red[kWideWaves];
    const int32_t total = map->total_vb;
    for (int32_t v = blockIdx.x; v < total; v += gridDim.x) {
        const int32_t s = vb_slot[v], lv = vb_local[v];
        const WideState W0 = st[s];
        const bool lead = lv == 0;  // this block commits the system's state
        if (W0.mode == kWideDone) {
            if (lead && threadIdx.x == 0) st_next[s] = W0;
            continue;
        }
        const WideSlot S = slots[s];
        const int32_t r0 = lv * kWideRows, r1 = min(S.n, r0 + kWideRows);
        const double bb = W0.bb;
        double s1 = 0.0, s2 = 0.0;
        if (W0.mode == kWideRun) {
            s1 = wide_part_sum(S.part_a, S.ntiles, s_red);  // p.q
            s2 = wide_part_sum(S.part, S.nvb, s_red);       // r.r
            const bool step = s1 > 0.0 && __builtin_isfinite(s1) && __builtin_isfinite(s2) && !(s2 <= S.tol2 * bb);
            if (step) {  // otherwise the solve stops or checks next
                const double beta = s2 / W0.rho;
                for (int32_t i = r0 + threadIdx.x; i < r1; i += kWideThreads) S.p[i] = S.r[i] + beta * S.p[i];
            }
        } else if (W0.mode == kWideCheck) {
            s2 = wide_part_sum(S.part, S.nvb, s_red);  // true r.r
            if (!(s2 <= S.tol2 * bb))
                for (int32_t i = r0 + threadIdx.x; i < r1; i += kWideThreads) S.p[i] = S.r[i];  // restart
        } else {
            if (lead) s2 = wide_part_sum(S.part, S.nvb, s_red);  // b.b
            for (int32_t i = r0 + threadIdx.x; i < r1; i += kWideThreads) S.p[i] = S.r[i];
        }
        if (lead && threadIdx.x == 0) {
            WideState W = W0;
            commit(W, S, s1, s2);
            st_next[s] = W;
        }
    }
}

spx_status wide_iteration_launch(const WideSlot *slots, const WideState *st, WideState *st_next,
                                 const WideMap *map, const int32_t *vb_slot, const int32_t *vb_local,
                                 const int32_t *ta_slot, const int32_t *ta_local, int grid, hipStream_t stream)
{
    wide_a_kernel<<<grid, kCsrThreads, 0, stream>>>(slots, st, map, ta_slot, ta_local);
    SPX_LAUNCHED();
    wide_b_kernel<<<grid, kWideThreads, 0, stream>>>(slots, st, map, vb_slot, vb_local);
    SPX_LAUNCHED();
    wide_c_kernel<<<grid, kWideThreads, 0, stream>>>(slots, st, st_next, map, vb_slot, vb_local);
    SPX_LAUNCHED();
    return SPX_OK;
}

}  // namespace spx
