// batch_wide.hip -- CG on many large systems at once, several work-groups per
// system, no synchronisation between work-groups inside a launch.
//
// Unpreconditioned CG from x0 = 0 in the single-reduction form of Chronopoulos
// and Gear (1989): besides r and p the recurrences carry w = A r and
// s = A p, so both inner products of a step (r.r and r.w) come from one
// pass and a step needs one grid-wide synchronisation fewer than the
// Hestenes-Stiefel order (the same Krylov iterates in exact arithmetic).
// One iteration is two grid-wide phases over every listed system (a launch
// boundary is the only global synchronisation):
//   A  w = A r (or w = A x in the true-residual mode), partial sums of r.w:
//      the load-balanced CSR tile kernel over every listed system's tiles;
//   V  gamma = r.r and delta = r.w from the partials; beta = gamma / gamma_old,
//      alpha = gamma / (delta - beta gamma / alpha_old) (beta = 0 and
//      alpha = gamma / delta when the recurrences start); p = r + beta p,
//      s = w + beta s, x += alpha p, r -= alpha s, partial sums of the new
//      r.r (true-residual mode: r = b - w; init: r = b). The first block of
//      each system commits its scalar state into the other of two state
//      buffers.
// The step is taken only while r.r is above the tolerance; below it the
// system checks its true residual (one product of x) and either finishes or
// restarts the recurrences from it.
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
// kernel runs with its dot epilogue in both modes (w.r in the run mode; the
// true-residual mode multiplies x and ignores the partial).
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
        const double *src = mode == kWideRun ? S.r : S.x;
        csr_tile<double, double, 1, kCsrThreads, kCsrTile, 1, kCsrLateGather>(
            k, S.n, S.nnz, S.ntiles, S.rowptr, S.col, S.val, src, S.w, 1.0, 0.0, src, S.part_a, S.csr_part);
    }
}

enum WideStep : int32_t { kStepTake = 0, kStepCheck = 1, kStepDone = 2 };

// The run mode's decision, taken alike by every block of the system from the
// two sums gamma = r.r and delta = r.w. On kStepTake, alpha and beta are set;
// on kStepDone, W holds the final status.
__device__ int32_t run_decision(WideState &W, const WideSlot &S, double gamma, double delta, double &alpha,
                                double &beta)
{
    W.spmv += 1;
    const double bb = W.truer == 2 ? gamma : W.bb;  // r = b: gamma is b.b
    W.bb = bb;
    W.rr = gamma;
    if (!__builtin_isfinite(gamma)) {
        W.status = kSlotNonfinite;
        return kStepDone;
    }
    if (gamma <= S.tol2 * bb) {  // also b = 0 (gamma = bb = 0)
        if (W.truer == 0) return kStepCheck;
        W.status = kSlotConverged;
        W.relres_true = bb > 0.0 ? sqrt(gamma / bb) : 0.0;
        return kStepDone;
    }
    if (W.iters >= S.maxit) {
        W.status = kSlotMaxit;
        return kStepDone;
    }
    beta = W.restart ? 0.0 : gamma / W.rho;
    const double den = W.restart ? delta : delta - beta * gamma / W.alpha;
    if (!__builtin_isfinite(delta) || !__builtin_isfinite(den)) {
        W.status = kSlotNonfinite;
        return kStepDone;
    }
    if (!(den > 0.0)) {  // p.A p <= 0: A is not positive definite along p
        W.status = kSlotBreakdown;
        return kStepDone;
    }
    alpha = gamma / den;
    return kStepTake;
}

// Vector phase and commit. Every block reads this iteration's state from st;
// the first virtual block of each system writes the updated state to
// st_next (the two buffers alternate from one iteration to the next).
__global__ __launch_bounds__(kWideThreads) void wide_v_kernel(const WideSlot *__restrict__ slots,
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
        const double *part_in = S.part + (W0.phase ? S.nvb : 0);
        double *part_out = S.part + (W0.phase ? 0 : S.nvb);
        WideState W = W0;
        bool wrote = false;  // this block stored a partial into part_out
        double t = 0.0;
        if (W0.mode == kWideRun) {
            const double gamma = wide_part_sum(part_in, S.nvb, s_red);
            const double delta = wide_part_sum(S.part_a, S.ntiles, s_red);
            double alpha = 0.0, beta = 0.0;
            const int32_t step = run_decision(W, S, gamma, delta, alpha, beta);
            if (step == kStepTake) {
                if (W0.restart) {
                    for (int32_t i = r0 + threadIdx.x; i < r1; i += kWideThreads) {
                        const double pi = S.r[i], si = S.w[i];
                        S.p[i] = pi;
                        S.s[i] = si;
                        S.x[i] += alpha * pi;
                        const double ri = S.r[i] - alpha * si;
                        S.r[i] = ri;
                        t += ri * ri;
                    }
                } else {
                    for (int32_t i = r0 + threadIdx.x; i < r1; i += kWideThreads) {
                        const double pi = S.r[i] + beta * S.p[i];
                        const double si = S.w[i] + beta * S.s[i];
                        S.p[i] = pi;
                        S.s[i] = si;
                        S.x[i] += alpha * pi;
                        const double ri = S.r[i] - alpha * si;
                        S.r[i] = ri;
                        t += ri * ri;
                    }
                }
                wrote = true;
                W.iters += 1;
                W.rho = gamma;
                W.alpha = alpha;
                W.restart = 0;
                W.truer = 0;
            } else if (step == kStepCheck) {
                W.mode = kWideCheck;
            } else {
                W.mode = kWideDone;
                if (W.status != kSlotConverged) W.relres_true = W.bb > 0.0 ? sqrt(W.rr / W.bb) : 0.0;
            }
        } else if (W0.mode == kWideCheck) {
            for (int32_t i = r0 + threadIdx.x; i < r1; i += kWideThreads) {
                const double ri = S.b[i] - S.w[i];
                S.r[i] = ri;
                t += ri * ri;
            }
            wrote = true;
            W.spmv += 1;
            W.mode = kWideRun;
            W.restart = 1;
            W.truer = 1;
        } else {  // init: x = 0 was written at admission
            for (int32_t i = r0 + threadIdx.x; i < r1; i += kWideThreads) {
                const double bi = S.b[i];
                S.r[i] = bi;
                t += bi * bi;
            }
            wrote = true;
            W.mode = kWideRun;
            W.restart = 1;
            W.truer = 2;
        }
        if (wrote) {
            t = wide_wg_sum(t, s_red);
            if (threadIdx.x == 0) part_out[lv] = t;
            W.phase = W0.phase ^ 1;
        }
        if (lead && threadIdx.x == 0) st_next[s] = W;
    }
}

spx_status wide_iteration_launch(const WideSlot *slots, const WideState *st, WideState *st_next,
                                 const WideMap *map, const int32_t *vb_slot, const int32_t *vb_local,
                                 const int32_t *ta_slot, const int32_t *ta_local, int grid, hipStream_t stream)
{
    wide_a_kernel<<<grid, kCsrThreads, 0, stream>>>(slots, st, map, ta_slot, ta_local);
    SPX_LAUNCHED();
    wide_v_kernel<<<grid, kWideThreads, 0, stream>>>(slots, st, st_next, map, vb_slot, vb_local);
    SPX_LAUNCHED();
    return SPX_OK;
}

}  // namespace spx
