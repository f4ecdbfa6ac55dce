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
// Nonsymmetric systems run unpreconditioned BiCGSTAB (van der Vorst 1992, in
// the order of the one-work-group kernel) on the same two kernels, one step
// as three product + vector pairs (bphase 0: v = A p with r_hat.v partials,
// then alpha and s = r - alpha v with s.s partials; bphase 1: t = A s with
// t.s and t.t partials, then omega, x and r = s - omega t with r.r and
// r_hat.r partials; bphase 2: no product, then beta and the new p). A small
// ||s|| or ||r|| is confirmed with the true residual, whose sum is read by
// one more pair (bphase 3), which also starts the recurrences after init.
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
        // one instantiation of the tile kernel for every case (its LDS
        // staging sets the occupancy); the second partial (y.y) is used by
        // BiCGSTAB's t = A s only
        const double *src = mode == kWideRun ? S.r : S.x;
        const double *dw = src;
        double *y = S.w;
        if (S.solver == kSlotBicgstab && mode == kWideRun) {
            const int32_t bp = st[s].bphase;
            if (bp == 0) {  // v = A p, r_hat.v
                src = S.p;
                dw = S.rh;
            } else if (bp == 1) {  // t = A s (s is held in r), t.s and t.t
                y = S.t;
            } else {
                continue;  // no product in this pair
            }
        }
        csr_tile<double, double, 2, kCsrThreads, kCsrTile, 1, kCsrLateGather>(
            k, S.n, S.nnz, S.ntiles, S.rowptr, S.col, S.val, src, y, 1.0, 0.0, dw, S.part_a, S.csr_part);
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

// BiCGSTAB's vector phase on one virtual block of one system; the lead block
// commits the state to *next. part_in / part_out: two rows of nvb partials.
__device__ void bicgstab_vector_phase(const WideSlot &S, const WideState &W0, bool lead, int32_t lv,
                                      const double *part_in, double *part_out, WideState *next, double *s_red)
{
    const int32_t r0 = lv * kWideRows, r1 = min(S.n, r0 + kWideRows);
    WideState W = W0;
    int nw = 0;  // partial rows this block stores into part_out
    double t0 = 0.0, t1 = 0.0;
    auto done = [&](int32_t status) {
        W.status = status;
        W.mode = kWideDone;
        if (status != kSlotConverged) W.relres_true = W.bb > 0.0 ? sqrt(W.rr / W.bb) : 0.0;
    };
    if (W0.mode == kWideInit) {  // x = 0 (written at admission): r = r_hat = b
        for (int32_t i = r0 + threadIdx.x; i < r1; i += kWideThreads) {
            const double bi = S.b[i];
            S.r[i] = bi;
            S.rh[i] = bi;
            t0 += bi * bi;
        }
        nw = 1;
        W.mode = kWideRun;
        W.bphase = 3;
        W.truer = 2;
    } else if (W0.mode == kWideCheck) {  // r = b - A x (A x in w), r_hat = r
        for (int32_t i = r0 + threadIdx.x; i < r1; i += kWideThreads) {
            const double ri = S.b[i] - S.w[i];
            S.r[i] = ri;
            S.rh[i] = ri;
            t0 += ri * ri;
        }
        nw = 1;
        W.spmv += 1;
        W.mode = kWideRun;
        W.bphase = 3;
        W.truer = 1;
    } else if (W0.bphase == 3) {  // a true residual's r.r: converged, or (re)start
        const double tr = wide_part_sum(part_in, S.nvb, s_red);
        if (W0.truer == 2) W.bb = tr;
        W.rr = tr;
        if (!__builtin_isfinite(tr)) {
            done(kSlotNonfinite);
        } else if (tr <= S.tol2 * W.bb) {  // also b = 0
            W.relres_true = W.bb > 0.0 ? sqrt(tr / W.bb) : 0.0;
            done(kSlotConverged);
        } else {
            for (int32_t i = r0 + threadIdx.x; i < r1; i += kWideThreads) S.p[i] = S.r[i];
            W.rho = tr;  // r_hat = r
            W.rho0 = W.alpha = W.omega = 1.0;
            W.truer = 0;
            W.bphase = 0;
        }
    } else if (W0.bphase == 0) {  // v = A p is in w: alpha, s = r - alpha v
        const double rhv = wide_part_sum(S.part_a, S.ntiles, s_red);
        if (W0.iters >= S.maxit) {
            done(kSlotMaxit);
        } else {
            W.iters += 1;
            W.spmv += 1;
            if (!__builtin_isfinite(rhv)) {
                done(kSlotNonfinite);
            } else if (rhv == 0.0) {
                done(kSlotBreakdown);
            } else {
                const double alpha = W0.rho / rhv;
                for (int32_t i = r0 + threadIdx.x; i < r1; i += kWideThreads) {
                    const double si = S.r[i] - alpha * S.w[i];
                    S.r[i] = si;
                    t0 += si * si;
                }
                nw = 1;
                W.alpha = alpha;
                W.bphase = 1;
            }
        }
    } else if (W0.bphase == 1) {  // t = A s is in t: omega, x, r = s - omega t
        const double ss = wide_part_sum(part_in, S.nvb, s_red);
        const double ts = wide_part_sum(S.part_a, S.ntiles, s_red);
        const double tt = wide_part_sum(S.part_a + S.ntiles, S.ntiles, s_red);
        W.rr = ss;
        const double alpha = W0.alpha;
        if (ss <= S.tol2 * W0.bb) {  // ||s|| small: x += alpha p, then confirm
            for (int32_t i = r0 + threadIdx.x; i < r1; i += kWideThreads) S.x[i] += alpha * S.p[i];
            W.mode = kWideCheck;
        } else {
            W.spmv += 1;  // t = A s
            if (!__builtin_isfinite(tt) || !__builtin_isfinite(ss)) {
                done(kSlotNonfinite);
            } else if (tt == 0.0) {
                done(kSlotBreakdown);
            } else {
                const double omega = ts / tt;
                for (int32_t i = r0 + threadIdx.x; i < r1; i += kWideThreads) {
                    const double si = S.r[i];
                    S.x[i] += alpha * S.p[i] + omega * si;
                    const double ri = si - omega * S.t[i];
                    S.r[i] = ri;
                    t0 += ri * ri;
                    t1 += S.rh[i] * ri;
                }
                nw = 2;
                W.omega = omega;
                W.bphase = 2;
            }
        }
    } else {  // bphase 2: r.r and r_hat.r: confirm, or beta and p
        const double rr = wide_part_sum(part_in, S.nvb, s_red);
        const double rho = wide_part_sum(part_in + S.nvb, S.nvb, s_red);
        W.rr = rr;
        if (!__builtin_isfinite(rr)) {
            done(kSlotNonfinite);
        } else if (rr <= S.tol2 * W0.bb) {
            W.mode = kWideCheck;
        } else if (W0.omega == 0.0 || rho == 0.0) {
            done(kSlotBreakdown);
        } else if (!__builtin_isfinite(rho)) {
            done(kSlotNonfinite);
        } else {
            const double beta = (rho / W0.rho) * (W0.alpha / W0.omega);
            const double omega = W0.omega;
            for (int32_t i = r0 + threadIdx.x; i < r1; i += kWideThreads)
                S.p[i] = S.r[i] + beta * (S.p[i] - omega * S.w[i]);
            W.rho0 = W0.rho;
            W.rho = rho;
            W.bphase = 0;
        }
    }
    if (nw > 0) {
        t0 = wide_wg_sum(t0, s_red);
        if (nw > 1) t1 = wide_wg_sum(t1, s_red);
        if (threadIdx.x == 0) {
            part_out[lv] = t0;
            if (nw > 1) part_out[S.nvb + lv] = t1;
        }
        W.phase = W0.phase ^ 1;
    }
    if (lead && threadIdx.x == 0) *next = W;
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
        const double *part_in = S.part + (W0.phase ? 2 * S.nvb : 0);
        double *part_out = S.part + (W0.phase ? 0 : 2 * S.nvb);
        if (S.solver == kSlotBicgstab) {
            bicgstab_vector_phase(S, W0, lead, lv, part_in, part_out, st_next + s, s_red);
            continue;
        }
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
