// krylov.hpp -- device-resident state and deterministic reductions of the
// Krylov solvers.
//
// Every iteration's scalars (rho, alpha, beta, omega, ...) live in a KState
// in device memory, so an iteration is a fixed sequence of kernel launches
// with no host round trip and can be captured in a hipGraph. Reductions are
// two-stage and deterministic: each work-group writes a partial to a fixed
// slot; a one-work-group finish kernel sums the partials in a fixed order and
// updates the scalars (one "finish" op per reduction). A flag in the state
// stops every later kernel of a captured block of iterations as soon as the
// solve has converged or failed.
#pragma once

#include "common.hpp"
#include "wave.hpp"

namespace spx {

enum KFlag : int32_t {
    kRunning = 0,
    kConverged = 1,   // recursive residual below tolerance
    kBreakdown = 2,
    kNonfinite = 3,
    kMaxit = 4,
    kHalfConverged = 5,  // BiCGSTAB: ||s|| below tolerance
    kZeroRhs = 6,
    kCycleEnd = 7,       // GMRES: cycle finished (lucky breakdown or estimate converged)
    kLongRow = 8,        // one-group CG: a row is longer than the cached form holds
};

enum KOp : int32_t {
    kOpNone = 0,
    kOpCgInit,     // t0 = b.b, t1 = r.z, t2 = r.r
    kOpCgAlpha,    // t0 = p.q
    kOpCgRho,      // t0 = r.z, t1 = r.r
    kOpBiInit,     // t0 = b.b, t1 = r.r
    kOpBiAlpha,    // t0 = rhat.v
    kOpBiS,        // t0 = s.s
    kOpBiOmega,    // t0 = t.s, t1 = t.t
    kOpBiRho,      // t0 = r.r, t1 = rhat.r
    kOpNorm2,      // t0 = w.w -> tmp[0]
    kOpCgRestart,  // t0 = r.z: restart the recurrences from the current r
    kOpBiRestart,  // t0 = r.r: restart BiCGSTAB with rhat = r
    kOpBicgAlpha,  // t0 = pt.q (BiCG)
    kOpBicgRho,    // t0 = (M^-1 r).rt, t1 = r.r (BiCG)
    kOpPipeInit,   // t0 = b.b, t1 = r.r (pipelined CG start)
    kOpPipeRestart,  // t0 = r.r: restart pipelined CG from the current r
    kOpPipeStep,   // t0 = r.u, t1 = w.u, t2 = r.r (pipelined CG iteration)
};

constexpr int kMaxDots = 64;  // GMRES restart length + 2 (multi-dot width)

struct KState {
    double rho, rho0, alpha, beta, omega, bb, tol2, rr;
    double tmp[4];
    int32_t flag, iters, maxit, spmv_count;
    int32_t restart_j, jend, pad0, pad1;
    double dots[2 * kMaxDots];  // GMRES multi-dot results
};

__device__ __forceinline__ bool finite(double v) { return __builtin_isfinite(v); }

// Scalar update after a reduction, run by one thread of the finisher kernel.
__device__ inline void finish_op(int op, const double *t, KState *st)
{
    switch (op) {
    case kOpCgInit:
        st->bb = t[0];
        st->rho = t[1];
        st->rr = t[2];
        if (!finite(t[0]) || !finite(t[2])) st->flag = kNonfinite;
        else if (t[0] == 0.0) st->flag = kZeroRhs;
        else if (t[2] <= st->tol2 * t[0]) st->flag = kConverged;
        break;
    case kOpCgAlpha:
        if (!finite(t[0])) st->flag = kNonfinite;
        else if (t[0] <= 0.0) st->flag = kBreakdown;
        else st->alpha = st->rho / t[0];
        break;
    case kOpCgRho:
        st->iters += 1;
        st->spmv_count += 1;
        st->rr = t[1];
        if (!finite(t[1]) || !finite(t[0])) {
            st->flag = kNonfinite;
        } else if (t[1] <= st->tol2 * st->bb) {
            st->flag = kConverged;
        } else {
            st->beta = t[0] / st->rho;
            st->rho = t[0];
            if (st->iters >= st->maxit) st->flag = kMaxit;
        }
        break;
    case kOpBiInit:
        st->bb = t[0];
        st->rr = t[1];
        st->rho = t[1];  // rhat = r, so rhat.r = r.r
        st->beta = 0.0;  // first direction p = r (p = v = 0 initially)
        st->omega = 1.0;
        st->alpha = 1.0;
        if (!finite(t[0]) || !finite(t[1])) st->flag = kNonfinite;
        else if (t[0] == 0.0) st->flag = kZeroRhs;
        else if (t[1] <= st->tol2 * t[0]) st->flag = kConverged;
        else if (t[1] == 0.0) st->flag = kBreakdown;
        break;
    case kOpBiAlpha:
        st->spmv_count += 1;
        if (!finite(t[0])) st->flag = kNonfinite;
        else if (t[0] == 0.0) st->flag = kBreakdown;
        else st->alpha = st->rho / t[0];
        break;
    case kOpBiS:
        st->rr = t[0];
        if (!finite(t[0])) st->flag = kNonfinite;
        else if (t[0] <= st->tol2 * st->bb) {
            st->flag = kHalfConverged;
            st->iters += 1;
        }
        break;
    case kOpBiOmega:
        st->spmv_count += 1;
        if (!finite(t[1]) || !finite(t[0])) st->flag = kNonfinite;
        else if (t[1] == 0.0) st->flag = kBreakdown;
        else st->omega = t[0] / t[1];
        break;
    case kOpBiRho:
        st->iters += 1;
        st->rr = t[0];
        if (!finite(t[0]) || !finite(t[1])) {
            st->flag = kNonfinite;
        } else if (t[0] <= st->tol2 * st->bb) {
            st->flag = kConverged;
        } else if (st->omega == 0.0 || t[1] == 0.0) {
            st->flag = kBreakdown;
        } else {
            st->beta = (t[1] / st->rho) * (st->alpha / st->omega);
            st->rho0 = st->rho;
            st->rho = t[1];
            if (st->iters >= st->maxit) st->flag = kMaxit;
        }
        break;
    case kOpBicgAlpha:
        if (!finite(t[0])) st->flag = kNonfinite;
        else if (t[0] == 0.0 || st->rho == 0.0) st->flag = kBreakdown;
        else st->alpha = st->rho / t[0];
        break;
    case kOpBicgRho:
        st->iters += 1;
        st->spmv_count += 2;
        st->rr = t[1];
        if (!finite(t[1]) || !finite(t[0])) {
            st->flag = kNonfinite;
        } else if (t[1] <= st->tol2 * st->bb) {
            st->flag = kConverged;
        } else if (t[0] == 0.0) {
            st->flag = kBreakdown;
        } else {
            st->beta = t[0] / st->rho;
            st->rho = t[0];
            if (st->iters >= st->maxit) st->flag = kMaxit;
        }
        break;
    case kOpPipeInit:
        st->bb = t[0];
        st->rr = t[1];
        st->restart_j = 0;
        if (!finite(t[0]) || !finite(t[1])) st->flag = kNonfinite;
        else if (t[0] == 0.0) st->flag = kZeroRhs;
        else if (t[1] <= st->tol2 * t[0]) st->flag = kConverged;
        break;
    case kOpPipeRestart:
        st->rr = t[0];
        st->restart_j = 0;
        st->flag = finite(t[0]) ? kRunning : kNonfinite;
        break;
    case kOpPipeStep: {
        // t0 = gamma = r.u, t1 = delta = w.u of the current residual; the
        // previous gamma and alpha are in rho and alpha; restart_j counts
        // steps since the (re)start
        st->rr = t[2];
        if (!finite(t[0]) || !finite(t[1]) || !finite(t[2])) {
            st->flag = kNonfinite;
            break;
        }
        if (t[2] <= st->tol2 * st->bb) {
            st->flag = kConverged;
            break;
        }
        if (st->iters >= st->maxit) {
            st->flag = kMaxit;
            break;
        }
        double beta = 0.0, den = t[1];
        if (st->restart_j > 0) {
            beta = t[0] / st->rho;
            den = t[1] - beta * t[0] / st->alpha;
        }
        if (!finite(den)) st->flag = kNonfinite;
        else if (den <= 0.0) st->flag = kBreakdown;
        else {
            st->alpha = t[0] / den;
            st->beta = beta;
            st->rho = t[0];
            st->restart_j += 1;
            st->iters += 1;
            st->spmv_count += 1;
        }
        break;
    }
    case kOpNorm2:
        st->tmp[0] = t[0];
        break;
    case kOpBiRestart:
        st->rho = t[0];
        st->rr = t[0];
        st->beta = 0.0;
        st->omega = 1.0;
        st->alpha = 1.0;
        st->flag = !finite(t[0]) ? kNonfinite : (t[0] == 0.0 ? kBreakdown : kRunning);
        break;
    case kOpCgRestart:
        st->rho = t[0];
        st->flag = finite(t[0]) ? kRunning : kNonfinite;
        break;
    default: break;
    }
}

// Work-group sum of v (all threads must call; result valid in thread 0).
template <typename T, int kThreads>
__device__ __forceinline__ T block_sum(T v, T *s_red)
{
    v = wave_sum(v);
    if (lane_id() == 0) s_red[threadIdx.x / kWave] = v;
    __syncthreads();
    T t = T(0);
    if (threadIdx.x == 0)
        for (int w = 0; w < kThreads / kWave; ++w) t += s_red[w];
    __syncthreads();
    return t;
}

// Two-stage deterministic reduction, stage 1: each work-group stores its NV
// block sums (valid in thread 0) to partials[k * nparts + part]. No fence:
// stage 2 (finish_kernel) is a separate launch, and the kernel boundary
// makes the partials visible across XCDs. (A last-arriving-group finish
// would need a device-scope release per work-group, which on gfx950 is an
// L2 write-back plus invalidate for every group.)
template <typename T, int NV>
__device__ __forceinline__ void write_partials(const T (&v)[NV], T *__restrict__ partials, int64_t nparts,
                                               int64_t part)
{
    if (threadIdx.x == 0)
        for (int k = 0; k < NV; ++k) partials[k * nparts + part] = v[k];
}

// Ops that belong to an iteration are skipped once the solve has stopped
// (their producing kernels skipped too); setup ops always run.
__device__ __forceinline__ bool op_runs_when_stopped(int op)
{
    return op == kOpCgInit || op == kOpBiInit || op == kOpNorm2 || op == kOpCgRestart || op == kOpBiRestart ||
           op == kOpPipeInit || op == kOpPipeRestart;
}

constexpr int kFinThreads = 1024;

// Stage 2: one work-group sums nv (<= 4) rows of partials in a fixed order
// and applies the scalar update `op`. Thread t adds partials t, t + 1024, ...
// of every row in that order (four strides' loads in flight), then the
// wavefront sums and the wavefronts' sums in order.
template <typename T>
__global__ __launch_bounds__(kFinThreads) void finish_kernel(const T *__restrict__ partials, int64_t nparts, int nv,
                                                            KState *st, int op)
{
    if (st->flag != kRunning && !op_runs_when_stopped(op)) return;
    constexpr int kW = kFinThreads / kWave;
    __shared__ T s_red[4][kW];
    T acc[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll 4
    for (int64_t i = threadIdx.x; i < nparts; i += kFinThreads)
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (k < nv) acc[k] += partials[k * nparts + i];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const T v = wave_sum(acc[k]);
        if (lane_id() == 0) s_red[k][threadIdx.x / kWave] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot[4] = {0.0, 0.0, 0.0, 0.0};
        for (int k = 0; k < nv; ++k) {
            T t = T(0);
            for (int w = 0; w < kW; ++w) t += s_red[k][w];
            tot[k] = (double)t;
        }
        finish_op(op, tot, st);
    }
}

template <typename T>
inline spx_status launch_finish(const T *partials, int64_t nparts, int nv, KState *st, int op, hipStream_t stream)
{
    finish_kernel<T><<<1, kFinThreads, 0, stream>>>(partials, nparts, nv, st, op);
    return hipGetLastError() == hipSuccess ? SPX_OK : SPX_ERR_HIP;
}

}  // namespace spx
