// small_cg.hip -- CG for small systems on one work-group (the latency path).
//
// A system of a few thousand rows moves well under a megabyte per CG
// iteration, so the five launches per iteration of the general driver are
// pure launch latency. Here one work-group of 1024 threads runs the whole
// solve in a single launch: thread t owns rows t, t + 1024, ... (up to kR = 4
// of them: four rows' state fits the 128 registers a thread of a 1024-thread
// group may hold) and keeps their row bounds, x, r and the Jacobi scaling in
// registers; the search direction p lives in LDS, where the product
// gathers it; the matrix entries are read from global memory (L2-resident
// at these sizes). Every dot product is a fixed-order work-group reduction
// (wavefront DPP sums, then the wavefront sums in order), so results are
// bitwise reproducible. The recurrences, the stopping test and the
// true-residual confirmation with restart are those of the general CG
// driver (Hestenes & Stiefel; the preconditioned form of Barrett et al.,
// "Templates", 1994).
#include "solver_common.hpp"
#include "small_cg.hpp"

namespace spx {

constexpr int kMaxWaves = 1024 / kWave;

// Work-group sums of NV values, result in every thread: wavefront sums, then
// lane i of every wavefront reads wavefront i's sum and a 16-lane butterfly
// adds them (the same fixed order in every wavefront). `par` alternates the
// LDS buffer so one barrier per reduction suffices.
template <int NV, int kWaves>
__device__ __forceinline__ void small_sum(double (&v)[NV], double (*s_red)[4 * kMaxWaves], int &par)
{
    const int w = threadIdx.x / kWave, l = lane_id();
#pragma unroll
    for (int j = 0; j < NV; ++j) v[j] = wave_sum(v[j]);
    if (l == 0)
#pragma unroll
        for (int j = 0; j < NV; ++j) s_red[par][j * kWaves + w] = v[j];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        const double t = l < kWaves ? s_red[par][j * kWaves + l] : 0.0;
        v[j] = readlane(subwave_sum<kWaves>(t), 0);
    }
    par ^= 1;
}

// sum_j val[j] * v[col[j]] over row bounds [a, b), v in LDS.
__device__ __forceinline__ double small_row(int32_t a, int32_t b, const int32_t *__restrict__ col,
                                            const double *__restrict__ val, const double *v)
{
    double s = 0.0;
#pragma unroll 2
    for (int32_t j = a; j < b; ++j) s += val[j] * v[col[j]];
    return s;
}

// kThreads threads, kR rows per thread; kL > 0: every row has at most kL
// entries and each thread keeps its rows' columns and values in registers
// for the whole solve (the product then only gathers p from LDS); kL = 0:
// the entries are read from global memory at every product.
template <int kThreads, int kR, int kL>
__global__ __launch_bounds__(kThreads) void small_cg_kernel(int32_t n, const int32_t *__restrict__ rowptr,
                                                                const int32_t *__restrict__ col,
                                                                const double *__restrict__ val,
                                                                const double *__restrict__ b, double *__restrict__ x,
                                                                const double *__restrict__ dinv, int x0_zero,
                                                                KState *st)
{
    constexpr int kWaves = kThreads / kWave;
    __shared__ double s_v[kThreads * kR];  // p (or x while the true residual is formed)
    __shared__ double s_red[2][4 * kMaxWaves];
    int par = 0;
    const int tid = threadIdx.x;
    const double tol2 = st->tol2;
    const int32_t maxit = st->maxit;
    int32_t ra[kR], rb[kR];
    double xr[kR], rv[kR], dv[kR], qv[kR];
#pragma unroll
    for (int k = 0; k < kR; ++k) {
        const int i = tid + k * kThreads;
        const bool in = i < n;
        ra[k] = in ? rowptr[i] : 0;
        rb[k] = in ? rowptr[i + 1] : 0;
        xr[k] = (in && !x0_zero) ? x[i] : 0.0;
        dv[k] = in ? (dinv ? dinv[i] : 1.0) : 0.0;
        if (!x0_zero) s_v[i] = xr[k];
    }
    int32_t cc[kL > 0 ? kR : 1][kL > 0 ? kL : 1];
    double vv[kL > 0 ? kR : 1][kL > 0 ? kL : 1];
    int32_t ln[kL > 0 ? kR : 1];  // row lengths (the cached form needs nothing else)
    if constexpr (kL > 0) {
        // the row-length hint is only a hint: a longer row sends the solve back
        // to the host, which runs the streaming form instead
        bool long_row = false;
#pragma unroll
        for (int k = 0; k < kR; ++k) long_row |= rb[k] - ra[k] > kL;
        if (__syncthreads_or(long_row)) {
            if (tid == 0) st->flag = kLongRow;
            return;
        }
#pragma unroll
        for (int k = 0; k < kR; ++k) {
            ln[k] = rb[k] - ra[k];
#pragma unroll
            for (int e = 0; e < kL; ++e) {
                const bool in = e < ln[k];
                cc[k][e] = in ? col[ra[k] + e] : 0;
                vv[k][e] = in ? val[ra[k] + e] : 0.0;
            }
        }
    }
    // product of row k with v (in LDS), entries in order
    auto row = [&](int k, const double *v) -> double {
        if constexpr (kL > 0) {
            double t = 0.0;
#pragma unroll
            for (int e = 0; e < kL; ++e)
                if (e < ln[k]) t += vv[k][e] * v[cc[k][e]];
            return t;
        } else {
            return small_row(ra[k], rb[k], col, val, v);
        }
    };
    if (!x0_zero) __syncthreads();
    // r = b - A x, b.b, r.r
    double s3[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < kR; ++k) {
        const int i = tid + k * kThreads;
        const double bi = i < n ? b[i] : 0.0;
        rv[k] = x0_zero ? bi : bi - row(k, s_v);
        s3[0] += bi * bi;
    }
    if (!x0_zero) __syncthreads();  // every gather of x is done before p overwrites it
    // p = z = M^{-1} r, rho = r.z
#pragma unroll
    for (int k = 0; k < kR; ++k) {
        const double z = rv[k] * dv[k];
        s_v[tid + k * kThreads] = z;
        s3[1] += rv[k] * z;
        s3[2] += rv[k] * rv[k];
    }
    small_sum<3, kWaves>(s3, s_red, par);  // its barrier also publishes p
    const double bb = s3[0];
    double rho = s3[1], rr = s3[2], true2 = -1.0;
    int32_t iters = 0, spmv = x0_zero ? 0 : 1, flag = kRunning;
    if (!__builtin_isfinite(bb) || !__builtin_isfinite(rr)) flag = kNonfinite;
    else if (bb == 0.0) flag = kZeroRhs;
    while (flag == kRunning) {
        if (rr <= tol2 * bb) {
            // confirm with the true residual b - A x (x staged in LDS)
            __syncthreads();  // gathers of p are done
#pragma unroll
            for (int k = 0; k < kR; ++k) s_v[tid + k * kThreads] = xr[k];
            __syncthreads();
            double t[1] = {0.0};
#pragma unroll
            for (int k = 0; k < kR; ++k) {
                const int i = tid + k * kThreads;
                const double bi = i < n ? b[i] : 0.0;
                rv[k] = bi - row(k, s_v);
                t[0] += rv[k] * rv[k];
            }
            spmv += 1;
            small_sum<1, kWaves>(t, s_red, par);  // its barrier: every gather of x is done
            true2 = t[0];
            if (!__builtin_isfinite(true2)) {
                flag = kNonfinite;
                break;
            }
            if (true2 <= tol2 * bb) {
                flag = kConverged;
                break;
            }
            if (iters >= maxit) {
                flag = kMaxit;
                break;
            }
            // restart the recurrences from the true residual
            double t2[2] = {0.0, 0.0};
#pragma unroll
            for (int k = 0; k < kR; ++k) {
                const double z = rv[k] * dv[k];
                s_v[tid + k * kThreads] = z;
                t2[0] += rv[k] * z;
                t2[1] += rv[k] * rv[k];
            }
            small_sum<2, kWaves>(t2, s_red, par);
            rho = t2[0];
            rr = t2[1];
            true2 = -1.0;
            continue;
        }
        if (iters >= maxit) {
            flag = kMaxit;
            break;
        }
        // q = A p and p.q
        double t[1] = {0.0};
#pragma unroll
        for (int k = 0; k < kR; ++k) {
            qv[k] = row(k, s_v);
            t[0] += s_v[tid + k * kThreads] * qv[k];
        }
        spmv += 1;
        small_sum<1, kWaves>(t, s_red, par);
        const double pq = t[0];
        if (!__builtin_isfinite(pq)) {
            flag = kNonfinite;
            break;
        }
        if (pq <= 0.0) {
            flag = kBreakdown;
            break;
        }
        const double alpha = rho / pq;
        double t2[2] = {0.0, 0.0};
#pragma unroll
        for (int k = 0; k < kR; ++k) {
            xr[k] += alpha * s_v[tid + k * kThreads];
            rv[k] = rv[k] - alpha * qv[k];
            const double z = rv[k] * dv[k];
            t2[0] += rv[k] * z;
            t2[1] += rv[k] * rv[k];
        }
        small_sum<2, kWaves>(t2, s_red, par);  // its barrier: every gather of p is done
        iters += 1;
        rr = t2[1];
        if (!__builtin_isfinite(rr) || !__builtin_isfinite(t2[0])) {
            flag = kNonfinite;
            break;
        }
        if (rr <= tol2 * bb) continue;  // confirmed at the top of the loop
        const double beta = t2[0] / rho;
        rho = t2[0];
#pragma unroll
        for (int k = 0; k < kR; ++k) {
            const int i = tid + k * kThreads;
            s_v[i] = rv[k] * dv[k] + beta * s_v[i];  // only this thread touches its own rows here
        }
        __syncthreads();  // p is published before the next product
    }
    const bool zero = flag == kZeroRhs;
#pragma unroll
    for (int k = 0; k < kR; ++k) {
        const int i = tid + k * kThreads;
        if (i < n) x[i] = zero ? 0.0 : xr[k];
    }
    if (tid == 0) {
        st->bb = bb;
        st->rr = rr;
        st->tmp[0] = zero ? 0.0 : true2;
        st->iters = iters;
        st->spmv_count = spmv;
        st->flag = flag;
    }
}

spx_status small_cg_launch(const spx_matrix &A, const double *b, double *x, const double *dinv, int x0_zero,
                           bool cached, KState *st, hipStream_t stream)
{
    const double *val = static_cast<const double *>(A.vals);
    if (cached)  // rows of at most 5 entries: 512 threads, 8 rows each, matrix in registers
        small_cg_kernel<512, 8, 5><<<1, 512, 0, stream>>>(A.nrows, A.rowptr, A.colidx, val, b, x, dinv, x0_zero, st);
    else
        small_cg_kernel<kSmallThreads, kSmallMaxRows / kSmallThreads, 0><<<1, kSmallThreads, 0, stream>>>(
            A.nrows, A.rowptr, A.colidx, val, b, x, dinv, x0_zero, st);
    SPX_LAUNCHED();
    return SPX_OK;
}

}  // namespace spx
