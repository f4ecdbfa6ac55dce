// solve_cg.hip -- preconditioned conjugate gradients on the GPU.
//
// Textbook PCG (Hestenes & Stiefel 1952; the preconditioned form of Barrett
// et al., "Templates", 1994) with a scalar Jacobi preconditioner, the solver
// the paper benchmarks in Section 4. One iteration is five launches:
//   1. q = A p fused with the partial sums of p.q (CSR and SELL-P epilogue;
//      a separate dot kernel for the other formats);
//   2. a one-work-group finisher sums them in a fixed order: alpha = rho / p.q;
//   3. x += alpha p, r -= alpha q, z = D^{-1} r, partial sums of r.z and r.r;
//   4. a finisher forms beta and tests ||r|| <= tol ||b||;
//   5. p = z + beta p.
// Scalars never leave the device; a block of `check_every` iterations is
// captured once into a hipGraph and replayed, and the host reads the state
// only between replays. When the recursive residual passes, the true residual
// b - A x decides; a miss restarts the recurrences from it.
// Small float64 CSR systems (at most kSmallMaxRows rows, scalar Jacobi or no
// preconditioner) run the whole solve in one launch instead (small_cg.hip).
// Float64 throughout for spx_cg_solve; the same driver runs in float32
// (float32 or binary16-stored matrix values) as the inner solver of
// mixed-precision iterative refinement.
#include <type_traits>

#include "convert.hpp"
#include "small_cg.hpp"
#include "solver_common.hpp"
#include "solvers.hpp"

namespace spx {

template <typename X>
__global__ __launch_bounds__(kVecThreads) void cg_init_kernel(int64_t n, const X *__restrict__ b,
                                                             const X *__restrict__ q, const X *__restrict__ dinv,
                                                             X *__restrict__ r, X *__restrict__ z, X *__restrict__ p,
                                                             X *__restrict__ partials, KState *st)
{
    __shared__ X s_red[kVecThreads / kWave];
    const int64_t base = (int64_t)blockIdx.x * kVecChunk;
    X bb = X(0), rz = X(0), rr = X(0);
#pragma unroll
    for (int u = 0; u < kVecItems; ++u) {
        const int64_t i = base + threadIdx.x + u * kVecThreads;
        if (i < n) {
            const X bi = b[i];
            const X ri = q ? bi - q[i] : bi;
            const X zi = dinv ? ri * dinv[i] : ri;
            r[i] = ri;
            if (dinv) z[i] = zi;
            p[i] = zi;
            bb += bi * bi;
            rz += ri * zi;
            rr += ri * ri;
        }
    }
    X v[3] = {block_sum<X, kVecThreads>(bb, s_red), block_sum<X, kVecThreads>(rz, s_red),
              block_sum<X, kVecThreads>(rr, s_red)};
    write_partials<X, 3>(v, partials, gridDim.x, blockIdx.x);
}

// Each thread takes kVecItems consecutive entries: one 16/32-byte load per
// vector when kVec (all pointers suitably aligned), else element by element.
template <typename X, bool kVec>
__global__ __launch_bounds__(kVecThreads) void cg_update_kernel(int64_t n, X *__restrict__ x, const X *__restrict__ p,
                                                               const X *__restrict__ q, X *__restrict__ r,
                                                               X *__restrict__ z, const X *__restrict__ dinv,
                                                               X *__restrict__ partials, KState *st)
{
    if (st->flag != kRunning) return;
    __shared__ X s_red[kVecThreads / kWave];
    typedef X XV __attribute__((ext_vector_type(kVecItems)));
    const X a = (X)st->alpha;
    const int64_t i0 = ((int64_t)blockIdx.x * kVecThreads + threadIdx.x) * kVecItems;
    X rz = X(0), rr = X(0);
    if (kVec && i0 + kVecItems <= n) {
        XV xv = *reinterpret_cast<const XV *>(x + i0);
        const XV pv = *reinterpret_cast<const XV *>(p + i0);
        const XV qv = *reinterpret_cast<const XV *>(q + i0);
        XV rv = *reinterpret_cast<const XV *>(r + i0);
        XV zv;
        const XV dv = dinv ? *reinterpret_cast<const XV *>(dinv + i0) : XV{};
#pragma unroll
        for (int u = 0; u < kVecItems; ++u) {
            xv[u] += a * pv[u];
            rv[u] = rv[u] - a * qv[u];
            zv[u] = dinv ? rv[u] * dv[u] : rv[u];
            rz += rv[u] * zv[u];
            rr += rv[u] * rv[u];
        }
        *reinterpret_cast<XV *>(x + i0) = xv;
        *reinterpret_cast<XV *>(r + i0) = rv;
        if (dinv) *reinterpret_cast<XV *>(z + i0) = zv;
    } else {
        for (int64_t i = i0; i < i0 + kVecItems && i < n; ++i) {
            x[i] += a * p[i];
            const X ri = r[i] - a * q[i];
            r[i] = ri;
            const X zi = dinv ? ri * dinv[i] : ri;
            if (dinv) z[i] = zi;
            rz += ri * zi;
            rr += ri * ri;
        }
    }
    X v[2] = {block_sum<X, kVecThreads>(rz, s_red), block_sum<X, kVecThreads>(rr, s_red)};
    write_partials<X, 2>(v, partials, gridDim.x, blockIdx.x);
}

template <typename X, bool kVec>
__global__ __launch_bounds__(kVecThreads) void cg_p_kernel(int64_t n, const X *__restrict__ z, X *__restrict__ p,
                                                          const KState *st)
{
    if (st->flag != kRunning) return;
    typedef X XV __attribute__((ext_vector_type(kVecItems)));
    const X be = (X)st->beta;
    const int64_t i0 = ((int64_t)blockIdx.x * kVecThreads + threadIdx.x) * kVecItems;
    if (kVec && i0 + kVecItems <= n) {
        const XV zv = *reinterpret_cast<const XV *>(z + i0);
        XV pv = *reinterpret_cast<const XV *>(p + i0);
#pragma unroll
        for (int u = 0; u < kVecItems; ++u) pv[u] = zv[u] + be * pv[u];
        *reinterpret_cast<XV *>(p + i0) = pv;
    } else {
        for (int64_t i = i0; i < i0 + kVecItems && i < n; ++i) p[i] = z[i] + be * p[i];
    }
}

template <typename X>
__global__ __launch_bounds__(kVecThreads) void cg_restart_kernel(int64_t n, const X *__restrict__ r,
                                                                const X *__restrict__ dinv, X *__restrict__ z,
                                                                X *__restrict__ p, X *__restrict__ partials,
                                                                KState *st)
{
    __shared__ X s_red[kVecThreads / kWave];
    const int64_t base = (int64_t)blockIdx.x * kVecChunk;
    X rz = X(0);
#pragma unroll
    for (int u = 0; u < kVecItems; ++u) {
        const int64_t i = base + threadIdx.x + u * kVecThreads;
        if (i < n) {
            const X ri = r[i];
            const X zi = dinv ? ri * dinv[i] : ri;
            if (dinv) z[i] = zi;
            p[i] = zi;
            rz += ri * zi;
        }
    }
    X v[1] = {block_sum<X, kVecThreads>(rz, s_red)};
    write_partials<X, 1>(v, partials, gridDim.x, blockIdx.x);
}

template <typename X>
__global__ void zero_kernel(int64_t n, X *__restrict__ x)
{
    const int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x;
    if (i < n) x[i] = X(0);
}

template <typename V, typename X>
struct CgBufs {
    X *r, *z, *p, *q, *d, *dinv, *partials;
    double *inv;  // block-Jacobi inverse blocks
    KState *st;
    int32_t *part;
};

template <typename V, typename X>
static CgBufs<V, X> cg_carve(Carve &c, const spx_matrix &A, int precond)
{
    const int64_t n = A.nrows;
    CgBufs<V, X> w{};
    w.st = c.take<KState>(1);
    w.r = c.take<X>(n);
    w.p = c.take<X>(n);
    w.q = c.take<X>(n);
    w.z = precond ? c.take<X>(n) : w.r;
    w.d = precond == 1 ? c.take<X>(n) : nullptr;
    w.dinv = precond == 1 ? c.take<X>(n) : nullptr;
    w.inv = precond >= 2 ? c.take<double>(ceil_div(n, precond) * precond * precond) : nullptr;
    w.partials = c.take<X>(3 * partial_slots(A));
    w.part = (A.fmt == SPX_CSR && A.csr_part == nullptr) ? c.take<int32_t>(csr_partition_bytes(A.nnz) / 4) : nullptr;
    return w;
}

template <typename V, typename X>
size_t cg_workspace(const spx_matrix &A, int precond)
{
    Carve c(nullptr, 0);
    (void)cg_carve<V, X>(c, A, precond);
    return c.off + 256;
}

// The one-launch solve of a small float64 CSR system (small_cg.hip) and the
// same bookkeeping as the general driver.
static spx_status small_cg_finish(const spx_matrix &A, const double *b, double *x, const SolveSpec &sp,
                                  const CgBufs<double, double> &w, SolveEnv *env, spx_solve_info *info,
                                  hipStream_t user_stream)
{
    hipStream_t s = env->stream;
    const int64_t n = A.nrows;
    const bool cached = A.max_row_len > 0 && A.max_row_len <= kSmallCachedLen;
    SPX_CHECK(small_cg_launch(A, b, x, sp.precond ? w.dinv : nullptr, sp.x0_zero, cached, w.st, s));
    KState hs;
    SPX_CHECK(read_state(env, w.st, &hs));
    if (hs.flag == kLongRow) {  // the row-length hint was too small
        SPX_CHECK(state_set_flag(w.st, kRunning, s));
        SPX_CHECK(small_cg_launch(A, b, x, sp.precond ? w.dinv : nullptr, sp.x0_zero, false, w.st, s));
        SPX_CHECK(read_state(env, w.st, &hs));
    }
    double true2 = hs.tmp[0];
    if (true2 < 0.0 && hs.bb > 0.0) {  // stopped before a true residual was formed
        SPX_CHECK(spmv_dispatch(A, x, w.q, 1.0, 0.0, s));
        SPX_CHECK(residual_norm<double>(n, b, w.q, w.r, w.partials, w.st, s));
        KState h2;
        SPX_CHECK(read_state(env, w.st, &h2));
        true2 = h2.tmp[0];
    }
    spx_status status = status_of_flag(hs.flag);
    if (hs.flag == kMaxit) set_error("cg: no convergence in %d iterations", sp.maxit);
    else if (hs.flag == kBreakdown) set_error("cg: breakdown (p'Ap <= 0)");
    else if (hs.flag == kNonfinite) set_error("cg: non-finite residual");
    SPX_HIP(hipEventRecord(env->ev1, s));
    SPX_HIP(hipEventSynchronize(env->ev1));
    float ms = 0.f;
    SPX_HIP(hipEventElapsedTime(&ms, env->ev0, env->ev1));
    info->status = status;
    info->iters = hs.iters;
    info->spmv_count = hs.spmv_count;
    info->relres_recursive = hs.bb > 0 ? sqrt(hs.rr / hs.bb) : 0.0;
    info->relres_true = hs.bb > 0 ? sqrt(true2 / hs.bb) : 0.0;
    info->device_ms = ms;
    SPX_HIP(hipEventRecord(env->join, s));
    SPX_HIP(hipStreamWaitEvent(user_stream, env->join, 0));
    return status;
}

template <typename V, typename X>
spx_status cg_run(const spx_matrix &A_in, const X *b, X *x, const SolveSpec &sp, void *ws, size_t ws_bytes,
                  spx_solve_info *info, hipStream_t user_stream)
{
    SolveEnv *env = nullptr;
    SPX_CHECK(solve_env(&env));
    hipStream_t s = env->stream;
    const int64_t n = A_in.nrows;
    Carve c(ws, ws_bytes);
    CgBufs<V, X> w = cg_carve<V, X>(c, A_in, sp.precond);
    SPX_REQUIRE(c.fits(), SPX_ERR_ARG, "cg: workspace of %zu bytes is too small (need %zu)", ws_bytes,
                cg_workspace<V, X>(A_in, sp.precond));
    spx_matrix A = A_in;
    *info = spx_solve_info{};

    SPX_HIP(hipEventRecord(env->join, user_stream));
    SPX_HIP(hipStreamWaitEvent(s, env->join, 0));
    SPX_HIP(hipEventRecord(env->ev0, s));
    // small float64 CSR systems: the whole solve in one work-group, one launch
    const bool small = std::is_same<V, double>::value && std::is_same<X, double>::value && A.fmt == SPX_CSR &&
                       n <= kSmallMaxRows && sp.precond <= 1 && sp.confirm_true;
    if (w.part && !small) {
        SPX_CHECK(csr_partition_launch(A, w.part, s));
        A.csr_part = w.part;
    }
    SPX_CHECK(state_init(w.st, sp.tol, sp.maxit, s));
    KState hs;
    const int32_t bs = sp.precond >= 2 ? sp.precond : 0;  // block-Jacobi block size
    if (sp.precond) {
        if (bs) SPX_CHECK(bj_setup<V>(A, bs, w.inv, w.st, s));
        else SPX_CHECK((jacobi_setup<V, X>(A, w.d, w.dinv, w.st, s)));
        SPX_CHECK(read_state(env, w.st, &hs));
        if (hs.flag != kRunning) {
            set_error(bs ? "cg: singular or non-finite diagonal block" : "cg: zero, missing or non-finite diagonal entry");
            return SPX_ERR_ZERO_DIAG;
        }
    }
    if constexpr (std::is_same<V, double>::value && std::is_same<X, double>::value) {
        if (small) return small_cg_finish(A, b, x, sp, w, env, info, user_stream);
    }
    const unsigned gv = (unsigned)vec_blocks(n);
    if (sp.x0_zero) {
        zero_kernel<X><<<(unsigned)ceil_div(n, kVecThreads), kVecThreads, 0, s>>>(n, x);
        cg_init_kernel<X><<<gv, kVecThreads, 0, s>>>(n, b, nullptr, w.dinv, w.r, w.z, w.p, w.partials, w.st);
    } else {
        SPX_CHECK(spmv_dispatch(A, x, w.q, 1.0, 0.0, s));
        cg_init_kernel<X><<<gv, kVecThreads, 0, s>>>(n, b, w.q, w.dinv, w.r, w.z, w.p, w.partials, w.st);
    }
    SPX_LAUNCHED();
    // block Jacobi: z = M^{-1} r, p = z and the r.z partials (row 1 of the init sums)
    if (bs) SPX_CHECK(bj_apply<X>(n, bs, w.inv, w.r, w.z, w.p, w.partials, 1, w.st, false, s));
    SPX_CHECK(launch_finish<X>(w.partials, gv, 3, w.st, kOpCgInit, s));
    SPX_CHECK(read_state(env, w.st, &hs));

    GraphGuard graph;
    const int m = sp.check_every > 0 ? sp.check_every : 16;
    // vector loads need every vector aligned to kVecItems entries (x is the
    // caller's; the workspace pieces are 256-byte aligned)
    const bool vec = (reinterpret_cast<uintptr_t>(x) % (kVecItems * sizeof(X))) == 0;
    auto iterations = [&]() -> spx_status {
        for (int it = 0; it < m; ++it) {
            SPX_CHECK((spmv_dot<V, X>(A, w.p, w.q, w.p, w.partials, w.st, kOpCgAlpha, s)));
            if (vec) {
                cg_update_kernel<X, true><<<gv, kVecThreads, 0, s>>>(n, x, w.p, w.q, w.r, sp.precond ? w.z : nullptr,
                                                                    w.dinv, w.partials, w.st);
            } else {
                cg_update_kernel<X, false><<<gv, kVecThreads, 0, s>>>(n, x, w.p, w.q, w.r,
                                                                     sp.precond ? w.z : nullptr, w.dinv, w.partials,
                                                                     w.st);
            }
            // block Jacobi: z = M^{-1} r and the r.z partials replace row 0
            if (bs) SPX_CHECK(bj_apply<X>(n, bs, w.inv, w.r, w.z, nullptr, w.partials, 0, w.st, true, s));
            SPX_CHECK(launch_finish<X>(w.partials, gv, 2, w.st, kOpCgRho, s));
            cg_p_kernel<X, true><<<gv, kVecThreads, 0, s>>>(n, w.z, w.p, w.st);
            SPX_LAUNCHED();
        }
        return SPX_OK;
    };
    spx_status status = SPX_OK;
    bool have_true = false;
    double true2 = 0.0;
    while (true) {
        if (hs.flag == kZeroRhs) {
            zero_kernel<X><<<(unsigned)ceil_div(n, kVecThreads), kVecThreads, 0, s>>>(n, x);
            SPX_LAUNCHED();
            status = SPX_OK;
            have_true = true;
            true2 = 0.0;
            break;
        }
        if (hs.flag == kConverged) {
            if (!sp.confirm_true) {
                status = SPX_OK;
                break;
            }
            SPX_CHECK(spmv_dispatch(A, x, w.q, 1.0, 0.0, s));
            SPX_CHECK(residual_norm<X>(n, b, w.q, w.r, w.partials, w.st, s));
            SPX_CHECK(read_state(env, w.st, &hs));
            have_true = true;
            true2 = hs.tmp[0];
            if (true2 <= hs.tol2 * hs.bb) {
                status = SPX_OK;
                break;
            }
            if (hs.iters >= sp.maxit) {
                status = SPX_ERR_NOT_CONVERGED;
                break;
            }
            // restart the recurrences from the true residual (already in r)
            cg_restart_kernel<X><<<gv, kVecThreads, 0, s>>>(n, w.r, w.dinv, w.z, w.p, w.partials, w.st);
            SPX_LAUNCHED();
            if (bs) SPX_CHECK(bj_apply<X>(n, bs, w.inv, w.r, w.z, w.p, w.partials, 0, w.st, false, s));
            SPX_CHECK(launch_finish<X>(w.partials, gv, 1, w.st, kOpCgRestart, s));
            SPX_CHECK(read_state(env, w.st, &hs));
            have_true = false;
            continue;
        }
        if (hs.flag != kRunning) {
            status = status_of_flag(hs.flag);
            if (hs.flag == kMaxit) set_error("cg: no convergence in %d iterations", sp.maxit);
            else if (hs.flag == kBreakdown) set_error("cg: breakdown (p'Ap <= 0)");
            else set_error("cg: non-finite residual");
            break;
        }
        if (graph.exec == nullptr) SPX_CHECK(capture_graph(s, &graph.exec, iterations));
        SPX_HIP(hipGraphLaunch(graph.exec, s));
        SPX_CHECK(read_state(env, w.st, &hs));
    }
    if (!have_true && hs.bb > 0.0) {
        SPX_CHECK(spmv_dispatch(A, x, w.q, 1.0, 0.0, s));
        SPX_CHECK(residual_norm<X>(n, b, w.q, w.r, w.partials, w.st, s));
        KState h2;
        SPX_CHECK(read_state(env, w.st, &h2));
        true2 = h2.tmp[0];
    }
    SPX_HIP(hipEventRecord(env->ev1, s));
    SPX_HIP(hipEventSynchronize(env->ev1));
    float ms = 0.f;
    SPX_HIP(hipEventElapsedTime(&ms, env->ev0, env->ev1));
    info->status = status;
    info->iters = hs.iters;
    info->spmv_count = hs.spmv_count + (sp.x0_zero ? 0 : 1);
    info->relres_recursive = hs.bb > 0 ? sqrt(hs.rr / hs.bb) : 0.0;
    info->relres_true = hs.bb > 0 ? sqrt(true2 / hs.bb) : 0.0;
    info->device_ms = ms;
    SPX_HIP(hipEventRecord(env->join, s));
    SPX_HIP(hipStreamWaitEvent(user_stream, env->join, 0));
    return status;
}

template size_t cg_workspace<double, double>(const spx_matrix &, int);
template size_t cg_workspace<float, float>(const spx_matrix &, int);
template size_t cg_workspace<_Float16, float>(const spx_matrix &, int);
template spx_status cg_run<double, double>(const spx_matrix &, const double *, double *, const SolveSpec &, void *,
                                           size_t, spx_solve_info *, hipStream_t);
template spx_status cg_run<float, float>(const spx_matrix &, const float *, float *, const SolveSpec &, void *,
                                         size_t, spx_solve_info *, hipStream_t);
template spx_status cg_run<_Float16, float>(const spx_matrix &, const float *, float *, const SolveSpec &, void *,
                                            size_t, spx_solve_info *, hipStream_t);

}  // namespace spx
