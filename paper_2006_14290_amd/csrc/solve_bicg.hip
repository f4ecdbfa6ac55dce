// solve_bicg.hip -- preconditioned BiCG on the GPU.
//
// BiCG (Fletcher 1976; the preconditioned form of Barrett et al.,
// "Templates", 1994), which the paper lists among the library's solvers
// (Section 1), with the shadow residual started as rt = r and the scalar
// Jacobi preconditioner (M = diag(A), so M^{-T} = M^{-1} and z = M^{-1} r is
// formed where it is needed instead of being stored). A^T is built once per
// solve in the workspace (stable device transpose), so both products are
// CSR products. One iteration is six launches:
//   1. qt = A^T pt;
//   2. q = A p fused with the partial sums of pt.q;
//   3. a one-work-group finisher: alpha = rho / pt.q;
//   4. x += alpha p, r -= alpha q, rt -= alpha qt, partial sums of
//      (M^{-1} r).rt and r.r;
//   5. a finisher forms beta = rho_new / rho and tests ||r|| <= tol ||b||;
//   6. p = M^{-1} r + beta p, pt = M^{-1} rt + beta pt.
// Scalars stay on the device; `check_every` iterations are captured once in
// a hipGraph and replayed. A recursive residual that passes is confirmed by
// the true residual b - A x; a miss restarts the recurrences from it with
// rt = r.
#include "solver_common.hpp"
#include "solvers.hpp"
#include "transpose.hpp"
#include "vec_io.hpp"

namespace spx {

// kInit: r = b - q (q = A x, or nullptr for x = 0), partial sums b.b,
// rho = (M^{-1} r).r, r.r. Otherwise r is given (restart) and only rho is
// summed. Both: rt = r, p = pt = M^{-1} r.
template <bool kInit>
__global__ __launch_bounds__(kVecThreads) void bicg_start_kernel(int64_t n, const double *__restrict__ b,
                                                                const double *__restrict__ q,
                                                                const double *__restrict__ dinv,
                                                                double *__restrict__ r, double *__restrict__ rt,
                                                                double *__restrict__ p, double *__restrict__ pt,
                                                                double *__restrict__ partials)
{
    __shared__ double s_red[kVecThreads / kWave];
    const int64_t i0 = vec_i0();
    double bb = 0.0, rho = 0.0, rr = 0.0;
#pragma unroll
    for (int u = 0; u < kVecItems; ++u) {
        const int64_t i = i0 + u;
        if (i < n) {
            double ri;
            if (kInit) {
                const double bi = b[i];
                ri = q ? bi - q[i] : bi;
                r[i] = ri;
                bb += bi * bi;
            } else {
                ri = r[i];
            }
            const double zi = dinv ? ri * dinv[i] : ri;
            rt[i] = ri;
            p[i] = zi;
            pt[i] = zi;
            rho += zi * ri;
            rr += ri * ri;
        }
    }
    if (kInit) {
        double v[3] = {block_sum<double, kVecThreads>(bb, s_red), block_sum<double, kVecThreads>(rho, s_red),
                       block_sum<double, kVecThreads>(rr, s_red)};
        write_partials<double, 3>(v, partials, gridDim.x, blockIdx.x);
    } else {
        double v[1] = {block_sum<double, kVecThreads>(rho, s_red)};
        write_partials<double, 1>(v, partials, gridDim.x, blockIdx.x);
    }
}

// x += alpha p, r -= alpha q, rt -= alpha qt; partial sums of
// (M^{-1} r).rt and r.r of the new residuals.
template <bool kVec>
__global__ __launch_bounds__(kVecThreads) void bicg_update_kernel(int64_t n, double *__restrict__ x,
                                                                 const double *__restrict__ p,
                                                                 const double *__restrict__ q, double *__restrict__ r,
                                                                 double *__restrict__ rt,
                                                                 const double *__restrict__ qt,
                                                                 const double *__restrict__ dinv,
                                                                 double *__restrict__ partials, const KState *st)
{
    if (st->flag != kRunning) return;
    __shared__ double s_red[kVecThreads / kWave];
    const double a = st->alpha;
    const int64_t i0 = vec_i0();
    vec4_t<double> xv = ld4<double, kVec>(x, i0, n), rv = ld4<double, kVec>(r, i0, n);
    vec4_t<double> tv = ld4<double, kVec>(rt, i0, n);
    const vec4_t<double> pv = ld4<double, kVec>(p, i0, n), qv = ld4<double, kVec>(q, i0, n);
    const vec4_t<double> qtv = ld4<double, kVec>(qt, i0, n);
    vec4_t<double> dv;
    if (dinv) dv = ld4<double, kVec>(dinv, i0, n);
    double rho = 0.0, rr = 0.0;
#pragma unroll
    for (int u = 0; u < kVecItems; ++u) {
        xv[u] += a * pv[u];
        rv[u] = rv[u] - a * qv[u];
        tv[u] = tv[u] - a * qtv[u];
        const double zi = dinv ? rv[u] * dv[u] : rv[u];
        rho += zi * tv[u];
        rr += rv[u] * rv[u];
    }
    st4<double, kVec>(x, i0, n, xv);
    st4<double, kVec>(r, i0, n, rv);
    st4<double, kVec>(rt, i0, n, tv);
    double v[2] = {block_sum<double, kVecThreads>(rho, s_red), block_sum<double, kVecThreads>(rr, s_red)};
    write_partials<double, 2>(v, partials, gridDim.x, blockIdx.x);
}

// p = M^{-1} r + beta p, pt = M^{-1} rt + beta pt.
template <bool kVec>
__global__ __launch_bounds__(kVecThreads) void bicg_dir_kernel(int64_t n, const double *__restrict__ r,
                                                              const double *__restrict__ rt,
                                                              const double *__restrict__ dinv,
                                                              double *__restrict__ p, double *__restrict__ pt,
                                                              const KState *st)
{
    if (st->flag != kRunning) return;
    const double be = st->beta;
    const int64_t i0 = vec_i0();
    const vec4_t<double> rv = ld4<double, kVec>(r, i0, n), tv = ld4<double, kVec>(rt, i0, n);
    vec4_t<double> pv = ld4<double, kVec>(p, i0, n), ptv = ld4<double, kVec>(pt, i0, n);
    vec4_t<double> dv;
    if (dinv) dv = ld4<double, kVec>(dinv, i0, n);
#pragma unroll
    for (int u = 0; u < kVecItems; ++u) {
        pv[u] = (dinv ? rv[u] * dv[u] : rv[u]) + be * pv[u];
        ptv[u] = (dinv ? tv[u] * dv[u] : tv[u]) + be * ptv[u];
    }
    st4<double, kVec>(p, i0, n, pv);
    st4<double, kVec>(pt, i0, n, ptv);
}

struct BicgBufs {
    KState *st;
    double *r, *rt, *p, *pt, *q, *qt, *d, *dinv, *partials, *val_t;
    int32_t *part, *rowptr_t, *col_t, *part_t;
    char *tws;  // transpose scratch
};

static BicgBufs bicg_carve(Carve &c, const spx_matrix &A, int precond)
{
    const int64_t n = A.nrows, nnz = A.nnz;
    BicgBufs w{};
    w.st = c.take<KState>(1);
    w.r = c.take<double>(n);
    w.rt = c.take<double>(n);
    w.p = c.take<double>(n);
    w.pt = c.take<double>(n);
    w.q = c.take<double>(n);
    w.qt = c.take<double>(n);
    w.d = precond ? c.take<double>(n) : nullptr;
    w.dinv = precond ? c.take<double>(n) : nullptr;
    w.partials = c.take<double>(3 * partial_slots(A));
    w.part = A.csr_part == nullptr ? c.take<int32_t>(csr_partition_bytes(nnz) / 4) : nullptr;
    w.rowptr_t = c.take<int32_t>(n + 1);
    w.col_t = c.take<int32_t>(nnz);
    w.val_t = c.take<double>(nnz);
    w.part_t = c.take<int32_t>(csr_partition_bytes(nnz) / 4);
    w.tws = c.take<char>(transpose_ws_bytes(nnz));
    return w;
}

size_t bicg_workspace(const spx_matrix &A, int precond)
{
    Carve c(nullptr, 0);
    (void)bicg_carve(c, A, precond);
    return c.off + 256;
}

spx_status bicg_run(const spx_matrix &A_in, const double *b, double *x, const SolveSpec &sp, void *ws,
                    size_t ws_bytes, spx_solve_info *info, hipStream_t user_stream)
{
    SolveEnv *env = nullptr;
    SPX_CHECK(solve_env(&env));
    hipStream_t s = env->stream;
    const int64_t n = A_in.nrows;
    Carve c(ws, ws_bytes);
    BicgBufs w = bicg_carve(c, A_in, sp.precond);
    SPX_REQUIRE(c.fits(), SPX_ERR_ARG, "bicg: workspace of %zu bytes is too small (need %zu)", ws_bytes,
                bicg_workspace(A_in, sp.precond));
    spx_matrix A = A_in;
    *info = spx_solve_info{};

    SPX_HIP(hipEventRecord(env->join, user_stream));
    SPX_HIP(hipStreamWaitEvent(s, env->join, 0));
    SPX_HIP(hipEventRecord(env->ev0, s));
    if (w.part) {
        SPX_CHECK(csr_partition_launch(A, w.part, s));
        A.csr_part = w.part;
    }
    // A^T in the workspace (its own tile partition; no row-length hint)
    spx_matrix At = A;
    At.rowptr = w.rowptr_t;
    At.colidx = w.col_t;
    At.vals = w.val_t;
    At.csr_part = nullptr;
    At.max_row_len = 0;
    SPX_CHECK(transpose_run(A, At, w.tws, (size_t)transpose_ws_bytes(A.nnz), s));
    SPX_CHECK(csr_partition_launch(At, w.part_t, s));
    At.csr_part = w.part_t;

    SPX_CHECK(state_init(w.st, sp.tol, sp.maxit, s));
    KState hs;
    if (sp.precond) {
        SPX_CHECK((jacobi_setup<double, double>(A, w.d, w.dinv, w.st, s)));
        SPX_CHECK(read_state(env, w.st, &hs));
        if (hs.flag != kRunning) {
            set_error("bicg: zero, missing or non-finite diagonal entry");
            return SPX_ERR_ZERO_DIAG;
        }
    }
    const unsigned gv = (unsigned)vec_blocks(n);
    if (sp.x0_zero) SPX_CHECK(fill_vector<double>(x, n, 0.0, s));  // x is write-only
    else SPX_CHECK(spmv_dispatch(A, x, w.q, 1.0, 0.0, s));
    bicg_start_kernel<true><<<gv, kVecThreads, 0, s>>>(n, b, sp.x0_zero ? nullptr : w.q, w.dinv, w.r, w.rt, w.p,
                                                       w.pt, w.partials);
    SPX_LAUNCHED();
    SPX_CHECK(launch_finish<double>(w.partials, gv, 3, w.st, kOpCgInit, s));
    SPX_CHECK(read_state(env, w.st, &hs));

    GraphGuard graph;
    const int m = sp.check_every > 0 ? sp.check_every : 16;
    // whole-group loads need x and the workspace (all its pieces sit at
    // multiples of 256 bytes from its start) aligned
    const bool vec = vec_aligned<double>({x, w.r});
    auto iterations = [&]() -> spx_status {
        for (int it = 0; it < m; ++it) {
            SPX_CHECK((csr_spmv_launch<double, double>(At, w.pt, w.qt, 1.0, 0.0, nullptr, nullptr, s, 0, w.st)));
            SPX_CHECK((spmv_dot<double, double>(A, w.p, w.q, w.pt, w.partials, w.st, kOpBicgAlpha, s)));
            if (vec)
                bicg_update_kernel<true><<<gv, kVecThreads, 0, s>>>(n, x, w.p, w.q, w.r, w.rt, w.qt, w.dinv,
                                                                    w.partials, w.st);
            else
                bicg_update_kernel<false><<<gv, kVecThreads, 0, s>>>(n, x, w.p, w.q, w.r, w.rt, w.qt, w.dinv,
                                                                     w.partials, w.st);
            SPX_LAUNCHED();
            SPX_CHECK(launch_finish<double>(w.partials, gv, 2, w.st, kOpBicgRho, s));
            if (vec) bicg_dir_kernel<true><<<gv, kVecThreads, 0, s>>>(n, w.r, w.rt, w.dinv, w.p, w.pt, w.st);
            else bicg_dir_kernel<false><<<gv, kVecThreads, 0, s>>>(n, w.r, w.rt, w.dinv, w.p, w.pt, w.st);
            SPX_LAUNCHED();
        }
        return SPX_OK;
    };
    spx_status status = SPX_OK;
    bool have_true = false;
    double true2 = 0.0;
    while (true) {
        if (hs.flag == kZeroRhs) {
            SPX_CHECK(fill_vector<double>(x, n, 0.0, s));
            status = SPX_OK;
            have_true = true;
            true2 = 0.0;
            break;
        }
        if (hs.flag == kConverged) {
            SPX_CHECK(spmv_dispatch(A, x, w.q, 1.0, 0.0, s));
            SPX_CHECK(residual_norm<double>(n, b, w.q, w.r, w.partials, w.st, s));
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
            // restart from the true residual (already in r) with rt = r
            bicg_start_kernel<false><<<gv, kVecThreads, 0, s>>>(n, nullptr, nullptr, w.dinv, w.r, w.rt, w.p, w.pt,
                                                                w.partials);
            SPX_LAUNCHED();
            SPX_CHECK(launch_finish<double>(w.partials, gv, 1, w.st, kOpCgRestart, s));
            SPX_CHECK(read_state(env, w.st, &hs));
            have_true = false;
            continue;
        }
        if (hs.flag != kRunning) {
            status = status_of_flag(hs.flag);
            if (hs.flag == kMaxit) set_error("bicg: no convergence in %d iterations", sp.maxit);
            else if (hs.flag == kBreakdown) set_error("bicg: breakdown (rho = 0 or pt'q = 0)");
            else set_error("bicg: non-finite residual");
            break;
        }
        if (graph.exec == nullptr) SPX_CHECK(capture_graph(s, &graph.exec, iterations));
        SPX_HIP(hipGraphLaunch(graph.exec, s));
        SPX_CHECK(read_state(env, w.st, &hs));
    }
    if (!have_true && hs.bb > 0.0) {
        SPX_CHECK(spmv_dispatch(A, x, w.q, 1.0, 0.0, s));
        SPX_CHECK(residual_norm<double>(n, b, w.q, w.r, w.partials, w.st, s));
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

}  // namespace spx
