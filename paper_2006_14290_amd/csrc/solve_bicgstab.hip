// solve_bicgstab.hip -- right-preconditioned BiCGSTAB on the GPU.
//
// Bi-CGSTAB (van der Vorst 1992) in the right-preconditioned form of
// Barrett et al., "Templates" (1994): the BiCG-family solver for the
// nonsymmetric systems among the paper's solvers (Section 1). Per iteration
// five launches, every scalar on the device:
//   P  p = r + beta (p - omega v),  p^ = D^{-1} p
//   A1 v = A p^ fused with rhat.v            -> alpha = rho / rhat.v
//   S  s = r - alpha v, s^ = D^{-1} s, s.s   -> half-step test ||s|| <= tol||b||
//   A2 t = A s^ fused with t.s and t.t       -> omega = t.s / t.t
//   X  x += alpha p^ + omega s^, r = s - omega t, r.r and rhat.r
//                                            -> convergence, beta, rho
// The first iteration uses beta = 0 with p = v = 0 (so p = r). A half-step
// exit applies x += alpha p^ on the host's next launch. Convergence is
// confirmed with the true residual; a miss restarts with rhat = r.
#include "solver_common.hpp"
#include "solvers.hpp"

namespace spx {

using X = double;

__global__ __launch_bounds__(kVecThreads) void bi_init_kernel(int64_t n, const X *__restrict__ b, const X *__restrict__ q,
                                                             X *__restrict__ r, X *__restrict__ rh, X *__restrict__ p,
                                                             X *__restrict__ v, X *__restrict__ partials, KState *st)
{
    __shared__ X s_red[kVecThreads / kWave];
    const int64_t base = (int64_t)blockIdx.x * kVecChunk;
    X bb = X(0), rr = X(0);
#pragma unroll
    for (int u = 0; u < kVecItems; ++u) {
        const int64_t i = base + threadIdx.x + u * kVecThreads;
        if (i < n) {
            const X bi = b[i];
            const X ri = q ? bi - q[i] : bi;
            r[i] = ri;
            rh[i] = ri;
            p[i] = X(0);
            v[i] = X(0);
            bb += bi * bi;
            rr += ri * ri;
        }
    }
    X vals[2] = {block_sum<X, kVecThreads>(bb, s_red), block_sum<X, kVecThreads>(rr, s_red)};
    write_partials<X, 2>(vals, partials, gridDim.x, blockIdx.x);
}

// restart from the current (true) residual r: rhat = r, p = v = 0
__global__ __launch_bounds__(kVecThreads) void bi_restart_kernel(int64_t n, const X *__restrict__ r, X *__restrict__ rh,
                                                                X *__restrict__ p, X *__restrict__ v,
                                                                X *__restrict__ partials, KState *st)
{
    __shared__ X s_red[kVecThreads / kWave];
    const int64_t base = (int64_t)blockIdx.x * kVecChunk;
    X rr = X(0);
#pragma unroll
    for (int u = 0; u < kVecItems; ++u) {
        const int64_t i = base + threadIdx.x + u * kVecThreads;
        if (i < n) {
            const X ri = r[i];
            rh[i] = ri;
            p[i] = X(0);
            v[i] = X(0);
            rr += ri * ri;
        }
    }
    X vals[1] = {block_sum<X, kVecThreads>(rr, s_red)};
    write_partials<X, 1>(vals, partials, gridDim.x, blockIdx.x);
}

__global__ __launch_bounds__(kVecThreads) void bi_p_kernel(int64_t n, const X *__restrict__ r, const X *__restrict__ v,
                                                          X *__restrict__ p, X *__restrict__ ph,
                                                          const X *__restrict__ dinv, const KState *st)
{
    if (st->flag != kRunning) return;
    const X be = st->beta, om = st->omega;
    const int64_t base = (int64_t)blockIdx.x * kVecChunk;
#pragma unroll
    for (int u = 0; u < kVecItems; ++u) {
        const int64_t i = base + threadIdx.x + u * kVecThreads;
        if (i < n) {
            const X pi = r[i] + be * (p[i] - om * v[i]);
            p[i] = pi;
            if (dinv) ph[i] = pi * dinv[i];
        }
    }
}

__global__ __launch_bounds__(kVecThreads) void bi_s_kernel(int64_t n, const X *__restrict__ r, const X *__restrict__ v,
                                                          X *__restrict__ s, X *__restrict__ sh,
                                                          const X *__restrict__ dinv, X *__restrict__ partials,
                                                          KState *st)
{
    if (st->flag != kRunning) return;
    __shared__ X s_red[kVecThreads / kWave];
    const X a = st->alpha;
    const int64_t base = (int64_t)blockIdx.x * kVecChunk;
    X ss = X(0);
#pragma unroll
    for (int u = 0; u < kVecItems; ++u) {
        const int64_t i = base + threadIdx.x + u * kVecThreads;
        if (i < n) {
            const X si = r[i] - a * v[i];
            s[i] = si;
            if (dinv) sh[i] = si * dinv[i];
            ss += si * si;
        }
    }
    X vals[1] = {block_sum<X, kVecThreads>(ss, s_red)};
    write_partials<X, 1>(vals, partials, gridDim.x, blockIdx.x);
}

__global__ __launch_bounds__(kVecThreads) void bi_x_kernel(int64_t n, X *__restrict__ x, const X *__restrict__ ph,
                                                          const X *__restrict__ sh, const X *__restrict__ s,
                                                          const X *__restrict__ t, X *__restrict__ r,
                                                          const X *__restrict__ rh, X *__restrict__ partials,
                                                          KState *st)
{
    if (st->flag != kRunning) return;
    __shared__ X s_red[kVecThreads / kWave];
    const X a = st->alpha, om = st->omega;
    const int64_t base = (int64_t)blockIdx.x * kVecChunk;
    X rr = X(0), rhr = X(0);
#pragma unroll
    for (int u = 0; u < kVecItems; ++u) {
        const int64_t i = base + threadIdx.x + u * kVecThreads;
        if (i < n) {
            x[i] += a * ph[i] + om * sh[i];
            const X ri = s[i] - om * t[i];
            r[i] = ri;
            rr += ri * ri;
            rhr += rh[i] * ri;
        }
    }
    X vals[2] = {block_sum<X, kVecThreads>(rr, s_red), block_sum<X, kVecThreads>(rhr, s_red)};
    write_partials<X, 2>(vals, partials, gridDim.x, blockIdx.x);
}

// half-step exit: x += alpha p^
__global__ __launch_bounds__(kVecThreads) void bi_half_kernel(int64_t n, X *__restrict__ x, const X *__restrict__ ph,
                                                             const KState *st)
{
    const X a = st->alpha;
    const int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x;
    if (i < n) x[i] += a * ph[i];
}

__global__ void zero_vec(int64_t n, X *__restrict__ x)
{
    const int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x;
    if (i < n) x[i] = X(0);
}

struct BiBufs {
    X *r, *rh, *p, *ph, *v, *s, *sh, *t, *q, *d, *dinv, *partials;
    KState *st;
    int32_t *part;
};

static BiBufs bi_carve(Carve &c, const spx_matrix &A, int precond)
{
    const int64_t n = A.nrows;
    BiBufs w{};
    w.st = c.take<KState>(1);
    w.r = c.take<X>(n);
    w.rh = c.take<X>(n);
    w.p = c.take<X>(n);
    w.v = c.take<X>(n);
    w.s = c.take<X>(n);
    w.t = c.take<X>(n);
    w.q = c.take<X>(n);
    w.ph = precond ? c.take<X>(n) : w.p;
    w.sh = precond ? c.take<X>(n) : w.s;
    w.d = precond ? c.take<X>(n) : nullptr;
    w.dinv = precond ? c.take<X>(n) : nullptr;
    w.partials = c.take<X>(3 * partial_slots(A));
    w.part = (A.fmt == SPX_CSR && A.csr_part == nullptr) ? c.take<int32_t>(csr_partition_bytes(A.nnz) / 4) : nullptr;
    return w;
}

size_t bicgstab_workspace(const spx_matrix &A, int precond)
{
    Carve c(nullptr, 0);
    (void)bi_carve(c, A, precond);
    return c.off + 256;
}

spx_status bicgstab_run(const spx_matrix &A_in, const double *b, double *x, const SolveSpec &sp, void *ws,
                        size_t ws_bytes, spx_solve_info *info, hipStream_t user_stream)
{
    SolveEnv *env = nullptr;
    SPX_CHECK(solve_env(&env));
    hipStream_t s = env->stream;
    const int64_t n = A_in.nrows;
    Carve c(ws, ws_bytes);
    BiBufs w = bi_carve(c, A_in, sp.precond);
    SPX_REQUIRE(c.fits(), SPX_ERR_ARG, "bicgstab: workspace of %zu bytes is too small (need %zu)", ws_bytes,
                bicgstab_workspace(A_in, sp.precond));
    spx_matrix A = A_in;
    *info = spx_solve_info{};
    SPX_HIP(hipEventRecord(env->join, user_stream));
    SPX_HIP(hipStreamWaitEvent(s, env->join, 0));
    SPX_HIP(hipEventRecord(env->ev0, s));
    if (w.part) {
        SPX_CHECK(csr_partition_launch(A, w.part, s));
        A.csr_part = w.part;
    }
    SPX_CHECK(state_init(w.st, sp.tol, sp.maxit, s));
    KState hs;
    if (sp.precond) {
        SPX_CHECK((jacobi_setup<double, double>(A, w.d, w.dinv, w.st, s)));
        SPX_CHECK(read_state(env, w.st, &hs));
        if (hs.flag != kRunning) {
            set_error("bicgstab: zero, missing or non-finite diagonal entry");
            return SPX_ERR_ZERO_DIAG;
        }
    }
    const unsigned gv = (unsigned)vec_blocks(n);
    const unsigned ge = (unsigned)ceil_div(n, kVecThreads);
    if (sp.x0_zero) {
        zero_vec<<<ge, kVecThreads, 0, s>>>(n, x);
        bi_init_kernel<<<gv, kVecThreads, 0, s>>>(n, b, nullptr, w.r, w.rh, w.p, w.v, w.partials, w.st);
    } else {
        SPX_CHECK(spmv_dispatch(A, x, w.q, 1.0, 0.0, s));
        bi_init_kernel<<<gv, kVecThreads, 0, s>>>(n, b, w.q, w.r, w.rh, w.p, w.v, w.partials, w.st);
    }
    SPX_LAUNCHED();
    SPX_CHECK(launch_finish<X>(w.partials, gv, 2, w.st, kOpBiInit, s));
    SPX_CHECK(read_state(env, w.st, &hs));

    GraphGuard graph;
    const int m = sp.check_every > 0 ? sp.check_every : 16;
    auto iterations = [&]() -> spx_status {
        for (int it = 0; it < m; ++it) {
            bi_p_kernel<<<gv, kVecThreads, 0, s>>>(n, w.r, w.v, w.p, w.ph, w.dinv, w.st);
            SPX_CHECK((spmv_dot<double, double>(A, w.ph, w.v, w.rh, w.partials, w.st, kOpBiAlpha, s)));
            bi_s_kernel<<<gv, kVecThreads, 0, s>>>(n, w.r, w.v, w.s, w.sh, w.dinv, w.partials, w.st);
            SPX_CHECK(launch_finish<X>(w.partials, gv, 1, w.st, kOpBiS, s));
            SPX_CHECK((spmv_dot2<double, double>(A, w.sh, w.t, w.s, w.partials, w.st, kOpBiOmega, s)));
            bi_x_kernel<<<gv, kVecThreads, 0, s>>>(n, x, w.ph, w.sh, w.s, w.t, w.r, w.rh, w.partials, w.st);
            SPX_LAUNCHED();
            SPX_CHECK(launch_finish<X>(w.partials, gv, 2, w.st, kOpBiRho, s));
        }
        return SPX_OK;
    };
    spx_status status = SPX_OK;
    bool have_true = false;
    double true2 = 0.0;
    while (true) {
        if (hs.flag == kZeroRhs) {
            zero_vec<<<ge, kVecThreads, 0, s>>>(n, x);
            SPX_LAUNCHED();
            have_true = true;
            true2 = 0.0;
            status = SPX_OK;
            break;
        }
        if (hs.flag == kConverged || hs.flag == kHalfConverged) {
            if (hs.flag == kHalfConverged) {
                bi_half_kernel<<<ge, kVecThreads, 0, s>>>(n, x, w.ph, w.st);
                SPX_LAUNCHED();
            }
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
                set_error("bicgstab: no convergence in %d iterations", sp.maxit);
                break;
            }
            bi_restart_kernel<<<gv, kVecThreads, 0, s>>>(n, w.r, w.rh, w.p, w.v, w.partials, w.st);
            SPX_LAUNCHED();
            SPX_CHECK(launch_finish<X>(w.partials, gv, 1, w.st, kOpBiRestart, s));
            SPX_CHECK(read_state(env, w.st, &hs));
            have_true = false;
            continue;
        }
        if (hs.flag != kRunning) {
            status = status_of_flag(hs.flag);
            if (hs.flag == kMaxit) set_error("bicgstab: no convergence in %d iterations", sp.maxit);
            else if (hs.flag == kBreakdown) set_error("bicgstab: breakdown (rho, rhat.v, t.t or omega is zero)");
            else set_error("bicgstab: non-finite residual");
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
