// solve_pipecg.hip -- pipelined preconditioned CG on the GPU.
//
// The pipelined CG of Ghysels & Vanroose ("Hiding global synchronization
// latency in the preconditioned Conjugate Gradient algorithm", Parallel
// Computing 40(7), 2014): CG's iterates in exact arithmetic, rearranged so
// that an iteration has a single reduction phase (gamma = r.u, delta = w.u
// and ||r||^2) that does not wait for the product with A. Kept besides x and
// r: u = M^{-1} r, w = A u, m = M^{-1} w, and the directions p, s = A p,
// q = M^{-1} s, z = A q (M = diag(A), or the identity, when u = r, m = w and
// q = s are the same vectors). One iteration is three launches:
//   1. a one-work-group finisher sums the previous update's partials, tests
//      ||r|| <= tol ||b||, and forms beta = gamma / gamma_prev and
//      alpha = gamma / (delta - beta gamma / alpha_prev);
//   2. nv = A m (any format);
//   3. z = nv + beta z, q = m + beta q, s = w + beta s, p = u + beta p,
//      x += alpha p, r -= alpha s, u -= alpha q, w -= alpha z, m = M^{-1} w,
//      with the partial sums of r.u, w.u and r.r.
// Against CG's five launches it moves more vector bytes (the update touches
// 20 vectors with Jacobi, 13 without, against CG's 11): on one GPU it pays
// where launches and reductions dominate (small systems); across GPUs the one
// reduction per iteration is the point. Scalars stay on the device and
// `check_every` iterations are replayed from a hipGraph; a recursive residual
// that passes is confirmed by the true residual, and a miss restarts the
// recurrences from it.
#include "solver_common.hpp"
#include "solvers.hpp"
#include "vec_io.hpp"

namespace spx {

// kInit: r = b - q (q = A x, or nullptr for x = 0) with partial sums b.b and
// r.r; otherwise r is given (restart) and only r.r is summed. Both: u = M^{-1} r.
template <bool kInit>
__global__ __launch_bounds__(kVecThreads) void pcg_start_kernel(int64_t n, const double *__restrict__ b,
                                                               const double *__restrict__ q,
                                                               const double *__restrict__ dinv,
                                                               double *__restrict__ r, double *__restrict__ u,
                                                               double *__restrict__ partials)
{
    __shared__ double s_red[kVecThreads / kWave];
    const int64_t i0 = vec_i0();
    double bb = 0.0, rr = 0.0;
#pragma unroll
    for (int k = 0; k < kVecItems; ++k) {
        const int64_t i = i0 + k;
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
            if (dinv) u[i] = ri * dinv[i];
            rr += ri * ri;
        }
    }
    if (kInit) {
        double v[2] = {block_sum<double, kVecThreads>(bb, s_red), block_sum<double, kVecThreads>(rr, s_red)};
        write_partials<double, 2>(v, partials, gridDim.x, blockIdx.x);
    } else {
        double v[1] = {block_sum<double, kVecThreads>(rr, s_red)};
        write_partials<double, 1>(v, partials, gridDim.x, blockIdx.x);
    }
}

// After w = A u: m = M^{-1} w and the partial sums r.u, w.u, r.r that the
// first iteration's finisher reduces.
__global__ __launch_bounds__(kVecThreads) void pcg_start2_kernel(int64_t n, const double *__restrict__ r,
                                                                const double *__restrict__ u,
                                                                const double *__restrict__ w,
                                                                const double *__restrict__ dinv,
                                                                double *__restrict__ m, double *__restrict__ partials)
{
    __shared__ double s_red[kVecThreads / kWave];
    const int64_t i0 = vec_i0();
    double g = 0.0, d = 0.0, rr = 0.0;
#pragma unroll
    for (int k = 0; k < kVecItems; ++k) {
        const int64_t i = i0 + k;
        if (i < n) {
            const double ri = r[i], ui = u[i], wi = w[i];
            if (dinv) m[i] = wi * dinv[i];
            g += ri * ui;
            d += wi * ui;
            rr += ri * ri;
        }
    }
    double v[3] = {block_sum<double, kVecThreads>(g, s_red), block_sum<double, kVecThreads>(d, s_red),
                   block_sum<double, kVecThreads>(rr, s_red)};
    write_partials<double, 3>(v, partials, gridDim.x, blockIdx.x);
}

// The recurrences of one iteration. kPrec: Jacobi (u, q, m are vectors of
// their own); otherwise u = r, q = s, m = w. beta = 0 (the first step after
// a (re)start) takes the new directions without reading the old ones.
template <bool kPrec, bool kVec>
__global__ __launch_bounds__(kVecThreads) void pcg_update_kernel(
    int64_t n, const double *__restrict__ nv, double *__restrict__ m, double *__restrict__ w, double *__restrict__ u,
    double *__restrict__ z, double *__restrict__ q, double *__restrict__ s, double *__restrict__ p,
    double *__restrict__ x, double *__restrict__ r, const double *__restrict__ dinv, double *__restrict__ partials,
    const KState *st)
{
    if (st->flag != kRunning) return;
    __shared__ double s_red[kVecThreads / kWave];
    typedef vec4_t<double> V4;
    const double a = st->alpha, be = st->beta;
    const bool fresh = be == 0.0;
    const int64_t i0 = vec_i0();
    const V4 nvv = ld4<double, kVec>(nv, i0, n);
    V4 wv = ld4<double, kVec>(w, i0, n), rv = ld4<double, kVec>(r, i0, n);
    V4 xv = ld4<double, kVec>(x, i0, n);
    V4 zv = nvv, sv = wv, pv, mv, uv, qv, dv;
    if (kPrec) {
        mv = ld4<double, kVec>(m, i0, n);
        uv = ld4<double, kVec>(u, i0, n);
        dv = ld4<double, kVec>(dinv, i0, n);
        pv = uv;
        qv = mv;
    } else {
        pv = rv;
    }
    if (!fresh) {
        const V4 zo = ld4<double, kVec>(z, i0, n), so = ld4<double, kVec>(s, i0, n), po = ld4<double, kVec>(p, i0, n);
        zv = nvv + be * zo;
        sv = wv + be * so;
        pv = pv + be * po;
        if (kPrec) qv = mv + be * ld4<double, kVec>(q, i0, n);
    }
    double g = 0.0, d = 0.0, rr = 0.0;
#pragma unroll
    for (int k = 0; k < kVecItems; ++k) {
        xv[k] += a * pv[k];
        rv[k] = rv[k] - a * sv[k];
        wv[k] = wv[k] - a * zv[k];
        if (kPrec) {
            uv[k] = uv[k] - a * qv[k];
            mv[k] = wv[k] * dv[k];
            g += rv[k] * uv[k];
            d += wv[k] * uv[k];
        } else {
            g += rv[k] * rv[k];
            d += wv[k] * rv[k];
        }
        rr += rv[k] * rv[k];
    }
    st4<double, kVec>(z, i0, n, zv);
    st4<double, kVec>(s, i0, n, sv);
    st4<double, kVec>(p, i0, n, pv);
    st4<double, kVec>(x, i0, n, xv);
    st4<double, kVec>(r, i0, n, rv);
    st4<double, kVec>(w, i0, n, wv);
    if (kPrec) {
        st4<double, kVec>(q, i0, n, qv);
        st4<double, kVec>(u, i0, n, uv);
        st4<double, kVec>(m, i0, n, mv);
    }
    double v[3] = {block_sum<double, kVecThreads>(g, s_red), block_sum<double, kVecThreads>(d, s_red),
                   block_sum<double, kVecThreads>(rr, s_red)};
    write_partials<double, 3>(v, partials, gridDim.x, blockIdx.x);
}

struct PcgBufs {
    KState *st;
    double *r, *u, *w, *m, *nv, *z, *q, *s, *p, *d, *dinv, *partials;
    int32_t *part;
};

static PcgBufs pcg_carve(Carve &c, const spx_matrix &A, int precond)
{
    const int64_t n = A.nrows;
    PcgBufs b{};
    b.st = c.take<KState>(1);
    b.r = c.take<double>(n);
    b.w = c.take<double>(n);
    b.nv = c.take<double>(n);
    b.z = c.take<double>(n);
    b.s = c.take<double>(n);
    b.p = c.take<double>(n);
    b.u = precond ? c.take<double>(n) : b.r;
    b.m = precond ? c.take<double>(n) : b.w;
    b.q = precond ? c.take<double>(n) : b.s;
    b.d = precond ? c.take<double>(n) : nullptr;
    b.dinv = precond ? c.take<double>(n) : nullptr;
    b.partials = c.take<double>(3 * partial_slots(A));
    b.part = (A.fmt == SPX_CSR && A.csr_part == nullptr) ? c.take<int32_t>(csr_partition_bytes(A.nnz) / 4) : nullptr;
    return b;
}

size_t pipecg_workspace(const spx_matrix &A, int precond)
{
    Carve c(nullptr, 0);
    (void)pcg_carve(c, A, precond);
    return c.off + 256;
}

spx_status pipecg_run(const spx_matrix &A_in, const double *b, double *x, const SolveSpec &sp, void *ws,
                      size_t ws_bytes, spx_solve_info *info, hipStream_t user_stream)
{
    SolveEnv *env = nullptr;
    SPX_CHECK(solve_env(&env));
    hipStream_t s = env->stream;
    const int64_t n = A_in.nrows;
    Carve c(ws, ws_bytes);
    PcgBufs w = pcg_carve(c, A_in, sp.precond);
    SPX_REQUIRE(c.fits(), SPX_ERR_ARG, "pipecg: workspace of %zu bytes is too small (need %zu)", ws_bytes,
                pipecg_workspace(A_in, sp.precond));
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
            set_error("pipecg: zero, missing or non-finite diagonal entry");
            return SPX_ERR_ZERO_DIAG;
        }
    }
    const unsigned gv = (unsigned)vec_blocks(n);
    if (sp.x0_zero) SPX_CHECK(fill_vector<double>(x, n, 0.0, s));  // x is write-only
    else SPX_CHECK(spmv_dispatch(A, x, w.nv, 1.0, 0.0, s));
    pcg_start_kernel<true><<<gv, kVecThreads, 0, s>>>(n, b, sp.x0_zero ? nullptr : w.nv, w.dinv, w.r, w.u,
                                                      w.partials);
    SPX_LAUNCHED();
    SPX_CHECK(launch_finish<double>(w.partials, gv, 2, w.st, kOpPipeInit, s));
    SPX_CHECK(read_state(env, w.st, &hs));
    int32_t starts = 0;  // products w = A u of (re)starts
    // w = A u, m = M^{-1} w and the first iteration's partials
    auto second_half = [&]() -> spx_status {
        SPX_CHECK(spmv_dispatch(A, w.u, w.w, 1.0, 0.0, s));
        pcg_start2_kernel<<<gv, kVecThreads, 0, s>>>(n, w.r, w.u, w.w, w.dinv, w.m, w.partials);
        SPX_LAUNCHED();
        ++starts;
        return SPX_OK;
    };
    if (hs.flag == kRunning) SPX_CHECK(second_half());

    GraphGuard graph;
    const int mm = sp.check_every > 0 ? sp.check_every : 16;
    // whole-group loads need x and the workspace (all its pieces sit at
    // multiples of 256 bytes from its start) aligned
    const bool vec = vec_aligned<double>({x, w.r});
    auto iterations = [&]() -> spx_status {
        for (int it = 0; it < mm; ++it) {
            SPX_CHECK(launch_finish<double>(w.partials, gv, 3, w.st, kOpPipeStep, s));
            SPX_CHECK((spmv_st<double, double>(A, w.m, w.nv, w.st, s)));
#define SPX_PCG_UPDATE(P, VEC)                                                                                    \
    pcg_update_kernel<P, VEC><<<gv, kVecThreads, 0, s>>>(n, w.nv, w.m, w.w, w.u, w.z, w.q, w.s, w.p, x, w.r, w.dinv, \
                                                        w.partials, w.st)
            if (sp.precond) {
                if (vec) SPX_PCG_UPDATE(true, true);
                else SPX_PCG_UPDATE(true, false);
            } else {
                if (vec) SPX_PCG_UPDATE(false, true);
                else SPX_PCG_UPDATE(false, false);
            }
#undef SPX_PCG_UPDATE
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
            SPX_CHECK(spmv_dispatch(A, x, w.nv, 1.0, 0.0, s));
            SPX_CHECK(residual_norm<double>(n, b, w.nv, w.r, w.partials, w.st, s));
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
            pcg_start_kernel<false><<<gv, kVecThreads, 0, s>>>(n, nullptr, nullptr, w.dinv, w.r, w.u, w.partials);
            SPX_LAUNCHED();
            SPX_CHECK(launch_finish<double>(w.partials, gv, 1, w.st, kOpPipeRestart, s));
            SPX_CHECK(second_half());
            SPX_CHECK(read_state(env, w.st, &hs));
            have_true = false;
            continue;
        }
        if (hs.flag != kRunning) {
            status = status_of_flag(hs.flag);
            if (hs.flag == kMaxit) set_error("pipecg: no convergence in %d iterations", sp.maxit);
            else if (hs.flag == kBreakdown) set_error("pipecg: breakdown (p'Ap <= 0)");
            else set_error("pipecg: non-finite residual");
            break;
        }
        if (graph.exec == nullptr) SPX_CHECK(capture_graph(s, &graph.exec, iterations));
        SPX_HIP(hipGraphLaunch(graph.exec, s));
        SPX_CHECK(read_state(env, w.st, &hs));
    }
    if (!have_true && hs.bb > 0.0) {
        SPX_CHECK(spmv_dispatch(A, x, w.nv, 1.0, 0.0, s));
        SPX_CHECK(residual_norm<double>(n, b, w.nv, w.r, w.partials, w.st, s));
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
    info->spmv_count = hs.spmv_count + starts + (sp.x0_zero ? 0 : 1);
    info->relres_recursive = hs.bb > 0 ? sqrt(hs.rr / hs.bb) : 0.0;
    info->relres_true = hs.bb > 0 ? sqrt(true2 / hs.bb) : 0.0;
    info->device_ms = ms;
    SPX_HIP(hipEventRecord(env->join, s));
    SPX_HIP(hipStreamWaitEvent(user_stream, env->join, 0));
    return status;
}

}  // namespace spx
