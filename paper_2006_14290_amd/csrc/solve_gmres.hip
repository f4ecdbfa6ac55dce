// solve_gmres.hip -- restarted, right-preconditioned GMRES(m) on the GPU.
//
// GMRES (Saad & Schultz 1986) as listed among the paper's solvers
// (Section 1), right-preconditioned with the scalar Jacobi M = diag(A):
// the Krylov space is that of A M^{-1}, and x = x0 + M^{-1} V y.
// Arnoldi orthogonalisation is classical Gram-Schmidt applied twice (CGS2,
// "twice is enough": Giraud, Langou, Rozloznik 2005): two passes of
//   h = V^T w (one multi-dot kernel: each work-group keeps its chunk of w in
//   registers and sweeps every basis vector), w -= V h,
// the second update fused with ||w||^2. A one-work-group finisher kernel that
// sums the partials of that reduction builds the Hessenberg column, applies the previous Givens rotations, forms
// the new one, updates the residual estimate |g_{j+1}| and decides whether the
// cycle ends (estimate below tolerance, lucky breakdown, or maxit). All of
// this stays on the device; one restart cycle (m Arnoldi steps) is a single
// captured hipGraph, replayed per cycle. At the end of a cycle one wavefront
// stages the triangle of H and g in LDS and one of its lanes back-substitutes
// H y = g there; then x += M^{-1} V y, and the next cycle starts from the true
// residual b - A x.
#include <cmath>

#include "solver_common.hpp"
#include "solvers.hpp"

namespace spx {

using X = double;

struct GmState {
    int m;
    double *H;   // (m+1) x m, column-major: H[j*(m+1) + i]
    double *g;   // m+1
    double *cs;  // m
    double *sn;  // m
    double *y;   // m
};

// cycle start: v0 = r / ||r|| (||r||^2 in st->tmp[0]), g = ||r|| e1
__global__ __launch_bounds__(kVecThreads) void gm_cycle_init_kernel(int64_t n, X *__restrict__ v0, KState *st,
                                                                   GmState gs)
{
    const double beta = sqrt(st->tmp[0]);
    const int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x;
    if (i < n) v0[i] = v0[i] / beta;
    if (i == 0) {
        for (int k = 0; k <= gs.m; ++k) gs.g[k] = 0.0;
        gs.g[0] = beta;
        st->jend = 0;
        st->flag = kRunning;
        st->tmp[1] = 1.0;
    }
}

// z = M^{-1} v_j, after normalising v_j = w / h_{j,j-1} (j > 0)
__global__ __launch_bounds__(kVecThreads) void gm_prep_kernel(int64_t n, X *__restrict__ vj, const X *__restrict__ dinv,
                                                             X *__restrict__ z, int normalise, const KState *st)
{
    if (st->flag != kRunning) return;
    const double inv = normalise ? 1.0 / st->tmp[1] : 1.0;
    const int64_t base = (int64_t)blockIdx.x * kVecChunk;
#pragma unroll
    for (int u = 0; u < kVecItems; ++u) {
        const int64_t i = base + threadIdx.x + u * kVecThreads;
        if (i < n) {
            const X v = normalise ? vj[i] * inv : vj[i];
            if (normalise) vj[i] = v;
            if (dinv) z[i] = v * dinv[i];
        }
    }
}

// h_i = v_i . w for i < nv: per-group partial sums (stage 1; the group keeps
// its chunk of w in registers and sweeps the basis vectors)
__global__ __launch_bounds__(kVecThreads) void gm_multidot_kernel(int64_t n, const X *__restrict__ V,
                                                                 const X *__restrict__ w, int nv,
                                                                 X *__restrict__ partials, const KState *st)
{
    if (st->flag != kRunning) return;
    __shared__ X s_red[kVecThreads / kWave];
    const int64_t base = (int64_t)blockIdx.x * kVecChunk;
    const int64_t nb = gridDim.x;
    X wl[kVecItems];
#pragma unroll
    for (int u = 0; u < kVecItems; ++u) {
        const int64_t i = base + threadIdx.x + u * kVecThreads;
        wl[u] = (i < n) ? w[i] : X(0);
    }
    for (int k = 0; k < nv; ++k) {
        const X *vk = V + (int64_t)k * n;
        X acc = X(0);
#pragma unroll
        for (int u = 0; u < kVecItems; ++u) {
            const int64_t i = base + threadIdx.x + u * kVecThreads;
            if (i < n) acc += vk[i] * wl[u];
        }
        const X t = block_sum<X, kVecThreads>(acc, s_red);
        if (threadIdx.x == 0) partials[(int64_t)k * nb + blockIdx.x] = t;
    }
}

// stage 2: st->dots[off + k] = sum of row k of the partials, fixed order:
// wavefront w takes rows w, w + 16, ...; lane l adds partials l, l + 64, ...
// of its row in that order, then the wavefront sum (no barrier).
__global__ __launch_bounds__(kFinThreads) void gm_multidot_finish(const X *__restrict__ partials, int64_t nb, int nv,
                                                                 KState *st, int off)
{
    if (st->flag != kRunning) return;
    constexpr int kW = kFinThreads / kWave;
    const int w = threadIdx.x / kWave, l = lane_id();
    for (int k = w; k < nv; k += kW) {
        X acc = X(0);
        const X *row = partials + (int64_t)k * nb;
#pragma unroll 8
        for (int64_t b = l; b < nb; b += kWave) acc += row[b];
        const X t = wave_sum(acc);
        if (l == 0) st->dots[off + k] = t;
    }
}

// w -= sum_i h_i v_i with h = st->dots[off..off+nv); optionally ||w||^2 and
// the Arnoldi step finish (Hessenberg column, Givens, cycle-end test).
__global__ __launch_bounds__(kVecThreads) void gm_update_kernel(int64_t n, const X *__restrict__ V, X *__restrict__ w,
                                                               int nv, int off, int final_pass,
                                                               X *__restrict__ partials, const KState *st)
{
    if (st->flag != kRunning) return;
    __shared__ X s_red[kVecThreads / kWave];
    __shared__ double s_h[kMaxDots];
    if (threadIdx.x < nv) s_h[threadIdx.x] = st->dots[off + threadIdx.x];
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kVecChunk;
    X wl[kVecItems];
#pragma unroll
    for (int u = 0; u < kVecItems; ++u) {
        const int64_t i = base + threadIdx.x + u * kVecThreads;
        wl[u] = (i < n) ? w[i] : X(0);
    }
    for (int k = 0; k < nv; ++k) {
        const X *vk = V + (int64_t)k * n;
        const X h = s_h[k];
#pragma unroll
        for (int u = 0; u < kVecItems; ++u) {
            const int64_t i = base + threadIdx.x + u * kVecThreads;
            if (i < n) wl[u] -= h * vk[i];
        }
    }
    X ww = X(0);
#pragma unroll
    for (int u = 0; u < kVecItems; ++u) {
        const int64_t i = base + threadIdx.x + u * kVecThreads;
        if (i < n) {
            w[i] = wl[u];
            ww += wl[u] * wl[u];
        }
    }
    if (!final_pass) return;
    const X t = block_sum<X, kVecThreads>(ww, s_red);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

// Arnoldi step finish: ||w||, Hessenberg column j, Givens rotations, the
// residual estimate and the cycle-end test (one work-group, fixed order).
__global__ __launch_bounds__(kFinThreads) void gm_step_finish(const X *__restrict__ partials, int64_t nb, int j,
                                                             KState *st, GmState gs)
{
    if (st->flag != kRunning) return;
    __shared__ X s_red[kFinThreads / kWave];
    X acc = X(0);
    for (int64_t b = threadIdx.x; b < nb; b += kFinThreads) acc += partials[b];
    const X w2 = block_sum<X, kFinThreads>(acc, s_red);
    if (threadIdx.x != 0) return;
    const int m = gs.m;
    double *hj = gs.H + (int64_t)j * (m + 1);
    for (int i = 0; i <= j; ++i) hj[i] = st->dots[i] + st->dots[kMaxDots + i];
    const double hn = sqrt(w2);
    hj[j + 1] = hn;
    for (int i = 0; i < j; ++i) {  // previous rotations
        const double a = hj[i], c = hj[i + 1];
        hj[i] = gs.cs[i] * a + gs.sn[i] * c;
        hj[i + 1] = -gs.sn[i] * a + gs.cs[i] * c;
    }
    const double rho = hypot(hj[j], hj[j + 1]);
    gs.cs[j] = hj[j] / rho;
    gs.sn[j] = hj[j + 1] / rho;
    hj[j] = rho;
    hj[j + 1] = 0.0;
    gs.g[j + 1] = -gs.sn[j] * gs.g[j];
    gs.g[j] = gs.cs[j] * gs.g[j];
    st->iters += 1;
    st->spmv_count += 1;
    st->jend = j + 1;
    st->tmp[1] = hn;
    st->rr = gs.g[j + 1] * gs.g[j + 1];
    if (!finite(gs.g[j + 1]) || !finite(hn)) st->flag = kNonfinite;
    else if (st->rr <= st->tol2 * st->bb || hn == 0.0 || st->iters >= st->maxit || j + 1 == m) st->flag = kCycleEnd;
}

// y = H(0:jend,0:jend)^{-1} g (back substitution)
__global__ __launch_bounds__(kWave) void gm_solve_kernel(KState *st, GmState gs)
{
    // the wavefront stages the triangle and g in LDS, then one lane runs
    // the substitution (in the same order) on LDS instead of on dependent
    // global loads
    __shared__ double s_h[(kMaxDots - 1) * kMaxDots];
    __shared__ double s_y[kMaxDots];
    const int jend = st->jend, m = gs.m;
    for (int t = threadIdx.x; t < jend * jend; t += kWave) {
        const int k = t / jend, i = t % jend;
        if (i <= k) s_h[k * kMaxDots + i] = gs.H[(int64_t)k * (m + 1) + i];
    }
    for (int t = threadIdx.x; t < jend; t += kWave) s_y[t] = gs.g[t];
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = jend - 1; i >= 0; --i) {
            double s = s_y[i];
            for (int k = i + 1; k < jend; ++k) s -= s_h[k * kMaxDots + i] * s_y[k];
            s_y[i] = s / s_h[i * kMaxDots + i];
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < jend; t += kWave) gs.y[t] = s_y[t];
}

// x += M^{-1} V y
__global__ __launch_bounds__(kVecThreads) void gm_xupdate_kernel(int64_t n, const X *__restrict__ V,
                                                                const X *__restrict__ dinv, X *__restrict__ x,
                                                                const KState *st, GmState gs)
{
    __shared__ double s_y[kMaxDots];
    const int jend = st->jend;
    if (threadIdx.x < jend) s_y[threadIdx.x] = gs.y[threadIdx.x];
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kVecChunk;
    X ul[kVecItems];
#pragma unroll
    for (int u = 0; u < kVecItems; ++u) ul[u] = X(0);
    for (int k = 0; k < jend; ++k) {
        const X *vk = V + (int64_t)k * n;
        const X yk = s_y[k];
#pragma unroll
        for (int u = 0; u < kVecItems; ++u) {
            const int64_t i = base + threadIdx.x + u * kVecThreads;
            if (i < n) ul[u] += yk * vk[i];
        }
    }
#pragma unroll
    for (int u = 0; u < kVecItems; ++u) {
        const int64_t i = base + threadIdx.x + u * kVecThreads;
        if (i < n) x[i] += dinv ? ul[u] * dinv[i] : ul[u];
    }
}

__global__ void gm_zero_vec(int64_t n, X *__restrict__ x)
{
    const int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x;
    if (i < n) x[i] = X(0);
}

// ||b||^2 -> st->bb (zero rhs flagged)
__global__ __launch_bounds__(kVecThreads) void gm_bnorm_kernel(int64_t n, const X *__restrict__ b,
                                                              X *__restrict__ partials, KState *st)
{
    __shared__ X s_red[kVecThreads / kWave];
    const int64_t base = (int64_t)blockIdx.x * kVecChunk;
    X acc = X(0);
#pragma unroll
    for (int u = 0; u < kVecItems; ++u) {
        const int64_t i = base + threadIdx.x + u * kVecThreads;
        if (i < n) acc += b[i] * b[i];
    }
    X v[1] = {block_sum<X, kVecThreads>(acc, s_red)};
    write_partials<X, 1>(v, partials, gridDim.x, blockIdx.x);
}

__global__ void gm_set_bb_kernel(KState *st)
{
    if (threadIdx.x == 0) {
        st->bb = st->tmp[0];
        if (!finite(st->bb)) st->flag = kNonfinite;
        else if (st->bb == 0.0) st->flag = kZeroRhs;
    }
}

struct GmBufs {
    X *V, *z, *q, *d, *dinv, *partials, *gmem;
    KState *st;
    int32_t *part;
};

static GmBufs gm_carve(Carve &c, const spx_matrix &A, int precond, int m)
{
    const int64_t n = A.nrows;
    GmBufs w{};
    w.st = c.take<KState>(1);
    w.V = c.take<X>((int64_t)(m + 1) * n);
    w.q = c.take<X>(n);
    w.z = precond ? c.take<X>(n) : nullptr;
    w.d = precond ? c.take<X>(n) : nullptr;
    w.dinv = precond ? c.take<X>(n) : nullptr;
    const int64_t vb = vec_blocks(n);
    const int64_t slots = spmv_dot_parts(A) > (m + 2) * vb ? spmv_dot_parts(A) : (m + 2) * vb;
    w.partials = c.take<X>(slots);
    w.gmem = c.take<X>((int64_t)(m + 1) * m + (m + 1) + 3 * m);
    w.part = (A.fmt == SPX_CSR && A.csr_part == nullptr) ? c.take<int32_t>(csr_partition_bytes(A.nnz) / 4) : nullptr;
    return w;
}

size_t gmres_workspace(const spx_matrix &A, int precond, int restart)
{
    Carve c(nullptr, 0);
    (void)gm_carve(c, A, precond, restart);
    return c.off + 256;
}

spx_status gmres_run(const spx_matrix &A_in, const double *b, double *x, const SolveSpec &sp, void *ws,
                     size_t ws_bytes, spx_solve_info *info, hipStream_t user_stream)
{
    const int m = sp.restart;
    SPX_REQUIRE(m >= 1 && m <= kMaxDots - 2, SPX_ERR_ARG, "gmres: restart must be in [1, %d]", kMaxDots - 2);
    SolveEnv *env = nullptr;
    SPX_CHECK(solve_env(&env));
    hipStream_t s = env->stream;
    const int64_t n = A_in.nrows;
    Carve c(ws, ws_bytes);
    GmBufs w = gm_carve(c, A_in, sp.precond, m);
    SPX_REQUIRE(c.fits(), SPX_ERR_ARG, "gmres: workspace of %zu bytes is too small (need %zu)", ws_bytes,
                gmres_workspace(A_in, sp.precond, m));
    spx_matrix A = A_in;
    *info = spx_solve_info{};
    GmState gs{m, w.gmem, w.gmem + (m + 1) * m, w.gmem + (m + 1) * m + (m + 1), w.gmem + (m + 1) * m + (m + 1) + m,
               w.gmem + (m + 1) * m + (m + 1) + 2 * m};

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
            set_error("gmres: zero, missing or non-finite diagonal entry");
            return SPX_ERR_ZERO_DIAG;
        }
    }
    const unsigned gv = (unsigned)vec_blocks(n);
    const unsigned ge = (unsigned)ceil_div(n, kVecThreads);
    if (sp.x0_zero) gm_zero_vec<<<ge, kVecThreads, 0, s>>>(n, x);
    gm_bnorm_kernel<<<gv, kVecThreads, 0, s>>>(n, b, w.partials, w.st);
    SPX_LAUNCHED();
    SPX_CHECK(launch_finish<X>(w.partials, gv, 1, w.st, kOpNorm2, s));
    gm_set_bb_kernel<<<1, 64, 0, s>>>(w.st);
    SPX_LAUNCHED();

    GraphGuard graph;
    auto cycle = [&]() -> spx_status {
        for (int j = 0; j < m; ++j) {
            X *vj = w.V + (int64_t)j * n;
            X *wv = w.V + (int64_t)(j + 1) * n;
            if (j > 0 || w.dinv) gm_prep_kernel<<<gv, kVecThreads, 0, s>>>(n, vj, w.dinv, w.z, j > 0 ? 1 : 0, w.st);
            const X *src = w.dinv ? w.z : vj;
            SPX_CHECK(spmv_dispatch(A, src, wv, 1.0, 0.0, s));
            gm_multidot_kernel<<<gv, kVecThreads, 0, s>>>(n, w.V, wv, j + 1, w.partials, w.st);
            gm_multidot_finish<<<1, kFinThreads, 0, s>>>(w.partials, gv, j + 1, w.st, 0);
            gm_update_kernel<<<gv, kVecThreads, 0, s>>>(n, w.V, wv, j + 1, 0, 0, w.partials, w.st);
            gm_multidot_kernel<<<gv, kVecThreads, 0, s>>>(n, w.V, wv, j + 1, w.partials, w.st);
            gm_multidot_finish<<<1, kFinThreads, 0, s>>>(w.partials, gv, j + 1, w.st, kMaxDots);
            gm_update_kernel<<<gv, kVecThreads, 0, s>>>(n, w.V, wv, j + 1, kMaxDots, 1, w.partials, w.st);
            gm_step_finish<<<1, kFinThreads, 0, s>>>(w.partials, gv, j, w.st, gs);
            SPX_LAUNCHED();
        }
        return SPX_OK;
    };
    spx_status status = SPX_OK;
    double true2 = 0.0;
    while (true) {
        // true residual into v0
        SPX_CHECK(spmv_dispatch(A, x, w.q, 1.0, 0.0, s));
        SPX_CHECK(residual_norm<double>(n, b, w.q, w.V, w.partials, w.st, s));
        SPX_CHECK(read_state(env, w.st, &hs));
        true2 = hs.tmp[0];
        if (hs.flag == kZeroRhs) {
            gm_zero_vec<<<ge, kVecThreads, 0, s>>>(n, x);
            SPX_LAUNCHED();
            true2 = 0.0;
            status = SPX_OK;
            break;
        }
        if (hs.flag == kNonfinite || !std::isfinite(true2)) {
            status = SPX_ERR_NONFINITE;
            set_error("gmres: non-finite residual");
            break;
        }
        if (true2 <= hs.tol2 * hs.bb) {
            status = SPX_OK;
            break;
        }
        if (hs.iters >= sp.maxit) {
            status = SPX_ERR_NOT_CONVERGED;
            set_error("gmres: no convergence in %d Arnoldi steps", sp.maxit);
            break;
        }
        gm_cycle_init_kernel<<<ge, kVecThreads, 0, s>>>(n, w.V, w.st, gs);
        SPX_LAUNCHED();
        if (graph.exec == nullptr) SPX_CHECK(capture_graph(s, &graph.exec, cycle));
        SPX_HIP(hipGraphLaunch(graph.exec, s));
        gm_solve_kernel<<<1, 64, 0, s>>>(w.st, gs);
        gm_xupdate_kernel<<<gv, kVecThreads, 0, s>>>(n, w.V, w.dinv, x, w.st, gs);
        SPX_LAUNCHED();
        SPX_CHECK(read_state(env, w.st, &hs));
        info->outer_iters += 1;
        if (hs.flag == kNonfinite) {
            status = SPX_ERR_NONFINITE;
            set_error("gmres: non-finite residual");
            break;
        }
    }
    SPX_HIP(hipEventRecord(env->ev1, s));
    SPX_HIP(hipEventSynchronize(env->ev1));
    float ms = 0.f;
    SPX_HIP(hipEventElapsedTime(&ms, env->ev0, env->ev1));
    info->status = status;
    info->iters = hs.iters;
    info->spmv_count = hs.spmv_count + info->outer_iters + 1;
    info->relres_recursive = hs.bb > 0 ? sqrt(hs.rr / hs.bb) : 0.0;
    info->relres_true = hs.bb > 0 ? sqrt(true2 / hs.bb) : 0.0;
    info->device_ms = ms;
    SPX_HIP(hipEventRecord(env->join, s));
    SPX_HIP(hipStreamWaitEvent(user_stream, env->join, 0));
    return status;
}

}  // namespace spx
