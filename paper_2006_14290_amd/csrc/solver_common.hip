// solver_common.hip -- shared pieces of the Krylov drivers.
#include "solver_common.hpp"

namespace spx {

spx_status solve_env(SolveEnv **env)
{
    static thread_local SolveEnv e;
    static thread_local int dev_of_env = -1;
    int dev = 0;
    SPX_HIP(hipGetDevice(&dev));
    if (e.stream == nullptr || dev_of_env != dev) {
        // one environment per thread and device; the previous device's one is released
        if (e.stream) {
            (void)hipStreamDestroy(e.stream);
            (void)hipHostFree(e.host_state);
            (void)hipEventDestroy(e.ev0);
            (void)hipEventDestroy(e.ev1);
            (void)hipEventDestroy(e.join);
            e = SolveEnv{};
        }
        SPX_HIP(hipStreamCreateWithFlags(&e.stream, hipStreamNonBlocking));
        SPX_HIP(hipHostMalloc(reinterpret_cast<void **>(&e.host_state), sizeof(KState), hipHostMallocDefault));
        SPX_HIP(hipEventCreate(&e.ev0));
        SPX_HIP(hipEventCreate(&e.ev1));
        SPX_HIP(hipEventCreateWithFlags(&e.join, hipEventDisableTiming));
        dev_of_env = dev;
    }
    *env = &e;
    return SPX_OK;
}

spx_status read_state(SolveEnv *env, const KState *dst, KState *out)
{
    SPX_HIP(hipMemcpyAsync(env->host_state, dst, sizeof(KState), hipMemcpyDeviceToHost, env->stream));
    SPX_HIP(hipStreamSynchronize(env->stream));
    *out = *env->host_state;
    return SPX_OK;
}

__global__ void state_init_kernel(KState *st, double tol, int32_t maxit)
{
    if (threadIdx.x == 0) {
        st->rho = st->rho0 = st->alpha = st->beta = st->omega = st->bb = st->rr = 0.0;
        st->omega = 1.0;
        for (int i = 0; i < 4; ++i) st->tmp[i] = 0.0;
        st->tol2 = tol * tol;
        st->flag = kRunning;
        st->iters = 0;
        st->maxit = maxit;
        st->spmv_count = 0;
        st->restart_j = 0;
        st->jend = 0;
    }
}

spx_status state_init(KState *st, double tol, int32_t maxit, hipStream_t stream)
{
    state_init_kernel<<<1, 64, 0, stream>>>(st, tol, maxit);
    SPX_LAUNCHED();
    return SPX_OK;
}

__global__ void state_flag_kernel(KState *st, int32_t flag)
{
    if (threadIdx.x == 0) st->flag = flag;
}

spx_status state_set_flag(KState *st, int32_t flag, hipStream_t stream)
{
    state_flag_kernel<<<1, 64, 0, stream>>>(st, flag);
    SPX_LAUNCHED();
    return SPX_OK;
}

// ------------------------------------------------------------------ Jacobi
template <typename X>
__global__ __launch_bounds__(kVecThreads) void fill_vec_kernel(X *a, int64_t n, X v)
{
    const int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x;
    if (i < n) a[i] = v;
}

template <typename X>
spx_status fill_vector(X *a, int64_t n, X v, hipStream_t stream)
{
    if (n <= 0) return SPX_OK;
    fill_vec_kernel<X><<<(unsigned)ceil_div(n, kVecThreads), kVecThreads, 0, stream>>>(a, n, v);
    SPX_LAUNCHED();
    return SPX_OK;
}
template spx_status fill_vector<double>(double *, int64_t, double, hipStream_t);
template spx_status fill_vector<float>(float *, int64_t, float, hipStream_t);

template <typename V, typename X>
spx_status spmv_st(const spx_matrix &A, const X *x, X *y, KState *st, hipStream_t stream)
{
    if (A.fmt == SPX_CSR) return csr_spmv_launch<V, X>(A, x, y, X(1), X(0), nullptr, nullptr, stream, 0, st);
    if (A.fmt == SPX_SELLP) return sellp_spmv_launch<V, X>(A, x, y, X(1), X(0), stream, 0, nullptr, nullptr, st);
    if (A.fmt == SPX_ELL) return ell_spmv_launch<V, X>(A, x, y, X(1), X(0), stream, 0, nullptr, nullptr, st);
    return spmv_dispatch(A, x, y, 1.0, 0.0, stream);
}
template spx_status spmv_st<double, double>(const spx_matrix &, const double *, double *, KState *, hipStream_t);

template <typename V, typename X>
__global__ __launch_bounds__(kVecThreads) void diag_csr_kernel(const int32_t *__restrict__ rowptr,
                                                              const int32_t *__restrict__ col,
                                                              const V *__restrict__ val, int32_t n, X *__restrict__ d)
{
    const int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x;
    if (i >= n) return;
    // columns ascend inside a row: binary search for column i
    int32_t lo = rowptr[i], hi = rowptr[i + 1];
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (col[mid] < i) lo = mid + 1;
        else hi = mid;
    }
    if (lo < rowptr[i + 1] && col[lo] == i) d[i] = widen(val[lo]);
}

template <typename V, typename X>
__global__ __launch_bounds__(kVecThreads) void diag_coo_kernel(const int32_t *__restrict__ row,
                                                              const int32_t *__restrict__ col,
                                                              const V *__restrict__ val, int64_t nnz, X *__restrict__ d)
{
    const int64_t p = (int64_t)blockIdx.x * kVecThreads + threadIdx.x;
    if (p < nnz && row[p] == col[p]) d[row[p]] = widen(val[p]);
}

template <typename V, typename X>
__global__ __launch_bounds__(kVecThreads) void diag_ell_kernel(const int32_t *__restrict__ ecol,
                                                              const V *__restrict__ eval, int32_t n, int32_t K,
                                                              int64_t ld, X *__restrict__ d)
{
    const int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x;
    if (i >= n) return;
    for (int32_t k = 0; k < K; ++k) {
        const int64_t q = (int64_t)k * ld + i;
        if (ecol[q] == i) d[i] = widen(eval[q]);
    }
}

template <typename V, typename X>
__global__ __launch_bounds__(kVecThreads) void diag_sellp_kernel(const int32_t *__restrict__ sets,
                                                                const int32_t *__restrict__ scol,
                                                                const V *__restrict__ sval, int32_t n, int32_t C,
                                                                X *__restrict__ d)
{
    const int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x;
    if (i >= n) return;
    const int64_t s = i / C, l = i % C;
    const int32_t k0 = sets[s], w = sets[s + 1] - k0;
    for (int32_t k = 0; k < w; ++k) {
        const int64_t q = ((int64_t)k0 + k) * C + l;
        if (scol[q] == i) d[i] = widen(sval[q]);
    }
}

template <typename X>
__global__ __launch_bounds__(kVecThreads) void dinv_kernel(const X *__restrict__ d, X *__restrict__ dinv, int64_t n,
                                                          KState *st)
{
    const int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x;
    bool bad = false;
    if (i < n) {
        const X v = d[i];
        bad = (v == X(0)) || !__builtin_isfinite(v);
        dinv[i] = X(1) / v;
    }
    if (ballot64(bad) && lane_id() == 0) atomicMax(&st->flag, (int32_t)kBreakdown);
}

template <typename V, typename X>
spx_status jacobi_setup(const spx_matrix &A, X *d, X *dinv, KState *st, hipStream_t stream)
{
    const int64_t n = A.nrows;
    if (n == 0) return SPX_OK;
    const unsigned g = (unsigned)ceil_div(n, kVecThreads);
    fill_vec_kernel<X><<<g, kVecThreads, 0, stream>>>(d, n, X(0));
    switch (A.fmt) {
    case SPX_CSR:
        diag_csr_kernel<V, X><<<g, kVecThreads, 0, stream>>>(A.rowptr, A.colidx, static_cast<const V *>(A.vals),
                                                             A.nrows, d);
        break;
    case SPX_COO:
        if (A.nnz > 0)
            diag_coo_kernel<V, X><<<(unsigned)ceil_div(A.nnz, kVecThreads), kVecThreads, 0, stream>>>(
                A.rowidx, A.colidx, static_cast<const V *>(A.vals), A.nnz, d);
        break;
    case SPX_ELL:
    case SPX_HYB:
        diag_ell_kernel<V, X><<<g, kVecThreads, 0, stream>>>(A.ell_col, static_cast<const V *>(A.ell_val), A.nrows,
                                                             A.ell_width, A.ell_ld, d);
        if (A.fmt == SPX_HYB && A.coo_nnz > 0)
            diag_coo_kernel<V, X><<<(unsigned)ceil_div(A.coo_nnz, kVecThreads), kVecThreads, 0, stream>>>(
                A.rowidx, A.colidx, static_cast<const V *>(A.vals), A.coo_nnz, d);
        break;
    case SPX_SELLP:
        diag_sellp_kernel<V, X><<<g, kVecThreads, 0, stream>>>(A.slice_sets, A.ell_col,
                                                               static_cast<const V *>(A.ell_val), A.nrows,
                                                               A.slice_size, d);
        break;
    default: break;
    }
    dinv_kernel<X><<<g, kVecThreads, 0, stream>>>(d, dinv, n, st);
    SPX_LAUNCHED();
    return SPX_OK;
}

// ------------------------------------------------------------------ dots
template <typename X>
__global__ __launch_bounds__(kVecThreads) void dot_kernel(int64_t n, const X *__restrict__ a, const X *__restrict__ b,
                                                         X *__restrict__ partials, KState *st, int op)
{
    if (st->flag != kRunning) return;
    __shared__ X s_red[kVecThreads / kWave];
    const int64_t base = (int64_t)blockIdx.x * kVecChunk;
    X acc = X(0);
#pragma unroll
    for (int u = 0; u < kVecItems; ++u) {
        const int64_t i = base + threadIdx.x + u * kVecThreads;
        if (i < n) acc += a[i] * b[i];
    }
    X v[1] = {block_sum<X, kVecThreads>(acc, s_red)};
    write_partials<X, 1>(v, partials, gridDim.x, blockIdx.x);
}

template <typename X>
__global__ __launch_bounds__(kVecThreads) void dot2_kernel(int64_t n, const X *__restrict__ a, const X *__restrict__ w,
                                                          X *__restrict__ partials, KState *st, int op)
{
    if (st->flag != kRunning) return;
    __shared__ X s_red[kVecThreads / kWave];
    const int64_t base = (int64_t)blockIdx.x * kVecChunk;
    X aw = X(0), aa = X(0);
#pragma unroll
    for (int u = 0; u < kVecItems; ++u) {
        const int64_t i = base + threadIdx.x + u * kVecThreads;
        if (i < n) {
            aw += a[i] * w[i];
            aa += a[i] * a[i];
        }
    }
    X v[2] = {block_sum<X, kVecThreads>(aw, s_red), block_sum<X, kVecThreads>(aa, s_red)};
    write_partials<X, 2>(v, partials, gridDim.x, blockIdx.x);
}

template <typename X>
__global__ __launch_bounds__(kVecThreads) void residual_kernel(int64_t n, const X *__restrict__ b,
                                                              const X *__restrict__ q, X *__restrict__ r,
                                                              X *__restrict__ partials, KState *st)
{
    __shared__ X s_red[kVecThreads / kWave];
    const int64_t base = (int64_t)blockIdx.x * kVecChunk;
    X acc = X(0);
#pragma unroll
    for (int u = 0; u < kVecItems; ++u) {
        const int64_t i = base + threadIdx.x + u * kVecThreads;
        if (i < n) {
            const X ri = b[i] - q[i];
            r[i] = ri;
            acc += ri * ri;
        }
    }
    X v[1] = {block_sum<X, kVecThreads>(acc, s_red)};
    write_partials<X, 1>(v, partials, gridDim.x, blockIdx.x);
}

template <typename V, typename X>
spx_status spmv_dot(const spx_matrix &A, const X *p, X *q, const X *w, X *partials, KState *st, int op,
                    hipStream_t stream)
{
    if (A.fmt == SPX_CSR) {
        SPX_CHECK((csr_spmv_launch<V, X>(A, p, q, X(1), X(0), w, partials, stream, 1, st, op)));
        return launch_finish<X>(partials, csr_dot_parts(A), 1, st, op, stream);
    }
    if (A.fmt == SPX_SELLP) {
        SPX_CHECK((sellp_spmv_launch<V, X>(A, p, q, X(1), X(0), stream, 1, w, partials, st)));
        return launch_finish<X>(partials, spmv_dot_parts(A), 1, st, op, stream);
    }
    if (A.fmt == SPX_ELL) {
        SPX_CHECK((ell_spmv_launch<V, X>(A, p, q, X(1), X(0), stream, 1, w, partials, st)));
        return launch_finish<X>(partials, spmv_dot_parts(A), 1, st, op, stream);
    }
    SPX_CHECK(spmv_dispatch(A, p, q, 1.0, 0.0, stream));
    dot_kernel<X><<<(unsigned)vec_blocks(A.nrows), kVecThreads, 0, stream>>>(A.nrows, w, q, partials, st, op);
    SPX_LAUNCHED();
    return launch_finish<X>(partials, vec_blocks(A.nrows), 1, st, op, stream);
}

template <typename V, typename X>
spx_status spmv_dot2(const spx_matrix &A, const X *sv, X *t, const X *w, X *partials, KState *st, int op,
                     hipStream_t stream)
{
    if (A.fmt == SPX_CSR) {
        SPX_CHECK((csr_spmv_launch<V, X>(A, sv, t, X(1), X(0), w, partials, stream, 2, st, op)));
        return launch_finish<X>(partials, csr_dot_parts(A), 2, st, op, stream);
    }
    if (A.fmt == SPX_SELLP) {
        SPX_CHECK((sellp_spmv_launch<V, X>(A, sv, t, X(1), X(0), stream, 2, w, partials, st)));
        return launch_finish<X>(partials, spmv_dot_parts(A), 2, st, op, stream);
    }
    if (A.fmt == SPX_ELL) {
        SPX_CHECK((ell_spmv_launch<V, X>(A, sv, t, X(1), X(0), stream, 2, w, partials, st)));
        return launch_finish<X>(partials, spmv_dot_parts(A), 2, st, op, stream);
    }
    SPX_CHECK(spmv_dispatch(A, sv, t, 1.0, 0.0, stream));
    dot2_kernel<X><<<(unsigned)vec_blocks(A.nrows), kVecThreads, 0, stream>>>(A.nrows, t, w, partials, st, op);
    SPX_LAUNCHED();
    return launch_finish<X>(partials, vec_blocks(A.nrows), 2, st, op, stream);
}

template <typename X>
spx_status residual_norm(int64_t n, const X *b, const X *q, X *r, X *partials, KState *st,
                         hipStream_t stream)
{
    residual_kernel<X><<<(unsigned)vec_blocks(n), kVecThreads, 0, stream>>>(n, b, q, r, partials, st);
    SPX_LAUNCHED();
    return launch_finish<X>(partials, vec_blocks(n), 1, st, kOpNorm2, stream);
}

template spx_status jacobi_setup<double, double>(const spx_matrix &, double *, double *, KState *, hipStream_t);
template spx_status jacobi_setup<float, float>(const spx_matrix &, float *, float *, KState *, hipStream_t);
template spx_status jacobi_setup<_Float16, float>(const spx_matrix &, float *, float *, KState *, hipStream_t);
template spx_status spmv_dot<double, double>(const spx_matrix &, const double *, double *, const double *, double *,
                                             KState *, int, hipStream_t);
template spx_status spmv_dot<float, float>(const spx_matrix &, const float *, float *, const float *, float *, KState *,
                                           int, hipStream_t);
template spx_status spmv_dot<_Float16, float>(const spx_matrix &, const float *, float *, const float *, float *,
                                              KState *, int, hipStream_t);
template spx_status spmv_dot2<double, double>(const spx_matrix &, const double *, double *, const double *, double *,
                                              KState *, int, hipStream_t);
template spx_status residual_norm<double>(int64_t, const double *, const double *, double *, double *, KState *,
                                          hipStream_t);
template spx_status residual_norm<float>(int64_t, const float *, const float *, float *, float *, KState *,
                                         hipStream_t);

}  // namespace spx
