// solve_ir.hip -- mixed-precision iterative refinement.
//
// Iterative refinement (Moler 1967; the mixed-precision analysis of Carson
// & Higham 2018) around an inner conjugate-gradient solve in float32:
//   x = 0; repeat: r = b - A64 x (float64, true residual) and stop when
//   ||r|| <= tol ||b||; s = ||r||_inf; rhat = fl32(r / s); inner CG on the
//   low-precision matrix (float32 values, or binary16-stored values widened
//   to float32 before each multiply-add; float32 vectors and sums) from zero
//   to relative residual max(inner_tol, tol ||b|| / (2 ||r||)) -- the last
//   step only needs to close the remaining gap; x += s * d (float64).
// Float64 is used only for the outer residual, the update of x and the
// stopping norms; every inner iteration moves float32 vectors and the
// low-precision matrix.
#include <algorithm>
#include <cmath>

#include "solver_common.hpp"
#include "solvers.hpp"

namespace spx {

// max |r_i| in two stages (no atomics): per work-group maxima into part[],
// then one work-group forms their maximum and stores its bit pattern (a
// non-negative double's bits are monotone in its value).
__global__ __launch_bounds__(kVecThreads) void ir_amax_kernel(int64_t n, const double *__restrict__ r,
                                                             double *__restrict__ part)
{
    __shared__ double s_m[kVecThreads / kWave];
    const int64_t base = (int64_t)blockIdx.x * kVecChunk;
    double m = 0.0;
#pragma unroll
    for (int u = 0; u < kVecItems; ++u) {
        const int64_t i = base + threadIdx.x + u * kVecThreads;
        if (i < n) m = fmax(m, fabs(r[i]));
    }
    for (int off = 32; off >= 1; off >>= 1) m = fmax(m, __shfl_xor(m, off));
    if (lane_id() == 0) s_m[threadIdx.x / kWave] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kVecThreads / kWave; ++w) m = fmax(m, s_m[w]);
        part[blockIdx.x] = m;
    }
}

__global__ __launch_bounds__(kFinThreads) void ir_amax_finish(const double *__restrict__ part, int64_t nb,
                                                             unsigned long long *__restrict__ amax_bits)
{
    __shared__ double s_m[kFinThreads / kWave];
    double m = 0.0;
#pragma unroll 8
    for (int64_t i = threadIdx.x; i < nb; i += kFinThreads) m = fmax(m, part[i]);
    for (int off = 32; off >= 1; off >>= 1) m = fmax(m, __shfl_xor(m, off));
    if (lane_id() == 0) s_m[threadIdx.x / kWave] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kFinThreads / kWave; ++w) m = fmax(m, s_m[w]);
        *amax_bits = __builtin_bit_cast(unsigned long long, m);
    }
}

__global__ __launch_bounds__(kVecThreads) void ir_scale_kernel(int64_t n, const double *__restrict__ r,
                                                              const unsigned long long *__restrict__ amax_bits,
                                                              float *__restrict__ rf)
{
    const double s = __builtin_bit_cast(double, *amax_bits);
    const int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x;
    if (i < n) rf[i] = (float)(r[i] / s);
}

__global__ __launch_bounds__(kVecThreads) void ir_update_kernel(int64_t n, double *__restrict__ x,
                                                               const float *__restrict__ d,
                                                               const unsigned long long *__restrict__ amax_bits)
{
    const double s = __builtin_bit_cast(double, *amax_bits);
    const int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x;
    if (i < n) x[i] += s * (double)d[i];
}

__global__ void ir_clear_kernel(int64_t n, double *__restrict__ x, unsigned long long *__restrict__ amax_bits)
{
    const int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x;
    if (i < n) x[i] = 0.0;
    if (i == 0) *amax_bits = 0ull;
}

struct IrBufs {
    double *r, *q, *partials;
    float *rf, *d;
    unsigned long long *amax;
    KState *st;
    int32_t *part64, *partlo;
    void *inner;
    size_t inner_bytes;
};

static size_t inner_bytes_of(const spx_matrix &Alow)
{
    return Alow.val_type == SPX_F16 ? cg_workspace<_Float16, float>(Alow, 0) : cg_workspace<float, float>(Alow, 0);
}

static IrBufs ir_carve(Carve &c, const spx_matrix &A64, const spx_matrix &Alow)
{
    const int64_t n = A64.nrows;
    IrBufs w{};
    w.st = c.take<KState>(1);
    w.r = c.take<double>(n);
    w.q = c.take<double>(n);
    w.rf = c.take<float>(n);
    w.d = c.take<float>(n);
    w.amax = c.take<unsigned long long>(1);
    w.partials = c.take<double>(3 * partial_slots(A64));
    w.part64 = (A64.fmt == SPX_CSR && A64.csr_part == nullptr) ? c.take<int32_t>(csr_partition_bytes(A64.nnz) / 4)
                                                                : nullptr;
    w.partlo = (Alow.fmt == SPX_CSR && Alow.csr_part == nullptr) ? c.take<int32_t>(csr_partition_bytes(Alow.nnz) / 4)
                                                                  : nullptr;
    spx_matrix lo = Alow;
    if (w.partlo) lo.csr_part = reinterpret_cast<const int32_t *>(16);  // partition present for the inner sizing
    w.inner_bytes = inner_bytes_of(lo);
    w.inner = c.take<char>((int64_t)w.inner_bytes);
    return w;
}

size_t ir_workspace(const spx_matrix &A64, const spx_matrix &Alow)
{
    Carve c(nullptr, 0);
    (void)ir_carve(c, A64, Alow);
    return c.off + 256;
}

spx_status ir_run(const spx_matrix &A64_in, const spx_matrix &Alow_in, const double *b, double *x, double tol,
                  double inner_tol, int32_t max_outer, int32_t inner_maxit, int32_t check_every, void *ws,
                  size_t ws_bytes, spx_solve_info *info, hipStream_t user_stream)
{
    SolveEnv *env = nullptr;
    SPX_CHECK(solve_env(&env));
    hipStream_t s = env->stream;
    const int64_t n = A64_in.nrows;
    Carve c(ws, ws_bytes);
    IrBufs w = ir_carve(c, A64_in, Alow_in);
    SPX_REQUIRE(c.fits(), SPX_ERR_ARG, "ir: workspace of %zu bytes is too small (need %zu)", ws_bytes,
                ir_workspace(A64_in, Alow_in));
    spx_matrix A64 = A64_in, Alow = Alow_in;
    *info = spx_solve_info{};
    hipEvent_t e0, e1;
    SPX_HIP(hipEventCreate(&e0));
    SPX_HIP(hipEventCreate(&e1));
    struct EvGuard {
        hipEvent_t a, b;
        ~EvGuard()
        {
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
        }
    } evg{e0, e1};
    SPX_HIP(hipEventRecord(env->join, user_stream));
    SPX_HIP(hipStreamWaitEvent(s, env->join, 0));
    SPX_HIP(hipEventRecord(e0, s));
    if (w.part64) {
        SPX_CHECK(csr_partition_launch(A64, w.part64, s));
        A64.csr_part = w.part64;
    }
    if (w.partlo) {
        SPX_CHECK(csr_partition_launch(Alow, w.partlo, s));
        Alow.csr_part = w.partlo;
    }
    SPX_CHECK(state_init(w.st, tol, 0, s));
    const unsigned ge = (unsigned)ceil_div(n, kVecThreads);
    const unsigned gv = (unsigned)vec_blocks(n);
    ir_clear_kernel<<<ge, kVecThreads, 0, s>>>(n, x, w.amax);
    SPX_LAUNCHED();
    // ||b||^2: the residual of x = 0 is b
    SPX_CHECK(spmv_dispatch(A64, x, w.q, 1.0, 0.0, s));
    SPX_CHECK(residual_norm<double>(n, b, w.q, w.r, w.partials, w.st, s));
    KState hs;
    SPX_CHECK(read_state(env, w.st, &hs));
    const double bb = hs.tmp[0];
    double rn2 = bb;
    spx_status status = SPX_ERR_NOT_CONVERGED;
    SolveSpec inner{inner_tol, inner_maxit, 0, 0, 1, check_every, 0};
    spx_solve_info ii;
    int outer = 0;
    while (true) {
        if (!std::isfinite(rn2)) {
            status = SPX_ERR_NONFINITE;
            set_error("ir: non-finite residual");
            break;
        }
        if (rn2 <= tol * tol * bb) {
            status = SPX_OK;
            break;
        }
        if (outer >= max_outer) {
            set_error("ir: no convergence in %d refinement steps", max_outer);
            break;
        }
        ir_amax_kernel<<<gv, kVecThreads, 0, s>>>(n, w.r, w.partials);
        ir_amax_finish<<<1, kFinThreads, 0, s>>>(w.partials, gv, w.amax);
        ir_scale_kernel<<<ge, kVecThreads, 0, s>>>(n, w.r, w.amax, w.rf);
        SPX_LAUNCHED();
        // the inner solve need not reduce the residual (much) beyond what is
        // left to reach tol ||b||
        inner.tol = std::max(inner_tol, 0.5 * tol * std::sqrt(bb / rn2));
        spx_status is;
        if (Alow.val_type == SPX_F16)
            is = cg_run<_Float16, float>(Alow, w.rf, w.d, inner, w.inner, w.inner_bytes, &ii, s);
        else
            is = cg_run<float, float>(Alow, w.rf, w.d, inner, w.inner, w.inner_bytes, &ii, s);
        info->iters += ii.iters;
        info->spmv_count += ii.spmv_count;
        outer += 1;
        if (is != SPX_OK && is != SPX_ERR_NOT_CONVERGED) {
            status = is;
            break;
        }
        ir_update_kernel<<<ge, kVecThreads, 0, s>>>(n, x, w.d, w.amax);
        SPX_LAUNCHED();
        SPX_CHECK(spmv_dispatch(A64, x, w.q, 1.0, 0.0, s));
        SPX_CHECK(residual_norm<double>(n, b, w.q, w.r, w.partials, w.st, s));
        SPX_CHECK(read_state(env, w.st, &hs));
        info->spmv_count += 1;
        rn2 = hs.tmp[0];
    }
    SPX_HIP(hipEventRecord(e1, s));
    SPX_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    SPX_HIP(hipEventElapsedTime(&ms, e0, e1));
    info->status = status;
    info->outer_iters = outer;
    info->relres_recursive = bb > 0 ? sqrt(rn2 / bb) : 0.0;
    info->relres_true = info->relres_recursive;
    info->device_ms = ms;
    SPX_HIP(hipEventRecord(env->join, s));
    SPX_HIP(hipStreamWaitEvent(user_stream, env->join, 0));
    return status;
}

}  // namespace spx
