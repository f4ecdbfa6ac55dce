// solver_common.hpp -- host helpers and vector kernels shared by the Krylov
// drivers: workspace carving, the Jacobi diagonal, the per-thread solve
// stream and pinned state mirror, and elementwise/reduction kernels.
#pragma once

#include "common.hpp"
#include "krylov.hpp"
#include "spmv.hpp"
#include "spmv_csr.hpp"

namespace spx {

constexpr int kVecThreads = 256;
constexpr int kVecItems = 4;                           // elements per thread
constexpr int kVecChunk = kVecThreads * kVecItems;     // elements per work-group

inline int64_t vec_blocks(int64_t n) { return n > 0 ? ceil_div(n, kVecChunk) : 1; }

// Partials written by the fused product + dot of A (CSR: one per tile;
// SELL-P: one per slice; other formats: the separate dot kernel's blocks),
// and the partials slots a solver needs (at least one vector pass).
inline int64_t spmv_dot_parts(const spx_matrix &A)
{
    if (A.fmt == SPX_CSR) return csr_dot_parts(A);
    if (A.fmt == SPX_SELLP) return sellp_dot_parts(A);
    if (A.fmt == SPX_ELL) return ell_dot_parts(A);
    return vec_blocks(A.nrows);
}
inline int64_t partial_slots(const spx_matrix &A)
{
    const int64_t a = spmv_dot_parts(A), b = vec_blocks(A.nrows);
    return a > b ? a : b;
}

// Bump allocator over a caller-provided workspace (256-byte aligned pieces).
struct Carve {
    char *base;
    size_t off = 0;
    size_t cap;
    explicit Carve(void *p, size_t c) : base(static_cast<char *>(p)), cap(c) {}
    template <typename T>
    T *take(int64_t count)
    {
        off = (off + 255) & ~size_t(255);
        T *p = reinterpret_cast<T *>(base ? base + off : nullptr);
        off += (size_t)(count > 0 ? count : 1) * sizeof(T);
        return p;
    }
    bool fits() const { return off <= cap; }
};

// Per-thread resources of a blocking solve: a private non-blocking stream
// (default priority) used for graph capture, and a pinned mirror of KState.
struct SolveEnv {
    hipStream_t stream = nullptr;
    KState *host_state = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr, join = nullptr;
};
spx_status solve_env(SolveEnv **env);

// Reads the device state into the pinned mirror (synchronizes the stream).
spx_status read_state(SolveEnv *env, const KState *dst, KState *out);

// Device state initialisation (fill kernel; no memset so it can be captured).
spx_status state_init(KState *st, double tol, int32_t maxit, hipStream_t stream);
spx_status state_set_flag(KState *st, int32_t flag, hipStream_t stream);

// a[0..n) = v (a kernel, so it can be captured).
template <typename X>
spx_status fill_vector(X *a, int64_t n, X v, hipStream_t stream);

// y = A x for any format; with a solver state, a set flag skips the product
// (CSR, ELL and SELL-P kernels; other formats always run).
template <typename V, typename X>
spx_status spmv_st(const spx_matrix &A, const X *x, X *y, KState *st, hipStream_t stream);

// dinv = 1 / diag(A) for any format; sets st->flag = kBreakdown on a zero,
// missing or non-finite diagonal entry (checked by the caller after a read).
template <typename V, typename X>
spx_status jacobi_setup(const spx_matrix &A, X *diag_tmp, X *dinv, KState *st, hipStream_t stream);

// Capture `body` (a sequence of launches on stream) into an executable graph.
template <typename F>
spx_status capture_graph(hipStream_t stream, hipGraphExec_t *exec, F &&body)
{
    hipGraph_t g = nullptr;
    SPX_HIP(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
    spx_status s = body();
    hipError_t e = hipStreamEndCapture(stream, &g);
    if (s != SPX_OK) {
        if (g) (void)hipGraphDestroy(g);
        return s;
    }
    if (e != hipSuccess) {
        set_error("hipStreamEndCapture: %s", hipGetErrorString(e));
        return SPX_ERR_HIP;
    }
    e = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        set_error("hipGraphInstantiate: %s", hipGetErrorString(e));
        return SPX_ERR_HIP;
    }
    return SPX_OK;
}

struct GraphGuard {
    hipGraphExec_t exec = nullptr;
    ~GraphGuard()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
    }
};

// Status of a finished solve from the device flag.
inline spx_status status_of_flag(int32_t flag)
{
    switch (flag) {
    case kConverged:
    case kHalfConverged:
    case kZeroRhs: return SPX_OK;
    case kBreakdown: return SPX_ERR_BREAKDOWN;
    case kNonfinite: return SPX_ERR_NONFINITE;
    case kMaxit: return SPX_ERR_NOT_CONVERGED;
    default: return SPX_ERR_NOT_CONVERGED;
    }
}

// Generic product q = A p (any format) plus the deterministic sum w.q
// finished by `op`; CSR fuses the sum into the product's epilogue.
template <typename V, typename X>
spx_status spmv_dot(const spx_matrix &A, const X *p, X *q, const X *w, X *partials, KState *st, int op,
                    hipStream_t stream);

// t = A s plus the two sums t.s and t.t finished by `op` (CSR: fused epilogue).
template <typename V, typename X>
spx_status spmv_dot2(const spx_matrix &A, const X *sv, X *t, const X *w, X *partials, KState *st, int op,
                     hipStream_t stream);

// r = b - q (q = A x) with ||r||^2 finished into st->tmp[0] (kOpNorm2).
template <typename X>
spx_status residual_norm(int64_t n, const X *b, const X *q, X *r, X *partials, KState *st,
                         hipStream_t stream);

}  // namespace spx
