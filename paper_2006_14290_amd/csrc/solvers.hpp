// solvers.hpp -- host drivers of the Krylov solvers.
#pragma once

#include "common.hpp"

namespace spx {

struct KState;

struct SolveSpec {
    double tol;
    int32_t maxit;
    int32_t restart;      // GMRES m
    int32_t precond;      // 0 none, 1 scalar Jacobi, bs >= 2 block Jacobi (CG only)
    int32_t x0_zero;
    int32_t check_every;  // iterations per captured graph launch
    int32_t confirm_true; // confirm convergence with the true residual
};

// Block-Jacobi (block size bs, a power of two <= 32; CSR matrices): the
// inverted diagonal blocks, column-major per block, in inv[nblocks*bs*bs].
template <typename V>
spx_status bj_setup(const spx_matrix &A, int32_t bs, double *inv, KState *st, hipStream_t stream);
// z = M^{-1} r, optionally p = z, partial sums of r.z at partials row `row`.
template <typename X>
spx_status bj_apply(int64_t n, int32_t bs, const double *inv, const X *r, X *z, X *p, X *partials, int row,
                    const KState *st, bool check_flag, hipStream_t stream);

template <typename V, typename X>
size_t cg_workspace(const spx_matrix &A, int precond);
template <typename V, typename X>
spx_status cg_run(const spx_matrix &A, const X *b, X *x, const SolveSpec &sp, void *ws, size_t ws_bytes,
                  spx_solve_info *info, hipStream_t user_stream);

size_t bicgstab_workspace(const spx_matrix &A, int precond);
spx_status bicgstab_run(const spx_matrix &A, const double *b, double *x, const SolveSpec &sp, void *ws,
                        size_t ws_bytes, spx_solve_info *info, hipStream_t user_stream);

size_t gmres_workspace(const spx_matrix &A, int precond, int restart);
spx_status gmres_run(const spx_matrix &A, const double *b, double *x, const SolveSpec &sp, void *ws,
                     size_t ws_bytes, spx_solve_info *info, hipStream_t user_stream);

size_t bicg_workspace(const spx_matrix &A, int precond);
spx_status bicg_run(const spx_matrix &A, const double *b, double *x, const SolveSpec &sp, void *ws,
                    size_t ws_bytes, spx_solve_info *info, hipStream_t user_stream);

size_t pipecg_workspace(const spx_matrix &A, int precond);
spx_status pipecg_run(const spx_matrix &A, const double *b, double *x, const SolveSpec &sp, void *ws,
                      size_t ws_bytes, spx_solve_info *info, hipStream_t user_stream);

size_t ir_workspace(const spx_matrix &A64, const spx_matrix &Alow);
spx_status ir_run(const spx_matrix &A64, const spx_matrix &Alow, const double *b, double *x, double tol,
                  double inner_tol, int32_t max_outer, int32_t inner_maxit, int32_t check_every, void *ws,
                  size_t ws_bytes, spx_solve_info *info, hipStream_t user_stream);

}  // namespace spx
