// capi_solve.cpp -- C entry points of the Krylov solvers.
#include "common.hpp"
#include "solvers.hpp"
#include "spmv.hpp"

using namespace spx;

static spx_status check_solve(const spx_matrix *A, const void *b, const void *x, const spx_solve_opts *opts,
                              const spx_solve_info *info, const char *who, bool block_jacobi = false)
{
    SPX_CHECK(check_matrix(A, who));
    SPX_REQUIRE(opts != nullptr && info != nullptr, SPX_ERR_ARG, "%s: null opts or info", who);
    SPX_REQUIRE(A->nrows == A->ncols, SPX_ERR_ARG, "%s: matrix is not square", who);
    SPX_REQUIRE(A->nrows == 0 || (b != nullptr && x != nullptr), SPX_ERR_ARG, "%s: null vector", who);
    SPX_REQUIRE(opts->tol >= 0.0, SPX_ERR_ARG, "%s: negative tolerance", who);
    SPX_REQUIRE(opts->maxit >= 0, SPX_ERR_ARG, "%s: negative maxit", who);
    const int32_t pc = opts->precond;
    if (block_jacobi && pc >= 2) {
        SPX_REQUIRE(pc <= 32 && (pc & (pc - 1)) == 0, SPX_ERR_ARG,
                    "%s: block-Jacobi block size %d is not a power of two <= 32", who, pc);
        SPX_REQUIRE(A->fmt == SPX_CSR, SPX_ERR_ARG, "%s: block Jacobi needs a CSR matrix", who);
        return SPX_OK;
    }
    SPX_REQUIRE(pc == 0 || pc == 1, SPX_ERR_ARG, "%s: precond must be 0 or 1%s", who,
                block_jacobi ? " or a block size 2..32" : "");
    return SPX_OK;
}

static SolveSpec spec_of(const spx_solve_opts *o)
{
    return SolveSpec{o->tol, o->maxit, o->restart, o->precond, o->x0_zero, o->check_every, 1};
}

extern "C" spx_status spx_solve_workspace(int32_t solver, const spx_matrix *A, const spx_solve_opts *opts,
                                          size_t *bytes)
{
    clear_error();
    SPX_CHECK(check_matrix(A, "spx_solve_workspace"));
    SPX_REQUIRE(opts != nullptr && bytes != nullptr, SPX_ERR_ARG, "spx_solve_workspace: null argument");
    switch (solver) {
    case SPX_SOLVER_CG: *bytes = cg_workspace<double, double>(*A, opts->precond); return SPX_OK;
    case SPX_SOLVER_BICGSTAB: *bytes = bicgstab_workspace(*A, opts->precond); return SPX_OK;
    case SPX_SOLVER_GMRES:
        SPX_REQUIRE(opts->restart >= 1 && opts->restart <= 62, SPX_ERR_ARG, "GMRES restart must be in [1, 62]");
        *bytes = gmres_workspace(*A, opts->precond, opts->restart);
        return SPX_OK;
    case SPX_SOLVER_BICG: *bytes = bicg_workspace(*A, opts->precond); return SPX_OK;
    case SPX_SOLVER_PIPECG: *bytes = pipecg_workspace(*A, opts->precond); return SPX_OK;
    default: break;
    }
    set_error("spx_solve_workspace: unknown solver %d", solver);
    return SPX_ERR_ARG;
}

extern "C" spx_status spx_cg_solve(const spx_matrix *A, const double *b, double *x, const spx_solve_opts *opts,
                                   void *ws, size_t ws_bytes, spx_solve_info *info, hipStream_t stream)
{
    clear_error();
    SPX_CHECK(check_solve(A, b, x, opts, info, "spx_cg_solve", true));
    SPX_REQUIRE(A->val_type == SPX_F64, SPX_ERR_ARG, "spx_cg_solve: matrix values must be SPX_F64");
    if (A->nrows == 0) {
        *info = spx_solve_info{};
        return SPX_OK;
    }
    return cg_run<double, double>(*A, b, x, spec_of(opts), ws, ws_bytes, info, stream);
}

extern "C" spx_status spx_bicgstab_solve(const spx_matrix *A, const double *b, double *x,
                                         const spx_solve_opts *opts, void *ws, size_t ws_bytes,
                                         spx_solve_info *info, hipStream_t stream)
{
    clear_error();
    SPX_CHECK(check_solve(A, b, x, opts, info, "spx_bicgstab_solve"));
    SPX_REQUIRE(A->val_type == SPX_F64, SPX_ERR_ARG, "spx_bicgstab_solve: matrix values must be SPX_F64");
    if (A->nrows == 0) {
        *info = spx_solve_info{};
        return SPX_OK;
    }
    return bicgstab_run(*A, b, x, spec_of(opts), ws, ws_bytes, info, stream);
}

extern "C" spx_status spx_gmres_solve(const spx_matrix *A, const double *b, double *x, const spx_solve_opts *opts,
                                      void *ws, size_t ws_bytes, spx_solve_info *info, hipStream_t stream)
{
    clear_error();
    SPX_CHECK(check_solve(A, b, x, opts, info, "spx_gmres_solve"));
    SPX_REQUIRE(A->val_type == SPX_F64, SPX_ERR_ARG, "spx_gmres_solve: matrix values must be SPX_F64");
    SPX_REQUIRE(opts->restart >= 1 && opts->restart <= 62, SPX_ERR_ARG, "spx_gmres_solve: restart must be in [1, 62]");
    if (A->nrows == 0) {
        *info = spx_solve_info{};
        return SPX_OK;
    }
    return gmres_run(*A, b, x, spec_of(opts), ws, ws_bytes, info, stream);
}

static spx_status check_ir(const spx_matrix *A64, const spx_matrix *Alow, const char *who)
{
    SPX_CHECK(check_matrix(A64, who));
    SPX_CHECK(check_matrix(Alow, who));
    SPX_REQUIRE(A64->val_type == SPX_F64, SPX_ERR_ARG, "%s: A64 must hold SPX_F64 values", who);
    SPX_REQUIRE(Alow->val_type == SPX_F32 || Alow->val_type == SPX_F16, SPX_ERR_ARG,
                "%s: Alow must hold SPX_F32 or SPX_F16 values", who);
    SPX_REQUIRE(A64->nrows == Alow->nrows && A64->ncols == Alow->ncols && A64->nrows == A64->ncols, SPX_ERR_ARG,
                "%s: A64 and Alow must be square and of the same size", who);
    return SPX_OK;
}

extern "C" spx_status spx_ir_workspace(const spx_matrix *A64, const spx_matrix *Alow, size_t *bytes)
{
    clear_error();
    SPX_CHECK(check_ir(A64, Alow, "spx_ir_workspace"));
    SPX_REQUIRE(bytes != nullptr, SPX_ERR_ARG, "spx_ir_workspace: null output");
    *bytes = ir_workspace(*A64, *Alow);
    return SPX_OK;
}

extern "C" spx_status spx_ir_solve(const spx_matrix *A64, const spx_matrix *Alow, const double *b, double *x,
                                   const spx_ir_opts *opts, void *ws, size_t ws_bytes, spx_solve_info *info,
                                   hipStream_t stream)
{
    clear_error();
    SPX_CHECK(check_ir(A64, Alow, "spx_ir_solve"));
    SPX_REQUIRE(opts != nullptr && info != nullptr, SPX_ERR_ARG, "spx_ir_solve: null opts or info");
    SPX_REQUIRE(A64->nrows == 0 || (b && x), SPX_ERR_ARG, "spx_ir_solve: null vector");
    SPX_REQUIRE(opts->tol >= 0 && opts->inner_tol > 0 && opts->max_outer >= 0 && opts->inner_maxit > 0, SPX_ERR_ARG,
                "spx_ir_solve: bad options");
    if (A64->nrows == 0) {
        *info = spx_solve_info{};
        return SPX_OK;
    }
    return ir_run(*A64, *Alow, b, x, opts->tol, opts->inner_tol, opts->max_outer, opts->inner_maxit,
                  opts->check_every, ws, ws_bytes, info, stream);
}

extern "C" spx_status spx_bicg_solve(const spx_matrix *A, const double *b, double *x, const spx_solve_opts *opts,
                                     void *ws, size_t ws_bytes, spx_solve_info *info, hipStream_t stream)
{
    clear_error();
    SPX_CHECK(check_solve(A, b, x, opts, info, "spx_bicg_solve"));
    SPX_REQUIRE(A->val_type == SPX_F64, SPX_ERR_ARG, "spx_bicg_solve: matrix values must be SPX_F64");
    SPX_REQUIRE(A->fmt == SPX_CSR, SPX_ERR_ARG, "spx_bicg_solve: the matrix must be CSR (A^T is built from it)");
    if (A->nrows == 0) {
        *info = spx_solve_info{};
        return SPX_OK;
    }
    return bicg_run(*A, b, x, spec_of(opts), ws, ws_bytes, info, stream);
}

extern "C" spx_status spx_pipecg_solve(const spx_matrix *A, const double *b, double *x, const spx_solve_opts *opts,
                                       void *ws, size_t ws_bytes, spx_solve_info *info, hipStream_t stream)
{
    clear_error();
    SPX_CHECK(check_solve(A, b, x, opts, info, "spx_pipecg_solve"));
    SPX_REQUIRE(A->val_type == SPX_F64, SPX_ERR_ARG, "spx_pipecg_solve: matrix values must be SPX_F64");
    if (A->nrows == 0) {
        *info = spx_solve_info{};
        return SPX_OK;
    }
    return pipecg_run(*A, b, x, spec_of(opts), ws, ws_bytes, info, stream);
}
