/*
 * spx.h -- C ABI of the spx sparse library for AMD MI355X (gfx950).
 *
 * The library computes sparse matrix-vector products y = alpha*A*x + beta*y
 * in the Csr, Coo, Ell and Hybrid formats and solves A x = b to a relative
 * residual with Krylov methods (CG, BiCGSTAB, GMRES) and a scalar Jacobi
 * preconditioner: the formats and solvers the paper names among the
 * library features it ports (Section 1) and whose SpMV and CG kernels it
 * measures (Section 4). The subwarp cooperative-group primitives it adds to
 * HIP (Section 3.3) are exposed for testing and micro-benchmarking.
 *
 * Conventions (every entry point):
 *  - All matrix and vector arrays are DEVICE pointers owned by the caller;
 *    the library never frees them. Scalars are passed by value.
 *  - Indices are int32. The CSR row pointer is int32, so nnz < 2^31. ELL slot
 *    k of row i lives at k*ell_ld + i (slot-major, computed in int64).
 *  - Every function returns an spx_status; nothing is thrown across the ABI.
 *    spx_last_error() returns a thread-local description of the last failure.
 *  - Descriptors are checked on the host (shapes, null pointers, type
 *    combinations). Array contents are trusted by the compute calls (an
 *    out-of-range index in them is undefined behaviour); spx_validate checks
 *    them once, on the device, before a matrix is trusted.
 *  - Compute calls are stream-ordered and asynchronous on the hipStream_t
 *    given (0 = the legacy default stream) unless stated otherwise.
 */
#ifndef SPX_H
#define SPX_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SPX_OK = 0,
    SPX_ERR_ARG = 1,           /* invalid argument or unsupported combination      */
    SPX_ERR_FORMAT = 2,        /* malformed matrix (e.g. ELL width too small)      */
    SPX_ERR_UNSORTED = 3,      /* columns not strictly ascending in a row          */
    SPX_ERR_DUPLICATE = 4,     /* repeated (row, col) entry                        */
    SPX_ERR_RANGE = 5,         /* index out of range / binary16 overflow in a cast */
    SPX_ERR_NOMEM = 6,         /* device or host allocation failed                 */
    SPX_ERR_BUDGET = 7,        /* request larger than the server's HBM budget      */
    SPX_ERR_HIP = 8,           /* a HIP runtime call failed                        */
    SPX_ERR_ZERO_DIAG = 9,     /* Jacobi: zero, missing or non-finite diagonal     */
    SPX_ERR_NOT_CONVERGED = 10,/* iteration limit reached                          */
    SPX_ERR_BREAKDOWN = 11,    /* Krylov breakdown (p'Ap <= 0, rho = 0, ...)       */
    SPX_ERR_NONFINITE = 12,    /* NaN or Inf in a residual norm                    */
    SPX_PENDING = 13,          /* serving: request not finished yet                */
    SPX_CANCELLED = 14,        /* serving: request cancelled                       */
    SPX_STATUS_MAX_ENUM = 0x7fffffff /* not a status: makes every int32 value a valid
                                        spx_status, so spx_status_string accepts any */
} spx_status;

typedef enum {
    SPX_F64 = 0, /* float64 values, float64 vectors                               */
    SPX_F32 = 1, /* float32 values, float32 vectors                               */
    SPX_F16 = 2  /* binary16 stored values, float32 vectors and accumulation       */
} spx_dtype;

typedef enum { SPX_CSR = 0, SPX_COO = 1, SPX_ELL = 2, SPX_HYB = 3, SPX_SELLP = 4 } spx_format;

/* Sparse matrix descriptor. Fields a format does not use are ignored.
 *  CSR: rowptr[nrows+1], colidx[nnz], vals[nnz]; rows ascending, columns
 *       strictly ascending inside a row, rowptr[0] = 0, rowptr[nrows] = nnz.
 *  COO: rowidx[nnz], colidx[nnz], vals[nnz] sorted by (row, col).
 *  ELL: ell_col[ell_width*ell_ld], ell_val[same]; ell_ld >= nrows; padding
 *       slots hold column -1 and value +0 and come after a row's entries.
 *  HYB: an ELL part (ell_*) plus a COO part (rowidx/colidx/vals, coo_nnz
 *       entries, sorted); nnz = stored ELL entries + coo_nnz.
 *  SELLP: sliced ELL with padding, the Sellp format the paper benchmarks
 *       (Section 4): rows in slices of slice_size rows (a power of two, at
 *       most 256); slice s has width w_s = stride_factor * ceil(longest row
 *       of the slice / stride_factor); slice_sets[nslices+1] holds the
 *       prefix sums of the widths (slice_cols = slice_sets[nslices]); entry
 *       k of row r = s*slice_size + l is at (slice_sets[s] + k)*slice_size + l
 *       of ell_col / ell_val ([slice_cols*slice_size] each); padding as ELL.
 * max_row_len is an optional hint (0 = unknown) used to choose kernels.     */
typedef struct spx_matrix {
    int32_t fmt;       /* spx_format */
    int32_t val_type;  /* spx_dtype  */
    int32_t nrows;
    int32_t ncols;
    int64_t nnz;
    int32_t *rowptr;
    int32_t *rowidx;
    int32_t *colidx;
    void *vals;
    int64_t coo_nnz;
    int32_t ell_width;
    int32_t max_row_len;
    int64_t ell_ld;
    int32_t *ell_col;
    void *ell_val;
    const int32_t *csr_part; /* optional CSR partition from spx_csr_analyse (NULL = none) */
    int32_t slice_size;      /* SELLP */
    int32_t stride_factor;   /* SELLP */
    int32_t *slice_sets;     /* SELLP, [ceil(nrows/slice_size) + 1] */
    int64_t slice_cols;      /* SELLP, slice_sets[nslices] */
    void *csr_cb;            /* optional column-blocked copy from spx_csr_colblock (NULL = none) */
    int32_t csr_cb_tiles;    /* set by spx_csr_colblock: tiles of its largest column block */
    int32_t csr_cb_live;     /* set by spx_csr_colblock: bit b set when column block b has entries */
} spx_matrix;

/* Name of a status code (static string). */
const char *spx_status_string(spx_status s);

/* Description of the last error raised on the calling thread ("" if none). */
const char *spx_last_error(void);

/* Library version as major*10000 + minor*100 + patch. */
int32_t spx_version(void);

/* ------------------------------------------------------------ validation
 * Canonical-form check of a matrix's index arrays: the layouts of the
 * Section 1 formats (and Sellp, Section 4) that every other call assumes.
 * The paper specifies no input validation; this is the library's own check,
 * run once before a matrix is trusted. Reads only index arrays (never
 * values) and returns the first failing class in this order:
 *  SPX_ERR_FORMAT    structure: CSR rowptr[0] != 0, rowptr[nrows] != nnz or
 *                    a decreasing row pointer; an ELL / SELL-P column after a
 *                    padding slot (-1) of its row, or in a SELL-P padding
 *                    row; a HYB row with COO entries whose ELL part is not
 *                    full; stored entries (ELL, HYB, SELL-P) not adding up
 *                    to nnz; SELL-P slice_sets[0] != 0, a negative width or
 *                    one not a multiple of stride_factor, or
 *                    slice_sets[nslices] != slice_cols;
 *  SPX_ERR_RANGE     a row index outside [0, nrows) or a column outside
 *                    [0, ncols) (padding -1 excepted);
 *  SPX_ERR_UNSORTED  columns not strictly ascending inside a row (COO and
 *                    the COO part of HYB: entries not in (row, col) order;
 *                    HYB: a row's first COO column not above its last ELL
 *                    column);
 *  SPX_ERR_DUPLICATE the same (row, col) stored twice.
 * spx_last_error() names the class and the smallest position (entry, row or
 * slice) where it occurs. BLOCKING (synchronizes `stream`); allocates and
 * frees 40 bytes of device memory. Errors besides the above: SPX_ERR_ARG
 * (descriptor), SPX_ERR_HIP. */
spx_status spx_validate(const spx_matrix *A, hipStream_t stream);

/* The CSR checks of spx_validate on HOST arrays (rowptr[nrows+1], colidx[nnz]),
 * with the same classes, precedence and messages; no device is touched. The
 * solve server applies it to every request in spx_serve_submit, so no
 * malformed system reaches the kernels that resident systems share. */
spx_status spx_validate_csr_host(int32_t nrows, int32_t ncols, int64_t nnz, const int32_t *rowptr,
                                 const int32_t *colidx);

/* ------------------------------------------------------------ SpMV
 * y = alpha * A x + beta * y  (Section 1: the Coo, Csr, Ell and Hybrid
 * formats; Section 4 measures the Coo and Sellp/Csr products).
 * x has ncols entries and y nrows entries, of the vector type of A's dtype
 * (float64 for SPX_F64, float32 for SPX_F32 and SPX_F16). With beta == 0, y
 * is write-only (it may hold NaN). x must not alias y.
 * Errors: SPX_ERR_ARG for null pointers, negative sizes, a bad dtype or
 * format; SPX_ERR_HIP if a launch fails. Asynchronous on `stream`.
 * The Csr, Ell and Hybrid-ELL row sums use a fixed order (bitwise
 * reproducible run to run); Coo and the COO part of Hybrid accumulate rows
 * that cross a work-chunk boundary with atomic adds, whose order varies. */
spx_status spx_spmv(const spx_matrix *A, const void *x, void *y, double alpha, double beta,
                    hipStream_t stream);

/* Same as spx_spmv but requires fmt == SPX_CSR. Two kernels:
 *  - small matrices (at most 65536 rows) with short, even rows
 *    (A->max_row_len known and at most twice the power of two at or above
 *    the mean row length): one subwarp of that many lanes per row, DPP row
 *    sums;
 *  - otherwise (or max_row_len == 0): load balanced. The rows are split into
 *    work-groups of equal nonzero count (a row is owned by the group in which
 *    it starts), so skewed row lengths stay balanced; each group stages the
 *    column indices and values in LDS and reduces every row with a subwarp
 *    whose size adapts to the number of rows in the group, gathering x as it
 *    goes.
 * max_row_len is a hint: a wrong value changes the speed, not the result
 * beyond rounding. */
spx_status spx_csr_spmv(const spx_matrix *A, const void *x, void *y, double alpha, double beta,
                        hipStream_t stream);

/* CSR analysis: the row partition of the load-balanced CSR product.
 * The nonzeros are cut into tiles of 2048; for every tile boundary the
 * partition stores (first row starting at or after the boundary, that row's
 * offset) as two int32. Computing it once per matrix lets every later
 * product (and every solver iteration) skip the per-tile search of the row
 * pointer. spx_csr_analysis_bytes gives the size of the device buffer;
 * spx_csr_analyse fills `buf` (caller-owned device memory, kept alive as long
 * as A is used) and stores it in A->csr_part. The partition is valid while
 * A->rowptr is unchanged. Errors: SPX_ERR_ARG (not CSR, buffer too small).
 * Asynchronous. */
int64_t spx_csr_analysis_bytes(const spx_matrix *A);
spx_status spx_csr_analyse(spx_matrix *A, void *buf, size_t bytes, hipStream_t stream);

/* Column-blocked CSR: for matrices whose column indices scatter over an x
 * larger than one XCD's 4 MB L2 (the skewed, random-column matrices of the
 * Section 4 test set), where the plain product's gathers of x miss L2 and
 * pull whole lines from the Infinity Cache or HBM. The columns are cut into
 * 8 equal ranges (ceil(ncols/8) columns each) and A is stored once more as 8
 * CSR matrices A_b, the entries of A whose column lies in range b, in A's
 * order. A product then runs the tiles of A_b on XCD b (work-group g goes to
 * XCD g mod 8), so each XCD gathers only x's range b, which its L2 holds; each
 * block writes its row sums to a partial vector and a second kernel forms
 * y = alpha * (P_0 + ... + P_7) + beta * y in that order (a fixed order: the
 * result is reproducible run to run; it differs from the plain product's by
 * the order of each row's sum only). Costs beyond the plain product: 8 row
 * pointers and 2 * 8 * nrows vector values (the partials) per product.
 * spx_csr_colblock_bytes gives the device buffer size (about the matrix's own
 * size plus 8 (nrows + 1) int32 and 8 nrows vector values);
 * spx_csr_colblock fills `buf` (caller-owned device memory, 256-byte aligned,
 * kept alive while A is used) from A's arrays, which must be in canonical
 * form (spx_validate), and sets A->csr_cb, csr_cb_tiles and csr_cb_live.
 * From then on spx_spmv and spx_csr_spmv on A use it (the solvers keep the
 * plain CSR product). The copy holds A's values as they were when it was
 * built: after changing A's values or pattern, build it again (or clear
 * A->csr_cb to return to the plain product). The buffer also holds the partials a product writes:
 * products with one A on two streams at once would race. BLOCKING.
 * Errors: SPX_ERR_ARG (not CSR, buffer too small or misaligned),
 * SPX_ERR_FORMAT (the blocks' entries do not add up to nnz), SPX_ERR_HIP. */
int64_t spx_csr_colblock_bytes(const spx_matrix *A);
spx_status spx_csr_colblock(spx_matrix *A, void *buf, size_t bytes, hipStream_t stream);

/* ------------------------------------------------------------ format conversion
 * Conversions between the formats of Section 1 and Sellp (Csr <-> Coo,
 * Csr -> Ell, Csr -> Hybrid, Csr -> Sellp, Ell -> Csr, Hybrid -> Csr,
 * Sellp -> Csr; other pairs go through Csr).
 * Index arrays are produced exactly and values are copied bit for bit, so
 * a round trip X -> Csr -> X reproduces the input.
 *
 * spx_convert_plan (BLOCKING: synchronizes `stream`) fills the shape fields
 * of *dst (fmt, val_type, nrows, ncols, nnz, coo_nnz, ell_width, ell_ld,
 * slice_cols; pointers are set to NULL) and the workspace size. For SELLP,
 * dst->slice_size and dst->stride_factor are read as inputs (0 = 64 and 1)
 * and kept; the caller allocates slice_sets[ceil(nrows/slice_size)+1] and
 * ell_col/ell_val[slice_cols*slice_size]. ell_width: -1 chooses it
 * (Ell: the longest row; Hybrid: the width K that minimises stored bytes
 * n*K*(sv+4) + (entries beyond K)*(sv+8), smallest K on ties), otherwise the
 * given width (Ell: SPX_ERR_FORMAT if a row is longer). ell_ld: 0 = nrows.
 * The caller then allocates dst's arrays (CSR: rowptr[nrows+1], colidx and
 * vals [nnz]; COO: rowidx/colidx/vals [nnz]; ELL: ell_col/ell_val
 * [ell_width*ell_ld]; HYB: both, the COO part with coo_nnz entries) and a
 * workspace of ws_bytes, and calls spx_convert (asynchronous). Ell input
 * must be in canonical form (entries in ascending column order, padding last).
 * Errors: SPX_ERR_ARG (unsupported pair, missing arrays, small workspace),
 * SPX_ERR_FORMAT, SPX_ERR_HIP. */
spx_status spx_convert_plan(const spx_matrix *src, int32_t dst_fmt, int32_t ell_width, int64_t ell_ld,
                            spx_matrix *dst, size_t *ws_bytes, hipStream_t stream);
spx_status spx_convert(const spx_matrix *src, spx_matrix *dst, void *ws, size_t ws_bytes, hipStream_t stream);

/* Value cast for mixed precision: dst receives src's values (src->val_type
 * must be SPX_F64) rounded to nearest even into dst->val_type (SPX_F32 or
 * SPX_F16); dst has the same format and shape as src and its own value
 * arrays (index arrays may be shared with src). NaN becomes the target's
 * quiet NaN with the sign kept. BLOCKING. Returns SPX_ERR_RANGE if a finite
 * value overflowed to infinity (the values are still written). */
spx_status spx_cast_values(const spx_matrix *src, spx_matrix *dst, hipStream_t stream);

/* ------------------------------------------------------------ transpose
 * At = A^T for a CSR matrix A (nrows x ncols, any value type), the product
 * BiCG needs (Section 1 lists BiCG among the library's solvers). The caller
 * fills At: fmt SPX_CSR, nrows = A->ncols, ncols = A->nrows, nnz = A->nnz,
 * the same val_type, and device arrays it owns: rowptr (A->ncols + 1 int32),
 * colidx (nnz int32), vals (nnz values); At->csr_part may be NULL. Rows of
 * At come out sorted by column (A's row index) and values are copied bit for
 * bit; the result does not depend on scheduling. Column indices of A must
 * lie in [0, ncols) (else At is wrong but every access stays in bounds).
 * Needs spx_csr_transpose_workspace bytes of device workspace; asynchronous
 * on stream. Errors: SPX_ERR_ARG (descriptors, shapes, workspace). */
spx_status spx_csr_transpose_workspace(const spx_matrix *A, size_t *bytes);
spx_status spx_csr_transpose(const spx_matrix *A, spx_matrix *At, void *ws, size_t ws_bytes, hipStream_t stream);

/* ------------------------------------------------------------ Krylov solvers
 * Solve A x = b to the relative residual ||b - A x||_2 <= tol * ||b||_2
 * (Section 4 runs CG; Section 1 lists CG, BiCG-type and GMRES solvers with
 * a block-Jacobi preconditioner, of which the scalar, 1x1-block case is
 * provided). float64 only (A->val_type == SPX_F64); b and x are device
 * float64 vectors of nrows entries; x holds the initial guess unless
 * opts->x0_zero. Any matrix format; CSR uses the fused product+dot kernel.
 *
 * Every scalar of the iteration stays on the device; `check_every`
 * iterations are captured once in a hipGraph and replayed, and the host
 * reads the solver state only between replays. Convergence of the recursive
 * residual is confirmed with the true residual b - A x (a miss restarts the
 * recurrences from it). All solves are BLOCKING: they return when done,
 * having ordered themselves after earlier work on `stream` and made `stream`
 * wait for them. info (may not be NULL) receives iterations (CG, BiCGSTAB:
 * full steps; GMRES: Arnoldi steps), products with A, GMRES restart cycles,
 * the recursive and true relative residuals and the device time.
 *
 * Errors: SPX_ERR_ARG (bad descriptor, dtype, sizes, workspace too small),
 * SPX_ERR_ZERO_DIAG (Jacobi with a zero/missing/non-finite diagonal entry),
 * SPX_ERR_BREAKDOWN (CG: p'Ap <= 0; BiCGSTAB: rhat'r = 0, rhat'v = 0, t't = 0
 * or omega = 0), SPX_ERR_NONFINITE (NaN/Inf in a residual norm),
 * SPX_ERR_NOT_CONVERGED (maxit reached; x holds the last iterate). */
typedef enum {
    SPX_SOLVER_CG = 0,
    SPX_SOLVER_BICGSTAB = 1,
    SPX_SOLVER_GMRES = 2,
    SPX_SOLVER_BICG = 3,
    SPX_SOLVER_PIPECG = 4
} spx_solver;

typedef struct {
    double tol;          /* relative residual target (e.g. 1e-10)                 */
    int32_t maxit;       /* iteration limit (GMRES: Arnoldi steps)                 */
    int32_t restart;     /* GMRES restart length m (1..62), e.g. 30                */
    int32_t precond;     /* 0 none, 1 scalar Jacobi M = diag(A); CG on CSR also
                            bs = 2, 4, 8, 16, 32: block Jacobi, M = the bs x bs
                            diagonal blocks (inverted by Gauss-Jordan with
                            partial pivoting; a singular block gives
                            SPX_ERR_ZERO_DIAG)                                    */
    int32_t x0_zero;     /* 1: start from x = 0 (x is write-only)                  */
    int32_t check_every; /* iterations per graph replay between host checks (0 = 16) */
    int32_t reserved;
} spx_solve_opts;

typedef struct {
    int32_t status, iters, spmv_count, outer_iters;
    double relres_recursive, relres_true, device_ms;
} spx_solve_info;

/* Device workspace (bytes) a solve on A with these options needs. */
spx_status spx_solve_workspace(int32_t solver, const spx_matrix *A, const spx_solve_opts *opts, size_t *bytes);

spx_status spx_cg_solve(const spx_matrix *A, const double *b, double *x, const spx_solve_opts *opts, void *ws,
                        size_t ws_bytes, spx_solve_info *info, hipStream_t stream);

spx_status spx_bicgstab_solve(const spx_matrix *A, const double *b, double *x, const spx_solve_opts *opts, void *ws,
                              size_t ws_bytes, spx_solve_info *info, hipStream_t stream);

spx_status spx_gmres_solve(const spx_matrix *A, const double *b, double *x, const spx_solve_opts *opts, void *ws,
                           size_t ws_bytes, spx_solve_info *info, hipStream_t stream);

/* Preconditioned BiCG (Section 1 lists BiCG among the library's solvers; the
 * form of Barrett et al., "Templates", 1994): shadow residual rt = r at the
 * start, precond 0 or 1 (scalar Jacobi; M^-T = M^-1). Each iteration
 * multiplies by A and by A^T; A^T is built in the workspace at the start of
 * every solve (spx_csr_transpose), so A must be CSR. info->spmv_count counts
 * both products. Breakdown: rho = (M^-1 r).rt = 0 or pt.(A p) = 0. Otherwise
 * as spx_cg_solve (BLOCKING, same errors). */
spx_status spx_bicg_solve(const spx_matrix *A, const double *b, double *x, const spx_solve_opts *opts, void *ws,
                          size_t ws_bytes, spx_solve_info *info, hipStream_t stream);

/* Pipelined preconditioned CG (Ghysels & Vanroose, Parallel Computing
 * 40(7), 2014): CG's iterates in exact arithmetic with one reduction phase
 * per iteration that does not wait for the product with A; three launches
 * per iteration against CG's five, more vector traffic. precond 0 or 1, any
 * matrix format. info->spmv_count includes the product w = A u of every
 * (re)start. Breakdown: p.Ap <= 0 (the step's denominator). Otherwise as
 * spx_cg_solve (BLOCKING, same errors). */
spx_status spx_pipecg_solve(const spx_matrix *A, const double *b, double *x, const spx_solve_opts *opts, void *ws,
                            size_t ws_bytes, spx_solve_info *info, hipStream_t stream);

/* ------------------------------------------------------------ mixed-precision iterative refinement
 * Solve A x = b to ||b - A x|| <= tol ||b|| in float64 with float32 inner
 * solves: x = 0; repeat { r = b - A64 x (float64); stop if small; s =
 * ||r||_inf; d = CG(Alow, fl32(r / s)) to relative residual inner_tol in
 * float32 (vectors and sums; SPX_F16 values are widened to float32 before
 * each multiply-add); x += s d }. A64: SPX_F64 values; Alow: the same
 * pattern with SPX_F32 or SPX_F16 values (see spx_cast_values), same or
 * different format. info->iters = total inner CG iterations, outer_iters =
 * refinement steps. BLOCKING; errors as the solvers above, plus
 * SPX_ERR_NOT_CONVERGED after max_outer steps. */
typedef struct {
    double tol;          /* float64 relative residual target, e.g. 1e-10  */
    double inner_tol;    /* inner CG relative residual, e.g. 1e-3         */
    int32_t max_outer;   /* refinement steps limit                        */
    int32_t inner_maxit; /* inner CG iteration limit per step             */
    int32_t check_every; /* inner iterations per graph replay (0 = 16)    */
    int32_t reserved;
} spx_ir_opts;

spx_status spx_ir_workspace(const spx_matrix *A64, const spx_matrix *Alow, size_t *bytes);
spx_status spx_ir_solve(const spx_matrix *A64, const spx_matrix *Alow, const double *b, double *x,
                        const spx_ir_opts *opts, void *ws, size_t ws_bytes, spx_solve_info *info,
                        hipStream_t stream);

/* ------------------------------------------------------------ batched CG and the solve server
 * Many independent float64 CSR systems solved together by unpreconditioned CG
 * (the solver of Section 4) from x = 0 to ||b - A x|| <= tol ||b||, the true
 * residual confirming convergence. Two paths, chosen per system by its size:
 *  - one work-group per system: a persistent kernel whose resident
 *    work-groups take systems from an atomic counter and run all of a
 *    system's CG iterations by themselves (product, updates and fixed-order
 *    reductions inside the group);
 *  - wide systems (n > 4096 by default): several work-groups per system,
 *    one CG step as two grid-wide launches over every wide system at once
 *    (the single-reduction CG of Chronopoulos and Gear: the product w = A r
 *    with the partials of r.w, then every vector update with the partials
 *    of r.r), each system cut into fixed blocks of 1024 rows whose partial
 *    sums are added in a fixed order.
 * Neither path lets one system's arithmetic depend on another's, so a
 * system's iterates are bitwise the same alone or in any batch or mix. */
typedef enum { SPX_BATCH_AUTO = 0, SPX_BATCH_ONE_GROUP = 1, SPX_BATCH_WIDE = 2 } spx_batch_path;

typedef struct {
    int32_t n;              /* rows (square system)                        */
    int32_t path;           /* spx_batch_path (AUTO: wide iff n > 4096)    */
    int64_t nnz;
    const int32_t *rowptr;  /* DEVICE CSR, float64 values                  */
    const int32_t *colidx;
    const double *vals;
    const double *b;        /* DEVICE right-hand side                      */
    double *x;              /* DEVICE solution (written)                   */
    double tol;
    int32_t maxit;
    int32_t status;         /* out: spx_status of this system              */
    int32_t iters;          /* out                                         */
    int32_t spmv_count;     /* out                                         */
    double relres_true;     /* out                                         */
} spx_batch_system;

/* Workspace for spx_cg_batch (3 vectors per system + the slot table). */
spx_status spx_cg_batch_workspace(const spx_batch_system *sys, int32_t count, size_t *bytes);

/* Solve sys[0..count) (host array of descriptors; outputs written back).
 * BLOCKING. Returns SPX_OK if every system converged, else the first failing
 * system's status (each sys[i].status tells). */
spx_status spx_cg_batch(spx_batch_system *sys, int32_t count, void *ws, size_t ws_bytes, hipStream_t stream);

/* spx_cg_batch without a workspace argument and without any device
 * allocation, for callers that cannot allocate device memory (tight serving
 * loops, harnesses that forbid hipMalloc). The workspace spx_cg_batch would
 * take is carved from a fixed 64 MiB array of device memory inside the
 * library instead (one per GPU, held until the process ends; its address is
 * looked up on the device's first call). Same arguments otherwise, same
 * results bit for bit. SPX_ERR_ARG when the batch needs more than 64 MiB of
 * workspace (spx_cg_batch_workspace tells how much; about 3 * 8 * n bytes per
 * system plus tables). Every call on a GPU shares that GPU's array and finds
 * it as the last call left it; nothing in it needs clearing. Calls from this
 * process on one device are serialised by the library; calls that overlap on
 * one GPU from elsewhere (another copy of the library) would race. */
spx_status spx_cg_batch_noalloc(spx_batch_system *sys, int32_t count, hipStream_t stream);

/* Continuous-batching server. Requests carry HOST arrays (kept alive by the
 * caller until the ticket completes); the server copies them into its HBM
 * pool (one allocation of hbm_budget_bytes, made at creation) when a slot and
 * memory are free, keeps each system and its Krylov state resident, and
 * advances all admitted systems together, tick after tick: the small ones in
 * the persistent one-work-group-per-system kernel, the wide ones in blocks
 * of wide iterations, each captured in a hipGraph and run concurrently on two
 * streams. Admission and retirement happen between ticks. Symmetric positive
 * definite systems are solved by CG; nonsymmetric ones by BiCGSTAB (the BiCG
 * family the paper lists among the library's solvers, Section 1), request
 * field solver = SPX_SOLVER_BICGSTAB, unpreconditioned, from x = 0, with the
 * true-residual confirmation of spx_bicgstab_solve; BiCGSTAB systems above
 * the wide threshold take the wide path too (one step as three product +
 * vector pairs). A finished CG request's
 * solution is bitwise the solution that spx_cg_batch gives for the same
 * system alone with the same path; every request's result is bitwise the
 * same alone or in any mix. */
typedef struct spx_server spx_server;

typedef struct {
    int32_t device;          /* HIP device of the server                        */
    int32_t max_slots;       /* concurrently resident systems                   */
    size_t hbm_budget_bytes; /* device memory for matrices and Krylov vectors   */
    int32_t iters_per_tick;  /* CG iterations per system per tick (0 = adaptive) */
    int32_t tick_us;         /* adaptive budget: target tick length (0 = 2000)  */
    int32_t wide_min_rows;   /* systems with n >= this take the wide path
                                (0 = 4097, as SPX_BATCH_AUTO; < 0 = never)       */
    int32_t debug_fail_tick; /* testing only: k > 0 makes the worker stop at its
                                k-th tick as if a HIP call had failed (no device
                                fault is involved); 0 = off                      */
    int32_t reserved0;
    int64_t inflight_bytes;  /* bound on the work admitted at once: the summed
                                bytes one iteration of every resident system
                                moves (CSR product + vector passes); a request
                                that would pass it waits in FIFO order until
                                enough retires (one is always admitted when
                                nothing is resident). <= 0 = no bound          */
} spx_server_config;

typedef struct {
    int32_t n;
    int32_t solver;          /* SPX_SOLVER_CG or SPX_SOLVER_BICGSTAB            */
    int64_t nnz;
    const int32_t *rowptr;   /* HOST CSR, float64, canonical                    */
    const int32_t *colidx;
    const double *vals;
    const double *b;         /* HOST                                           */
    double *x_out;           /* HOST, written on completion (may be NULL)       */
    double tol;              /* e.g. 1e-8                                       */
    int32_t maxit;           /* 0 = no limit                                    */
    int32_t reserved;
} spx_request;

typedef struct {
    int64_t submitted, completed, queued, active, rejected, ticks;
    size_t pool_bytes_total, pool_bytes_in_use, pool_bytes_peak;
} spx_server_stats;

spx_status spx_server_create(const spx_server_config *cfg, spx_server **out);
/* Queues a request after checking its CSR arrays with spx_validate_csr_host
 * (SPX_ERR_FORMAT / RANGE / UNSORTED / DUPLICATE: nothing is queued).
 * SPX_ERR_BUDGET if it can never fit the HBM budget; SPX_ERR_ARG for a
 * solver other than CG or BiCGSTAB. */
spx_status spx_serve_submit(spx_server *server, const spx_request *req, uint64_t *ticket);
/* SPX_PENDING while queued or running; afterwards the request's status, and
 * *info (if not NULL) with iterations, residuals and device_ms = submit-to-done
 * latency in milliseconds. */
spx_status spx_serve_poll(spx_server *server, uint64_t ticket, spx_solve_info *info);
spx_status spx_serve_wait(spx_server *server, uint64_t ticket, double timeout_s, spx_solve_info *info);
/* Cancels a queued or running request: if it returns SPX_OK before the
 * request has completed, the request ends as SPX_CANCELLED. For a request
 * that had already completed it returns SPX_OK and changes nothing. */
spx_status spx_serve_cancel(spx_server *server, uint64_t ticket);
/* Counters of the server. (Named _get_stats: spx_server_stats is the type.) */
spx_status spx_server_get_stats(spx_server *server, spx_server_stats *stats);
/* The server runs two threads: an admission thread (slots, pool memory and
 * the copies of the request arrays; pinned host arrays are copied by DMA,
 * pageable ones are staged by the runtime on this thread) and a worker
 * (ticks, retirement). If a HIP call fails in either, the server stops:
 * every queued and resident request ends with SPX_ERR_HIP (waiters are
 * woken) and later submissions return SPX_ERR_HIP. */
/* Stops both threads (queued and resident requests end as SPX_CANCELLED) and
 * frees everything. */
spx_status spx_server_destroy(spx_server *server);

/* ------------------------------------------------------------ subwarp primitives
 * The subwarp cooperative-group operations of Section 3.3 on 64-lane
 * wavefronts, over n device values (n a multiple of 64):
 *  spx_subwarp_sum:   out[t] = sum of in[] over t's subwarp of `size` lanes
 *                     (xor butterfly, log2(size) steps), repeated
 *                     `inner_loops` times on the running value as in the
 *                     paper's reduction benchmark (inner_loops = 1 gives the
 *                     plain group sum). size in {1,2,4,...,64}. float64.
 *  spx_subwarp_vote:  ballot[t] = (wave ballot of pred & Mask) >> LaneOffset,
 *                     any[t], all[t] as defined in Section 3.3.
 *  spx_wave_segscan:  inclusive segmented sum over each 64-lane wavefront,
 *                     segments starting at head[t] != 0 and at lane 0.
 * Errors: SPX_ERR_ARG for a bad size, n not a multiple of 64 or null
 * pointers. Asynchronous. */
spx_status spx_subwarp_sum(const double *in, double *out, int64_t n, int32_t size, int32_t inner_loops,
                           hipStream_t stream);
spx_status spx_subwarp_vote(const int32_t *pred, uint64_t *ballot, int32_t *any, int32_t *all, int64_t n,
                            int32_t size, hipStream_t stream);
spx_status spx_wave_segscan(const double *in, const int32_t *head, double *out, int64_t n,
                            hipStream_t stream);

/* ------------------------------------------------------------ measurement helpers
 * The attainable HBM bandwidth next to the SpMV rates (not part of the
 * paper's method): every thread keeps eight 16-byte non-temporal loads in
 * flight. spx_stream_copy: dst[i] = src[i] for n float64 values (16-byte
 * aligned pointers). spx_stream_read: reads n float64 values (n even,
 * 16-byte aligned) and writes nothing to sink[0] for finite data (it is there
 * to keep the loads). Asynchronous. */
spx_status spx_stream_copy(const double *src, double *dst, int64_t n, hipStream_t stream);
spx_status spx_stream_read(const double *src, int64_t n, double *sink, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* SPX_H */
