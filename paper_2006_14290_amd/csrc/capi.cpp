// capi.cpp -- status strings, thread-local error text, descriptor checks and
// the format/dtype dispatch of the SpMV entry points.
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "common.hpp"
#include "convert.hpp"
#include "transpose.hpp"
#include "spmv.hpp"
#include "spmv_colblock.hpp"
#include "spmv_csr.hpp"

namespace spx {

static thread_local char g_last_error[512] = "";

void set_error(const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
    va_end(ap);
}

void clear_error() { g_last_error[0] = '\0'; }

spx_status check_matrix(const spx_matrix *A, const char *who)
{
    SPX_REQUIRE(A != nullptr, SPX_ERR_ARG, "%s: null matrix descriptor", who);
    SPX_REQUIRE(A->nrows >= 0 && A->ncols >= 0 && A->nnz >= 0, SPX_ERR_ARG, "%s: negative size", who);
    SPX_REQUIRE(A->val_type >= SPX_F64 && A->val_type <= SPX_F16, SPX_ERR_ARG, "%s: bad val_type %d", who,
                A->val_type);
    switch (A->fmt) {
    case SPX_CSR:
        SPX_REQUIRE(A->rowptr != nullptr, SPX_ERR_ARG, "%s: CSR needs rowptr", who);
        SPX_REQUIRE(A->nnz == 0 || (A->colidx && A->vals), SPX_ERR_ARG, "%s: CSR needs colidx and vals", who);
        SPX_REQUIRE(A->nnz <= INT32_MAX, SPX_ERR_ARG, "%s: CSR nnz exceeds int32", who);
        break;
    case SPX_COO:
        SPX_REQUIRE(A->nnz == 0 || (A->rowidx && A->colidx && A->vals), SPX_ERR_ARG,
                    "%s: COO needs rowidx, colidx and vals", who);
        break;
    case SPX_ELL:
        SPX_REQUIRE(A->ell_width >= 0, SPX_ERR_ARG, "%s: negative ell_width", who);
        SPX_REQUIRE(A->ell_ld >= A->nrows, SPX_ERR_ARG, "%s: ell_ld < nrows", who);
        SPX_REQUIRE(A->ell_width == 0 || A->nrows == 0 || (A->ell_col && A->ell_val), SPX_ERR_ARG,
                    "%s: ELL needs ell_col and ell_val", who);
        break;
    case SPX_HYB:
        SPX_REQUIRE(A->ell_width >= 0 && A->coo_nnz >= 0, SPX_ERR_ARG, "%s: negative HYB sizes", who);
        SPX_REQUIRE(A->ell_ld >= A->nrows, SPX_ERR_ARG, "%s: ell_ld < nrows", who);
        SPX_REQUIRE(A->ell_width == 0 || A->nrows == 0 || (A->ell_col && A->ell_val), SPX_ERR_ARG,
                    "%s: HYB needs ell_col and ell_val", who);
        SPX_REQUIRE(A->coo_nnz == 0 || (A->rowidx && A->colidx && A->vals), SPX_ERR_ARG,
                    "%s: HYB needs its COO arrays", who);
        break;
    case SPX_SELLP:
        SPX_REQUIRE(A->slice_size >= 1 && A->slice_size <= 256 && (A->slice_size & (A->slice_size - 1)) == 0,
                    SPX_ERR_ARG, "%s: SELLP slice_size %d is not a power of two <= 256", who, A->slice_size);
        SPX_REQUIRE(A->stride_factor >= 1, SPX_ERR_ARG, "%s: SELLP stride_factor < 1", who);
        SPX_REQUIRE(A->slice_cols >= 0 && A->slice_cols <= INT32_MAX, SPX_ERR_ARG, "%s: bad SELLP slice_cols", who);
        SPX_REQUIRE(A->nrows == 0 || A->slice_sets != nullptr, SPX_ERR_ARG, "%s: SELLP needs slice_sets", who);
        SPX_REQUIRE(A->slice_cols == 0 || (A->ell_col && A->ell_val), SPX_ERR_ARG,
                    "%s: SELLP needs ell_col and ell_val", who);
        break;
    default:
        SPX_REQUIRE(false, SPX_ERR_ARG, "%s: bad format %d", who, A->fmt);
    }
    return SPX_OK;
}

template <typename V, typename X>
static spx_status spmv_typed(const spx_matrix &A, const void *x, void *y, double alpha, double beta,
                             hipStream_t stream, bool colblock)
{
    const X *xx = static_cast<const X *>(x);
    X *yy = static_cast<X *>(y);
    const X a = static_cast<X>(alpha), b = static_cast<X>(beta);
    switch (A.fmt) {
    case SPX_CSR:
        if (colblock && A.csr_cb != nullptr) return colblock_spmv_launch<V, X>(A, xx, yy, a, b, stream);
        return csr_spmv_launch<V, X>(A, xx, yy, a, b, nullptr, nullptr, stream);
    case SPX_COO: return coo_spmv_launch<V, X>(A, xx, yy, a, b, stream);
    case SPX_ELL: return ell_spmv_launch<V, X>(A, xx, yy, a, b, stream);
    case SPX_HYB: return hyb_spmv_launch<V, X>(A, xx, yy, a, b, stream);
    case SPX_SELLP: return sellp_spmv_launch<V, X>(A, xx, yy, a, b, stream);
    default: break;
    }
    set_error("spmv: bad format");
    return SPX_ERR_ARG;
}

spx_status spmv_dispatch(const spx_matrix &A, const void *x, void *y, double alpha, double beta, hipStream_t stream,
                         bool colblock)
{
    if (A.nrows == 0) return SPX_OK;
    switch (A.val_type) {
    case SPX_F64: return spmv_typed<double, double>(A, x, y, alpha, beta, stream, colblock);
    case SPX_F32: return spmv_typed<float, float>(A, x, y, alpha, beta, stream, colblock);
    case SPX_F16: return spmv_typed<_Float16, float>(A, x, y, alpha, beta, stream, colblock);
    default: break;
    }
    set_error("spmv: bad val_type");
    return SPX_ERR_ARG;
}

}  // namespace spx

using namespace spx;

extern "C" const char *spx_status_string(spx_status s)
{
    switch (s) {
    case SPX_OK: return "SPX_OK";
    case SPX_ERR_ARG: return "SPX_ERR_ARG";
    case SPX_ERR_FORMAT: return "SPX_ERR_FORMAT";
    case SPX_ERR_UNSORTED: return "SPX_ERR_UNSORTED";
    case SPX_ERR_DUPLICATE: return "SPX_ERR_DUPLICATE";
    case SPX_ERR_RANGE: return "SPX_ERR_RANGE";
    case SPX_ERR_NOMEM: return "SPX_ERR_NOMEM";
    case SPX_ERR_BUDGET: return "SPX_ERR_BUDGET";
    case SPX_ERR_HIP: return "SPX_ERR_HIP";
    case SPX_ERR_ZERO_DIAG: return "SPX_ERR_ZERO_DIAG";
    case SPX_ERR_NOT_CONVERGED: return "SPX_ERR_NOT_CONVERGED";
    case SPX_ERR_BREAKDOWN: return "SPX_ERR_BREAKDOWN";
    case SPX_ERR_NONFINITE: return "SPX_ERR_NONFINITE";
    case SPX_PENDING: return "SPX_PENDING";
    case SPX_CANCELLED: return "SPX_CANCELLED";
    default: break;
    }
    return "SPX_UNKNOWN";
}

extern "C" const char *spx_last_error(void) { return g_last_error; }

extern "C" int32_t spx_version(void) { return 100; }

extern "C" spx_status spx_spmv(const spx_matrix *A, const void *x, void *y, double alpha, double beta,
                               hipStream_t stream)
{
    clear_error();
    SPX_CHECK(check_matrix(A, "spx_spmv"));
    SPX_REQUIRE(A->nrows == 0 || (y != nullptr && (A->ncols == 0 || x != nullptr)), SPX_ERR_ARG,
                "spx_spmv: null vector");
    SPX_REQUIRE(x != y || A->nrows == 0, SPX_ERR_ARG, "spx_spmv: x aliases y");
    return spmv_dispatch(*A, x, y, alpha, beta, stream, true);
}

extern "C" spx_status spx_csr_spmv(const spx_matrix *A, const void *x, void *y, double alpha, double beta,
                                   hipStream_t stream)
{
    clear_error();
    SPX_CHECK(check_matrix(A, "spx_csr_spmv"));
    SPX_REQUIRE(A->fmt == SPX_CSR, SPX_ERR_ARG, "spx_csr_spmv: matrix is not CSR");
    SPX_REQUIRE(A->nrows == 0 || (y != nullptr && (A->ncols == 0 || x != nullptr)), SPX_ERR_ARG,
                "spx_csr_spmv: null vector");
    SPX_REQUIRE(x != y || A->nrows == 0, SPX_ERR_ARG, "spx_csr_spmv: x aliases y");
    return spmv_dispatch(*A, x, y, alpha, beta, stream, true);
}

extern "C" int64_t spx_csr_analysis_bytes(const spx_matrix *A)
{
    if (A == nullptr || A->fmt != SPX_CSR || A->nnz < 0) return 0;
    return csr_partition_bytes(A->nnz);
}

extern "C" spx_status spx_csr_analyse(spx_matrix *A, void *buf, size_t bytes, hipStream_t stream)
{
    clear_error();
    SPX_CHECK(check_matrix(A, "spx_csr_analyse"));
    SPX_REQUIRE(A->fmt == SPX_CSR, SPX_ERR_ARG, "spx_csr_analyse: matrix is not CSR");
    SPX_REQUIRE(buf != nullptr, SPX_ERR_ARG, "spx_csr_analyse: null buffer");
    SPX_REQUIRE((int64_t)bytes >= csr_partition_bytes(A->nnz), SPX_ERR_ARG,
                "spx_csr_analyse: buffer of %zu bytes is smaller than the %lld needed", bytes,
                (long long)csr_partition_bytes(A->nnz));
    A->csr_part = nullptr;
    if (A->nrows > 0) SPX_CHECK(csr_partition_launch(*A, static_cast<int32_t *>(buf), stream));
    A->csr_part = static_cast<const int32_t *>(buf);
    return SPX_OK;
}

extern "C" int64_t spx_csr_colblock_bytes(const spx_matrix *A)
{
    if (A == nullptr || A->fmt != SPX_CSR || A->nnz < 0 || A->nrows < 0) return 0;
    return colblock_bytes(*A);
}

extern "C" spx_status spx_csr_colblock(spx_matrix *A, void *buf, size_t bytes, hipStream_t stream)
{
    clear_error();
    SPX_CHECK(check_matrix(A, "spx_csr_colblock"));
    SPX_REQUIRE(A->fmt == SPX_CSR, SPX_ERR_ARG, "spx_csr_colblock: matrix is not CSR");
    return colblock_build(*A, buf, bytes, stream);
}

extern "C" spx_status spx_convert_plan(const spx_matrix *src, int32_t dst_fmt, int32_t ell_width, int64_t ell_ld,
                                       spx_matrix *dst, size_t *ws_bytes, hipStream_t stream)
{
    clear_error();
    SPX_CHECK(check_matrix(src, "spx_convert_plan"));
    SPX_REQUIRE(dst != nullptr && ws_bytes != nullptr, SPX_ERR_ARG, "spx_convert_plan: null output");
    SPX_REQUIRE(dst_fmt >= SPX_CSR && dst_fmt <= SPX_SELLP, SPX_ERR_ARG, "spx_convert_plan: bad format %d", dst_fmt);
    return convert_plan(*src, dst_fmt, ell_width, ell_ld, dst, ws_bytes, stream);
}

extern "C" spx_status spx_convert(const spx_matrix *src, spx_matrix *dst, void *ws, size_t ws_bytes,
                                  hipStream_t stream)
{
    clear_error();
    SPX_CHECK(check_matrix(src, "spx_convert"));
    SPX_CHECK(check_matrix(dst, "spx_convert (dst)"));
    SPX_REQUIRE(src->nrows == dst->nrows && src->ncols == dst->ncols && src->val_type == dst->val_type,
                SPX_ERR_ARG, "spx_convert: dst shape or dtype differs from src");
    SPX_REQUIRE(dst->fmt != SPX_COO || dst->nnz == src->nnz, SPX_ERR_ARG, "spx_convert: dst nnz differs from plan");
    return convert_run(*src, *dst, ws, ws_bytes, stream);
}

extern "C" spx_status spx_csr_transpose_workspace(const spx_matrix *A, size_t *bytes)
{
    clear_error();
    SPX_CHECK(check_matrix(A, "spx_csr_transpose_workspace"));
    SPX_REQUIRE(bytes != nullptr, SPX_ERR_ARG, "spx_csr_transpose_workspace: null bytes");
    SPX_REQUIRE(A->fmt == SPX_CSR, SPX_ERR_ARG, "spx_csr_transpose_workspace: the matrix must be CSR");
    *bytes = (size_t)transpose_ws_bytes(A->nnz);
    return SPX_OK;
}

extern "C" spx_status spx_csr_transpose(const spx_matrix *A, spx_matrix *At, void *ws, size_t ws_bytes,
                                        hipStream_t stream)
{
    clear_error();
    SPX_CHECK(check_matrix(A, "spx_csr_transpose"));
    SPX_CHECK(check_matrix(At, "spx_csr_transpose (At)"));
    SPX_REQUIRE(A->fmt == SPX_CSR && At->fmt == SPX_CSR, SPX_ERR_ARG, "spx_csr_transpose: both matrices must be CSR");
    SPX_REQUIRE(At->nrows == A->ncols && At->ncols == A->nrows && At->nnz == A->nnz && At->val_type == A->val_type,
                SPX_ERR_ARG, "spx_csr_transpose: At must be ncols x nrows with the same nnz and val_type");
    SPX_REQUIRE(A->ncols <= INT32_MAX && A->nrows <= INT32_MAX, SPX_ERR_ARG, "spx_csr_transpose: too many rows");
    return transpose_run(*A, *At, ws, ws_bytes, stream);
}

extern "C" spx_status spx_cast_values(const spx_matrix *src, spx_matrix *dst, hipStream_t stream)
{
    clear_error();
    SPX_CHECK(check_matrix(src, "spx_cast_values"));
    SPX_CHECK(check_matrix(dst, "spx_cast_values (dst)"));
    SPX_REQUIRE(src->val_type == SPX_F64, SPX_ERR_ARG, "spx_cast_values: source must be SPX_F64");
    SPX_REQUIRE(dst->val_type == SPX_F32 || dst->val_type == SPX_F16, SPX_ERR_ARG,
                "spx_cast_values: target must be SPX_F32 or SPX_F16");
    SPX_REQUIRE(src->fmt == dst->fmt && src->nrows == dst->nrows && src->nnz == dst->nnz &&
                    src->ell_width == dst->ell_width && src->ell_ld == dst->ell_ld && src->coo_nnz == dst->coo_nnz &&
                    (src->fmt != SPX_SELLP ||
                     (src->slice_size == dst->slice_size && src->slice_cols == dst->slice_cols)),
                SPX_ERR_ARG, "spx_cast_values: dst shape differs from src");
    int64_t ovf = 0, o = 0;
    if (src->fmt == SPX_CSR || src->fmt == SPX_COO) {
        SPX_CHECK(cast_values(static_cast<const double *>(src->vals), src->nnz, dst->val_type, dst->vals, &o, stream));
        ovf += o;
    } else if (src->fmt == SPX_SELLP) {
        SPX_CHECK(cast_values(static_cast<const double *>(src->ell_val), src->slice_cols * src->slice_size,
                              dst->val_type, dst->ell_val, &o, stream));
        ovf += o;
    } else {
        SPX_CHECK(cast_values(static_cast<const double *>(src->ell_val), (int64_t)src->ell_width * src->ell_ld,
                              dst->val_type, dst->ell_val, &o, stream));
        ovf += o;
        if (src->fmt == SPX_HYB) {
            SPX_CHECK(cast_values(static_cast<const double *>(src->vals), src->coo_nnz, dst->val_type, dst->vals, &o,
                                  stream));
            ovf += o;
        }
    }
    SPX_REQUIRE(ovf == 0, SPX_ERR_RANGE, "spx_cast_values: %lld finite values overflowed", (long long)ovf);
    return SPX_OK;
}
