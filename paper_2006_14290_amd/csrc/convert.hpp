// convert.hpp -- format conversion, casts and the device prefix scan.
#pragma once

#include "common.hpp"

namespace spx {

int64_t scan_ws_bytes(int64_t n);
template <typename T>
spx_status inclusive_scan(T *a, int64_t n, void *ws, hipStream_t stream);

// row_out[p] = row of entry p of a CSR row pointer with n rows.
spx_status csr_rows_launch(const int32_t *rowptr, int32_t n, int32_t *row_out, hipStream_t stream);
spx_status csr_max_row_len(const spx_matrix &A, int32_t *out, hipStream_t stream);
int64_t convert_ws_bytes(const spx_matrix &src, int32_t dst_fmt, int32_t slice_size);
spx_status convert_plan(const spx_matrix &src, int32_t dst_fmt, int32_t ell_width, int64_t ell_ld, spx_matrix *dst,
                        size_t *ws_bytes, hipStream_t stream);
spx_status convert_run(const spx_matrix &src, spx_matrix &dst, void *ws, size_t ws_bytes, hipStream_t stream);
spx_status cast_values(const double *src, int64_t n, int32_t dst_type, void *dst, int64_t *overflow,
                       hipStream_t stream);

}  // namespace spx
