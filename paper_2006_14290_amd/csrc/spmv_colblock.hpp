// spmv_colblock.hpp -- the column-blocked CSR product (spx_csr_colblock).
#pragma once

#include "common.hpp"

namespace spx {

constexpr int kCbBlocks = 8;  // column blocks, one per XCD

// Columns per block: ceil(ncols / kCbBlocks) (at least 1).
int32_t colblock_width(int32_t ncols);
// Device bytes of the column-blocked copy of A (spx_csr_colblock_bytes).
int64_t colblock_bytes(const spx_matrix &A);
// Builds the copy in buf and records it in A (csr_cb, csr_cb_tiles). BLOCKING.
spx_status colblock_build(spx_matrix &A, void *buf, size_t bytes, hipStream_t stream);
// y = alpha*A*x + beta*y through A's column-blocked copy.
template <typename V, typename X>
spx_status colblock_spmv_launch(const spx_matrix &A, const X *x, X *y, X alpha, X beta, hipStream_t stream);

}  // namespace spx
