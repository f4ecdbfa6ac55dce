// spmv_csr.hpp -- launch interface of the load-balanced CSR product.
#pragma once

#include "common.hpp"

namespace spx {

constexpr int kCsrThreads = 512;  // work-group size (8 wavefronts)
constexpr int kCsrTile = 4096;    // nonzeros per tile and per LDS pass

inline int64_t csr_tiles(int64_t nnz) { return nnz > 0 ? ceil_div(nnz, kCsrTile) : 1; }

// y = alpha*A*x + beta*y for a CSR matrix with stored value type V and vector
// type X. If dot_with != nullptr, also writes one partial of sum_i y_i *
// dot_with_i per tile to dot_partials[csr_tiles(nnz)] (fixed order).
// Writes the tile partition (2 * (csr_tiles(nnz) + 1) int32) of A.
spx_status csr_partition_launch(const spx_matrix &A, int32_t *part, hipStream_t stream);
inline int64_t csr_partition_bytes(int64_t nnz) { return 2 * (csr_tiles(nnz) + 1) * (int64_t)sizeof(int32_t); }

template <typename V, typename X>
spx_status csr_spmv_launch(const spx_matrix &A, const X *x, X *y, X alpha, X beta, const X *dot_with,
                           X *dot_partials, hipStream_t stream);

}  // namespace spx
