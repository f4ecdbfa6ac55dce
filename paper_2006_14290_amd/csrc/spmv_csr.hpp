// spmv_csr.hpp -- launch interface of the load-balanced CSR product.
#pragma once

#include "common.hpp"

namespace spx {

constexpr int kCsrThreads = 512;  // work-group size (8 wavefronts)
constexpr int kCsrTile = 4096;    // nonzeros per tile and per LDS pass

inline int64_t csr_tiles(int64_t nnz) { return nnz > 0 ? ceil_div(nnz, kCsrTile) : 1; }

struct KState;

// y = alpha*A*x + beta*y for a CSR matrix with stored value type V and vector
// type X. epi = 1: also sum_i y_i*dot_with_i; epi = 2: that and sum_i y_i^2,
// one partial per tile in dot_partials[epi][csr_tiles(nnz)] (fixed order).
// With a solver state st, a set st->flag skips the work (the caller reduces
// the partials with finish_kernel).
// Writes the tile partition (2 * (csr_tiles(nnz) + 1) int32) of A.
spx_status csr_partition_launch(const spx_matrix &A, int32_t *part, hipStream_t stream);
inline int64_t csr_partition_bytes(int64_t nnz) { return 2 * (csr_tiles(nnz) + 1) * (int64_t)sizeof(int32_t); }

template <typename V, typename X>
spx_status csr_spmv_launch(const spx_matrix &A, const X *x, X *y, X alpha, X beta, const X *dot_with,
                           X *dot_partials, hipStream_t stream, int epi = 0, KState *st = nullptr, int op = 0,
                           int ticket = 0);

}  // namespace spx
