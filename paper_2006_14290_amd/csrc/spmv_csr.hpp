// spmv_csr.hpp -- launch interface of the load-balanced CSR product.
#pragma once

#include "common.hpp"

namespace spx {

constexpr int kCsrThreads = 256;  // work-group size (4 wavefronts)
constexpr int kCsrTile = 2048;    // nonzeros per tile and per LDS pass
constexpr int kCsrSlack = 64;     // a pass may run this many entries past its tile
constexpr bool kCsrLateGather = true;  // gather x while reducing rows (see csr_spmv_kernel)
constexpr int kRowThreads = 256;  // row-per-subwarp kernel: work-group size
constexpr int kRowU = 4;          // rows per subwarp in the row-per-subwarp kernel
constexpr int kRowIters = 8;      // row groups per work-group in the row-per-subwarp kernel
constexpr int kRowMaxRows = 65536;  // larger matrices take the load-balanced kernel

inline int64_t csr_tiles(int64_t nnz) { return nnz > 0 ? ceil_div(nnz, kCsrTile) : 1; }

struct KState;

// y = alpha*A*x + beta*y for a CSR matrix with stored value type V and vector
// type X. epi = 1: also sum_i y_i*dot_with_i; epi = 2: that and sum_i y_i^2,
// one partial per tile in dot_partials[epi][csr_tiles(nnz)] (fixed order).
// With a solver state st, a set st->flag skips the work (the caller reduces
// the partials with finish_kernel).
// Subwarp width of the row-per-subwarp kernel for A, or 0 when A takes the
// load-balanced kernel: A is small (at most kRowMaxRows rows) and its rows
// are short and even (max_row_len known and at most twice the power of two
// at or above the mean row length).
int csr_rows_sub(const spx_matrix &A);
// Number of dot partials the CSR product with epi > 0 writes for A.
int64_t csr_dot_parts(const spx_matrix &A);

// Writes the tile partition (2 * (csr_tiles(nnz) + 1) int32) of A.
spx_status csr_partition_launch(const spx_matrix &A, int32_t *part, hipStream_t stream);
inline int64_t csr_partition_bytes(int64_t nnz) { return 2 * (csr_tiles(nnz) + 1) * (int64_t)sizeof(int32_t); }

template <typename V, typename X>
spx_status csr_spmv_launch(const spx_matrix &A, const X *x, X *y, X alpha, X beta, const X *dot_with,
                           X *dot_partials, hipStream_t stream, int epi = 0, KState *st = nullptr, int op = 0);

}  // namespace spx
