// transpose.hpp -- CSR transpose on the device (a stable radix sort of the
// column indices; see transpose.hip).
#pragma once

#include "common.hpp"

namespace spx {

// Workspace bytes of transpose_run for a matrix with nnz entries.
int64_t transpose_ws_bytes(int64_t nnz);

// At = A^T for a CSR matrix A (At: ncols x nrows CSR of the same value type,
// its arrays caller-owned: rowptr A.ncols + 1, colidx and vals A.nnz).
// Asynchronous on stream.
spx_status transpose_run(const spx_matrix &A, spx_matrix &At, void *ws, size_t ws_bytes, hipStream_t stream);

}  // namespace spx
