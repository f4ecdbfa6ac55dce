// small_cg.hpp -- CG for small systems on one work-group (see small_cg.hip).
#pragma once

#include "common.hpp"
#include "krylov.hpp"

namespace spx {

constexpr int kSmallThreads = 1024;           // one work-group
constexpr int kSmallMaxRows = 4 * kSmallThreads;  // rows per solve at most

// Runs the whole float64 CG solve (x0 = 0 or given, M = diag(A) when dinv is
// not null) of a CSR system with at most kSmallMaxRows rows in one launch.
// Reads st->tol2 and st->maxit; writes st->bb, rr (recursive r.r), tmp[0]
// (true r.r, or -1 when not formed), iters, spmv_count and flag. cached:
// the form that holds the matrix in registers, for rows of at most
// kSmallCachedLen entries; it only sets flag = kLongRow (and leaves x alone)
// when a row is longer.
constexpr int kSmallCachedLen = 5;
spx_status small_cg_launch(const spx_matrix &A, const double *b, double *x, const double *dinv, int x0_zero,
                           bool cached, KState *st, hipStream_t stream);

}  // namespace spx
