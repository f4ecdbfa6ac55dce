// spmv.hpp -- launch interfaces of the COO, ELL and hybrid products and the
// shared descriptor check.
#pragma once

#include "common.hpp"

namespace spx {

spx_status check_matrix(const spx_matrix *A, const char *who);
// Canonical-form checks of host CSR arrays (spx_validate_csr_host).
spx_status validate_csr_host(int32_t nrows, int32_t ncols, int64_t nnz, const int32_t *rowptr, const int32_t *col);
// colblock: use A's column-blocked copy when it has one (the public product
// entry points); the solvers call it with false (plain CSR product).
spx_status spmv_dispatch(const spx_matrix &A, const void *x, void *y, double alpha, double beta,
                         hipStream_t stream, bool colblock = false);

constexpr int kCooThreads = 256;
constexpr int kCooTiles = 4;                      // 64-entry tiles per wavefront chunk
constexpr int kCooChunk = 64 * kCooTiles;          // entries per wavefront chunk
constexpr int64_t kCooTargetSpans = 16384;         // wavefront spans to aim for
constexpr int64_t kCooMaxSpan = 8;                 // chunks per span at most
constexpr int kEllThreads = 256;
constexpr int kSellThreads = 256;

template <typename V, typename X>
spx_status coo_spmv_launch(const spx_matrix &A, const X *x, X *y, X alpha, X beta, hipStream_t stream);
struct KState;
// epi = 1: also one partial of sum_i y_i*dot_with_i per work-group
// (ell_dot_parts(A) of them); epi = 2: that and sum_i y_i^2; a set st->flag
// skips the launch.
template <typename V, typename X>
spx_status ell_spmv_launch(const spx_matrix &A, const X *x, X *y, X alpha, X beta, hipStream_t stream, int epi = 0,
                           const X *dot_with = nullptr, X *partials = nullptr, const KState *st = nullptr);
int64_t ell_dot_parts(const spx_matrix &A);
template <typename V, typename X>
spx_status hyb_spmv_launch(const spx_matrix &A, const X *x, X *y, X alpha, X beta, hipStream_t stream);
// epi = 1: also the partials of sum_i y_i*dot_with_i (sellp_dot_parts(A) of
// them); epi = 2: that and sum_i y_i^2 (partials[epi][parts]); a set
// st->flag skips the launch.
int64_t sellp_dot_parts(const spx_matrix &A);
template <typename V, typename X>
spx_status sellp_spmv_launch(const spx_matrix &A, const X *x, X *y, X alpha, X beta, hipStream_t stream,
                             int epi = 0, const X *dot_with = nullptr, X *partials = nullptr,
                             const KState *st = nullptr);

}  // namespace spx
