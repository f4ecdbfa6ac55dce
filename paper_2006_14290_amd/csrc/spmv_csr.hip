// spmv_csr.hip -- load-balanced CSR sparse matrix-vector product for gfx950.
//
// y = alpha * A x + beta * y over the Csr format (Section 1 of the paper
// lists it among the library's formats; Section 4 measures its SpMV).
//
// Work split: the nonzeros are cut into tiles of kTile entries; tile k owns
// every row that STARTS inside [k*kTile, (k+1)*kTile) and processes the whole
// nonzero range of those rows. Each work-group finds its rows with two
// wavefront-cooperative 64-ary searches of the row pointer, streams the
// range in passes of kTile products staged in LDS (coalesced, non-temporal
// loads of values and column indices; gathers of x through the caches), and
// reduces the rows of a pass with subwarps whose size is chosen from the
// number of rows in the pass (Section 3.3's subwarp model: many short rows ->
// small subwarps, one long row -> a whole wavefront). A row longer than a pass
// carries its partial sum in LDS to the next pass. Every row is written once
// by its owner: no atomics, and the summation order is fixed, so results are
// bitwise reproducible.
//
// Bytes moved (the roofline unit): nnz*(sv+4) + (nrows+1)*4 + ncols*sx +
// nrows*sx (+ nrows*sx when beta != 0).
#include "common.hpp"
#include "krylov.hpp"
#include "spmv_csr.hpp"
#include "spmv_csr_tile.hpp"
#include "wave.hpp"

namespace spx {

// One work-group per tile (XCD-remapped block id); see csr_tile. With a
// solver state, a set flag skips the launch.
template <typename V, typename X, int kEpi, int kThreads, int kTile, int kVec, bool kLate>
__global__ __launch_bounds__(kThreads) void csr_spmv_kernel(
    int32_t nrows, int64_t nnz, int64_t ntiles, int64_t grid_padded, const int32_t *__restrict__ rowptr,
    const int32_t *__restrict__ col, const V *__restrict__ val, const X *__restrict__ x, X *__restrict__ y,
    X alpha, X beta, const X *__restrict__ dot_with, X *__restrict__ dot_partials, const int32_t *__restrict__ part,
    KState *__restrict__ st, int op)
{
    if (st != nullptr && st->flag != kRunning) return;
    const int64_t k = xcd_remap(blockIdx.x, grid_padded);
    if (k >= ntiles) return;
    csr_tile<V, X, kEpi, kThreads, kTile, kVec, kLate>(k, nrows, nnz, ntiles, rowptr, col, val, x, y, alpha, beta,
                                                       dot_with, dot_partials, part);
}

// Row-per-subwarp CSR product for short, regular rows (the "classical"
// strategy: a subwarp of kSub lanes per row, kSub the power of two at or
// above the mean row length). A block takes kRowU * kRowThreads / kSub
// consecutive rows; at step u the subwarps of a wavefront hold adjacent rows,
// so every load instruction reads one contiguous stretch of col / val. The
// first kSub entries of all kRowU rows are loaded before the first gather;
// longer rows continue in a loop. Rows are reduced with DPP (fixed order).
// A block repeats this kRowIters times over the following rows.
template <typename V, typename X, int kEpi, int kSub>
__global__ __launch_bounds__(kRowThreads) void csr_rows_kernel(
    int32_t nrows, int64_t nblocks, int64_t grid_padded, const int32_t *__restrict__ rowptr,
    const int32_t *__restrict__ col, const V *__restrict__ val, const X *__restrict__ x, X *__restrict__ y, X alpha,
    X beta, const X *__restrict__ dot_with, X *__restrict__ dot_partials, KState *__restrict__ st)
{
    if (st != nullptr && st->flag != kRunning) return;
    constexpr int kSubs = kRowThreads / kSub;
    constexpr int64_t kStep = (int64_t)kSubs * kRowU;  // rows per block iteration
    const int64_t blk = xcd_remap(blockIdx.x, grid_padded);
    if (blk >= nblocks) return;
    const int tid = threadIdx.x, sw = tid / kSub, sl = tid % kSub;
    X d1 = X(0), d2 = X(0);
    for (int it = 0; it < kRowIters; ++it) {
        const int64_t base = (blk * kRowIters + it) * kStep + sw;
        if (base - sw >= nrows) break;  // uniform across the block
        int32_t a[kRowU], b[kRowU], c[kRowU];
        V v[kRowU];
#pragma unroll
        for (int u = 0; u < kRowU; ++u) {
            const int64_t row = base + (int64_t)u * kSubs;
            a[u] = 0;
            b[u] = 0;
            if (row < nrows) {
                a[u] = rowptr[row];
                b[u] = rowptr[row + 1];
            }
        }
#pragma unroll
        for (int u = 0; u < kRowU; ++u) {
            const int32_t k = a[u] + sl;
            c[u] = -1;
            v[u] = V(0);
            if (k < b[u]) {
                c[u] = ld_stream(col + k);
                v[u] = ld_stream(val + k);
            }
        }
        X sum[kRowU];
#pragma unroll
        for (int u = 0; u < kRowU; ++u) sum[u] = c[u] >= 0 ? widen(v[u]) * x[c[u]] : X(0);
#pragma unroll
        for (int u = 0; u < kRowU; ++u)
            for (int32_t k = a[u] + sl + kSub; k < b[u]; k += kSub)
                sum[u] += widen(ld_stream(val + k)) * x[ld_stream(col + k)];
#pragma unroll
        for (int u = 0; u < kRowU; ++u) {
            const X t = subwave_sum<kSub>(sum[u]);
            const int64_t row = base + (int64_t)u * kSubs;
            if (sl == 0 && row < nrows) {
                X out = alpha * t;
                if (beta != X(0)) out += beta * y[row];
                y[row] = out;
                if constexpr (kEpi >= 1) d1 += out * dot_with[row];
                if constexpr (kEpi >= 2) d2 += out * out;
            }
        }
    }
    if constexpr (kEpi > 0) {
        __shared__ X s_red[kRowThreads / kWave];
        X vv[kEpi];
        vv[0] = block_sum<X, kRowThreads>(d1, s_red);
        if constexpr (kEpi >= 2) vv[kEpi - 1] = block_sum<X, kRowThreads>(d2, s_red);
        write_partials<X, kEpi>(vv, dot_partials, nblocks, blk);
    }
}

// One wavefront per tile boundary k in [0, ntiles]: the first row starting
// at or after k*kCsrTile (nrows for the final boundary) and its offset.
__global__ __launch_bounds__(256) void csr_partition_kernel(int32_t nrows, int64_t nnz, int64_t ntiles,
                                                           const int32_t *__restrict__ rowptr,
                                                           int32_t *__restrict__ part)
{
    const int64_t k = (int64_t)blockIdx.x * (256 / kWave) + threadIdx.x / kWave;
    if (k > ntiles) return;
    int32_t v = (int32_t)nnz;
    int64_t r = nrows;
    if (k < ntiles) r = lower_bound_wave(rowptr, 0, nrows, k * kCsrTile, &v);
    if (lane_id() == 0) {
        part[2 * k] = (int32_t)r;
        part[2 * k + 1] = v;
    }
}

spx_status csr_partition_launch(const spx_matrix &A, int32_t *part, hipStream_t stream)
{
    const int64_t ntiles = csr_tiles(A.nnz);
    csr_partition_kernel<<<(unsigned)ceil_div(ntiles + 1, 256 / kWave), 256, 0, stream>>>(A.nrows, A.nnz, ntiles,
                                                                                          A.rowptr, part);
    SPX_LAUNCHED();
    return SPX_OK;
}

int csr_rows_sub(const spx_matrix &A)
{
    // measured on gfx950: the row-per-subwarp kernel wins only on small
    // matrices (a few launches' worth of work, where the load-balanced
    // kernel's staging and barriers dominate); the load-balanced kernel
    // streams large banded matrices faster
    if (A.nrows <= 0 || A.nrows > kRowMaxRows || A.max_row_len <= 0 || A.nnz <= 0) return 0;
    const int64_t mean = ceil_div(A.nnz, A.nrows);
    int sub = 4;
    while (sub < 64 && sub < mean) sub <<= 1;
    return A.max_row_len <= 2 * sub ? sub : 0;
}

int64_t csr_dot_parts(const spx_matrix &A)
{
    const int sub = csr_rows_sub(A);
    if (sub == 0) return csr_tiles(A.nnz);
    return ceil_div(A.nrows, (int64_t)(kRowThreads / sub) * kRowU * kRowIters);
}

template <typename V, typename X>
spx_status csr_spmv_launch(const spx_matrix &A, const X *x, X *y, X alpha, X beta, const X *dot_with,
                           X *dot_partials, hipStream_t stream, int epi, KState *st, int op)
{
    const V *val = static_cast<const V *>(A.vals);
    const int sub = csr_rows_sub(A);
    if (sub > 0) {
        const int64_t nblocks = csr_dot_parts(A);
        const int64_t grid = pad_to_xcds(nblocks);
#define SPX_ROWS_LAUNCH(E, SUB)                                                                                      \
    csr_rows_kernel<V, X, E, SUB><<<(unsigned)grid, kRowThreads, 0, stream>>>(A.nrows, nblocks, grid, A.rowptr,         \
                                                                               A.colidx, val, x, y, alpha, beta,       \
                                                                               dot_with, dot_partials, st)
#define SPX_ROWS_EPI(SUB)                                                                                            \
    if (epi == 2) SPX_ROWS_LAUNCH(2, SUB);                                                                           \
    else if (epi == 1) SPX_ROWS_LAUNCH(1, SUB);                                                                      \
    else SPX_ROWS_LAUNCH(0, SUB);
        switch (sub) {
        case 4: SPX_ROWS_EPI(4) break;
        case 8: SPX_ROWS_EPI(8) break;
        case 16: SPX_ROWS_EPI(16) break;
        case 32: SPX_ROWS_EPI(32) break;
        default: SPX_ROWS_EPI(64) break;
        }
#undef SPX_ROWS_EPI
#undef SPX_ROWS_LAUNCH
        SPX_LAUNCHED();
        return SPX_OK;
    }
    const int64_t ntiles = csr_tiles(A.nnz);
    const int64_t grid = pad_to_xcds(ntiles);
    // 16-byte value vectors (and matching column vectors) when both arrays
    // are 16-byte aligned, else one entry per load
    constexpr int kVec = 16 / (int)sizeof(V);
    const bool vec = ((reinterpret_cast<uintptr_t>(A.colidx) | reinterpret_cast<uintptr_t>(val)) & 15) == 0;
#define SPX_CSR_LAUNCH(E, VEC)                                                                                   \
    csr_spmv_kernel<V, X, E, kCsrThreads, kCsrTile, VEC, kCsrLateGather><<<(unsigned)grid, kCsrThreads, 0, stream>>>( \
        A.nrows, A.nnz, ntiles, grid, A.rowptr, A.colidx, val, x, y, alpha, beta, dot_with, dot_partials, A.csr_part, \
        st, op)
    if (vec) {
        if (epi == 2) SPX_CSR_LAUNCH(2, kVec);
        else if (epi == 1) SPX_CSR_LAUNCH(1, kVec);
        else SPX_CSR_LAUNCH(0, kVec);
    } else {
        if (epi == 2) SPX_CSR_LAUNCH(2, 1);
        else if (epi == 1) SPX_CSR_LAUNCH(1, 1);
        else SPX_CSR_LAUNCH(0, 1);
    }
#undef SPX_CSR_LAUNCH
    SPX_LAUNCHED();
    return SPX_OK;
}

template spx_status csr_spmv_launch<double, double>(const spx_matrix &, const double *, double *, double, double,
                                                    const double *, double *, hipStream_t, int, KState *, int);
template spx_status csr_spmv_launch<float, float>(const spx_matrix &, const float *, float *, float, float,
                                                  const float *, float *, hipStream_t, int, KState *, int);
template spx_status csr_spmv_launch<_Float16, float>(const spx_matrix &, const float *, float *, float, float,
                                                     const float *, float *, hipStream_t, int, KState *, int);

}  // namespace spx
