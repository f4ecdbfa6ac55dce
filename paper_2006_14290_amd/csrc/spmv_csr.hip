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
#include "wave.hpp"

namespace spx {

// First index r in [lo, hi] with rowptr[r] >= key, assuming the answer lies in
// [lo, hi]; *val receives rowptr[r]. Executed by one whole wavefront (64-ary
// search: one dependent load per round); every lane returns the answer.
__device__ int64_t lower_bound_wave(const int32_t *__restrict__ rowptr, int64_t lo, int64_t hi, int64_t key,
                                    int32_t *val)
{
    const int l = lane_id();
    while (hi - lo >= kWave) {
        const int64_t step = (hi - lo) / kWave;
        const int64_t p = lo + l * step;
        const int32_t v = rowptr[p];
        const lane_mask_t m = ballot64(v >= key);
        if (m & 1ull) {  // rowptr[lo] >= key and the answer is >= lo
            *val = readlane(v, 0);
            return lo;
        }
        const int j = m ? __builtin_ctzll(m) : kWave;  // first probe at or above key
        const int64_t nlo = lo + (int64_t)(j - 1) * step + 1;
        const int64_t nhi = (j < kWave) ? lo + (int64_t)j * step : hi;
        lo = nlo;
        hi = nhi;
    }
    const int64_t p = lo + l;
    const int32_t v = (p <= hi) ? rowptr[p] : 0;
    const lane_mask_t m = ballot64((p <= hi) && (v >= key));
    const int j = m ? __builtin_ctzll(m) : (int)(hi - lo);
    *val = readlane(v, j);
    return lo + j;
}

// One work-group per tile of kTile nonzeros (XCD-remapped block id). The
// group owns the rows that start inside its tile: it reads their bounds from
// the precomputed partition (or finds them with two wavefront searches),
// issues every value/column load of the pass before the first gather, stages
// the products in LDS and reduces each row with an adaptive subwarp. Rows
// longer than the rest of the pass continue in further passes, carrying their
// partial sum in LDS.
// kEpi: 0 = plain product; 1 = also sum_i y_i*w_i; 2 = also sum_i y_i*w_i
// and sum_i y_i*y_i. With a solver state the sums are reduced across tiles
// (deterministically) and finished by `op`; a set state flag skips the launch.
template <typename V, typename X, int kEpi, int kThreads, int kTile, int kVec, bool kLate>
__global__ __launch_bounds__(kThreads) void csr_spmv_kernel(
    int32_t nrows, int64_t nnz, int64_t ntiles, int64_t grid_padded, const int32_t *__restrict__ rowptr,
    const int32_t *__restrict__ col, const V *__restrict__ val, const X *__restrict__ x, X *__restrict__ y,
    X alpha, X beta, const X *__restrict__ dot_with, X *__restrict__ dot_partials, const int32_t *__restrict__ part,
    KState *__restrict__ st, int op)
{
    if (kEpi > 0 && st != nullptr && st->flag != kRunning) return;
    using A = X;  // accumulation type
    constexpr int kPer = kTile / kThreads;
    constexpr int kNV = kPer / kVec;  // vector loads per thread and pass
    static_assert(kPer % kVec == 0, "tile must split into whole vectors");
    typedef V VV __attribute__((ext_vector_type(kVec)));
    typedef int32_t CV __attribute__((ext_vector_type(kVec)));
    // kLate: the pass's columns and values are staged and x is gathered while
    // the rows are reduced (a subwarp's lanes then sit on neighbouring rows,
    // so a gather instruction touches few cache lines on banded matrices);
    // otherwise the products are formed while staging.
    constexpr size_t kLdsBytes = kLate ? (size_t)kTile * (sizeof(int32_t) + sizeof(V)) : (size_t)kTile * sizeof(A);
    __shared__ __align__(16) unsigned char s_raw[kLdsBytes];
    A *prod = reinterpret_cast<A *>(s_raw);
    V *s_val = reinterpret_cast<V *>(s_raw);
    int32_t *s_col = reinterpret_cast<int32_t *>(s_raw + (size_t)kTile * sizeof(V));
    __shared__ int32_t s_rp[kThreads + 1];
    __shared__ int64_t s_b[4];
    __shared__ A s_carry;

    const int64_t k = xcd_remap(blockIdx.x, grid_padded);
    if (k >= ntiles) return;
    const int tid = threadIdx.x;
    const int wid = tid / kWave;

    int64_t ra, rb, s, e;
    if (part != nullptr) {
        ra = part[2 * k];
        s = part[2 * k + 1];
        rb = part[2 * k + 2];
        e = part[2 * k + 3];
    } else {
        if (wid == 0) {
            int32_t v;
            const int64_t r0 = lower_bound_wave(rowptr, 0, nrows, k * kTile, &v);
            if (lane_id() == 0) {
                s_b[0] = r0;
                s_b[2] = v;
            }
        } else if (wid == 1) {
            int32_t v = (int32_t)nnz;
            const int64_t r1 = (k == ntiles - 1) ? (int64_t)nrows : lower_bound_wave(rowptr, 0, nrows, (k + 1) * kTile, &v);
            if (lane_id() == 0) {
                s_b[1] = r1;
                s_b[3] = v;
            }
        }
        __syncthreads();
        ra = s_b[0];
        rb = s_b[1];
        s = s_b[2];
        e = s_b[3];
    }
    if (tid == 0) s_carry = A(0);

    A dot_acc = A(0), dot_acc2 = A(0);
    int64_t r = ra;          // first row not yet written
    bool continued = false;  // row r holds a partial sum from an earlier pass
    int64_t w0 = s;
    while (true) {
        // A pass covers the kVec-aligned window [a0, a0 + kTile) of the
        // nonzeros; entries before w0 (the previous owner's) or from w1 on
        // are loaded only as far as they share a vector with ours, and are
        // never summed.
        const int64_t a0 = w0 & ~(int64_t)(kVec - 1);
        const int64_t w1 = (e - a0 > kTile) ? a0 + kTile : e;
        const bool last = (w1 == e);
        __syncthreads();  // s_carry / prod / s_rp of the previous pass are consumed
        const A carry_in = s_carry;
        // every value and column load of the pass goes out before the first
        // gather; the row pointers of the first row batch are fetched alongside
        CV cc[kNV];
        VV vv[kNV];
#pragma unroll
        for (int u = 0; u < kNV; ++u) {
            const int64_t base = a0 + ((int64_t)u * kThreads + tid) * kVec;
            if (base < w1 && base + kVec <= nnz) {
                cc[u] = ld_stream(reinterpret_cast<const CV *>(col + base));
                vv[u] = ld_stream(reinterpret_cast<const VV *>(val + base));
            } else {
#pragma unroll
                for (int j = 0; j < kVec; ++j) {
                    const bool ok = base < w1 && base + j < nnz;
                    cc[u][j] = ok ? col[base + j] : 0;
                    vv[u][j] = ok ? val[base + j] : V(0);
                }
            }
        }
        int64_t row_t = r + tid;
        int32_t rp_t = 0, rp_t1 = 0;
        if (row_t < rb) {
            rp_t = rowptr[row_t];
            rp_t1 = rowptr[row_t + 1];
        }
#pragma unroll
        for (int u = 0; u < kNV; ++u) {
            if constexpr (kLate) {
                *reinterpret_cast<VV *>(&s_val[(u * kThreads + tid) * kVec]) = vv[u];
                *reinterpret_cast<CV *>(&s_col[(u * kThreads + tid) * kVec]) = cc[u];
            } else {
                typedef A AV __attribute__((ext_vector_type(kVec)));
                const int64_t base = a0 + ((int64_t)u * kThreads + tid) * kVec;
                AV pv;
#pragma unroll
                for (int j = 0; j < kVec; ++j) pv[j] = (base + j < w1) ? widen(vv[u][j]) * x[cc[u][j]] : A(0);
                *reinterpret_cast<AV *>(&prod[(u * kThreads + tid) * kVec]) = pv;
            }
        }
        // rows of this pass, in batches of up to kThreads rows
        bool first_batch = true;
        bool cont_out = false;
        while (true) {
            if (!first_batch) {
                row_t = r + tid;
                if (row_t < rb) {
                    rp_t = rowptr[row_t];
                    rp_t1 = rowptr[row_t + 1];
                }
            }
            const bool touch = (row_t < rb) && (last || rp_t < w1);
            if (touch) {
                if (tid == 0) s_rp[0] = rp_t;
                s_rp[tid + 1] = rp_t1;
            }
            const int nb = __syncthreads_count(touch);
            if (nb == 0) break;
            // every touching row ends inside the pass except possibly the last one
            const int nfin = (last || s_rp[nb] <= w1) ? nb : nb - 1;
            int size = kThreads / nb;
            size = size >= 64 ? 64 : (size >= 32 ? 32 : (size >= 16 ? 16 : (size >= 8 ? 8 : (size >= 4 ? 4 : (size >= 2 ? 2 : 1)))));
            const int groups = kThreads / size;
            const int g = tid / size;
            const int sl = tid % size;
            for (int j0 = 0; j0 < nb; j0 += groups) {
                const int j = j0 + g;
                A sum = A(0);
                if (j < nb) {
                    const int a = (int)((s_rp[j] > w0 ? s_rp[j] : w0) - a0);
                    const int b = (int)((s_rp[j + 1] < w1 ? s_rp[j + 1] : w1) - a0);
                    if constexpr (kLate) {
#pragma unroll 4
                        for (int p = a + sl; p < b; p += size) sum += widen(s_val[p]) * x[s_col[p]];
                    } else {
                        for (int p = a + sl; p < b; p += size) sum += prod[p];
                    }
                }
                sum = subwave_sum_dyn(sum, size);
                if (j < nb && sl == 0) {
                    if (j == 0 && first_batch && continued) sum += carry_in;
                    const int64_t row = r + j;
                    if (j < nfin) {
                        X out = alpha * sum;
                        if (beta != X(0)) out += beta * y[row];
                        y[row] = out;
                        if constexpr (kEpi >= 1) dot_acc += out * dot_with[row];
                        if constexpr (kEpi >= 2) dot_acc2 += out * out;
                    } else {
                        s_carry = sum;  // the one row continuing into the next pass
                    }
                }
            }
            r += nfin;
            first_batch = false;
            cont_out = nfin < nb;
            if (nfin < kThreads) break;
            __syncthreads();  // s_rp is rewritten by the next batch
        }
        if (last) break;
        continued = cont_out;
        w0 = w1;
    }
    if constexpr (kEpi > 0) {
        __shared__ A s_red[kThreads / kWave];
        A v[kEpi];
        v[0] = block_sum<A, kThreads>(dot_acc, s_red);
        if constexpr (kEpi >= 2) v[kEpi - 1] = block_sum<A, kThreads>(dot_acc2, s_red);
        write_partials<A, kEpi>(v, dot_partials, ntiles, k);
    }
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
    if (kEpi > 0 && st != nullptr && st->flag != kRunning) return;
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
