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
#include "spmv_csr.hpp"
#include "wave.hpp"

namespace spx {

// First index r in [lo, hi] with rowptr[r] >= key, assuming the answer lies in
// [lo, hi]. Executed by one whole wavefront; every lane returns the answer.
__device__ int64_t lower_bound_wave(const int32_t *__restrict__ rowptr, int64_t lo, int64_t hi, int64_t key)
{
    const int l = lane_id();
    while (hi - lo >= kWave) {
        const int64_t step = (hi - lo) / kWave;
        const int64_t p = lo + l * step;
        const lane_mask_t m = ballot64(rowptr[p] >= key);
        if (m & 1ull) return lo;  // rowptr[lo] >= key and the answer is >= lo
        const int j = m ? __builtin_ctzll(m) : kWave;  // first probe at or above key
        const int64_t nlo = lo + (int64_t)(j - 1) * step + 1;
        const int64_t nhi = (j < kWave) ? lo + (int64_t)j * step : hi;
        lo = nlo;
        hi = nhi;
    }
    const int64_t p = lo + l;
    const bool pred = (p <= hi) && (rowptr[p] >= key);
    const lane_mask_t m = ballot64(pred);
    return m ? lo + __builtin_ctzll(m) : hi;
}

template <typename V, typename X, bool kEpiDot>
__global__ __launch_bounds__(kCsrThreads) void csr_spmv_kernel(
    int32_t nrows, int64_t nnz, int64_t ntiles, int64_t grid_padded, const int32_t *__restrict__ rowptr,
    const int32_t *__restrict__ col, const V *__restrict__ val, const X *__restrict__ x, X *__restrict__ y,
    X alpha, X beta, const X *__restrict__ dot_with, X *__restrict__ dot_partials)
{
    using A = X;  // accumulation type
    __shared__ A prod[kCsrTile];
    __shared__ int32_t s_rp[kCsrThreads + 1];
    __shared__ int64_t s_bounds[2];
    __shared__ A s_carry;
    __shared__ A s_dot[kCsrThreads / kWave];

    const int64_t k = xcd_remap(blockIdx.x, grid_padded);
    if (k >= ntiles) return;
    const int tid = threadIdx.x;
    const int wid = tid / kWave;

    if (wid == 0) {
        const int64_t ra = lower_bound_wave(rowptr, 0, nrows, k * kCsrTile);
        if (lane_id() == 0) s_bounds[0] = ra;
    } else if (wid == 1) {
        const int64_t rb = (k == ntiles - 1) ? (int64_t)nrows : lower_bound_wave(rowptr, 0, nrows, (k + 1) * kCsrTile);
        if (lane_id() == 0) s_bounds[1] = rb;
    }
    if (tid == 0) s_carry = A(0);
    __syncthreads();
    const int64_t ra = s_bounds[0], rb = s_bounds[1];
    const int64_t s = rowptr[ra], e = rowptr[rb];

    A dot_acc = A(0);
    int64_t r = ra;          // first row not yet written
    bool continued = false;  // row r holds a partial sum from an earlier pass
    int64_t w0 = s;
    while (true) {
        const int64_t w1 = (e - w0 > kCsrTile) ? w0 + kCsrTile : e;
        const bool last = (w1 == e);
        const A carry_in = s_carry;  // written before the previous barrier
        // stage products of this pass
        const int cnt = (int)(w1 - w0);
        for (int i = tid; i < cnt; i += kCsrThreads) {
            const int64_t p = w0 + i;
            prod[i] = widen(ld_stream(val + p)) * x[ld_stream(col + p)];
        }
        // rows of this pass, in batches of up to kCsrThreads rows
        bool first_batch = true;
        while (true) {
            const int64_t row_t = r + tid;
            int32_t rp_t = 0, rp_t1 = 0;
            if (row_t < rb) {
                rp_t = rowptr[row_t];
                rp_t1 = rowptr[row_t + 1];
            }
            const bool touch = (row_t < rb) && (last || rp_t < w1);
            const bool fin = touch && (last || rp_t1 <= w1);
            if (touch) {
                if (tid == 0) s_rp[0] = rp_t;
                s_rp[tid + 1] = rp_t1;
            }
            const int nb = __syncthreads_count(touch);
            const int nfin = __syncthreads_count(fin);
            if (nb == 0) break;
            // subwarp size: largest power of two with nb * size <= threads, capped at 64
            int size = kCsrThreads / nb;
            size = size >= 64 ? 64 : (size >= 32 ? 32 : (size >= 16 ? 16 : (size >= 8 ? 8 : (size >= 4 ? 4 : (size >= 2 ? 2 : 1)))));
            const int groups = kCsrThreads / size;
            const int g = tid / size;
            const int sl = tid % size;
            for (int j0 = 0; j0 < nb; j0 += groups) {
                const int j = j0 + g;
                A sum = A(0);
                if (j < nb) {
                    const int64_t a = (s_rp[j] > w0 ? s_rp[j] : w0) - w0;
                    const int64_t b = (s_rp[j + 1] < w1 ? s_rp[j + 1] : w1) - w0;
                    for (int64_t p = a + sl; p < b; p += size) sum += prod[p];
                }
                sum = subwave_sum_dyn(sum, size);
                if (j < nb && sl == 0) {
                    if (j == 0 && first_batch && continued) sum += carry_in;
                    const int64_t row = r + j;
                    if (j < nfin) {
                        X out = alpha * sum;
                        if (beta != X(0)) out += beta * y[row];
                        y[row] = out;
                        if constexpr (kEpiDot) dot_acc += out * dot_with[row];
                    } else {
                        s_carry = sum;  // the one row continuing into the next pass
                    }
                }
            }
            r += nfin;
            first_batch = false;
            __syncthreads();
            if (nfin < kCsrThreads) break;
        }
        continued = (r < rb) && (rowptr[r] < w1);
        if (last) break;
        w0 = w1;
        __syncthreads();
    }
    if constexpr (kEpiDot) {
        dot_acc = wave_sum(dot_acc);
        if (lane_id() == 0) s_dot[wid] = dot_acc;
        __syncthreads();
        if (tid == 0) {
            A t = A(0);
            for (int w = 0; w < kCsrThreads / kWave; ++w) t += s_dot[w];
            dot_partials[k] = t;
        }
    }
}

template <typename V, typename X>
spx_status csr_spmv_launch(const spx_matrix &A, const X *x, X *y, X alpha, X beta, const X *dot_with,
                           X *dot_partials, hipStream_t stream)
{
    const int64_t ntiles = csr_tiles(A.nnz);
    const int64_t grid = pad_to_xcds(ntiles);
    const V *val = static_cast<const V *>(A.vals);
    if (dot_with)
        csr_spmv_kernel<V, X, true><<<dim3((unsigned)grid), dim3(kCsrThreads), 0, stream>>>(
            A.nrows, A.nnz, ntiles, grid, A.rowptr, A.colidx, val, x, y, alpha, beta, dot_with, dot_partials);
    else
        csr_spmv_kernel<V, X, false><<<dim3((unsigned)grid), dim3(kCsrThreads), 0, stream>>>(
            A.nrows, A.nnz, ntiles, grid, A.rowptr, A.colidx, val, x, y, alpha, beta, nullptr, nullptr);
    SPX_LAUNCHED();
    return SPX_OK;
}

template spx_status csr_spmv_launch<double, double>(const spx_matrix &, const double *, double *, double, double,
                                                    const double *, double *, hipStream_t);
template spx_status csr_spmv_launch<float, float>(const spx_matrix &, const float *, float *, float, float,
                                                  const float *, float *, hipStream_t);
template spx_status csr_spmv_launch<_Float16, float>(const spx_matrix &, const float *, float *, float, float,
                                                     const float *, float *, hipStream_t);

}  // namespace spx
