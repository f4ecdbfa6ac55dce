// block_jacobi.hip -- block-Jacobi preconditioner for CG.
//
// Block-Jacobi is among the preconditioners the paper lists for the library
// (Section 1); the scalar Jacobi is its 1x1 case. Block k covers rows and
// columns [k*bs, min(n, (k+1)*bs)), bs a power of two <= 32. Setup: one
// wavefront per block gathers the dense diagonal block from the CSR rows into
// LDS next to an identity and runs Gauss-Jordan elimination with partial
// pivoting (largest |pivot|, lowest row on ties); the inverse is stored
// column-major per block (inv[k*bs*bs + j*bs + i] = (D_k^{-1})_{ij}) so that
// the threads of a block read it coalesced when applying it. A zero or
// non-finite pivot sets the solver flag to breakdown.
#include "solver_common.hpp"
#include "solvers.hpp"

namespace spx {

// One wavefront per block of BS rows. The augmented block [D_k | I] sits in
// LDS with an odd row stride, so a column read by the pivot search (lane r
// reads row r) touches distinct banks. Lane c owns column c: after the pivot
// row is normalised, every lane c != j eliminates column j from its own
// column (a_rc -= a_rj * a_jc for r != j). Column j itself is not updated
// (it is never read again: later steps read only later pivot columns and the
// right half), so no lane writes what another reads within a step and a step
// needs no barrier per row.
template <typename V, int BS>
__global__ __launch_bounds__(kWave) void bj_setup_kernel(const int32_t *__restrict__ rowptr,
                                                        const int32_t *__restrict__ col,
                                                        const V *__restrict__ val, int32_t n,
                                                        double *__restrict__ inv, KState *st)
{
    constexpr int S = 2 * BS + 1;
    __shared__ double a[BS * S];
    const int64_t k = blockIdx.x;
    const int64_t i0 = k * BS;
    const int m = (int)min((int64_t)BS, n - i0);
    const int w = 2 * m;
    const int lane = threadIdx.x;
    for (int t = lane; t < BS * S; t += kWave) a[t] = 0.0;
    __syncthreads();
    if (lane < m) {
        for (int32_t p = rowptr[i0 + lane]; p < rowptr[i0 + lane + 1]; ++p) {
            const int32_t c = col[p];
            if (c >= i0 && c < i0 + m) a[lane * S + (c - i0)] = (double)val[p];
        }
        a[lane * S + m + lane] = 1.0;
    }
    __syncthreads();
    bool ok = true;
    for (int j = 0; j < m; ++j) {
        // pivot: largest |a_rj| over r >= j, lowest r on ties (wavefront argmax)
        double v = (lane >= j && lane < m) ? fabs(a[lane * S + j]) : -1.0;
        int idx = lane;
        for (int off = kWave / 2; off >= 1; off >>= 1) {
            const double ov = __shfl_xor(v, off);
            const int oi = __shfl_xor(idx, off);
            if (ov > v || (ov == v && oi < idx)) {
                v = ov;
                idx = oi;
            }
        }
        const int piv = idx;
        const double d = a[piv * S + j];
        if (d == 0.0 || !__builtin_isfinite(d)) {
            ok = false;
            break;
        }
        __syncthreads();  // every lane has read d before the swap moves it
        if (piv != j && lane < w) {
            const double t = a[j * S + lane];
            a[j * S + lane] = a[piv * S + lane];
            a[piv * S + lane] = t;
        }
        __syncthreads();
        if (lane < w) a[j * S + lane] /= d;
        __syncthreads();
        if (lane < w && lane != j) {
            const double pj = a[j * S + lane];
            for (int r = 0; r < m; ++r)
                if (r != j) a[r * S + lane] -= a[r * S + j] * pj;
        }
        __syncthreads();
    }
    if (!ok) {
        if (lane == 0) atomicMax(&st->flag, (int32_t)kBreakdown);
        return;
    }
    // column-major inverse; rows / columns past m of a last, smaller block are 0
    for (int t = lane; t < BS * BS; t += kWave) {
        const int j = t / BS, i = t % BS;
        inv[k * BS * BS + t] = (i < m && j < m) ? a[i * S + m + j] : 0.0;
    }
}

// z = blockdiag(D_k^{-1}) r (each entry summed over its block's columns in
// order), optionally p = z, and the work-group partial of sum r_i z_i at
// partials[row * gridDim.x + blockIdx.x] (the layout of the vector kernels).
// check_flag: skip once the solve has stopped (inside iteration graphs).
template <typename X>
__global__ __launch_bounds__(kVecThreads) void bj_apply_kernel(int64_t n, int32_t bs,
                                                              const double *__restrict__ inv,
                                                              const X *__restrict__ r, X *__restrict__ z,
                                                              X *__restrict__ p, X *__restrict__ partials, int row,
                                                              const KState *st, int check_flag)
{
    if (check_flag && st->flag != kRunning) return;
    __shared__ X s_red[kVecThreads / kWave];
    const int64_t base = (int64_t)blockIdx.x * kVecChunk;
    X rz = X(0);
#pragma unroll
    for (int u = 0; u < kVecItems; ++u) {
        const int64_t i = base + threadIdx.x + u * kVecThreads;
        if (i < n) {
            const int64_t k = i / bs, i0 = k * bs;
            const int m = (int)min((int64_t)bs, n - i0);
            const double *blk = inv + k * bs * bs + (i - i0);
            X s = X(0);
            for (int j = 0; j < m; ++j) s += (X)blk[j * bs] * r[i0 + j];
            z[i] = s;
            if (p) p[i] = s;
            rz += r[i] * s;
        }
    }
    X v[1] = {block_sum<X, kVecThreads>(rz, s_red)};
    write_partials<X, 1>(v, partials + (int64_t)row * gridDim.x, gridDim.x, blockIdx.x);
}

template <typename V>
spx_status bj_setup(const spx_matrix &A, int32_t bs, double *inv, KState *st, hipStream_t stream)
{
    const int64_t nb = ceil_div(A.nrows, bs);
    if (nb == 0) return SPX_OK;
    const V *val = static_cast<const V *>(A.vals);
#define SPX_BJ_SETUP(BS)                                                                                             \
    bj_setup_kernel<V, BS><<<(unsigned)nb, kWave, 0, stream>>>(A.rowptr, A.colidx, val, A.nrows, inv, st)
    switch (bs) {
    case 1: SPX_BJ_SETUP(1); break;
    case 2: SPX_BJ_SETUP(2); break;
    case 4: SPX_BJ_SETUP(4); break;
    case 8: SPX_BJ_SETUP(8); break;
    case 16: SPX_BJ_SETUP(16); break;
    case 32: SPX_BJ_SETUP(32); break;
    default: SPX_REQUIRE(false, SPX_ERR_ARG, "block-Jacobi block size %d is not a power of two <= 32", bs);
    }
#undef SPX_BJ_SETUP
    SPX_LAUNCHED();
    return SPX_OK;
}

template <typename X>
spx_status bj_apply(int64_t n, int32_t bs, const double *inv, const X *r, X *z, X *p, X *partials, int row,
                    const KState *st, bool check_flag, hipStream_t stream)
{
    bj_apply_kernel<X><<<(unsigned)vec_blocks(n), kVecThreads, 0, stream>>>(n, bs, inv, r, z, p, partials, row, st,
                                                                            check_flag ? 1 : 0);
    SPX_LAUNCHED();
    return SPX_OK;
}

template spx_status bj_setup<double>(const spx_matrix &, int32_t, double *, KState *, hipStream_t);
template spx_status bj_setup<float>(const spx_matrix &, int32_t, double *, KState *, hipStream_t);
template spx_status bj_setup<_Float16>(const spx_matrix &, int32_t, double *, KState *, hipStream_t);
template spx_status bj_apply<double>(int64_t, int32_t, const double *, const double *, double *, double *, double *,
                                     int, const KState *, bool, hipStream_t);
template spx_status bj_apply<float>(int64_t, int32_t, const double *, const float *, float *, float *, float *, int,
                                    const KState *, bool, hipStream_t);

}  // namespace spx
