// spmv_colblock.hip -- the CSR product for matrices whose column indices
// scatter over a vector too large for one XCD's L2 (Zipf-like rows of random
// columns, Section 4's skewed matrices): the columns are cut into kCbBlocks
// (8) equal ranges, one per XCD, and the matrix is stored once more as
// kCbBlocks CSR matrices A_b (the entries of A whose column falls in range b,
// in A's row-major order). Work-group g of the product runs on XCD g mod 8
// (the dispatcher deals work-groups round robin) and takes a tile of A_{g mod
// 8}, so each XCD gathers only its 1/8 of x, which its 4 MB L2 holds, instead
// of pulling random lines of all of x from beyond L2. Each block writes its
// row sums to its own partial vector P_b; a second kernel forms
// y = alpha * (P_0 + P_1 + ... + P_7) + beta * y in that fixed order, so the
// result does not depend on scheduling (it differs from the plain CSR
// product's only by the order of the row sum).
//
// Device buffer (caller-owned, 256-byte aligned), regions 256-byte aligned:
//   table   int64 base[kCbBlocks + 1] (entry offset of block b's arrays; each
//           block starts on a multiple of 16 entries) and int64 bnnz[kCbBlocks]
//   rowptr  kCbBlocks x (nrows + 1) int32, block b's row pointer from 0
//   part    kCbBlocks x 2 (csr_tiles(nnz) + 1) int32: each block's tile
//           partition (as spx_csr_analyse), stride for the whole matrix
//   P       kCbBlocks x nrows partial sums in the vector type
//   col     nnz + 16 kCbBlocks int32
//   val     nnz + 16 kCbBlocks values
// Bytes moved per product beyond the CSR algorithmic bytes:
// kCbBlocks (nrows + 1) 4 (block row pointers) + 2 kCbBlocks nrows sx
// (partials written and read).
#include <algorithm>

#include "common.hpp"
#include "convert.hpp"
#include "spmv_colblock.hpp"
#include "spmv_csr.hpp"
#include "spmv_csr_tile.hpp"

namespace spx {

namespace {

constexpr int64_t kCbAlign = 16;  // entries: keeps every block's 16-byte vector loads aligned

size_t a256(size_t b) { return (b + 255) & ~size_t(255); }

struct CbLayout {
    size_t table, rowptr, part, partials, col, val, total;
    int64_t part_stride;  // int32 per block partition
};

CbLayout cb_layout(int64_t n, int64_t nnz, size_t sv, size_t sx)
{
    CbLayout L{};
    const int64_t cap = nnz + kCbAlign * kCbBlocks;
    L.part_stride = 2 * (csr_tiles(nnz) + 1);
    size_t off = 0;
    L.table = off;
    off += 256;
    L.rowptr = off;
    off += a256((size_t)kCbBlocks * (size_t)(n + 1) * 4);
    L.part = off;
    off += a256((size_t)kCbBlocks * (size_t)L.part_stride * 4);
    L.partials = off;
    off += a256((size_t)kCbBlocks * (size_t)n * sx);
    L.col = off;
    off += a256((size_t)cap * 4);
    L.val = off;
    off += a256((size_t)cap * sv);
    L.total = off;
    return L;
}

size_t val_bytes(int32_t t) { return t == SPX_F64 ? 8 : (t == SPX_F32 ? 4 : 2); }
size_t vec_bytes(int32_t t) { return t == SPX_F64 ? 8 : 4; }

// First p in [lo, hi) with col[p] >= key (hi if none).
__device__ __forceinline__ int32_t row_lower_bound(const int32_t *__restrict__ col, int32_t lo, int32_t hi, int32_t key)
{
    while (lo < hi) {
        const int32_t mid = lo + (hi - lo) / 2;
        if (col[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Thread per row: the number of the row's entries in each column block,
// written to rowptr_b[i + 1] (block b's row pointer before its scan).
__global__ __launch_bounds__(256) void cb_count_kernel(const int32_t *__restrict__ rowptr,
                                                       const int32_t *__restrict__ col, int32_t n, int32_t width,
                                                       int32_t *__restrict__ brp)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int32_t a = rowptr[i], e = rowptr[i + 1];
    int32_t lo = a;
#pragma unroll
    for (int b = 0; b < kCbBlocks; ++b) {
        const int64_t lim = (int64_t)(b + 1) * width;
        const int32_t hi = (b == kCbBlocks - 1 || lim > INT32_MAX) ? e : row_lower_bound(col, lo, e, (int32_t)lim);
        brp[(int64_t)b * (n + 1) + i + 1] = hi - lo;
        lo = hi;
    }
    if (i == 0) {
#pragma unroll
        for (int b = 0; b < kCbBlocks; ++b) brp[(int64_t)b * (n + 1)] = 0;
    }
}

// One wavefront per row: every entry of the row goes to its block's arrays,
// keeping row-major order. The row's entries of block b are contiguous in A
// (columns ascend), starting after the entries of blocks 0..b-1.
template <typename W>
__global__ __launch_bounds__(256) void cb_scatter_kernel(const int32_t *__restrict__ rowptr,
                                                         const int32_t *__restrict__ col, const W *__restrict__ val,
                                                         int32_t n, int32_t width, const int32_t *__restrict__ brp,
                                                         const int64_t *__restrict__ base, int32_t *__restrict__ ocol,
                                                         W *__restrict__ oval)
{
    const int64_t i = (int64_t)blockIdx.x * (256 / kWave) + threadIdx.x / kWave;
    if (i >= n) return;
    const int l = lane_id();
    const int32_t a = rowptr[i], e = rowptr[i + 1];
    // per block: destination of the block's first entry of this row, and the
    // source position of that entry
    int64_t dst0[kCbBlocks];
    int32_t src0[kCbBlocks], cnt[kCbBlocks];
    int32_t s = a;
#pragma unroll
    for (int b = 0; b < kCbBlocks; ++b) {
        const int32_t r0 = brp[(int64_t)b * (n + 1) + i], r1 = brp[(int64_t)b * (n + 1) + i + 1];
        dst0[b] = base[b] + r0;
        src0[b] = s;
        cnt[b] = r1 - r0;
        s += r1 - r0;
    }
    for (int32_t p = a + l; p < e; p += kWave) {
        const int32_t c = col[p];
        int b = c / width;
        b = b < 0 ? 0 : (b < kCbBlocks ? b : kCbBlocks - 1);  // as the count kernel places them
        int64_t d = -1;
#pragma unroll
        for (int q = 0; q < kCbBlocks; ++q)
            if (q == b && p >= src0[q] && p - src0[q] < cnt[q]) d = dst0[q] + (p - src0[q]);
        if (d < 0) continue;  // only a row whose columns are not ascending gets here
        ocol[d] = c;
        oval[d] = val[p];
    }
}

// Work-group g: tile g / kCbBlocks of block g % kCbBlocks (the XCD it runs on).
template <typename V, typename X>
__global__ __launch_bounds__(kCsrThreads) void cb_spmv_kernel(int32_t nrows, const int64_t *__restrict__ table,
                                                              const int32_t *__restrict__ brp,
                                                              const int32_t *__restrict__ part, int64_t part_stride,
                                                              const int32_t *__restrict__ col,
                                                              const V *__restrict__ val, const X *__restrict__ x,
                                                              X *__restrict__ partials)
{
    const int b = (int)(blockIdx.x % kCbBlocks);
    const int64_t t = blockIdx.x / kCbBlocks;
    const int64_t bnnz = table[kCbBlocks + 1 + b];
    const int64_t ntiles = (bnnz + kCsrTile - 1) / kCsrTile;
    if (bnnz == 0 || t >= ntiles) return;  // an empty block adds nothing (the finisher skips it)
    const int64_t off = table[b];
    constexpr int kVec = 16 / (int)sizeof(V);
    // the columns of a block are scattered over its range: each thread
    // gathers x for its own staged entries at once (one round of gathers in
    // flight) instead of the row-ordered gathers that serve banded matrices
    // (measured on the Zipf(1.5) matrix, float64: 1.24 ms against 2.08 ms)
    csr_tile<V, X, 0, kCsrThreads, kCsrTile, kVec, false>(
        t, nrows, bnnz, ntiles, brp + (int64_t)b * (nrows + 1), col + off, val + off, x,
        partials + (int64_t)b * nrows, X(1), X(0), nullptr, nullptr, part + (int64_t)b * part_stride);
}

// y = alpha * (P_0 + ... + P_7) + beta * y, the partials added in block order.
// Blocks without entries (bit b of `live` clear) contribute nothing.
template <typename X>
__global__ __launch_bounds__(256) void cb_finish_kernel(const X *__restrict__ partials, int64_t n, uint32_t live,
                                                        X *__restrict__ y, X alpha, X beta)
{
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
        X s = X(0);
#pragma unroll
        for (int b = 0; b < kCbBlocks; ++b)
            if (live & (1u << b)) s += partials[(int64_t)b * n + i];
        X out = alpha * s;
        if (beta != X(0)) out += beta * y[i];
        y[i] = out;
    }
}

template <typename W>
spx_status cb_scatter_launch(const spx_matrix &A, int32_t width, const int32_t *brp, const int64_t *base,
                             int32_t *ocol, void *oval, hipStream_t stream)
{
    const unsigned grid = (unsigned)ceil_div(A.nrows, 256 / kWave);
    cb_scatter_kernel<W><<<grid, 256, 0, stream>>>(A.rowptr, A.colidx, static_cast<const W *>(A.vals), A.nrows, width,
                                                   brp, base, ocol, static_cast<W *>(oval));
    SPX_LAUNCHED();
    return SPX_OK;
}

}  // namespace

int32_t colblock_width(int32_t ncols) { return (int32_t)std::max<int64_t>(1, ceil_div(ncols, kCbBlocks)); }

int64_t colblock_bytes(const spx_matrix &A)
{
    return (int64_t)cb_layout(A.nrows, A.nnz, val_bytes(A.val_type), vec_bytes(A.val_type)).total;
}

spx_status colblock_build(spx_matrix &A, void *buf, size_t bytes, hipStream_t stream)
{
    const int64_t n = A.nrows, nnz = A.nnz;
    const CbLayout L = cb_layout(n, nnz, val_bytes(A.val_type), vec_bytes(A.val_type));
    SPX_REQUIRE(buf != nullptr && bytes >= L.total, SPX_ERR_ARG,
                "spx_csr_colblock: buffer of %zu bytes is smaller than the %zu needed", bytes, L.total);
    SPX_REQUIRE(reinterpret_cast<uintptr_t>(buf) % 256 == 0, SPX_ERR_ARG,
                "spx_csr_colblock: buffer must be 256-byte aligned");
    char *B = static_cast<char *>(buf);
    int64_t *table = reinterpret_cast<int64_t *>(B + L.table);
    int32_t *brp = reinterpret_cast<int32_t *>(B + L.rowptr);
    int32_t *part = reinterpret_cast<int32_t *>(B + L.part);
    int32_t *ocol = reinterpret_cast<int32_t *>(B + L.col);
    void *oval = B + L.val;
    const int32_t width = colblock_width(A.ncols);
    A.csr_cb = nullptr;
    A.csr_cb_tiles = 0;
    A.csr_cb_live = 0;
    int64_t h_table[2 * kCbBlocks + 1] = {};
    if (n > 0) {
        cb_count_kernel<<<(unsigned)ceil_div(n, 256), 256, 0, stream>>>(A.rowptr, A.colidx, (int32_t)n, width, brp);
        SPX_LAUNCHED();
        // the partial-sum region is free until the first product: scan workspace
        void *scan_ws = B + L.partials;
        SPX_REQUIRE(L.col - L.partials >= (size_t)scan_ws_bytes(n), SPX_ERR_ARG, "spx_csr_colblock: internal layout");
        for (int b = 0; b < kCbBlocks; ++b)
            SPX_CHECK(inclusive_scan<int32_t>(brp + (int64_t)b * (n + 1) + 1, n, scan_ws, stream));
        int32_t h_nnz[kCbBlocks];
        for (int b = 0; b < kCbBlocks; ++b)
            SPX_HIP(hipMemcpyAsync(&h_nnz[b], brp + (int64_t)b * (n + 1) + n, sizeof(int32_t), hipMemcpyDeviceToHost,
                                   stream));
        SPX_HIP(hipStreamSynchronize(stream));
        int64_t off = 0, total = 0;
        for (int b = 0; b < kCbBlocks; ++b) {
            h_table[b] = off;
            h_table[kCbBlocks + 1 + b] = h_nnz[b];
            off += ceil_div(h_nnz[b], kCbAlign) * kCbAlign;
            total += h_nnz[b];
        }
        h_table[kCbBlocks] = off;
        SPX_REQUIRE(total == nnz, SPX_ERR_FORMAT,
                    "spx_csr_colblock: the blocks hold %lld entries, the matrix %lld (rowptr or columns malformed)",
                    (long long)total, (long long)nnz);
    }
    SPX_HIP(hipMemcpyAsync(table, h_table, sizeof(h_table), hipMemcpyHostToDevice, stream));
    if (n > 0) {
        switch (A.val_type) {
        case SPX_F64: SPX_CHECK(cb_scatter_launch<uint64_t>(A, width, brp, table, ocol, oval, stream)); break;
        case SPX_F32: SPX_CHECK(cb_scatter_launch<uint32_t>(A, width, brp, table, ocol, oval, stream)); break;
        default: SPX_CHECK(cb_scatter_launch<uint16_t>(A, width, brp, table, ocol, oval, stream)); break;
        }
    }
    int32_t tiles = 1, live = 0;
    for (int b = 0; b < kCbBlocks && n > 0; ++b) {
        if (h_table[kCbBlocks + 1 + b] > 0) live |= 1 << b;
        spx_matrix d{};
        d.fmt = SPX_CSR;
        d.val_type = A.val_type;
        d.nrows = (int32_t)n;
        d.ncols = A.ncols;
        d.nnz = h_table[kCbBlocks + 1 + b];
        d.rowptr = brp + (int64_t)b * (n + 1);
        SPX_CHECK(csr_partition_launch(d, part + (int64_t)b * L.part_stride, stream));
        tiles = std::max<int32_t>(tiles, (int32_t)csr_tiles(d.nnz));
    }
    SPX_HIP(hipStreamSynchronize(stream));  // h_table is read by the copy above
    A.csr_cb = buf;
    A.csr_cb_tiles = tiles;
    A.csr_cb_live = live;
    return SPX_OK;
}

template <typename V, typename X>
spx_status colblock_spmv_launch(const spx_matrix &A, const X *x, X *y, X alpha, X beta, hipStream_t stream)
{
    const int64_t n = A.nrows;
    if (n == 0) return SPX_OK;
    const CbLayout L = cb_layout(n, A.nnz, sizeof(V), sizeof(X));
    char *B = static_cast<char *>(A.csr_cb);
    X *partials = reinterpret_cast<X *>(B + L.partials);
    const int64_t grid = (int64_t)kCbBlocks * std::max<int32_t>(1, A.csr_cb_tiles);
    SPX_REQUIRE(grid <= INT32_MAX, SPX_ERR_ARG, "spx_spmv: column-blocked grid too large");
    cb_spmv_kernel<V, X><<<(unsigned)grid, kCsrThreads, 0, stream>>>(
        A.nrows, reinterpret_cast<const int64_t *>(B + L.table), reinterpret_cast<const int32_t *>(B + L.rowptr),
        reinterpret_cast<const int32_t *>(B + L.part), L.part_stride, reinterpret_cast<const int32_t *>(B + L.col),
        reinterpret_cast<const V *>(B + L.val), x, partials);
    SPX_LAUNCHED();
    const int64_t fg = std::min<int64_t>(ceil_div(n, 256), 8192);
    cb_finish_kernel<X><<<(unsigned)fg, 256, 0, stream>>>(partials, n, (uint32_t)A.csr_cb_live, y, alpha, beta);
    SPX_LAUNCHED();
    return SPX_OK;
}

template spx_status colblock_spmv_launch<double, double>(const spx_matrix &, const double *, double *, double, double,
                                                         hipStream_t);
template spx_status colblock_spmv_launch<float, float>(const spx_matrix &, const float *, float *, float, float,
                                                       hipStream_t);
template spx_status colblock_spmv_launch<_Float16, float>(const spx_matrix &, const float *, float *, float, float,
                                                          hipStream_t);

}  // namespace spx
