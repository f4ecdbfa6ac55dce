// transpose.hip -- CSR transpose on the device.
//
// In CSR, A^T is A's entries ordered by (column, row). A's entries are
// already in row order, so a stable sort of their column indices yields that
// order. The sort is a least-significant-digit radix sort with 8-bit digits,
// ceil(bits(ncols - 1) / 8) passes, carrying each entry's position k in A:
//   1. per tile of kRxTile entries, a 256-bin digit histogram, stored
//      digit-major (hist[1 + d * ntiles + tile]);
//   2. an exclusive scan of those counts gives each (digit, tile) its first
//      output slot, so equal digits keep tile order;
//   3. each tile re-reads its entries in index order, ranks every entry
//      among equal digits before it (wavefront ballots on the 8 digit bits,
//      then per-wavefront counts in LDS) and scatters key and position.
// Then A^T's column indices are row(k), its values val[k], and its row
// pointer entry for column c is the first sorted position whose key is >= c
// (a binary search per column). Every step is deterministic: results do not
// depend on the order in which work-groups run.
#include "convert.hpp"
#include "transpose.hpp"
#include "wave.hpp"

namespace spx {

constexpr int kRxThreads = 256;
constexpr int kRxItems = 8;
constexpr int kRxTile = kRxThreads * kRxItems;  // entries per work-group
constexpr int kRxBins = 256;
constexpr int kRxWaves = kRxThreads / kWave;

static int64_t rx_tiles(int64_t nnz) { return nnz > 0 ? ceil_div(nnz, kRxTile) : 1; }

// Radix passes needed for keys in [0, ncols).
static int rx_passes(int32_t ncols)
{
    int bits = 0;
    while (bits < 31 && (int64_t(1) << bits) < (int64_t)ncols) ++bits;
    return (bits + 7) / 8;
}

__global__ __launch_bounds__(kRxThreads) void rx_hist_kernel(const int32_t *__restrict__ keys, int64_t nnz, int shift,
                                                            int64_t ntiles, int32_t *__restrict__ hist)
{
    __shared__ int32_t h[kRxBins];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kRxTile;
#pragma unroll
    for (int j = 0; j < kRxItems; ++j) {
        const int64_t e = base + j * kRxThreads + threadIdx.x;
        if (e < nnz) atomicAdd(&h[((uint32_t)keys[e] >> shift) & (kRxBins - 1)], 1);
    }
    __syncthreads();
    hist[1 + (int64_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
    if (blockIdx.x == 0 && threadIdx.x == 0) hist[0] = 0;
}

// offs[d * ntiles + tile]: first output slot of digit d in this tile.
// perm_in == nullptr: the positions are the identity (first pass).
__global__ __launch_bounds__(kRxThreads) void rx_scatter_kernel(const int32_t *__restrict__ keys_in,
                                                               const int32_t *__restrict__ perm_in, int64_t nnz,
                                                               int shift, int64_t ntiles,
                                                               const int32_t *__restrict__ offs,
                                                               int32_t *__restrict__ keys_out,
                                                               int32_t *__restrict__ perm_out)
{
    __shared__ int32_t run[kRxBins];
    __shared__ int32_t cnt[kRxWaves][kRxBins];
    const int w = threadIdx.x / kWave;
    run[threadIdx.x] = offs[(int64_t)threadIdx.x * ntiles + blockIdx.x];
#pragma unroll
    for (int v = 0; v < kRxWaves; ++v) cnt[v][threadIdx.x] = 0;
    __syncthreads();
    const lane_mask_t below = (lane_mask_t(1) << lane_id()) - 1;
    const int64_t base = (int64_t)blockIdx.x * kRxTile;
    for (int j = 0; j < kRxItems; ++j) {
        const int64_t e = base + j * kRxThreads + threadIdx.x;
        const bool valid = e < nnz;
        const int32_t key = valid ? keys_in[e] : 0;
        const int d = (int)(((uint32_t)key >> shift) & (kRxBins - 1));
        // lanes of this wavefront holding the same digit
        lane_mask_t peers = ballot64(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1;
            const lane_mask_t m = ballot64(bit);
            peers &= bit ? m : ~m;
        }
        const int rank = __popcll(peers & below);
        const bool leader = valid && rank == 0;
        const int count = __popcll(peers);
        if (leader) cnt[w][d] = count;
        __syncthreads();
        if (valid) {
            int32_t pos = run[d] + rank;
            for (int v = 0; v < w; ++v) pos += cnt[v][d];
            keys_out[pos] = key;
            perm_out[pos] = perm_in ? perm_in[e] : (int32_t)e;
        }
        __syncthreads();
        // every read of run[] and cnt[] for this step is done; the next
        // step's writes to cnt[w][*] come from this same wavefront, in order
        if (leader) {
            atomicAdd(&run[d], count);
            cnt[w][d] = 0;
        }
    }
}

// rowptr_t[c] = first position p with keys[p] >= c (c = 0 .. ncols).
__global__ __launch_bounds__(kRxThreads) void rx_rowptr_kernel(const int32_t *__restrict__ keys, int64_t nnz,
                                                              int32_t ncols, int32_t *__restrict__ rowptr_t)
{
    const int64_t c = (int64_t)blockIdx.x * kRxThreads + threadIdx.x;
    if (c > ncols) return;
    int64_t lo = 0, hi = nnz;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((int64_t)keys[mid] < c) lo = mid + 1;
        else hi = mid;
    }
    rowptr_t[c] = (int32_t)lo;
}

// col_t[p] = row of entry perm[p], val_t[p] = val[perm[p]] (perm == nullptr:
// identity). T is an unsigned integer of the value's width (bit copy).
template <typename T>
__global__ __launch_bounds__(kRxThreads) void rx_gather_kernel(const int32_t *__restrict__ perm, int64_t nnz,
                                                              const int32_t *__restrict__ rowof,
                                                              const T *__restrict__ val, int32_t *__restrict__ col_t,
                                                              T *__restrict__ val_t)
{
    const int64_t p = (int64_t)blockIdx.x * kRxThreads + threadIdx.x;
    if (p >= nnz) return;
    const int32_t k = perm ? perm[p] : (int32_t)p;
    col_t[p] = rowof[k];
    val_t[p] = val[k];
}

struct RxBufs {
    int32_t *rowof, *k0, *k1, *p0, *p1, *hist;
    void *scan;
};

static RxBufs rx_carve(char *base, int64_t nnz, size_t *total)
{
    size_t off = 0;
    auto take = [&](size_t bytes) {
        off = (off + 255) & ~size_t(255);
        char *p = base ? base + off : nullptr;
        off += bytes > 0 ? bytes : 1;
        return p;
    };
    const int64_t ntiles = rx_tiles(nnz);
    const size_t e = (size_t)(nnz > 0 ? nnz : 1) * sizeof(int32_t);
    RxBufs b;
    b.rowof = reinterpret_cast<int32_t *>(take(e));
    b.k0 = reinterpret_cast<int32_t *>(take(e));
    b.k1 = reinterpret_cast<int32_t *>(take(e));
    b.p0 = reinterpret_cast<int32_t *>(take(e));
    b.p1 = reinterpret_cast<int32_t *>(take(e));
    b.hist = reinterpret_cast<int32_t *>(take((size_t)(kRxBins * ntiles + 1) * sizeof(int32_t)));
    b.scan = take((size_t)scan_ws_bytes(kRxBins * ntiles));
    *total = off + 256;
    return b;
}

int64_t transpose_ws_bytes(int64_t nnz)
{
    size_t total = 0;
    (void)rx_carve(nullptr, nnz, &total);
    return (int64_t)total;
}

spx_status transpose_run(const spx_matrix &A, spx_matrix &At, void *ws, size_t ws_bytes, hipStream_t stream)
{
    const int64_t nnz = A.nnz;
    const int32_t ncols = (int32_t)A.ncols;
    const size_t need = (size_t)transpose_ws_bytes(nnz);
    SPX_REQUIRE(ws != nullptr && ws_bytes >= need, SPX_ERR_ARG,
                "csr transpose: workspace of %zu bytes is too small (need %zu)", ws_bytes, need);
    // round the base up to 256 bytes inside the slack the size includes
    char *base = reinterpret_cast<char *>((reinterpret_cast<uintptr_t>(ws) + 255) & ~uintptr_t(255));
    size_t total = 0;
    RxBufs b = rx_carve(base, nnz, &total);
    const unsigned grow = (unsigned)ceil_div((int64_t)ncols + 1, kRxThreads);
    if (nnz == 0) {
        rx_rowptr_kernel<<<grow, kRxThreads, 0, stream>>>(b.k0, 0, ncols, At.rowptr);
        SPX_LAUNCHED();
        return SPX_OK;
    }
    SPX_CHECK(csr_rows_launch(A.rowptr, (int32_t)A.nrows, b.rowof, stream));
    const int64_t ntiles = rx_tiles(nnz);
    const int passes = rx_passes(ncols);
    const int32_t *keys = A.colidx;
    const int32_t *perm = nullptr;
    int32_t *kout = b.k0, *pout = b.p0;
    for (int pass = 0; pass < passes; ++pass) {
        const int shift = 8 * pass;
        rx_hist_kernel<<<(unsigned)ntiles, kRxThreads, 0, stream>>>(keys, nnz, shift, ntiles, b.hist);
        SPX_LAUNCHED();
        SPX_CHECK(inclusive_scan<int32_t>(b.hist + 1, kRxBins * ntiles, b.scan, stream));
        rx_scatter_kernel<<<(unsigned)ntiles, kRxThreads, 0, stream>>>(keys, perm, nnz, shift, ntiles, b.hist, kout,
                                                                       pout);
        SPX_LAUNCHED();
        keys = kout;
        perm = pout;
        kout = (kout == b.k0) ? b.k1 : b.k0;
        pout = (pout == b.p0) ? b.p1 : b.p0;
    }
    rx_rowptr_kernel<<<grow, kRxThreads, 0, stream>>>(keys, nnz, ncols, At.rowptr);
    SPX_LAUNCHED();
    const unsigned g = (unsigned)ceil_div(nnz, kRxThreads);
    switch (A.val_type) {
    case SPX_F64:
        rx_gather_kernel<uint64_t><<<g, kRxThreads, 0, stream>>>(perm, nnz, b.rowof,
                                                                 static_cast<const uint64_t *>(A.vals), At.colidx,
                                                                 static_cast<uint64_t *>(At.vals));
        break;
    case SPX_F32:
        rx_gather_kernel<uint32_t><<<g, kRxThreads, 0, stream>>>(perm, nnz, b.rowof,
                                                                 static_cast<const uint32_t *>(A.vals), At.colidx,
                                                                 static_cast<uint32_t *>(At.vals));
        break;
    default:
        rx_gather_kernel<uint16_t><<<g, kRxThreads, 0, stream>>>(perm, nnz, b.rowof,
                                                                 static_cast<const uint16_t *>(A.vals), At.colidx,
                                                                 static_cast<uint16_t *>(At.vals));
        break;
    }
    SPX_LAUNCHED();
    return SPX_OK;
}

}  // namespace spx
