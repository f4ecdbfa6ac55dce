// validate.hip -- canonical-form checks of a matrix's index arrays.
//
// spx_validate reads only index arrays (row pointers, row and column indices,
// ELL / SELL-P slot columns, slice offsets), never values, and classifies what
// it finds into four classes, reported in this order of precedence:
//   SPX_ERR_FORMAT     structure: CSR row pointer not starting at 0, not
//                      ending at nnz or decreasing; an ELL / SELL-P entry
//                      after a padding slot; a HYB row with COO entries
//                      whose ELL part is not full; stored entries not
//                      adding up to nnz; SELL-P slice offsets malformed;
//   SPX_ERR_RANGE      a row or column index outside the matrix;
//   SPX_ERR_UNSORTED   columns not ascending inside a row (COO: entries not
//                      in (row, col) order);
//   SPX_ERR_DUPLICATE  the same (row, col) stored twice.
// Every kernel records, per class, the smallest position (entry or row) where
// it saw the class, with an atomic minimum; the host reads the four words
// back. Entry checks run only once the structure checks have passed, so no
// kernel follows a malformed row pointer or slice offset.
//
// spx_validate_csr_host applies the same CSR checks to host arrays with plain
// loops; the solve server runs it on every request before queueing it.
#include <algorithm>

#include "common.hpp"
#include "spmv.hpp"
#include "wave.hpp"

namespace spx {
namespace {

enum { kVFormat = 0, kVRange = 1, kVUnsorted = 2, kVDuplicate = 3, kVClasses = 4, kVCount = 4 };
constexpr int kVThreads = 256;
constexpr unsigned long long kNone = ~0ull;

__device__ __forceinline__ void vflag(unsigned long long *res, int cls, int64_t pos)
{
    if ((unsigned long long)pos < res[cls]) atomicMin(&res[cls], (unsigned long long)pos);
}

// Columns c0, c1 of adjacent entries of one row.
__device__ __forceinline__ void vpair(unsigned long long *res, int32_t c0, int32_t c1, int64_t pos)
{
    if (c0 > c1) vflag(res, kVUnsorted, pos);
    else if (c0 == c1) vflag(res, kVDuplicate, pos);
}

__global__ void vinit_kernel(unsigned long long *res)
{
    if (threadIdx.x < kVClasses) res[threadIdx.x] = kNone;
    if (threadIdx.x == kVCount) res[kVCount] = 0;
}

// ---------------------------------------------------------------- CSR
__global__ __launch_bounds__(kVThreads) void v_rowptr_kernel(const int32_t *__restrict__ rowptr, int32_t n,
                                                             int64_t nnz, unsigned long long *res)
{
    const int64_t i = (int64_t)blockIdx.x * kVThreads + threadIdx.x;
    if (i > n) return;
    const int64_t a = rowptr[i];
    if (i == 0 && a != 0) vflag(res, kVFormat, 0);
    if (i == n && a != nnz) vflag(res, kVFormat, n);
    if (i < n && (int64_t)rowptr[i + 1] < a) vflag(res, kVFormat, i);
}

// One wavefront per row: lane l checks entries l, l + 64, ... against the
// column range and against their successor in the row.
__global__ __launch_bounds__(kVThreads) void v_csr_entries_kernel(const int32_t *__restrict__ rowptr,
                                                                  const int32_t *__restrict__ col, int32_t n,
                                                                  int32_t ncols, unsigned long long *res)
{
    const int64_t row = (int64_t)blockIdx.x * (kVThreads / kWave) + threadIdx.x / kWave;
    if (row >= n) return;
    const int64_t b = rowptr[row], e = rowptr[row + 1];
    for (int64_t p = b + (threadIdx.x % kWave); p < e; p += kWave) {
        const int32_t c = col[p];
        if (c < 0 || c >= ncols) vflag(res, kVRange, p);
        if (p + 1 < e) vpair(res, c, col[p + 1], p);
    }
}

// ---------------------------------------------------------------- COO
__global__ __launch_bounds__(kVThreads) void v_coo_kernel(const int32_t *__restrict__ row,
                                                          const int32_t *__restrict__ col, int64_t nnz, int32_t nrows,
                                                          int32_t ncols, unsigned long long *res)
{
    const int64_t p = (int64_t)blockIdx.x * kVThreads + threadIdx.x;
    if (p >= nnz) return;
    const int32_t r = row[p], c = col[p];
    if (r < 0 || r >= nrows || c < 0 || c >= ncols) vflag(res, kVRange, p);
    if (p + 1 < nnz) {
        const int32_t r1 = row[p + 1];
        if (r > r1) vflag(res, kVUnsorted, p);
        else if (r == r1) vpair(res, c, col[p + 1], p);
    }
}

// ---------------------------------------------------------------- ELL / SELL-P rows
// One thread per row; slot k of the row at base + k * stride. Counts the
// stored entries (one atomic per work-group).
__device__ __forceinline__ int64_t v_slot_row(const int32_t *__restrict__ ecol, int64_t base, int64_t stride,
                                              int32_t width, int32_t ncols, bool exists, int64_t row,
                                              unsigned long long *res)
{
    int32_t prev = -1;
    bool pad = false;
    int64_t stored = 0;
    for (int32_t k = 0; k < width; ++k) {
        const int32_t c = ecol[base + (int64_t)k * stride];
        if (c == -1) {
            pad = true;
            continue;
        }
        if (pad || !exists) vflag(res, kVFormat, row);
        if (c < -1 || c >= ncols) {
            vflag(res, kVRange, row);
        } else if (prev >= 0) {
            vpair(res, prev, c, row);
        }
        prev = c;
        ++stored;
    }
    return stored;
}

__device__ __forceinline__ void v_add_count(int64_t v, unsigned long long *res)
{
    __shared__ unsigned long long s_cnt;
    if (threadIdx.x == 0) s_cnt = 0;
    __syncthreads();
    if (v) atomicAdd(&s_cnt, (unsigned long long)v);
    __syncthreads();
    if (threadIdx.x == 0 && s_cnt) atomicAdd(&res[kVCount], s_cnt);
}

__global__ __launch_bounds__(kVThreads) void v_ell_kernel(const int32_t *__restrict__ ecol, int32_t n, int32_t K,
                                                          int64_t ld, int32_t ncols, unsigned long long *res)
{
    const int64_t i = (int64_t)blockIdx.x * kVThreads + threadIdx.x;
    int64_t stored = 0;
    if (i < n) stored = v_slot_row(ecol, i, ld, K, ncols, true, i, res);
    v_add_count(stored, res);
}

__global__ __launch_bounds__(kVThreads) void v_sets_kernel(const int32_t *__restrict__ sets, int64_t ns,
                                                           int64_t slice_cols, int32_t T, unsigned long long *res)
{
    const int64_t s = (int64_t)blockIdx.x * kVThreads + threadIdx.x;
    if (s > ns) return;
    const int64_t a = sets[s];
    if (s == 0 && a != 0) vflag(res, kVFormat, 0);
    if (s == ns && a != slice_cols) vflag(res, kVFormat, ns);
    if (s < ns) {
        const int64_t w = (int64_t)sets[s + 1] - a;
        if (w < 0 || w % T != 0) vflag(res, kVFormat, s);
    }
}

__global__ __launch_bounds__(kVThreads) void v_sellp_kernel(const int32_t *__restrict__ sets,
                                                            const int32_t *__restrict__ scol, int32_t n, int32_t C,
                                                            int64_t nslices, int32_t ncols, unsigned long long *res)
{
    const int64_t r = (int64_t)blockIdx.x * kVThreads + threadIdx.x;  // rows of the padded last slice included
    int64_t stored = 0;
    if (r < nslices * C) {
        const int64_t s = r / C, l = r % C;
        const int64_t w = (int64_t)sets[s + 1] - sets[s];
        stored = v_slot_row(scol, (int64_t)sets[s] * C + l, C, (int32_t)w, ncols, r < n, r, res);
    }
    v_add_count(stored, res);
}

// ---------------------------------------------------------------- HYB cross check
// A COO entry of row r needs r's ELL part full (K stored entries) and, if it
// is the first COO entry of r, a column beyond the ELL part's last one.
__global__ __launch_bounds__(kVThreads) void v_hyb_cross_kernel(const int32_t *__restrict__ ecol, int32_t K,
                                                                int64_t ld, const int32_t *__restrict__ row,
                                                                const int32_t *__restrict__ col, int64_t cnnz,
                                                                int32_t nrows, unsigned long long *res)
{
    const int64_t p = (int64_t)blockIdx.x * kVThreads + threadIdx.x;
    if (p >= cnnz || K == 0) return;
    const int32_t r = row[p];
    if (r < 0 || r >= nrows) return;  // a range error, flagged by the COO check
    const int32_t last = ecol[(int64_t)(K - 1) * ld + r];
    if (last == -1) {
        vflag(res, kVFormat, p);
    } else if (p == 0 || row[p - 1] != r) {
        vpair(res, last, col[p], p);
    }
}

unsigned grid_for(int64_t items, int64_t per_block) { return (unsigned)ceil_div(std::max<int64_t>(items, 1), per_block); }

spx_status read_results(unsigned long long *dres, unsigned long long *h, hipStream_t stream)
{
    SPX_HIP(hipMemcpyAsync(h, dres, sizeof(unsigned long long) * (kVCount + 1), hipMemcpyDeviceToHost, stream));
    SPX_HIP(hipStreamSynchronize(stream));
    return SPX_OK;
}

spx_status report(const unsigned long long *h, const char *fmt_name)
{
    static const char *what[kVClasses] = {"malformed structure", "index out of range", "unsorted entries",
                                          "duplicate entry"};
    static const spx_status code[kVClasses] = {SPX_ERR_FORMAT, SPX_ERR_RANGE, SPX_ERR_UNSORTED, SPX_ERR_DUPLICATE};
    for (int c = 0; c < kVClasses; ++c)
        if (h[c] != kNone) {
            set_error("spx_validate: %s: %s at position %llu", fmt_name, what[c], (unsigned long long)h[c]);
            return code[c];
        }
    return SPX_OK;
}

struct DevWords {
    unsigned long long *p = nullptr;
    ~DevWords()
    {
        if (p) (void)hipFree(p);
    }
};

spx_status validate_device(const spx_matrix &A, hipStream_t stream)
{
    DevWords d;
    SPX_HIP(hipMalloc(reinterpret_cast<void **>(&d.p), sizeof(unsigned long long) * (kVCount + 1)));
    unsigned long long *res = d.p;
    unsigned long long h[kVCount + 1];
    vinit_kernel<<<1, 64, 0, stream>>>(res);
    SPX_LAUNCHED();
    const int32_t n = A.nrows, nc = A.ncols;
    switch (A.fmt) {
    case SPX_CSR: {
        v_rowptr_kernel<<<grid_for((int64_t)n + 1, kVThreads), kVThreads, 0, stream>>>(A.rowptr, n, A.nnz, res);
        SPX_LAUNCHED();
        SPX_CHECK(read_results(res, h, stream));
        if (h[kVFormat] != kNone) return report(h, "CSR row pointer");
        if (n > 0 && A.nnz > 0) {
            v_csr_entries_kernel<<<grid_for(n, kVThreads / kWave), kVThreads, 0, stream>>>(A.rowptr, A.colidx, n, nc,
                                                                                         res);
            SPX_LAUNCHED();
        }
        SPX_CHECK(read_results(res, h, stream));
        return report(h, "CSR");
    }
    case SPX_COO:
        if (A.nnz > 0) {
            v_coo_kernel<<<grid_for(A.nnz, kVThreads), kVThreads, 0, stream>>>(A.rowidx, A.colidx, A.nnz, n, nc, res);
            SPX_LAUNCHED();
        }
        SPX_CHECK(read_results(res, h, stream));
        return report(h, "COO");
    case SPX_ELL:
    case SPX_HYB: {
        if (n > 0 && A.ell_width > 0) {
            v_ell_kernel<<<grid_for(n, kVThreads), kVThreads, 0, stream>>>(A.ell_col, n, A.ell_width, A.ell_ld, nc,
                                                                          res);
            SPX_LAUNCHED();
        }
        const int64_t cnnz = A.fmt == SPX_HYB ? A.coo_nnz : 0;
        if (cnnz > 0) {
            v_coo_kernel<<<grid_for(cnnz, kVThreads), kVThreads, 0, stream>>>(A.rowidx, A.colidx, cnnz, n, nc, res);
            SPX_LAUNCHED();
            if (n > 0) {
                v_hyb_cross_kernel<<<grid_for(cnnz, kVThreads), kVThreads, 0, stream>>>(
                    A.ell_col, A.ell_width, A.ell_ld, A.rowidx, A.colidx, cnnz, n, res);
                SPX_LAUNCHED();
            }
        }
        SPX_CHECK(read_results(res, h, stream));
        if (h[kVFormat] == kNone && (int64_t)h[kVCount] + cnnz != A.nnz) h[kVFormat] = (unsigned long long)A.nnz;
        return report(h, A.fmt == SPX_ELL ? "ELL" : "HYB");
    }
    case SPX_SELLP: {
        const int64_t ns = ceil_div(n, A.slice_size);
        v_sets_kernel<<<grid_for(ns + 1, kVThreads), kVThreads, 0, stream>>>(A.slice_sets, ns, A.slice_cols,
                                                                           A.stride_factor, res);
        SPX_LAUNCHED();
        SPX_CHECK(read_results(res, h, stream));
        if (h[kVFormat] != kNone) return report(h, "SELLP slice offsets");
        if (ns > 0) {
            v_sellp_kernel<<<grid_for(ns * A.slice_size, kVThreads), kVThreads, 0, stream>>>(
                A.slice_sets, A.ell_col, n, A.slice_size, ns, nc, res);
            SPX_LAUNCHED();
        }
        SPX_CHECK(read_results(res, h, stream));
        if (h[kVFormat] == kNone && (int64_t)h[kVCount] != A.nnz) h[kVFormat] = (unsigned long long)A.nnz;
        return report(h, "SELLP");
    }
    default: break;
    }
    set_error("spx_validate: bad format %d", A.fmt);
    return SPX_ERR_ARG;
}

}  // namespace

spx_status validate_csr_host(int32_t nrows, int32_t ncols, int64_t nnz, const int32_t *rowptr, const int32_t *col)
{
    SPX_REQUIRE(nrows >= 0 && ncols >= 0 && nnz >= 0 && rowptr != nullptr && (nnz == 0 || col != nullptr),
                SPX_ERR_ARG, "spx_validate_csr_host: bad arguments");
    SPX_REQUIRE(rowptr[0] == 0, SPX_ERR_FORMAT, "spx_validate_csr_host: rowptr[0] = %d, not 0", rowptr[0]);
    for (int32_t i = 0; i < nrows; ++i)
        SPX_REQUIRE(rowptr[i + 1] >= rowptr[i], SPX_ERR_FORMAT, "spx_validate_csr_host: rowptr decreases at row %d", i);
    SPX_REQUIRE(rowptr[nrows] == nnz, SPX_ERR_FORMAT, "spx_validate_csr_host: rowptr[n] = %d, nnz = %lld",
                rowptr[nrows], (long long)nnz);
    // one pass; the first entry of each class by position is remembered and
    // the class of highest precedence is reported, as spx_validate does
    int64_t first[kVClasses] = {-1, -1, -1, -1};
    for (int32_t i = 0; i < nrows; ++i) {
        const int32_t b = rowptr[i], e = rowptr[i + 1];
        bool ok = true;
        for (int32_t p = b; p < e; ++p) ok &= (col[p] >= 0) & (col[p] < ncols) & (p + 1 >= e || col[p] < col[p + 1]);
        if (ok) continue;
        for (int32_t p = b; p < e; ++p) {
            int cls = -1;
            if (col[p] < 0 || col[p] >= ncols) {
                cls = kVRange;
                if (first[cls] < 0) first[cls] = p;
            }
            if (p + 1 < e && col[p] >= col[p + 1]) {
                cls = col[p] > col[p + 1] ? kVUnsorted : kVDuplicate;
                if (first[cls] < 0) first[cls] = p;
            }
        }
    }
    unsigned long long h[kVCount + 1];
    for (int c = 0; c < kVClasses; ++c) h[c] = first[c] < 0 ? kNone : (unsigned long long)first[c];
    h[kVCount] = 0;
    const spx_status st = report(h, "host CSR");
    return st;
}

}  // namespace spx

using namespace spx;

extern "C" spx_status spx_validate(const spx_matrix *A, hipStream_t stream)
{
    clear_error();
    SPX_CHECK(check_matrix(A, "spx_validate"));
    return validate_device(*A, stream);
}

extern "C" spx_status spx_validate_csr_host(int32_t nrows, int32_t ncols, int64_t nnz, const int32_t *rowptr,
                                            const int32_t *colidx)
{
    clear_error();
    return validate_csr_host(nrows, ncols, nnz, rowptr, colidx);
}
