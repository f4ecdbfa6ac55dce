// convert.hip -- format conversion and value casts on the GPU.
//
// Formats as in Section 1 of the paper (Coo, Csr, Ell, Hybrid). Every
// conversion is integer index work plus bit-for-bit value copies, so results
// are exact; casts to float32 / binary16 round to nearest even.
//
//  CSR -> COO   row index of every entry: a wavefront takes 64 rows; short
//               rows are expanded by their own lane, rows longer than 64 by the
//               whole wavefront (coalesced stores).
//  COO -> CSR   rowptr from the sorted row array: entry p writes rowptr[i] = p
//               for every row i in (row[p-1], row[p]] (one pass, coalesced).
//  CSR -> ELL   one lane per row writes its K slots (slot-major, coalesced).
//  CSR -> HYB   first K entries of a row -> ELL slots; the rest -> COO part at
//               an offset from an exclusive scan of max(0, len - K).
//  ELL -> CSR   per-row counts of stored slots, scan, then a copy in slot order.
//  HYB -> CSR   ELL counts plus COO counts (from the COO row pointer), scan,
//               then a per-row merge of the two ascending lists.
#include <vector>

#include "common.hpp"
#include "convert.hpp"
#include "spmv.hpp"
#include "wave.hpp"

namespace spx {

constexpr int kCvThreads = 256;
constexpr int kCvStageRows = 128;   // rows per work-group of the staged conversions
constexpr int kCvStageNnz = 4096;   // their LDS capacity in entries
constexpr int kScanItems = 4;                           // per thread
constexpr int kScanBlock = kCvThreads * kScanItems;     // elements per scan block

// ------------------------------------------------------------------ scan
// Inclusive prefix sum in place over n values of T, three phases: per-block
// sums, a single-block scan of those sums, per-block scan plus offset.
template <typename T>
__device__ __forceinline__ T block_inclusive_scan(T v, T *s_tmp, T *total)
{
    // wavefront scan by DPP-free shuffles through LDS (Hillis-Steele over the block)
    const int tid = threadIdx.x;
    s_tmp[tid] = v;
    __syncthreads();
    for (int off = 1; off < kCvThreads; off <<= 1) {
        T add = (tid >= off) ? s_tmp[tid - off] : T(0);
        __syncthreads();
        s_tmp[tid] += add;
        __syncthreads();
    }
    T r = s_tmp[tid];
    if (total) *total = s_tmp[kCvThreads - 1];
    __syncthreads();
    return r;
}

template <typename T>
__global__ __launch_bounds__(kCvThreads) void scan_block_sums(const T *__restrict__ a, int64_t n, T *__restrict__ sums)
{
    __shared__ T s_tmp[kCvThreads];
    const int64_t base = (int64_t)blockIdx.x * kScanBlock;
    T v = T(0);
#pragma unroll
    for (int u = 0; u < kScanItems; ++u) {
        const int64_t i = base + threadIdx.x * kScanItems + u;
        if (i < n) v += a[i];
    }
    T total;
    block_inclusive_scan(v, s_tmp, &total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

template <typename T>
__global__ __launch_bounds__(kCvThreads) void scan_sums_serial(T *__restrict__ sums, int64_t nb)
{
    // exclusive scan of the block sums by one work-group, kCvThreads at a time
    __shared__ T s_tmp[kCvThreads];
    T carry = T(0);
    for (int64_t c = 0; c < nb; c += kCvThreads) {
        const int64_t i = c + threadIdx.x;
        const T v = (i < nb) ? sums[i] : T(0);
        T total;
        const T inc = block_inclusive_scan(v, s_tmp, &total);
        if (i < nb) sums[i] = carry + inc - v;
        carry += total;
    }
}

template <typename T>
__global__ __launch_bounds__(kCvThreads) void scan_apply(T *__restrict__ a, int64_t n, const T *__restrict__ sums)
{
    __shared__ T s_tmp[kCvThreads];
    const int64_t base = (int64_t)blockIdx.x * kScanBlock;
    T v[kScanItems];
    T local = T(0);
#pragma unroll
    for (int u = 0; u < kScanItems; ++u) {
        const int64_t i = base + threadIdx.x * kScanItems + u;
        v[u] = (i < n) ? a[i] : T(0);
        local += v[u];
    }
    const T inc = block_inclusive_scan<T>(local, s_tmp, nullptr);
    T run = sums[blockIdx.x] + inc - local;
#pragma unroll
    for (int u = 0; u < kScanItems; ++u) {
        const int64_t i = base + threadIdx.x * kScanItems + u;
        run += v[u];
        if (i < n) a[i] = run;
    }
}

int64_t scan_ws_bytes(int64_t n) { return (ceil_div(n > 0 ? n : 1, kScanBlock) + 1) * 8; }

template <typename T>
spx_status inclusive_scan(T *a, int64_t n, void *ws, hipStream_t stream)
{
    if (n <= 0) return SPX_OK;
    const int64_t nb = ceil_div(n, kScanBlock);
    T *sums = static_cast<T *>(ws);
    scan_block_sums<T><<<(unsigned)nb, kCvThreads, 0, stream>>>(a, n, sums);
    scan_sums_serial<T><<<1, kCvThreads, 0, stream>>>(sums, nb);
    scan_apply<T><<<(unsigned)nb, kCvThreads, 0, stream>>>(a, n, sums);
    SPX_LAUNCHED();
    return SPX_OK;
}

// ------------------------------------------------------------------ small helpers
template <typename T>
__global__ void fill_kernel(T *__restrict__ a, int64_t n, T v)
{
    const int64_t i = (int64_t)blockIdx.x * kCvThreads + threadIdx.x;
    if (i < n) a[i] = v;
}

template <typename T>
static spx_status fill(T *a, int64_t n, T v, hipStream_t stream)
{
    if (n <= 0) return SPX_OK;
    fill_kernel<T><<<(unsigned)ceil_div(n, kCvThreads), kCvThreads, 0, stream>>>(a, n, v);
    SPX_LAUNCHED();
    return SPX_OK;
}

// Row-length statistics: max over rows, and the histogram of lengths. A
// block takes kStatRows consecutive rows (thread t reads rows t, t + 256, ...:
// coalesced) and combines them in LDS, so the global atomics are one per
// block (max) or one per non-empty bin and block (histogram) instead of one
// per wavefront or row on a handful of addresses.
constexpr int kStatItems = 16;
constexpr int kStatRows = kCvThreads * kStatItems;
constexpr int kHistLdsBins = 4096;  // row lengths below this are counted in LDS

__global__ __launch_bounds__(kCvThreads) void row_len_max_kernel(const int32_t *__restrict__ rowptr, int32_t n,
                                                                int32_t *__restrict__ out)
{
    __shared__ int32_t s_max[kCvThreads / kWave];
    const int64_t base = (int64_t)blockIdx.x * kStatRows;
    int32_t l = 0;
#pragma unroll 4
    for (int u = 0; u < kStatItems; ++u) {
        const int64_t i = base + (int64_t)u * kCvThreads + threadIdx.x;
        if (i < n) {
            const int32_t v = rowptr[i + 1] - rowptr[i];
            l = v > l ? v : l;
        }
    }
    for (int off = 32; off >= 1; off >>= 1) {
        const int o = __shfl_xor(l, off);
        l = o > l ? o : l;
    }
    if (lane_id() == 0) s_max[threadIdx.x / kWave] = l;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t m = s_max[0];
        for (int w = 1; w < kCvThreads / kWave; ++w) m = s_max[w] > m ? s_max[w] : m;
        atomicMax(out, m);
    }
}

// hist has nb = max row length + 1 bins.
__global__ __launch_bounds__(kCvThreads) void row_len_hist_kernel(const int32_t *__restrict__ rowptr, int32_t n,
                                                                 int64_t nb, unsigned long long *__restrict__ hist)
{
    __shared__ uint32_t h[kHistLdsBins];
    const int lds_bins = nb < kHistLdsBins ? (int)nb : kHistLdsBins;
    for (int t = threadIdx.x; t < lds_bins; t += kCvThreads) h[t] = 0u;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kStatRows;
    for (int u = 0; u < kStatItems; ++u) {
        const int64_t i = base + (int64_t)u * kCvThreads + threadIdx.x;
        if (i < n) {
            const int32_t len = rowptr[i + 1] - rowptr[i];
            if (len < lds_bins) atomicAdd(&h[len], 1u);
            else atomicAdd(hist + len, 1ull);
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < lds_bins; t += kCvThreads)
        if (h[t] != 0u) atomicAdd(hist + t, (unsigned long long)h[t]);
}

// ------------------------------------------------------------------ CSR -> COO
// A block takes kCvThreads consecutive rows and writes the row index of
// each of their entries [A, B) in entry order (consecutive threads write
// consecutive entries); the row of entry p is found by bisection over the
// block's row pointers in LDS (empty rows are skipped by the bisection).
__global__ __launch_bounds__(kCvThreads) void csr_rows_kernel(const int32_t *__restrict__ rowptr, int32_t n,
                                                             int32_t *__restrict__ row_out)
{
    __shared__ int32_t s_rp[kCvThreads + 1];
    const int64_t r0 = (int64_t)blockIdx.x * kCvThreads;
    const int64_t rend = r0 + kCvThreads < (int64_t)n ? r0 + kCvThreads : (int64_t)n;
    const int nr = (int)(rend - r0);  // 1 .. kCvThreads
    if (threadIdx.x <= nr) s_rp[threadIdx.x] = rowptr[r0 + threadIdx.x];
    if (threadIdx.x == 0 && nr == kCvThreads) s_rp[kCvThreads] = rowptr[rend];
    __syncthreads();
    const int32_t A = s_rp[0], B = s_rp[nr];
    for (int64_t p = (int64_t)A + threadIdx.x; p < B; p += kCvThreads) {
        int lo = 0, hi = nr;  // s_rp[lo] <= p < s_rp[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (s_rp[mid] <= p) lo = mid;
            else hi = mid;
        }
        row_out[p] = (int32_t)(r0 + lo);
    }
}

spx_status csr_rows_launch(const int32_t *rowptr, int32_t n, int32_t *row_out, hipStream_t stream)
{
    if (n <= 0) return SPX_OK;
    csr_rows_kernel<<<(unsigned)ceil_div(n, kCvThreads), kCvThreads, 0, stream>>>(rowptr, n, row_out);
    SPX_LAUNCHED();
    return SPX_OK;
}

// ------------------------------------------------------------------ COO -> CSR
__global__ __launch_bounds__(kCvThreads) void coo_rowptr_kernel(const int32_t *__restrict__ row, int64_t nnz,
                                                               int32_t n, int32_t *__restrict__ rowptr)
{
    const int64_t p = (int64_t)blockIdx.x * kCvThreads + threadIdx.x;
    if (p >= nnz) return;
    const int32_t r = row[p];
    const int32_t rp = (p > 0) ? row[p - 1] : -1;
    for (int32_t i = rp + 1; i <= r; ++i) rowptr[i] = (int32_t)p;
    if (p == nnz - 1)
        for (int32_t i = r + 1; i <= n; ++i) rowptr[i] = (int32_t)nnz;
}

// ------------------------------------------------------------------ CSR -> ELL / HYB (ELL part)
// Conversions that turn rows into slot columns (or back) go through LDS:
// the kCvStageRows consecutive rows of a work-group occupy one contiguous
// stretch of the CSR arrays, read (or written) coalesced there, while each
// thread walks its own row in LDS. A block whose rows hold more than
// kCvStageNnz entries reads / writes the CSR arrays directly instead.
struct StageRange {
    int32_t base, cnt;
    bool staged;
};

__device__ __forceinline__ StageRange stage_range(const int32_t *__restrict__ rowptr, int32_t n, int64_t r0)
{
    StageRange g{0, 0, false};
    if (r0 < n) {
        const int64_t r1 = min((int64_t)n, r0 + kCvStageRows);
        g.base = rowptr[r0];
        g.cnt = rowptr[r1] - g.base;
    }
    g.staged = g.cnt <= kCvStageNnz;
    return g;
}

template <typename V>
__device__ __forceinline__ void stage_in(const int32_t *__restrict__ col, const V *__restrict__ val,
                                         const StageRange &g, int32_t *s_col, V *s_val)
{
    for (int32_t j = threadIdx.x; j < g.cnt; j += kCvStageRows) {
        s_col[j] = col[g.base + j];
        s_val[j] = val[g.base + j];
    }
    __syncthreads();
}

template <typename V>
__device__ __forceinline__ void stage_out(int32_t *__restrict__ col, V *__restrict__ val, const StageRange &g,
                                          const int32_t *s_col, const V *s_val)
{
    __syncthreads();
    for (int32_t j = threadIdx.x; j < g.cnt; j += kCvStageRows) {
        col[g.base + j] = s_col[j];
        val[g.base + j] = s_val[j];
    }
}

template <typename V>
__global__ __launch_bounds__(kCvStageRows) void csr_to_ell_kernel(const int32_t *__restrict__ rowptr,
                                                                 const int32_t *__restrict__ col,
                                                                 const V *__restrict__ val, int32_t n, int32_t K,
                                                                 int64_t ld, int32_t *__restrict__ ecol,
                                                                 V *__restrict__ eval)
{
    __shared__ int32_t s_col[kCvStageNnz];
    __shared__ V s_val[kCvStageNnz];
    const int64_t r0 = (int64_t)blockIdx.x * kCvStageRows;
    const int64_t i = r0 + threadIdx.x;
    const StageRange g = stage_range(rowptr, n, r0);
    if (g.staged) stage_in(col, val, g, s_col, s_val);
    if (i >= ld) return;
    const int32_t a = (i < n) ? rowptr[i] : 0;
    const int32_t len = (i < n) ? rowptr[i + 1] - a : 0;
    for (int32_t k = 0; k < K; ++k) {
        const int64_t q = (int64_t)k * ld + i;
        if (k < len) {
            ecol[q] = g.staged ? s_col[a - g.base + k] : col[a + k];
            eval[q] = g.staged ? s_val[a - g.base + k] : val[a + k];
        } else {
            ecol[q] = -1;
            eval[q] = V(0);
        }
    }
}

__global__ __launch_bounds__(kCvThreads) void hyb_excess_kernel(const int32_t *__restrict__ rowptr, int32_t n,
                                                               int32_t K, int64_t *__restrict__ ex)
{
    const int64_t i = (int64_t)blockIdx.x * kCvThreads + threadIdx.x;
    if (i < n) {
        const int32_t len = rowptr[i + 1] - rowptr[i];
        ex[i] = len > K ? len - K : 0;
    }
}

// COO part of a HYB: entries k >= K of row i go to [off_i, off_i + len - K),
// off_i = inclusive_scan(excess)[i] - excess_i.
template <typename V>
__global__ __launch_bounds__(kCvThreads) void hyb_coo_kernel(const int32_t *__restrict__ rowptr,
                                                            const int32_t *__restrict__ col,
                                                            const V *__restrict__ val, int32_t n, int32_t K,
                                                            const int64_t *__restrict__ incl,
                                                            int32_t *__restrict__ crow, int32_t *__restrict__ ccol,
                                                            V *__restrict__ cval)
{
    const int64_t i = (int64_t)blockIdx.x * kCvThreads + threadIdx.x;
    const int32_t a = (i < n) ? rowptr[i] + K : 0;
    const int32_t b = (i < n) ? rowptr[i + 1] : 0;
    const int64_t off = (i < n) ? incl[i] - (b > a ? b - a : 0) : 0;
    const bool longrow = (b - a) > kWave;
    if (!longrow)
        for (int32_t p = a; p < b; ++p) {
            crow[off + (p - a)] = (int32_t)i;
            ccol[off + (p - a)] = col[p];
            cval[off + (p - a)] = val[p];
        }
    lane_mask_t m = ballot64(longrow);
    while (m) {
        const int src = __builtin_ctzll(m);
        m &= m - 1;
        const int32_t ra = readlane(a, src), rb = readlane(b, src);
        const int32_t rid = readlane((int)i, src);
        const int64_t o = (int64_t)(uint32_t)readlane((int)(off & 0xffffffff), src) |
                          ((int64_t)readlane((int)(off >> 32), src) << 32);
        for (int32_t p = ra + lane_id(); p < rb; p += kWave) {
            crow[o + (p - ra)] = rid;
            ccol[o + (p - ra)] = col[p];
            cval[o + (p - ra)] = val[p];
        }
    }
}

// ------------------------------------------------------------------ ELL -> CSR and HYB -> CSR
// rowptr[i+1] = stored ELL slots of row i (+ COO entries of row i if coo_rp)
__global__ __launch_bounds__(kCvThreads) void ell_count_kernel(const int32_t *__restrict__ ecol, int32_t n,
                                                              int32_t K, int64_t ld,
                                                              const int32_t *__restrict__ coo_rp,
                                                              int32_t *__restrict__ rowptr)
{
    const int64_t i = (int64_t)blockIdx.x * kCvThreads + threadIdx.x;
    if (i == 0) rowptr[0] = 0;
    if (i >= n) return;
    int32_t c = 0;
    for (int32_t k = 0; k < K; ++k) c += ecol[(int64_t)k * ld + i] >= 0;
    if (coo_rp) c += coo_rp[i + 1] - coo_rp[i];
    rowptr[i + 1] = c;
}

// Row i of the CSR result: the row's ELL entries (slot order, padding
// dropped) merged with its COO entries (if any), ascending by column.
template <typename V>
__global__ __launch_bounds__(kCvStageRows) void ell_hyb_to_csr_kernel(
    const int32_t *__restrict__ ecol, const V *__restrict__ eval, int32_t n, int32_t K, int64_t ld,
    const int32_t *__restrict__ coo_rp, const int32_t *__restrict__ ccol, const V *__restrict__ cval,
    const int32_t *__restrict__ rowptr, int32_t *__restrict__ col, V *__restrict__ val)
{
    __shared__ int32_t s_col[kCvStageNnz];
    __shared__ V s_val[kCvStageNnz];
    const int64_t r0 = (int64_t)blockIdx.x * kCvStageRows;
    const int64_t i = r0 + threadIdx.x;
    const StageRange g = stage_range(rowptr, n, r0);
    // entry o of the CSR result goes to LDS slot o - base when staged
    auto put = [&](int32_t o, int32_t c, V v) {
        if (g.staged) {
            s_col[o - g.base] = c;
            s_val[o - g.base] = v;
        } else {
            col[o] = c;
            val[o] = v;
        }
    };
    if (i < n) {
        int32_t o = rowptr[i];
        int32_t cb = coo_rp ? coo_rp[i] : 0;
        const int32_t ce = coo_rp ? coo_rp[i + 1] : 0;
        for (int32_t k = 0; k < K; ++k) {
            const int64_t q = (int64_t)k * ld + i;
            const int32_t c = ecol[q];
            if (c < 0) continue;
            while (cb < ce && ccol[cb] < c) {  // COO entries with a smaller column come first
                put(o++, ccol[cb], cval[cb]);
                ++cb;
            }
            put(o++, c, eval[q]);
        }
        for (; cb < ce; ++cb) put(o++, ccol[cb], cval[cb]);
    }
    if (g.staged) stage_out(col, val, g, s_col, s_val);
}

// ------------------------------------------------------------------ casts
// float64 -> binary16, round to nearest even, from the bit pattern: 10
// fraction bits kept, the dropped bits decide the rounding; results below
// 2^-14 are counted in units of 2^-24 (subnormals). NaN -> quiet NaN with
// the sign kept; a finite input that rounds past 65504 -> inf (flagged).
__device__ __forceinline__ uint16_t f64_to_f16_bits(double d, int *overflow)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, d);
    const uint16_t sign = (uint16_t)((b >> 48) & 0x8000u);
    const uint64_t a = b & 0x7FFFFFFFFFFFFFFFull;
    if (a >= 0x7FF0000000000000ull) return sign | (a > 0x7FF0000000000000ull ? 0x7E00u : 0x7C00u);
    const int e = (int)(a >> 52) - 1023;
    const uint64_t m = a & 0xFFFFFFFFFFFFFull;
    if (e >= -14) {
        uint64_t hm = m >> 42;
        const uint64_t rem = m & ((1ull << 42) - 1);
        const uint64_t half = 1ull << 41;
        hm += (rem > half || (rem == half && (hm & 1))) ? 1 : 0;
        int ee = e;
        if (hm == 1024) {
            hm = 0;
            ee += 1;
        }
        if (ee > 15) {
            *overflow = 1;
            return sign | 0x7C00u;
        }
        return sign | (uint16_t)((ee + 15) << 10) | (uint16_t)hm;
    }
    const int shift = 28 - e;  // value / 2^-24 = (m | 2^52) >> shift
    if (shift > 63) return sign;
    const uint64_t M = m | (1ull << 52);
    uint64_t q = M >> shift;
    const uint64_t rem = M & ((1ull << shift) - 1);
    const uint64_t half = 1ull << (shift - 1);
    q += (rem > half || (rem == half && (q & 1))) ? 1 : 0;
    return sign | (uint16_t)q;
}

__device__ __forceinline__ uint32_t f64_to_f32_bits(double d, int *overflow)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, d);
    if ((b & 0x7FFFFFFFFFFFFFFFull) > 0x7FF0000000000000ull)
        return (uint32_t)((b >> 32) & 0x80000000u) | 0x7FC00000u;
    const float f = (float)d;  // v_cvt_f32_f64: round to nearest even
    const uint32_t u = __builtin_bit_cast(uint32_t, f);
    if ((u & 0x7FFFFFFFu) == 0x7F800000u && (b & 0x7FFFFFFFFFFFFFFFull) != 0x7FF0000000000000ull) *overflow = 1;
    return u;
}

__global__ __launch_bounds__(kCvThreads) void cast_kernel(const double *__restrict__ src, int64_t n, int32_t dst_type,
                                                         void *__restrict__ dst, unsigned long long *__restrict__ ovf)
{
    const int64_t i = (int64_t)blockIdx.x * kCvThreads + threadIdx.x;
    int o = 0;
    if (i < n) {
        if (dst_type == SPX_F32)
            static_cast<uint32_t *>(dst)[i] = f64_to_f32_bits(src[i], &o);
        else
            static_cast<uint16_t *>(dst)[i] = f64_to_f16_bits(src[i], &o);
    }
    const lane_mask_t m = ballot64(o != 0);
    if (m && lane_id() == 0) atomicAdd(ovf, (unsigned long long)__builtin_popcountll(m));
}


// ------------------------------------------------------------------ SELL-P
// Width of every slice: stride_factor * ceil(longest row in the slice /
// stride_factor), one thread per slice. Written as int32 (out32, shifted by
// one so that an inclusive scan gives slice_sets) or int64 (out64).
__global__ __launch_bounds__(kCvThreads) void sellp_width_kernel(const int32_t *__restrict__ rowptr, int32_t n,
                                                                int32_t C, int32_t T, int64_t nslices,
                                                                int32_t *__restrict__ out32,
                                                                int64_t *__restrict__ out64)
{
    const int64_t s = (int64_t)blockIdx.x * kCvThreads + threadIdx.x;
    if (s == 0 && out32) out32[0] = 0;
    if (s >= nslices) return;
    int32_t m = 0;
    const int64_t r1 = min((int64_t)n, (s + 1) * C);
    for (int64_t r = s * C; r < r1; ++r) m = max(m, rowptr[r + 1] - rowptr[r]);
    const int32_t w = ((m + T - 1) / T) * T;
    if (out32) out32[s + 1] = w;
    if (out64) out64[s] = w;
}

// One thread per (slice, lane): row s*C + l written slot by slot (lanes of a
// slice are adjacent, so each slot column is written coalesced).
template <typename V>
__global__ __launch_bounds__(kCvStageRows) void csr_to_sellp_kernel(const int32_t *__restrict__ rowptr,
                                                                   const int32_t *__restrict__ col,
                                                                   const V *__restrict__ val, int32_t n, int32_t C,
                                                                   int64_t nslices, const int32_t *__restrict__ sets,
                                                                   int32_t *__restrict__ scol, V *__restrict__ sval)
{
    __shared__ int32_t s_col[kCvStageNnz];
    __shared__ V s_val[kCvStageNnz];
    const int64_t r0 = (int64_t)blockIdx.x * kCvStageRows;
    const int64_t r = r0 + threadIdx.x;  // = slice * C + lane
    const StageRange g = stage_range(rowptr, n, r0);
    if (g.staged) stage_in(col, val, g, s_col, s_val);
    if (r >= nslices * C) return;
    const int64_t s = r / C, l = r % C;
    const int32_t a = (r < n) ? rowptr[r] : 0;
    const int32_t len = (r < n) ? rowptr[r + 1] - a : 0;
    const int32_t k0 = sets[s], w = sets[s + 1] - k0;
    for (int32_t k = 0; k < w; ++k) {
        const int64_t q = ((int64_t)k0 + k) * C + l;
        if (k < len) {
            scol[q] = g.staged ? s_col[a - g.base + k] : col[a + k];
            sval[q] = g.staged ? s_val[a - g.base + k] : val[a + k];
        } else {
            scol[q] = -1;
            sval[q] = V(0);
        }
    }
}

__global__ __launch_bounds__(kCvThreads) void sellp_count_kernel(const int32_t *__restrict__ sets,
                                                                const int32_t *__restrict__ scol, int32_t n,
                                                                int32_t C, int32_t *__restrict__ rowptr)
{
    const int64_t r = (int64_t)blockIdx.x * kCvThreads + threadIdx.x;
    if (r == 0) rowptr[0] = 0;
    if (r >= n) return;
    const int64_t s = r / C, l = r % C;
    const int32_t k0 = sets[s], w = sets[s + 1] - k0;
    int32_t c = 0;
    for (int32_t k = 0; k < w; ++k) c += scol[((int64_t)k0 + k) * C + l] >= 0;
    rowptr[r + 1] = c;
}

template <typename V>
__global__ __launch_bounds__(kCvStageRows) void sellp_to_csr_kernel(const int32_t *__restrict__ sets,
                                                                   const int32_t *__restrict__ scol,
                                                                   const V *__restrict__ sval, int32_t n, int32_t C,
                                                                   const int32_t *__restrict__ rowptr,
                                                                   int32_t *__restrict__ col, V *__restrict__ val)
{
    __shared__ int32_t s_col[kCvStageNnz];
    __shared__ V s_val[kCvStageNnz];
    const int64_t r0 = (int64_t)blockIdx.x * kCvStageRows;
    const int64_t r = r0 + threadIdx.x;
    const StageRange g = stage_range(rowptr, n, r0);
    if (r < n) {
        const int64_t s = r / C, l = r % C;
        const int32_t k0 = sets[s], w = sets[s + 1] - k0;
        int32_t o = rowptr[r];
        for (int32_t k = 0; k < w; ++k) {
            const int64_t q = ((int64_t)k0 + k) * C + l;
            if (scol[q] >= 0) {
                if (g.staged) {
                    s_col[o - g.base] = scol[q];
                    s_val[o - g.base] = sval[q];
                } else {
                    col[o] = scol[q];
                    val[o] = sval[q];
                }
                ++o;
            }
        }
    }
    if (g.staged) stage_out(col, val, g, s_col, s_val);
}

// ------------------------------------------------------------------ host side
static size_t val_size(int32_t t) { return t == SPX_F64 ? 8 : (t == SPX_F32 ? 4 : 2); }

template <typename T>
static spx_status read_scalar(const T *dptr, T *host, hipStream_t stream)
{
    SPX_HIP(hipMemcpyAsync(host, dptr, sizeof(T), hipMemcpyDeviceToHost, stream));
    SPX_HIP(hipStreamSynchronize(stream));
    return SPX_OK;
}

// A small device scratch for plan-time reductions (sizes only), freed on return.
struct DevScratch {
    void *p = nullptr;
    ~DevScratch()
    {
        if (p) (void)hipFree(p);
    }
};

spx_status csr_max_row_len(const spx_matrix &A, int32_t *out, hipStream_t stream)
{
    DevScratch d;
    SPX_HIP(hipMalloc(&d.p, sizeof(int32_t)));
    int32_t *dm = static_cast<int32_t *>(d.p);
    SPX_CHECK(fill<int32_t>(dm, 1, 0, stream));
    if (A.nrows > 0) {
        row_len_max_kernel<<<(unsigned)ceil_div(A.nrows, kStatRows), kCvThreads, 0, stream>>>(A.rowptr, A.nrows, dm);
        SPX_LAUNCHED();
    }
    return read_scalar(dm, out, stream);
}

// Automatic HYB width: argmin over K of n*K*(sv+si) + sum max(0, len-K)*(sv+2si),
// smallest K on ties, from the device histogram of row lengths.
static spx_status hyb_auto_width(const spx_matrix &A, int32_t maxlen, int32_t *K_out, hipStream_t stream)
{
    DevScratch d;
    const size_t nb = (size_t)maxlen + 1;
    SPX_HIP(hipMalloc(&d.p, nb * sizeof(unsigned long long)));
    auto *hist = static_cast<unsigned long long *>(d.p);
    SPX_CHECK(fill<unsigned long long>(hist, (int64_t)nb, 0ull, stream));
    if (A.nrows > 0) {
        row_len_hist_kernel<<<(unsigned)ceil_div(A.nrows, kStatRows), kCvThreads, 0, stream>>>(A.rowptr, A.nrows,
                                                                                               (int64_t)nb, hist);
        SPX_LAUNCHED();
    }
    std::vector<unsigned long long> h(nb);
    SPX_HIP(hipMemcpyAsync(h.data(), hist, nb * sizeof(unsigned long long), hipMemcpyDeviceToHost, stream));
    SPX_HIP(hipStreamSynchronize(stream));
    const double sv = (double)val_size(A.val_type), si = 4.0;
    // excess(K) = sum_{L > K} (L - K) h[L]; rows_above(K) = sum_{L > K} h[L]
    double excess = 0.0, above = 0.0;
    for (size_t L = 1; L < nb; ++L) {
        excess += (double)L * (double)h[L];
        above += (double)h[L];
    }
    int32_t best = 0;
    double best_bytes = excess * (sv + 2 * si);
    for (int32_t K = 1; K <= maxlen; ++K) {
        excess -= above;            // every row longer than K-1 loses one excess entry
        above -= (double)h[K];      // rows of length exactly K are no longer above
        const double bytes = (double)A.nrows * K * (sv + si) + excess * (sv + 2 * si);
        if (bytes < best_bytes) {
            best_bytes = bytes;
            best = K;
        }
    }
    *K_out = best;
    return SPX_OK;
}

static int32_t sellp_c(int32_t c) { return c > 0 ? c : 64; }
static int32_t sellp_t(int32_t t) { return t > 0 ? t : 1; }

int64_t convert_ws_bytes(const spx_matrix &src, int32_t dst_fmt, int32_t slice_size)
{
    const int64_t n = src.nrows;
    if (src.fmt == SPX_CSR && dst_fmt == SPX_SELLP) return scan_ws_bytes(ceil_div(n, sellp_c(slice_size)) + 1);
    if (src.fmt == SPX_SELLP && dst_fmt == SPX_CSR) return scan_ws_bytes(n);
    if (src.fmt == SPX_CSR && dst_fmt == SPX_HYB) return (n + 1) * 8 + scan_ws_bytes(n);
    if (dst_fmt == SPX_CSR && (src.fmt == SPX_ELL || src.fmt == SPX_HYB)) return (n + 1) * 8 + scan_ws_bytes(n);
    return 0;
}

spx_status convert_plan(const spx_matrix &src, int32_t dst_fmt, int32_t ell_width, int64_t ell_ld, spx_matrix *dst,
                        size_t *ws_bytes, hipStream_t stream)
{
    spx_matrix d{};
    d.fmt = dst_fmt;
    d.val_type = src.val_type;
    d.nrows = src.nrows;
    d.ncols = src.ncols;
    const int64_t n = src.nrows;
    if (src.fmt == SPX_CSR && dst_fmt == SPX_COO) {
        d.nnz = src.nnz;
    } else if (src.fmt == SPX_COO && dst_fmt == SPX_CSR) {
        d.nnz = src.nnz;
    } else if (src.fmt == SPX_CSR && (dst_fmt == SPX_ELL || dst_fmt == SPX_HYB)) {
        int32_t maxlen = 0;
        SPX_CHECK(csr_max_row_len(src, &maxlen, stream));
        int32_t K = ell_width;
        if (dst_fmt == SPX_ELL) {
            if (K < 0) K = maxlen;
            SPX_REQUIRE(K >= maxlen, SPX_ERR_FORMAT, "convert: ELL width %d below the longest row (%d)", K, maxlen);
            d.nnz = src.nnz;
        } else {
            if (K < 0) SPX_CHECK(hyb_auto_width(src, maxlen, &K, stream));
            // coo_nnz = sum max(0, len - K): reuse the excess kernel + a scan on a scratch
            DevScratch s;
            SPX_HIP(hipMalloc(&s.p, (size_t)(n + 1) * 8 + (size_t)scan_ws_bytes(n)));
            int64_t *ex = static_cast<int64_t *>(s.p);
            int64_t tot = 0;
            if (n > 0) {
                hyb_excess_kernel<<<(unsigned)ceil_div(n, kCvThreads), kCvThreads, 0, stream>>>(src.rowptr, src.nrows,
                                                                                               K, ex);
                SPX_LAUNCHED();
                SPX_CHECK(inclusive_scan<int64_t>(ex, n, ex + n + 1, stream));
                SPX_CHECK(read_scalar(ex + n - 1, &tot, stream));
            }
            d.coo_nnz = tot;
            d.nnz = src.nnz;
        }
        d.ell_width = K;
        d.ell_ld = ell_ld > 0 ? ell_ld : n;
        SPX_REQUIRE(d.ell_ld >= n, SPX_ERR_ARG, "convert: ell_ld < nrows");
    } else if ((src.fmt == SPX_ELL || src.fmt == SPX_HYB) && dst_fmt == SPX_CSR) {
        // count the stored entries on the device (padding dropped)
        DevScratch s;
        SPX_HIP(hipMalloc(&s.p, (size_t)(n + 1) * 8 + (size_t)scan_ws_bytes(n)));
        int32_t *crp = static_cast<int32_t *>(s.p);
        int32_t *cnt = crp + (n + 1);
        int32_t tot = 0;
        if (n > 0) {
            const int32_t *coo_rp = nullptr;
            if (src.fmt == SPX_HYB && src.coo_nnz > 0) {
                coo_rowptr_kernel<<<(unsigned)ceil_div(src.coo_nnz, kCvThreads), kCvThreads, 0, stream>>>(
                    src.rowidx, src.coo_nnz, src.nrows, crp);
                SPX_LAUNCHED();
                coo_rp = crp;
            }
            ell_count_kernel<<<(unsigned)ceil_div(n, kCvThreads), kCvThreads, 0, stream>>>(
                src.ell_col, src.nrows, src.ell_width, src.ell_ld, coo_rp, cnt);
            SPX_LAUNCHED();
            SPX_CHECK(inclusive_scan<int32_t>(cnt + 1, n, static_cast<char *>(s.p) + (size_t)(n + 1) * 8, stream));
            SPX_CHECK(read_scalar(cnt + n, &tot, stream));
        }
        d.nnz = tot;
    } else if (src.fmt == SPX_CSR && dst_fmt == SPX_SELLP) {
        const int32_t C = sellp_c(dst->slice_size), T = sellp_t(dst->stride_factor);
        SPX_REQUIRE(C <= 256 && (C & (C - 1)) == 0, SPX_ERR_ARG, "convert: slice_size %d is not a power of two <= 256",
                    C);
        const int64_t ns = ceil_div(n, C);
        DevScratch s;
        SPX_HIP(hipMalloc(&s.p, (size_t)(ns + 1) * 8 + (size_t)scan_ws_bytes(ns + 1)));
        int64_t *w = static_cast<int64_t *>(s.p);
        int64_t tot = 0;
        if (ns > 0) {
            sellp_width_kernel<<<(unsigned)ceil_div(ns, kCvThreads), kCvThreads, 0, stream>>>(src.rowptr, src.nrows, C,
                                                                                             T, ns, nullptr, w);
            SPX_LAUNCHED();
            SPX_CHECK(inclusive_scan<int64_t>(w, ns, w + ns + 1, stream));
            SPX_CHECK(read_scalar(w + ns - 1, &tot, stream));
        }
        SPX_REQUIRE(tot <= INT32_MAX, SPX_ERR_RANGE, "convert: SELLP slice widths sum to %lld > int32",
                    (long long)tot);
        d.nnz = src.nnz;
        d.slice_size = C;
        d.stride_factor = T;
        d.slice_cols = tot;
    } else if (src.fmt == SPX_SELLP && dst_fmt == SPX_CSR) {
        DevScratch s;
        SPX_HIP(hipMalloc(&s.p, (size_t)(n + 1) * 4 + (size_t)scan_ws_bytes(n)));
        int32_t *cnt = static_cast<int32_t *>(s.p);
        int32_t tot = 0;
        if (n > 0) {
            sellp_count_kernel<<<(unsigned)ceil_div(n, kCvThreads), kCvThreads, 0, stream>>>(
                src.slice_sets, src.ell_col, src.nrows, src.slice_size, cnt);
            SPX_LAUNCHED();
            SPX_CHECK(inclusive_scan<int32_t>(cnt + 1, n, static_cast<char *>(s.p) + (size_t)(n + 1) * 4, stream));
            SPX_CHECK(read_scalar(cnt + n, &tot, stream));
        }
        d.nnz = tot;
    } else if (src.fmt == dst_fmt) {
        SPX_REQUIRE(false, SPX_ERR_ARG, "convert: source and destination formats are the same");
    } else {
        SPX_REQUIRE(false, SPX_ERR_ARG, "convert: %d -> %d is not supported (convert through CSR)", src.fmt,
                    dst_fmt);
    }
    *dst = d;
    *ws_bytes = (size_t)convert_ws_bytes(src, dst_fmt, d.slice_size);
    return SPX_OK;
}

template <typename V>
static spx_status convert_typed(const spx_matrix &src, spx_matrix &dst, void *ws, hipStream_t stream)
{
    const int32_t n = src.nrows;
    const unsigned gr = (unsigned)ceil_div(n > 0 ? n : 1, kCvThreads);
    if (src.fmt == SPX_CSR && dst.fmt == SPX_COO) {
        if (n > 0) {
            csr_rows_kernel<<<gr, kCvThreads, 0, stream>>>(src.rowptr, n, dst.rowidx);
            SPX_LAUNCHED();
        }
        if (src.nnz > 0) {
            SPX_HIP(hipMemcpyAsync(dst.colidx, src.colidx, src.nnz * 4, hipMemcpyDeviceToDevice, stream));
            SPX_HIP(hipMemcpyAsync(dst.vals, src.vals, src.nnz * sizeof(V), hipMemcpyDeviceToDevice, stream));
        }
        return SPX_OK;
    }
    if (src.fmt == SPX_COO && dst.fmt == SPX_CSR) {
        if (src.nnz == 0) return fill<int32_t>(dst.rowptr, n + 1, 0, stream);
        coo_rowptr_kernel<<<(unsigned)ceil_div(src.nnz, kCvThreads), kCvThreads, 0, stream>>>(src.rowidx, src.nnz, n,
                                                                                             dst.rowptr);
        SPX_LAUNCHED();
        SPX_HIP(hipMemcpyAsync(dst.colidx, src.colidx, src.nnz * 4, hipMemcpyDeviceToDevice, stream));
        SPX_HIP(hipMemcpyAsync(dst.vals, src.vals, src.nnz * sizeof(V), hipMemcpyDeviceToDevice, stream));
        return SPX_OK;
    }
    if (src.fmt == SPX_CSR && (dst.fmt == SPX_ELL || dst.fmt == SPX_HYB)) {
        if (dst.ell_width > 0 && dst.ell_ld > 0) {
            csr_to_ell_kernel<V><<<(unsigned)ceil_div(dst.ell_ld, kCvStageRows), kCvStageRows, 0, stream>>>(
                src.rowptr, src.colidx, static_cast<const V *>(src.vals), n, dst.ell_width, dst.ell_ld, dst.ell_col,
                static_cast<V *>(dst.ell_val));
            SPX_LAUNCHED();
        }
        if (dst.fmt == SPX_HYB && n > 0 && dst.coo_nnz > 0) {
            int64_t *ex = static_cast<int64_t *>(ws);
            hyb_excess_kernel<<<gr, kCvThreads, 0, stream>>>(src.rowptr, n, dst.ell_width, ex);
            SPX_LAUNCHED();
            SPX_CHECK(inclusive_scan<int64_t>(ex, n, ex + n + 1, stream));
            hyb_coo_kernel<V><<<gr, kCvThreads, 0, stream>>>(src.rowptr, src.colidx, static_cast<const V *>(src.vals),
                                                             n, dst.ell_width, ex, dst.rowidx, dst.colidx,
                                                             static_cast<V *>(dst.vals));
            SPX_LAUNCHED();
        }
        return SPX_OK;
    }
    if ((src.fmt == SPX_ELL || src.fmt == SPX_HYB) && dst.fmt == SPX_CSR) {
        if (n == 0) return fill<int32_t>(dst.rowptr, 1, 0, stream);
        const int32_t *coo_rp = nullptr;
        if (src.fmt == SPX_HYB && src.coo_nnz > 0) {
            int32_t *crp = static_cast<int32_t *>(ws);
            coo_rowptr_kernel<<<(unsigned)ceil_div(src.coo_nnz, kCvThreads), kCvThreads, 0, stream>>>(
                src.rowidx, src.coo_nnz, n, crp);
            SPX_LAUNCHED();
            coo_rp = crp;
        }
        void *scan_ws = static_cast<char *>(ws) + (size_t)(n + 1) * 8;
        ell_count_kernel<<<gr, kCvThreads, 0, stream>>>(src.ell_col, n, src.ell_width, src.ell_ld, coo_rp, dst.rowptr);
        SPX_LAUNCHED();
        SPX_CHECK(inclusive_scan<int32_t>(dst.rowptr + 1, n, scan_ws, stream));
        ell_hyb_to_csr_kernel<V><<<(unsigned)ceil_div(n, kCvStageRows), kCvStageRows, 0, stream>>>(
            src.ell_col, static_cast<const V *>(src.ell_val), n, src.ell_width, src.ell_ld, coo_rp, src.colidx,
            static_cast<const V *>(src.vals), dst.rowptr, dst.colidx, static_cast<V *>(dst.vals));
        SPX_LAUNCHED();
        return SPX_OK;
    }
    if (src.fmt == SPX_CSR && dst.fmt == SPX_SELLP) {
        const int32_t C = dst.slice_size;
        const int64_t ns = ceil_div(n, C);
        sellp_width_kernel<<<(unsigned)ceil_div(ns + 1, kCvThreads), kCvThreads, 0, stream>>>(
            src.rowptr, n, C, dst.stride_factor, ns, dst.slice_sets, nullptr);
        SPX_LAUNCHED();
        if (ns > 0) {
            SPX_CHECK(inclusive_scan<int32_t>(dst.slice_sets + 1, ns, ws, stream));
            csr_to_sellp_kernel<V><<<(unsigned)ceil_div(ns * C, kCvStageRows), kCvStageRows, 0, stream>>>(
                src.rowptr, src.colidx, static_cast<const V *>(src.vals), n, C, ns, dst.slice_sets, dst.ell_col,
                static_cast<V *>(dst.ell_val));
            SPX_LAUNCHED();
        }
        return SPX_OK;
    }
    if (src.fmt == SPX_SELLP && dst.fmt == SPX_CSR) {
        if (n == 0) return fill<int32_t>(dst.rowptr, 1, 0, stream);
        sellp_count_kernel<<<gr, kCvThreads, 0, stream>>>(src.slice_sets, src.ell_col, n, src.slice_size, dst.rowptr);
        SPX_LAUNCHED();
        SPX_CHECK(inclusive_scan<int32_t>(dst.rowptr + 1, n, ws, stream));
        sellp_to_csr_kernel<V><<<(unsigned)ceil_div(n, kCvStageRows), kCvStageRows, 0, stream>>>(
            src.slice_sets, src.ell_col, static_cast<const V *>(src.ell_val), n, src.slice_size, dst.rowptr,
            dst.colidx, static_cast<V *>(dst.vals));
        SPX_LAUNCHED();
        return SPX_OK;
    }
    set_error("convert: unsupported pair %d -> %d", src.fmt, dst.fmt);
    return SPX_ERR_ARG;
}

spx_status convert_run(const spx_matrix &src, spx_matrix &dst, void *ws, size_t ws_bytes, hipStream_t stream)
{
    const int64_t need = convert_ws_bytes(src, dst.fmt, dst.slice_size);
    SPX_REQUIRE((int64_t)ws_bytes >= need && (ws != nullptr || need == 0), SPX_ERR_ARG,
                "convert: workspace of %zu bytes is smaller than the %lld needed", ws_bytes, (long long)need);
    switch (val_size(src.val_type)) {
    case 8: return convert_typed<uint64_t>(src, dst, ws, stream);
    case 4: return convert_typed<uint32_t>(src, dst, ws, stream);
    default: return convert_typed<uint16_t>(src, dst, ws, stream);
    }
}

spx_status cast_values(const double *src, int64_t n, int32_t dst_type, void *dst, int64_t *overflow,
                       hipStream_t stream)
{
    DevScratch d;
    SPX_HIP(hipMalloc(&d.p, sizeof(unsigned long long)));
    auto *ovf = static_cast<unsigned long long *>(d.p);
    SPX_CHECK(fill<unsigned long long>(ovf, 1, 0ull, stream));
    if (n > 0) {
        cast_kernel<<<(unsigned)ceil_div(n, kCvThreads), kCvThreads, 0, stream>>>(src, n, dst_type, dst, ovf);
        SPX_LAUNCHED();
    }
    unsigned long long h = 0;
    SPX_CHECK(read_scalar(ovf, &h, stream));
    *overflow = (int64_t)h;
    return SPX_OK;
}

}  // namespace spx
