// spmv_formats.hip -- COO, ELL and hybrid ELL+COO products for gfx950.
//
// COO (Section 4: the Coo product "relies on atomic operations"): entries
// sorted by row are cut into wavefront spans of a few chunks of kCooChunk
// entries. A wavefront walks its span chunk by chunk (all loads of a chunk
// issued first) in 64-entry tiles: coalesced loads of row, column and value,
// gathered x, then one segmented inclusive scan across the 64 lanes (DPP row
// shifts + row broadcasts, wave.hpp) keyed by the row index. The last segment
// of a tile is carried in registers into the next tile and chunk. A row
// wholly inside a span is written with a plain store; a row that crosses a
// span boundary is accumulated with a float atomic add after a small pre-pass
// has set it to beta*y (the only non-deterministic order).
// Rows without entries (gaps between consecutive row indices) are written
// beta*y by the chunk that sees the gap.
//
// ELL: slot-major layout (slot k of row i at k*ld + i), one lane per row,
// so every slot load is a contiguous 64-lane access. Padding slots (column -1)
// skip the gather; since padding follows a row's entries, a wavefront stops
// as soon as all of its rows have reached padding.
//
// HYB: the ELL kernel writes y = alpha*A_ell*x + beta*y, then the COO kernel
// adds the COO part (plain read-modify-write for rows inside a chunk, atomics
// for rows crossing a chunk boundary).
#include "common.hpp"
#include "krylov.hpp"
#include "spmv.hpp"
#include "wave.hpp"

namespace spx {

template <typename X>
__device__ __forceinline__ X scaled(X v, X beta)
{
    return beta == X(0) ? X(0) : beta * v;
}

// Pre-pass: a row crossing a chunk boundary is set to beta*y exactly once,
// by the first boundary that falls strictly inside it.
template <typename X>
__global__ __launch_bounds__(256) void coo_split_init_kernel(int64_t nnz, int64_t nspans, int64_t span,
                                                            const int32_t *__restrict__ row, X *__restrict__ y,
                                                            X beta)
{
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x + 1;  // boundary k*span, k >= 1
    if (k >= nspans) return;
    const int64_t b = k * span;
    const int32_t r = row[b];
    if (row[b - 1] != r) return;                  // boundary between rows: no split
    if (k >= 2 && row[b - span - 1] == r) return;  // an earlier boundary is inside r too
    y[r] = beta == X(0) ? X(0) : beta * y[r];
}

template <typename X>
__global__ __launch_bounds__(256) void scale_kernel(int64_t n, X *__restrict__ y, X beta)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) y[i] = scaled(y[i], beta);
}

// Complete segment (row r, sum) of chunk [c0, c1): atomics if it may share
// its row with a neighbouring chunk. row_before / row_after are the rows of
// the entries just outside the chunk (-1 if none).
// kBetaZero: beta == 0, so y is written without being read (no dependent
// load in the tile loop).
template <typename X, bool kAccumulate, bool kBetaZero>
__device__ __forceinline__ void coo_write(int32_t r, X sum, bool chunk_start_seg, bool chunk_end_seg,
                                          int32_t row_before, int32_t row_after, X *__restrict__ y, X alpha, X beta)
{
    const bool left = chunk_start_seg && row_before == r;
    const bool right = chunk_end_seg && row_after == r;
    if (left || right) {
        unsafeAtomicAdd(y + r, alpha * sum);
    } else if (kAccumulate) {
        y[r] += alpha * sum;
    } else if (kBetaZero) {
        y[r] = alpha * sum;
    } else {
        y[r] = alpha * sum + scaled(y[r], beta);
    }
}

template <typename V, typename X, bool kAccumulate, bool kBetaZero>
__global__ __launch_bounds__(kCooThreads) void coo_spmv_kernel(int32_t nrows, int64_t nnz, int64_t nspans,
                                                               int64_t span, int64_t grid_padded,
                                                               const int32_t *__restrict__ row,
                                                               const int32_t *__restrict__ col,
                                                               const V *__restrict__ val, const X *__restrict__ x,
                                                               X *__restrict__ y, X alpha, X beta)
{
    const int lane = lane_id();
    const int64_t blk = xcd_remap(blockIdx.x, grid_padded);
    const int64_t w = blk * (kCooThreads / kWave) + threadIdx.x / kWave;
    if (w >= nspans) return;
    // this wavefront's span [s0, s1): consecutive chunks of kCooChunk entries
    // whose open row is carried from chunk to chunk in registers; only rows
    // crossing the span's ends need atomics
    const int64_t s0 = w * span;
    const int64_t s1 = (s0 + span < nnz) ? s0 + span : nnz;
    const int32_t row_before = s0 > 0 ? row[s0 - 1] : -1;
    const int32_t row_after = s1 < nnz ? row[s1] : -1;

    int32_t carry_row = -1;
    X carry_val = X(0);
    bool carry_start = false;  // carried segment began at the span start
    for (int64_t c0 = s0; c0 < s1; c0 += kCooChunk) {
        const int64_t c1 = (c0 + kCooChunk < s1) ? c0 + kCooChunk : s1;
        // issue every load of the chunk first (memory-level parallelism); the
        // chunk base is wave-uniform so the loads use scalar base + 32-bit offsets
        const int32_t *__restrict__ rowc = row + c0;
        const int32_t *__restrict__ colc = col + c0;
        const V *__restrict__ valc = val + c0;
        const int cn = (int)(c1 - c0);
        int32_t r[kCooTiles], c[kCooTiles];
        X p[kCooTiles];
#pragma unroll
        for (int t = 0; t < kCooTiles; ++t) {
            const int o = t * kWave + lane;
            r[t] = -1;
            c[t] = 0;
            p[t] = X(0);
            if (o < cn) {
                r[t] = ld_stream(rowc + o);
                c[t] = ld_stream(colc + o);
                p[t] = widen(ld_stream(valc + o));
            }
        }
        const int32_t chunk_before = c0 > 0 ? row[c0 - 1] : -1;
#pragma unroll
        for (int t = 0; t < kCooTiles; ++t)
            if (r[t] >= 0) p[t] *= x[c[t]];

#pragma unroll
        for (int t = 0; t < kCooTiles; ++t) {
            const int64_t tb = c0 + t * kWave;
            if (tb >= c1) break;
            const int64_t e = tb + lane;
            const bool valid = e < c1;
            const int32_t rr = r[t];
            const int32_t r0 = readlane(rr, 0);
            const bool span_first = (c0 == s0) && t == 0;
            // the carried segment ends before this tile: write it
            if (carry_row >= 0 && r0 != carry_row) {
                if (lane == 0)
                    coo_write<X, kAccumulate, kBetaZero>(carry_row, carry_val, carry_start, false, row_before,
                                                         row_after, y, alpha, beta);
                carry_row = -1;
            }
            const bool merged = (carry_row >= 0);  // lane 0 continues the carried segment
            const int32_t first_prev = (t == 0) ? chunk_before : readlane(r[t > 0 ? t - 1 : 0], kWave - 1);
            const int32_t rprev = wave_shift_up1(rr, first_prev);
            const bool head = !valid || lane == 0 || rr != rprev;
            X v = p[t];
            if (lane == 0 && merged) v += carry_val;
            // gaps: rows strictly between the previous entry's row and this one are empty
            if (!kAccumulate && valid && rr != rprev)
                for (int32_t g = rprev + 1; g < rr; ++g) y[g] = kBetaZero ? X(0) : scaled(y[g], beta);
            if (!kAccumulate && valid && e == nnz - 1)
                for (int32_t g = rr + 1; g < nrows; ++g) y[g] = kBetaZero ? X(0) : scaled(y[g], beta);
            const X sv = wave_segscan(v, head);
            // the last valid lane of the tile and the segment it closes are carried on
            const int tail_e = (c1 - tb < kWave) ? (int)(c1 - tb - 1) : kWave - 1;
            const lane_mask_t heads = ballot64(head && lane > 0);
            const lane_mask_t upto_me = (lane == kWave - 1) ? ~0ull : ((2ull << lane) - 1);
            const bool seg0 = (heads & upto_me & ~1ull) == 0;  // my segment holds lane 0
            const bool start_seg = seg0 && (span_first || (merged && carry_start));
            // a lane closes a segment when the next lane starts a new one
            const int32_t rn = wave_shift_down1(rr, -2);
            if (lane < tail_e && rn != rr)
                coo_write<X, kAccumulate, kBetaZero>(rr, sv, start_seg, false, row_before, row_after, y, alpha,
                                                     beta);
            carry_row = readlane(rr, tail_e);
            carry_val = readlane(sv, tail_e);
            const lane_mask_t upto_tail = (tail_e == kWave - 1) ? ~0ull : ((2ull << tail_e) - 1);
            const bool last_seg_has_lane0 = (heads & upto_tail & ~1ull) == 0;
            carry_start = last_seg_has_lane0 && (span_first || (merged && carry_start));
        }
    }
    if (carry_row >= 0 && lane == 0)
        coo_write<X, kAccumulate, kBetaZero>(carry_row, carry_val, carry_start, true, row_before, row_after, y, alpha,
                                             beta);
}

// One thread per kR consecutive rows (kR = 2 loads the two rows' slots as
// one vector when ld is even and the arrays are aligned), four slot columns
// in flight; a wavefront stops once all its rows are into their padding.
// kEpi: 0 = plain product; 1 = also the block's sum of y_i*w_i; 2 = that and
// the sum of y_i^2 (one partial per work-group, reduced later in a fixed
// order; a set solver flag skips the launch).
template <typename V, typename X, int kEpi, int kR>
__global__ __launch_bounds__(kEllThreads) void ell_spmv_kernel(int32_t nrows, int32_t K, int64_t ld,
                                                               int64_t grid_padded, const int32_t *__restrict__ ecol,
                                                               const V *__restrict__ eval, const X *__restrict__ x,
                                                               X *__restrict__ y, X alpha, X beta,
                                                               const X *__restrict__ dot_with,
                                                               X *__restrict__ partials, const KState *st)
{
    if (st != nullptr && st->flag != kRunning) return;
    typedef int32_t CR __attribute__((ext_vector_type(kR)));
    typedef V VR __attribute__((ext_vector_type(kR)));
    const int64_t nblocks = ((int64_t)nrows + kEllThreads * kR - 1) / (kEllThreads * kR);
    const int64_t blk = xcd_remap(blockIdx.x, grid_padded);
    if (blk >= nblocks) return;
    const int64_t i0 = (blk * kEllThreads + threadIdx.x) * kR;
    const bool in = i0 < nrows;
    X sum[kR];
#pragma unroll
    for (int r = 0; r < kR; ++r) sum[r] = X(0);
    constexpr int U = 4;
    for (int k = 0; k < K; k += U) {
        CR cc[U];
        VR vv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
#pragma unroll
            for (int r = 0; r < kR; ++r) {
                cc[u][r] = -1;
                vv[u][r] = V(0);
            }
            if (in && k + u < K) {
                const int64_t q = (int64_t)(k + u) * ld + i0;
                cc[u] = ld_stream(reinterpret_cast<const CR *>(ecol + q));
                vv[u] = ld_stream(reinterpret_cast<const VR *>(eval + q));
#pragma unroll
                for (int r = 1; r < kR; ++r)
                    if (i0 + r >= nrows) cc[u][r] = -1;  // a slot past the last row is not the matrix's
            }
        }
        bool live = false;
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int r = 0; r < kR; ++r)
                if (cc[u][r] >= 0) sum[r] += widen(vv[u][r]) * x[cc[u][r]];
#pragma unroll
        for (int r = 0; r < kR; ++r) live |= cc[U - 1][r] >= 0;
        if (ballot64(live) == 0) break;  // every row of the wavefront is into its padding
    }
    X d1 = X(0), d2 = X(0);
#pragma unroll
    for (int r = 0; r < kR; ++r) {
        const int64_t i = i0 + r;
        if (i < nrows) {
            X out = alpha * sum[r];
            if (beta != X(0)) out += beta * y[i];  // y is not read when beta == 0
            y[i] = out;
            if constexpr (kEpi >= 1) d1 += out * dot_with[i];
            if constexpr (kEpi >= 2) d2 += out * out;
        }
    }
    if constexpr (kEpi > 0) {
        __shared__ X s_red[kEllThreads / kWave];
        X v[kEpi];
        v[0] = block_sum<X, kEllThreads>(d1, s_red);
        if constexpr (kEpi >= 2) v[kEpi - 1] = block_sum<X, kEllThreads>(d2, s_red);
        write_partials<X, kEpi>(v, partials, nblocks, blk);
    }
}

template <typename V, typename X, bool kAccumulate>
static spx_status coo_part(int32_t nrows, int64_t nnz, const int32_t *row, const int32_t *col, const V *val,
                           const X *x, X *y, X alpha, X beta, hipStream_t stream)
{
    if (nnz == 0) {
        if (!kAccumulate) {
            scale_kernel<X><<<(unsigned)ceil_div(nrows, 256), 256, 0, stream>>>(nrows, y, beta);
            SPX_LAUNCHED();
        }
        return SPX_OK;
    }
    // chunks per wavefront span: enough spans to fill the GPU several times
    // over, at most kCooMaxSpan chunks (fewer spans, fewer boundary atomics)
    const int64_t nchunks = ceil_div(nnz, kCooChunk);
    int64_t per = ceil_div(nchunks, kCooTargetSpans);
    per = per < 1 ? 1 : (per > kCooMaxSpan ? kCooMaxSpan : per);
    const int64_t span = per * kCooChunk;
    const int64_t nspans = ceil_div(nnz, span);
    if (!kAccumulate && nspans > 1) {
        coo_split_init_kernel<X><<<(unsigned)ceil_div(nspans - 1, 256), 256, 0, stream>>>(nnz, nspans, span, row, y,
                                                                                          beta);
        SPX_LAUNCHED();
    }
    const int64_t blocks = ceil_div(nspans, kCooThreads / kWave);
    const int64_t grid = pad_to_xcds(blocks);
    if (!kAccumulate && beta == X(0))
        coo_spmv_kernel<V, X, false, true><<<(unsigned)grid, kCooThreads, 0, stream>>>(
            nrows, nnz, nspans, span, grid, row, col, val, x, y, alpha, beta);
    else
        coo_spmv_kernel<V, X, kAccumulate, false><<<(unsigned)grid, kCooThreads, 0, stream>>>(
            nrows, nnz, nspans, span, grid, row, col, val, x, y, alpha, beta);
    SPX_LAUNCHED();
    return SPX_OK;
}

template <typename V, typename X>
spx_status coo_spmv_launch(const spx_matrix &A, const X *x, X *y, X alpha, X beta, hipStream_t stream)
{
    return coo_part<V, X, false>(A.nrows, A.nnz, A.rowidx, A.colidx, static_cast<const V *>(A.vals), x, y, alpha,
                                 beta, stream);
}

// Two rows per thread when the slot columns can be read two rows at a time:
// even leading dimension (so a pair never straddles a slot column; with an
// odd nrows the last pair's second row is in-bounds padding) and arrays
// aligned to two entries.
static int ell_rows_per_thread(const spx_matrix &A)
{
    const size_t sv = A.val_type == SPX_F64 ? 8 : (A.val_type == SPX_F32 ? 4 : 2);
    const bool even = (A.ell_ld % 2) == 0;
    const bool aligned = (reinterpret_cast<uintptr_t>(A.ell_col) % 8 == 0) &&
                         (reinterpret_cast<uintptr_t>(A.ell_val) % (2 * sv) == 0);
    return even && aligned ? 2 : 1;
}

int64_t ell_dot_parts(const spx_matrix &A)
{
    return A.nrows > 0 ? ceil_div(A.nrows, (int64_t)kEllThreads * ell_rows_per_thread(A)) : 1;
}

template <typename V, typename X>
spx_status ell_spmv_launch(const spx_matrix &A, const X *x, X *y, X alpha, X beta, hipStream_t stream, int epi,
                           const X *dot_with, X *partials, const KState *st)
{
    const int kr = ell_rows_per_thread(A);
    const int64_t blocks = ceil_div(A.nrows, (int64_t)kEllThreads * kr);
    const int64_t grid = pad_to_xcds(blocks);
#define SPX_ELL_LAUNCH(E, R)                                                                                        \
    ell_spmv_kernel<V, X, E, R><<<(unsigned)grid, kEllThreads, 0, stream>>>(                                        \
        A.nrows, A.ell_width, A.ell_ld, grid, A.ell_col, static_cast<const V *>(A.ell_val), x, y, alpha, beta,      \
        dot_with, partials, st)
    if (kr == 2) {
        if (epi == 2) SPX_ELL_LAUNCH(2, 2);
        else if (epi == 1) SPX_ELL_LAUNCH(1, 2);
        else SPX_ELL_LAUNCH(0, 2);
    } else {
        if (epi == 2) SPX_ELL_LAUNCH(2, 1);
        else if (epi == 1) SPX_ELL_LAUNCH(1, 1);
        else SPX_ELL_LAUNCH(0, 1);
    }
#undef SPX_ELL_LAUNCH
    SPX_LAUNCHED();
    return SPX_OK;
}

template <typename V, typename X>
spx_status hyb_spmv_launch(const spx_matrix &A, const X *x, X *y, X alpha, X beta, hipStream_t stream)
{
    SPX_CHECK(ell_spmv_launch<V, X>(A, x, y, alpha, beta, stream));
    return coo_part<V, X, true>(A.nrows, A.coo_nnz, A.rowidx, A.colidx, static_cast<const V *>(A.vals), x, y, alpha,
                                beta, stream);
}

// SELL-P: one work-group of kSellThreads per slice. Lane l = tid % C owns row
// s*C + l; the G = kSellThreads / C lane groups take the slice's slot
// columns round robin (group g: columns g, g + G, ...), each slot column
// read coalesced across the lanes; the G partial sums of a row are added in
// group order. Padding slots (column -1) contribute nothing.
// kEpi: 0 = plain product; 1 = also the slice's sum of y_i*w_i; 2 = that and
// sum of y_i^2 (one partial per slice, reduced later in a fixed order; a set
// solver flag skips the launch).
template <typename V, typename X, int kEpi>
__global__ __launch_bounds__(kSellThreads) void sellp_spmv_kernel(int32_t nrows, int32_t C, int32_t log2c,
                                                                 int64_t nslices, int64_t grid_padded,
                                                                 const int32_t *__restrict__ sets,
                                                                 const int32_t *__restrict__ scol,
                                                                 const V *__restrict__ sval, const X *__restrict__ x,
                                                                 X *__restrict__ y, X alpha, X beta,
                                                                 const X *__restrict__ dot_with,
                                                                 X *__restrict__ partials, const KState *st)
{
    if (st != nullptr && st->flag != kRunning) return;
    __shared__ X part[kSellThreads];
    const int64_t s = xcd_remap(blockIdx.x, grid_padded);
    if (s >= nslices) return;
    const int tid = threadIdx.x;
    const int l = tid & (C - 1), g = tid >> log2c;
    const int G = kSellThreads >> log2c;
    const int32_t k0 = sets[s], w = sets[s + 1] - k0;
    const int32_t *__restrict__ cs = scol + (int64_t)k0 * C + l;
    const V *__restrict__ vs = sval + (int64_t)k0 * C + l;
    X sum = X(0);
    constexpr int U = 4;
    int32_t k = g;
    for (; k + (U - 1) * G < w; k += U * G) {
        int32_t cc[U];
        X vv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t q = (int64_t)(k + u * G) * C;
            cc[u] = ld_stream(cs + q);
            vv[u] = widen(ld_stream(vs + q));
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (cc[u] >= 0) sum += vv[u] * x[cc[u]];
    }
    for (; k < w; k += G) {
        const int64_t q = (int64_t)k * C;
        const int32_t c = ld_stream(cs + q);
        const X v = widen(ld_stream(vs + q));
        if (c >= 0) sum += v * x[c];
    }
    part[tid] = sum;
    __syncthreads();
    const int64_t row = s * C + l;
    X d1 = X(0), d2 = X(0);
    if (g == 0 && row < nrows) {
        X t = part[l];
        for (int j = 1; j < G; ++j) t += part[j * C + l];
        X out = alpha * t;
        if (beta != X(0)) out += beta * y[row];
        y[row] = out;
        if constexpr (kEpi >= 1) d1 = out * dot_with[row];
        if constexpr (kEpi >= 2) d2 = out * out;
    }
    if constexpr (kEpi > 0) {
        __shared__ X s_red[kSellThreads / kWave];
        X v[kEpi];
        v[0] = block_sum<X, kSellThreads>(d1, s_red);
        if constexpr (kEpi >= 2) v[kEpi - 1] = block_sum<X, kSellThreads>(d2, s_red);
        write_partials<X, kEpi>(v, partials, nslices, s);
    }
}

// SELL-P with 64-row slices: one wavefront per slice, one lane per row, four
// slot columns in flight per lane (the slot columns are read coalesced and,
// on banded matrices, so are the gathers of x); no cross-lane reduction.
template <typename V, typename X, int kEpi>
__global__ __launch_bounds__(kSellThreads) void sellp64_spmv_kernel(int32_t nrows, int64_t nslices,
                                                                   int64_t grid_padded,
                                                                   const int32_t *__restrict__ sets,
                                                                   const int32_t *__restrict__ scol,
                                                                   const V *__restrict__ sval,
                                                                   const X *__restrict__ x, X *__restrict__ y,
                                                                   X alpha, X beta, const X *__restrict__ dot_with,
                                                                   X *__restrict__ partials, const KState *st)
{
    if (st != nullptr && st->flag != kRunning) return;
    constexpr int kSlices = kSellThreads / kWave;  // slices per work-group
    const int64_t blk = xcd_remap(blockIdx.x, grid_padded);
    const int64_t nblocks = (nslices + kSlices - 1) / kSlices;
    if (blk >= nblocks) return;
    const int64_t s = blk * kSlices + threadIdx.x / kWave;
    const int l = lane_id();
    X d1 = X(0), d2 = X(0);
    if (s < nslices) {
        const int32_t k0 = sets[s], w = sets[s + 1] - k0;
        const int32_t *__restrict__ cs = scol + (int64_t)k0 * kWave + l;
        const V *__restrict__ vs = sval + (int64_t)k0 * kWave + l;
        X sum = X(0);
        constexpr int U = 4;
        int32_t k = 0;
        for (; k + U <= w; k += U) {
            int32_t cc[U];
            X vv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                cc[u] = ld_stream(cs + (int64_t)(k + u) * kWave);
                vv[u] = widen(ld_stream(vs + (int64_t)(k + u) * kWave));
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (cc[u] >= 0) sum += vv[u] * x[cc[u]];
        }
        for (; k < w; ++k) {
            const int32_t c = ld_stream(cs + (int64_t)k * kWave);
            const X v = widen(ld_stream(vs + (int64_t)k * kWave));
            if (c >= 0) sum += v * x[c];
        }
        const int64_t row = s * kWave + l;
        if (row < nrows) {
            X out = alpha * sum;
            if (beta != X(0)) out += beta * y[row];
            y[row] = out;
            if constexpr (kEpi >= 1) d1 = out * dot_with[row];
            if constexpr (kEpi >= 2) d2 = out * out;
        }
    }
    if constexpr (kEpi > 0) {
        __shared__ X s_red[kSellThreads / kWave];
        X v[kEpi];
        v[0] = block_sum<X, kSellThreads>(d1, s_red);
        if constexpr (kEpi >= 2) v[kEpi - 1] = block_sum<X, kSellThreads>(d2, s_red);
        write_partials<X, kEpi>(v, partials, nblocks, blk);
    }
}

int64_t sellp_dot_parts(const spx_matrix &A)
{
    const int64_t ns = A.nrows > 0 ? ceil_div(A.nrows, A.slice_size) : 1;
    return A.slice_size == kWave ? ceil_div(ns, kSellThreads / kWave) : ns;
}

template <typename V, typename X>
spx_status sellp_spmv_launch(const spx_matrix &A, const X *x, X *y, X alpha, X beta, hipStream_t stream, int epi,
                             const X *dot_with, X *partials, const KState *st)
{
    const int32_t C = A.slice_size;
    const int64_t ns = ceil_div(A.nrows, C);
    if (C == kWave) {
        const int64_t nblocks = sellp_dot_parts(A);
        const int64_t grid = pad_to_xcds(nblocks);
#define SPX_SELL64_LAUNCH(E)                                                                                       \
    sellp64_spmv_kernel<V, X, E><<<(unsigned)grid, kSellThreads, 0, stream>>>(                                     \
        A.nrows, ns, grid, A.slice_sets, A.ell_col, static_cast<const V *>(A.ell_val), x, y, alpha, beta, dot_with, \
        partials, st)
        if (epi == 2) SPX_SELL64_LAUNCH(2);
        else if (epi == 1) SPX_SELL64_LAUNCH(1);
        else SPX_SELL64_LAUNCH(0);
#undef SPX_SELL64_LAUNCH
        SPX_LAUNCHED();
        return SPX_OK;
    }
    int32_t log2c = 0;
    while ((1 << log2c) < C) ++log2c;
    const int64_t grid = pad_to_xcds(ns);
#define SPX_SELL_LAUNCH(E)                                                                                         \
    sellp_spmv_kernel<V, X, E><<<(unsigned)grid, kSellThreads, 0, stream>>>(                                       \
        A.nrows, C, log2c, ns, grid, A.slice_sets, A.ell_col, static_cast<const V *>(A.ell_val), x, y, alpha, beta, \
        dot_with, partials, st)
    if (epi == 2) SPX_SELL_LAUNCH(2);
    else if (epi == 1) SPX_SELL_LAUNCH(1);
    else SPX_SELL_LAUNCH(0);
#undef SPX_SELL_LAUNCH
    SPX_LAUNCHED();
    return SPX_OK;
}

#define SPX_INST(V, X)                                                                                          \
    template spx_status coo_spmv_launch<V, X>(const spx_matrix &, const X *, X *, X, X, hipStream_t);          \
    template spx_status ell_spmv_launch<V, X>(const spx_matrix &, const X *, X *, X, X, hipStream_t, int,        \
                                              const X *, X *, const KState *);                                    \
    template spx_status hyb_spmv_launch<V, X>(const spx_matrix &, const X *, X *, X, X, hipStream_t);          \
    template spx_status sellp_spmv_launch<V, X>(const spx_matrix &, const X *, X *, X, X, hipStream_t, int,      \
                                                const X *, X *, const KState *);
SPX_INST(double, double)
SPX_INST(float, float)
SPX_INST(_Float16, float)
#undef SPX_INST

}  // namespace spx
