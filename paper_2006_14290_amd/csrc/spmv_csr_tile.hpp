// spmv_csr_tile.hpp -- one tile of the load-balanced CSR product, as a
// device function shared by the CSR kernel and the wide batched solver.
#pragma once

#include "common.hpp"
#include "krylov.hpp"
#include "spmv_csr.hpp"
#include "wave.hpp"

namespace spx {

// First index r in [lo, hi] with rowptr[r] >= key, assuming the answer lies in
// [lo, hi]; *val receives rowptr[r]. Executed by one whole wavefront (64-ary
// search: one dependent load per round); every lane returns the answer.
__device__ inline int64_t lower_bound_wave(const int32_t *__restrict__ rowptr, int64_t lo, int64_t hi, int64_t key,
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

// Tile k of kTile nonzeros, processed by the calling work-group, which
// owns the rows that start inside its tile: it reads their bounds from
// the precomputed partition (or finds them with two wavefront searches),
// issues every value/column load of the pass before the first gather, stages
// the products in LDS and reduces each row with an adaptive subwarp. Rows
// longer than the rest of the pass continue in further passes, carrying their
// partial sum in LDS.
// kEpi: 0 = plain product; 1 = also sum_i y_i*w_i; 2 = also sum_i y_i*w_i
// and sum_i y_i*y_i. With a solver state the sums are reduced across tiles
// (deterministically, one partial per tile at dot_partials[j * ntiles + k]).
template <typename V, typename X, int kEpi, int kThreads, int kTile, int kVec, bool kLate>
__device__ __forceinline__ void csr_tile(int64_t k, int32_t nrows, int64_t nnz, int64_t ntiles,
                                         const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                                         const V *__restrict__ val, const X *__restrict__ x, X *__restrict__ y,
                                         X alpha, X beta, const X *__restrict__ dot_with,
                                         X *__restrict__ dot_partials, const int32_t *__restrict__ part)
{
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
    // kSlack extra entries let a pass run up to kSlack entries past the
    // tile, so the row that crosses into the next tile usually finishes in
    // the same pass instead of costing a second round of loads
    constexpr int kSlack = kCsrSlack;
    constexpr int kStage = kTile + kSlack;
    static_assert(kSlack % kVec == 0 && kSlack / kVec <= kThreads, "slack must split into whole vectors");
    // values are staged in their arithmetic type (binary16 is widened to
    // float once, while staging, instead of at every use in the row loop)
    using SV = typename acc_of<V>::type;
    typedef SV SVV __attribute__((ext_vector_type(kVec)));
    constexpr size_t kLdsBytes = kLate ? (size_t)kStage * (sizeof(int32_t) + sizeof(SV)) : (size_t)kStage * sizeof(A);
    __shared__ __align__(16) unsigned char s_raw[kLdsBytes];
    A *prod = reinterpret_cast<A *>(s_raw);
    SV *s_val = reinterpret_cast<SV *>(s_raw);
    int32_t *s_col = reinterpret_cast<int32_t *>(s_raw + (size_t)kStage * sizeof(SV));
    __shared__ int32_t s_rp[kThreads + 1];
    __shared__ int64_t s_b[4];
    __shared__ A s_carry;

    const int tid = threadIdx.x;
    __syncthreads();  // LDS of a previous tile handled by this work-group is consumed
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
        const int64_t w1 = (e - a0 > kStage) ? a0 + kTile : e;
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
        // the slack entries [a0 + kTile, w1), one vector per thread
        CV cs;
        VV vs;
        const int64_t sbase = a0 + kTile + (int64_t)tid * kVec;
        const bool slack = tid < kSlack / kVec && sbase < w1;
        if (slack) {
#pragma unroll
            for (int j = 0; j < kVec; ++j) {
                const bool ok = sbase + j < w1;
                cs[j] = ok ? col[sbase + j] : 0;
                vs[j] = ok ? val[sbase + j] : V(0);
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
                SVV sv;
#pragma unroll
                for (int j = 0; j < kVec; ++j) sv[j] = widen(vv[u][j]);
                *reinterpret_cast<SVV *>(&s_val[(u * kThreads + tid) * kVec]) = sv;
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
        if (slack) {
            if constexpr (kLate) {
                SVV sv;
#pragma unroll
                for (int j = 0; j < kVec; ++j) sv[j] = widen(vs[j]);
                *reinterpret_cast<SVV *>(&s_val[kTile + tid * kVec]) = sv;
                *reinterpret_cast<CV *>(&s_col[kTile + tid * kVec]) = cs;
            } else {
                typedef A AV __attribute__((ext_vector_type(kVec)));
                AV pv;
#pragma unroll
                for (int j = 0; j < kVec; ++j) pv[j] = (sbase + j < w1) ? widen(vs[j]) * x[cs[j]] : A(0);
                *reinterpret_cast<AV *>(&prod[kTile + tid * kVec]) = pv;
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
                        for (int p = a + sl; p < b; p += size) sum += s_val[p] * x[s_col[p]];
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


}  // namespace spx
