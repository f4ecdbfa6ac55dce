/*
 * spx_oracle.c -- CPU oracle for the sparse matrix-vector product, format
 * conversion and Krylov solvers of the library.
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this code. It shares no code, header
 * or table with the GPU path: everything here is written out plainly, in
 * float64, in the order of the textbook definition, so that it can be checked
 * against the definitions by eye.
 *
 * The paper validates every GPU kernel against sequential CPU "reference"
 * kernels (Section 3.1, Section 3.5); this file plays that role. The matrix
 * formats (Coo, Csr, Ell, Hybrid) and solvers (CG, BiCG family, GMRES) are the
 * ones the paper lists among the library's features (Section 1); their
 * definitions follow the standard literature named at each function.
 *
 * Conventions: indices are int32, the CSR row pointer is int32 (nnz < 2^31),
 * ELL slot offsets are computed in int64. All arrays are caller-owned.
 * Functions return 0 on success and a negative ORC_E* code on bad input.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum {
    ORC_OK = 0,
    ORC_NOT_CONVERGED = 1,
    ORC_BREAKDOWN = 2,
    ORC_NONFINITE = 3,
    ORC_ZERO_DIAG = 4,
    ORC_EARG = -1,
    ORC_EFORMAT = -2,
    ORC_ERANGE = -3,
    ORC_ENOMEM = -4,
};

/* ------------------------------------------------------------------------ */
/* Error-free transformations (Ogita, Rump, Oishi, "Accurate sum and dot     */
/* product", SIAM J. Sci. Comput. 26(6), 2005): TwoSum (Knuth) and           */
/* TwoProduct via a fused multiply-add. The file is compiled with            */
/* -ffp-contract=off so that no other expression is fused.                   */
/* ------------------------------------------------------------------------ */
static void two_sum(double a, double b, double *s, double *e)
{
    double x = a + b;
    double z = x - a;
    *e = (a - (x - z)) + (b - z);
    *s = x;
}

static void two_prod(double a, double b, double *p, double *e)
{
    double x = a * b;
    *e = fma(a, b, -x);
    *p = x;
}

/* Dot2 accumulator: (hi, lo) keeps the sum as if computed in twice the
 * working precision, then rounded once. */
typedef struct { double hi, lo; } dot2_t;

static void dot2_add_prod(dot2_t *acc, double a, double b)
{
    double h, r, q;
    two_prod(a, b, &h, &r);
    two_sum(acc->hi, h, &acc->hi, &q);
    acc->lo += q + r;
}

static void dot2_add(dot2_t *acc, double a)
{
    double q;
    two_sum(acc->hi, a, &acc->hi, &q);
    acc->lo += q;
}

static double dot2_value(const dot2_t *acc) { return acc->hi + acc->lo; }

/* ------------------------------------------------------------------------ */
/* SpMV: y_i = alpha * sum_{p in row i} val[p] * x[col[p]] + beta * y_i.     */
/* With beta == 0 y is not read (BLAS convention).                           */
/* ------------------------------------------------------------------------ */

/* Plain float64, sequential summation in storage order. */
void orc_csr_spmv(int32_t n, const int32_t *rowptr, const int32_t *col, const double *val,
                  const double *x, double *y, double alpha, double beta)
{
    for (int32_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int32_t p = rowptr[i]; p < rowptr[i + 1]; ++p)
            s += val[p] * x[col[p]];
        y[i] = (beta == 0.0) ? alpha * s : alpha * s + beta * y[i];
    }
}

/* Dot2-accurate product: the row sum is computed as if in quadruple-like
 * precision and rounded once, so its error is about u*|sum| + O(u^2)*(|A||x|)_i.
 * absax (may be NULL) receives (|A| |x|)_i, the scale of the tolerance. */
void orc_csr_spmv_dot2(int32_t n, const int32_t *rowptr, const int32_t *col, const double *val,
                       const double *x, double *y, double alpha, double beta, double *absax)
{
    for (int32_t i = 0; i < n; ++i) {
        dot2_t acc = {0.0, 0.0};
        double a = 0.0;
        for (int32_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            dot2_add_prod(&acc, val[p], x[col[p]]);
            a += fabs(val[p]) * fabs(x[col[p]]);
        }
        double s = dot2_value(&acc);
        if (absax) absax[i] = a;
        y[i] = (beta == 0.0) ? alpha * s : alpha * s + beta * y[i];
    }
}

/* Plain float64 product straight from COO triples (row-major order). */
void orc_coo_spmv(int32_t n, int64_t nnz, const int32_t *row, const int32_t *col, const double *val,
                  const double *x, double *y, double alpha, double beta)
{
    double *acc = (double *)calloc((size_t)n > 0 ? (size_t)n : 1, sizeof(double));
    for (int64_t p = 0; p < nnz; ++p) acc[row[p]] += val[p] * x[col[p]];
    for (int32_t i = 0; i < n; ++i) y[i] = (beta == 0.0) ? alpha * acc[i] : alpha * acc[i] + beta * y[i];
    free(acc);
}

/* Plain float64 product straight from slot-major ELL (slot k of row i at
 * k*ld + i; column -1 marks padding). */
void orc_ell_spmv(int32_t n, int32_t K, int64_t ld, const int32_t *ecol, const double *eval,
                  const double *x, double *y, double alpha, double beta)
{
    for (int32_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int32_t k = 0; k < K; ++k) {
            int64_t q = (int64_t)k * ld + i;
            if (ecol[q] >= 0) s += eval[q] * x[ecol[q]];
        }
        y[i] = (beta == 0.0) ? alpha * s : alpha * s + beta * y[i];
    }
}

/* ------------------------------------------------------------------------ */
/* Canonical-form check of a CSR matrix.                                     */
/* Returns 0, ORC_EFORMAT (bad row pointer), -10 (unsorted), -11 (duplicate) */
/* or ORC_ERANGE (column out of range).                                      */
/* ------------------------------------------------------------------------ */
int orc_csr_check(int32_t n, int32_t ncols, const int32_t *rowptr, const int32_t *col)
{
    if (rowptr[0] != 0) return ORC_EFORMAT;
    for (int32_t i = 0; i < n; ++i) {
        if (rowptr[i + 1] < rowptr[i]) return ORC_EFORMAT;
        for (int32_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            if (col[p] < 0 || col[p] >= ncols) return ORC_ERANGE;
            if (p > rowptr[i]) {
                if (col[p] == col[p - 1]) return -11;
                if (col[p] < col[p - 1]) return -10;
            }
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Format conversion. Values are copied bit for bit (memcpy of the 8 bytes). */
/* ------------------------------------------------------------------------ */

/* COO row index of every stored entry, in CSR storage order. */
void orc_csr_to_coo(int32_t n, const int32_t *rowptr, int32_t *row_out)
{
    for (int32_t i = 0; i < n; ++i)
        for (int32_t p = rowptr[i]; p < rowptr[i + 1]; ++p) row_out[p] = i;
}

/* Row pointer from a row-major sorted COO row array. */
int orc_coo_to_csr(int32_t n, int64_t nnz, const int32_t *row, int32_t *rowptr_out)
{
    for (int32_t i = 0; i <= n; ++i) rowptr_out[i] = 0;
    for (int64_t p = 0; p < nnz; ++p) {
        if (row[p] < 0 || row[p] >= n) return ORC_ERANGE;
        if (p > 0 && row[p] < row[p - 1]) return -10;
        rowptr_out[row[p] + 1] += 1;
    }
    for (int32_t i = 0; i < n; ++i) rowptr_out[i + 1] += rowptr_out[i];
    return ORC_OK;
}

/* Largest row length. */
int32_t orc_max_row_length(int32_t n, const int32_t *rowptr)
{
    int32_t m = 0;
    for (int32_t i = 0; i < n; ++i)
        if (rowptr[i + 1] - rowptr[i] > m) m = rowptr[i + 1] - rowptr[i];
    return m;
}

/* CSR -> ELL of width K with leading dimension ld >= n. Slot k of row i
 * holds the row's k-th entry (ascending column) if k < len_i, else column -1
 * and value +0.0. Fails with ORC_EFORMAT if some row is longer than K. */
int orc_csr_to_ell(int32_t n, const int32_t *rowptr, const int32_t *col, const double *val,
                   int32_t K, int64_t ld, int32_t *ecol, double *eval)
{
    if (ld < n) return ORC_EARG;
    for (int32_t i = 0; i < n; ++i) {
        int32_t len = rowptr[i + 1] - rowptr[i];
        if (len > K) return ORC_EFORMAT;
        for (int32_t k = 0; k < K; ++k) {
            int64_t q = (int64_t)k * ld + i;
            if (k < len) {
                ecol[q] = col[rowptr[i] + k];
                memcpy(&eval[q], &val[rowptr[i] + k], sizeof(double));
            } else {
                ecol[q] = -1;
                eval[q] = 0.0;
            }
        }
    }
    return ORC_OK;
}

/* Number of stored (non-padding) slots of an ELL matrix. */
int64_t orc_ell_count(int32_t n, int32_t K, int64_t ld, const int32_t *ecol)
{
    int64_t c = 0;
    for (int32_t i = 0; i < n; ++i)
        for (int32_t k = 0; k < K; ++k)
            if (ecol[(int64_t)k * ld + i] >= 0) ++c;
    return c;
}

/* Stored entries of row i of an ELL matrix in slot order, padding dropped. */
static int32_t ell_row(int32_t i, int32_t K, int64_t ld, const int32_t *ecol, const double *eval,
                       int32_t *c_out, double *v_out)
{
    int32_t m = 0;
    for (int32_t k = 0; k < K; ++k) {
        int64_t q = (int64_t)k * ld + i;
        if (ecol[q] >= 0) {
            c_out[m] = ecol[q];
            memcpy(&v_out[m], &eval[q], sizeof(double));
            ++m;
        }
    }
    return m;
}

/* Merge of two column-ascending entry lists into one ascending list. */
static int32_t merge_row(const int32_t *ca, const double *va, int32_t na,
                         const int32_t *cb, const double *vb, int32_t nb,
                         int32_t *c_out, double *v_out)
{
    int32_t ia = 0, ib = 0, m = 0;
    while (ia < na || ib < nb) {
        int take_a = (ib >= nb) || (ia < na && ca[ia] <= cb[ib]);
        if (take_a) { c_out[m] = ca[ia]; memcpy(&v_out[m], &va[ia], sizeof(double)); ++ia; }
        else        { c_out[m] = cb[ib]; memcpy(&v_out[m], &vb[ib], sizeof(double)); ++ib; }
        ++m;
    }
    return m;
}

/* ELL -> CSR: padding slots dropped, entries kept in ascending column order
 * (slot entries of a canonical ELL already are). rowptr/col/val must have room
 * for n+1 / orc_ell_count entries. */
int orc_ell_to_csr(int32_t n, int32_t K, int64_t ld, const int32_t *ecol, const double *eval,
                   int32_t *rowptr, int32_t *col, double *val)
{
    int32_t *tc = (int32_t *)malloc(sizeof(int32_t) * (K > 0 ? K : 1));
    double *tv = (double *)malloc(sizeof(double) * (K > 0 ? K : 1));
    int32_t *sc = (int32_t *)malloc(sizeof(int32_t) * (K > 0 ? K : 1));
    double *sv = (double *)malloc(sizeof(double) * (K > 0 ? K : 1));
    if (!tc || !tv || !sc || !sv) { free(tc); free(tv); free(sc); free(sv); return ORC_ENOMEM; }
    rowptr[0] = 0;
    for (int32_t i = 0; i < n; ++i) {
        int32_t m = ell_row(i, K, ld, ecol, eval, tc, tv);
        /* insertion sort by column (stable), in case slots are not ascending */
        int32_t s = 0;
        for (int32_t a = 0; a < m; ++a) {
            int32_t b = s;
            while (b > 0 && sc[b - 1] > tc[a]) { sc[b] = sc[b - 1]; memcpy(&sv[b], &sv[b - 1], 8); --b; }
            sc[b] = tc[a];
            memcpy(&sv[b], &tv[a], 8);
            ++s;
        }
        for (int32_t a = 0; a < s; ++a) { col[rowptr[i] + a] = sc[a]; memcpy(&val[rowptr[i] + a], &sv[a], 8); }
        rowptr[i + 1] = rowptr[i] + s;
    }
    free(tc); free(tv); free(sc); free(sv);
    return ORC_OK;
}

/* Number of entries a CSR matrix keeps in the COO part of a width-K HYB. */
int64_t orc_hyb_coo_count(int32_t n, const int32_t *rowptr, int32_t K)
{
    int64_t c = 0;
    for (int32_t i = 0; i < n; ++i) {
        int32_t len = rowptr[i + 1] - rowptr[i];
        if (len > K) c += len - K;
    }
    return c;
}

/* CSR -> HYB(K): the ELL part holds the first min(len_i, K) entries of each
 * row (ELL layout as orc_csr_to_ell), the COO part the remaining entries in
 * row-major order. */
int orc_csr_to_hyb(int32_t n, const int32_t *rowptr, const int32_t *col, const double *val,
                   int32_t K, int64_t ld, int32_t *ecol, double *eval,
                   int32_t *crow, int32_t *ccol, double *cval)
{
    if (ld < n || K < 0) return ORC_EARG;
    int64_t c = 0;
    for (int32_t i = 0; i < n; ++i) {
        int32_t len = rowptr[i + 1] - rowptr[i];
        for (int32_t k = 0; k < K; ++k) {
            int64_t q = (int64_t)k * ld + i;
            if (k < len) {
                ecol[q] = col[rowptr[i] + k];
                memcpy(&eval[q], &val[rowptr[i] + k], 8);
            } else {
                ecol[q] = -1;
                eval[q] = 0.0;
            }
        }
        for (int32_t k = K; k < len; ++k) {
            crow[c] = i;
            ccol[c] = col[rowptr[i] + k];
            memcpy(&cval[c], &val[rowptr[i] + k], 8);
            ++c;
        }
    }
    return ORC_OK;
}

/* HYB -> CSR: per row, the ELL part (padding dropped) is merged with the
 * row's COO entries, ascending by column. The COO part must be row-sorted. */
int orc_hyb_to_csr(int32_t n, int32_t K, int64_t ld, const int32_t *ecol, const double *eval,
                   int64_t cnnz, const int32_t *crow, const int32_t *ccol, const double *cval,
                   int32_t *rowptr, int32_t *col, double *val)
{
    int32_t *tc = (int32_t *)malloc(sizeof(int32_t) * (K > 0 ? K : 1));
    double *tv = (double *)malloc(sizeof(double) * (K > 0 ? K : 1));
    if (!tc || !tv) { free(tc); free(tv); return ORC_ENOMEM; }
    int64_t c = 0;
    rowptr[0] = 0;
    for (int32_t i = 0; i < n; ++i) {
        int32_t m = ell_row(i, K, ld, ecol, eval, tc, tv);
        int64_t c0 = c;
        while (c < cnnz && crow[c] == i) ++c;
        if (c < cnnz && crow[c] < i) { free(tc); free(tv); return -10; }
        int32_t r = merge_row(tc, tv, m, ccol + c0, cval + c0, (int32_t)(c - c0),
                              col + rowptr[i], val + rowptr[i]);
        rowptr[i + 1] = rowptr[i] + r;
    }
    free(tc); free(tv);
    if (c != cnnz) return ORC_EFORMAT;
    return ORC_OK;
}

/* Automatic HYB width: the K in [0, maxlen] that minimises the stored bytes
 *   bytes(K) = n*K*(sv+si) + sum_i max(0, len_i - K) * (sv + 2*si),
 * smallest K on ties. Evaluated directly for every K over the histogram of
 * row lengths. */
int32_t orc_hyb_auto_width(int32_t n, const int32_t *rowptr, int32_t sv, int32_t si)
{
    int32_t maxlen = orc_max_row_length(n, rowptr);
    int64_t *hist = (int64_t *)calloc((size_t)maxlen + 1, sizeof(int64_t));
    for (int32_t i = 0; i < n; ++i) hist[rowptr[i + 1] - rowptr[i]] += 1;
    int32_t best_k = 0;
    double best = -1.0;
    for (int32_t K = 0; K <= maxlen; ++K) {
        double excess = 0.0;
        for (int32_t L = K + 1; L <= maxlen; ++L) excess += (double)hist[L] * (double)(L - K);
        double bytes = (double)n * K * (sv + si) + excess * (sv + 2 * si);
        if (best < 0.0 || bytes < best) { best = bytes; best_k = K; }
    }
    free(hist);
    return best_k;
}

/* ------------------------------------------------------------------------ */
/* SELL-P, the sliced ELL format with padding that the paper benchmarks as   */
/* Sellp (Section 4); layout as in Anzt, Tomov and Dongarra (2014): rows are */
/* grouped in slices of C consecutive rows; slice s stores its rows'         */
/* entries column-major within the slice, with width                         */
/*   w_s = T * ceil(max row length in the slice / T)                        */
/* (T is the stride factor); slice_sets[s] is the sum of the widths of the   */
/* slices before s, so entry k of row r = s*C + l sits at                    */
/*   (slice_sets[s] + k) * C + l.                                            */
/* Padding slots (and the lanes of a last, partial slice) hold column -1 and */
/* value +0. A row's entries occupy its first slots, ascending by column.    */
/* ------------------------------------------------------------------------ */

/* slice_sets[0..nslices]; returns ORC_ERANGE if the total width overflows
 * int32, ORC_EARG for C < 1 or T < 1. */
int orc_sellp_shape(int32_t n, const int32_t *rowptr, int32_t C, int32_t T, int32_t *slice_sets)
{
    if (C < 1 || T < 1) return ORC_EARG;
    int32_t nslices = (n + C - 1) / C;
    int64_t acc = 0;
    slice_sets[0] = 0;
    for (int32_t s = 0; s < nslices; ++s) {
        int32_t m = 0;
        for (int32_t r = s * C; r < n && r < (s + 1) * C; ++r) {
            int32_t len = rowptr[r + 1] - rowptr[r];
            if (len > m) m = len;
        }
        int32_t w = ((m + T - 1) / T) * T;
        acc += w;
        if (acc > INT32_MAX) return ORC_ERANGE;
        slice_sets[s + 1] = (int32_t)acc;
    }
    return ORC_OK;
}

int orc_csr_to_sellp(int32_t n, const int32_t *rowptr, const int32_t *col, const double *val, int32_t C,
                     const int32_t *slice_sets, int32_t *scol, double *sval)
{
    if (C < 1) return ORC_EARG;
    int32_t nslices = (n + C - 1) / C;
    for (int32_t s = 0; s < nslices; ++s) {
        int32_t w = slice_sets[s + 1] - slice_sets[s];
        for (int32_t l = 0; l < C; ++l) {
            int32_t r = s * C + l;
            int32_t len = (r < n) ? rowptr[r + 1] - rowptr[r] : 0;
            if (len > w) return ORC_EFORMAT;
            for (int32_t k = 0; k < w; ++k) {
                int64_t q = ((int64_t)slice_sets[s] + k) * C + l;
                if (k < len) {
                    scol[q] = col[rowptr[r] + k];
                    memcpy(&sval[q], &val[rowptr[r] + k], 8);
                } else {
                    scol[q] = -1;
                    sval[q] = 0.0;
                }
            }
        }
    }
    return ORC_OK;
}

/* y = alpha * A x + beta * y; each row summed in slot order. */
void orc_sellp_spmv(int32_t n, int32_t C, const int32_t *slice_sets, const int32_t *scol, const double *sval,
                    const double *x, double *y, double alpha, double beta)
{
    for (int32_t r = 0; r < n; ++r) {
        int32_t s = r / C, l = r % C;
        double acc = 0.0;
        for (int32_t k = 0; k < slice_sets[s + 1] - slice_sets[s]; ++k) {
            int64_t q = ((int64_t)slice_sets[s] + k) * C + l;
            if (scol[q] >= 0) acc += sval[q] * x[scol[q]];
        }
        y[r] = (beta == 0.0) ? alpha * acc : alpha * acc + beta * y[r];
    }
}

/* Stored entries of each row (slots up to the first padding slot). Returns
 * ORC_EFORMAT if a stored entry follows padding in some row. */
int64_t orc_sellp_count(int32_t n, int32_t C, const int32_t *slice_sets, const int32_t *scol)
{
    int64_t total = 0;
    for (int32_t r = 0; r < n; ++r) {
        int32_t s = r / C, l = r % C, w = slice_sets[s + 1] - slice_sets[s];
        int32_t k = 0;
        while (k < w && scol[((int64_t)slice_sets[s] + k) * C + l] >= 0) ++k;
        for (int32_t j = k; j < w; ++j)
            if (scol[((int64_t)slice_sets[s] + j) * C + l] >= 0) return ORC_EFORMAT;
        total += k;
    }
    return total;
}

int orc_sellp_to_csr(int32_t n, int32_t C, const int32_t *slice_sets, const int32_t *scol, const double *sval,
                     int32_t *rowptr, int32_t *col, double *val)
{
    rowptr[0] = 0;
    for (int32_t r = 0; r < n; ++r) {
        int32_t s = r / C, l = r % C, w = slice_sets[s + 1] - slice_sets[s];
        int32_t c = rowptr[r];
        for (int32_t k = 0; k < w; ++k) {
            int64_t q = ((int64_t)slice_sets[s] + k) * C + l;
            if (scol[q] < 0) break;
            col[c] = scol[q];
            memcpy(&val[c], &sval[q], 8);
            ++c;
        }
        rowptr[r + 1] = c;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Value casts, round to nearest even (IEEE 754).                           */
/* NaN maps to the canonical quiet NaN of the target with the sign kept.     */
/* ------------------------------------------------------------------------ */

/* float64 -> binary16 bits. Returns 1 when a finite input overflows to inf. */
static int f64_to_f16_bits(double d, uint16_t *out)
{
    uint64_t b;
    memcpy(&b, &d, 8);
    uint16_t sign = (uint16_t)((b >> 63) << 15);
    double a = fabs(d);
    if (isnan(d)) { *out = sign | 0x7E00u; return 0; }
    if (isinf(d)) { *out = sign | 0x7C00u; return 0; }
    /* binary16: 5 exponent bits (bias 15), 10 fraction bits; largest finite
     * 65504; subnormal spacing 2^-24. */
    if (a < ldexp(1.0, -14)) {
        double r = nearbyint(ldexp(a, 24));  /* units of 2^-24, rounded once */
        *out = sign | (uint16_t)r;           /* r == 1024 is the smallest normal */
        return 0;
    }
    int e;
    frexp(a, &e);                            /* a = f * 2^e, f in [0.5, 1) */
    e -= 1;                                  /* a in [2^e, 2^(e+1)) */
    double r = nearbyint(ldexp(a, 10 - e));  /* in [1024, 2048] */
    if (r == 2048.0) { r = 1024.0; e += 1; }
    if (e > 15) { *out = sign | 0x7C00u; return 1; }
    *out = sign | (uint16_t)((e + 15) << 10) | (uint16_t)((uint32_t)r - 1024u);
    return 0;
}

/* float64 -> float32 bits (the C conversion rounds to nearest even). */
static uint32_t f64_to_f32_bits(double d)
{
    uint64_t b;
    memcpy(&b, &d, 8);
    if (isnan(d)) return (uint32_t)((b >> 63) << 31) | 0x7FC00000u;
    float f = (float)d;
    uint32_t u;
    memcpy(&u, &f, 4);
    return u;
}

/* Cast of a value array. dst_type 1 = float32 (4-byte words), 2 = binary16
 * (2-byte words). Returns the number of finite inputs that overflowed. */
int64_t orc_cast_values(int64_t nnz, const double *src, int32_t dst_type, void *dst)
{
    int64_t overflow = 0;
    for (int64_t p = 0; p < nnz; ++p) {
        if (dst_type == 1) {
            uint32_t u = f64_to_f32_bits(src[p]);
            if (isfinite(src[p]) && (u & 0x7F800000u) == 0x7F800000u) ++overflow;
            ((uint32_t *)dst)[p] = u;
        } else {
            uint16_t h;
            overflow += f64_to_f16_bits(src[p], &h);
            ((uint16_t *)dst)[p] = h;
        }
    }
    return overflow;
}

/* binary16 bits -> float64 (exact). */
double orc_f16_to_f64(uint16_t h)
{
    int sign = h >> 15, e = (h >> 10) & 0x1F, f = h & 0x3FF;
    double v;
    if (e == 0) v = ldexp((double)f, -24);
    else if (e == 31) v = f ? NAN : INFINITY;
    else v = ldexp((double)(f + 1024), e - 25);
    return sign ? -v : v;
}

/* ------------------------------------------------------------------------ */
/* Vector helpers (plain float64 loops).                                     */
/* ------------------------------------------------------------------------ */
static double dot(int32_t n, const double *a, const double *b)
{
    double s = 0.0;
    for (int32_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

static double nrm2(int32_t n, const double *a) { return sqrt(dot(n, a, a)); }

/* Residual r = b - A x with every row sum taken by Dot2 (b enters the same
 * accumulator), and its 2-norm. */
double orc_residual(int32_t n, const int32_t *rowptr, const int32_t *col, const double *val,
                    const double *b, const double *x, double *r)
{
    double s2 = 0.0;
    for (int32_t i = 0; i < n; ++i) {
        dot2_t acc = {0.0, 0.0};
        dot2_add(&acc, b[i]);
        for (int32_t p = rowptr[i]; p < rowptr[i + 1]; ++p) dot2_add_prod(&acc, -val[p], x[col[p]]);
        double ri = dot2_value(&acc);
        if (r) r[i] = ri;
        s2 += ri * ri;
    }
    return sqrt(s2);
}

/* Scalar Jacobi preconditioner: M = diag(A). dinv[i] = 1 / a_ii. A missing,
 * zero or non-finite diagonal entry is ORC_ZERO_DIAG. */
int orc_jacobi_setup(int32_t n, const int32_t *rowptr, const int32_t *col, const double *val,
                     double *diag)
{
    for (int32_t i = 0; i < n; ++i) {
        double d = 0.0;
        for (int32_t p = rowptr[i]; p < rowptr[i + 1]; ++p)
            if (col[p] == i) d = val[p];
        if (d == 0.0 || !isfinite(d)) return ORC_ZERO_DIAG;
        diag[i] = d;
    }
    return ORC_OK;
}

/* z = M^{-1} r (M = diag, or identity when diag == NULL). */
static void apply_prec(int32_t n, const double *diag, const double *r, double *z)
{
    for (int32_t i = 0; i < n; ++i) z[i] = diag ? r[i] / diag[i] : r[i];
}

/* ------------------------------------------------------------------------ */
/* Block-Jacobi preconditioner (the paper's Section 1 names block-Jacobi     */
/* among the library's preconditioners; scalar Jacobi is its 1x1 case).      */
/* Block k holds rows and columns [k*bs, min(n, (k+1)*bs)); its dense        */
/* diagonal submatrix D_k is inverted by Gauss-Jordan elimination with       */
/* partial pivoting (largest |pivot|, first row on ties): for each pivot     */
/* column j, swap the pivot row into place, divide row j of [D | I] by the   */
/* pivot, then subtract a_rj * (row j) from every other row r. inv holds     */
/* nblocks blocks of bs*bs doubles, row-major; a last, smaller block of m    */
/* rows uses the leading m x m part. Returns ORC_ZERO_DIAG for a zero or     */
/* non-finite pivot.                                                         */
/* ------------------------------------------------------------------------ */
int orc_block_jacobi_setup(int32_t n, const int32_t *rowptr, const int32_t *col, const double *val, int32_t bs,
                           double *inv)
{
    if (bs < 1) return ORC_EARG;
    int32_t nb = (n + bs - 1) / bs;
    double *a = malloc(sizeof(double) * (size_t)bs * 2 * bs);
    if (!a) return ORC_ENOMEM;
    int status = ORC_OK;
    for (int32_t k = 0; k < nb && status == ORC_OK; ++k) {
        int32_t i0 = k * bs, m = (n - i0 < bs) ? n - i0 : bs, w = 2 * m;
        memset(a, 0, sizeof(double) * (size_t)m * w);
        for (int32_t r = 0; r < m; ++r) {
            for (int32_t p = rowptr[i0 + r]; p < rowptr[i0 + r + 1]; ++p)
                if (col[p] >= i0 && col[p] < i0 + m) a[r * w + (col[p] - i0)] = val[p];
            a[r * w + m + r] = 1.0;
        }
        for (int32_t j = 0; j < m; ++j) {
            int32_t piv = j;
            for (int32_t r = j + 1; r < m; ++r)
                if (fabs(a[r * w + j]) > fabs(a[piv * w + j])) piv = r;
            double d = a[piv * w + j];
            if (d == 0.0 || !isfinite(d)) { status = ORC_ZERO_DIAG; break; }
            if (piv != j)
                for (int32_t c = 0; c < w; ++c) {
                    double t = a[j * w + c];
                    a[j * w + c] = a[piv * w + c];
                    a[piv * w + c] = t;
                }
            for (int32_t c = 0; c < w; ++c) a[j * w + c] /= d;
            for (int32_t r = 0; r < m; ++r) {
                if (r == j) continue;
                double f = a[r * w + j];
                for (int32_t c = 0; c < w; ++c) a[r * w + c] -= f * a[j * w + c];
            }
        }
        for (int32_t r = 0; r < bs; ++r)
            for (int32_t c = 0; c < bs; ++c)
                inv[(size_t)k * bs * bs + (size_t)r * bs + c] = (r < m && c < m) ? a[r * w + m + c] : 0.0;
    }
    free(a);
    return status;
}

/* z = blockdiag(D_k^{-1}) r, each entry summed over the block's columns in
 * order. */
void orc_block_jacobi_apply(int32_t n, int32_t bs, const double *inv, const double *r, double *z)
{
    for (int32_t i = 0; i < n; ++i) {
        int32_t k = i / bs, i0 = k * bs, m = (n - i0 < bs) ? n - i0 : bs;
        double s = 0.0;
        for (int32_t j = 0; j < m; ++j) s += inv[(size_t)k * bs * bs + (size_t)(i - i0) * bs + j] * r[i0 + j];
        z[i] = s;
    }
}

/* A preconditioner: none (kind 0), scalar Jacobi (kind 1, diag), or block
 * Jacobi with kind x kind blocks (kind >= 2, inv). */
typedef struct {
    int32_t kind;
    double *diag, *inv;
} orc_prec;

static int prec_setup(orc_prec *P, int32_t kind, int32_t n, const int32_t *rowptr, const int32_t *col,
                      const double *val)
{
    P->kind = kind;
    P->diag = NULL;
    P->inv = NULL;
    if (kind == 1) {
        P->diag = malloc(sizeof(double) * (n > 0 ? n : 1));
        if (!P->diag) return ORC_ENOMEM;
        return orc_jacobi_setup(n, rowptr, col, val, P->diag);
    }
    if (kind >= 2) {
        int32_t nb = (n + kind - 1) / kind;
        P->inv = malloc(sizeof(double) * (size_t)(nb > 0 ? nb : 1) * kind * kind);
        if (!P->inv) return ORC_ENOMEM;
        return orc_block_jacobi_setup(n, rowptr, col, val, kind, P->inv);
    }
    return ORC_OK;
}

static void prec_apply(const orc_prec *P, int32_t n, const double *r, double *z)
{
    if (P->kind >= 2) orc_block_jacobi_apply(n, P->kind, P->inv, r, z);
    else apply_prec(n, P->diag, r, z);
}

static void prec_free(orc_prec *P)
{
    free(P->diag);
    free(P->inv);
}

typedef struct {
    int32_t status, iters, spmv_count, outer_iters;
    double relres_recursive, relres_true;
} orc_info;

/* ------------------------------------------------------------------------ */
/* Preconditioned conjugate gradients (Hestenes & Stiefel 1952; the          */
/* preconditioned form of Barrett et al., "Templates for the Solution of     */
/* Linear Systems", 1994). Stopping test on the unpreconditioned 2-norm of   */
/* the residual relative to ||b||; when the recursive residual passes, the   */
/* true residual b - A x decides, and a miss restarts the recurrences from   */
/* it. Iterations count the products q = A p.                                */
/* precond: 0 none, 1 scalar Jacobi, b >= 2 block Jacobi with b x b blocks.  */
/* x holds x0 on entry unless x0_zero.                                       */
/* ------------------------------------------------------------------------ */
int orc_cg(int32_t n, const int32_t *rowptr, const int32_t *col, const double *val,
           const double *b, double *x, double tol, int32_t maxit, int32_t precond, int32_t x0_zero,
           orc_info *info)
{
    memset(info, 0, sizeof(*info));
    double *r = malloc(sizeof(double) * n), *z = malloc(sizeof(double) * n);
    double *p = malloc(sizeof(double) * n), *q = malloc(sizeof(double) * n);
    orc_prec P;
    int ps = prec_setup(&P, precond, n, rowptr, col, val);
    if (!r || !z || !p || !q || ps == ORC_ENOMEM) { info->status = ORC_ENOMEM; goto out; }
    if (ps != ORC_OK) {
        info->status = ORC_ZERO_DIAG;
        goto out;
    }
    if (x0_zero) memset(x, 0, sizeof(double) * n);
    double bn = nrm2(n, b);
    if (!isfinite(bn)) { info->status = ORC_NONFINITE; goto out; }
    if (bn == 0.0) {
        memset(x, 0, sizeof(double) * n);
        info->status = ORC_OK;
        goto out;
    }
    /* r = b - A x */
    orc_csr_spmv(n, rowptr, col, val, x, q, 1.0, 0.0);
    for (int32_t i = 0; i < n; ++i) r[i] = b[i] - q[i];
    int restart = 1;
    double rho = 0.0;
    info->status = ORC_NOT_CONVERGED;
    if (nrm2(n, r) <= tol * bn) {
        info->status = ORC_OK;
        restart = 0;
        maxit = 0;
    }
    while (info->status == ORC_NOT_CONVERGED) {
        if (restart) {
            prec_apply(&P, n, r, z);
            memcpy(p, z, sizeof(double) * n);
            rho = dot(n, r, z);
            restart = 0;
        }
        if (info->iters >= maxit) break;
        orc_csr_spmv(n, rowptr, col, val, p, q, 1.0, 0.0);
        info->iters += 1;
        info->spmv_count += 1;
        double pq = dot(n, p, q);
        if (!isfinite(pq)) { info->status = ORC_NONFINITE; break; }
        if (pq <= 0.0) { info->status = ORC_BREAKDOWN; break; }
        double alpha = rho / pq;
        for (int32_t i = 0; i < n; ++i) x[i] += alpha * p[i];
        for (int32_t i = 0; i < n; ++i) r[i] -= alpha * q[i];
        double rn = nrm2(n, r);
        info->relres_recursive = rn / bn;
        if (!isfinite(rn)) { info->status = ORC_NONFINITE; break; }
        if (rn <= tol * bn) {
            double tn = orc_residual(n, rowptr, col, val, b, x, r);  /* r <- true residual */
            if (tn <= tol * bn) { info->status = ORC_OK; break; }
            restart = 1;
            continue;
        }
        prec_apply(&P, n, r, z);
        double rho_new = dot(n, r, z);
        double beta = rho_new / rho;
        rho = rho_new;
        for (int32_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
    }
    info->relres_true = orc_residual(n, rowptr, col, val, b, x, NULL) / bn;
out:
    free(r); free(z); free(p); free(q);
    prec_free(&P);
    return info->status;
}

/* ------------------------------------------------------------------------ */
/* BiCGSTAB (van der Vorst 1992), right-preconditioned as in Barrett et al., */
/* "Templates" (1994). One iteration = two products with A. Convergence is    */
/* tested on s (half step) and on r (full step), each confirmed by the true  */
/* residual; a true residual that misses restarts from it with r_hat = r.    */
/* ------------------------------------------------------------------------ */
int orc_bicgstab(int32_t n, const int32_t *rowptr, const int32_t *col, const double *val,
                 const double *b, double *x, double tol, int32_t maxit, int32_t precond,
                 int32_t x0_zero, orc_info *info)
{
    memset(info, 0, sizeof(*info));
    double *r = malloc(sizeof(double) * n), *rh = malloc(sizeof(double) * n);
    double *p = malloc(sizeof(double) * n), *v = malloc(sizeof(double) * n);
    double *ph = malloc(sizeof(double) * n), *s = malloc(sizeof(double) * n);
    double *sh = malloc(sizeof(double) * n), *t = malloc(sizeof(double) * n);
    double *diag = precond ? malloc(sizeof(double) * n) : NULL;
    if (!r || !rh || !p || !v || !ph || !s || !sh || !t || (precond && !diag)) {
        info->status = ORC_ENOMEM;
        goto out;
    }
    if (precond && orc_jacobi_setup(n, rowptr, col, val, diag) != ORC_OK) {
        info->status = ORC_ZERO_DIAG;
        goto out;
    }
    if (x0_zero) memset(x, 0, sizeof(double) * n);
    double bn = nrm2(n, b);
    if (!isfinite(bn)) { info->status = ORC_NONFINITE; goto out; }
    if (bn == 0.0) { memset(x, 0, sizeof(double) * n); info->status = ORC_OK; goto out; }
    orc_csr_spmv(n, rowptr, col, val, x, t, 1.0, 0.0);
    for (int32_t i = 0; i < n; ++i) r[i] = b[i] - t[i];
    double rho0 = 1.0, alpha = 1.0, omega = 1.0;
    int first = 1;
    info->status = ORC_NOT_CONVERGED;
    if (nrm2(n, r) <= tol * bn) {
        info->status = ORC_OK;
        goto done;
    }
    memcpy(rh, r, sizeof(double) * n);
    while (info->iters < maxit) {
        info->iters += 1;
        double rho = dot(n, rh, r);
        if (!isfinite(rho)) { info->status = ORC_NONFINITE; break; }
        if (rho == 0.0) { info->status = ORC_BREAKDOWN; break; }
        if (first) {
            memcpy(p, r, sizeof(double) * n);
            first = 0;
        } else {
            double beta = (rho / rho0) * (alpha / omega);
            for (int32_t i = 0; i < n; ++i) p[i] = r[i] + beta * (p[i] - omega * v[i]);
        }
        apply_prec(n, diag, p, ph);
        orc_csr_spmv(n, rowptr, col, val, ph, v, 1.0, 0.0);
        info->spmv_count += 1;
        double rhv = dot(n, rh, v);
        if (rhv == 0.0 || !isfinite(rhv)) { info->status = isfinite(rhv) ? ORC_BREAKDOWN : ORC_NONFINITE; break; }
        alpha = rho / rhv;
        for (int32_t i = 0; i < n; ++i) s[i] = r[i] - alpha * v[i];
        double sn = nrm2(n, s);
        info->relres_recursive = sn / bn;
        if (sn <= tol * bn) {
            for (int32_t i = 0; i < n; ++i) x[i] += alpha * ph[i];
            double tn = orc_residual(n, rowptr, col, val, b, x, r);
            if (tn <= tol * bn) { info->status = ORC_OK; break; }
            memcpy(rh, r, sizeof(double) * n);
            rho0 = alpha = omega = 1.0;
            first = 1;
            continue;
        }
        apply_prec(n, diag, s, sh);
        orc_csr_spmv(n, rowptr, col, val, sh, t, 1.0, 0.0);
        info->spmv_count += 1;
        double tt = dot(n, t, t);
        if (!isfinite(tt)) { info->status = ORC_NONFINITE; break; }
        if (tt == 0.0) { info->status = ORC_BREAKDOWN; break; }
        omega = dot(n, t, s) / tt;
        for (int32_t i = 0; i < n; ++i) x[i] += alpha * ph[i] + omega * sh[i];
        for (int32_t i = 0; i < n; ++i) r[i] = s[i] - omega * t[i];
        rho0 = rho;
        double rn = nrm2(n, r);
        info->relres_recursive = rn / bn;
        if (!isfinite(rn)) { info->status = ORC_NONFINITE; break; }
        if (rn <= tol * bn) {
            double tn = orc_residual(n, rowptr, col, val, b, x, r);
            if (tn <= tol * bn) { info->status = ORC_OK; break; }
            memcpy(rh, r, sizeof(double) * n);
            rho0 = alpha = omega = 1.0;
            first = 1;
            continue;
        }
        if (omega == 0.0) { info->status = ORC_BREAKDOWN; break; }
    }
done:
    info->relres_true = orc_residual(n, rowptr, col, val, b, x, NULL) / bn;
out:
    free(r); free(rh); free(p); free(v); free(ph); free(s); free(sh); free(t); free(diag);
    return info->status;
}

/* ------------------------------------------------------------------------ */
/* Transpose of an nrows x ncols CSR matrix: (A^T)_{ji} = A_{ij}. A counting */
/* sort by column: count each column's entries, prefix-sum the counts into   */
/* the row pointer of A^T (ncols + 1 entries), then walk A's rows in         */
/* increasing order appending every entry to its column, so the rows of A^T  */
/* come out sorted by column index.                                          */
/* ------------------------------------------------------------------------ */
int orc_csr_transpose(int32_t nrows, int32_t ncols, const int32_t *rowptr, const int32_t *col,
                      const double *val, int32_t *rowptr_t, int32_t *col_t, double *val_t)
{
    if (nrows < 0 || ncols < 0) return ORC_EARG;
    int32_t *next = malloc(sizeof(int32_t) * (ncols > 0 ? ncols : 1));
    if (!next) return ORC_ENOMEM;
    for (int32_t j = 0; j <= ncols; ++j) rowptr_t[j] = 0;
    for (int32_t p = 0; p < rowptr[nrows]; ++p) {
        if (col[p] < 0 || col[p] >= ncols) {
            free(next);
            return ORC_ERANGE;
        }
        rowptr_t[col[p] + 1] += 1;
    }
    for (int32_t j = 0; j < ncols; ++j) rowptr_t[j + 1] += rowptr_t[j];
    for (int32_t j = 0; j < ncols; ++j) next[j] = rowptr_t[j];
    for (int32_t i = 0; i < nrows; ++i)
        for (int32_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            int32_t d = next[col[p]]++;
            col_t[d] = i;
            val_t[d] = val[p];
        }
    free(next);
    return ORC_OK;
}

/* y = A^T x from the definition y_j = sum_i a_ij x_i: y = 0, then A's rows  */
/* in increasing i add a_ij x_i to y_j (A square, n x n).                   */
static void csr_spmv_t(int32_t n, const int32_t *rowptr, const int32_t *col, const double *val,
                       const double *x, double *y)
{
    for (int32_t j = 0; j < n; ++j) y[j] = 0.0;
    for (int32_t i = 0; i < n; ++i)
        for (int32_t p = rowptr[i]; p < rowptr[i + 1]; ++p) y[col[p]] += val[p] * x[i];
}

/* ------------------------------------------------------------------------ */
/* Preconditioned BiCG (Fletcher 1976, in the form of Barrett et al.,        */
/* "Templates", 1994); the paper lists BiCG among the library's solvers      */
/* (Section 1). The shadow residual starts as r~ = r. With M = diag(A)       */
/* (Jacobi) M^{-T} = M^{-1}. One iteration:                                 */
/*   z = M^{-1} r, z~ = M^{-T} r~, rho = z . r~ (zero: breakdown);           */
/*   p = z, p~ = z~ on the first step, else with beta = rho / rho_prev       */
/*   p = z + beta p, p~ = z~ + beta p~;                                      */
/*   q = A p, q~ = A^T p~, alpha = rho / (p~ . q) (zero: breakdown);         */
/*   x += alpha p, r -= alpha q, r~ -= alpha q~.                             */
/* Stopping as orc_cg; a true residual that misses restarts from it with     */
/* r~ = r. Each iteration counts two products (A and A^T). hist, if not      */
/* NULL, receives r and r~ at the start of iterations 1 .. nhist (2n doubles */
/* per iteration: r, then r~).                                               */
/* ------------------------------------------------------------------------ */
int orc_bicg(int32_t n, const int32_t *rowptr, const int32_t *col, const double *val,
             const double *b, double *x, double tol, int32_t maxit, int32_t precond, int32_t x0_zero,
             double *hist, int32_t nhist, orc_info *info)
{
    memset(info, 0, sizeof(*info));
    size_t nb = sizeof(double) * (size_t)(n > 0 ? n : 1);
    double *r = malloc(nb), *rt = malloc(nb), *z = malloc(nb), *zt = malloc(nb);
    double *p = malloc(nb), *pt = malloc(nb), *q = malloc(nb), *qt = malloc(nb);
    double *diag = precond ? malloc(nb) : NULL;
    if (!r || !rt || !z || !zt || !p || !pt || !q || !qt || (precond && !diag)) {
        info->status = ORC_ENOMEM;
        goto out;
    }
    if (precond && orc_jacobi_setup(n, rowptr, col, val, diag) != ORC_OK) {
        info->status = ORC_ZERO_DIAG;
        goto out;
    }
    if (x0_zero) memset(x, 0, sizeof(double) * n);
    double bn = nrm2(n, b);
    if (!isfinite(bn)) { info->status = ORC_NONFINITE; goto out; }
    if (bn == 0.0) { memset(x, 0, sizeof(double) * n); info->status = ORC_OK; goto out; }
    orc_csr_spmv(n, rowptr, col, val, x, q, 1.0, 0.0);
    for (int32_t i = 0; i < n; ++i) r[i] = b[i] - q[i];
    info->status = ORC_NOT_CONVERGED;
    if (nrm2(n, r) <= tol * bn) {
        info->status = ORC_OK;
        goto done;
    }
    int restart = 1, first = 1;
    double rho_prev = 1.0;
    while (info->iters < maxit) {
        if (restart) {
            memcpy(rt, r, sizeof(double) * n);
            restart = 0;
            first = 1;
        }
        if (hist && info->iters < nhist) {
            memcpy(hist + (size_t)2 * n * info->iters, r, sizeof(double) * n);
            memcpy(hist + (size_t)2 * n * info->iters + n, rt, sizeof(double) * n);
        }
        apply_prec(n, diag, r, z);
        apply_prec(n, diag, rt, zt);
        double rho = dot(n, z, rt);
        if (!isfinite(rho)) { info->status = ORC_NONFINITE; break; }
        if (rho == 0.0) { info->status = ORC_BREAKDOWN; break; }
        if (first) {
            memcpy(p, z, sizeof(double) * n);
            memcpy(pt, zt, sizeof(double) * n);
            first = 0;
        } else {
            double beta = rho / rho_prev;
            for (int32_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
            for (int32_t i = 0; i < n; ++i) pt[i] = zt[i] + beta * pt[i];
        }
        rho_prev = rho;
        orc_csr_spmv(n, rowptr, col, val, p, q, 1.0, 0.0);
        csr_spmv_t(n, rowptr, col, val, pt, qt);
        info->iters += 1;
        info->spmv_count += 2;
        double ptq = dot(n, pt, q);
        if (!isfinite(ptq)) { info->status = ORC_NONFINITE; break; }
        if (ptq == 0.0) { info->status = ORC_BREAKDOWN; break; }
        double alpha = rho / ptq;
        for (int32_t i = 0; i < n; ++i) x[i] += alpha * p[i];
        for (int32_t i = 0; i < n; ++i) r[i] -= alpha * q[i];
        for (int32_t i = 0; i < n; ++i) rt[i] -= alpha * qt[i];
        double rn = nrm2(n, r);
        info->relres_recursive = rn / bn;
        if (!isfinite(rn)) { info->status = ORC_NONFINITE; break; }
        if (rn <= tol * bn) {
            double tn = orc_residual(n, rowptr, col, val, b, x, r);
            if (tn <= tol * bn) { info->status = ORC_OK; break; }
            restart = 1;
        }
    }
done:
    info->relres_true = orc_residual(n, rowptr, col, val, b, x, NULL) / bn;
out:
    free(r); free(rt); free(z); free(zt); free(p); free(pt); free(q); free(qt); free(diag);
    return info->status;
}

/* ------------------------------------------------------------------------ */
/* Pipelined preconditioned CG (Ghysels & Vanroose, "Hiding global           */
/* synchronization latency in the preconditioned Conjugate Gradient          */
/* algorithm", Parallel Computing 40(7), 2014). The iterates of orc_cg in    */
/* exact arithmetic, rearranged so that an iteration has a single reduction  */
/* phase which can overlap the product with A. Kept alongside x and r:       */
/* u = M^{-1} r, w = A u, and the directions p, s = A p, q = M^{-1} s,       */
/* z = A q. Iteration i (M = diag(A) or the identity):                      */
/*   gamma = r . u, delta = w . u;  m = M^{-1} w, nv = A m;                 */
/*   i = 0: beta = 0, alpha = gamma / delta;                                */
/*   else   beta = gamma / gamma_prev,                                      */
/*          alpha = gamma / (delta - beta gamma / alpha_prev);              */
/*   (a denominator <= 0 is a breakdown: it equals p . A p);                */
/*   z = nv + beta z, q = m + beta q, s = w + beta s, p = u + beta p;       */
/*   x += alpha p, r -= alpha s, u -= alpha q, w -= alpha z.                */
/* Stopping as orc_cg on ||r||; a true residual that misses restarts the     */
/* recurrences from it (u = M^{-1} r, w = A u, i = 0). One product per       */
/* iteration plus one per (re)start.                                        */
/* ------------------------------------------------------------------------ */
int orc_pipecg(int32_t n, const int32_t *rowptr, const int32_t *col, const double *val,
               const double *b, double *x, double tol, int32_t maxit, int32_t precond, int32_t x0_zero,
               orc_info *info)
{
    memset(info, 0, sizeof(*info));
    size_t nb = sizeof(double) * (size_t)(n > 0 ? n : 1);
    double *r = malloc(nb), *u = malloc(nb), *w = malloc(nb), *m = malloc(nb), *nv = malloc(nb);
    double *z = malloc(nb), *q = malloc(nb), *s = malloc(nb), *p = malloc(nb);
    double *diag = precond ? malloc(nb) : NULL;
    if (!r || !u || !w || !m || !nv || !z || !q || !s || !p || (precond && !diag)) {
        info->status = ORC_ENOMEM;
        goto out;
    }
    if (precond && orc_jacobi_setup(n, rowptr, col, val, diag) != ORC_OK) {
        info->status = ORC_ZERO_DIAG;
        goto out;
    }
    if (x0_zero) memset(x, 0, sizeof(double) * n);
    double bn = nrm2(n, b);
    if (!isfinite(bn)) { info->status = ORC_NONFINITE; goto out; }
    if (bn == 0.0) { memset(x, 0, sizeof(double) * n); info->status = ORC_OK; goto out; }
    orc_csr_spmv(n, rowptr, col, val, x, nv, 1.0, 0.0);
    for (int32_t i = 0; i < n; ++i) r[i] = b[i] - nv[i];
    info->status = ORC_NOT_CONVERGED;
    if (nrm2(n, r) <= tol * bn) {
        info->status = ORC_OK;
        goto done;
    }
    int restart = 1, step = 0;
    double gamma_prev = 1.0, alpha_prev = 1.0;
    while (info->iters < maxit) {
        if (restart) {
            apply_prec(n, diag, r, u);
            orc_csr_spmv(n, rowptr, col, val, u, w, 1.0, 0.0);
            info->spmv_count += 1;
            restart = 0;
            step = 0;
        }
        double gamma = dot(n, r, u), delta = dot(n, w, u);
        apply_prec(n, diag, w, m);
        orc_csr_spmv(n, rowptr, col, val, m, nv, 1.0, 0.0);
        info->iters += 1;
        info->spmv_count += 1;
        if (!isfinite(gamma) || !isfinite(delta)) { info->status = ORC_NONFINITE; break; }
        double beta = 0.0, den = delta;
        if (step > 0) {
            beta = gamma / gamma_prev;
            den = delta - beta * gamma / alpha_prev;
        }
        if (!isfinite(den)) { info->status = ORC_NONFINITE; break; }
        if (den <= 0.0) { info->status = ORC_BREAKDOWN; break; }
        double alpha = gamma / den;
        if (step == 0) {
            memcpy(z, nv, nb);
            memcpy(q, m, nb);
            memcpy(s, w, nb);
            memcpy(p, u, nb);
        } else {
            for (int32_t i = 0; i < n; ++i) z[i] = nv[i] + beta * z[i];
            for (int32_t i = 0; i < n; ++i) q[i] = m[i] + beta * q[i];
            for (int32_t i = 0; i < n; ++i) s[i] = w[i] + beta * s[i];
            for (int32_t i = 0; i < n; ++i) p[i] = u[i] + beta * p[i];
        }
        for (int32_t i = 0; i < n; ++i) x[i] += alpha * p[i];
        for (int32_t i = 0; i < n; ++i) r[i] -= alpha * s[i];
        for (int32_t i = 0; i < n; ++i) u[i] -= alpha * q[i];
        for (int32_t i = 0; i < n; ++i) w[i] -= alpha * z[i];
        gamma_prev = gamma;
        alpha_prev = alpha;
        step += 1;
        double rn = nrm2(n, r);
        info->relres_recursive = rn / bn;
        if (!isfinite(rn)) { info->status = ORC_NONFINITE; break; }
        if (rn <= tol * bn) {
            double tn = orc_residual(n, rowptr, col, val, b, x, r);
            if (tn <= tol * bn) { info->status = ORC_OK; break; }
            restart = 1;
        }
    }
done:
    info->relres_true = orc_residual(n, rowptr, col, val, b, x, NULL) / bn;
out:
    free(r); free(u); free(w); free(m); free(nv); free(z); free(q); free(s); free(p); free(diag);
    return info->status;
}

/* ------------------------------------------------------------------------ */
/* Arnoldi with modified Gram-Schmidt (Saad, "Iterative Methods for Sparse   */
/* Linear Systems", 2nd ed., 2003, Ch. 6). Column j of V (length n, column-  */
/* major, n x (m+1)) is the j-th basis vector; H is (m+1) x m column-major.  */
/* One step: w = A M^{-1} v_j, h_ij = w . v_i, w -= h_ij v_i (i = 0..j),     */
/* h_{j+1,j} = ||w||, v_{j+1} = w / h_{j+1,j}. Returns h_{j+1,j}.           */
/* ------------------------------------------------------------------------ */
static double arnoldi_step(int32_t n, const int32_t *rowptr, const int32_t *col, const double *val,
                           const double *diag, double *V, double *H, int32_t m, int32_t j,
                           double *tmp)
{
    double *w = V + (int64_t)(j + 1) * n;
    apply_prec(n, diag, V + (int64_t)j * n, tmp);
    orc_csr_spmv(n, rowptr, col, val, tmp, w, 1.0, 0.0);
    for (int32_t i = 0; i <= j; ++i) {
        const double *vi = V + (int64_t)i * n;
        double h = dot(n, w, vi);
        H[(int64_t)j * (m + 1) + i] = h;
        for (int32_t k = 0; k < n; ++k) w[k] -= h * vi[k];
    }
    double hn = nrm2(n, w);
    H[(int64_t)j * (m + 1) + j + 1] = hn;
    if (hn != 0.0)
        for (int32_t k = 0; k < n; ++k) w[k] /= hn;
    return hn;
}

/* m Arnoldi steps from v0 (normalised here). Exposed for the Arnoldi
 * identity test A M^{-1} V_m = V_{m+1} Hbar_m. Returns the number of steps
 * taken (fewer than m on an exact breakdown). */
int32_t orc_arnoldi(int32_t n, const int32_t *rowptr, const int32_t *col, const double *val,
                    const double *v0, int32_t m, int32_t precond, double *V, double *H)
{
    double *diag = precond ? malloc(sizeof(double) * n) : NULL;
    double *tmp = malloc(sizeof(double) * n);
    if (precond) orc_jacobi_setup(n, rowptr, col, val, diag);
    memset(H, 0, sizeof(double) * (size_t)(m + 1) * m);
    double b0 = nrm2(n, v0);
    for (int32_t k = 0; k < n; ++k) V[k] = v0[k] / b0;
    int32_t j = 0;
    for (; j < m; ++j)
        if (arnoldi_step(n, rowptr, col, val, diag, V, H, m, j, tmp) == 0.0) { ++j; break; }
    free(diag);
    free(tmp);
    return j;
}

/* Restarted GMRES(m) (Saad & Schultz 1986), right preconditioned, MGS
 * Arnoldi, Givens rotations on the Hessenberg matrix. maxit counts Arnoldi
 * steps; every cycle starts from the true residual. */
int orc_gmres(int32_t n, const int32_t *rowptr, const int32_t *col, const double *val,
              const double *b, double *x, double tol, int32_t maxit, int32_t m, int32_t precond,
              int32_t x0_zero, orc_info *info)
{
    memset(info, 0, sizeof(*info));
    double *V = malloc(sizeof(double) * (size_t)n * (m + 1));
    double *H = malloc(sizeof(double) * (size_t)(m + 1) * m);
    double *cs = malloc(sizeof(double) * m), *sn = malloc(sizeof(double) * m);
    double *g = malloc(sizeof(double) * (m + 1)), *y = malloc(sizeof(double) * m);
    double *tmp = malloc(sizeof(double) * n), *u = malloc(sizeof(double) * n);
    double *diag = precond ? malloc(sizeof(double) * n) : NULL;
    if (!V || !H || !cs || !sn || !g || !y || !tmp || !u || (precond && !diag)) {
        info->status = ORC_ENOMEM;
        goto out;
    }
    if (precond && orc_jacobi_setup(n, rowptr, col, val, diag) != ORC_OK) {
        info->status = ORC_ZERO_DIAG;
        goto out;
    }
    if (x0_zero) memset(x, 0, sizeof(double) * n);
    double bn = nrm2(n, b);
    if (!isfinite(bn)) { info->status = ORC_NONFINITE; goto out; }
    if (bn == 0.0) { memset(x, 0, sizeof(double) * n); info->status = ORC_OK; goto out; }
    info->status = ORC_NOT_CONVERGED;
    while (1) {
        double beta = orc_residual(n, rowptr, col, val, b, x, V);  /* V[:,0] <- r */
        info->relres_recursive = beta / bn;
        if (!isfinite(beta)) { info->status = ORC_NONFINITE; break; }
        if (beta <= tol * bn) { info->status = ORC_OK; break; }
        if (info->iters >= maxit) break;
        info->outer_iters += 1;
        for (int32_t k = 0; k < n; ++k) V[k] /= beta;
        memset(H, 0, sizeof(double) * (size_t)(m + 1) * m);
        for (int32_t i = 0; i <= m; ++i) g[i] = 0.0;
        g[0] = beta;
        int32_t jend = 0;
        for (int32_t j = 0; j < m && info->iters < maxit; ++j) {
            double *Hj = H + (int64_t)j * (m + 1);
            double hn = arnoldi_step(n, rowptr, col, val, diag, V, H, m, j, tmp);
            info->iters += 1;
            info->spmv_count += 1;
            for (int32_t i = 0; i < j; ++i) {  /* previous rotations */
                double a = Hj[i], c = Hj[i + 1];
                Hj[i] = cs[i] * a + sn[i] * c;
                Hj[i + 1] = -sn[i] * a + cs[i] * c;
            }
            double rho = hypot(Hj[j], Hj[j + 1]);
            cs[j] = Hj[j] / rho;
            sn[j] = Hj[j + 1] / rho;
            Hj[j] = rho;
            Hj[j + 1] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            jend = j + 1;
            info->relres_recursive = fabs(g[j + 1]) / bn;
            if (!isfinite(g[j + 1])) { info->status = ORC_NONFINITE; goto done; }
            if (fabs(g[j + 1]) <= tol * bn || hn == 0.0) break;
        }
        /* back substitution H(0:jend, 0:jend) y = g(0:jend) */
        for (int32_t i = jend - 1; i >= 0; --i) {
            double s = g[i];
            for (int32_t k = i + 1; k < jend; ++k) s -= H[(int64_t)k * (m + 1) + i] * y[k];
            y[i] = s / H[(int64_t)i * (m + 1) + i];
        }
        /* x += M^{-1} (V y) */
        for (int32_t k = 0; k < n; ++k) u[k] = 0.0;
        for (int32_t i = 0; i < jend; ++i)
            for (int32_t k = 0; k < n; ++k) u[k] += y[i] * V[(int64_t)i * n + k];
        apply_prec(n, diag, u, tmp);
        for (int32_t k = 0; k < n; ++k) x[k] += tmp[k];
    }
done:
    info->relres_true = orc_residual(n, rowptr, col, val, b, x, NULL) / bn;
out:
    free(V); free(H); free(cs); free(sn); free(g); free(y); free(tmp); free(u); free(diag);
    return info->status;
}

/* ------------------------------------------------------------------------ */
/* Mixed-precision iterative refinement (Moler 1967; Carson & Higham 2018).  */
/* Outer loop in float64: r = b - A64 x, stop when ||r|| <= tol ||b||;       */
/* scale s = ||r||_inf, rhs = fl32(r / s); inner unpreconditioned CG in      */
/* float32 (vectors and accumulation) on the low-precision matrix, whose     */
/* values are given as float32 (binary16-stored values are passed widened,   */
/* which is exact), from zero to relative residual                          */
/* max(inner_tol, tol ||b|| / (2 ||r||)); x += s * d. The inner CG stops on  */
/* its recursive residual.                                                   */
/* ------------------------------------------------------------------------ */
static int32_t cg_f32(int32_t n, const int32_t *rowptr, const int32_t *col, const float *val,
                      const float *b, float *x, float tol, int32_t maxit,
                      float *r, float *p, float *q)
{
    float bb = 0.0f;
    for (int32_t i = 0; i < n; ++i) bb += b[i] * b[i];
    float bn = sqrtf(bb);
    for (int32_t i = 0; i < n; ++i) { x[i] = 0.0f; r[i] = b[i]; p[i] = b[i]; }
    float rho = bb;
    int32_t it = 0;
    if (bn == 0.0f) return 0;
    while (it < maxit) {
        for (int32_t i = 0; i < n; ++i) {
            float s = 0.0f;
            for (int32_t k = rowptr[i]; k < rowptr[i + 1]; ++k) s += val[k] * p[col[k]];
            q[i] = s;
        }
        ++it;
        float pq = 0.0f;
        for (int32_t i = 0; i < n; ++i) pq += p[i] * q[i];
        if (!(pq > 0.0f) || !isfinite(pq)) return -it;
        float alpha = rho / pq;
        for (int32_t i = 0; i < n; ++i) x[i] += alpha * p[i];
        for (int32_t i = 0; i < n; ++i) r[i] -= alpha * q[i];
        float rr = 0.0f;
        for (int32_t i = 0; i < n; ++i) rr += r[i] * r[i];
        if (sqrtf(rr) <= tol * bn) break;
        float beta = rr / rho;
        rho = rr;
        for (int32_t i = 0; i < n; ++i) p[i] = r[i] + beta * p[i];
    }
    return it;
}

int orc_ir(int32_t n, const int32_t *rowptr, const int32_t *col, const double *val64,
           const float *val_low, const double *b, double *x, double tol, double inner_tol,
           int32_t max_outer, int32_t inner_maxit, orc_info *info)
{
    memset(info, 0, sizeof(*info));
    double *r = malloc(sizeof(double) * n);
    float *rl = malloc(sizeof(float) * n), *d = malloc(sizeof(float) * n);
    float *w1 = malloc(sizeof(float) * n), *w2 = malloc(sizeof(float) * n), *w3 = malloc(sizeof(float) * n);
    if (!r || !rl || !d || !w1 || !w2 || !w3) { info->status = ORC_ENOMEM; goto out; }
    memset(x, 0, sizeof(double) * n);
    double bn = nrm2(n, b);
    if (bn == 0.0) { info->status = ORC_OK; goto out; }
    info->status = ORC_NOT_CONVERGED;
    for (int32_t outer = 0;; ++outer) {
        double rn = orc_residual(n, rowptr, col, val64, b, x, r);
        info->spmv_count += 1;
        info->relres_true = rn / bn;
        info->relres_recursive = rn / bn;
        if (!isfinite(rn)) { info->status = ORC_NONFINITE; break; }
        if (rn <= tol * bn) { info->status = ORC_OK; break; }
        if (outer >= max_outer) break;
        double s = 0.0;
        for (int32_t i = 0; i < n; ++i) if (fabs(r[i]) > s) s = fabs(r[i]);
        for (int32_t i = 0; i < n; ++i) rl[i] = (float)(r[i] / s);
        /* the inner solve only has to close the remaining gap to tol * ||b||
         * (with a factor 2 of margin), never less than inner_tol */
        double itol = 0.5 * tol * bn / rn;
        if (itol < inner_tol) itol = inner_tol;
        int32_t it = cg_f32(n, rowptr, col, val_low, rl, d, (float)itol, inner_maxit, w1, w2, w3);
        info->outer_iters += 1;
        if (it < 0) { info->iters += -it; info->spmv_count += -it; info->status = ORC_BREAKDOWN; break; }
        info->iters += it;
        info->spmv_count += it;
        for (int32_t i = 0; i < n; ++i) x[i] += s * (double)d[i];
    }
out:
    free(r); free(rl); free(d); free(w1); free(w2); free(w3);
    return info->status;
}

/* ------------------------------------------------------------------------ */
/* Subwarp group model (Section 3.3): contiguous groups of Size lanes inside */
/* a warp of warpsize lanes. For thread tid:                                 */
/*   Rank       = tid % Size                                                 */
/*   LaneOffset = floor((tid % warpsize) / Size) * Size                      */
/*   Mask       = (~0 >> (warpsize - Size)) << LaneOffset                    */
/* with ~0 a warpsize-bit mask. ballot = (warp ballot & Mask) >> LaneOffset, */
/* any = (warp ballot & Mask) != 0, all = (warp ballot & Mask) == Mask.      */
/* ------------------------------------------------------------------------ */
void orc_subwarp_params(int32_t tid, int32_t size, int32_t warpsize, int32_t *rank,
                        int32_t *lane_offset, uint64_t *mask)
{
    uint64_t full = (warpsize == 64) ? ~(uint64_t)0 : (((uint64_t)1 << warpsize) - 1);
    *rank = tid % size;
    *lane_offset = ((tid % warpsize) / size) * size;
    *mask = (full >> (warpsize - size)) << *lane_offset;
}

/* Per-thread subwarp ballot / any / all of pred over nthreads threads. */
void orc_subwarp_vote(const int32_t *pred, int32_t nthreads, int32_t size, int32_t warpsize,
                      uint64_t *ballot, int32_t *any, int32_t *all)
{
    for (int32_t t = 0; t < nthreads; ++t) {
        int32_t w0 = (t / warpsize) * warpsize;
        uint64_t warp_ballot = 0;
        for (int32_t l = 0; l < warpsize && w0 + l < nthreads; ++l)
            if (pred[w0 + l]) warp_ballot |= (uint64_t)1 << l;
        int32_t rank, off;
        uint64_t mask;
        orc_subwarp_params(t, size, warpsize, &rank, &off, &mask);
        ballot[t] = (warp_ballot & mask) >> off;
        any[t] = (warp_ballot & mask) != 0;
        all[t] = (warp_ballot & mask) == mask;
    }
}

/* Subwarp sum by the xor butterfly of the reduction kernel in Section 3.3:
 * for bitmask = 1, 2, 4, ... < Size every lane adds the value its partner
 * lane (lane ^ bitmask) held before the step. log2(Size) steps; every lane
 * of a group ends with the group sum. nthreads must be a multiple of Size. */
int32_t orc_subwarp_reduce(const double *in, double *out, int32_t nthreads, int32_t size)
{
    double *cur = malloc(sizeof(double) * nthreads), *prev = malloc(sizeof(double) * nthreads);
    memcpy(cur, in, sizeof(double) * nthreads);
    int32_t steps = 0;
    for (int32_t bitmask = 1; bitmask < size; bitmask <<= 1) {
        memcpy(prev, cur, sizeof(double) * nthreads);
        for (int32_t t = 0; t < nthreads; ++t) cur[t] = prev[t] + prev[t ^ bitmask];
        ++steps;
    }
    memcpy(out, cur, sizeof(double) * nthreads);
    free(cur);
    free(prev);
    return steps;
}

/* Inclusive segmented sum: a segment starts at every head flag and at every
 * multiple of width; out[t] = in[t] + out[t-1] inside a segment. */
void orc_segmented_scan(const double *in, const int32_t *head, double *out, int32_t nthreads,
                        int32_t width)
{
    for (int32_t t = 0; t < nthreads; ++t) {
        if (head[t] || t % width == 0) out[t] = in[t];
        else out[t] = out[t - 1] + in[t];
    }
}
