"""Pins of the oracle's format conversions and value casts: bitwise round
trips, closed-form counts, an independent library (scipy / numpy casts) and
hand-evaluated IEEE 754 binary16 roundings."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
from paper_2006_14290_amd import synth as S


def _bits(a):
    return np.ascontiguousarray(a).view(np.uint64 if a.dtype == np.float64 else np.uint32)


def _special_matrix():
    A = S.random_small(50, 0.2, seed=21, empty_rows=(0, 13, 49), long_rows=(7,))
    v = A.val.copy()
    v[0] = -0.0
    v[1] = np.frombuffer(np.uint64(0x7FF800000000BEEF).tobytes(), np.float64)[0]  # NaN payload
    v[2] = 0.0  # explicit zero stays stored
    return S.CSR(A.n, A.rowptr, A.col, v)


def _same_csr(A, B):
    np.testing.assert_array_equal(np.asarray(A.rowptr, np.int32), np.asarray(B.rowptr, np.int32))
    np.testing.assert_array_equal(np.asarray(A.col, np.int32), np.asarray(B.col, np.int32))
    np.testing.assert_array_equal(_bits(np.asarray(A.val)), _bits(np.asarray(B.val)))


def test_coo_rows_match_scipy():
    A = _special_matrix()
    row = O.csr_to_coo_rows(A)
    m = sp.csr_matrix((np.ones(A.nnz), A.col, A.rowptr), shape=(A.n, A.n)).tocoo()
    np.testing.assert_array_equal(row, m.row)
    np.testing.assert_array_equal(O.coo_to_csr_rowptr(A.n, row), A.rowptr)


@pytest.mark.parametrize("ld_extra", [0, 7])
def test_ell_round_trip_and_layout(ld_extra):
    A = _special_matrix()
    K = O.max_row_length(A)
    assert K == int(np.diff(A.rowptr).max())
    E = O.csr_to_ell(A, ld=A.n + ld_extra)
    assert E.K == K
    lens = np.diff(A.rowptr)
    for i in (0, 7, 13, 20):
        for k in range(K):
            q = k * E.ld + i
            if k < lens[i]:
                assert E.col[q] == A.col[A.rowptr[i] + k]
            else:
                assert E.col[q] == -1 and _bits(E.val[q:q + 1])[0] == 0
    _same_csr(A, O.ell_to_csr(E))
    with pytest.raises(ValueError):
        O.csr_to_ell(A, K=K - 1)


@pytest.mark.parametrize("K", [0, 1, 3, None])
def test_hyb_round_trip_and_counts(K):
    A = _special_matrix()
    H = O.csr_to_hyb(A, K=K)
    K = H.ell.K
    lens = np.diff(A.rowptr).astype(np.int64)
    assert len(H.row) == np.maximum(lens - K, 0).sum()
    assert np.all(np.diff(H.row) >= 0)
    _same_csr(A, O.hyb_to_csr(H))


def _hand_hyb_matrix():
    # six rows of lengths 1, 3, 0, 5, 2, 0 (columns ascending, values 1..13 in entry order)
    rowptr = np.array([0, 1, 4, 4, 9, 11, 11], np.int32)
    col = np.array([4, 0, 2, 5, 0, 1, 2, 3, 5, 1, 4], np.int32)
    return S.CSR(6, rowptr, col, np.arange(1.0, 12.0))


def test_hyb_split_hand_worked_width2():
    """The split the Hybrid format of Section 1 implies (ELL part = each row's
    first min(len, K) entries, COO part = the rest in row-major order),
    written out by hand for K = 2 and a leading dimension above n."""
    H = O.csr_to_hyb(_hand_hyb_matrix(), K=2, ld=8)
    E = H.ell
    assert (E.K, E.ld) == (2, 8)
    # slot 0 then slot 1, eight rows each (rows 6 and 7 are beyond n: never written)
    exp_col = [4, 0, -1, 0, 1, -1, -1, -1,
               -1, 2, -1, 1, 4, -1, -1, -1]
    exp_val = [1, 2, 0, 5, 10, 0, 0, 0,
               0, 3, 0, 6, 11, 0, 0, 0]
    np.testing.assert_array_equal(E.col, exp_col)
    np.testing.assert_array_equal(_bits(E.val), _bits(np.array(exp_val, np.float64)))
    # COO part: row 1's third entry, then row 3's last three, in row-major order
    np.testing.assert_array_equal(H.row, [1, 3, 3, 3])
    np.testing.assert_array_equal(H.col, [5, 2, 3, 5])
    np.testing.assert_array_equal(H.val, [4.0, 7.0, 8.0, 9.0])


def test_hyb_split_hand_worked_wide_and_zero():
    A = _hand_hyb_matrix()
    # K above every row length: everything in the ELL part, left-packed, no COO part
    H = O.csr_to_hyb(A, K=7)
    assert len(H.row) == 0 and H.ell.ld == 6
    lens = [1, 3, 0, 5, 2, 0]
    exp = np.full((7, 6), -1, np.int32)
    for i, L in enumerate(lens):
        exp[:L, i] = A.col[A.rowptr[i]:A.rowptr[i] + L]
    np.testing.assert_array_equal(H.ell.col.reshape(7, 6), exp)
    # K = 0: the COO part is the whole matrix in CSR entry order
    H0 = O.csr_to_hyb(A, K=0)
    assert H0.ell.col.size == 0
    np.testing.assert_array_equal(H0.row, [0, 1, 1, 1, 3, 3, 3, 3, 3, 4, 4])
    np.testing.assert_array_equal(H0.col, A.col)
    np.testing.assert_array_equal(H0.val, A.val)


def test_hyb_auto_width_hand_examples():
    # lengths [1,1,1,10], sv=8, si=4: bytes(K) = 4*K*12 + excess*16
    # K=0: 208, K=1: 48+144=192, K=2: 96+128=224 -> K=1
    A = S.CSR(4, np.array([0, 1, 2, 3, 13], np.int32), np.array([0, 1, 2] + list(range(10)), np.int32),
              np.ones(13))
    assert O.hyb_auto_width(A, 8, 4) == 1
    # all rows equal length L -> K = L (no COO part is cheapest)
    B = S.poisson2d(1)
    assert O.hyb_auto_width(B) == 1
    # one huge row among empty rows -> K = 0 (pure COO)
    C = S.CSR(5, np.array([0, 0, 0, 0, 0, 5], np.int32), np.arange(5, dtype=np.int32), np.ones(5))
    assert O.hyb_auto_width(C) == 0


def _auto_k_threshold(lens, sv, si):
    """Equivalent rule: the first K at which the fraction of rows longer than
    K drops below (sv+si)/(sv+2si) (the marginal bytes of one more ELL column
    versus the COO entries it absorbs); ties keep the smaller K."""
    n = lens.size
    thr = (sv + si) / (sv + 2 * si)
    K = 0
    while K < lens.max() and (lens > K).sum() / n > thr:
        K += 1
    return K


@pytest.mark.parametrize("maker", ["27pt", "zipf", "rand"])
@pytest.mark.parametrize("sv", [8, 4])
def test_hyb_auto_width_threshold_rule(maker, sv):
    if maker == "27pt":
        A = S.stencil27_random(40)  # (38/40)^3 of the rows are full: K = 27
    elif maker == "zipf":
        A = S.zipf_matrix(20000, seed=1)
    else:
        A = S.random_small(300, 0.03, seed=5)
    lens = np.diff(A.rowptr).astype(np.int64)
    assert O.hyb_auto_width(A, sv, 4) == _auto_k_threshold(lens, sv, 4)
    if maker == "27pt":
        assert O.hyb_auto_width(A, sv, 4) == 27
    if maker == "zipf":
        assert O.hyb_auto_width(A, sv, 4) == 1


def test_stencil_nnz_closed_forms():
    assert S.poisson2d(64).nnz == 20224
    for N in (3, 10):
        assert S.stencil27_random(N).nnz == (3 * N - 2) ** 3
        assert S.poisson3d_7pt(N).nnz == 7 * N ** 3 - 6 * N ** 2
    assert O.max_row_length(S.stencil27_random(6)) == 27


def test_cast_f16_hand_values():
    cases = [
        (1.0, 0x3C00, 0), (-2.0, 0xC000, 0), (65504.0, 0x7BFF, 0),
        (65519.99, 0x7BFF, 0), (65520.0, 0x7C00, 1), (-1e6, 0xFC00, 1),
        (2.0 ** -24, 0x0001, 0), (2.0 ** -25, 0x0000, 0), (3 * 2.0 ** -25, 0x0002, 0),
        (2.0 ** -14, 0x0400, 0), (1 + 2.0 ** -11, 0x3C00, 0), (1 + 3 * 2.0 ** -11, 0x3C02, 0),
        (-0.0, 0x8000, 0), (np.inf, 0x7C00, 0), (0.1, 0x2E66, 0), (1023 * 2.0 ** -24 + 2.0 ** -25, 0x0400, 0),
    ]
    vals = np.array([c[0] for c in cases])
    h, ov = O.cast_values(vals, "f16")
    got = h.view(np.uint16)
    for (v, exp, _), g in zip(cases, got):
        assert int(g) == exp, (v, hex(int(g)), hex(exp))
    assert ov == sum(c[2] for c in cases)
    nan, _ = O.cast_values(np.array([np.nan, -np.nan]), "f16")
    assert list(nan.view(np.uint16)) == [0x7E00, 0xFE00]


def test_cast_matches_numpy_rne():
    rng = np.random.default_rng(3)
    v = np.concatenate([rng.uniform(-1, 1, 5000), rng.standard_normal(5000) * 1e4,
                        np.ldexp(rng.uniform(-1, 1, 2000), rng.integers(-30, 0, 2000)),
                        np.ldexp(rng.uniform(-1, 1, 2000), rng.integers(-160, 130, 2000))])
    h, _ = O.cast_values(v, "f16")
    with np.errstate(over="ignore"):
        ref16 = v.astype(np.float16)
    np.testing.assert_array_equal(h.view(np.uint16), ref16.view(np.uint16))
    f, _ = O.cast_values(v, "f32")
    with np.errstate(over="ignore"):
        ref32 = v.astype(np.float32)
    np.testing.assert_array_equal(f.view(np.uint32), ref32.view(np.uint32))
    for bits in (0x0001, 0x03FF, 0x0400, 0x3C00, 0x7BFF, 0xC000):
        assert O.f16_to_f64(bits) == float(np.array([bits], np.uint16).view(np.float16)[0])


def test_isotropic_7pt_exact_in_f16():
    A = S.poisson3d_7pt(6)
    h, ov = O.cast_values(A.val, "f16")
    assert ov == 0
    np.testing.assert_array_equal(h.astype(np.float64), A.val)
