"""Pins of the oracle's SELL-P format (the sliced ELL with padding that the
paper benchmarks as Sellp, Section 4): a layout worked out by hand, the two
degenerate slice sizes that reduce to CSR (one row per slice) and to ELL
(one slice), bitwise round trips, exact rational products and the padding
count evaluated independently with numpy."""
import numpy as np
import pytest

import oracle as O
from paper_2006_14290_amd import synth as S
from test_oracle_formats import _bits, _same_csr, _special_matrix
from test_oracle_spmv import U, exact_matvec


def _hand_matrix():
    # rows of lengths 1, 3, 0, 2, 4 (n = 5)
    d = np.zeros((5, 5))
    d[0, 0] = 1
    d[1, 1], d[1, 2], d[1, 4] = 2, 3, 4
    d[3, 0], d[3, 3] = 5, 6
    d[4, 0], d[4, 1], d[4, 2], d[4, 3] = 7, 8, 9, 10
    return S.from_dense(d)


def test_sellp_hand_layout():
    # C = 2, T = 2: slices {0,1} (max 3 -> width 4), {2,3} (max 2 -> 2), {4} (max 4 -> 4)
    P = O.csr_to_sellp(_hand_matrix(), C=2, T=2)
    np.testing.assert_array_equal(P.slice_sets, [0, 4, 6, 10])
    # slot (slice_sets[s] + k) * C + l of row s*C + l
    np.testing.assert_array_equal(
        P.col, [0, 1, -1, 2, -1, 4, -1, -1, -1, 0, -1, 3, 0, -1, 1, -1, 2, -1, 3, -1])
    np.testing.assert_array_equal(
        P.val, [1, 2, 0, 3, 0, 4, 0, 0, 0, 5, 0, 6, 7, 0, 8, 0, 9, 0, 10, 0])


def test_sellp_one_row_per_slice_is_csr():
    A = _special_matrix()
    P = O.csr_to_sellp(A, C=1, T=1)
    np.testing.assert_array_equal(P.slice_sets, A.rowptr)
    np.testing.assert_array_equal(P.col, A.col)
    np.testing.assert_array_equal(_bits(P.val), _bits(A.val))


def test_sellp_one_slice_is_ell():
    A = _special_matrix()
    P = O.csr_to_sellp(A, C=A.n, T=1)
    E = O.csr_to_ell(A)
    np.testing.assert_array_equal(P.slice_sets, [0, E.K])
    np.testing.assert_array_equal(P.col, E.col)
    np.testing.assert_array_equal(_bits(P.val), _bits(E.val))


@pytest.mark.parametrize("C,T", [(1, 1), (2, 1), (64, 1), (64, 4), (7, 3), (100, 8)])
def test_sellp_round_trip(C, T):
    A = _special_matrix()
    P = O.csr_to_sellp(A, C=C, T=T)
    _same_csr(A, O.sellp_to_csr(P))
    assert np.all(np.diff(P.slice_sets) % T == 0)


@pytest.mark.parametrize("C,T", [(64, 1), (8, 2), (3, 1)])
def test_sellp_product_exact(C, T):
    A = S.random_small(70, 0.12, seed=31, empty_rows=(0, 1, 69), long_rows=(5, 64))
    x = S.uniform_vector(A.n, seed=7)
    ex = np.array([float(v) for v in exact_matvec(A, x)])
    _, absax = O.csr_spmv_dot2(A, x)
    k = np.maximum(np.diff(A.rowptr), 1)
    bound = (k * U / (1 - k * U)) * absax * 1.0000001
    P = O.csr_to_sellp(A, C=C, T=T)
    y = O.sellp_spmv(P, x)
    assert np.all(np.abs(y - ex) <= bound)
    yb = O.sellp_spmv(P, x, y=np.ones(A.n), alpha=-2.0, beta=0.5)
    assert np.all(np.abs(yb - (-2.0 * ex + 0.5)) <= 2 * bound + U)


def test_sellp_padding_count_27pt():
    A = S.stencil27_random(12, seed=0)
    lens = np.diff(A.rowptr)
    for C, T in ((64, 1), (32, 4)):
        P = O.csr_to_sellp(A, C=C, T=T)
        nsl = -(-A.n // C)
        widths = [int(-(-lens[s * C:(s + 1) * C].max() // T) * T) for s in range(nsl)]
        assert int(P.slice_sets[-1]) == sum(widths)
        assert int((P.col >= 0).sum()) == A.nnz
