"""Canonical-form checks of host CSR arrays through the C ABI
(spx_validate_csr_host, the check spx_serve_submit applies to every
request). Pure host code: runs without a GPU and touches no device."""
import numpy as np
import pytest

from paper_2006_14290_amd import synth as S

spx = pytest.importorskip("paper_2006_14290_amd.spx")


def _small():
    return S.random_small(40, 0.15, seed=4, empty_rows=(0, 17, 39), long_rows=(5,))


def _check(rowptr, col, n=None, ncols=None, nnz=None):
    n = len(rowptr) - 1 if n is None else n
    return spx.validate_csr_host(n, n if ncols is None else ncols, rowptr, col, nnz)


def test_canonical_matrices_pass():
    for A in (_small(), S.poisson2d(9), S.stencil27_random(5), S.zipf_matrix(3000, seed=2)):
        assert _check(A.rowptr, A.col) == spx.OK
    # empty matrix and all-empty rows
    assert _check(np.zeros(1, np.int32), np.zeros(0, np.int32)) == spx.OK
    assert _check(np.zeros(6, np.int32), np.zeros(0, np.int32)) == spx.OK


def test_row_pointer_errors_are_format():
    A = _small()
    rp = A.rowptr.copy()
    rp[0] = 1
    assert _check(rp, A.col) == spx.ERR_FORMAT
    rp = A.rowptr.copy()
    rp[10], rp[11] = rp[11], rp[10]  # a decreasing step (rows 9..11 are non-empty)
    assert rp[11] < rp[10]
    assert _check(rp, A.col) == spx.ERR_FORMAT
    assert "decreases" in spx.last_error()
    # rowptr[n] != nnz
    assert _check(A.rowptr, A.col, nnz=A.nnz - 1) == spx.ERR_FORMAT


@pytest.mark.parametrize("bad", [-1, 40, 1 << 30])
def test_column_out_of_range(bad):
    A = _small()
    col = A.col.copy()
    p = A.rowptr[21] + 1 if A.rowptr[22] - A.rowptr[21] > 1 else A.rowptr[5]
    col[p] = bad
    assert _check(A.rowptr, col) == spx.ERR_RANGE
    assert f"position {p}" in spx.last_error()
    # a narrower matrix: the last column becomes out of range
    assert _check(A.rowptr, A.col, ncols=int(A.col.max())) == spx.ERR_RANGE


def test_unsorted_and_duplicate_rows():
    A = _small()
    lens = np.diff(A.rowptr)
    i = int(np.flatnonzero(lens >= 3)[0])
    b = A.rowptr[i]
    col = A.col.copy()
    col[b], col[b + 1] = col[b + 1], col[b]
    assert _check(A.rowptr, col) == spx.ERR_UNSORTED
    col = A.col.copy()
    col[b + 1] = col[b]
    assert _check(A.rowptr, col) == spx.ERR_DUPLICATE
    assert f"position {b}" in spx.last_error()


def test_precedence_range_over_unsorted_over_duplicate():
    A = _small()
    lens = np.diff(A.rowptr)
    rows = np.flatnonzero(lens >= 3)
    r0, r1, r2 = (int(r) for r in rows[:3])
    col = A.col.copy()
    col[A.rowptr[r0] + 1] = col[A.rowptr[r0]]                               # duplicate, first by position
    col[A.rowptr[r1]], col[A.rowptr[r1] + 1] = col[A.rowptr[r1] + 1], col[A.rowptr[r1]]  # unsorted
    assert _check(A.rowptr, col) == spx.ERR_UNSORTED
    col[A.rowptr[r2] + 2] = 40                                              # range, last by position
    assert _check(A.rowptr, col) == spx.ERR_RANGE
    # rows that cross each other's boundary are not compared: descending at a row start is fine
    B = S.CSR(3, np.array([0, 2, 4, 5], np.int32), np.array([1, 2, 0, 1, 2], np.int32), np.ones(5))
    assert _check(B.rowptr, B.col) == spx.OK


def test_argument_errors():
    assert spx._lib.spx_validate_csr_host(-1, 3, 0, None, None) == spx.ERR_ARG
    assert spx._lib.spx_validate_csr_host(3, 3, 2, None, None) == spx.ERR_ARG
