"""Pins of the oracle's SpMV and subwarp model against facts independent of it:
exact rational dense products, closed forms of stencil operators, and the
paper's subwarp definitions evaluated by hand (Section 3.3)."""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
from paper_2006_14290_amd import synth as S

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
U = 2.0 ** -53


def exact_matvec(A, x):
    """Exact dense product with rational arithmetic, rounded once at the end."""
    out = []
    for i in range(A.n):
        s = Fraction(0)
        for p in range(A.rowptr[i], A.rowptr[i + 1]):
            s += Fraction(float(A.val[p])) * Fraction(float(x[A.col[p]]))
        out.append(s)
    return out


def _cases():
    yield S.random_small(37, 0.2, seed=1, empty_rows=(0, 5, 36), long_rows=(3, 20))
    yield S.random_small(64, 0.05, seed=2, empty_rows=tuple(range(10, 20)))
    yield S.random_small(1, 1.0, seed=3)
    yield S.random_small(65, 0.5, seed=4, long_rows=(64,))
    a = np.zeros((6, 6))
    a[1, 1] = 0.0  # explicit zero kept below
    yield S.from_dense(a, keep_zeros=True)


@pytest.mark.parametrize("case", list(range(5)))
def test_spmv_vs_exact_rational(case):
    A = list(_cases())[case]
    x = S.uniform_vector(A.n, seed=case)
    ex = exact_matvec(A, x)
    y2, absax = O.csr_spmv_dot2(A, x)
    y1 = O.csr_spmv(A, x)
    lens = np.diff(A.rowptr)
    for i in range(A.n):
        e = float(ex[i])
        # Dot2 result: faithful to the exact sum (error u|s| + O(u^2)|A||x|)
        assert abs(y2[i] - e) <= U * abs(e) + 1e-28 * absax[i]
        # plain sequential sum: gamma_k bound (Higham, Ch. 3)
        k = max(int(lens[i]), 1)
        assert abs(y1[i] - e) <= (k * U / (1 - k * U)) * absax[i] * 1.0000001
        if absax[i] == 0:
            assert y1[i] == 0.0 and y2[i] == 0.0


def test_alpha_beta_semantics():
    A = S.random_small(30, 0.3, seed=5, empty_rows=(7,))
    x = S.uniform_vector(A.n, seed=1)
    y0 = S.uniform_vector(A.n, seed=2)
    ex = exact_matvec(A, x)
    y, _ = O.csr_spmv_dot2(A, x, y0, alpha=-2.5, beta=0.75)
    for i in range(A.n):
        e = -2.5 * float(ex[i]) + 0.75 * y0[i]
        assert abs(y[i] - e) <= 4 * U * (abs(2.5 * float(ex[i])) + abs(0.75 * y0[i])) + 1e-300
    # beta == 0: y is write-only, NaN in it does not propagate
    ynan = np.full(A.n, np.nan)
    y, _ = O.csr_spmv_dot2(A, x, ynan, alpha=1.0, beta=0.0)
    assert np.all(np.isfinite(y))
    y = O.csr_spmv(A, x, ynan, alpha=1.0, beta=0.0)
    assert np.all(np.isfinite(y))
    assert y[7] == 0.0


def _missing_neighbour_sum(shape, coeff_axis, f):
    """Closed form of (A f)(p) for a stencil with eliminated Dirichlet boundary
    and f linear on the infinite grid: the infinite stencil annihilates f, so
    the product equals the sum, over neighbours that fall outside the grid, of
    coefficient times f there."""
    d = len(shape)
    grids = np.meshgrid(*[np.arange(s) for s in shape], indexing="ij")
    coords = [g.transpose(tuple(range(d - 1, -1, -1))).reshape(-1) for g in grids]
    out = np.zeros(coords[0].size)
    for a in range(d):
        for sgn in (-1, 1):
            q = [c.copy() for c in coords]
            q[a] = q[a] + sgn
            outside = (q[a] < 0) | (q[a] >= shape[a])
            out[outside] += coeff_axis[a] * f(q)[outside]
    return out, coords


@pytest.mark.parametrize("N", [1, 2, 7, 16])
def test_poisson2d_closed_forms(N):
    A = S.poisson2d(N)
    assert A.nnz == 5 * N * N - 4 * N
    one = np.ones(A.n)
    y = O.csr_spmv(A, one)
    exp, coords = _missing_neighbour_sum((N, N), (1.0, 1.0), lambda q: np.ones(q[0].size))
    np.testing.assert_array_equal(y, exp)
    # a linear grid function is annihilated at interior rows (column-permutation detector)
    for fx in (lambda q: q[0].astype(float), lambda q: 3.0 * q[1] - 2.0 * q[0] + 5.0):
        g = fx(coords)
        y = O.csr_spmv(A, g)
        exp, _ = _missing_neighbour_sum((N, N), (1.0, 1.0), fx)
        np.testing.assert_array_equal(y, exp)
    # quadratic: A_inf (i^2) = -2 everywhere
    g = coords[0].astype(float) ** 2
    y = O.csr_spmv(A, g)
    exp, _ = _missing_neighbour_sum((N, N), (1.0, 1.0), lambda q: q[0].astype(float) ** 2)
    np.testing.assert_array_equal(y, exp - 2.0)


@pytest.mark.parametrize("N,c", [(5, (1.0, 1.0, 1.0)), (6, (1.0, 1.0, 0.01)), (3, (2.0, 0.5, 0.25))])
def test_poisson3d_closed_forms(N, c):
    A = S.poisson3d_7pt(N, *c)
    assert A.nnz == 7 * N ** 3 - 6 * N ** 2
    one = np.ones(A.n)
    f = lambda q: 2.0 * q[0] - q[1] + 3.0 * q[2] + 1.0  # noqa: E731
    exp, coords = _missing_neighbour_sum((N, N, N), c, f)
    y = O.csr_spmv(A, f(coords))
    # exact for integer coefficients; the 0.01 coefficient rounds (|err| <= a few ulps)
    tol = 0.0 if all(float(v).is_integer() or v in (0.5, 0.25) for v in c) else 64 * U * 4.02 * 30
    assert np.max(np.abs(y - exp)) <= tol
    exp1, _ = _missing_neighbour_sum((N, N, N), c, lambda q: np.ones(q[0].size))
    y1 = O.csr_spmv(A, one)
    assert np.max(np.abs(y1 - exp1)) <= (0.0 if tol == 0.0 else 8 * U * 4.02)


def test_convdiff_row_sums():
    # Interior rows of the upwind operator sum to 0 (diag 36 = 3*11 + 3*1).
    N = 6
    A = S.convdiff3d_upwind(N)
    y = O.csr_spmv(A, np.ones(A.n))
    lens = np.diff(A.rowptr)
    assert np.all(y[lens == 7] == 0.0)
    assert np.all(y[lens < 7] > 0.0)


def test_27pt_counts_and_bruteforce():
    N = 5
    A = S.stencil27_random(N, seed=3)
    assert A.nnz == (3 * N - 2) ** 3
    assert O.csr_check(A) == 0
    x = S.uniform_vector(A.n, seed=9)
    ex = exact_matvec(A, x)
    y2, absax = O.csr_spmv_dot2(A, x)
    for i in range(A.n):
        assert abs(y2[i] - float(ex[i])) <= U * abs(float(ex[i])) + 1e-28 * absax[i]


def test_coo_and_ell_products_match_exact():
    A = S.random_small(40, 0.15, seed=11, empty_rows=(2, 3), long_rows=(39,))
    x = S.uniform_vector(A.n, seed=3)
    ex = np.array([float(v) for v in exact_matvec(A, x)])
    _, absax = O.csr_spmv_dot2(A, x)
    k = np.maximum(np.diff(A.rowptr), 1)
    bound = (k * U / (1 - k * U)) * absax * 1.0000001
    row = O.csr_to_coo_rows(A)
    yc = O.coo_spmv(A.n, row, A.col, A.val, x)
    assert np.all(np.abs(yc - ex) <= bound)
    E = O.csr_to_ell(A, ld=A.n + 13)
    ye = O.ell_spmv(A.n, E.K, E.ld, E.col, E.val, x)
    assert np.all(np.abs(ye - ex) <= bound)


def test_csr_check_codes():
    A = S.random_small(10, 0.5, seed=1)
    assert O.csr_check(A) == 0
    bad = S.CSR(A.n, A.rowptr.copy(), A.col.copy(), A.val.copy())
    r = int(np.argmax(np.diff(A.rowptr) >= 2))
    p = A.rowptr[r]
    bad.col[p], bad.col[p + 1] = bad.col[p + 1], bad.col[p]
    assert O.csr_check(bad) == -10
    bad.col[p] = bad.col[p + 1]
    assert O.csr_check(bad) == -11
    bad = S.CSR(A.n, A.rowptr.copy(), A.col.copy(), A.val.copy())
    bad.col[0] = A.n
    assert O.csr_check(bad) == -3


# ---------------------------------------------------------------- subwarp model
def _golden():
    with open(os.path.join(GOLDEN, "subwarp_model.json")) as f:
        return json.load(f)


def test_subwarp_params_golden():
    g = _golden()
    for c in g["params"]:
        r, o, m = O.subwarp_params(c["tid"], c["size"], c["warpsize"])
        assert (r, o, m) == (c["rank"], c["lane_offset"], int(c["mask"], 16)), c


def test_subwarp_vote_golden_and_bruteforce():
    g = _golden()["ballot_odd_lanes"]
    pred = np.arange(128) % 2
    b, a, l = O.subwarp_vote(pred, g["size"])
    assert np.all(b == int(g["ballot"], 16)) and np.all(a == g["any"]) and np.all(l == g["all"])
    rng = np.random.default_rng(0)
    for size in (1, 2, 4, 8, 16, 32, 64):
        pred = (rng.random(192) < 0.5).astype(np.int32)
        pred[64:64 + size] = 1  # one all-true group
        pred[128:128 + size] = 0  # one all-false group
        b, a, l = O.subwarp_vote(pred, size)
        for t in range(pred.size):
            g0 = (t // size) * size
            bits = sum(int(pred[g0 + k]) << k for k in range(size))
            assert int(b[t]) == bits
            assert a[t] == (bits != 0)
            assert l[t] == (bits == (1 << size) - 1)


def test_subwarp_reduce_steps_and_sums():
    g = _golden()
    for size, steps in g["reduce_steps"].items():
        size = int(size)
        data = np.arange(128, dtype=np.float64)
        out, st = O.subwarp_reduce(data, size)
        assert st == steps
        groups = data.reshape(-1, size).sum(axis=1)  # integers: exact
        np.testing.assert_array_equal(out, np.repeat(groups, size))
    assert round(g["reduce_steps"]["4"] / g["reduce_steps"]["64"], 3) == g["theory_ratio_wave64_size4_vs_64"]
    assert round(g["reduce_steps"]["4"] / g["reduce_steps"]["32"], 3) == g["theory_ratio_warp32_size4_vs_32"]


def test_segmented_scan_bruteforce():
    rng = np.random.default_rng(1)
    data = rng.integers(-50, 50, 256).astype(np.float64)
    head = (rng.random(256) < 0.2).astype(np.int32)
    out = O.segmented_scan(data, head, 64)
    start = 0
    for t in range(256):
        if head[t] or t % 64 == 0:
            start = t
        assert out[t] == data[start:t + 1].sum()
