"""GPU CSR transpose, BiCG and pipelined CG against the oracle.

Transpose: bit-exact against the oracle's counting-sort transpose (rows,
columns and value bits) on ragged, empty, rectangular, heavy-column and
multi-tile inputs, float64/float32/binary16 values, and at the 128^3
convection-diffusion size. BiCG and pipelined CG: the true relative residual
is recomputed on the host with the oracle's Dot2 residual, iteration counts
are compared with the oracle's, and the status codes are forced by input."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2006_14290_amd import synth as S

from gpu_util import dev, host

pytestmark = pytest.mark.gpu

spx = pytest.importorskip("paper_2006_14290_amd.spx")


def _problem(A, seed=0):
    xs = S.uniform_vector(A.n, seed=seed, purpose="xstar")
    b, _ = O.csr_spmv_dot2(A, xs)
    return xs, b


def _true_relres(A, b, x):
    _, rn = O.residual(A, b, x)
    return rn / np.linalg.norm(b)


def _check_transpose(A, ncols=None, dtype=None):
    nc = A.n if ncols is None else ncols
    dt = spx.F64 if dtype is None else dtype
    Ad = spx.csr_from_host(A, dtype=dt)
    if ncols is not None:
        Ad.ncols = ncols
    At = spx.csr_transpose(Ad)
    rpt, ct, vt = O.csr_transpose(A, ncols=nc)
    np.testing.assert_array_equal(host(At.rowptr), rpt)
    np.testing.assert_array_equal(host(At.colidx)[: A.nnz], ct)
    # values are copied bit for bit: compare with the stored (rounded) values
    vref = vt.astype({spx.F64: np.float64, spx.F32: np.float32, spx.F16: np.float16}[dt])
    got = host(At.vals)[: A.nnz]
    np.testing.assert_array_equal(got.view(np.uint8), vref.view(np.uint8))
    return At


# ------------------------------------------------------------------ transpose
@pytest.mark.parametrize("seed", [0, 1])
def test_transpose_random_ragged(seed):
    print(f"case transpose random seed {seed}", flush=True)
    A = S.random_small(3001, 0.004, seed=seed, empty_rows=(0, 7, 3000), long_rows=(5, 1234))
    _check_transpose(A)


@pytest.mark.parametrize("dtype", ["f64", "f32", "f16"])
def test_transpose_value_types(dtype):
    A = S.convdiff3d_upwind(21)  # n = 9261, several tiles
    _check_transpose(A, dtype={"f64": spx.F64, "f32": spx.F32, "f16": spx.F16}[dtype])


def test_transpose_heavy_columns_and_involution():
    """Zipf column degrees (a few columns hold a large share of the entries)
    and ncols > 2^16 (three radix passes); transposing twice is the identity."""
    A = S.zipf_matrix(100000, a=1.5, kmax=500, seed=3)
    At = _check_transpose(A)
    Att = spx.csr_transpose(At)
    np.testing.assert_array_equal(host(Att.rowptr), A.rowptr)
    np.testing.assert_array_equal(host(Att.colidx)[: A.nnz], A.col)
    np.testing.assert_array_equal(host(Att.vals)[: A.nnz].view(np.uint64), A.val.view(np.uint64))


def test_transpose_rectangular_small_and_empty():
    # 13 rows, 300 columns (two radix passes), and 300 rows x 1 column (no pass)
    rng = np.random.default_rng(5)
    for nrows, ncols in ((13, 300), (300, 1), (1, 1), (2, 70000)):
        d = rng.uniform(-1, 1, (nrows, ncols)) * (rng.random((nrows, ncols)) < (0.0005 if ncols > 1000 else 0.3))
        rows, cols = np.nonzero(d)
        rowptr = np.zeros(nrows + 1, np.int64)
        np.add.at(rowptr, rows + 1, 1)
        A = S.CSR(nrows, np.cumsum(rowptr).astype(np.int32), cols.astype(np.int32), d[rows, cols])
        _check_transpose(A, ncols=ncols)
    E = S.CSR(9, np.zeros(10, np.int32), np.zeros(0, np.int32), np.zeros(0))
    At = spx.csr_transpose(spx.csr_from_host(E))
    assert not host(At.rowptr).any()


def test_transpose_shape_errors():
    A = spx.csr_from_host(S.poisson2d(5))
    bad = spx.Matrix(spx.CSR, spx.F32, A.ncols, A.nrows, A.nnz, rowptr=A.rowptr.clone(), colidx=A.colidx.clone(),
                     vals=A.vals.float())
    ws = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    st = spx._lib.spx_csr_transpose(spx.ctypes.byref(A.desc()), spx.ctypes.byref(bad.desc()), spx._ptr(ws),
                                    ws.numel(), spx._stream(None))
    assert st == spx.ERR_ARG
    st = spx._lib.spx_csr_transpose(spx.ctypes.byref(A.desc()), spx.ctypes.byref(A.desc()), spx._ptr(ws), 16,
                                    spx._stream(None))
    assert st == spx.ERR_ARG


@pytest.mark.timeout(300)
def test_transpose_full_convdiff_128():
    print("case transpose convdiff 128^3", flush=True)
    A = S.convdiff3d_upwind(128)
    _check_transpose(A)


# ------------------------------------------------------------------ BiCG
@pytest.mark.parametrize("precond", [0, 1])
def test_bicg_convdiff_vs_oracle(precond):
    print(f"case bicg convdiff 16^3 precond {precond}", flush=True)
    A = S.convdiff3d_upwind(16, peclet=10.0)
    xs, b = _problem(A)
    xo, io = O.bicg(A, b, tol=1e-10, precond=precond)
    assert io["status"] == O.OK
    x, info = spx.bicg_solve(spx.csr_from_host(A), dev(b), tol=1e-10, precond=precond, check_every=8)
    x = host(x)
    assert info["status"] == spx.OK, info
    assert _true_relres(A, b, x) <= 1e-10
    assert abs(info["iters"] - io["iters"]) <= 0.1 * io["iters"] + 5, (info["iters"], io["iters"])
    assert info["spmv_count"] == 2 * info["iters"]
    assert np.linalg.norm(x - xo) <= 1e-6 * np.linalg.norm(xo)


def test_bicg_symmetric_matches_cg():
    """On a symmetric matrix BiCG with rt = r takes CG's steps."""
    A = S.spd_diag_dominant(30000, seed=6)
    xs, b = _problem(A, 6)
    Ad = spx.csr_from_host(A)
    xb, ib = spx.bicg_solve(Ad, dev(b), tol=1e-10, precond=1)
    xc, ic = spx.cg_solve(Ad, dev(b), tol=1e-10, precond=1)
    assert ib["status"] == ic["status"] == spx.OK
    assert abs(ib["iters"] - ic["iters"]) <= 1
    assert _true_relres(A, b, host(xb)) <= 1e-10


def test_bicg_x0_unaligned_and_reproducible():
    A = S.convdiff3d_upwind(12)
    xs, b = _problem(A, 2)
    Ad = spx.csr_from_host(A)
    x0 = S.uniform_vector(A.n, seed=8)
    x, info = spx.bicg_solve(Ad, dev(b), x=dev(x0), tol=1e-10, precond=1)
    assert info["status"] == spx.OK
    assert _true_relres(A, b, host(x)) <= 1e-10
    _, io = O.bicg(A, b, tol=1e-10, precond=1, x0=x0)
    assert abs(info["iters"] - io["iters"]) <= 0.1 * io["iters"] + 5
    big = torch.zeros(A.n + 1, dtype=torch.float64, device="cuda")
    xu = big[1:]
    assert xu.data_ptr() % 32 != 0
    xu, iu = spx.bicg_solve(Ad, dev(b), xu, tol=1e-10, precond=1)
    xa, ia = spx.bicg_solve(Ad, dev(b), tol=1e-10, precond=1)
    xa2, ia2 = spx.bicg_solve(Ad, dev(b), tol=1e-10, precond=1)
    assert iu["iters"] == ia["iters"] == ia2["iters"]
    np.testing.assert_array_equal(host(xa).view(np.uint64), host(xu).view(np.uint64))
    np.testing.assert_array_equal(host(xa).view(np.uint64), host(xa2).view(np.uint64))


def test_bicg_status_codes():
    # [[0,1],[1,0]], b = e0: pt.q = 0 on the first step
    A = S.from_dense(np.array([[0.0, 1.0], [1.0, 0.0]]))
    _, info = spx.bicg_solve(spx.csr_from_host(A), dev(np.array([1.0, 0.0])), tol=1e-10)
    assert info["status"] == spx.ERR_BREAKDOWN and info["iters"] == 0
    with pytest.raises(spx.SpxError, match="ZERO_DIAG"):
        spx.bicg_solve(spx.csr_from_host(A), dev(np.array([1.0, 0.0])), precond=1)
    P = S.convdiff3d_upwind(10)
    xs, b = _problem(P)
    _, info = spx.bicg_solve(spx.csr_from_host(P), dev(b), tol=1e-12, maxit=4)
    assert info["status"] == spx.ERR_NOT_CONVERGED and info["iters"] == 4
    bn = b.copy()
    bn[3] = np.nan
    _, info = spx.bicg_solve(spx.csr_from_host(P), dev(bn))
    assert info["status"] == spx.ERR_NONFINITE
    x, info = spx.bicg_solve(spx.csr_from_host(P), dev(np.zeros(P.n)))
    assert info["status"] == spx.OK and info["iters"] == 0 and not host(x).any()
    D = S.from_dense(np.diag(np.arange(1.0, 9.0)))
    x, info = spx.bicg_solve(spx.csr_from_host(D), dev(np.ones(8)), precond=1)
    assert info["status"] == spx.OK and info["iters"] == 1
    np.testing.assert_allclose(host(x), 1.0 / np.arange(1.0, 9.0), rtol=1e-15)
    with pytest.raises(spx.SpxError, match="ARG"):
        spx.bicg_solve(spx.convert(spx.csr_from_host(P), spx.ELL), dev(b))


@pytest.mark.timeout(600)
def test_bicg_full_convdiff_128():
    print("case bicg convdiff 128^3", flush=True)
    A = S.convdiff3d_upwind(128)
    xs, b = _problem(A)
    x, info = spx.bicg_solve(spx.csr_from_host(A), dev(b), tol=1e-10, precond=1, maxit=5000)
    assert info["status"] == spx.OK, info
    assert _true_relres(A, b, host(x)) <= 1e-10
    print("bicg convdiff 128^3:", info, flush=True)


# ------------------------------------------------------------------ pipelined CG
@pytest.mark.parametrize("precond", [0, 1])
@pytest.mark.parametrize("fmt", ["csr", "ell", "sellp", "coo"])
def test_pipecg_vs_oracle(fmt, precond):
    print(f"case pipecg aniso 20^3 {fmt} precond {precond}", flush=True)
    A = S.poisson3d_7pt(20, 1, 1, 0.05)
    xs, b = _problem(A)
    xo, io = O.pipecg(A, b, tol=1e-10, precond=precond)
    assert io["status"] == O.OK
    Ad = spx.csr_from_host(A)
    if fmt != "csr":
        Ad = spx.convert(Ad, {"ell": spx.ELL, "sellp": spx.SELLP, "coo": spx.COO}[fmt])
    x, info = spx.pipecg_solve(Ad, dev(b), tol=1e-10, precond=precond, check_every=8)
    x = host(x)
    assert info["status"] == spx.OK, info
    assert _true_relres(A, b, x) <= 1e-10
    assert abs(info["iters"] - io["iters"]) <= 0.1 * io["iters"] + 5, (info["iters"], io["iters"])
    _, ic = spx.cg_solve(spx.csr_from_host(A), dev(b), tol=1e-10, precond=precond)
    assert abs(info["iters"] - ic["iters"]) <= 0.1 * ic["iters"] + 5


def test_pipecg_x0_unaligned_and_reproducible():
    A = S.spd_diag_dominant(20000, seed=4)
    xs, b = _problem(A, 4)
    Ad = spx.csr_from_host(A)
    x0 = S.uniform_vector(A.n, seed=5)
    x, info = spx.pipecg_solve(Ad, dev(b), x=dev(x0), tol=1e-10, precond=1)
    assert info["status"] == spx.OK
    assert _true_relres(A, b, host(x)) <= 1e-10
    _, io = O.pipecg(A, b, tol=1e-10, precond=1, x0=x0)
    assert abs(info["iters"] - io["iters"]) <= 0.1 * io["iters"] + 5
    big = torch.zeros(A.n + 1, dtype=torch.float64, device="cuda")
    xu = big[1:]
    xu, iu = spx.pipecg_solve(Ad, dev(b), xu, tol=1e-10, precond=1)
    xa, ia = spx.pipecg_solve(Ad, dev(b), tol=1e-10, precond=1)
    xa2, _ = spx.pipecg_solve(Ad, dev(b), tol=1e-10, precond=1)
    assert iu["iters"] == ia["iters"]
    np.testing.assert_array_equal(host(xa).view(np.uint64), host(xu).view(np.uint64))
    np.testing.assert_array_equal(host(xa).view(np.uint64), host(xa2).view(np.uint64))


def test_pipecg_status_codes():
    ind = S.from_dense(np.diag([1.0, -1.0] * 3))
    _, info = spx.pipecg_solve(spx.csr_from_host(ind), dev(np.ones(6)), tol=1e-12)
    assert info["status"] == spx.ERR_BREAKDOWN
    P = S.poisson2d(16)
    xs, b = _problem(P)
    _, info = spx.pipecg_solve(spx.csr_from_host(P), dev(b), tol=1e-12, maxit=3)
    assert info["status"] == spx.ERR_NOT_CONVERGED and info["iters"] == 3
    bn = b.copy()
    bn[0] = np.inf
    _, info = spx.pipecg_solve(spx.csr_from_host(P), dev(bn))
    assert info["status"] == spx.ERR_NONFINITE
    x, info = spx.pipecg_solve(spx.csr_from_host(P), dev(np.zeros(P.n)))
    assert info["status"] == spx.OK and info["iters"] == 0 and not host(x).any()
    Z = S.from_dense(np.diag([1.0, 0.0, 2.0]), keep_zeros=True)
    with pytest.raises(spx.SpxError, match="ZERO_DIAG"):
        spx.pipecg_solve(spx.csr_from_host(Z), dev(np.ones(3)), precond=1)
    one = S.from_dense(np.array([[4.0]]))
    x, info = spx.pipecg_solve(spx.csr_from_host(one), dev(np.array([2.0])))
    assert info["status"] == spx.OK and info["iters"] == 1 and host(x)[0] == 0.5


@pytest.mark.timeout(600)
def test_pipecg_full_aniso_128():
    print("case pipecg aniso 128^3", flush=True)
    A = S.poisson3d_7pt(128, 1, 1, 0.01)
    xs, b = _problem(A)
    x, info = spx.pipecg_solve(spx.csr_from_host(A), dev(b), tol=1e-10, precond=1, maxit=5000)
    assert info["status"] == spx.OK, info
    assert _true_relres(A, b, host(x)) <= 1e-10
    print("pipecg aniso 128^3:", info, flush=True)


# ------------------------------------------------------------------ restarts
@pytest.mark.parametrize("solver", ["cg_small", "cg_general", "pipecg", "bicg"])
def test_unreachable_tolerance_restarts_and_stops(solver):
    """With tol = 1e-17 the recursive residual of CG eventually passes while
    the true residual cannot: the solver confirms, restarts from the true
    residual, and stops at maxit with an accurate iterate. Every solver stops
    within maxit."""
    print(f"case restarts {solver}", flush=True)
    A = S.poisson2d(30) if solver != "bicg" else S.convdiff3d_upwind(10)
    xs, b = _problem(A, 3)
    Ad = spx.csr_from_host(A)
    if solver == "cg_general":
        Ad = spx.convert(Ad, spx.ELL)  # the multi-launch driver
    fn = {"cg_small": spx.cg_solve, "cg_general": spx.cg_solve, "pipecg": spx.pipecg_solve,
          "bicg": spx.bicg_solve}[solver]
    x, info = fn(Ad, dev(b), tol=1e-17, maxit=600, precond=1)
    assert info["status"] in (spx.OK, spx.ERR_NOT_CONVERGED, spx.ERR_BREAKDOWN), info
    assert info["iters"] <= 600
    if solver in ("cg_small", "cg_general"):
        # CG restarts until maxit and keeps an iterate at the attainable accuracy
        assert info["status"] == spx.ERR_NOT_CONVERGED and info["iters"] == 600, info
        assert _true_relres(A, b, host(x)) <= 1e-13
    else:
        # pipelined CG and BiCG end at rounding level with a breakdown (their
        # step denominators lose their sign; the oracle's pipelined CG does the
        # same on this system), keeping an iterate within the usual tolerance
        assert _true_relres(A, b, host(x)) <= 1e-10


def test_batch_unreachable_tolerance_stops():
    A = S.poisson2d(30)
    xs, b = _problem(A, 4)
    Ad = spx.csr_from_host(A)
    xb, ib = spx.cg_batch([Ad], [dev(b)], tol=1e-17, maxit=500)
    assert ib[0]["status"] in (spx.OK, spx.ERR_NOT_CONVERGED), ib
    assert ib[0]["iters"] <= 500
    assert _true_relres(A, b, host(xb[0])) <= 1e-13
