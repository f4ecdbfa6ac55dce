"""spx_cg_batch_noalloc (the batched CG that takes its workspace from the
library's fixed device scratch instead of a caller's buffer) against
spx_cg_batch: two calls in a row, the second on fewer and smaller systems,
each result bitwise the workspace entry point's, and every solution checked
through the oracle's true residual. Also: a batch too large for the scratch
is refused before anything runs."""
import numpy as np
import pytest

import oracle as O
from paper_2006_14290_amd import synth as S

from gpu_util import dev, host

pytestmark = pytest.mark.gpu

spx = pytest.importorskip("paper_2006_14290_amd.spx")


def _system(kind, size, seed):
    A = S.poisson2d(size) if kind == "poisson" else S.spd_diag_dominant(size, seed=seed)
    xs = S.uniform_vector(A.n, seed=seed, purpose="xstar")
    b, _ = O.csr_spmv_dot2(A, xs)
    return A, b


# the first call: one-group systems (small-system kernel and general kernel)
# and wide systems; the second call: fewer, smaller systems
FIRST = [("poisson", 32, 1), ("spd", 1000, 2), ("poisson", 70, 3), ("spd", 6000, 4), ("poisson", 150, 5),
         ("spd", 30000, 6), ("poisson", 45, 7)]
SECOND = [("spd", 1200, 8), ("poisson", 40, 9), ("poisson", 130, 10)]


def _relres(A, b, x):
    _, rn = O.residual(A, b, x)
    return rn / np.linalg.norm(b)


def _check_call(cases, tol):
    print(f"case noalloc batch of {len(cases)} systems, tol {tol}", flush=True)
    systems = [_system(*c) for c in cases]
    mats = [spx.csr_from_host(A) for A, _ in systems]
    bs = [dev(b) for _, b in systems]
    xw, iw = spx.cg_batch(mats, bs, tol=tol)
    xn, inn = spx.cg_batch(mats, bs, tol=tol, noalloc=True)
    for (A, b), a, ia, z, iz in zip(systems, xw, iw, xn, inn):
        assert ia["status"] == spx.OK and iz["status"] == spx.OK, (ia, iz)
        assert ia == iz
        a, z = host(a), host(z)
        np.testing.assert_array_equal(a.view(np.uint64), z.view(np.uint64))
        assert _relres(A, b, z) <= tol


def test_noalloc_batch_matches_workspace_batch_twice():
    _check_call(FIRST, 1e-8)
    _check_call(SECOND, 1e-9)


def test_noalloc_batch_refuses_oversize():
    n = 3_000_000  # 3 vectors of n float64 = 72 MB > 64 MiB of scratch
    rowptr = np.arange(n + 1, dtype=np.int32)
    col = np.arange(n, dtype=np.int32)
    A = S.CSR(n, rowptr, col, np.full(n, 2.0))
    Ad = spx.csr_from_host(A)
    with pytest.raises(spx.SpxError, match="ERR_ARG"):
        spx.cg_batch([Ad], [dev(np.ones(n))], tol=1e-8, noalloc=True)
    # the workspace entry point still solves it
    x, info = spx.cg_batch([Ad], [dev(np.ones(n))], tol=1e-8)
    assert info[0]["status"] == spx.OK
    assert np.allclose(host(x[0]), 0.5)
