"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke run.

This module builds matrices and vectors only. It holds none of the arithmetic
of the method itself (no products, no reductions, no solver steps), so both the
GPU path and the CPU oracle can be fed from it without sharing any code.

The paper evaluates on more than 2,800 SuiteSparse matrices (Section 4), which
are not available here; the generators below produce matrices with the shapes,
sizes and row-length distributions of the workloads this library is measured
on instead:

* 2D 5-point and 3D 7/27-point stencils on lexicographically ordered grids
  (index ``i + Nx*(j + Ny*k)``, x fastest), homogeneous Dirichlet boundary
  eliminated, unit spacing;
* a random matrix whose row lengths follow Zipf(a) clipped to ``[1, kmax]``
  with distinct, uniformly random, ascending column indices;
* random symmetric diagonally dominant SPD matrices;
* i.i.d. uniform[-1, 1) vectors.

Every draw comes from numpy's PCG64 ``default_rng`` seeded through a
``SeedSequence`` spawned into one independent stream per purpose, so that,
for example, changing the values never changes the pattern.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass

import numpy as np

# One independent random stream per purpose, spawned from the user seed.
_STREAMS = ("pattern", "values", "x", "xstar", "arrivals", "sizes", "rhs")


def rng(seed: int, purpose: str) -> np.random.Generator:
    """Independent PCG64 generator for ``purpose`` derived from ``seed``."""
    idx = _STREAMS.index(purpose)
    child = np.random.SeedSequence(int(seed)).spawn(len(_STREAMS))[idx]
    return np.random.default_rng(child)


@dataclass
class CSR:
    """Host CSR matrix in canonical form (rows ascending, columns strictly
    ascending inside a row, explicit zeros kept). Indices are int32."""

    n: int
    rowptr: np.ndarray  # int32 [n+1]
    col: np.ndarray  # int32 [nnz]
    val: np.ndarray  # float64 [nnz]

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def row_lengths(self) -> np.ndarray:
        return np.diff(self.rowptr.astype(np.int64))


def _finish(n: int, rowptr64: np.ndarray, col64: np.ndarray, val: np.ndarray) -> CSR:
    if rowptr64[-1] > np.iinfo(np.int32).max:
        raise ValueError("nnz exceeds int32 range")
    return CSR(
        n=int(n),
        rowptr=np.ascontiguousarray(rowptr64, dtype=np.int32),
        col=np.ascontiguousarray(col64, dtype=np.int32),
        val=np.ascontiguousarray(val, dtype=np.float64),
    )


def stencil(shape, offsets, coeffs=None, seed: int = 0) -> CSR:
    """Matrix of a constant-pattern stencil on a lexicographic grid.

    ``shape`` is ``(Nx,)``, ``(Nx, Ny)`` or ``(Nx, Ny, Nz)``; ``offsets`` is a
    list of integer offset tuples of the same rank. Neighbours that fall outside
    the grid are dropped (eliminated Dirichlet boundary). ``coeffs`` gives one
    value per offset; ``None`` draws every stored value i.i.d. uniform[-1, 1)
    from the ``values`` stream, in row-major storage order.
    """
    shape = tuple(int(s) for s in shape)
    d = len(shape)
    offsets = [tuple(int(v) for v in o) for o in offsets]
    strides = [int(np.prod(shape[:a])) for a in range(d)]
    lin = [sum(o[a] * strides[a] for a in range(d)) for o in offsets]
    order = np.argsort(lin, kind="stable")  # ascending linear offset = ascending column
    offsets = [offsets[i] for i in order]
    lin = [lin[i] for i in order]
    if coeffs is not None:
        coeffs = [float(coeffs[i]) for i in order]
    n = int(np.prod(shape))
    grids = np.meshgrid(*[np.arange(s, dtype=np.int64) for s in shape], indexing="ij")
    # meshgrid 'ij' puts axis 0 first; flatten so that x (axis 0) runs fastest.
    coords = [g.transpose(tuple(range(d - 1, -1, -1))).reshape(-1) for g in grids]
    valid = np.ones((n, len(offsets)), dtype=bool)
    for k, o in enumerate(offsets):
        for a in range(d):
            if o[a] != 0:
                c = coords[a] + o[a]
                valid[:, k] &= (c >= 0) & (c < shape[a])
    rows = np.arange(n, dtype=np.int64)
    colmat = rows[:, None] + np.asarray(lin, dtype=np.int64)[None, :]
    lens = valid.sum(axis=1)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(lens, out=rowptr[1:])
    col = colmat[valid]
    del colmat
    if coeffs is None:
        val = rng(seed, "values").uniform(-1.0, 1.0, col.size)
    else:
        val = np.broadcast_to(np.asarray(coeffs, dtype=np.float64)[None, :], valid.shape)[valid]
    return _finish(n, rowptr, col, val)


def offsets_5pt():
    return [(0, -1), (-1, 0), (0, 0), (1, 0), (0, 1)]


def offsets_7pt():
    return [(0, 0, -1), (0, -1, 0), (-1, 0, 0), (0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)]


def offsets_27pt():
    return [t for t in itertools.product((-1, 0, 1), repeat=3)]


def poisson2d(N: int) -> CSR:
    """2D 5-point Poisson, diagonal 4, neighbours -1, on an N x N grid."""
    off = offsets_5pt()
    coeffs = [4.0 if o == (0, 0) else -1.0 for o in off]
    return stencil((N, N), off, coeffs)


def poisson3d_7pt(N: int, cx: float = 1.0, cy: float = 1.0, cz: float = 1.0) -> CSR:
    """3D 7-point (possibly anisotropic) Poisson on an N^3 grid.

    Off-diagonals are ``-c`` along each axis and the diagonal is
    ``2*(cx + cy + cz)`` evaluated in float64 (4.02 for 1/1/0.01)."""
    off = offsets_7pt()
    diag = 2.0 * (cx + cy + cz)
    axis_c = (cx, cy, cz)
    coeffs = []
    for o in off:
        if o == (0, 0, 0):
            coeffs.append(diag)
        else:
            a = [i for i in range(3) if o[i] != 0][0]
            coeffs.append(-axis_c[a])
    return stencil((N, N, N), off, coeffs)


def convdiff3d_upwind(N: int, peclet: float = 10.0) -> CSR:
    """Nonsymmetric 3D 7-point convection-diffusion, first-order upwind.

    Unit diffusion with equal wind along +x, +y, +z and per-axis cell Peclet
    number ``peclet``, scaled by h^2/nu: diagonal ``6 + 3*peclet``, the upwind
    neighbour (offset -1 on an axis) ``-(1 + peclet)``, the downwind neighbour
    ``-1``. This is an M-matrix (36, -11, -1 at Peclet 10)."""
    off = offsets_7pt()
    coeffs = []
    for o in off:
        if o == (0, 0, 0):
            coeffs.append(6.0 + 3.0 * peclet)
        elif sum(o) < 0:
            coeffs.append(-(1.0 + peclet))
        else:
            coeffs.append(-1.0)
    return stencil((N, N, N), off, coeffs)


def stencil27_random(N: int, seed: int = 0) -> CSR:
    """3D 27-point pattern on an N^3 grid with i.i.d. uniform[-1, 1) values."""
    return stencil((N, N, N), offsets_27pt(), None, seed=seed)


def zipf_matrix(n: int, a: float = 1.5, kmax: int = 10000, seed: int = 0) -> CSR:
    """Random n x n matrix with Zipf(a) row lengths clipped to [1, kmax].

    Lengths are ``min(zipf(a), kmax)`` (numpy's Zipf draws are >= 1). Columns
    in a row are distinct and uniform over ``[0, n)``: draws with replacement
    are deduplicated and topped up until the row is full, then sorted. Values
    are i.i.d. uniform[-1, 1)."""
    kmax = min(int(kmax), int(n))
    rp = rng(seed, "pattern")
    lens = np.minimum(rp.zipf(a, n), kmax).astype(np.int64)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(lens, out=rowptr[1:])
    nnz = int(rowptr[-1])
    key = np.repeat(np.arange(n, dtype=np.int64) * n, lens)
    key += rp.integers(0, n, nnz, dtype=np.int64)
    key.sort()
    dup = np.flatnonzero(key[1:] == key[:-1]) + 1
    if dup.size:
        for r in np.unique(key[dup] // n):
            s, e = int(rowptr[r]), int(rowptr[r + 1])
            c = np.unique(key[s:e] - r * n)
            while c.size < e - s:
                c = np.unique(np.concatenate([c, rp.integers(0, n, (e - s) - c.size, dtype=np.int64)]))
            key[s:e] = r * n + c
    col = key % n
    del key
    val = rng(seed, "values").uniform(-1.0, 1.0, nnz)
    return _finish(n, rowptr, col, val)


def spd_diag_dominant(n: int, kmin: int = 5, kmax: int = 30, seed: int = 0, device=None) -> CSR:
    """Random symmetric, strictly diagonally dominant SPD matrix.

    Each row i draws a target length k ~ U{kmin..kmax} and (k-1)//2 partner
    columns j != i uniformly; each pair (i, j) gets one uniform[-1, 1) value
    placed at (i, j) and mirrored to (j, i) (a pair drawn twice keeps its first
    value). The diagonal is ``sum_j |a_ij| + 1``, summed left to right along
    the row. With `device` (a torch device such as "cuda") the random draws
    are the same and the sorting and assembly run in torch there: the same
    matrix, bit for bit, much faster for large n."""
    rp = rng(seed, "pattern")
    rv = rng(seed, "values")
    k = rp.integers(kmin, kmax + 1, n)
    m = (k - 1) // 2
    src = np.repeat(np.arange(n, dtype=np.int64), m)
    dst = rp.integers(0, n - 1, src.size, dtype=np.int64)
    v = rv.uniform(-1.0, 1.0, src.size)
    if device is not None:
        return _spd_assemble_torch(n, src, dst, v, device)
    dst += dst >= src  # uniform over [0, n) without i
    lo = np.minimum(src, dst)
    hi = np.maximum(src, dst)
    # pairs in (lo, hi) order, the first draw of each kept
    o = np.argsort(lo * n + hi, kind="stable")
    key = (lo * n + hi)[o]
    keep = np.ones(key.size, bool)
    keep[1:] = key[1:] != key[:-1]
    o = o[keep]
    ulo, uhi, uv = lo[o], hi[o], v[o]  # upper entries (row lo, col hi), sorted by (row, col)
    o2 = np.argsort(uhi * n + ulo, kind="stable")
    llo, lhi, lv = ulo[o2], uhi[o2], uv[o2]  # lower entries (row hi, col lo), sorted by (row, col)
    cnt_lo = np.bincount(lhi, minlength=n)  # entries left of the diagonal per row
    cnt_up = np.bincount(ulo, minlength=n)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(cnt_lo + 1 + cnt_up, out=rowptr[1:])
    nnz = int(rowptr[-1])
    col = np.empty(nnz, np.int64)
    val = np.zeros(nnz)
    # a row holds its lower entries, the diagonal, then its upper entries
    lstart = np.zeros(n, np.int64)
    np.cumsum(cnt_lo[:-1], out=lstart[1:])
    ustart = np.zeros(n, np.int64)
    np.cumsum(cnt_up[:-1], out=ustart[1:])
    pl = rowptr[lhi] + (np.arange(lhi.size) - lstart[lhi])
    pu = rowptr[ulo] + cnt_lo[ulo] + 1 + (np.arange(ulo.size) - ustart[ulo])
    pd = rowptr[:-1] + cnt_lo
    col[pl], val[pl] = llo, lv
    col[pu], val[pu] = uhi, uv
    col[pd] = np.arange(n)
    rows = np.repeat(np.arange(n), np.diff(rowptr))
    val[pd] = np.bincount(rows, weights=np.abs(val), minlength=n) + 1.0
    return _finish(n, rowptr, col, val)


def _spd_assemble_torch(n, src, dst, v, device) -> CSR:
    """The assembly steps of spd_diag_dominant in torch on `device`."""
    import torch

    dev = torch.device(device)
    src = torch.from_numpy(src).to(dev)
    dst = torch.from_numpy(dst).to(dev)
    v = torch.from_numpy(v).to(dev)
    dst = dst + (dst >= src).to(dst.dtype)
    lo = torch.minimum(src, dst)
    hi = torch.maximum(src, dst)
    key, o = torch.sort(lo * n + hi, stable=True)
    keep = torch.ones_like(key, dtype=torch.bool)
    keep[1:] = key[1:] != key[:-1]
    o = o[keep]
    ulo, uhi, uv = lo[o], hi[o], v[o]
    _, o2 = torch.sort(uhi * n + ulo, stable=True)
    llo, lhi, lv = ulo[o2], uhi[o2], uv[o2]
    cnt_lo = torch.bincount(lhi, minlength=n)
    cnt_up = torch.bincount(ulo, minlength=n)
    lens = cnt_lo + 1 + cnt_up
    rowptr = torch.zeros(n + 1, dtype=torch.int64, device=dev)
    rowptr[1:] = torch.cumsum(lens, 0)
    nnz = int(rowptr[-1])
    col = torch.empty(nnz, dtype=torch.int64, device=dev)
    val = torch.zeros(nnz, dtype=torch.float64, device=dev)
    lstart = torch.cumsum(cnt_lo, 0) - cnt_lo
    ustart = torch.cumsum(cnt_up, 0) - cnt_up
    pl = rowptr[lhi] + (torch.arange(lhi.numel(), device=dev) - lstart[lhi])
    pu = rowptr[ulo] + cnt_lo[ulo] + 1 + (torch.arange(ulo.numel(), device=dev) - ustart[ulo])
    pd = rowptr[:-1] + cnt_lo
    col[pl], val[pl] = llo, lv
    col[pu], val[pu] = uhi, uv
    col[pd] = torch.arange(n, device=dev)
    # row sums of |a_ij| left to right (as the host path's bincount adds them)
    a = val.abs()
    acc = torch.zeros(n, dtype=torch.float64, device=dev)
    start = rowptr[:-1]
    for j in range(int(lens.max())):
        idx = start + j
        live = j < lens
        acc += torch.where(live, a[torch.where(live, idx, 0)], torch.zeros((), dtype=a.dtype, device=dev))
    val[pd] = acc + 1.0
    return _finish(n, rowptr.cpu().numpy(), col.cpu().numpy(), val.cpu().numpy())


def uniform_vector(n: int, seed: int = 0, purpose: str = "x") -> np.ndarray:
    """i.i.d. uniform[-1, 1) float64 vector from the ``purpose`` stream."""
    return rng(seed, purpose).uniform(-1.0, 1.0, int(n))


def random_small(n: int, density: float, seed: int = 0, empty_rows=(), long_rows=()) -> CSR:
    """Small random test matrix with chosen empty and dense rows.

    ``empty_rows`` get no entries, ``long_rows`` get every column; the other
    rows keep each column with probability ``density``."""
    rp = rng(seed, "pattern")
    mask = rp.random((n, n)) < density
    for r in empty_rows:
        mask[r, :] = False
    for r in long_rows:
        mask[r, :] = True
    rows, cols = np.nonzero(mask)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(mask.sum(axis=1), out=rowptr[1:])
    val = rng(seed, "values").uniform(-1.0, 1.0, rows.size)
    return _finish(n, rowptr, cols, val)


def from_dense(a: np.ndarray, keep_zeros=False) -> CSR:
    """CSR of a small dense array (stores nonzeros, or every entry)."""
    a = np.asarray(a, dtype=np.float64)
    mask = np.ones(a.shape, bool) if keep_zeros else (a != 0)
    rows, cols = np.nonzero(mask)
    rowptr = np.zeros(a.shape[0] + 1, dtype=np.int64)
    np.cumsum(mask.sum(axis=1), out=rowptr[1:])
    return _finish(a.shape[0], rowptr, cols, a[rows, cols])


def poisson_arrivals(count: int, rate: float, seed: int = 0) -> np.ndarray:
    """Arrival times (s) of a Poisson process of the given rate (1/s)."""
    gaps = rng(seed, "arrivals").exponential(1.0 / rate, int(count))
    return np.cumsum(gaps)
