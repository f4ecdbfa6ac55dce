"""Helpers shared by the GPU parity tests."""
import numpy as np
import torch

U64 = 2.0 ** -53
U32 = 2.0 ** -24


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def gamma(k, u):
    k = np.asarray(k, dtype=np.float64)
    return k * u / (1.0 - k * u)


def assert_spmv_f64(y, yref, absax, beta_y=None, tol=1e-14):
    """Per-row parity bar for float64 products: |y - y_ref| <= tol*(|A||x|)_i
    (+ tol*|beta*y_i|); a row with (|A||x|)_i == 0 must be exactly zero."""
    bound = tol * absax
    if beta_y is not None:
        bound = bound + tol * np.abs(beta_y)
    err = np.abs(y - yref)
    bad = np.flatnonzero(~(err <= bound))
    assert bad.size == 0, (f"{bad.size} rows out of tolerance; first {bad[:5]}: y={y[bad[:5]]} "
                           f"ref={yref[bad[:5]]} bound={bound[bad[:5]]}")
    zero = (absax == 0) if beta_y is None else (absax == 0) & (beta_y == 0)
    assert np.all(y[zero] == 0.0)


def assert_spmv_low(y, yref, absax, rowlen, beta_y=None):
    """float32 / binary16-value products: first-order bound gamma_{k+2}(2^-24)
    times (|A||x|)_i (+ |beta*y_i|) with k the row length (Higham, Ch. 3)."""
    g = gamma(rowlen + 2, U32)
    bound = g * absax
    if beta_y is not None:
        bound = bound + g * np.abs(beta_y) + U32 * np.abs(beta_y)
    err = np.abs(y.astype(np.float64) - yref)
    bad = np.flatnonzero(~(err <= bound))
    assert bad.size == 0, (f"{bad.size} rows out of tolerance; first {bad[:5]}: y={y[bad[:5]]} "
                           f"ref={yref[bad[:5]]} bound={bound[bad[:5]]}")
