"""Seeded synthetic inputs shared by the HIP path, the CPU oracle, the tests and the benchmark.

This module generates *data* only: coefficient fields, initial states, random
test blocks and request traces.  It holds none of the method's arithmetic (no
finite-volume fluxes, no time coupling, no solver), so both sides can consume
the same bytes without sharing any computation.

Array conventions: a grid field with ``n = (nx, ny[, nz])`` cells is a numpy
array of shape ``(nz, ny, nx)`` (or ``(ny, nx)`` in 2D) in C order, so that its
flattened index is ``ix + nx*iy + nx*ny*iz``.  Cell centres of the unit
square/cube sit at ``(i + 1/2) / n``.
"""
from __future__ import annotations

import numpy as np
from scipy import ndimage


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def field_shape(n) -> tuple:
    """numpy shape (slowest axis first) of a field on a grid with per-axis cell counts ``n``."""
    n = tuple(int(v) for v in n)
    return tuple(reversed(n))


def cell_centres(n):
    """Per-axis cell-centre coordinates on the unit square/cube (list, x first)."""
    return [(np.arange(int(m), dtype=np.float64) + 0.5) / int(m) for m in n]


def gaussian_field(n, corr_len_cells: float, seed: int) -> np.ndarray:
    """Stationary Gaussian random field with zero mean and unit sample variance.

    White noise N(0,1) drawn from PCG64(seed) is smoothed along every axis by a
    normalised Gaussian kernel of standard deviation ``corr_len_cells`` cells
    (reflective boundary), then centred and scaled to unit sample variance.
    """
    shape = field_shape(n)
    g = _rng(seed).standard_normal(shape)
    if corr_len_cells > 0:
        radius = int(np.ceil(3.0 * corr_len_cells))
        x = np.arange(-radius, radius + 1, dtype=np.float64)
        w = np.exp(-0.5 * (x / corr_len_cells) ** 2)
        w /= w.sum()
        for ax in range(g.ndim):
            g = ndimage.convolve1d(g, w, axis=ax, mode="reflect")
    g -= g.mean()
    g /= g.std()
    return g


def lognormal_field(n, log_mean: float, log_std: float, corr_len_cells: float, seed: int) -> np.ndarray:
    """Cell-wise coefficient ``exp(log_mean + log_std * g)`` with ``g`` from :func:`gaussian_field`.

    Returned flattened (length N, float64) in the grid's linear cell order.
    """
    g = gaussian_field(n, corr_len_cells, seed)
    return np.exp(log_mean + log_std * g).ravel()


def sin_product(n) -> np.ndarray:
    """``prod_d sin(pi x_d)`` at the cell centres, flattened (float64)."""
    cs = cell_centres(n)
    vals = [np.sin(np.pi * c) for c in cs]
    out = vals[0]
    for v in vals[1:]:
        out = np.multiply.outer(v, out)
    return np.ascontiguousarray(out).ravel()


def smooth_random(n, seed: int, max_mode: int = 4) -> np.ndarray:
    """Seeded smooth field in [0, 1]: a random cosine series, min-max scaled.

    Modes ``(k_x, k_y[, k_z])`` with every ``k_d <= max_mode`` get N(0,1)
    amplitudes damped by ``1 / (1 + |k|^2)``; the sum is evaluated at the cell
    centres and mapped affinely onto [0, 1].
    """
    rng = _rng(seed)
    cs = cell_centres(n)
    dim = len(cs)
    ks = np.stack(np.meshgrid(*[np.arange(max_mode + 1)] * dim, indexing="ij"), -1).reshape(-1, dim)
    amp = rng.standard_normal(len(ks)) / (1.0 + (ks ** 2).sum(1))
    field = np.zeros(field_shape(n))
    for a, kv in zip(amp, ks):
        term = np.cos(np.pi * kv[0] * cs[0])
        for d in range(1, dim):
            term = np.multiply.outer(np.cos(np.pi * kv[d] * cs[d]), term)
        field += a * term
    lo, hi = field.min(), field.max()
    return ((field - lo) / (hi - lo)).ravel()


def random_block(N: int, k: int, seed: int, dtype=np.float64) -> np.ndarray:
    """Row-major N x k block with N(0,1) entries."""
    return _rng(seed).standard_normal((N, k)).astype(dtype)


def random_csr(N: int, seed: int, min_row: int = 0, max_row: int = 9, diag: bool = True):
    """Random square CSR pattern and values (rowptr int32, col int32, val float64).

    Row lengths are uniform in [min_row, max_row]; column indices are distinct
    and sorted within a row; with ``diag`` every row contains its diagonal.
    """
    rng = _rng(seed)
    rowptr = np.zeros(N + 1, dtype=np.int64)
    cols = []
    for r in range(N):
        m = int(rng.integers(min_row, max_row + 1))
        m = min(m, N)
        c = rng.choice(N, size=m, replace=False) if m else np.zeros(0, dtype=np.int64)
        if diag and r not in c:
            c = np.append(c, r) if m < N else c
        c = np.sort(c)
        cols.append(c)
        rowptr[r + 1] = rowptr[r] + len(c)
    col = np.concatenate(cols).astype(np.int32) if cols else np.zeros(0, np.int32)
    val = rng.standard_normal(len(col))
    return rowptr.astype(np.int32), col, val


def poisson_trace(n_requests: int, rate_per_s: float, seed: int, sizes, widths):
    """Arrival times (s, cumulative exponential gaps), grid sizes and block widths of a request trace."""
    rng = _rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, size=n_requests)
    t = np.cumsum(gaps)
    n = rng.choice(np.asarray(sizes), size=n_requests)
    k = rng.choice(np.asarray(widths), size=n_requests)
    return t, n, k
