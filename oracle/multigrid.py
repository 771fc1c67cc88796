"""Geometric multigrid V-cycle for ``A = a M + b K`` on a structured grid (oracle side; test
infrastructure only).

The paper preconditions its inner Krylov solves with AMG (Sec. 4.1) and gives no details; the library
uses a geometric V-cycle in its place.  This module writes that V-cycle out from its definition with
scipy sparse matrices, so that one application can be compared entry by entry:

* level 0 is the fine grid with ``M_0 = I`` and ``K_0 = K``; level ``l+1`` aggregates 2 x 2 x 2 cells
  of level ``l`` (one cell along an axis of odd length at its end); with the piecewise-constant
  prolongation ``P_l`` (``P[i, I] = 1`` when fine cell i lies in aggregate I) the coarse operators are
  the Galerkin products ``K_{l+1} = P^T K_l P`` and ``M_{l+1} = P^T M_l P``;
* coarsening stops once a level has at most 64 cells (or after 16 levels);
* cells are coloured red (even coordinate sum on their level's grid) and black; the 7-point stencil,
  which the Galerkin products keep, couples only cells of opposite colours;
* ``V(l, f)``: on the coarsest level, 12 damped Jacobi sweeps from zero with ``w_c = 0.8``;
  otherwise, from ``x = 0``, one Gauss-Seidel half-sweep over the red cells and one over the black
  cells, ``x_c = V(l+1, P^T (f - A x))``, ``z = x + s P x_c``, then the half-sweeps in the adjoint
  order (black, then red).  A half-sweep solves each row of its colour with the other colour
  fixed; as no two cells of one colour are coupled, it equals a Gauss-Seidel pass over that colour
  in any order.  The cycle is symmetric because the post-smoother is the adjoint of the
  pre-smoother.
* the coarse correction is scaled by ``s = 1.4``: the Galerkin operator of a piecewise-constant
  aggregation is stiffer than the fine operator on smooth modes (a 2x2x2 aggregate couples to a
  face neighbour through four fine faces: twice the coupling of a 2h re-discretisation in 3-D), so
  the unscaled correction falls short.

Parity unpinned by the paper (it prints no multigrid); the CPU tests pin this module by the algebraic
facts it must satisfy (Galerkin row sums, the uniform-coefficient coarse stencil, agreement of the
smoothing with a cell-by-cell Gauss-Seidel loop, exactness when A is diagonal, symmetry and positive
definiteness of the cycle, contraction as a stationary solver).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

COARSE_SCALE = 1.4   # scale of the prolonged coarse correction
COARSE_OMEGA = 0.8   # damping of the coarsest level's sweeps
COARSEST_MAX = 64
COARSE_SWEEPS = 12
MAX_LEVELS = 16


def _dims(n):
    n = tuple(int(v) for v in n)
    return n + (1,) * (3 - len(n))


def prolongation(n):
    """Piecewise-constant prolongation from the aggregates of grid ``n`` (cells ix + nx*iy + nx*ny*iz)
    to grid ``n``; returns (P, coarse dims)."""
    nx, ny, nz = _dims(n)
    cx, cy, cz = (nx + 1) // 2, (ny + 1) // 2, (nz + 1) // 2
    iz, iy, ix = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    fine = (ix + nx * iy + nx * ny * iz).ravel()
    coarse = ((ix // 2) + cx * (iy // 2) + cx * cy * (iz // 2)).ravel()
    N, Nc = nx * ny * nz, cx * cy * cz
    P = sp.csr_matrix((np.ones(N), (fine, coarse)), shape=(N, Nc))
    return P, (cx, cy, cz)


def red_cells(dims):
    """Mask of the red cells (even ix + iy + iz) of grid ``dims`` (cells ix + nx*iy + nx*ny*iz)."""
    nx, ny, nz = dims
    iz, iy, ix = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return ((ix + iy + iz) % 2 == 0).ravel()


def half_sweep(A, f, x, cells):
    """Gauss-Seidel over the masked cells: each solves its own row with every other cell fixed."""
    x = np.array(x, dtype=np.float64, copy=True)
    r = f - A @ x
    x[cells] += r[cells] / A.diagonal()[cells, None]
    return x


def hierarchy(K, n):
    """Galerkin hierarchy: list of (K_l, m_l diagonal mass, P_l or None, dims)."""
    levels = []
    Kl = sp.csr_matrix(K, dtype=np.float64)
    ml = np.ones(Kl.shape[0])
    dims = _dims(n)
    while True:
        N = Kl.shape[0]
        if N <= COARSEST_MAX or len(levels) + 1 >= MAX_LEVELS:
            levels.append((Kl, ml, None, dims))
            return levels
        P, cdims = prolongation(dims)
        levels.append((Kl, ml, P, dims))
        Kl = (P.T @ Kl @ P).tocsr()
        ml = P.T @ ml
        dims = cdims


def vcycle(levels, a, b, f, lvl=0):
    """One V-cycle z = V(f) on level ``lvl`` for the columns of ``f`` (N x k)."""
    K, m, P, dims = levels[lvl]
    A = (sp.diags(a * m) + b * K).tocsr()
    f = np.asarray(f, dtype=np.float64)
    if P is None:
        dinv = 1.0 / A.diagonal()
        x = COARSE_OMEGA * dinv[:, None] * f
        for _ in range(COARSE_SWEEPS - 1):
            x = x + COARSE_OMEGA * dinv[:, None] * (f - A @ x)
        return x
    red = red_cells(dims)
    x = half_sweep(A, f, np.zeros_like(f), red)
    x = half_sweep(A, f, x, ~red)
    xc = vcycle(levels, a, b, P.T @ (f - A @ x), lvl + 1)
    z = x + COARSE_SCALE * (P @ xc)
    z = half_sweep(A, f, z, ~red)
    return half_sweep(A, f, z, red)
