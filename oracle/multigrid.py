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
* ``V(l, f)``: on the coarsest level, 12 damped Jacobi sweeps from zero with ``w_c = 0.8``;
  otherwise ``x = w D^-1 f``, ``x_c = V(l+1, P^T (f - A x))``, ``z = x + s P x_c``,
  ``z += w D^-1 (f - A z)``, with ``D = diag(A_l)``, ``w = 0.9`` and the coarse correction scaled by
  ``s = 1.4``.  The scale compensates the Galerkin operator of a piecewise-constant aggregation,
  which is stiffer than the fine operator on smooth modes (a 2x2x2 aggregate couples to a face
  neighbour through four fine faces: twice the coupling of a 2h re-discretisation in 3-D), so the
  unscaled correction falls short.

Parity unpinned by the paper (it prints no multigrid); the CPU tests pin this module by the algebraic
facts it must satisfy (Galerkin row sums, the uniform-coefficient coarse stencil, symmetry and
positive definiteness of the cycle, contraction as a stationary solver).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

OMEGA = 0.9          # damping of the pre- and post-sweeps
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
    K, m, P, _ = levels[lvl]
    A = (sp.diags(a * m) + b * K).tocsr()
    dinv = 1.0 / A.diagonal()
    f = np.asarray(f, dtype=np.float64)
    if P is None:
        x = COARSE_OMEGA * dinv[:, None] * f
        for _ in range(COARSE_SWEEPS - 1):
            x = x + COARSE_OMEGA * dinv[:, None] * (f - A @ x)
        return x
    x = OMEGA * dinv[:, None] * f
    fc = P.T @ (f - A @ x)
    xc = vcycle(levels, a, b, fc, lvl + 1)
    z = x + COARSE_SCALE * (P @ xc)
    return z + OMEGA * dinv[:, None] * (f - A @ z)
