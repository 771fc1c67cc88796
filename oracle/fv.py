"""Cell-centred finite-volume operators on the unit square / cube (oracle side).

The paper's experiments use a cell-centred FV discretisation (Sec. 4.1) and
state the semi-discrete problem as ``M y' + K y = b`` (Sec. 1, eq. problem), or
``M y' + f(t, y) = 0`` with ``f(t, y) = K[y] y - b(t)`` in the nonlinear case
(Sec. 2.2).  The paper gives no flux formulas; this module fixes them:

* uniform grid, ``n_d`` cells along axis ``d``, ``h_d = 1/n_d``, cell centres
  at ``(i + 1/2) h_d``, linear index ``ix + nx*iy + nx*ny*iz``;
* every row is divided by the cell volume, so the mass matrix is ``M = I``;
* diffusion: interior face ``P|Q`` normal to axis ``d`` with coefficient
  ``c_f`` contributes ``c_f (u_P - u_Q) / h_d^2`` to row ``P`` and the negative
  to row ``Q``; a linear coefficient field uses the harmonic face mean
  ``c_f = 2 c_P c_Q / (c_P + c_Q)``;
* Dirichlet face with value ``g`` (half a cell from the centre):
  ``2 c_P (u_P - g) / h_d^2``; zero-flux (Neumann) face: nothing;
* convection ``div(v u)`` by first-order upwinding: the flux ``w u_up`` with
  ``w = v . n`` leaves the upwind cell's row positive and enters the other
  row negative; boundary outflow ``w u_P``, boundary inflow ``w g``.

The PDE is ``u_t + div(v u - c grad u) = 0`` (linear) and
``u_t = div(D(u) grad u) + r(u)`` (nonlinear), i.e. ``f(u) = -div_h(D grad_h u) - r(u)``.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


class Grid:
    """Uniform cell-centred grid of ``[0,1]^dim`` with ``n = (nx, ny[, nz])`` cells."""

    def __init__(self, n):
        self.n = tuple(int(v) for v in n)
        self.dim = len(self.n)
        if self.dim not in (1, 2, 3):
            raise ValueError("grid must be 1-, 2- or 3-dimensional")
        self.h = tuple(1.0 / v for v in self.n)
        self.N = int(np.prod(self.n))
        self.shape = tuple(reversed(self.n))  # numpy shape, slowest axis first
        self._idx = np.arange(self.N).reshape(self.shape)

    def _array_axis(self, d: int) -> int:
        return self.dim - 1 - d

    def interior_faces(self, d: int):
        """(P, Q) flat cell indices of every interior face normal to axis d; Q = P + e_d."""
        ax = self._array_axis(d)
        m = self.n[d]
        P = np.take(self._idx, np.arange(0, m - 1), axis=ax).ravel()
        Q = np.take(self._idx, np.arange(1, m), axis=ax).ravel()
        return P, Q

    def boundary_cells(self, d: int, side: int):
        """Flat indices of the cells touching the low (side 0) or high (side 1) face of axis d."""
        ax = self._array_axis(d)
        i = 0 if side == 0 else self.n[d] - 1
        return np.take(self._idx, [i], axis=ax).ravel()


def _bc_of(bc, d, side):
    """Boundary spec of face (d, side): ('dirichlet', g) or ('neumann',). Default: Dirichlet 0."""
    if bc is None:
        return ("dirichlet", 0.0)
    spec = bc.get((d, side), bc.get("default", ("dirichlet", 0.0)))
    if spec[0] not in ("dirichlet", "neumann"):
        raise ValueError(f"unknown boundary condition {spec!r}")
    return spec


def assemble_linear(n, kappa=1.0, velocity=None, bc=None):
    """Assemble ``K`` (CSR) and ``b`` for ``u_t + div(v u - kappa grad u) = 0`` with ``M = I``.

    ``kappa`` is a scalar or a per-cell array (harmonic face means); ``velocity``
    a constant vector; ``bc`` maps ``(axis, side)`` (or ``"default"``) to
    ``("dirichlet", g)`` or ``("neumann",)``.
    """
    g = Grid(n)
    N = g.N
    kap = np.full(N, float(kappa)) if np.isscalar(kappa) else np.asarray(kappa, dtype=np.float64).ravel()
    if kap.shape != (N,):
        raise ValueError("kappa must be scalar or have one value per cell")
    vel = np.zeros(g.dim) if velocity is None else np.asarray(velocity, dtype=np.float64)
    rows, cols, vals = [], [], []
    b = np.zeros(N)

    def add(r, c, v):
        rows.append(np.asarray(r))
        cols.append(np.asarray(c))
        vals.append(np.broadcast_to(np.asarray(v, dtype=np.float64), np.shape(r)).copy())

    for d in range(g.dim):
        h = g.h[d]
        P, Q = g.interior_faces(d)
        ksum = kap[P] + kap[Q]
        kf = np.divide(2.0 * kap[P] * kap[Q], ksum, out=np.zeros_like(ksum), where=ksum > 0)
        t = kf / h ** 2
        add(P, P, t)
        add(P, Q, -t)
        add(Q, Q, t)
        add(Q, P, -t)
        w = vel[d]
        if w > 0:
            add(P, P, w / h)
            add(Q, P, -w / h)
        elif w < 0:
            add(P, Q, w / h)
            add(Q, Q, -w / h)
        for side in (0, 1):
            cells = g.boundary_cells(d, side)
            spec = _bc_of(bc, d, side)
            if spec[0] == "neumann":
                continue
            gval = float(spec[1])
            tb = 2.0 * kap[cells] / h ** 2
            add(cells, cells, tb)
            b[cells] += tb * gval
            w_out = -vel[d] if side == 0 else vel[d]
            if w_out > 0:
                add(cells, cells, w_out / h)
            elif w_out < 0:
                b[cells] -= w_out * gval / h
    K = sp.coo_matrix(
        (np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(N, N)
    ).tocsr()
    K.sum_duplicates()
    K.sort_indices()
    return K, b


class NonlinearDiffusionReaction:
    """``f(u) = -div_h(D(u) grad_h u) - r(u)`` with polynomial ``D`` and ``r`` (Sec. 2.2).

    ``D(u) = sum_i dcoef[i] u^i`` and ``r(u) = sum_i rcoef[i] u^i``.  The face
    coefficient is the arithmetic mean ``(D(u_P) + D(u_Q)) / 2``; a Dirichlet
    face with value ``g`` uses ``(D(u_P) + D(g)) / 2`` and the half-cell
    distance.  Boundaries default to zero flux (Neumann).
    """

    def __init__(self, n, dcoef=(1.0, 0.0, 1.0), rcoef=(0.0, 0.0, 0.0, -1.0), bc=None):
        self.grid = Grid(n)
        self.dcoef = np.asarray(dcoef, dtype=np.float64)
        self.rcoef = np.asarray(rcoef, dtype=np.float64)
        self.bc = {"default": ("neumann",)} if bc is None else bc
        self._faces = []
        for d in range(self.grid.dim):
            P, Q = self.grid.interior_faces(d)
            self._faces.append((P, Q, 1.0 / self.grid.h[d] ** 2))
        self._bfaces = []
        for d in range(self.grid.dim):
            for side in (0, 1):
                spec = _bc_of(self.bc, d, side)
                if spec[0] == "dirichlet":
                    self._bfaces.append((self.grid.boundary_cells(d, side), float(spec[1]), 2.0 / self.grid.h[d] ** 2))

    def D(self, u):
        return np.polynomial.polynomial.polyval(u, self.dcoef)

    def dD(self, u):
        return np.polynomial.polynomial.polyval(u, np.polynomial.polynomial.polyder(self.dcoef))

    def r(self, u):
        return np.polynomial.polynomial.polyval(u, self.rcoef)

    def dr(self, u):
        return np.polynomial.polynomial.polyval(u, np.polynomial.polynomial.polyder(self.rcoef))

    def f(self, u):
        u = np.asarray(u, dtype=np.float64)
        out = -self.r(u)
        Du = self.D(u)
        for P, Q, w in self._faces:
            flux = 0.5 * (Du[P] + Du[Q]) * (u[P] - u[Q]) * w
            np.add.at(out, P, flux)
            np.add.at(out, Q, -flux)
        for cells, gval, w in self._bfaces:
            out[cells] += 0.5 * (Du[cells] + self.D(gval)) * (u[cells] - gval) * w
        return out

    def jac(self, u):
        """Exact Jacobian ``df/du`` (CSR)."""
        u = np.asarray(u, dtype=np.float64)
        N = self.grid.N
        Du, dDu = self.D(u), self.dD(u)
        rows, cols, vals = [np.arange(N)], [np.arange(N)], [-self.dr(u)]
        for P, Q, w in self._faces:
            Df = 0.5 * (Du[P] + Du[Q])
            diff = u[P] - u[Q]
            # flux_PQ = Df * diff * w enters row P (+) and row Q (-)
            dflux_dP = (Df + 0.5 * dDu[P] * diff) * w
            dflux_dQ = (-Df + 0.5 * dDu[Q] * diff) * w
            rows += [P, P, Q, Q]
            cols += [P, Q, P, Q]
            vals += [dflux_dP, dflux_dQ, -dflux_dP, -dflux_dQ]
        for cells, gval, w in self._bfaces:
            Df = 0.5 * (Du[cells] + self.D(gval))
            rows.append(cells)
            cols.append(cells)
            vals.append((Df + 0.5 * dDu[cells] * (u[cells] - gval)) * w)
        J = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(N, N)).tocsr()
        J.sum_duplicates()
        J.sort_indices()
        return J
