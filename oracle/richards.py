"""Richards' equation on a cell-centred FV grid (oracle side; Sec. 4.3, eq. RelationshipsThetaK).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The equation for the pressure head psi is ``d/dt theta(psi) - div(K(psi) grad(psi + z)) = 0`` with
the van Genuchten closure of eq. RelationshipsThetaK: effective saturation
``Se = (1 + (alpha |psi|)^n)^(-m)``, ``m = 1 - 1/n``, for psi < 0 (Se = 1 otherwise),
``theta = theta_r + (theta_s - theta_r) Se`` and, as printed in the paper, the Mualem conductivity
in terms of ``s = theta / theta_s``: ``K = Ks s^(1/2) (1 - (1 - s^(1/m))^m)^2``.

Discretisation (the paper uses FE; the FV choices are this library's readings):
* unit cube, ``z`` is the last axis (height of the cell centre), every row divided by the volume;
* interior face P|Q along axis d: ``K_f (H_P - H_Q) / h_d^2`` with the total head ``H = psi + z``
  and ``K_f = harm(Ks_P, Ks_Q) * (kr(psi_P) + kr(psi_Q)) / 2`` (kr = K / Ks);
* top face (z = 1): Dirichlet ``psi = g`` half a cell away, ``2 Ks_P (kr_P + kr(g))/2 (H_P - H_g)/h^2``,
  or no flow;
* bottom face (z = 0): free drainage (unit head gradient), outflow ``Ks_P kr(psi_P) / h``, or no flow;
* lateral faces: no flow.

Semi-discrete problem: ``d/dt theta(psi) + F(psi) = 0`` with ``F(psi) = -div_h(K grad_h H)``.
With a nonlinear time derivative the mass term of the all-at-once system is split like the
stiffness term (Sec. 2.2, Remark on additional nonlinearity): the window residual is
``theta(Y) A1^T + F(Y) A2^T - B0`` with ``B0`` built from ``theta(psi^n)``.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .fv import Grid


class VanGenuchten:
    """Closure of eq. RelationshipsThetaK with parameters theta_r, theta_s, alpha, n."""

    def __init__(self, theta_r=0.05, theta_s=0.4, alpha=2.0, n=2.0):
        self.tr, self.ts, self.alpha, self.n = float(theta_r), float(theta_s), float(alpha), float(n)
        self.m = 1.0 - 1.0 / self.n

    def se(self, psi):
        psi = np.asarray(psi, dtype=np.float64)
        neg = psi < 0.0
        out = np.ones_like(psi)
        out[neg] = (1.0 + (self.alpha * -psi[neg]) ** self.n) ** (-self.m)
        return out

    def dse(self, psi):
        psi = np.asarray(psi, dtype=np.float64)
        neg = psi < 0.0
        out = np.zeros_like(psi)
        a = self.alpha * -psi[neg]
        # d/dpsi (1 + a^n)^(-m) with a = -alpha psi
        out[neg] = self.m * self.n * self.alpha * a ** (self.n - 1.0) * (1.0 + a ** self.n) ** (-self.m - 1.0)
        return out

    def theta(self, psi):
        return self.tr + (self.ts - self.tr) * self.se(psi)

    def dtheta(self, psi):
        return (self.ts - self.tr) * self.dse(psi)

    def kr(self, psi):
        s = self.theta(psi) / self.ts
        return np.sqrt(s) * (1.0 - (1.0 - s ** (1.0 / self.m)) ** self.m) ** 2

    def dkr(self, psi):
        s = self.theta(psi) / self.ts
        ds = self.dtheta(psi) / self.ts
        w = 1.0 - s ** (1.0 / self.m)
        g = 1.0 - w ** self.m
        # d/ds [s^(1/2) g^2], g = 1 - (1 - s^(1/m))^m
        with np.errstate(divide="ignore", invalid="ignore"):
            dg = np.where(w > 0.0, self.m * w ** (self.m - 1.0) * (1.0 / self.m) * s ** (1.0 / self.m - 1.0), 0.0)
        dks = 0.5 / np.sqrt(s) * g * g + np.sqrt(s) * 2.0 * g * dg
        return dks * ds


class Richards:
    """``F(psi)``, ``theta(psi)`` and their derivatives on the grid ``n`` (z = last axis)."""

    def __init__(self, n, ks, vg=None, top=("dirichlet", 0.0), bottom="free_drainage"):
        self.grid = Grid(n)
        g = self.grid
        self.vg = vg or VanGenuchten()
        self.ks = np.broadcast_to(np.asarray(ks, dtype=np.float64), (g.N,)).copy()
        self.top, self.bottom = top, bottom
        zc = (np.arange(g.n[-1]) + 0.5) * g.h[-1]
        self.z = np.broadcast_to(zc.reshape((-1,) + (1,) * (g.dim - 1)), g.shape).ravel().copy()
        self._faces = []
        for d in range(g.dim):
            P, Q = g.interior_faces(d)
            kf = 2.0 * self.ks[P] * self.ks[Q] / (self.ks[P] + self.ks[Q])
            self._faces.append((P, Q, kf / g.h[d] ** 2))
        zd = g.dim - 1
        self._top = g.boundary_cells(zd, 1)
        self._bot = g.boundary_cells(zd, 0)
        self._hz = g.h[zd]

    def theta(self, psi):
        return self.vg.theta(psi)

    def dtheta(self, psi):
        return self.vg.dtheta(psi)

    def f(self, psi):
        psi = np.asarray(psi, dtype=np.float64)
        kr = self.vg.kr(psi)
        H = psi + self.z
        out = np.zeros_like(psi)
        for P, Q, w in self._faces:
            q = w * 0.5 * (kr[P] + kr[Q]) * (H[P] - H[Q])
            np.add.at(out, P, q)
            np.add.at(out, Q, -q)
        if self.top[0] == "dirichlet":
            gv = float(self.top[1])
            c = self._top
            krg = self.vg.kr(np.array([gv]))[0]
            out[c] += 2.0 * self.ks[c] * 0.5 * (kr[c] + krg) * (H[c] - (gv + 1.0)) / self._hz ** 2
        if self.bottom == "free_drainage":
            c = self._bot
            out[c] += self.ks[c] * kr[c] / self._hz
        return out

    def jac(self, psi):
        """Exact ``dF/dpsi`` (CSR)."""
        psi = np.asarray(psi, dtype=np.float64)
        N = self.grid.N
        kr, dkr = self.vg.kr(psi), self.vg.dkr(psi)
        H = psi + self.z
        rows, cols, vals = [], [], []
        diag = np.zeros(N)
        for P, Q, w in self._faces:
            m = 0.5 * (kr[P] + kr[Q])
            dH = H[P] - H[Q]
            dq_dP = w * (m + 0.5 * dkr[P] * dH)   # q = w m dH enters row P (+) and row Q (-)
            dq_dQ = w * (-m + 0.5 * dkr[Q] * dH)
            np.add.at(diag, P, dq_dP)
            np.add.at(diag, Q, -dq_dQ)
            rows += [P, Q]
            cols += [Q, P]
            vals += [dq_dQ, -dq_dP]
        if self.top[0] == "dirichlet":
            gv = float(self.top[1])
            c = self._top
            krg = self.vg.kr(np.array([gv]))[0]
            dH = H[c] - (gv + 1.0)
            diag[c] += 2.0 * self.ks[c] * (0.5 * (kr[c] + krg) + 0.5 * dkr[c] * dH) / self._hz ** 2
        if self.bottom == "free_drainage":
            c = self._bot
            diag[c] += self.ks[c] * dkr[c] / self._hz
        rows.append(np.arange(N))
        cols.append(np.arange(N))
        vals.append(diag)
        return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(N, N))


def window_residual(model, A1, A2, Y, B0):
    """``theta(Y) A1^T + F(Y) A2^T - B0`` column by column (Sec. 2.2 with a split mass term)."""
    Th = np.column_stack([model.theta(Y[:, j]) for j in range(Y.shape[1])])
    F = np.column_stack([model.f(Y[:, j]) for j in range(Y.shape[1])])
    return Th @ A1.T + F @ A2.T - B0


def implicit_euler(model, psi0, tau, n_steps, newton_rtol=1e-12, max_newton=60, lin=None):
    """Sequential implicit Euler with Newton's method and direct solves:
    ``G(psi) = (theta(psi) - theta(psi^n)) / tau + F(psi) = 0`` for every step (the plain
    definition the all-at-once iteration must reproduce).  ``lin = L`` replaces theta' in the
    Jacobian by the constant L (the L-scheme).  A step stops when
    ``||G|| <= newton_rtol * ||theta(psi^n) / tau||``.  Returns ``(psis, iterations)``."""
    psi = np.asarray(psi0, dtype=np.float64).copy()
    out, its = [psi.copy()], []
    for _ in range(n_steps):
        th_n = model.theta(psi)
        scale = np.linalg.norm(th_n / tau)
        x = psi.copy()
        for it in range(max_newton + 1):
            G = (model.theta(x) - th_n) / tau + model.f(x)
            if np.linalg.norm(G) <= newton_rtol * scale:
                break
            if it == max_newton:
                raise RuntimeError("implicit Euler Newton did not converge")
            m = model.dtheta(x) if lin is None else np.full_like(x, lin)
            J = (sp.diags(m / tau) + model.jac(x)).tocsc()
            x = x - spla.spsolve(J, G)
        psi = x
        out.append(psi.copy())
        its.append(it)
    return out, its
