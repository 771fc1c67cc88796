"""Sequential stiffly accurate DIRK time stepping (oracle side).

This is the plain definition of what the all-at-once block method must
reproduce: the all-at-once system of Sec. 2.1 is the stage equations of
eq. stiffly-accurate-DIRK stacked together, and the splitting / Newton loop of
Algorithm 1 only changes how that solution is reached.  Stage ``i`` of step
``n`` solves (stage-index reading of eq. stiffly-accurate-DIRK)

    (1/tau) M (y_i - y^n) + sum_{j<=i} a_ij f(y_j) = 0,   y^{n+1} = y_m,

with ``f(y) = K y - b`` (linear) or a nonlinear ``f`` (Sec. 2.2).  An explicit
first stage is ``y_1 = y^n``.  Each implicit stage is solved by a direct sparse
LU (default) or by a Jacobi-preconditioned Krylov method from scipy.

``rk_linear`` covers fully implicit tableaux (the remark on fully implicit
Runge-Kutta methods after Algorithm 1) by solving the coupled stages of a step
together.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .timecoupling import implicit_part, resolve


def linear_solve(A, rhs, x0=None, kind="direct", rtol=1e-13):
    """Solve ``A x = rhs``: sparse LU, or Jacobi-preconditioned CG / GMRES(50) / BiCGStab.

    Iterative solves stop at ``||rhs - A x|| <= rtol ||rhs||``.
    """
    if kind == "direct":
        return spla.spsolve(sp.csc_matrix(A), rhs)
    dinv = 1.0 / A.diagonal()
    P = spla.LinearOperator(A.shape, matvec=lambda v: dinv * v, dtype=np.float64)
    x0 = np.zeros_like(rhs) if x0 is None else x0
    if kind == "cg":
        x, info = spla.cg(A, rhs, x0=x0, rtol=rtol, atol=0.0, maxiter=100000, M=P)
    elif kind == "gmres":
        x, info = spla.gmres(A, rhs, x0=x0, rtol=rtol, atol=0.0, restart=50, maxiter=100000, M=P)
    elif kind == "bicgstab":
        x, info = spla.bicgstab(A, rhs, x0=x0, rtol=rtol, atol=0.0, maxiter=100000, M=P)
    else:
        raise ValueError(f"unknown solver {kind!r}")
    if info != 0:
        raise RuntimeError(f"{kind} did not converge (info={info})")
    return x


def _mass(M, N):
    return sp.identity(N, format="csr") if M is None else M


def dirk_linear(K, b, y0, tau, method, n_steps, theta=0.5, M=None, solver="direct", rtol=1e-13):
    """Step ``M y' + K y = b`` (constant ``b``) ``n_steps`` times.

    ``method`` is a method name or a custom stiffly accurate ``(A, c)`` (``timecoupling.resolve``).
    Returns ``(ys, stages)``: ``ys[n]`` is ``y^n`` (``ys[0] = y0``) and
    ``stages[n]`` the list of implicit-stage vectors of step ``n``.
    """
    A, _, c = resolve(method, theta)
    Ai, ae, _, _ = implicit_part(A, c)
    mi = Ai.shape[0]
    N = K.shape[0]
    M = _mass(M, N)
    y = np.asarray(y0, dtype=np.float64).copy()
    ys, stages_all = [y.copy()], []
    for _ in range(n_steps):
        My = M @ y
        f_yn = K @ y - b
        st, fst = [], []
        for q in range(mi):
            rhs = My / tau - ae[q] * f_yn + Ai[q, q] * b
            for j in range(q):
                rhs = rhs - Ai[q, j] * fst[j]
            J = (M / tau + Ai[q, q] * K).tocsr()
            yq = linear_solve(J, rhs, x0=(st[-1] if st else y), kind=solver, rtol=rtol)
            st.append(yq)
            fst.append(K @ yq - b)
        y = st[-1].copy()
        ys.append(y.copy())
        stages_all.append(st)
    return ys, stages_all


def rk_linear(K, b, y0, tau, method, n_steps, M=None):
    """Step ``M y' + K y = b`` with any stiffly accurate Runge-Kutta tableau, one step at a time.

    All ``m`` stages of a step are solved together: with ``f(y) = K y - b`` the stage equations
    ``(1/tau) M (y_i - y^n) + sum_j a_ij f(y_j) = 0`` (Sec. 2 with the sum over every stage, which
    is the fully implicit case of the remark after Algorithm 1) are, stacked stage by stage,

        (I_m (x) M/tau + A (x) K) [y_1; ...; y_m] = 1 (x) M y^n / tau + (A 1) (x) b,

    solved by one sparse LU of the ``mN x mN`` matrix.  ``y^{n+1} = y_m``.  An explicit first
    stage (a zero first row) is kept as an ordinary stage, whose equation then gives ``y_1 = y^n``.
    Returns ``(ys, stages)`` like ``dirk_linear``.
    """
    A, _, _ = resolve(method)
    m = A.shape[0]
    N = K.shape[0]
    M = _mass(M, N)
    Mt = sp.csr_matrix(M) / tau
    big = (sp.kron(sp.identity(m), Mt) + sp.kron(sp.csr_matrix(A), sp.csr_matrix(K))).tocsc()
    lu = spla.splu(big)
    rowsum = A.sum(axis=1)
    y = np.asarray(y0, dtype=np.float64).copy()
    ys, stages_all = [y.copy()], []
    for _ in range(n_steps):
        rhs = np.concatenate([Mt @ y + rowsum[i] * b for i in range(m)])
        Ys = lu.solve(rhs)
        st = [Ys[i * N:(i + 1) * N].copy() for i in range(m)]
        y = st[-1].copy()
        ys.append(y.copy())
        stages_all.append(st)
    return ys, stages_all


def dirk_nonlinear(fop, y0, tau, method, n_steps, theta=0.5, M=None, solver="direct",
                   rtol=1e-13, newton_rtol=1e-12, max_newton=50):
    """Step ``M y' + f(y) = 0`` with Newton's method (exact Jacobian) on every implicit stage.

    ``fop`` provides ``f(y)`` and ``jac(y)``.  A stage stops when
    ``||G(y)|| <= newton_rtol * ||M y^n / tau||`` with ``G`` the stage residual.
    Returns ``(ys, stages, newton_iterations_per_step)``.
    """
    A, _, c = resolve(method, theta)
    Ai, ae, _, _ = implicit_part(A, c)
    mi = Ai.shape[0]
    y = np.asarray(y0, dtype=np.float64).copy()
    N = y.shape[0]
    M = _mass(M, N)
    ys, stages_all, iters = [y.copy()], [], []
    for _ in range(n_steps):
        My = M @ y
        f_yn = fop.f(y)
        st, fst = [], []
        its = 0
        for q in range(mi):
            known = -My / tau + ae[q] * f_yn
            for j in range(q):
                known = known + Ai[q, j] * fst[j]
            x = (st[-1] if st else y).copy()
            scale = np.linalg.norm(My / tau)
            for it in range(max_newton + 1):
                G = M @ x / tau + known + Ai[q, q] * fop.f(x)
                if np.linalg.norm(G) <= newton_rtol * scale:
                    break
                if it == max_newton:
                    raise RuntimeError("stage Newton did not converge")
                J = (M / tau + Ai[q, q] * fop.jac(x)).tocsr()
                x = x - linear_solve(J, G, kind=solver, rtol=rtol)
                its += 1
            st.append(x)
            fst.append(fop.f(x))
        y = st[-1].copy()
        ys.append(y.copy())
        stages_all.append(st)
        iters.append(its)
    return ys, stages_all, iters
