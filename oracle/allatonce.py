"""All-at-once system, matrix-equation residual and splitting fixed point (oracle side).

Sec. 2.1: the stages of ``s`` steps solve
``[A1 (x) M + A2 (x) K] vec Y = [A2 (x) I] vec B + vec B0`` (eq.
general-system-time-steps) where ``vec`` stacks the columns of the N x k block
``Y``.  With ``(C (x) A) vec X = vec(A X C^T)`` this is the matrix equation
``M Y A1^T + K Y A2^T = B A2^T + B0``; its residual (Sec. 2.2, with the sign of
the ``F`` term read so that it agrees with the linear system) is

    R(Y) = M Y A1^T + F(T, Y) A2^T - B0,   F(T, Y)_j = f(T_j, Y_j) = K Y_j - b_j.

The splitting (eq. matrix-splitting) keeps ``(1/tau) M + beta K`` on the left
and iterates eq. matrix-fixed-point-equation.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def vec(Y):
    """Stack the columns of Y into one vector."""
    return np.asarray(Y).ravel(order="F")


def unvec(v, N):
    return np.asarray(v).reshape((-1, N)).T.copy()


def _dense(A):
    return A.toarray() if sp.issparse(A) else np.asarray(A, dtype=np.float64)


def kron_operator(M, K, A1, A2):
    """Dense ``A1 (x) M + A2 (x) K`` (tiny problems only)."""
    return np.kron(A1, _dense(M)) + np.kron(A2, _dense(K))


def solve_dense(M, K, A1, A2, B, B0):
    """Brute-force solve of the all-at-once system; returns the N x k block Y."""
    N = K.shape[0]
    rhs = np.kron(A2, np.eye(N)) @ vec(B) + vec(B0)
    return unvec(np.linalg.solve(kron_operator(M, K, A1, A2), rhs), N)


def solve_sparse(M, K, A1, A2, B, B0):
    """The all-at-once system of eq. general-system-time-steps solved directly with a sparse LU of
    ``A1 (x) M + A2 (x) K`` (moderate sizes); returns the N x k block Y."""
    N = K.shape[0]
    M = sp.csr_matrix(M) if sp.issparse(M) else sp.csr_matrix(np.asarray(M, dtype=np.float64))
    Kop = sp.kron(sp.csr_matrix(A1), M) + sp.kron(sp.csr_matrix(A2), sp.csr_matrix(K))
    rhs = vec(np.asarray(B) @ np.asarray(A2).T + np.asarray(B0))
    return unvec(spla.spsolve(Kop.tocsc(), rhs), N)


def residual_linear(M, K, A1, A2, Y, B, B0):
    """``R = M Y A1^T + (K Y - B) A2^T - B0`` (matrix form)."""
    return M @ Y @ A1.T + (K @ Y - B) @ A2.T - B0


def residual_nonlinear(M, fcols, A1, A2, Y, B0):
    """``R = M Y A1^T + F A2^T - B0`` with ``F[:, j] = fcols(j, Y[:, j])``."""
    F = np.column_stack([fcols(j, Y[:, j]) for j in range(Y.shape[1])])
    return M @ Y @ A1.T + F @ A2.T - B0


def splitting_sweep(M, K, A1, A2, tau, beta, Y, B, B0):
    """One sweep of eq. matrix-fixed-point-equation with an exact (direct) solve.

    ``(M/tau + beta K) Y_new = -M Y (A1 - I/tau)^T - K Y (A2 - beta I)^T + B A2^T + B0``
    """
    k = Y.shape[1]
    I = np.eye(k)
    rhs = -(M @ Y @ (A1 - I / tau).T) - K @ Y @ (A2 - beta * I).T + B @ A2.T + B0
    J = sp.csc_matrix(M / tau + beta * K)
    lu = spla.splu(J)
    return np.column_stack([lu.solve(rhs[:, j]) for j in range(k)])


def splitting_sweep_diag(M, K, A1, A2, Y, B, B0):
    """One sweep of the splitting that keeps every column's own diagonal coefficients (the remark
    after eq. matrix-fixed-point-equation: with M a scaled identity the left-hand side
    ``D (x) M + beta I (x) K``, D diagonal, still admits vectorized block Krylov solves).  Column j:

    ``(A1_jj M + A2_jj K) y_j_new = [-M Y (A1 - diag A1)^T - K Y (A2 - diag A2)^T + B A2^T + B0]_j``

    with an exact (direct) solve per column.  For a DIRK window the off-diagonal parts are strictly
    lower triangular, so k sweeps reach the all-at-once solution whatever the diagonal."""
    k = Y.shape[1]
    d1, d2 = np.diag(A1), np.diag(A2)
    rhs = -(M @ Y @ (A1 - np.diag(d1)).T) - K @ Y @ (A2 - np.diag(d2)).T + B @ A2.T + B0
    out = np.empty_like(rhs)
    for j in range(k):
        out[:, j] = spla.spsolve(sp.csc_matrix(d1[j] * M + d2[j] * K), rhs[:, j])
    return out
