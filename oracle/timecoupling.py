"""Butcher tableaux and all-at-once time-coupling matrices (oracle side).

Sec. 2 writes one step of an m-stage stiffly accurate DIRK method for
``M y' + f(t, y) = 0`` as (eq. stiffly-accurate-DIRK, stage index ``i``):

    (1/tau) M (y_i - y^n) + sum_{j<=i} a_ij f(t^n + c_j tau, y_j) = 0,
    y^{n+1} = y_m.

Sec. 2.1 stacks the stages (and, eq. time-stepping-matrices-multiple-parallel-
time-steps, ``s`` consecutive steps) into ``[A1 (x) M + A2 (x) K] vec Y = ...``.
An explicit first stage (``a_11 = 0``) is eliminated first (Sec. 2.1): its
couplings ``a_i1`` move into ``A2`` (below the diagonal blocks, where ``A1``
carries ``-1/tau``) and into ``B0``.  Example 2 prints the result for the
theta-method.

Pipelining (Sec. 2.2, eq. matrix-equation-pipelining) uses the k x k
sub-blocks of these matrices that start at the diagonal index of the front
stage, and a ``B0`` whose nonzero columns are those stages of the front step
that lie in the window.  The paper's ``B0`` display mixes the stage and column
index and its sign; the reading used here (stage ``q`` of the front step,
``f = K y - b``) is

    B0_q = (1/tau) M y^n - sum_{j < front} a_qj f(y_j) - a_q1^expl f(y^n).
"""
from __future__ import annotations

import math

import numpy as np


def tableau(name: str, theta: float = 0.5):
    """Butcher tableau ``(A, b, c)`` of a stiffly accurate method.

    * ``"ie"``: implicit Euler.
    * ``"theta"``: the theta-method as a 2-stage stiffly accurate scheme with
      an explicit first stage (Sec. 2.1, Example 1).
    * ``"sdirk2"``: the 2-stage L-stable SDIRK with ``gamma = 1 - 1/sqrt(2)``
      (the paper does not print its second-order DIRK; this is the reading).
    * ``"radau2"``: the 2-stage Radau IIA collocation method (order 3, stiffly
      accurate, L-stable), a fully implicit scheme for the remark on fully
      implicit Runge-Kutta methods that follows Algorithm 1.
    """
    name = name.lower()
    if name == "ie":
        A = np.array([[1.0]])
        b = np.array([1.0])
        c = np.array([1.0])
    elif name == "theta":
        A = np.array([[0.0, 0.0], [1.0 - theta, theta]])
        b = np.array([1.0 - theta, theta])
        c = np.array([0.0, 1.0])
    elif name == "sdirk2":
        g = 1.0 - 1.0 / math.sqrt(2.0)
        A = np.array([[g, 0.0], [1.0 - g, g]])
        b = np.array([1.0 - g, g])
        c = np.array([g, 1.0])
    elif name == "radau2":
        A = np.array([[5.0 / 12.0, -1.0 / 12.0], [0.75, 0.25]])
        b = np.array([0.75, 0.25])
        c = np.array([1.0 / 3.0, 1.0])
    else:
        raise ValueError(f"unknown method {name!r}")
    return A, b, c


def custom_tableau(A, c, tol: float = 1e-12):
    """Tableau ``(A, b, c)`` of a user-given stiffly accurate method: ``b`` is the last row of ``A``
    (Sec. 2, eq. stiffly-accurate-DIRK: the step result is the last stage).  The stage times must be
    the row sums ``c_i = sum_j a_ij`` and the last one must be 1 (so that ``sum_i b_i = 1``);
    otherwise the tableau does not define a consistent stiffly accurate method and ``ValueError`` is
    raised."""
    A = np.array(A, dtype=np.float64)
    c = np.array(c, dtype=np.float64)
    m = A.shape[0]
    if A.shape != (m, m) or c.shape != (m,) or m < 1:
        raise ValueError("A must be m x m and c of length m")
    if not (np.all(np.isfinite(A)) and np.all(np.isfinite(c))):
        raise ValueError("tableau entries must be finite")
    if np.any(np.abs(A.sum(axis=1) - c) > tol * np.maximum(1.0, np.abs(c))):
        raise ValueError("stage times must be the row sums of A")
    if abs(c[-1] - 1.0) > tol:
        raise ValueError("a stiffly accurate method ends at c_m = 1")
    return A, A[-1].copy(), c


def resolve(method, theta: float = 0.5):
    """``(A, b, c)`` for a method name (see ``tableau``) or a custom ``(A, c)`` pair."""
    if isinstance(method, str):
        return tableau(method, theta)
    A, c = method
    return custom_tableau(A, c)


def is_fully_implicit(A) -> bool:
    """True when some stage couples to a later one (an entry above the diagonal)."""
    return bool(np.any(np.triu(np.asarray(A, dtype=np.float64), 1)))


def averaged_beta(A) -> float:
    """Splitting coefficient of a fully implicit tableau: the remark on fully implicit Runge-Kutta
    methods (after Algorithm 1) replaces the stage-wise Jacobian by an averaged one.  Reading: a
    single ``J = M/tau + beta K`` for every stage with ``beta = |det A|^(1/m)``, the geometric mean
    of the moduli of A's eigenvalues (sqrt(1/6) for 2-stage Radau IIA)."""
    A = np.asarray(A, dtype=np.float64)
    return float(abs(np.linalg.det(A)) ** (1.0 / A.shape[0]))


def is_stiffly_accurate(A, b) -> bool:
    """``b_i = a_{m,i}`` for all i (Sec. 2)."""
    return bool(np.array_equal(np.asarray(A)[-1], np.asarray(b)))


def implicit_part(A, c):
    """Split off an explicit first stage (``a_11 = 0`` and first row zero).

    Returns ``(A_impl, a_expl, c_impl, explicit)`` where ``a_expl[i]`` is the
    coupling of implicit stage ``i`` to the eliminated stage (zeros if none).
    """
    A = np.asarray(A, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    if A[0, 0] == 0.0 and not np.any(A[0]):
        return A[1:, 1:].copy(), A[1:, 0].copy(), c[1:].copy(), True
    return A.copy(), np.zeros(A.shape[0]), c.copy(), False


def time_stepping_matrices(A, c, s: int, tau: float):
    """``A1, A2`` for ``s`` consecutive steps (eq. time-stepping-matrices-multiple-parallel-time-steps).

    Size ``s*m' x s*m'`` with ``m'`` the number of implicit stages.  ``A1`` is
    ``(1/tau) I`` with ``-1/tau`` coupling every stage of step ``j+1`` to the
    last stage of step ``j``; ``A2`` is block diagonal in ``A_impl`` plus the
    eliminated explicit-stage couplings at the positions of those ``-1/tau``.
    """
    Ai, ae, _, explicit = implicit_part(A, c)
    mi = Ai.shape[0]
    k = s * mi
    A1 = np.eye(k) / tau
    A2 = np.zeros((k, k))
    for j in range(s):
        A2[j * mi:(j + 1) * mi, j * mi:(j + 1) * mi] = Ai
    for j in range(1, s):
        for i in range(mi):
            A1[j * mi + i, j * mi - 1] = -1.0 / tau
            if explicit:
                A2[j * mi + i, j * mi - 1] = ae[i]
    return A1, A2


def window_matrices(A, c, k: int, phase: int, tau: float):
    """Pipelined window ``A1^(n,k), A2^(n,k)`` (Sec. 2.2): the k x k blocks from diagonal index ``phase``.

    ``phase`` is the implicit-stage index (0-based) of the window's front column
    within its time step.
    """
    Ai, _, _, _ = implicit_part(A, c)
    mi = Ai.shape[0]
    if not 0 <= phase < mi:
        raise ValueError("phase must be an implicit stage index")
    s = -(-(phase + k) // mi)
    A1, A2 = time_stepping_matrices(A, c, s, tau)
    return A1[phase:phase + k, phase:phase + k].copy(), A2[phase:phase + k, phase:phase + k].copy(), float(A2[phase, phase])


def window_b0(A, c, k: int, phase: int, tau: float, My_n, f_yn, f_stages):
    """Columns of ``B0^(n,k)`` for a window whose front is implicit stage ``phase`` of step n.

    ``My_n`` is ``M y^n``; ``f_yn`` is ``f(t^n, y^n)`` (used only when an explicit
    first stage was eliminated); ``f_stages[j]`` is ``f`` at the already
    converged implicit stage ``j < phase`` of step n.  Returns an ``N x k``
    array (columns past the front step are zero).
    """
    Ai, ae, _, explicit = implicit_part(A, c)
    mi = Ai.shape[0]
    N = np.asarray(My_n).shape[0]
    B0 = np.zeros((N, k))
    for i in range(k):
        q = phase + i
        if q >= mi:
            break
        col = np.asarray(My_n, dtype=np.float64) / tau
        for j in range(phase):
            col = col - Ai[q, j] * f_stages[j]
        if explicit:
            col = col - ae[q] * f_yn
        B0[:, i] = col
    return B0
