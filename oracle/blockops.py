"""Plain definitions of the block kernels (oracle side).

Sec. 3 names the block operator ``Y <- A X`` on an N x k block as the main
ingredient of a block Krylov iteration; block Krylov methods (Sec. 1,
eq. basic-matrix-equation) add k x k Gram matrices ``X^T Y`` and right
multiplications by k x k coefficient matrices.  These are the definitions the
HIP kernels are compared against, in FP64.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def csr(rowptr, col, val, N):
    return sp.csr_matrix((np.asarray(val, np.float64), np.asarray(col), np.asarray(rowptr)), shape=(N, N))


def block_operator(K, X, alpha=0.0, beta=1.0, mdiag=None):
    """``alpha M X + beta K X`` with ``M = diag(mdiag)`` (identity if None)."""
    X = np.asarray(X, dtype=np.float64)
    MX = X if mdiag is None else np.asarray(mdiag)[:, None] * X
    return alpha * MX + beta * (K @ X)


def gram(X, Y):
    """``X^T Y`` (k x k)."""
    return np.asarray(X, np.float64).T @ np.asarray(Y, np.float64)


def right_multiply(X, C):
    """``X C`` for an N x k block and a k x k matrix."""
    return np.asarray(X, np.float64) @ np.asarray(C, np.float64)


def block_solve(K, alpha, beta, B, mdiag=None):
    """Exact solution of ``(alpha M + beta K) X = B`` column by column (sparse LU)."""
    N = K.shape[0]
    Mm = sp.identity(N) if mdiag is None else sp.diags(mdiag)
    lu = spla.splu(sp.csc_matrix(alpha * Mm + beta * K))
    B = np.asarray(B, np.float64)
    return np.column_stack([lu.solve(B[:, j]) for j in range(B.shape[1])])
