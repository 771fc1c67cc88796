"""Pins for user-given stiffly accurate DIRK tableaux (Sec. 2, eq. stiffly-accurate-DIRK) and for the
splitting that keeps each column's own diagonal (the remark after eq. matrix-fixed-point-equation on
left-hand sides ``D (x) M + beta I (x) K``).  Two tableaux with distinct diagonal entries:

* T2: A = [[1/3, 0], [3/4, 1/4]], c = (1/3, 1) (order 2);
* T3: A = [[0, 0, 0], [1/4, 1/4, 0], [1/3, 1/3, 1/3]], c = (0, 1/2, 1), an explicit first stage
  that the all-at-once form eliminates (Sec. 2.1), implicit diagonal 1/4, 1/3 (order 2).
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import allatonce as aao
from oracle import fv, stepping
from oracle import timecoupling as tc
from paper_2504_02117_amd import inputs

T2 = (np.array([[1 / 3, 0.0], [0.75, 0.25]]), np.array([1 / 3, 1.0]))
T3 = (np.array([[0.0, 0.0, 0.0], [0.25, 0.25, 0.0], [1 / 3, 1 / 3, 1 / 3]]), np.array([0.0, 0.5, 1.0]))
TABLEAUX = {"T2": T2, "T3": T3}


@pytest.mark.parametrize("name", ["T2", "T3"])
def test_custom_tableau_is_stiffly_accurate_and_second_order(name):
    A, b, c = tc.resolve(TABLEAUX[name])
    assert tc.is_stiffly_accurate(A, b)
    assert not tc.is_fully_implicit(A)
    assert b.sum() == pytest.approx(1.0, abs=1e-15)
    assert b @ c == pytest.approx(0.5, abs=1e-15)          # order 2
    # not order 3: one of the two third-order conditions fails
    assert abs(b @ c ** 2 - 1.0 / 3.0) > 1e-3 or abs(b @ (A @ c) - 1.0 / 6.0) > 1e-3
    Ai, _, _, _ = tc.implicit_part(A, c)
    assert len(set(np.diag(Ai))) == Ai.shape[0]             # distinct diagonal entries


def test_custom_tableau_rejections():
    with pytest.raises(ValueError):  # c is not the row sums
        tc.custom_tableau([[0.5, 0.0], [0.5, 0.5]], [0.4, 1.0])
    with pytest.raises(ValueError):  # does not end at c = 1 (sum of b != 1)
        tc.custom_tableau([[0.5, 0.0], [0.25, 0.5]], [0.5, 0.75])
    with pytest.raises(ValueError):  # not square
        tc.custom_tableau(np.ones((2, 3)), [1.0, 1.0])


@pytest.mark.parametrize("name", ["T2", "T3"])
def test_custom_dirk_eigenvector_decay(name):
    """Pi sin(pi x_d) is an exact eigenvector of the Dirichlet FV Laplacian, so the stepped solution
    is R(-tau lambda)^n times it, with R(z) = 1 + z b^T (I - z A)^-1 1 from the tableau alone."""
    n, tau, steps = (9, 11), 4e-3, 5
    K, b = fv.assemble_linear(n)
    u0 = inputs.sin_product(n)
    lam = sum(4 * m * m * math.sin(math.pi / (2 * m)) ** 2 for m in n)
    A, bw, _ = tc.resolve(TABLEAUX[name])
    z = -tau * lam
    R = 1 + z * bw @ np.linalg.solve(np.eye(A.shape[0]) - z * A, np.ones(A.shape[0]))
    ys, _ = stepping.dirk_linear(K, b, u0, tau, TABLEAUX[name], steps)
    for s in range(steps + 1):
        np.testing.assert_allclose(ys[s], R ** s * u0, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("name", ["T2", "T3"])
def test_custom_dirk_matches_coupled_stage_solve(name):
    """Stage-by-stage stepping equals the all-stages-at-once sparse LU of each step."""
    n = (7, 6, 5)
    kap = inputs.lognormal_field(n, 0.0, 1.0, 1.5, 21)
    K, b = fv.assemble_linear(n, kappa=kap, bc={"default": ("dirichlet", 0.25)})
    y0 = inputs.smooth_random(n, 22)
    ys, _ = stepping.dirk_linear(K, b, y0, 0.02, TABLEAUX[name], 4)
    yr, _ = stepping.rk_linear(K, b, y0, 0.02, TABLEAUX[name], 4)
    for s in range(5):
        np.testing.assert_allclose(ys[s], yr[s], rtol=1e-12, atol=1e-12)


def test_custom_reproduces_named_sdirk2():
    g = 1 - 1 / math.sqrt(2)
    custom = (np.array([[g, 0.0], [1 - g, g]]), np.array([g, 1.0]))
    K, b = fv.assemble_linear((8, 7), bc={"default": ("dirichlet", 1.0)})
    y0 = inputs.smooth_random((8, 7), 3)
    ya, _ = stepping.dirk_linear(K, b, y0, 0.05, "sdirk2", 3)
    yb, _ = stepping.dirk_linear(K, b, y0, 0.05, custom, 3)
    for s in range(4):
        np.testing.assert_array_equal(ya[s], yb[s])


@pytest.mark.parametrize("name", ["T2", "T3"])
@pytest.mark.parametrize("s", [1, 3])
def test_diagonal_splitting_is_exact_after_k_sweeps(name, s):
    """The splitting that keeps each column's diagonal coefficients reaches the all-at-once solution
    (= sequential stepping) after k sweeps for a DIRK window, while the splitting with the front
    column's coefficient beta for every column does not when the diagonal entries differ."""
    n = (5, 4)
    kap = inputs.lognormal_field(n, 0.0, 1.0, 1.0, 5)
    K, b = fv.assemble_linear(n, kappa=kap, bc={"default": ("dirichlet", 0.5)})
    N = K.shape[0]
    tau = 0.05
    A, _, c = tc.resolve(TABLEAUX[name])
    A1, A2 = tc.time_stepping_matrices(A, c, s, tau)
    k = A1.shape[0]
    y0 = inputs.smooth_random(n, 6)
    B = np.tile(b[:, None], (1, k))
    B0 = tc.window_b0(A, c, k, 0, tau, y0, K @ y0 - b, [])
    M = sp.identity(N, format="csr")
    exact = aao.solve_dense(M, K, A1, A2, B, B0)
    _, st = stepping.dirk_linear(K, b, y0, tau, TABLEAUX[name], s)
    np.testing.assert_allclose(exact, np.column_stack([v for step in st for v in step]), rtol=1e-11, atol=1e-11)
    Yd = np.zeros((N, k))
    Yf = np.zeros((N, k))
    for _ in range(k):
        Yd = aao.splitting_sweep_diag(M, K, A1, A2, Yd, B, B0)
        Yf = aao.splitting_sweep(M, K, A1, A2, tau, A2[0, 0], Yf, B, B0)
    scale = np.abs(exact).max()
    assert np.abs(Yd - exact).max() <= 1e-11 * scale
    assert np.abs(Yf - exact).max() > 1e-6 * scale
