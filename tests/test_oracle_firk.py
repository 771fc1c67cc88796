"""Pins for the fully implicit Runge-Kutta case (the remark on fully implicit methods after
Algorithm 1): the 2-stage Radau IIA tableau, sequential stepping with all stages solved together,
the all-at-once system for several steps, and the averaged-Jacobian splitting."""
import math

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import allatonce as aao
from oracle import fv, stepping
from oracle import timecoupling as tc
from paper_2504_02117_amd import inputs


def test_radau2_order_and_collocation_conditions():
    A, b, c = tc.tableau("radau2")
    # order 3: the rooted-tree conditions up to order 3
    assert b.sum() == pytest.approx(1.0, abs=1e-15)
    assert b @ c == pytest.approx(0.5, abs=1e-15)
    assert b @ c ** 2 == pytest.approx(1.0 / 3.0, abs=1e-15)
    assert b @ (A @ c) == pytest.approx(1.0 / 6.0, abs=1e-15)
    # collocation at c: sum_j a_ij c_j^(q-1) = c_i^q / q for q = 1, 2
    np.testing.assert_allclose(A.sum(1), c, atol=1e-15)
    np.testing.assert_allclose(A @ c, c ** 2 / 2, atol=1e-15)
    # Radau IIA nodes: roots of the right Radau polynomial, with c_m = 1
    assert c[-1] == 1.0 and c[0] == pytest.approx(1.0 / 3.0, abs=1e-15)
    assert tc.is_stiffly_accurate(A, b)
    assert tc.is_fully_implicit(A)
    for name in ("ie", "theta", "sdirk2"):
        assert not tc.is_fully_implicit(tc.tableau(name)[0])


def _R_radau2(z):
    return (1 + z / 3) / (1 - 2 * z / 3 + z * z / 6)


def test_radau2_stability_function():
    # R(z) = 1 + z b^T (I - z A)^{-1} 1 must equal the (1,2)-Pade approximant of exp, which is
    # the stability function of 2-stage Radau IIA: local error O(z^4) and R(-inf) = 0.
    A, b, _ = tc.tableau("radau2")
    for z in [-0.1, -1.0, -10.0, -1e3, 0.5]:
        R_tab = 1 + z * b @ np.linalg.solve(np.eye(2) - z * A, np.ones(2))
        assert R_tab == pytest.approx(_R_radau2(z), rel=1e-13)
    for z in [1e-2, 2e-2]:
        assert abs(_R_radau2(-z) - math.exp(-z)) < 0.05 * z ** 4  # error constant 1/72
    assert abs(_R_radau2(-1e9)) < 1e-8


@pytest.mark.parametrize("method", ["radau2", "sdirk2", "ie"])
def test_rk_linear_eigenvector_decay(method):
    # Pi sin(pi x_d) is an exact eigenvector of the Dirichlet FV Laplacian (lambda in closed form),
    # so the discrete solution decays exactly as R(-tau lambda)^n.
    n, tau, steps = (10, 12), 3e-3, 5
    K, b = fv.assemble_linear(n)
    u0 = inputs.sin_product(n)
    lam = sum(4 * m * m * math.sin(math.pi / (2 * m)) ** 2 for m in n)
    g = 1 - 1 / math.sqrt(2)
    R = {"radau2": _R_radau2, "ie": lambda z: 1 / (1 - z),
         "sdirk2": lambda z: (1 + (1 - 2 * g) * z) / (1 - g * z) ** 2}[method]
    ys, st = stepping.rk_linear(K, b, u0, tau, method, steps)
    for s in range(steps + 1):
        np.testing.assert_allclose(ys[s], R(-tau * lam) ** s * u0, rtol=0, atol=1e-12)
    if method == "radau2":
        # the first stage: amplitude of the stage system (I - z A)^{-1} 1 at the exact eigenvalue
        A, _, _ = tc.tableau("radau2")
        z = -tau * lam
        stage_amp = np.linalg.solve(np.eye(2) - z * A, np.ones(2))
        np.testing.assert_allclose(st[0][0], stage_amp[0] * u0, rtol=0, atol=1e-12)


@pytest.mark.parametrize("method", ["ie", "sdirk2", "theta"])
def test_rk_linear_equals_stagewise_dirk(method):
    # For a lower-triangular tableau the coupled solve equals stage-by-stage substitution (the theta
    # method keeps its explicit first stage here as an ordinary stage with y_1 = y^n).
    n = (5, 6)
    kap = inputs.lognormal_field(n, 0.0, 1.0, 1.5, 4)
    K, b = fv.assemble_linear(n, kappa=kap, velocity=(1.0, 0.5), bc={"default": ("dirichlet", 0.2)})
    y0 = inputs.smooth_random(n, 5)
    ys_c, _ = stepping.rk_linear(K, b, y0, 0.02, method, 4)
    ys_s, _ = stepping.dirk_linear(K, b, y0, 0.02, method, 4, theta=0.5)
    for a_, b_ in zip(ys_c, ys_s):
        np.testing.assert_allclose(a_, b_, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("s", [1, 2, 3])
def test_radau2_allatonce_equals_sequential(s):
    # s steps of Radau IIA stacked (eq. time-stepping-matrices-multiple-parallel-time-steps with a
    # full 2 x 2 diagonal block): the brute-force dense Kronecker solve equals sequential stepping.
    n = (4, 4)
    kap = inputs.lognormal_field(n, 0.0, 1.0, 1.0, 11)
    K, b = fv.assemble_linear(n, kappa=kap, velocity=(1.0, -0.5), bc={"default": ("dirichlet", 0.4)})
    N = K.shape[0]
    tau = 0.03
    y0 = inputs.smooth_random(n, 7)
    A, _, c = tc.tableau("radau2")
    A1, A2 = tc.time_stepping_matrices(A, c, s, tau)
    k = A1.shape[0]
    assert A2[0, 1] == pytest.approx(-1.0 / 12.0)  # upper entry inside the step block
    B = np.tile(b[:, None], (1, k))
    B0 = tc.window_b0(A, c, k, 0, tau, y0, K @ y0 - b, [])
    assert np.abs(B0[:, :2] - y0[:, None] / tau).max() < 1e-12 and not B0[:, 2:].any()
    Y = aao.solve_dense(sp.identity(N), K, A1, A2, B, B0)
    ys, st = stepping.rk_linear(K, b, y0, tau, "radau2", s)
    seq = np.column_stack([v for step in st for v in step])
    np.testing.assert_allclose(Y, seq, rtol=1e-12, atol=1e-12)


def test_averaged_beta():
    A, _, _ = tc.tableau("radau2")
    assert tc.averaged_beta(A) == pytest.approx(math.sqrt(1.0 / 6.0), rel=1e-15)
    # for a uniform diagonal DIRK the geometric mean is the diagonal itself
    g = 1 - 1 / math.sqrt(2)
    assert tc.averaged_beta(tc.tableau("sdirk2")[0]) == pytest.approx(g, rel=1e-14)


def test_averaged_splitting_converges_but_is_not_nilpotent():
    # With a full tableau block the splitting remainder is not strictly lower triangular: after k
    # sweeps the error is still far from zero, but the iteration contracts.  In the stiff limit a
    # mode with eigenvalue mu of A is damped by |1 - mu/beta| per sweep (0.606 for Radau IIA with
    # the averaged beta), which bounds the observed asymptotic rate.
    n = (6, 6)
    K, b = fv.assemble_linear(n, kappa=inputs.lognormal_field(n, 0.0, 1.0, 1.5, 3))
    N = K.shape[0]
    tau = 0.05
    y0 = inputs.smooth_random(n, 2)
    A, _, c = tc.tableau("radau2")
    s = 2
    A1, A2 = tc.time_stepping_matrices(A, c, s, tau)
    k = A1.shape[0]
    beta = tc.averaged_beta(A)
    B = np.tile(b[:, None], (1, k))
    B0 = tc.window_b0(A, c, k, 0, tau, y0, K @ y0 - b, [])
    Yex = aao.solve_dense(sp.identity(N), K, A1, A2, B, B0)
    Y = np.tile(y0[:, None], (1, k))
    errs = []
    for _ in range(80):
        Y = aao.splitting_sweep(sp.identity(N), K, A1, A2, tau, beta, Y, B, B0)
        errs.append(np.abs(Y - Yex).max())
    assert errs[k - 1] > 1e-4 * errs[0]
    assert errs[-1] < 1e-10 * np.abs(Yex).max()
    mu = np.linalg.eigvals(A)
    bound = max(abs(1 - mu / beta))
    assert bound == pytest.approx(0.6058, abs=1e-3)
    rate = (errs[39] / errs[19]) ** (1 / 20)  # before the rounding floor
    assert 0.5 < rate <= bound + 1e-3
