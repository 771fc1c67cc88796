"""Pins for the all-at-once formulation (Sec. 2.1, 2.2): Kronecker identity, equivalence with
sequential stepping, pipelined-window residuals and the nilpotent splitting."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import allatonce as aao
from oracle import fv, stepping
from oracle import timecoupling as tc
from paper_2504_02117_amd import inputs


def _problem(n=(4, 4), g=0.4):
    kap = inputs.lognormal_field(n, 0.0, 1.0, 1.0, 11)
    K, b = fv.assemble_linear(n, kappa=kap, velocity=(1.0, -0.5), bc={"default": ("dirichlet", g)})
    return K, b


def test_kronecker_identity_orientation():
    # (C (x) A) vec X = vec(A X C^T): the matrix residual must equal the Kronecker form.
    rng = np.random.default_rng(0)
    N, k = 5, 3
    M = np.diag(rng.uniform(1, 2, N))
    K = rng.standard_normal((N, N))
    A1, A2 = rng.standard_normal((2, k, k))
    Y, B, B0 = rng.standard_normal((3, N, k))
    R = aao.residual_linear(M, K, A1, A2, Y, B, B0)
    r_kron = aao.kron_operator(M, K, A1, A2) @ aao.vec(Y) - np.kron(A2, np.eye(N)) @ aao.vec(B) - aao.vec(B0)
    np.testing.assert_allclose(aao.vec(R), r_kron, rtol=1e-13, atol=1e-13)
    # a transposed coupling would not match
    R_bad = M @ Y @ A1 + (K @ Y - B) @ A2 - B0
    assert np.abs(aao.vec(R_bad) - r_kron).max() > 1e-3


@pytest.mark.parametrize("method,theta", [("ie", 1.0), ("theta", 0.5), ("theta", 1.0), ("sdirk2", 0.5)])
@pytest.mark.parametrize("s", [1, 2, 4])
def test_allatonce_equals_sequential(method, theta, s):
    K, b = _problem()
    N = K.shape[0]
    tau = 0.03
    y0 = inputs.smooth_random((4, 4), 7)
    A, _, c = tc.tableau(method, theta)
    A1, A2 = tc.time_stepping_matrices(A, c, s, tau)
    k = A1.shape[0]
    B = np.tile(b[:, None], (1, k))
    B0 = tc.window_b0(A, c, k, 0, tau, y0, K @ y0 - b, [])
    Y = aao.solve_dense(sp.identity(N), K, A1, A2, B, B0)
    ys, st = stepping.dirk_linear(K, b, y0, tau, method, s, theta=theta)
    seq = np.column_stack([v for step in st for v in step])
    np.testing.assert_allclose(Y, seq, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(Y[:, -1], ys[-1], rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("method,theta", [("ie", 1.0), ("sdirk2", 0.5)])
@pytest.mark.parametrize("s", [1, 3])
def test_sparse_allatonce_solve_equals_sequential(method, theta, s):
    """The sparse direct solve of the window system reproduces sequential stepping."""
    n = (6, 5, 4)
    kap = inputs.lognormal_field(n, 0.0, 1.0, 1.5, 12)
    K, b = fv.assemble_linear(n, kappa=kap, velocity=(0.5, 0.0, -1.0), bc={"default": ("dirichlet", 0.3)})
    N = K.shape[0]
    tau = 0.02
    y0 = inputs.smooth_random(n, 8)
    A, _, c = tc.tableau(method, theta)
    A1, A2 = tc.time_stepping_matrices(A, c, s, tau)
    k = A1.shape[0]
    B = np.tile(b[:, None], (1, k))
    B0 = tc.window_b0(A, c, k, 0, tau, y0, K @ y0 - b, [])
    Y = aao.solve_sparse(sp.identity(N), K, A1, A2, B, B0)
    _, st = stepping.dirk_linear(K, b, y0, tau, method, s, theta=theta)
    seq = np.column_stack([v for step in st for v in step])
    np.testing.assert_allclose(Y, seq, rtol=1e-11, atol=1e-11)


@pytest.mark.parametrize("method", ["ie", "theta", "sdirk2"])
@pytest.mark.parametrize("k", [1, 3, 4])
def test_pipelined_window_residual_vanishes(method, k):
    # Window starting at any implicit stage of step 1: stacking the sequential stages that follow
    # makes the residual M Y A1^T + (K Y - B) A2^T - B0 vanish.
    K, b = _problem()
    N = K.shape[0]
    tau = 0.05
    y0 = inputs.smooth_random((4, 4), 3)
    A, _, c = tc.tableau(method, 0.5)
    mi = tc.implicit_part(A, c)[0].shape[0]
    ys, st = stepping.dirk_linear(K, b, y0, tau, method, 6, theta=0.5)
    flat = [(n, q, v) for n, step in enumerate(st) for q, v in enumerate(step)]
    for phase in range(mi):
        start = mi + phase  # front column: stage `phase` of step index 1
        Y = np.column_stack([flat[start + i][2] for i in range(k)])
        A1, A2, beta = tc.window_matrices(A, c, k, phase, tau)
        yn = ys[1]
        f_st = [K @ st[1][j] - b for j in range(phase)]
        B0 = tc.window_b0(A, c, k, phase, tau, yn, K @ yn - b, f_st)
        R = aao.residual_linear(sp.identity(N), K, A1, A2, Y, np.tile(b[:, None], (1, k)), B0)
        assert np.abs(R).max() < 1e-10 * np.abs(yn).max() / tau
        assert beta == pytest.approx(tc.implicit_part(A, c)[0][phase, phase])


@pytest.mark.parametrize("method", ["ie", "theta", "sdirk2"])
def test_splitting_is_nilpotent(method):
    # Exact inner solves: the fixed point of eq. matrix-fixed-point-equation reaches the all-at-once
    # solution after exactly k sweeps (strictly lower-triangular remainders), not before.
    K, b = _problem()
    N = K.shape[0]
    tau = 0.05
    y0 = inputs.smooth_random((4, 4), 9)
    A, _, c = tc.tableau(method, 0.5)
    A1, A2, beta = tc.window_matrices(A, c, 4, 0, tau)
    B = np.tile(b[:, None], (1, 4))
    B0 = tc.window_b0(A, c, 4, 0, tau, y0, K @ y0 - b, [])
    Yex = aao.solve_dense(sp.identity(N), K, A1, A2, B, B0)
    Y = np.tile(y0[:, None], (1, 4))
    errs = []
    for _ in range(4):
        Y = aao.splitting_sweep(sp.identity(N), K, A1, A2, tau, beta, Y, B, B0)
        errs.append(np.abs(Y - Yex).max())
    assert errs[-1] < 1e-12
    assert errs[-2] > 1e-9
    # and the Newton form of Algorithm 1 (Y - J^{-1} R) is the same sweep in the linear case
    Y0 = np.tile(y0[:, None], (1, 4))
    R = aao.residual_linear(sp.identity(N), K, A1, A2, Y0, B, B0)
    J = (sp.identity(N) / tau + beta * K).tocsc()
    V = np.column_stack([stepping.linear_solve(J, R[:, j]) for j in range(4)])
    Ysw = aao.splitting_sweep(sp.identity(N), K, A1, A2, tau, beta, Y0, B, B0)
    np.testing.assert_allclose(Y0 - V, Ysw, rtol=1e-11, atol=1e-11)


def test_nonlinear_window_residual_vanishes():
    n = (5, 4)
    op = fv.NonlinearDiffusionReaction(n)
    tau = 0.01
    y0 = inputs.smooth_random(n, 4)
    A, _, c = tc.tableau("sdirk2")
    ys, st, _ = stepping.dirk_nonlinear(op, y0, tau, "sdirk2", 3)
    N = y0.size
    for phase in (0, 1):
        k = 3
        flat = [v for step in st for v in step]
        Y = np.column_stack(flat[2 + phase:2 + phase + k])
        A1, A2, _ = tc.window_matrices(A, c, k, phase, tau)
        f_st = [op.f(st[1][j]) for j in range(phase)]
        B0 = tc.window_b0(A, c, k, phase, tau, ys[1], op.f(ys[1]), f_st)
        R = aao.residual_nonlinear(sp.identity(N), lambda j, y: op.f(y), A1, A2, Y, B0)
        assert np.abs(R).max() < 1e-9 * np.abs(ys[1]).max() / tau
