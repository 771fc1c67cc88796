"""Pins for the oracle's nonlinear diffusion-reaction operator and Newton stepping."""
import math

import numpy as np
import pytest

from oracle import fv, stepping
from paper_2504_02117_amd import inputs


@pytest.mark.parametrize("bc", [None, {"default": ("dirichlet", 0.25)}])
def test_jacobian_matches_finite_differences(bc):
    n = (5, 4)
    op = fv.NonlinearDiffusionReaction(n, dcoef=(1.0, 0.3, 1.0), rcoef=(0.1, -0.2, 0.0, -1.0), bc=bc)
    u = inputs.smooth_random(n, 1)
    J = op.jac(u).toarray()
    eps = 1e-6
    Jfd = np.empty_like(J)
    for j in range(u.size):
        e = np.zeros_like(u)
        e[j] = eps
        Jfd[:, j] = (op.f(u + e) - op.f(u - e)) / (2 * eps)
    np.testing.assert_allclose(J, Jfd, rtol=0, atol=1e-6 * np.abs(J).max())


def test_f_linear_limit_matches_linear_assembly():
    # D == 1 and r == 0 reduce f to the constant-coefficient Laplacian K u.
    n = (6, 5)
    op = fv.NonlinearDiffusionReaction(n, dcoef=(1.0,), rcoef=(0.0,), bc={"default": ("dirichlet", 0.0)})
    K, b = fv.assemble_linear(n)
    u = inputs.smooth_random(n, 2)
    np.testing.assert_allclose(op.f(u), K @ u - b, rtol=1e-13, atol=1e-10)


def _scalar_stage(known, a, tau):
    # a y^3 + y/tau + known = 0, unique real root (monotone cubic)
    roots = np.roots([a, 0.0, 1.0 / tau, known])
    real = roots[np.abs(roots.imag) < 1e-9].real
    assert real.size == 1
    return real[0]


def test_constant_state_reduces_to_scalar_ode():
    # Zero-flux boundaries and a spatially constant state: f(u) = u^3 (r = -u^3), so each SDIRK2
    # stage is a scalar cubic, solved here by polynomial roots.
    n = (4, 4)
    op = fv.NonlinearDiffusionReaction(n)
    tau, u0, steps = 0.05, 0.8, 10
    ys, _, _ = stepping.dirk_nonlinear(op, np.full(16, u0), tau, "sdirk2", steps)
    g = 1 - 1 / math.sqrt(2)
    y = u0
    for s in range(steps):
        y1 = _scalar_stage(-y / tau, g, tau)
        y2 = _scalar_stage(-y / tau + (1 - g) * y1 ** 3, g, tau)
        y = y2
        np.testing.assert_allclose(ys[s + 1], y, rtol=5e-12)  # stage Newton stops at 1e-12 relative


def test_second_order_in_time():
    op = fv.NonlinearDiffusionReaction((2, 2))
    u0, T = 0.9, 0.4
    exact = u0 / math.sqrt(1 + 2 * u0 ** 2 * T)
    errs = []
    for steps in (10, 20, 40):
        ys, _, _ = stepping.dirk_nonlinear(op, np.full(4, u0), T / steps, "sdirk2", steps)
        errs.append(abs(ys[-1][0] - exact))
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5


def test_zero_flux_diffusion_conserves_mass():
    n = (6, 6)
    op = fv.NonlinearDiffusionReaction(n, rcoef=(0.0,))
    u0 = inputs.smooth_random(n, 5)
    ys, _, iters = stepping.dirk_nonlinear(op, u0, 1e-3, "sdirk2", 4)
    assert abs(ys[-1].sum() - u0.sum()) < 1e-11 * u0.sum()
    assert all(i >= 2 for i in iters)
