"""Pins for the oracle's FV operators and sequential stepping."""
import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import fv, stepping
from paper_2504_02117_amd import inputs


def test_nnz_formula_and_symmetry():
    for n in [(8, 8), (6, 5, 4)]:
        K, b = fv.assemble_linear(n, kappa=inputs.lognormal_field(n, 0, 1, 1.5, 3))
        g = fv.Grid(n)
        faces = sum(g.N // g.n[d] * (g.n[d] - 1) for d in range(g.dim))
        assert K.nnz == g.N + 2 * faces
        assert abs(K - K.T).max() < 1e-12 * abs(K).max()
        assert not b.any()
        off = K - sp.diags(K.diagonal())
        assert off.max() <= 0 and K.diagonal().min() > 0


def test_config_sizes():
    # 128^3 7-point: N = 2 097 152, nnz = 7N - 6 n^2; 1024^2 5-point: nnz = 5N - 4n; 32^2: 4992.
    for n, dim in [(128, 3), (1024, 2), (32, 2)]:
        N = n ** dim
        nnz = (2 * dim + 1) * N - 2 * dim * n ** (dim - 1)
        assert {(128, 3): 14581760, (1024, 2): 5238784, (32, 2): 4992}[(n, dim)] == nnz
    K, _ = fv.assemble_linear((32, 32), velocity=(1.0, 0.5))
    assert K.nnz == 4992


@pytest.mark.parametrize("n", [(16, 16), (12, 10), (8, 8, 8), (6, 7, 5)])
def test_sin_product_is_exact_eigenvector(n):
    K, _ = fv.assemble_linear(n)
    u = inputs.sin_product(n)
    lam = sum(4 * m * m * math.sin(math.pi / (2 * m)) ** 2 for m in n)
    np.testing.assert_allclose(K @ u, lam * u, rtol=0, atol=1e-11 * lam)


def _R(method, z):
    g = 1 - 1 / math.sqrt(2)
    return {
        "ie": 1 / (1 - z),
        "theta": (1 + 0.5 * z) / (1 - 0.5 * z),
        "sdirk2": (1 + (1 - 2 * g) * z) / (1 - g * z) ** 2,
    }[method]


@pytest.mark.parametrize("method", ["ie", "theta", "sdirk2"])
@pytest.mark.parametrize("solver", ["direct", "cg"])
def test_eigenvector_decay(method, solver):
    n, tau, steps = (12, 12), 2e-3, 6
    K, b = fv.assemble_linear(n)
    u0 = inputs.sin_product(n)
    lam = sum(4 * m * m * math.sin(math.pi / (2 * m)) ** 2 for m in n)
    ys, _ = stepping.dirk_linear(K, b, u0, tau, method, steps, theta=0.5, solver=solver, rtol=1e-14)
    for s in range(steps + 1):
        np.testing.assert_allclose(ys[s], _R(method, -tau * lam) ** s * u0, rtol=0, atol=1e-12)


def test_harmonic_mean_series_resistance_1d():
    # Steady 1D diffusion through cells of piecewise-constant kappa: the FV solution with harmonic
    # faces equals the exact piecewise-linear solution (constant flux through resistances h/kappa).
    n = 9
    kap = np.exp(np.random.default_rng(0).standard_normal(n) * 1.5)
    g0, g1 = 2.0, -1.0
    K, b = fv.assemble_linear((n,), kappa=kap, bc={(0, 0): ("dirichlet", g0), (0, 1): ("dirichlet", g1)})
    u = spla.spsolve(K.tocsc(), b)
    h = 1.0 / n
    q = (g0 - g1) / np.sum(h / kap)
    exact = np.empty(n)
    exact[0] = g0 - q * h / (2 * kap[0])
    for i in range(n - 1):
        exact[i + 1] = exact[i] - q * (h / (2 * kap[i]) + h / (2 * kap[i + 1]))
    np.testing.assert_allclose(u, exact, rtol=1e-12, atol=1e-12)


def test_upwind_pure_convection_is_lower_triangular():
    n = (10, 9)
    K, b = fv.assemble_linear(n, kappa=0.0, velocity=(1.0, 0.5), bc={"default": ("dirichlet", 0.3)})
    assert abs(sp.triu(K, 1)).max() == 0  # stored zeros of the (vanishing) diffusion part allowed
    assert b.any()  # inflow faces x=0 and y=0 carry g
    tau = 0.05
    y0 = inputs.sin_product(n)
    J = (sp.identity(K.shape[0]) / tau + K).tocsr()
    rhs = y0 / tau + b
    x_fwd = spla.spsolve_triangular(J, rhs, lower=True)
    ys, _ = stepping.dirk_linear(K, b, y0, tau, "ie", 1)
    np.testing.assert_allclose(ys[1], x_fwd, rtol=1e-13, atol=1e-13)
    # outflow faces (x=1, y=1) carry no inflow term: b vanishes on cells touching only them
    g = fv.Grid(n)
    assert b[g.boundary_cells(0, 1)[1:]].tolist() == [0.0] * (n[1] - 1)


def test_convection_inflow_value():
    # one cell, velocity +x, inflow value g: IE step of u' + v(u - g)/h ... on a 1-cell grid
    K, b = fv.assemble_linear((1,), kappa=0.0, velocity=(2.0,), bc={"default": ("dirichlet", 3.0)})
    # flux in at x=0: -w g with w = -2 (outward normal -x) -> b = 2*3/h = 6 ; outflow at x=1: K = 2/h
    assert K.toarray()[0, 0] == pytest.approx(2.0) and b[0] == pytest.approx(6.0)


def test_neumann_conserves_mass_and_dirichlet_max_principle():
    n = (10, 8)
    kap = inputs.lognormal_field(n, 0, 1, 2, 5)
    u0 = inputs.smooth_random(n, 2)
    K, b = fv.assemble_linear(n, kappa=kap, bc={"default": ("neumann",)})
    ys, _ = stepping.dirk_linear(K, b, u0, 1e-2, "ie", 5)
    assert abs(ys[-1].sum() - u0.sum()) < 1e-11 * u0.sum()
    K, b = fv.assemble_linear(n, kappa=kap)
    ys, _ = stepping.dirk_linear(K, b, u0, 1e-2, "ie", 5)
    for y in ys:
        assert y.min() >= -1e-14 and y.max() <= u0.max() + 1e-14


@pytest.mark.parametrize("kind", ["cg", "gmres", "bicgstab"])
def test_iterative_solvers_match_direct(kind):
    n = (12, 11)
    K, b = fv.assemble_linear(n, kappa=inputs.lognormal_field(n, 0, 1, 2, 1),
                              velocity=None if kind == "cg" else (1.0, 0.5))
    J = (sp.identity(K.shape[0]) * 50 + K).tocsr()
    rhs = inputs.random_block(K.shape[0], 1, 3)[:, 0]
    x = stepping.linear_solve(J, rhs, kind=kind, rtol=1e-13)
    xd = stepping.linear_solve(J, rhs, kind="direct")
    np.testing.assert_allclose(x, xd, rtol=0, atol=1e-10 * abs(xd).max())
