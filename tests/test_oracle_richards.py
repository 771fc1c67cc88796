"""Pins of the Richards oracle (Sec. 4.3, eq. RelationshipsThetaK) against facts fixed by the paper
and by the physics: closed forms of the van Genuchten closure, the Lipschitz constant the paper
prints for its silt-loam soil, flow invariants of the discrete operator (hydrostatic rest, unit
gradient drainage, steady infiltration, conservation), finite-difference derivatives, and a
root-finder check of the implicit Euler step."""
import numpy as np
import pytest
import scipy.optimize as so
import scipy.sparse as sp

from oracle import richards as ri
from oracle import timecoupling as otc
from paper_2504_02117_amd import inputs

VG = ri.VanGenuchten(theta_r=0.05, theta_s=0.4, alpha=2.0, n=2.0)
# silt loam of the paper's benchmark table
SILT = ri.VanGenuchten(theta_r=0.131, theta_s=0.396, alpha=0.423, n=2.06)


def test_theta_closed_forms():
    for vg in (VG, SILT):
        assert vg.theta(np.array([0.0]))[0] == vg.ts
        np.testing.assert_array_equal(vg.theta(np.array([0.3, 5.0])), [vg.ts, vg.ts])
        assert abs(vg.theta(np.array([-1e9]))[0] - vg.tr) < 1e-6
        # (alpha |psi|)^n = 1: Se = 2^(-m)
        psi = -1.0 / vg.alpha
        m = 1.0 - 1.0 / vg.n
        assert abs(vg.theta(np.array([psi]))[0] - (vg.tr + (vg.ts - vg.tr) * 2.0 ** (-m))) < 1e-15
    # alpha = 2, n = 2 (m = 1/2): theta(-1) = 0.05 + 0.35 / sqrt(5)
    assert abs(VG.theta(np.array([-1.0]))[0] - (0.05 + 0.35 / np.sqrt(5.0))) < 1e-15


def test_conductivity_closed_forms():
    for vg in (VG, SILT):
        assert abs(vg.kr(np.array([0.0]))[0] - 1.0) < 1e-15  # K(0) = Ks
        # with s = theta / theta_s as printed, the dry limit is s_r = theta_r / theta_s, not 0
        sr = vg.tr / vg.ts
        dry = np.sqrt(sr) * (1.0 - (1.0 - sr ** (1.0 / vg.m)) ** vg.m) ** 2
        assert abs(vg.kr(np.array([-1e9]))[0] - dry) < 1e-9
    # alpha = 2, n = 2, psi = -1: s = theta/theta_s, K/Ks = s^(1/2) (1 - (1 - s^2)^(1/2))^2
    s = (0.05 + 0.35 / np.sqrt(5.0)) / 0.4
    want = np.sqrt(s) * (1.0 - np.sqrt(1.0 - s * s)) ** 2
    assert abs(VG.kr(np.array([-1.0]))[0] - want) < 1e-15


def test_closure_monotone():
    psi = -np.logspace(-4, 3, 4000)[::-1]  # increasing from -1e3 to -1e-4
    for vg in (VG, SILT):
        assert np.all(np.diff(vg.theta(psi)) > 0)
        assert np.all(np.diff(vg.kr(psi)) > 0)
        assert np.all(vg.dtheta(psi) > 0) and np.all(vg.dkr(psi) > 0)


def test_silt_loam_lipschitz_constant_matches_paper():
    """The paper's L-scheme constant for its silt loam is the Lipschitz constant of theta, printed
    as 4.501e-2.  Its maximiser has the closed form (alpha |psi|)^n = m (m = 1 - 1/n)."""
    vg = SILT
    m, n, a = vg.m, vg.n, vg.alpha
    astar = m ** (1.0 / n)
    closed = (vg.ts - vg.tr) * a * m * n * astar ** (n - 1.0) * (1.0 + astar ** n) ** (-m - 1.0)
    got = vg.dtheta(np.array([-astar / a]))[0]
    assert abs(got - closed) < 1e-15
    assert abs(got - 4.501e-2) < 5e-6
    grid = -np.logspace(-4, 3, 200001)
    assert vg.dtheta(grid).max() <= got * (1 + 1e-12)


@pytest.mark.parametrize("vg", [VG, SILT])
def test_derivatives_match_finite_differences(vg):
    psi = np.concatenate([-np.logspace(-2, 1.5, 60), [-0.7, -3.3]])
    h = 1e-6 * np.maximum(1.0, np.abs(psi))
    fd_t = (vg.theta(psi + h) - vg.theta(psi - h)) / (2 * h)
    fd_k = (vg.kr(psi + h) - vg.kr(psi - h)) / (2 * h)
    np.testing.assert_allclose(vg.dtheta(psi), fd_t, rtol=1e-6, atol=1e-12)
    np.testing.assert_allclose(vg.dkr(psi), fd_k, rtol=1e-5, atol=1e-12)
    # saturated side: no change
    np.testing.assert_array_equal(vg.dtheta(np.array([0.0, 0.5])), [0.0, 0.0])
    np.testing.assert_array_equal(vg.dkr(np.array([0.0, 0.5])), [0.0, 0.0])


def _ks(n, seed=7):
    return inputs.lognormal_field(n, 0.0, 1.5, 3.0, seed).ravel()


@pytest.mark.parametrize("n", [(12,), (9, 7), (6, 5, 8)])
def test_hydrostatic_state_is_at_rest(n):
    """psi = c - z gives a constant total head: with no-flow faces F = 0 for any Ks field."""
    model = ri.Richards(n, _ks(n), VG, top=("none",), bottom="none")
    for c in (-2.0, 0.4):
        psi = c - model.z
        assert np.abs(model.f(psi)).max() < 1e-12


@pytest.mark.parametrize("n", [(10,), (6, 9), (4, 5, 7)])
def test_uniform_head_drains_with_unit_gradient(n):
    """Uniform psi with homogeneous Ks: every vertical face carries Ks kr / h downwards.  With a
    no-flow top and a free-drainage bottom only the top layer loses water, at Ks kr / h_z."""
    g_ks = 0.7
    model = ri.Richards(n, g_ks, VG, top=("none",), bottom="free_drainage")
    psi = np.full(model.grid.N, -0.8)
    F = model.f(psi)
    top = model.grid.boundary_cells(len(n) - 1, 1)
    want = np.zeros_like(F)
    want[top] = g_ks * VG.kr(np.array([-0.8]))[0] * n[-1]
    assert np.abs(F - want).max() < 1e-12


@pytest.mark.parametrize("n", [(11,), (5, 8), (3, 4, 9)])
def test_steady_infiltration_at_top_value(n):
    """Top Dirichlet g, free-drainage bottom, psi = g everywhere and Ks varying only laterally:
    a steady unit-gradient flow, F = 0."""
    N = int(np.prod(n))
    shape = inputs.field_shape(n)  # z is the slowest axis
    lat = np.linspace(0.5, 2.0, N // n[-1]).reshape(shape[1:])
    ks = np.broadcast_to(lat[None], shape)
    for g in (-1.2, 0.0, 0.3):
        model = ri.Richards(n, ks.ravel(), VG, top=("dirichlet", g), bottom="free_drainage")
        assert np.abs(model.f(np.full(N, g))).max() < 1e-12 * max(1.0, n[-1])


def test_layered_saturated_column_matches_darcy():
    """Saturated (kr = 1) steady downward flux q through a layered column: integrating Darcy's law
    dH/dz = q / Ks(z) cell by cell from the top face gives heads at the cell centres on which F
    vanishes except in the bottom cell (no-flow bottom), where the inflow q accumulates: F = -q/h.
    Exact for piecewise-constant Ks because the face conductance is the series (harmonic) one."""
    nz = 9
    ks = np.array([0.3, 2.0, 0.8, 5.0, 1.0, 0.05, 0.7, 3.0, 1.4])
    h = 1.0 / nz
    g, q = 6.0, 0.02
    zc = (np.arange(nz) + 0.5) * h
    H = np.empty(nz)
    H[-1] = (g + 1.0) - q * (h / 2) / ks[-1]
    for i in range(nz - 2, -1, -1):
        H[i] = H[i + 1] - q * (h / 2) * (1.0 / ks[i + 1] + 1.0 / ks[i])
    psi = H - zc
    assert psi.min() > 0.0
    model = ri.Richards((nz,), ks, VG, top=("dirichlet", g), bottom="none")
    F = model.f(psi)
    want = np.zeros(nz)
    want[0] = -q / h
    assert np.abs(F - want).max() < 1e-12


def test_no_flow_conserves_mass():
    n = (5, 6, 7)
    model = ri.Richards(n, _ks(n), VG, top=("none",), bottom="none")
    psi = -np.abs(inputs.smooth_random(n, 3)) * 2.0 - 0.1
    assert abs(model.f(psi).sum()) < 1e-11 * np.abs(model.f(psi)).max()
    # implicit Euler keeps sum(theta) up to the Newton tolerance
    out, _ = ri.implicit_euler(model, psi, 1e-3, 3)
    tot = [model.theta(p).sum() for p in out]
    assert max(abs(t - tot[0]) for t in tot) < 1e-10 * tot[0]


def test_boundary_fluxes_balance():
    """sum(F) over the cells equals the net outflow through the top and bottom faces."""
    n = (4, 5, 6)
    model = ri.Richards(n, _ks(n), VG, top=("dirichlet", -0.1), bottom="free_drainage")
    psi = -np.abs(inputs.smooth_random(n, 8)) - 0.2
    F = model.f(psi)
    hz = 1.0 / n[-1]
    top = model.grid.boundary_cells(2, 1)
    bot = model.grid.boundary_cells(2, 0)
    kr = VG.kr(psi)
    krg = VG.kr(np.array([-0.1]))[0]
    H = psi + model.z
    out_top = (2.0 * model.ks[top] * 0.5 * (kr[top] + krg) * (H[top] - (-0.1 + 1.0)) / hz ** 2).sum()
    out_bot = (model.ks[bot] * kr[bot] / hz).sum()
    assert abs(F.sum() - (out_top + out_bot)) < 1e-10 * np.abs(F).sum()


@pytest.mark.parametrize("top,bottom", [(("dirichlet", 0.0), "free_drainage"), (("none",), "none")])
def test_jacobian_matches_finite_differences(top, bottom):
    n = (4, 3, 5)
    model = ri.Richards(n, _ks(n, 2), VG, top=top, bottom=bottom)
    psi = -np.abs(inputs.smooth_random(n, 1)) * 1.5 - 0.05
    psi[::7] = 0.2  # a few saturated cells
    J = model.jac(psi).toarray()
    N = psi.size
    fd = np.empty((N, N))
    for j in range(N):
        h = 1e-6
        e = np.zeros(N)
        e[j] = h
        fd[:, j] = (model.f(psi + e) - model.f(psi - e)) / (2 * h)
    assert np.abs(J - fd).max() < 1e-6 * np.abs(J).max()


def test_implicit_euler_step_is_a_root():
    """The Newton/direct IE step agrees with an independent root finder on a small column."""
    n = (8,)
    model = ri.Richards(n, np.linspace(0.5, 1.5, 8), VG, top=("dirichlet", 0.0), bottom="free_drainage")
    psi0 = np.full(8, -1.0)
    tau = 5e-3
    out, its = ri.implicit_euler(model, psi0, tau, 1)
    th0 = model.theta(psi0)
    root = so.fsolve(lambda x: (model.theta(x) - th0) / tau + model.f(x), psi0, xtol=1e-12)
    assert np.abs(out[1] - root).max() < 1e-10
    assert its[0] >= 2


def test_window_residual_vanishes_on_sequential_solution():
    """theta(Y) A1^T + F(Y) A2^T - B0 is zero on the implicit Euler trajectory (IE windows)."""
    n = (3, 4, 5)
    model = ri.Richards(n, _ks(n), VG, top=("dirichlet", 0.0), bottom="free_drainage")
    psi0 = -np.abs(inputs.smooth_random(n, 6)) - 0.3
    tau, k = 2e-3, 4
    out, _ = ri.implicit_euler(model, psi0, tau, k)
    A, _, c = otc.tableau("ie")
    A1, A2, _ = otc.window_matrices(A, c, k, 0, tau)
    B0 = otc.window_b0(A, c, k, 0, tau, model.theta(psi0), model.f(psi0), [])
    Y = np.column_stack(out[1:])
    R = ri.window_residual(model, A1, A2, Y, B0)
    assert np.abs(R).max() < 1e-9 * np.abs(model.theta(psi0) / tau).max()
    # and not on a perturbed window
    Y2 = Y.copy()
    Y2[:, 2] += 1e-3
    assert np.abs(ri.window_residual(model, A1, A2, Y2, B0)).max() > 1e-3
