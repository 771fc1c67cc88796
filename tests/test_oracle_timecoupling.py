"""Pins for the oracle's time coupling (Sec. 2.1, Example 2; Sec. 2.2 pipelining)."""
import math
import os

import numpy as np
import pytest

from oracle import timecoupling as tc

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "example2_theta.txt")


def _read_golden():
    mats, name, rows = {}, None, []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if line[0].isalpha():
            if name:
                mats[name] = np.array(rows, dtype=float)
            name, rows = line, []
        else:
            rows.append([float(v) for v in line.split()])
    mats[name] = np.array(rows, dtype=float)
    return mats


@pytest.mark.parametrize("theta", [0.5, 0.3])
def test_example2_theta_matrices(theta):
    g = _read_golden()
    A, b, c = tc.tableau("theta", theta)
    A1, A2 = tc.time_stepping_matrices(A, c, s=4, tau=0.25)
    np.testing.assert_allclose(A1, g[f"A1 theta={theta}"], rtol=0, atol=1e-15)
    np.testing.assert_allclose(A2, g[f"A2 theta={theta}"], rtol=0, atol=1e-15)


@pytest.mark.parametrize("theta", [1.0, 0.5])
def test_example2_theta_b0(theta):
    rng = np.random.default_rng(1)
    N, tau = 7, 0.1
    My, Ky, bn = rng.standard_normal((3, N))
    A, b, c = tc.tableau("theta", theta)
    B0 = tc.window_b0(A, c, k=4, phase=0, tau=tau, My_n=My, f_yn=Ky - bn, f_stages=[])
    np.testing.assert_allclose(B0[:, 0], My / tau - (1 - theta) * (Ky - bn), rtol=1e-15, atol=1e-15)
    assert not B0[:, 1:].any()


def test_single_step_theta_is_example1():
    # s = 1 reduces the all-at-once system to (M/tau + theta K) y^{n+1} = theta b + M y^n/tau + (1-theta)(b - K y^n).
    A, b, c = tc.tableau("theta", 0.7)
    A1, A2 = tc.time_stepping_matrices(A, c, s=1, tau=0.2)
    assert A1.shape == (1, 1) and A1[0, 0] == pytest.approx(5.0) and A2[0, 0] == pytest.approx(0.7)


@pytest.mark.parametrize("name", ["ie", "theta", "sdirk2"])
def test_tableaux_stiffly_accurate(name):
    A, b, c = tc.tableau(name)
    assert tc.is_stiffly_accurate(A, b)
    np.testing.assert_allclose(A.sum(1), c, atol=1e-15)  # row-sum condition c_i = sum_j a_ij


def test_sdirk2_order_and_l_stability():
    # Stability function from the tableau must match the closed form (1+(1-2g)z)/(1-gz)^2,
    # agree with exp(z) to second order and vanish at infinity.
    A, b, c = tc.tableau("sdirk2")
    g = 1 - 1 / math.sqrt(2)
    for z in [-0.1, -1.0, -10.0, -1e3]:
        R_tab = 1 + z * b @ np.linalg.solve(np.eye(2) - z * A, np.ones(2))
        R_closed = (1 + (1 - 2 * g) * z) / (1 - g * z) ** 2
        assert R_tab == pytest.approx(R_closed, rel=1e-13)
    z = 1e-3
    R = (1 + (1 - 2 * g) * z) / (1 - g * z) ** 2
    assert abs(R - math.exp(z)) < 1e-9 * 1.0  # local error O(z^3)
    assert abs((1 + (1 - 2 * g) * 1e8) / (1 - g * 1e8) ** 2) < 1e-7


def test_sdirk2_multi_step_structure():
    # eq. time-stepping-matrices-multiple-parallel-time-steps for m = 2, s = 3:
    # A1 couples both stages of step j+1 to the last stage of step j; A2 is block diagonal.
    A, b, c = tc.tableau("sdirk2")
    tau = 0.5
    A1, A2 = tc.time_stepping_matrices(A, c, s=3, tau=tau)
    expect_A1 = np.eye(6) / tau
    for r in (2, 3):
        expect_A1[r, 1] = -1 / tau
    for r in (4, 5):
        expect_A1[r, 3] = -1 / tau
    np.testing.assert_array_equal(A1, expect_A1)
    expect_A2 = np.zeros((6, 6))
    for j in range(3):
        expect_A2[2 * j:2 * j + 2, 2 * j:2 * j + 2] = A
    np.testing.assert_array_equal(A2, expect_A2)


def test_splitting_parts_strictly_lower():
    # The splitting of eq. matrix-splitting leaves strictly lower-triangular remainders for IE, theta, SDIRK2.
    for name in ["ie", "theta", "sdirk2"]:
        A, b, c = tc.tableau(name)
        for phase in range(tc.implicit_part(A, c)[0].shape[0]):
            A1, A2, beta = tc.window_matrices(A, c, k=5, phase=phase, tau=0.3)
            assert not np.triu(A1 - np.eye(5) / 0.3).any()
            assert not np.triu(A2 - beta * np.eye(5)).any()
