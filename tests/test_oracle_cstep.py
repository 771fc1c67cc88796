"""Pins for the C form of the oracle's sequential implicit Euler (oracle/seqstep.c).

Each test checks it against something outside the C code: the closed-form decay of the exact
discrete eigenvector, a sparse LU solve of every step (scipy), and the scipy CG form of the oracle.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import cstep, fv, stepping
from paper_2504_02117_amd import inputs


def test_eigenvector_decay_closed_form():
    # Pi sin(pi x_d) is an exact eigenvector of the Dirichlet FV Laplacian with
    # lambda = sum_d 4 n_d^2 sin^2(pi / (2 n_d)); implicit Euler multiplies it by 1 / (1 + tau lambda).
    n, tau, steps = (10, 9, 8), 3e-3, 5
    K, b = fv.assemble_linear(n)
    u0 = inputs.sin_product(n)
    lam = sum(4 * m * m * math.sin(math.pi / (2 * m)) ** 2 for m in n)
    ys, its, _ = cstep.ie_steps(K, b, u0, tau, steps, rtol=1e-14, threads=2)
    for s in range(steps + 1):
        np.testing.assert_allclose(ys[s], u0 / (1 + tau * lam) ** s, rtol=0, atol=1e-12)
    assert all(i >= 0 for i in its)


@pytest.mark.parametrize("n", [(23, 17), (9, 11, 7)])
def test_matches_sparse_lu_per_step(n):
    # heterogeneous coefficient, nonzero Dirichlet data (b != 0): each step against a direct solve
    kap = inputs.lognormal_field(n, 0.0, 2.0, 2.0, 5)
    bc = {"default": ("dirichlet", 0.0), (0, 0): ("dirichlet", 1.5), (1, 1): ("neumann",)}
    K, b = fv.assemble_linear(n, kappa=kap, bc=bc)
    assert b.any()
    tau, steps = 1e-3, 4
    u0 = inputs.smooth_random(n, 2)
    ys, _, _ = cstep.ie_steps(K, b, u0, tau, steps, rtol=1e-14)
    J = sp.csc_matrix(sp.identity(K.shape[0]) / tau + K)
    y = u0.copy()
    for s in range(steps):
        y = spla.spsolve(J, y / tau + b)
        assert np.linalg.norm(ys[s + 1] - y) <= 1e-12 * np.linalg.norm(y)


def test_thread_count_changes_only_rounding_and_matches_scipy_form():
    n = (20, 18, 16)
    kap = inputs.lognormal_field(n, 0.0, 2.0, 2.5, 1)
    K, b = fv.assemble_linear(n, kappa=kap)
    u0 = inputs.sin_product(n)
    y1, it1, used1 = cstep.ie_steps(K, b, u0, 1e-3, 3, rtol=1e-12, threads=1)
    y4, it4, used4 = cstep.ie_steps(K, b, u0, 1e-3, 3, rtol=1e-12, threads=4)
    assert used1 == 1 and used4 == 4
    ref, _ = stepping.dirk_linear(K, b, u0, 1e-3, "ie", 3)
    for s in range(1, 4):
        nr = np.linalg.norm(ref[s])
        assert np.linalg.norm(y1[s] - y4[s]) <= 1e-10 * nr
        assert np.linalg.norm(y1[s] - ref[s]) <= 1e-9 * nr


def test_residual_meets_tolerance_in_the_true_norm():
    n = (30, 30)
    kap = inputs.lognormal_field(n, 0.0, 2.0, 3.0, 7)
    K, b = fv.assemble_linear(n, kappa=kap)
    u0 = inputs.sin_product(n)
    tau = 1e-3
    for rtol in (1e-6, 1e-10):
        ys, _, _ = cstep.ie_steps(K, b, u0, tau, 2, rtol=rtol)
        J = sp.identity(K.shape[0]) / tau + K
        for s in range(2):
            rhs = ys[s] / tau + b
            assert np.linalg.norm(rhs - J @ ys[s + 1]) <= rtol * np.linalg.norm(rhs)
