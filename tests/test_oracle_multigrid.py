"""Pins for the oracle's multigrid V-cycle: Galerkin coarse operators (row sums, the uniform-coefficient
coarse stencil), and the cycle's symmetry, positive definiteness and contraction."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import fv, multigrid as mg
from paper_2504_02117_amd import inputs


def test_prolongation_counts_cells_once():
    for n in [(5, 4, 3), (7,), (6, 5), (1, 7, 9)]:
        P, cdims = mg.prolongation(n)
        assert P.shape == (int(np.prod(n)), int(np.prod(cdims)))
        np.testing.assert_array_equal(P.sum(axis=1).A.ravel(), 1.0)  # every fine cell in one aggregate
        assert P.sum() == np.prod(n)


def test_galerkin_row_sums_and_mass():
    # P^T K P 1 = P^T (K 1): the coarse row sums are the aggregate sums of the fine row sums, and the
    # coarse mass counts the fine cells of each aggregate
    n = (9, 8, 7)
    K, _ = fv.assemble_linear(n, kappa=inputs.lognormal_field(n, 0.0, 2.0, 2.0, 1))
    lv = mg.hierarchy(K, n)
    for (Kf, mf, P, _), (Kc, mc, _, _) in zip(lv[:-1], lv[1:]):
        np.testing.assert_allclose(Kc @ np.ones(Kc.shape[0]), P.T @ (Kf @ np.ones(Kf.shape[0])), rtol=1e-12,
                                   atol=1e-9 * abs(Kf).max())
        np.testing.assert_array_equal(mc, P.T @ mf)
    assert lv[-1][0].shape[0] <= mg.COARSEST_MAX


def test_uniform_coefficient_coarse_stencil():
    # unit coefficient, zero Neumann everywhere: an interior 2x2x2 aggregate couples to each face
    # neighbour through 4 fine faces (-4/h^2) and its diagonal is 8 * 6/h^2 - 2 * 12/h^2 = 24/h^2
    n = (8, 8, 8)
    h2 = 64.0
    neu = {(d, s): ("neumann",) for d in range(3) for s in range(2)}
    K, _ = fv.assemble_linear(n, kappa=1.0, bc=neu)
    Kc = mg.hierarchy(K, n)[1][0].toarray()
    I = 1 + 4 * 1 + 16 * 1  # coarse cell (1, 1, 1) of the 4^3 level: interior
    assert Kc[I, I] == pytest.approx(24 * h2)
    for s in (1, 4, 16):
        assert Kc[I, I + s] == pytest.approx(-4 * h2)
        assert Kc[I, I - s] == pytest.approx(-4 * h2)
    assert abs(Kc.sum(axis=1)).max() < 1e-9 * h2  # Neumann: zero row sums survive coarsening


@pytest.mark.parametrize("n", [(12, 10, 9), (33, 29), (100,)])
def test_vcycle_symmetric_positive_definite(n):
    K, _ = fv.assemble_linear(n, kappa=inputs.lognormal_field(n, 0.0, 2.0, 2.0, 3) if len(n) > 1 else 1.0)
    lv = mg.hierarchy(K, n)
    N = K.shape[0]
    rng = np.random.default_rng(0)
    X = rng.standard_normal((N, 3))
    BX = mg.vcycle(lv, 1e3, 0.7, X)
    G = X.T @ BX
    np.testing.assert_allclose(G, G.T, rtol=1e-12, atol=1e-12 * abs(G).max())
    assert np.all(np.linalg.eigvalsh(0.5 * (G + G.T)) > 0)


def test_vcycle_contracts_as_a_solver():
    # x <- x + V(f - A x) on a heterogeneous 16^3 problem with a weak mass term: the error falls by
    # at least half per cycle (damped Jacobi alone barely moves the smooth error here)
    n = (16, 16, 16)
    K, _ = fv.assemble_linear(n, kappa=inputs.lognormal_field(n, 0.0, 2.0, 3.0, 2))
    a, b = 10.0, 1.0
    A = (a * sp.identity(K.shape[0]) + b * K).tocsr()
    lv = mg.hierarchy(K, n)
    x_true = np.random.default_rng(1).standard_normal((K.shape[0], 1))
    f = A @ x_true
    x = np.zeros_like(f)
    err0 = np.linalg.norm(x - x_true)
    for _ in range(6):
        x = x + mg.vcycle(lv, a, b, f - A @ x)
    assert np.linalg.norm(x - x_true) < err0 * 0.5 ** 6
