"""Pins for the oracle's multigrid V-cycle: Galerkin coarse operators (row sums, the uniform-coefficient
coarse stencil), the cycle's closed form when A is a multiple of the mass, and its symmetry,
positive definiteness and contraction."""
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


def _mass_only_cycle(f, counts, a, w, s, wc, sweeps, P):
    """The V-cycle for b = 0 worked out by hand: A_l = a diag(m_l) is diagonal, so each damped Jacobi
    sweep scales its residual by (1 - w), the coarsest solve leaves (1 - wc)^sweeps of the exact
    answer f / (a m), and the post-sweep gives z' = (1 - w) z + w f / (a m)."""
    m = counts[0]
    if len(P) == 0:
        return (1.0 - (1.0 - wc) ** sweeps) * f / (a * m)[:, None]
    x = w * f / (a * m)[:, None]
    fc = P[0].T @ ((1.0 - w) * f)  # f - A x = (1 - w) f
    xc = _mass_only_cycle(fc, counts[1:], a, w, s, wc, sweeps, P[1:])
    z = x + s * (P[0] @ xc)
    return (1.0 - w) * z + w * f / (a * m)[:, None]


@pytest.mark.parametrize("n", [(8, 4, 4), (16, 8, 8), (9, 7, 5)])
def test_vcycle_closed_form_without_stiffness(n):
    # with b = 0 every level is diagonal and the cycle has a closed form in the damping factors, the
    # coarse scale and the sweep count; the cell counts m_l come from the aggregation alone
    K, _ = fv.assemble_linear(n, kappa=inputs.lognormal_field(n, 0.0, 1.0, 2.0, 4))
    lv = mg.hierarchy(K, n)
    assert len(lv) >= 2
    Ps = [P for (_, _, P, _) in lv[:-1]]
    counts, c = [], np.ones(K.shape[0])
    for P in [None] + Ps:
        if P is not None:
            c = P.T @ c  # cells per aggregate, counted again from the prolongations
        counts.append(c)
    f = np.random.default_rng(5).standard_normal((K.shape[0], 2))
    a = 7.0
    want = _mass_only_cycle(f, counts, a, 0.9, 1.4, 0.8, 12, Ps)
    np.testing.assert_allclose(mg.vcycle(lv, a, 0.0, f), want, rtol=1e-13, atol=1e-15)


def test_coarse_scale_shortens_the_iteration():
    # the scaled coarse correction is a better preconditioner than the plain one on a heterogeneous
    # problem with a deep hierarchy: fewer CG iterations to the same residual (the reason for the
    # scale; on 512^2 the count falls from 90 to 47, on 128^3 from 31 to 24)
    n = (256, 256)
    K, _ = fv.assemble_linear(n, kappa=inputs.lognormal_field(n, 0.0, 2.0, 8.0, 0))
    a, b = 1e3, 1.0
    A = (a * sp.identity(K.shape[0]) + b * K).tocsr()
    lv = mg.hierarchy(K, n)
    f = np.random.default_rng(2).standard_normal((K.shape[0], 1))

    def pcg_iters(scale):
        old = mg.COARSE_SCALE
        mg.COARSE_SCALE = scale
        try:
            x = np.zeros_like(f)
            r = f.copy()
            z = mg.vcycle(lv, a, b, r)
            p = z.copy()
            rz = float((r * z).sum())
            for it in range(1, 200):
                q = A @ p
                al = rz / float((p * q).sum())
                x += al * p
                r -= al * q
                if np.linalg.norm(r) < 1e-8 * np.linalg.norm(f):
                    return it
                z = mg.vcycle(lv, a, b, r)
                rz, rz0 = float((r * z).sum()), rz
                p = z + (rz / rz0) * p
            return 200
        finally:
            mg.COARSE_SCALE = old

    assert pcg_iters(mg.COARSE_SCALE) < 0.8 * pcg_iters(1.0)
