"""Pins for the oracle's block kernels: brute force on tiny inputs."""
import numpy as np

from oracle import blockops
from paper_2504_02117_amd import inputs


def test_block_operator_brute_force():
    N, k = 13, 3
    rowptr, col, val = inputs.random_csr(N, 0, 0, 5)
    X = inputs.random_block(N, k, 1)
    md = np.linspace(1.0, 2.0, N)
    K = blockops.csr(rowptr, col, val, N)
    Y = blockops.block_operator(K, X, alpha=0.7, beta=-1.3, mdiag=md)
    ref = np.zeros((N, k))
    for r in range(N):
        for c in range(k):
            acc = 0.0
            for j in range(rowptr[r], rowptr[r + 1]):
                acc += val[j] * X[col[j], c]
            ref[r, c] = 0.7 * md[r] * X[r, c] - 1.3 * acc
    np.testing.assert_allclose(Y, ref, rtol=1e-14, atol=1e-14)


def test_gram_brute_force():
    X, Y = inputs.random_block(9, 4, 2), inputs.random_block(9, 4, 3)
    G = blockops.gram(X, Y)
    for a in range(4):
        for b in range(4):
            assert abs(G[a, b] - sum(X[r, a] * Y[r, b] for r in range(9))) < 1e-13


def test_block_solve_against_dense():
    N, k = 11, 3
    rowptr, col, val = inputs.random_csr(N, 4, 1, 4)
    K = blockops.csr(rowptr, col, val, N)
    B = inputs.random_block(N, k, 5)
    X = blockops.block_solve(K, 10.0, 1.0, B)
    Xd = np.linalg.solve(10.0 * np.eye(N) + K.toarray(), B)
    np.testing.assert_allclose(X, Xd, rtol=1e-12, atol=1e-12)


def test_inputs_are_seeded_and_ordered():
    a = inputs.lognormal_field((8, 6, 4), 0.0, 2.0, 2.0, 0)
    b = inputs.lognormal_field((8, 6, 4), 0.0, 2.0, 2.0, 0)
    assert np.array_equal(a, b) and a.shape == (192,)
    g = np.log(a) / 2.0
    assert abs(g.mean()) < 1e-12 and abs(g.std() - 1) < 1e-12
    u = inputs.sin_product((4, 3))
    # cell (ix=1, iy=2) has linear index 1 + 4*2 = 9, centre (0.375, 5/6)
    assert u[9] == np.sin(np.pi * 0.375) * np.sin(np.pi * 5 / 6)
