"""GPU parity for the index-free stencil form of the block operator (symmetric 5/7-point FV
operators; the BOP of Sec. 3 without its column-index stream): the operator itself against the
oracle's sparse matrix on several grids (3-D, 2-D, 1-D, degenerate axes, ragged sizes), the fused
SpMM + Gram of narrow block CG, block solves, Algorithm 1 with DIRK and Radau IIA tableaux, the full
128^3 operator on sampled rows, and the rejection of non-symmetric operators."""
import sys

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import blockops, fv, stepping
from paper_2504_02117_amd import inputs

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2504_02117_amd import bkts
    assert torch.cuda.is_available()
    ctx = bkts.bkts_ctx_create(0, torch.cuda.current_stream())
    yield torch, bkts, ctx
    torch.cuda.synchronize()
    bkts.bkts_ctx_destroy(ctx)


def dev(torch, a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def stencil_op(env, n, kappa, bc=None, velocity=(0.0, 0.0, 0.0)):
    torch, bkts, ctx = env
    bc_type = [bkts.BKTS_BC_DIRICHLET] * 6
    bc_value = [0.0] * 6
    for (d, side), spec in (bc or {}).items():
        f = 2 * d + side
        if spec[0] == "neumann":
            bc_type[f] = bkts.BKTS_BC_NEUMANN
        else:
            bc_value[f] = spec[1]
    op = bkts.bkts_fv_assemble(ctx, n, kappa=None if kappa is None else dev(torch, kappa), kappa_const=1.0,
                               velocity=velocity, bc_type=bc_type, bc_value=bc_value, fmt=bkts.BKTS_FMT_STENCIL)
    K, b = fv.assemble_linear(n, kappa=kappa, velocity=velocity[:len(n)], bc=bc or {})
    return op, K, b


GRIDS = [
    ((20, 19, 18), {(0, 0): ("dirichlet", 1.0), (2, 1): ("neumann",)}),
    ((33, 29), {(1, 1): ("neumann",)}),
    ((257,), {}),
    ((1, 7, 9), {}),   # nx = 1: the x and y offsets coincide
    ((5, 1, 4), {}),   # ny = 1: the y and z offsets coincide
]


@pytest.mark.parametrize("gi", range(len(GRIDS)))
@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 8, 16, 32])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_stencil_spmm_matches_oracle(env, gi, k, dtype):
    torch, bkts, ctx = env
    n, bc = GRIDS[gi]
    say(f"stencil spmm n={n} k={k} {dtype}")
    kap = inputs.lognormal_field(n, 0.0, 1.5, 2.0, 3) if len(n) > 1 else np.exp(np.linspace(-2, 2, n[0]))
    op, K, _ = stencil_op(env, n, kap, bc)
    try:
        N = K.shape[0]
        X = inputs.random_block(N, k, 11 + k)
        tdt = torch.float64 if dtype == "f64" else torch.float32
        Xd = dev(torch, X, tdt)
        Yd = torch.full((N, k), 7.0, dtype=tdt, device="cuda")
        bkts.bkts_spmm(ctx, op, Xd, Yd, alpha=-2.5, beta=1.0)
        if dtype == "f64":
            ref = blockops.block_operator(K, X, -2.5, 1.0)
            tol = 1e-13
        else:
            Kf = sp.csr_matrix((K.data.astype(np.float32).astype(np.float64), K.indices, K.indptr), shape=K.shape)
            ref = blockops.block_operator(Kf, X.astype(np.float32).astype(np.float64), -2.5, 1.0)
            tol = 2e-6
        got = Yd.double().cpu().numpy()
        scale = abs(K).sum(1).A.ravel()[:, None] * abs(X).max() + 2.5 * abs(X).max()
        assert (abs(got - ref) / scale).max() < tol
    finally:
        bkts.bkts_op_destroy(op)


@pytest.mark.parametrize("k", [8, 16, 32])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_stencil_spmm_tiled_ragged(env, k, dtype):
    """Wide rows on a 3-D grid whose sizes are not multiples of the x-y tile, with several z-planes
    per workgroup and a shorter last z-chunk (71 planes), against the oracle's operator."""
    torch, bkts, ctx = env
    n = (45, 37, 71)
    say(f"stencil spmm tiled n={n} k={k} {dtype}")
    kap = inputs.lognormal_field(n, 0.0, 1.5, 3.0, 7)
    op, K, _ = stencil_op(env, n, kap, {(0, 1): ("dirichlet", 2.0), (1, 0): ("neumann",)})
    try:
        N = K.shape[0]
        X = inputs.random_block(N, k, 5 + k)
        tdt = torch.float64 if dtype == "f64" else torch.float32
        Xd = dev(torch, X, tdt)
        Yd = torch.full((N, k), 7.0, dtype=tdt, device="cuda")
        bkts.bkts_spmm(ctx, op, Xd, Yd, alpha=0.75, beta=-1.5)
        if dtype == "f64":
            ref = blockops.block_operator(K, X, 0.75, -1.5)
            tol = 1e-13
        else:
            Kf = sp.csr_matrix((K.data.astype(np.float32).astype(np.float64), K.indices, K.indptr), shape=K.shape)
            ref = blockops.block_operator(Kf, X.astype(np.float32).astype(np.float64), 0.75, -1.5)
            tol = 2e-6
        got = Yd.double().cpu().numpy()
        scale = abs(K).sum(1).A.ravel()[:, None] * abs(X).max() + 1.5 * abs(X).max()
        assert (abs(got - ref) / scale).max() < tol
    finally:
        bkts.bkts_op_destroy(op)


@pytest.mark.parametrize("k", [3, 16])
def test_stencil_spmm_strided_and_source(env, k):
    """Leading dimensions that rule out 16-byte access, and the operator inside the refinement
    residual R = B - (a I + b K) X (a source block)."""
    torch, bkts, ctx = env
    n = (17, 15, 13)
    op, K, _ = stencil_op(env, n, inputs.lognormal_field(n, 0.0, 2.0, 3.0, 4))
    try:
        N = K.shape[0]
        X = inputs.random_block(N, k, 2)
        Xbig = torch.zeros((N, k + 3), dtype=torch.float64, device="cuda")
        Xbig[:, :k] = dev(torch, X)
        Ybig = torch.full((N, k + 3), 7.0, dtype=torch.float64, device="cuda")
        bkts.bkts_spmm(ctx, op, Xbig[:, :k], Ybig[:, :k], alpha=3.0, beta=0.5)
        got = Ybig.cpu().numpy()
        ref = blockops.block_operator(K, X, 3.0, 0.5)
        scale = abs(K).sum(1).A.ravel()[:, None] * abs(X).max()
        assert (abs(got[:, :k] - ref) / scale).max() < 1e-13
        assert (got[:, k:] == 7.0).all()
    finally:
        bkts.bkts_op_destroy(op)


def test_stencil_matches_sell_csr_export(env):
    """The stencil operator keeps the assembled CSR (export) identical to the SELL operator's."""
    torch, bkts, ctx = env
    n = (12, 11, 10)
    kap = inputs.lognormal_field(n, 0.0, 2.0, 3.0, 8)
    op_s, K, b = stencil_op(env, n, kap, {(0, 0): ("dirichlet", 0.5)})
    op_l = bkts.bkts_fv_assemble(ctx, n, kappa=dev(torch, kap), bc_type=[0] * 6, bc_value=[0.5, 0, 0, 0, 0, 0],
                                 fmt=bkts.BKTS_FMT_SELL)
    try:
        a = bkts.bkts_op_export_csr(op_s)
        c = bkts.bkts_op_export_csr(op_l)
        for x, y in zip(a, c):
            np.testing.assert_array_equal(x, y)
    finally:
        bkts.bkts_op_destroy(op_s)
        bkts.bkts_op_destroy(op_l)


def test_stencil_rejects_nonsymmetric_and_raw_csr(env):
    torch, bkts, ctx = env
    with pytest.raises(bkts.BktsError) as e:
        stencil_op(env, (8, 7, 6), None, velocity=(1.0, 0.5, 0.0))
    assert e.value.status == bkts.BKTS_EINVAL
    K, _ = fv.assemble_linear((6, 5))
    K = K.tocsr()
    rp = dev(torch, K.indptr.astype(np.int32))
    ci = dev(torch, K.indices.astype(np.int32))
    va = dev(torch, K.data)
    with pytest.raises(bkts.BktsError) as e:
        bkts.bkts_op_create_csr(ctx, K.shape[0], K.nnz, rp, ci, va, fmt=bkts.BKTS_FMT_STENCIL)
    assert e.value.status == bkts.BKTS_EINVAL


@pytest.mark.parametrize("k", [1, 2, 4, 8, 16])
@pytest.mark.parametrize("precision", [0, 1])
def test_stencil_block_solve_matches_direct(env, k, precision):
    """Block CG on the stencil operator (the fused SpMM + Gram for k <= 4) against k sparse LU solves."""
    torch, bkts, ctx = env
    n = (14, 13, 12)
    say(f"stencil block solve k={k} precision={precision}")
    op, K, _ = stencil_op(env, n, inputs.lognormal_field(n, 0.0, 2.0, 3.0, 5))
    try:
        N = K.shape[0]
        tau = 1e-3
        B = inputs.random_block(N, k, 30 + k)
        want = blockops.block_solve(K, 1.0 / tau, 1.0, B)
        Xd = torch.zeros((N, k), dtype=torch.float64, device="cuda")
        opts = bkts.solve_opts(precision=precision, rtol=1e-11, inner_rtol=1e-4)
        info = bkts.bkts_block_solve(ctx, op, 1.0 / tau, 1.0, dev(torch, B), Xd, opts)
        got = Xd.cpu().numpy()
        assert info.converged == 1
        err = np.linalg.norm(got - want, axis=0) / np.linalg.norm(want, axis=0)
        assert err.max() < 1e-9
    finally:
        bkts.bkts_op_destroy(op)


@pytest.mark.parametrize("method,name,k", [(0, "ie", 4), (2, "sdirk2", 8), (4, "radau2", 4)])
def test_stencil_advance_matches_sequential_oracle(env, method, name, k):
    torch, bkts, ctx = env
    n = (10, 9, 8)
    steps, tau = 5, 2e-3
    say(f"stencil advance {name} k={k}")
    op, K, b = stencil_op(env, n, inputs.lognormal_field(n, 0.0, 1.5, 2.0, 9), {(0, 0): ("dirichlet", 1.0)})
    tc = bkts.bkts_tc_create(ctx, method, k, tau)
    try:
        N = K.shape[0]
        y0 = inputs.smooth_random(n, 3)
        hist = torch.zeros((steps, N), dtype=torch.float64, device="cuda")
        inner = bkts.solve_opts(precision=1, rtol=1e-3, inner_rtol=1e-4)
        info = bkts.bkts_advance(ctx, op, tc, dev(torch, y0), steps, inner=inner, outer_rtol=1e-12, max_outer=300,
                                 y_hist=hist)
        if name == "radau2":
            ys, _ = stepping.rk_linear(K, b, y0, tau, name, steps)
        else:
            ys, _ = stepping.dirk_linear(K, b, y0, tau, name, steps)
        got = hist.cpu().numpy()
        for s in range(steps):
            assert np.linalg.norm(got[s] - ys[s + 1]) / np.linalg.norm(ys[s + 1]) < 1e-8, s
        assert info.accepted_steps == steps
    finally:
        bkts.bkts_tc_destroy(tc)
        bkts.bkts_op_destroy(op)


def test_stencil_full_size_128cubed_sampled(env):
    """The 128^3 lognormal (sigma=2, correlation 8 cells) headline operator in stencil form: sampled
    rows of the FP32 k = 4 and FP64 k = 16 block operators against the oracle's rows."""
    torch, bkts, ctx = env
    n = (128, 128, 128)
    say("stencil full-size 128^3")
    kap = inputs.lognormal_field(n, 0.0, 2.0, 8.0, 0)
    op, K, _ = stencil_op(env, n, kap)
    try:
        N = K.shape[0]
        rows = np.random.default_rng(1).choice(N, 4000, replace=False)
        Kr = K[rows]
        for k, dtype in ((4, "f32"), (16, "f64")):
            X = inputs.random_block(N, k, 6)
            tdt = torch.float64 if dtype == "f64" else torch.float32
            Xd = dev(torch, X, tdt)
            Yd = torch.empty_like(Xd)
            bkts.bkts_spmm(ctx, op, Xd, Yd, alpha=1e3, beta=1.0)
            got = Yd.double().cpu().numpy()[rows]
            if dtype == "f64":
                ref = 1e3 * X[rows] + Kr @ X
                tol = 1e-13
            else:
                Xf = X.astype(np.float32).astype(np.float64)
                Kf = sp.csr_matrix((Kr.data.astype(np.float32).astype(np.float64), Kr.indices, Kr.indptr),
                                   shape=Kr.shape)
                ref = 1e3 * Xf[rows] + Kf @ Xf
                tol = 2e-6
            scale = abs(Kr).sum(1).A.ravel()[:, None] * abs(X).max() + 1e3 * abs(X).max()
            assert (abs(got - ref) / scale).max() < tol
            del Xd, Yd
    finally:
        bkts.bkts_op_destroy(op)


@pytest.mark.parametrize("method,name", [(0, "ie"), (2, "sdirk2"), (4, "radau2")])
@pytest.mark.parametrize("k", [1, 2, 4, 6])
def test_stencil_residual_matches_oracle(env, method, name, k):
    """The fused all-at-once residual on the stencil form (row-per-thread kernel for k <= 4, the tiled
    kernel above), with a nonzero source and B0 columns, every phase, against the oracle."""
    from oracle import allatonce as aao
    from oracle import timecoupling as otc
    torch, bkts, ctx = env
    if name == "radau2" and k % 2:
        pytest.skip("Radau IIA windows hold whole steps")
    n = (11, 9, 7)
    op, K, b = stencil_op(env, n, inputs.lognormal_field(n, 0.0, 1.0, 2.0, 2), {(0, 0): ("dirichlet", 1.0)})
    tau = 0.01
    tc = bkts.bkts_tc_create(ctx, method, k, tau)
    try:
        N = K.shape[0]
        A, _, c = otc.tableau(name)
        mi = otc.implicit_part(A, c)[0].shape[0]
        phases = [0] if name == "radau2" else range(mi)
        for phase in phases:
            Y = inputs.random_block(N, k, 20 + phase)
            nb0 = min(mi - phase, k)
            B0 = inputs.random_block(N, nb0, 30 + phase)
            R = torch.empty((N, k), dtype=torch.float64, device="cuda")
            norms = bkts.bkts_residual(ctx, op, tc, torch.from_numpy(Y).cuda(), R, B0=torch.from_numpy(B0).cuda(),
                                       phase=phase)
            A1, A2, _ = otc.window_matrices(A, c, k, phase, tau)
            B0full = np.zeros((N, k))
            B0full[:, :nb0] = B0
            ref = aao.residual_linear(sp.identity(N), K, A1, A2, Y, np.tile(b[:, None], (1, k)), B0full)
            got = R.cpu().numpy()
            scale = (abs(K).sum(1).A.ravel()[:, None] + 2 / tau) * 4
            assert (abs(got - ref) / scale).max() < 1e-13
            np.testing.assert_allclose(norms, (ref ** 2).sum(0), rtol=1e-11)
    finally:
        bkts.bkts_tc_destroy(tc)
        bkts.bkts_op_destroy(op)
