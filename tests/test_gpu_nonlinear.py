"""GPU parity of the Newton form of Algorithm 1 (nonlinear diffusion-reaction, Sec. 2.2): the
column-wise f, its Jacobian, the fused nonlinear window residual, one Newton step and the full
pipelined stepper, each through the C ABI against the oracle on the same seeded inputs."""
import sys

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import allatonce as aao
from oracle import fv, stepping
from oracle import timecoupling as otc
from paper_2504_02117_amd import inputs

pytestmark = pytest.mark.gpu

# D(u) = 1 + u^2, r(u) = -u^3: the diffusion-reaction problem of the nonlinear experiments
DCOEF = (1.0, 0.0, 1.0, 0.0)
RCOEF = (0.0, 0.0, 0.0, -1.0)


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


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def make(env, n, bc=None, dcoef=DCOEF, rcoef=RCOEF):
    """Device operator and oracle operator for the same problem.  ``bc`` maps (axis, side) to
    ('dirichlet', g) or ('neumann',); unspecified faces are zero flux."""
    torch, bkts, ctx = env
    bc_type = [bkts.BKTS_BC_NEUMANN] * 6
    bc_value = [0.0] * 6
    obc = {"default": ("neumann",)}
    for (d, side), spec in (bc or {}).items():
        if spec[0] == "dirichlet":
            bc_type[2 * d + side] = bkts.BKTS_BC_DIRICHLET
            bc_value[2 * d + side] = spec[1]
        obc[(d, side)] = spec
    nl = bkts.bkts_nlop_create(ctx, n, dcoef=dcoef, rcoef=rcoef, bc_type=bc_type, bc_value=bc_value)
    ref = fv.NonlinearDiffusionReaction(n, dcoef=dcoef, rcoef=rcoef, bc=obc)
    return nl, ref


GRIDS = [
    dict(n=(40, 37)),
    dict(n=(9, 8, 7), bc={(0, 0): ("dirichlet", 1.0), (2, 1): ("dirichlet", -0.5)}),
    dict(n=(301,), bc={(0, 1): ("dirichlet", 0.25)}),
    dict(n=(1, 1)),
    dict(n=(64, 33), bc={(1, 0): ("dirichlet", 0.5)}),
]


def _block(n, k, seed):
    N = int(np.prod(n))
    return np.column_stack([inputs.smooth_random(n, seed + j) for j in range(k)]) * 1.5 - 0.25 \
        if N > 1 else np.random.default_rng(seed).random((1, k))


@pytest.mark.parametrize("gi", range(len(GRIDS)))
def test_nl_eval_matches_oracle(env, gi):
    torch, bkts, ctx = env
    g = GRIDS[gi]
    say(f"nl_eval {g}")
    nl, ref = make(env, g["n"], g.get("bc"))
    try:
        k = 5
        Y = _block(g["n"], k, 11)
        Yd = dev(torch, Y)
        Fd = torch.full((Y.shape[0], k + 2), np.nan, dtype=torch.float64, device="cuda")
        bkts.bkts_nl_eval(ctx, nl, Yd, Fd[:, 1:k + 1])
        got = Fd.cpu().numpy()
        want = np.column_stack([ref.f(Y[:, j]) for j in range(k)])
        scale = np.abs(want).max() + 1.0
        assert np.abs(got[:, 1:k + 1] - want).max() / scale < 1e-13
        assert np.isnan(got[:, 0]).all() and np.isnan(got[:, k + 1]).all()  # outside the view untouched
    finally:
        bkts.bkts_nlop_destroy(nl)


@pytest.mark.parametrize("gi", range(len(GRIDS)))
def test_nl_jacobian_matches_oracle(env, gi):
    torch, bkts, ctx = env
    g = GRIDS[gi]
    say(f"nl_jacobian {g}")
    nl, ref = make(env, g["n"], g.get("bc"))
    try:
        u = _block(g["n"], 1, 3)[:, 0]
        alpha, beta = 1e3, 0.29
        J = bkts.bkts_nl_jacobian(ctx, nl, dev(torch, u), alpha, beta)
        rowptr, col, val, _ = bkts.bkts_op_export_csr(J)
        N = u.shape[0]
        got = sp.csr_matrix((val, col, rowptr), shape=(N, N))
        want = (alpha * sp.identity(N) + beta * ref.jac(u)).tocsr()
        diff = abs(got - want).max()
        assert diff / abs(want).max() < 1e-14
        # sorted columns, as the stencil is stored
        for r in range(min(N, 200)):
            assert np.all(np.diff(col[rowptr[r]:rowptr[r + 1]]) > 0)
        # a second call with another point reuses the storage and refreshes the values
        u2 = u * 0.5 + 0.1
        J2 = bkts.bkts_nl_jacobian(ctx, nl, dev(torch, u2), 1.0, 1.0)
        assert J2 == J
        _, _, val2, _ = bkts.bkts_op_export_csr(J2)
        want2 = (sp.identity(N) + ref.jac(u2)).tocsr()
        got2 = sp.csr_matrix((val2, col, rowptr), shape=(N, N))
        assert abs(got2 - want2).max() / abs(want2).max() < 1e-14
    finally:
        bkts.bkts_nlop_destroy(nl)


@pytest.mark.parametrize("k,phase", [(1, 0), (4, 0), (4, 1), (7, 1), (16, 0), (16, 1)])
def test_nl_residual_matches_oracle(env, k, phase):
    torch, bkts, ctx = env
    n = (53, 47)
    tau = 1e-2
    say(f"nl_residual k={k} phase={phase}")
    nl, ref = make(env, n, {(0, 0): ("dirichlet", 1.0)})
    tc = bkts.bkts_tc_create(ctx, bkts.BKTS_SDIRK2, k, tau)
    try:
        A, _, c = otc.tableau("sdirk2")
        A1, A2, _ = otc.window_matrices(A, c, k, phase, tau)
        Y = _block(n, k, 21)
        yn = inputs.smooth_random(n, 5)
        fst = [ref.f(Y[:, 0] * 0.9)]
        B0 = otc.window_b0(A, c, k, phase, tau, yn, ref.f(yn), fst[:phase])
        nb0 = min(2 - phase, k)
        want = aao.residual_nonlinear(sp.identity(Y.shape[0]), lambda j, y: ref.f(y), A1, A2, Y, B0)
        Yd = dev(torch, Y)
        Rd = torch.empty_like(Yd)
        norms = bkts.bkts_nl_residual(ctx, nl, tc, Yd, Rd, B0=dev(torch, B0[:, :nb0]), phase=phase)
        got = Rd.cpu().numpy()
        scale = np.abs(want).max()
        assert np.abs(got - want).max() / scale < 1e-13
        np.testing.assert_allclose(norms, (want ** 2).sum(0), rtol=1e-11)
    finally:
        bkts.bkts_tc_destroy(tc)
        bkts.bkts_nlop_destroy(nl)


@pytest.mark.parametrize("krylov,mg", [(1, False), (2, False), (1, True), (2, True)])
@pytest.mark.parametrize("precision", [0, 1])
def test_newton_step_matches_direct(env, krylov, mg, precision):
    """One Newton iteration: Y - J^{-1} R(Y) with J = I/tau + a_kk Df(Y_0), J^{-1} by a direct solve
    (mg: preconditioned by the V-cycle of the symmetric part of J)."""
    torch, bkts, ctx = env
    n = (48, 40)
    k, tau = 4, 5e-3
    say(f"newton_step krylov={krylov} mg={mg} precision={precision}")
    nl, ref = make(env, n)
    tc = bkts.bkts_tc_create(ctx, bkts.BKTS_SDIRK2, k, tau)
    try:
        A, _, c = otc.tableau("sdirk2")
        A1, A2, beta = otc.window_matrices(A, c, k, 0, tau)
        N = int(np.prod(n))
        yn = inputs.smooth_random(n, 9)
        Y = np.column_stack([yn] * k)
        B0 = otc.window_b0(A, c, k, 0, tau, yn, ref.f(yn), [])
        R = aao.residual_nonlinear(sp.identity(N), lambda j, y: ref.f(y), A1, A2, Y, B0)
        J = (sp.identity(N) / tau + beta * ref.jac(Y[:, 0])).tocsc()
        lu = spla.splu(J)
        want = Y - np.column_stack([lu.solve(R[:, j]) for j in range(k)])
        Yd = dev(torch, Y)
        opts = bkts.solve_opts(krylov=krylov, precision=precision, rtol=1e-13, inner_rtol=1e-6, maxit=4000)
        if mg:
            opts.precond = bkts.BKTS_PREC_MG
        norms, info = bkts.bkts_newton_step(ctx, nl, tc, Yd, B0=dev(torch, B0[:, :2]), phase=0, opts=opts)
        np.testing.assert_allclose(norms, (R ** 2).sum(0), rtol=1e-11)
        got = Yd.cpu().numpy()
        rel = np.linalg.norm(got - want) / np.linalg.norm(want)
        assert rel < 1e-10, rel
        say(f"  iterations={info.iterations} refinements={info.refinements} rel={rel:.2e}")
    finally:
        bkts.bkts_tc_destroy(tc)
        bkts.bkts_nlop_destroy(nl)


@pytest.mark.parametrize("k,krylov,precision,mg", [(2, 2, 1, False), (4, 2, 1, False), (16, 2, 1, False),
                                                    (4, 1, 0, False), (3, 2, 0, False), (4, 2, 1, True),
                                                    (3, 2, 0, True)])
def test_nl_stepper_matches_sequential_newton(env, k, krylov, precision, mg):
    """Algorithm 1 in Newton form (SDIRK2, D = 1 + u^2, r = -u^3, zero flux, smooth initial data in
    [0, 1]) against per-stage Newton with exact Jacobians and direct solves (mg: BiCGStab
    preconditioned by the V-cycle of the symmetric part of each Jacobian)."""
    torch, bkts, ctx = env
    n = (36, 30)
    steps, tau = 6, 2e-3
    say(f"nl stepper k={k} krylov={krylov} precision={precision} mg={mg}")
    nl, ref = make(env, n)
    tc = bkts.bkts_tc_create(ctx, bkts.BKTS_SDIRK2, k, tau)
    st = None
    try:
        N = int(np.prod(n))
        y0 = inputs.smooth_random(n, 4)
        ys, _, _ = stepping.dirk_nonlinear(ref, y0, tau, "sdirk2", steps)
        st = bkts.bkts_nl_stepper_create(ctx, nl, tc, dev(torch, y0))
        hist = torch.zeros((steps, N), dtype=torch.float64, device="cuda")
        inner = bkts.solve_opts(krylov=krylov, precision=precision, rtol=1e-3, inner_rtol=1e-3, maxit=2000)
        if mg:
            inner.precond = bkts.BKTS_PREC_MG
        info = bkts.bkts_stepper_advance(st, steps, inner=inner, outer_rtol=1e-12, max_outer=100, y_hist=hist)
        assert info.accepted_steps == steps
        got = hist.cpu().numpy()
        for s in range(steps):
            rel = np.linalg.norm(got[s] - ys[s + 1]) / np.linalg.norm(ys[s + 1])
            assert rel < 1e-8, (s, rel)
        yl = torch.empty(N, dtype=torch.float64, device="cuda")
        assert bkts.bkts_stepper_state(st, yl) == steps
        np.testing.assert_array_equal(yl.cpu().numpy(), got[-1])
        say(f"  outer={info.outer_iterations} krylov={info.krylov_iterations} rel_last={rel:.2e}")
    finally:
        if st:
            bkts.bkts_stepper_destroy(st)
        bkts.bkts_tc_destroy(tc)
        bkts.bkts_nlop_destroy(nl)


def test_nl_stepper_multigrid_is_repeatable(env):
    """The multigrid-preconditioned Newton form reduces in a fixed order: two runs from the same
    state give the same bits (the hierarchy of the Jacobian's symmetric part is rebuilt in place)."""
    torch, bkts, ctx = env
    n = (36, 30)
    steps, tau = 4, 2e-3
    nl, _ = make(env, n)
    tc = bkts.bkts_tc_create(ctx, bkts.BKTS_SDIRK2, 4, tau)
    try:
        N = int(np.prod(n))
        y0 = inputs.smooth_random(n, 4)
        inner = bkts.solve_opts(krylov=2, precision=1, rtol=1e-3, inner_rtol=1e-3, maxit=2000)
        inner.precond = bkts.BKTS_PREC_MG
        runs = []
        for _ in range(2):
            st = bkts.bkts_nl_stepper_create(ctx, nl, tc, dev(torch, y0))
            try:
                hist = torch.zeros((steps, N), dtype=torch.float64, device="cuda")
                info = bkts.bkts_stepper_advance(st, steps, inner=inner, outer_rtol=1e-12, max_outer=100, y_hist=hist)
                assert info.accepted_steps == steps
                runs.append(hist.cpu().numpy())
            finally:
                bkts.bkts_stepper_destroy(st)
        np.testing.assert_array_equal(runs[0], runs[1])
    finally:
        bkts.bkts_tc_destroy(tc)
        bkts.bkts_nlop_destroy(nl)


def test_nl_argument_errors(env):
    torch, bkts, ctx = env
    with pytest.raises(bkts.BktsError):
        bkts.bkts_nlop_create(ctx, (0, 4))
    nl, _ = make(env, (6, 5))
    tc = bkts.bkts_tc_create(ctx, bkts.BKTS_SDIRK2, 4, 1e-2)
    try:
        Y = torch.zeros((30, 4), dtype=torch.float64, device="cuda")
        with pytest.raises(bkts.BktsError):
            bkts.bkts_nl_residual(ctx, nl, tc, Y, Y)  # aliasing
        with pytest.raises(bkts.BktsError):
            bkts.bkts_nl_residual(ctx, nl, tc, Y, torch.empty_like(Y), phase=2)
    finally:
        bkts.bkts_tc_destroy(tc)
        bkts.bkts_nlop_destroy(nl)
