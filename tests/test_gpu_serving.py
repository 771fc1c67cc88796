"""GPU tests of the serving loop: every request's window against the oracle's sequential stepping,
bitwise equality of a request alone and inside a mix of other requests, HBM-budgeted admission
and continuous batching (requests admitted while others run), for grouped window-splitting
requests (mode 0) and pipelined multigrid requests on worker lanes (mode 1)."""
import sys
import time

import numpy as np
import pytest

from oracle import fv, stepping
from paper_2504_02117_amd import inputs

pytestmark = pytest.mark.gpu

METHODS = {"ie": 0, "theta": 1, "sdirk2": 2}


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


class Req:
    """One synthetic request: 2-D lognormal diffusion (seed = tag), y0 = sin-product."""

    def __init__(self, torch, n, k, tag, method="ie", tau=1e-3, sigma=1.0, mode=0, window=0):
        self.n, self.k, self.tag, self.method, self.tau = n, k, tag, method, tau
        self.mode, self.window = mode, window
        self.kappa = inputs.lognormal_field(n, 0.0, sigma, 4.0, tag)
        self.y0 = inputs.sin_product(n)
        self.N = int(np.prod(n))
        self.kd = torch.from_numpy(self.kappa).cuda()
        self.y0d = torch.from_numpy(self.y0).cuda()
        self.out = torch.full((self.N, k), np.nan, dtype=torch.float64, device="cuda")

    def request(self, bkts, rtol=1e-12, inner_rtol=1e-3):
        return bkts.make_request(self.n, self.y0d, self.out, self.k, self.tau, kappa=self.kd,
                                 method=METHODS[self.method], rtol=rtol, inner_rtol=inner_rtol, tag=self.tag,
                                 mode=self.mode, window=self.window)

    def oracle_columns(self):
        """Window columns by sequential stepping: every implicit stage in order."""
        K, b = fv.assemble_linear(self.n, kappa=self.kappa)
        per_step = 2 if self.method == "sdirk2" else 1
        steps = -(-self.k // per_step)
        _, stages = stepping.dirk_linear(K, b, self.y0, self.tau, self.method, steps)
        cols = [s for st in stages for s in (st if self.method == "sdirk2" else [st[-1]])]
        return np.column_stack(cols[:self.k])


def run_all(bkts, srv, reqs, timeout=120.0):
    tickets = {bkts.bkts_server_submit(srv, r.request(bkts)): r for r in reqs}
    got = {}
    t_end = time.time() + timeout
    while len(got) < len(tickets):
        assert time.time() < t_end, "serving timed out"
        bkts.bkts_server_wait(srv, 1, 1.0)
        for res in bkts.bkts_server_poll(srv):
            got[res.ticket] = res
    return {tickets[t]: r for t, r in got.items()}


def check_against_oracle(r, res):
    assert res.status == 0, (r.n, r.k, res.status)
    got = r.out.cpu().numpy()
    want = r.oracle_columns()
    for j in range(r.k):
        rel = np.linalg.norm(got[:, j] - want[:, j]) / np.linalg.norm(want[:, j])
        assert rel < 1e-8, (r.n, r.k, r.method, j, rel)


@pytest.mark.parametrize("n,k,method,mode,window", [
    ((16, 16), 4, "ie", 0, 0), ((24, 20), 1, "ie", 0, 0), ((33, 31), 8, "ie", 0, 0),
    ((20, 18), 3, "sdirk2", 0, 0), ((18, 18), 16, "ie", 0, 0), ((12, 10), 32, "ie", 0, 0),
    ((21, 19), 5, "theta", 0, 0), ((40, 8), 2, "sdirk2", 0, 0),
    ((16, 16), 4, "ie", 1, 0), ((24, 20), 1, "ie", 1, 0), ((33, 31), 8, "ie", 1, 0), ((70, 66), 16, "ie", 1, 0),
    ((12, 10), 32, "ie", 1, 0), ((45, 43), 7, "ie", 1, 2), ((30, 28), 5, "ie", 1, 5)])
def test_request_matches_oracle(env, n, k, method, mode, window):
    torch, bkts, ctx = env
    say(f"serving single n={n} k={k} {method} mode={mode} window={window}")
    srv = bkts.bkts_server_create(ctx, 1 << 30, 8)
    try:
        r = Req(torch, n, k, 7, method=method, mode=mode, window=window)
        torch.cuda.synchronize()
        res = run_all(bkts, srv, [r])[r]
        check_against_oracle(r, res)
        say(f"  outer={res.outer_iterations} krylov={res.krylov_iterations} rel={res.rel_residual:.2e}")
    finally:
        bkts.bkts_server_destroy(srv)


@pytest.mark.parametrize("probe_mode", [0, 1])
def test_alone_equals_mix_and_batching(env, probe_mode):
    """The same request alone and among 11 others of mixed sizes, widths and modes: bitwise equal
    outputs, each within 1e-8 of the oracle; later requests join while earlier ones run."""
    torch, bkts, ctx = env
    say(f"serving alone vs mix, probe mode {probe_mode}")
    probe_shape = ((48, 40), 8)
    alone = Req(torch, probe_shape[0], probe_shape[1], 3, mode=probe_mode)
    torch.cuda.synchronize()
    srv = bkts.bkts_server_create(ctx, 1 << 30, 4)
    try:
        res_alone = run_all(bkts, srv, [alone])[alone]
        check_against_oracle(alone, res_alone)
        ref = alone.out.cpu().numpy()
    finally:
        bkts.bkts_server_destroy(srv)
    rng = np.random.default_rng(1)
    mix = []
    for i in range(11):
        n = int(rng.choice([16, 24, 32, 64]))
        k = int(rng.choice([1, 4, 8, 16, 32]))
        mix.append(Req(torch, (n, n), k, 100 + i, mode=i % 2))
    probe = Req(torch, probe_shape[0], probe_shape[1], 3, mode=probe_mode)
    torch.cuda.synchronize()
    srv = bkts.bkts_server_create(ctx, 1 << 30, 6)
    try:
        # the probe arrives in the middle of the stream of requests
        first = {bkts.bkts_server_submit(srv, r.request(bkts)): r for r in mix[:6]}
        time.sleep(0.02)
        tp = bkts.bkts_server_submit(srv, probe.request(bkts))
        rest = {bkts.bkts_server_submit(srv, r.request(bkts)): r for r in mix[6:]}
        want = {**first, tp: probe, **rest}
        got = {}
        t_end = time.time() + 180
        while len(got) < len(want):
            assert time.time() < t_end
            bkts.bkts_server_wait(srv, 1, 1.0)
            for res in bkts.bkts_server_poll(srv):
                got[res.ticket] = res
        st = bkts.bkts_server_stats_get(srv)
    finally:
        bkts.bkts_server_destroy(srv)
    np.testing.assert_array_equal(probe.out.cpu().numpy(), ref)
    assert got[tp].outer_iterations == res_alone.outer_iterations
    assert got[tp].krylov_iterations == res_alone.krylov_iterations
    for t, r in want.items():
        check_against_oracle(r, got[t])
    assert st.max_active >= 2, st.max_active
    assert st.grouped_launches > 0
    # continuous batching: some request was admitted while another one was still running
    spans = sorted((got[t].t_admit, got[t].t_done) for t in want)
    assert any(spans[i + 1][0] < spans[i][1] for i in range(len(spans) - 1))
    say(f"  rounds={st.rounds} launches={st.grouped_launches} max_active={st.max_active}")


@pytest.mark.parametrize("mode", [0, 1])
def test_admission_respects_budget(env, mode):
    torch, bkts, ctx = env
    say(f"serving budget, mode {mode}")
    reqs = [Req(torch, (64, 64), 16, 200 + i, mode=mode) for i in range(4)]
    torch.cuda.synchronize()
    fp = None
    srv = bkts.bkts_server_create(ctx, 1 << 40, 8)
    try:
        fp = run_all(bkts, srv, reqs[:1])[reqs[0]].footprint_bytes
    finally:
        bkts.bkts_server_destroy(srv)
    budget = int(fp * 2.5)  # two at a time
    srv = bkts.bkts_server_create(ctx, budget, 8)
    try:
        got = run_all(bkts, srv, reqs)
        st = bkts.bkts_server_stats_get(srv)
    finally:
        bkts.bkts_server_destroy(srv)
    assert st.bytes_peak <= budget
    assert st.max_active == 2
    for r, res in got.items():
        check_against_oracle(r, res)


def test_submit_errors(env):
    torch, bkts, ctx = env
    srv = bkts.bkts_server_create(ctx, 1 << 20, 2)
    try:
        r = Req(torch, (128, 128), 16, 1)
        with pytest.raises(bkts.BktsError) as e:
            bkts.bkts_server_submit(srv, r.request(bkts))  # needs more than 1 MiB
        assert e.value.status == bkts.BKTS_ENOMEM
        bad = r.request(bkts)
        bad.k = 33
        with pytest.raises(bkts.BktsError) as e:
            bkts.bkts_server_submit(srv, bad)
        assert e.value.status == bkts.BKTS_EINVAL
        small = Req(torch, (8, 8), 4, 2)
        for field, value in (("mode", 2), ("window", 5), ("window", -1)):
            bad = small.request(bkts)
            setattr(bad, field, value)
            with pytest.raises(bkts.BktsError) as e:
                bkts.bkts_server_submit(srv, bad)
            assert e.value.status == bkts.BKTS_EINVAL, (field, value)
        bad = Req(torch, (8, 8), 4, 2, method="sdirk2", mode=1).request(bkts)  # pipelined: implicit Euler only
        with pytest.raises(bkts.BktsError) as e:
            bkts.bkts_server_submit(srv, bad)
        assert e.value.status == bkts.BKTS_EINVAL
        assert bkts.bkts_server_poll(srv) == []
    finally:
        bkts.bkts_server_destroy(srv)
