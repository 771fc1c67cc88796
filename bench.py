"""Benchmark: pipelined block Krylov time stepping on one MI355X.

Workload (the 128^3 heterogeneous-diffusion case): 3-D unit cube, 128^3 cell-centred FV cells,
7-point diffusion with a lognormal coefficient (log-mean 0, log-std 2, Gaussian correlation
length 8 cells, seed 0, harmonic face means), homogeneous Dirichlet boundary, implicit Euler
with tau = 1e-3 from u0 = sin(pi x) sin(pi y) sin(pi z).  All inputs are seeded and synthetic.

A "step" is one accepted time step of Algorithm 1 (residual, block solves, shift), each step
converged to a front-column relative residual of 1e-8.  The block form uses k time columns
with FP32 block-CG inner solves (multigrid V-cycle preconditioner on the stencil form of the
operator) inside the FP64 outer refinement; the plain form is the same library at k = 1 in FP64
(inner = outer = 1e-8, i.e. one solve per step) with the same operator and preconditioner.

Prints ONE compact JSON line on stdout (the full record, with every leg and sweep, goes to
--full-out).  `value` = DOF * accepted steps / second of the block form, the median of --repeats
timed runs (each a fresh stepper: warmup steps, then the timed steps), inputs resident in HBM
before the timed region; `roofline` is the kernel category with the largest share of kernel time
in the median run, its average launch time measured with HIP events inside the library over the
timed region; `oracle_rel_error` is the error of the headline configuration's first steps against
the FP64 oracle's sequential steps; `cpu_baseline` is the oracle stepping a bounded sample of the
same workload on the host (plain C on every core, and the scipy form on one core beside it).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import statistics
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TIMER_PERIOD = 8  # time every 8th launch of each kernel (keeps the event overhead off the loop)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=16)
    p.add_argument("--warmup", type=int, default=16)
    p.add_argument("--repeats", type=int, default=5,
                   help="timed runs of the headline (fresh stepper, warmup + timed steps each); value = median")
    p.add_argument("--err-steps", type=int, default=3,
                   help="untimed headline steps from u0 checked against the oracle (0 = skip)")
    p.add_argument("--full-out", default="bench_out/bench_full.json",
                   help="where the full JSON record goes (the stdout line is the compact summary)")
    p.add_argument("--n", type=int, default=128)
    p.add_argument("--k", type=int, default=4)
    p.add_argument("--precision", choices=["f32", "f64"], default="f32")
    p.add_argument("--inner-rtol", type=float, default=0.1,
                   help="inner (FP32 block-CG) relative tolerance per outer iteration; the outer loop converges "
                        "every accepted step to 1e-8 regardless")
    p.add_argument("--format", choices=["stencil", "sell"], default="stencil",
                   help="storage of the 128^3 operator: the index-free stencil form (diagonal + one array per "
                        "neighbour offset) or SELL-C; the other format's block and plain forms are timed beside it")
    p.add_argument("--no-format-compare", dest="format_compare", action="store_false")
    p.add_argument("--precond", choices=["jacobi", "mg"], default="mg",
                   help="preconditioner of the inner block CG of the headline forms (mg needs the stencil format)")
    p.add_argument("--plain-steps", type=int, default=8)
    p.add_argument("--no-plain", action="store_true")
    p.add_argument("--no-cpu", action="store_true")
    p.add_argument("--cpu-steps", type=int, default=3)
    p.add_argument("--no-kernel-timers", action="store_true",
                   help="time the block form without the in-library kernel timers (no roofline)")
    p.add_argument("--calibrate-copy", action="store_true",
                   help="first run 3 plain 256 MiB device copies (reference dispatches for HBM counters)")
    p.add_argument("--serve-requests", type=int, default=512,
                   help="requests in the serving trace (0 = skip the serving leg)")
    p.add_argument("--serve-mode", type=int, default=1, choices=[0, 1],
                   help="0: grouped window splitting (Jacobi); 1: pipelined Algorithm 1 with multigrid on lanes")
    p.add_argument("--serve-rate", type=float, default=200.0, help="mean arrivals per second")
    p.add_argument("--serve-budget-gib", type=float, default=4.0)
    p.add_argument("--serve-slots", type=int, default=64)
    p.add_argument("--serve-inner-rtol", type=float, default=0.1)
    p.add_argument("--no-serve-plain", dest="serve_plain", action="store_false",
                   help="skip the plain FP64 one-at-a-time replay of the serving trace")
    p.add_argument("--nl-n", type=int, default=1024, help="nonlinear leg: grid n x n (0 = skip)")
    p.add_argument("--nl-k", type=int, default=16, help="nonlinear leg: window columns (8 steps x 2 stages)")
    p.add_argument("--nl-steps", type=int, default=8)
    p.add_argument("--nl-inner-rtol", type=float, default=0.1,
                   help="inner tolerance of the timed block form (the paper's 1e-5 is timed beside it)")
    p.add_argument("--ri-n", type=int, default=96, help="Richards leg: grid n^3 (0 = skip)")
    p.add_argument("--ri-k", type=int, default=16, help="Richards leg: window columns (implicit Euler steps)")
    p.add_argument("--ri-steps", type=int, default=4)
    p.add_argument("--ri-inner-rtol", type=float, default=1e-4,
                   help="inner tolerance (looser tolerances let Newton diverge at 96^3, tau=1e-3)")
    p.add_argument("--accel", type=str, default="4,8,16",
                   help="window-solve leg: comma list of window widths solved whole by FGMRES on the all-at-once "
                        "operator and by the plain splitting iteration (empty = skip)")
    p.add_argument("--accel-inner-rtol", type=float, default=0.1)
    p.add_argument("--firk-ks", type=str, default="2,4,8",
                   help="Radau IIA leg: window widths (2 columns per step) of the pipelined form ('' = skip)")
    p.add_argument("--firk-steps", type=int, default=4)
    p.add_argument("--firk-inner-rtol", type=float, default=0.1)
    p.add_argument("--spmm-ks", type=str, default="1,4,8,16,32",
                   help="block-operator sweep widths ('' = skip)")
    p.add_argument("--spmm-reps", type=int, default=30)
    p.add_argument("--sweep", type=str, default="1f32,4f64,4f32@0.01,8,16,32",
                   help="comma list of extra block forms to time: <k>[f32|f64][@inner_rtol] (defaults: --precision, "
                        "--inner-rtol)")
    return p.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_table(bkts, ctx):
    """Per-category launch duration from the library's in-dispatch event timers.  The duration of a
    category is the median of its timed launches (the mean is kept as mean_us): a short kernel's
    event interval now and then takes in a stall of the queue ahead of it, which the median ignores
    and the mean does not."""
    out = {}
    for name in bkts.KERNELS:
        n, ms, by = bkts.bkts_profile_query(ctx, name)
        if n:
            med_ms = statistics.median(bkts.bkts_profile_samples(ctx, name))
            tot = med_ms * n
            out[name] = {"launches": n, "avg_us": 1e3 * med_ms, "mean_us": 1e3 * ms / n, "total_ms": tot,
                         "bytes_per_launch": by / n, "GBps": (by / n / 1e9) / (med_ms / 1e3) if med_ms > 0 else None}
    tot = sum(v["total_ms"] for v in out.values())
    for v in out.values():
        v["share"] = v["total_ms"] / tot if tot > 0 else None
    return out


def kernel_name(cat, k, fmt="sell", precond="jacobi"):
    """The kernel behind a profiling category in the block-CG inner solve at width k."""
    row = k in (1, 2, 4)  # one thread per row; wider blocks use column tiles (MFMA for the updates)
    if row and fmt == "stencil" and precond == "mg":  # V-cycle fused into the iteration
        fused = {"cg_update": "rk_cg_xr_kernel", "cg_pupdate": "rk_cg_xp_kernel"}
        if cat in fused:
            return fused[cat]
    if fmt == "stencil":
        spmm = "rk_st_spmm_gram_kernel" if row else "st_spmm_kernel"
    else:
        spmm = "rk_spmm_gram_kernel" if row else spmm_kernel_name(k, "f32")
    return {"spmm": spmm,
            "cg_update": "rk_cg_update_kernel" if row else "mf_cg_update_kernel",
            "cg_pupdate": "rk_cg_pupdate_kernel" if row else "mf_cg_pupdate_kernel",
            "gram": "rk_gram_kernel" if row else "mf_gram_kernel",
            "residual": "st_residual_row_kernel" if (fmt == "stencil" and row) else "residual_kernel",
            "norms": "colnorm_kernel", "cast": "cast_scale_kernel",
            "small": "finalize / k x k kernels", "other": "vector kernels",
            "mg_restrict": "mg_restrict_kernel", "mg_prolong": "mg_prolong_kernel",
            "mg_coarse": "multigrid kernels of the coarser levels"}.get(cat, cat)


def roofline_of(kt, cat, k, precision, fmt="sell", precond="jacobi"):
    """HBM roofline of one profiling category: algorithmic bytes per launch / average launch time."""
    v = kt[cat]
    bpl = v["bytes_per_launch"]
    achieved = bpl / (v["avg_us"] * 1e-6) / 1e9
    name = kernel_name(cat, k, fmt, precond)
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic_for(name, precision, k), "kernel": name,
            "category": cat, "algorithmic_bytes_per_launch": bpl, "avg_launch_us": v["avg_us"],
            "timed_launches": v["launches"], "timer_period": TIMER_PERIOD,
            "share_of_kernel_time": v["share"]}


def traffic_for(kernel, precision, k):
    """Counter-based HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated) from the committed
    counter summary, or None when there is none for this kernel or its source changed since."""
    path = os.path.join(ROOT, "profiles", "counters.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
        e = d.get(f"{kernel} {precision} k={k}")
        if not e:
            return None
        for src, sha in e["sources"].items():
            if hashlib.sha256(open(os.path.join(ROOT, src), "rb").read()).hexdigest() != sha:
                return None
        return e["hbm_bytes_per_launch"]
    except (OSError, ValueError, KeyError):
        return None


def spmm_kernel_name(k, precision, fmt="sell"):
    """Kernel that bkts_spmm launches on a uniform-width SELL operator (or the stencil form of a 3-D
    grid) at width k, for contiguous blocks."""
    kp = 1
    while kp < k:
        kp *= 2
    sv = 4 if precision == "f32" else 8
    if fmt == "stencil":
        return "st_tile_kernel" if k == kp and 64 <= kp * sv <= 256 else "st_spmm_kernel"
    return "spmm_coop_kernel" if kp * sv >= 64 else "spmm_ell_kernel"


def run_spmm_sweep(torch, bkts, ctx, a, kd, n):
    """Block operator alone at every width, FP64 and FP32, on the 128^3 lognormal operator.

    Three assembled copies of the operator and three (X, Y) pairs are used in rotation so that the
    working set of consecutive launches exceeds the 256 MiB Infinity Cache (each launch reads cold
    data). Time per launch comes from the library's in-dispatch event timers."""
    N = n[0] * n[1] * n[2]
    out = {"copy": stream_copy_rate(torch)}
    for fmt, code in (("sell", bkts.BKTS_FMT_SELL), ("stencil", bkts.BKTS_FMT_STENCIL)):
        out.update(spmm_sweep_format(torch, bkts, ctx, a, kd, n, N, fmt, code))
    return out


def stream_copy_rate(torch, mib=256, reps=12):
    """Practical streaming ceiling: device-to-device copies of `mib` MiB in rotation over three buffer
    pairs (cold in the Infinity Cache), read + write bytes over the median copy time."""
    n = (mib << 20) // 8
    src = [torch.full((n,), 1.0, dtype=torch.float64, device="cuda") for _ in range(3)]
    dst = [torch.empty_like(x) for x in src]
    times = []
    for i in range(reps + 3):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst[i % 3].copy_(src[i % 3])
        e1.record()
        e1.synchronize()
        if i >= 3:
            times.append(e0.elapsed_time(e1))
    del src, dst
    ms = statistics.median(times)
    gbs = 2.0 * (mib << 20) / (ms * 1e-3) / 1e9
    log(f"  copy {mib} MiB: {1e3 * ms:.1f} us  {gbs:.0f} GB/s  frac {gbs / HBM_PEAK_GBS:.3f}")
    return {"avg_us": 1e3 * ms, "GBps": gbs, "frac": gbs / HBM_PEAK_GBS, "bytes_per_copy": 2.0 * (mib << 20),
            "kernel": "device-to-device copy (torch copy_)"}


def spmm_sweep_format(torch, bkts, ctx, a, kd, n, N, fmt, code):
    ops = [bkts.bkts_fv_assemble(ctx, n, kappa=kd, fmt=code) for _ in range(3)]
    _, nnz = bkts.bkts_op_info(ops[0])
    out = {}
    for prec, dt, sv in (("f64", torch.float64, 8), ("f32", torch.float32, 4)):
        for k in [int(v) for v in a.spmm_ks.split(",") if v.strip()]:
            gen = torch.Generator(device="cuda").manual_seed(k)
            Xs = [torch.randn((N, k), dtype=dt, device="cuda", generator=gen) for _ in range(3)]
            Ys = [torch.empty_like(x) for x in Xs]
            for i in range(3):
                bkts.bkts_spmm(ctx, ops[i], Xs[i], Ys[i], alpha=1e3, beta=1.0)
            torch.cuda.synchronize()
            bkts.bkts_profile_enable(ctx, True, 1)
            for i in range(a.spmm_reps):
                j = i % 3
                bkts.bkts_spmm(ctx, ops[j], Xs[j], Ys[j], alpha=1e3, beta=1.0)
            torch.cuda.synchronize()
            cnt, ms, by = bkts.bkts_profile_query(ctx, "spmm")
            bkts.bkts_profile_enable(ctx, False)
            us = 1e3 * ms / cnt
            bpl = by / cnt
            gbs = bpl / (us * 1e-6) / 1e9
            key = f"{prec} k={k}" if fmt == "sell" else f"{fmt} {prec} k={k}"
            out[key] = {"avg_us": us, "GBps": gbs, "frac": gbs / HBM_PEAK_GBS,
                        "algorithmic_bytes_per_launch": bpl, "flop_per_byte": 2.0 * nnz * k / bpl,
                        "kernel": spmm_kernel_name(k, prec, fmt), "format": fmt, "launches": cnt,
                        "traffic": traffic_for(spmm_kernel_name(k, prec, fmt), prec, k)}
            log(f"  spmm {fmt:7s} {prec} k={k:2d}: {us:7.1f} us  {gbs:6.0f} GB/s  frac {gbs / HBM_PEAK_GBS:.3f}  "
                f"AI {2.0 * nnz * k / bpl:.3f} flop/B")
            del Xs, Ys
    for o in ops:
        bkts.bkts_op_destroy(o)
    torch.cuda.synchronize()
    return out


def calibrate_copy(torch):
    """Plain device-to-device copies of a known size (256 MiB), for scaling the HBM byte counters."""
    a = torch.empty(1 << 25, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    del a, b


def run_form(torch, bkts, ctx, op, y0, k, precision, inner_rtol, warmup, steps, profile, precond="jacobi"):
    """Time `steps` accepted steps of a persistent stepper after `warmup` untimed ones."""
    tc = bkts.bkts_tc_create(ctx, bkts.BKTS_IE, k, 1e-3)
    st = bkts.bkts_stepper_create(ctx, op, tc, y0)
    prec = bkts.BKTS_PRECISION_F32_REFINE if precision == "f32" else bkts.BKTS_PRECISION_F64
    pc = bkts.BKTS_PREC_MG if precond == "mg" else bkts.BKTS_PREC_JACOBI
    inner = bkts.solve_opts(precond=pc, precision=prec, rtol=inner_rtol, inner_rtol=inner_rtol, maxit=100000)
    N = y0.numel()
    try:
        if warmup:
            bkts.bkts_stepper_advance(st, warmup, inner=inner, outer_rtol=1e-8, max_outer=400)
        hist = torch.empty((steps, N), dtype=torch.float64, device="cuda")
        bkts.bkts_profile_enable(ctx, profile, period=TIMER_PERIOD)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = bkts.bkts_stepper_advance(st, steps, inner=inner, outer_rtol=1e-8, max_outer=400, y_hist=hist)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        kt = kernel_table(bkts, ctx) if profile else {}
        bkts.bkts_profile_enable(ctx, False)
        return dict(seconds=dt, info=info, kernels=kt, hist=hist, value=N * steps / dt)
    finally:
        bkts.bkts_stepper_destroy(st)
        bkts.bkts_tc_destroy(tc)


def run_serving(torch, bkts, ctx, a):
    """Replay a seeded Poisson trace of heterogeneous 2-D diffusion solves through the serving loop."""
    import numpy as np

    from paper_2504_02117_amd import inputs
    rng = np.random.default_rng(0)
    m = a.serve_requests
    gaps = rng.exponential(1.0 / a.serve_rate, m)
    arrivals = np.cumsum(gaps) - gaps[0]
    sizes = rng.choice([64, 128, 256, 512], m)
    widths = rng.choice([4, 8, 16, 32], m)
    reqs = []
    log(f"serving: building {m} requests")
    y0s = {}
    for i in range(m):
        n = (int(sizes[i]), int(sizes[i]))
        if n not in y0s:
            y0s[n] = torch.from_numpy(inputs.sin_product(n)).cuda()
        kd = torch.from_numpy(inputs.lognormal_field(n, 0.0, 2.0, 8.0, 1000 + i)).cuda()
        out = torch.empty((n[0] * n[1], int(widths[i])), dtype=torch.float64, device="cuda")
        reqs.append((n, kd, out))
        if (i + 1) % 128 == 0:
            log(f"  built {i + 1}")
    torch.cuda.synchronize()
    srv = bkts.bkts_server_create(ctx, int(a.serve_budget_gib * (1 << 30)), a.serve_slots)
    results = {}
    try:
        t0 = bkts.bkts_server_clock(srv)
        tickets = {}
        for i, (n, kd, out) in enumerate(reqs):
            while bkts.bkts_server_clock(srv) < t0 + arrivals[i]:
                for r in bkts.bkts_server_poll(srv):
                    results[r.ticket] = r
                time.sleep(min(5e-4, max(0.0, t0 + arrivals[i] - bkts.bkts_server_clock(srv))))
            req = bkts.make_request(n, y0s[n], out, int(widths[i]), 1e-3, kappa=kd, rtol=1e-8,
                                    inner_rtol=a.serve_inner_rtol, tag=i, mode=a.serve_mode)
            tickets[bkts.bkts_server_submit(srv, req)] = i
        log(f"  all {m} submitted at t={bkts.bkts_server_clock(srv) - t0:.2f} s, {len(results)} done")
        last = time.time()
        while len(results) < m:
            bkts.bkts_server_wait(srv, 1, 1.0)
            for r in bkts.bkts_server_poll(srv):
                results[r.ticket] = r
            if time.time() - last > 10.0:
                last = time.time()
                log(f"  {len(results)}/{m} done at t={bkts.bkts_server_clock(srv) - t0:.1f} s")
        st = bkts.bkts_server_stats_get(srv)
    finally:
        bkts.bkts_server_destroy(srv)
    lat, wait, work, bad = [], [], [], 0
    elem_it, outer_tot = 0.0, 0
    t_end = 0.0
    for t, r in results.items():
        i = tickets[t]
        arr = t0 + arrivals[i]
        lat.append(r.t_done - arr)
        wait.append(r.t_admit - arr)
        t_end = max(t_end, r.t_done)
        bad += r.status != 0
        work.append(sizes[i] ** 2 * widths[i])
        elem_it += float(r.krylov_iterations) * sizes[i] ** 2 * widths[i]
        outer_tot += r.outer_iterations
    makespan = t_end - t0
    fifo = run_serving_plain(torch, bkts, ctx, reqs, arrivals, widths, sizes, y0s) if a.serve_plain else None
    # oracle check of the smallest requests of the trace
    from oracle import fv, stepping
    errs = []
    for i in [j for j in range(m) if sizes[j] == 64][:2]:
        n, kd, out = reqs[i]
        K, b = fv.assemble_linear(n, kappa=kd.cpu().numpy())
        ys, _ = stepping.dirk_linear(K, b, y0s[n].cpu().numpy(), 1e-3, "ie", int(widths[i]))
        got = out.cpu().numpy()
        errs.append(max(np.linalg.norm(got[:, j] - ys[j + 1]) / np.linalg.norm(ys[j + 1]) for j in range(widths[i])))
    return {"requests": m, "failed": int(bad), "rate_per_s": a.serve_rate, "makespan_s": makespan,
            "throughput_dof_timesteps_per_s": float(np.sum(work)) / makespan,
            "latency_p50_ms": 1e3 * float(np.percentile(lat, 50)), "latency_p99_ms": 1e3 * float(np.percentile(lat, 99)),
            "queue_wait_p50_ms": 1e3 * float(np.percentile(wait, 50)),
            "queue_wait_p99_ms": 1e3 * float(np.percentile(wait, 99)),
            "rounds": st.rounds, "grouped_launches": st.grouped_launches, "max_active": st.max_active,
            "mean_outer_iterations": outer_tot / m,
            "krylov_element_iterations": elem_it,
            "inner_stream_GBps": 44.0 * elem_it / makespan / 1e9,
            "hbm_budget_bytes": int(a.serve_budget_gib * (1 << 30)), "hbm_peak_reserved_bytes": st.bytes_peak,
            "oracle_max_rel_err_sampled": max(errs) if errs else None, "inner_rtol": a.serve_inner_rtol,
            "plain_fifo": fifo,
            "speedup_vs_plain_fifo": (fifo["makespan_s"] / makespan) if fifo else None,
            "mode": a.serve_mode,
            "workload": "2-D lognormal diffusion (log-std 2, corr. 8 cells, seed 1000+i), n in {64,128,256,512}, "
                        "k in {4,8,16,32}, implicit Euler tau=1e-3, k steps per request, Poisson arrivals; "
                        + ("pipelined Algorithm 1 (window min(k,4)), FP32 multigrid block CG inside FP64 to 1e-8 "
                           "per step, on worker lanes" if a.serve_mode == 1 else
                           "one window of k steps by grouped splitting, FP32 Jacobi block CG inside FP64 "
                           "Newton to 1e-8")}


def run_serving_plain(torch, bkts, ctx, reqs, arrivals, widths, sizes, y0s):
    """The same trace served one request at a time in arrival order by plain FP64 k = 1 stepping (CG
    preconditioned by the same multigrid V-cycle on the stencil form, inner = outer = 1e-8): each
    request's operator is assembled when it starts, and its k steps are taken one after another.
    Arrivals are replayed on the same clock as the served form."""
    import numpy as np
    log(f"serving baseline: plain FP64 k=1 stepping, one request at a time in arrival order")
    inner = bkts.solve_opts(precond=bkts.BKTS_PREC_MG, precision=bkts.BKTS_PRECISION_F64, rtol=1e-8,
                            inner_rtol=1e-8, maxit=100000)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat, done, its = [], 0.0, 0
    for i, (n, kd, out) in enumerate(reqs):
        now = time.perf_counter() - t0
        if now < arrivals[i]:
            time.sleep(arrivals[i] - now)
        k = int(widths[i])
        op = bkts.bkts_fv_assemble(ctx, n, kappa=kd, fmt=bkts.BKTS_FMT_STENCIL)
        tc = bkts.bkts_tc_create(ctx, bkts.BKTS_IE, 1, 1e-3)
        st = bkts.bkts_stepper_create(ctx, op, tc, y0s[n])
        hist = torch.empty((k, n[0] * n[1]), dtype=torch.float64, device="cuda")
        try:
            info = bkts.bkts_stepper_advance(st, k, inner=inner, outer_rtol=1e-8, max_outer=400, y_hist=hist)
            its += info.krylov_iterations
            torch.empty_like(out).copy_(hist.t())  # the result in the served layout (N x k)
            torch.cuda.synchronize()
        finally:
            bkts.bkts_stepper_destroy(st)
            bkts.bkts_tc_destroy(tc)
            bkts.bkts_op_destroy(op)
        done = time.perf_counter() - t0
        lat.append(done - arrivals[i])
    work = float(np.sum(np.asarray(sizes, dtype=np.float64) ** 2 * widths))
    log(f"  plain FIFO: makespan {done:.2f} s, {work / done:.4g} DOF*steps/s, p50 "
        f"{1e3 * np.percentile(lat, 50):.0f} ms, p99 {1e3 * np.percentile(lat, 99):.0f} ms")
    return {"makespan_s": done, "throughput_dof_timesteps_per_s": work / done,
            "latency_p50_ms": 1e3 * float(np.percentile(lat, 50)),
            "latency_p99_ms": 1e3 * float(np.percentile(lat, 99)), "krylov_iterations": its,
            "config": "FP64 k=1 CG + multigrid (stencil form), inner = outer = 1e-8, one request at a time, "
                      "operator assembled per request"}


def run_nonlinear(torch, bkts, ctx, a):
    """Newton form of Algorithm 1: D(u) = 1 + u^2, r(u) = -u^3, zero flux, SDIRK2, tau = 1e-4."""
    import numpy as np

    from paper_2504_02117_amd import inputs

    def form(n, k, precision, steps, warmup, profile, tol, hist=False, precond=None):
        nl = bkts.bkts_nlop_create(ctx, n, dcoef=(1, 0, 1, 0), rcoef=(0, 0, 0, -1))
        tc = bkts.bkts_tc_create(ctx, bkts.BKTS_SDIRK2, k, 1e-4)
        y0 = torch.from_numpy(inputs.smooth_random(n, 0)).cuda()
        st = bkts.bkts_nl_stepper_create(ctx, nl, tc, y0)
        inner = bkts.solve_opts(krylov=bkts.BKTS_BICGSTAB, precision=precision, rtol=tol, inner_rtol=tol, maxit=20000)
        if precond is not None:
            inner.precond = precond
        N = n[0] * n[1]
        try:
            if warmup:
                bkts.bkts_stepper_advance(st, warmup, inner=inner, outer_rtol=1e-8, max_outer=400)
            h = torch.empty((steps, N), dtype=torch.float64, device="cuda") if hist else None
            bkts.bkts_profile_enable(ctx, profile, period=TIMER_PERIOD)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = bkts.bkts_stepper_advance(st, steps, inner=inner, outer_rtol=1e-8, max_outer=400, y_hist=h)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            kt = kernel_table(bkts, ctx) if profile else {}
            bkts.bkts_profile_enable(ctx, False)
            return dict(seconds=dt, info=info, kernels=kt, value=N * steps / dt, hist=h, y0=y0)
        finally:
            bkts.bkts_stepper_destroy(st)
            bkts.bkts_tc_destroy(tc)
            bkts.bkts_nlop_destroy(nl)

    n = (a.nl_n, a.nl_n)
    F32, F64 = bkts.BKTS_PRECISION_F32_REFINE, bkts.BKTS_PRECISION_F64
    MG = bkts.BKTS_PREC_MG
    log(f"nonlinear leg {n}: block k={a.nl_k} FP32 inner {a.nl_inner_rtol:g}, {a.nl_steps} steps, multigrid")
    blk = form(n, a.nl_k, F32, a.nl_steps, 2, True, a.nl_inner_rtol, precond=MG)
    log(f"  {blk['value']:.4g} DOF*steps/s, outer={blk['info'].outer_iterations} krylov={blk['info'].krylov_iterations}")
    jac = form(n, a.nl_k, F32, a.nl_steps, 2, False, a.nl_inner_rtol)
    log(f"  block k={a.nl_k} with Jacobi: {jac['value']:.4g} DOF*steps/s")
    paper = form(n, a.nl_k, F32, a.nl_steps, 2, False, 1e-5)
    log(f"  block, inner 1e-5: {paper['value']:.4g} DOF*steps/s")
    narrow = form(n, 4, F32, a.nl_steps, 2, False, a.nl_inner_rtol)
    log(f"  block k=4 (2 steps x 2 stages), inner {a.nl_inner_rtol:g}: {narrow['value']:.4g} DOF*steps/s")
    plains = {tol: form(n, 1, F64, max(2, a.nl_steps // 2), 1, False, tol) for tol in (1e-5, a.nl_inner_rtol)}
    best = max(plains, key=lambda t: plains[t]["value"])
    pl = plains[best]
    log(f"  plain k=1 FP64: " + ", ".join(f"inner {t:g}: {v['value']:.4g}" for t, v in plains.items()))
    # BiCGStab preconditioned by the V-cycle of each Jacobian's symmetric part
    mg_k4 = form(n, 4, F32, a.nl_steps, 2, False, a.nl_inner_rtol, precond=MG)
    mg_plain = form(n, 1, F64, max(2, a.nl_steps // 2), 1, False, a.nl_inner_rtol, precond=MG)
    log(f"  multigrid: block k=4 {mg_k4['value']:.4g}, plain k=1 FP64 {mg_plain['value']:.4g} DOF*steps/s "
        f"(krylov {mg_k4['info'].krylov_iterations} and {mg_plain['info'].krylov_iterations})")
    # parity of the same configuration at 256^2 against the oracle's per-stage Newton
    from oracle import fv as ofv, stepping
    m = (256, 256)
    chk = form(m, a.nl_k, F32, 4, 0, False, a.nl_inner_rtol, hist=True, precond=MG)
    ref = ofv.NonlinearDiffusionReaction(m, dcoef=(1, 0, 1), rcoef=(0, 0, 0, -1))
    ys, _, _ = stepping.dirk_nonlinear(ref, chk["y0"].cpu().numpy(), 1e-4, "sdirk2", 4)
    got = chk["hist"].cpu().numpy()
    err = max(float(np.linalg.norm(got[s_] - ys[s_ + 1]) / np.linalg.norm(ys[s_ + 1])) for s_ in range(4))
    roof = None
    if blk["kernels"]:
        dom = max((c for c in blk["kernels"] if c not in ("small", "other", "mg_coarse")),
                  key=lambda c: blk["kernels"][c]["total_ms"])
        roof = roofline_of(blk["kernels"], dom, a.nl_k, "f32")
        roof["kernel"] = {"spmm": spmm_kernel_name(a.nl_k, "f32"), "residual": "nl_residual_kernel",
                          "norms": "coldots_kernel (BiCGStab column dots) and colnorm_kernel"}.get(dom, roof["kernel"])
    return {"workload": f"nonlinear diffusion-reaction {a.nl_n}^2 FV, D(u)=1+u^2, r(u)=-u^3, zero flux, SDIRK2 "
                        f"tau=1e-4, {a.nl_k} columns ({a.nl_k // 2} steps x 2 stages), Newton to 1e-8, per-column "
                        f"(vectorized) BiCGStab inner {a.nl_inner_rtol:g} in FP32 preconditioned by the multigrid "
                        f"V-cycle of the symmetric part of each Newton Jacobian (the 'jacobi', 'k4' and 'plain' entries "
                        f"and the inner 1e-5 form: Jacobi), seeded smooth u0 in [0,1]",
            "value": blk["value"], "unit": "DOF*timesteps/s", "ms_per_step": 1e3 * blk["seconds"] / a.nl_steps,
            "outer_iterations": blk["info"].outer_iterations, "krylov_iterations": blk["info"].krylov_iterations,
            "paper_inner_1e-5": {"value": paper["value"], "outer_iterations": paper["info"].outer_iterations,
                                 "krylov_iterations": paper["info"].krylov_iterations},
            "k4": {"value": narrow["value"], "outer_iterations": narrow["info"].outer_iterations},
            "multigrid": {"k4": mg_k4["value"], "plain": mg_plain["value"],
                          "krylov_iterations": {"k4": mg_k4["info"].krylov_iterations,
                                                "plain": mg_plain["info"].krylov_iterations}},
            "plain": {"value": pl["value"], "config": f"k=1 (stage by stage), FP64 BiCGStab, inner {best:g} (the "
                                                      f"faster of 1e-5 and {a.nl_inner_rtol:g}), outer 1e-8",
                      "all": {f"{t:g}": v["value"] for t, v in plains.items()}},
            "jacobi": {"value": jac["value"], "krylov_iterations": jac["info"].krylov_iterations},
            "speedup_vs_plain": blk["value"] / max(pl["value"], mg_plain["value"]),
            "oracle_max_rel_err_256": err, "roofline": roof,
            "kernels": {kk: {"avg_us": vv["avg_us"], "GBps": vv["GBps"]} for kk, vv in blk["kernels"].items()}}


def run_accel(torch, bkts, ctx, a, op, u0):
    """One implicit-Euler window of k steps on the 128^3 operator, solved whole to ||R||_F <= 1e-8 ||F||_F:
    FGMRES(30) on the all-at-once operator with the block-CG J^-1 solve as right preconditioner, against the
    plain splitting iteration with the same inner solve."""
    tau = 1e-3
    N = u0.shape[0]
    out, keep = {}, None
    for kk in [int(v) for v in a.accel.split(",") if v.strip()]:
        tc = bkts.bkts_tc_create(ctx, bkts.BKTS_IE, kk, tau)
        B0 = (u0 / tau).reshape(N, 1).contiguous()
        inner = bkts.solve_opts(krylov=bkts.BKTS_CG, precision=bkts.BKTS_PRECISION_F32_REFINE,
                                precond=bkts.BKTS_PREC_MG if a.precond == "mg" else bkts.BKTS_PREC_JACOBI,
                                rtol=a.accel_inner_rtol, inner_rtol=a.accel_inner_rtol, maxit=4000)
        try:
            row = {}
            for name, method in (("fgmres", bkts.BKTS_WINDOW_FGMRES), ("splitting", bkts.BKTS_WINDOW_SPLITTING)):
                Y = u0.reshape(N, 1).repeat(1, kk).contiguous()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                info = bkts.bkts_window_solve(ctx, op, tc, Y, B0=B0, method=method, inner=inner, rtol=1e-8,
                                              restart=30, maxit=200)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                row[name] = {"value": N * kk / dt, "seconds": dt, "iterations": info.iterations,
                             "precond_applications": info.precond_applications,
                             "inner_iterations": info.inner_iterations, "rel_residual": info.rel_residual}
                log(f"  window k={kk} {name}: {N * kk / dt:.4g} DOF*steps/s, {info.iterations} its, "
                    f"{info.precond_applications} J-solves, {info.inner_iterations} inner its, "
                    f"rel. residual {info.rel_residual:.2e}")
                if keep is None and name == "fgmres":
                    keep = (kk, Y.cpu().numpy())
                del Y
            row["fgmres_speedup_vs_splitting"] = row["fgmres"]["value"] / row["splitting"]["value"]
            out[f"k={kk}"] = row
        finally:
            bkts.bkts_tc_destroy(tc)
    return {"workload": f"heterogeneous diffusion {a.n}^3 (the headline operator), one implicit-Euler window of k "
                        f"steps from u0 solved whole to ||R||_F <= 1e-8 ||F||_F; J^-1 = FP32 block CG + {a.precond} "
                        f"at inner rtol {a.accel_inner_rtol:g}; FGMRES restart 30",
            "unit": "DOF*timesteps/s", "forms": out}, keep


def run_firk(torch, bkts, ctx, a, op, u0, kd, n):
    """2-stage Radau IIA on the 128^3 operator (fully implicit; averaged splitting coefficient).

    Forms, each advancing the same number of steps from u0 to a 1e-8 residual per accepted step:
    Algorithm 1 accepting whole steps with windows of 1, 2 and 4 steps (2, 4, 8 columns), and
    sequential stepping in which every step's 2-column window is solved by FGMRES on the
    all-at-once operator (right-preconditioned by the block J^-1 solve) or by the plain splitting."""
    import numpy as np
    tau, steps = 1e-3, a.firk_steps
    N = u0.shape[0]
    prec = bkts.BKTS_PRECISION_F32_REFINE
    inner = bkts.solve_opts(krylov=bkts.BKTS_CG, precision=prec, rtol=a.firk_inner_rtol,
                            precond=bkts.BKTS_PREC_MG if a.precond == "mg" else bkts.BKTS_PREC_JACOBI,
                            inner_rtol=a.firk_inner_rtol, maxit=100000)
    forms = {}
    for kk in [int(v) for v in a.firk_ks.split(",") if v.strip()]:
        tc = bkts.bkts_tc_create(ctx, bkts.BKTS_RADAU2, kk, tau)
        st = bkts.bkts_stepper_create(ctx, op, tc, u0)
        try:
            bkts.bkts_stepper_advance(st, 1, inner=inner, outer_rtol=1e-8, max_outer=1000)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = bkts.bkts_stepper_advance(st, steps, inner=inner, outer_rtol=1e-8, max_outer=1000)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
        finally:
            bkts.bkts_stepper_destroy(st)
            bkts.bkts_tc_destroy(tc)
        forms[f"pipelined k={kk} ({kk // 2} steps)"] = {
            "value": N * steps / dt, "outer_iterations": info.outer_iterations,
            "krylov_iterations": info.krylov_iterations}
        log(f"  Radau IIA pipelined k={kk}: {N * steps / dt:.4g} DOF*steps/s, outer {info.outer_iterations}, "
            f"krylov {info.krylov_iterations}")
    tc = bkts.bkts_tc_create(ctx, bkts.BKTS_RADAU2, 2, tau)
    try:
        for name, method in (("fgmres", bkts.BKTS_WINDOW_FGMRES), ("splitting", bkts.BKTS_WINDOW_SPLITTING)):
            y = u0.clone()
            its = pre = inn = 0
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                B0 = (y / tau).reshape(N, 1).repeat(1, 2).contiguous()
                Y = y.reshape(N, 1).repeat(1, 2).contiguous()
                info = bkts.bkts_window_solve(ctx, op, tc, Y, B0=B0, method=method, inner=inner, rtol=1e-8,
                                              restart=30, maxit=1000)
                its += info.iterations
                pre += info.precond_applications
                inn += info.inner_iterations
                y = Y[:, 1].contiguous()
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            forms[f"sequential window {name}"] = {"value": N * steps / dt, "outer_iterations": its,
                                                  "precond_applications": pre, "krylov_iterations": inn}
            log(f"  Radau IIA sequential {name}: {N * steps / dt:.4g} DOF*steps/s, {its} its, {pre} J-solves")
    finally:
        bkts.bkts_tc_destroy(tc)
    # oracle check on a small grid: pipelined k=4 against sequential coupled-stage stepping
    from oracle import fv, stepping
    m = (16, 16, 16)
    kap = inputs_lognormal(m)
    K, b = fv.assemble_linear(m, kappa=kap)
    y0 = u0_small(m)
    op_s = bkts.bkts_fv_assemble(ctx, m, kappa=torch.from_numpy(kap).cuda(), fmt=bkts.BKTS_FMT_STENCIL)
    tc = bkts.bkts_tc_create(ctx, bkts.BKTS_RADAU2, 4, tau)
    try:
        hist = torch.empty((4, y0.shape[0]), dtype=torch.float64, device="cuda")
        bkts.bkts_advance(ctx, op_s, tc, torch.from_numpy(y0).cuda(), 4, inner=inner, outer_rtol=1e-8,
                          max_outer=1000, y_hist=hist)
        ys, _ = stepping.rk_linear(K, b, y0, tau, "radau2", 4)
        got = hist.cpu().numpy()
        err = max(np.linalg.norm(got[s] - ys[s + 1]) / np.linalg.norm(ys[s + 1]) for s in range(4))
    finally:
        bkts.bkts_tc_destroy(tc)
        bkts.bkts_op_destroy(op_s)
    best = max(forms, key=lambda f: forms[f]["value"])
    return {"workload": f"heterogeneous diffusion {a.n}^3 (the headline operator), 2-stage Radau IIA tau=1e-3, "
                        f"{steps} steps to a 1e-8 residual per accepted step, averaged splitting coefficient "
                        f"|det A|^(1/2), J^-1 = FP32 block CG + {a.precond} at inner rtol {a.firk_inner_rtol}",
            "unit": "DOF*timesteps/s", "forms": forms, "best": best,
            "oracle_max_rel_err_16cubed": err}


def inputs_lognormal(m):
    from paper_2504_02117_amd import inputs
    return inputs.lognormal_field(m, 0.0, 2.0, 8.0 * m[0] / 128.0, 0)


def u0_small(m):
    from paper_2504_02117_amd import inputs
    return inputs.sin_product(m)


def run_richards(torch, bkts, ctx, a):
    """Richards' equation (Sec. 4.3): van Genuchten closure (alpha=2, n=2, theta_r=0.05, theta_s=0.4),
    lognormal Ks (log-std 1.5, corr. 8 cells), hydrostatic start psi0 = -z, Dirichlet psi = -0.3 on top,
    free drainage below, implicit Euler tau = 1e-3, Newton to 1e-8."""
    import numpy as np

    from paper_2504_02117_amd import inputs

    tau, g = 1e-3, -0.3

    def setup(n, corr):
        ks = torch.from_numpy(inputs.lognormal_field(n, 0.0, 1.5, corr, 1).ravel()).cuda()
        z = (np.arange(n[2]) + 0.5) / n[2]
        y0 = np.ascontiguousarray(np.broadcast_to(-z[:, None, None], inputs.field_shape(n)).ravel())
        return ks, y0

    def form(n, ks, y0, k, krylov, precision, steps, warmup, profile, hist=False, precond=None):
        nl = bkts.bkts_richards_create(ctx, n, ks, top=bkts.BKTS_RI_DIRICHLET, top_value=g,
                                       bottom=bkts.BKTS_RI_FREE_DRAINAGE)
        tc = bkts.bkts_tc_create(ctx, bkts.BKTS_IE, k, tau)
        st = bkts.bkts_nl_stepper_create(ctx, nl, tc, torch.from_numpy(y0).cuda())
        inner = bkts.solve_opts(krylov=krylov, precision=precision, rtol=a.ri_inner_rtol,
                                inner_rtol=a.ri_inner_rtol, maxit=4000, restart=30)
        if precond is not None:
            inner.precond = precond
        N = n[0] * n[1] * n[2]
        t_start = time.perf_counter()

        def cb(step, t, y, user):
            log(f"    step {step} ({time.perf_counter() - t_start:.1f} s)")
        try:
            if warmup:
                bkts.bkts_stepper_advance(st, warmup, inner=inner, outer_rtol=1e-8, max_outer=60, cb=cb)
            h = torch.empty((steps, N), dtype=torch.float64, device="cuda") if hist else None
            bkts.bkts_profile_enable(ctx, profile, period=TIMER_PERIOD)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = bkts.bkts_stepper_advance(st, steps, inner=inner, outer_rtol=1e-8, max_outer=60, y_hist=h)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            kt = kernel_table(bkts, ctx) if profile else {}
            bkts.bkts_profile_enable(ctx, False)
            return dict(seconds=dt, info=info, kernels=kt, value=N * steps / dt, hist=h)
        finally:
            bkts.bkts_stepper_destroy(st)
            bkts.bkts_tc_destroy(tc)
            bkts.bkts_nlop_destroy(nl)

    GM, BI = bkts.BKTS_GMRES, bkts.BKTS_BICGSTAB
    F32, F64 = bkts.BKTS_PRECISION_F32_REFINE, bkts.BKTS_PRECISION_F64
    n = (a.ri_n,) * 3
    ks, y0 = setup(n, 8.0)
    MG = bkts.BKTS_PREC_MG
    res = {}
    # Jacobi forms, then BiCGStab preconditioned by the V-cycle of the Jacobian's symmetric part
    for name, k, kry, prec, pc in (("block_gmres", a.ri_k, GM, F32, None), ("block_bicgstab", a.ri_k, BI, F32, None),
                                   ("block_bicgstab_k4", 4, BI, F32, None),  # the width the paper finds best
                                   ("plain_gmres", 1, GM, F64, None), ("plain_bicgstab", 1, BI, F64, None),
                                   ("block_gmres_mg", a.ri_k, GM, F32, MG),
                                   ("block_bicgstab_mg", a.ri_k, BI, F32, MG), ("block_bicgstab_k4_mg", 4, BI, F32, MG),
                                   ("plain_bicgstab_mg", 1, BI, F64, MG)):
        log(f"Richards leg {n}: {name} k={k}, inner {a.ri_inner_rtol:g}, {a.ri_steps} steps")
        r = form(n, ks, y0, k, kry, prec, a.ri_steps, 1, True, precond=pc)
        log(f"  {r['value']:.4g} DOF*steps/s, outer={r['info'].outer_iterations} "
            f"krylov={r['info'].krylov_iterations}")
        res[name] = r
    # parity of the block GMRES configuration on a 16 x 16 x 20 grid against sequential implicit Euler
    from oracle import richards as ori
    m = (16, 16, 20)
    ks_m, y0_m = setup(m, 8.0 * 16 / 96)
    chk = form(m, ks_m, y0_m, a.ri_k, GM, F32, 4, 0, False, hist=True, precond=MG)
    ref = ori.Richards(m, ks_m.cpu().numpy(), ori.VanGenuchten(), top=("dirichlet", g), bottom="free_drainage")
    ys, _ = ori.implicit_euler(ref, y0_m, tau, 4)
    got = chk["hist"].cpu().numpy()
    err = max(float(np.abs(got[s_] - ys[s_ + 1]).max() / np.abs(ys[s_ + 1]).max()) for s_ in range(4))
    blk = res["block_gmres_mg"]  # the configured form (Newton + block GMRES, k columns) with the V-cycle
    roof = None
    if blk["kernels"]:
        dom = max((c for c in blk["kernels"] if c not in ("small", "other", "mg_coarse")),
                  key=lambda c: blk["kernels"][c]["total_ms"])
        roof = roofline_of(blk["kernels"], dom, a.ri_k, "f32")
        roof["kernel"] = {"spmm": spmm_kernel_name(a.ri_k, "f32"), "residual": "nl_residual_kernel",
                          "gram": "mf_mgram_kernel and mf_gram_kernel (block Gram-Schmidt)"}.get(dom, roof["kernel"])
    best = max(res, key=lambda t: res[t]["value"])
    return {"workload": f"Richards' equation {a.ri_n}^3 FV, van Genuchten alpha=2 n=2 theta_r=0.05 theta_s=0.4, "
                        f"lognormal Ks (log-std 1.5, corr. 8 cells), psi0=-z, Dirichlet psi=-0.3 on top, free "
                        f"drainage below, implicit Euler tau=1e-3, {a.ri_k} columns, Newton to 1e-8, block GMRES(30) "
                        f"inner {a.ri_inner_rtol:g} in FP32 with FP64 residuals, preconditioned by the multigrid V-cycle "
                        f"of the symmetric part of each Newton Jacobian (value: block_gmres_mg; forms without _mg: Jacobi)",
            "value": blk["value"], "unit": "DOF*timesteps/s", "ms_per_step": 1e3 * blk["seconds"] / a.ri_steps,
            "forms": {kk: {"value": v["value"], "outer_iterations": v["info"].outer_iterations,
                           "krylov_iterations": v["info"].krylov_iterations,
                           "kernels": {c: {"avg_us": x["avg_us"], "launches": x["launches"], "share": x["share"]}
                                       for c, x in v["kernels"].items()}} for kk, v in res.items()},
            "fastest_form": best,
            "speedup_vs_plain": blk["value"] / max(v["value"] for kk, v in res.items() if kk.startswith("plain")),
            "best_block_vs_best_plain": max(v["value"] for kk, v in res.items() if kk.startswith("block"))
            / max(v["value"] for kk, v in res.items() if kk.startswith("plain")),
            "oracle_max_rel_err_16x16x20": err, "roofline": roof,
            "kernels": {kk: {"avg_us": vv["avg_us"], "GBps": vv["GBps"]} for kk, vv in blk["kernels"].items()}}


def headline_error(torch, bkts, ctx, op, y0, a, K, b, u0):
    """Relative 2-norm error of the headline configuration's first accepted steps against the oracle.

    An untimed run of the same stepper (k, precision, inner tolerance, preconditioner, outer 1e-8)
    from u0, against the oracle's sequential implicit Euler (plain C Jacobi-PCG to a 1e-12 residual,
    every host core)."""
    import numpy as np

    from oracle import cstep
    steps = a.err_steps
    r = run_form(torch, bkts, ctx, op, y0, a.k, a.precision, a.inner_rtol, 0, steps, False, a.precond)
    got = r["hist"].cpu().numpy()
    t = time.perf_counter()
    ys, its, used = cstep.ie_steps(K, b, u0, 1e-3, steps, rtol=1e-12)
    log(f"  oracle reference: {steps} steps to 1e-12 on {used} threads in {time.perf_counter() - t:.1f} s")
    errs = [float(np.linalg.norm(got[s] - ys[s + 1]) / np.linalg.norm(ys[s + 1])) for s in range(steps)]
    return {"max": max(errs), "per_step": errs, "steps": steps,
            "reference": "oracle sequential implicit Euler, Jacobi-PCG to a 1e-12 relative residual (plain C)"}


def cpu_baselines(a, K, b, u0, N):
    """The oracle timed on the host: the plain C form on every core (the reported value) and the
    scipy form on one core, each stepping a bounded sample of the headline workload to 1e-8."""
    from threadpoolctl import threadpool_limits

    from oracle import cstep, stepping
    steps = a.cpu_steps
    log(f"oracle time stepping on the host: {steps} IE steps to 1e-8, C on all cores, then scipy on one")
    t = time.perf_counter()
    _, its, used = cstep.ie_steps(K, b, u0, 1e-3, steps, rtol=1e-8)
    cs = time.perf_counter() - t
    with threadpool_limits(1):
        t = time.perf_counter()
        stepping.dirk_linear(K, b, u0, 1e-3, "ie", steps, solver="cg", rtol=1e-8)
        ps = time.perf_counter() - t
    log(f"  C on {used} threads: {N * steps / cs:.4g} DOF*steps/s; scipy on 1 core: {N * steps / ps:.4g}")
    return {"value": N * steps / cs, "unit": "DOF*timesteps/s", "cores": used, "kind": "oracle",
            "sample": f"{steps} implicit-Euler steps of the 128^3 workload, Jacobi-PCG to a 1e-8 relative "
                      f"residual per step, {cs:.1f} s (plain C oracle, OpenMP, {used} threads)",
            "one_core": {"value": N * steps / ps, "cores": 1, "seconds": ps,
                         "sample": f"the same {steps} steps with the scipy oracle (Jacobi-CG), BLAS limited to 1"},
            "cg_iterations": its, "cpu_model": _cpu_model(), "nproc": os.cpu_count()}


def pick_roofline(kt, k, precision, fmt, precond="jacobi"):
    """Roofline of the category with the largest share of kernel time (no exclusions), plus the
    categories made of small latency-bound launches, reported by their launch counts."""
    if not kt:
        return None, None
    dom = max(kt, key=lambda c: kt[c]["total_ms"])
    roof = roofline_of(kt, dom, k, precision, fmt, precond)
    lat = {c: {"launches": kt[c]["launches"], "avg_us": kt[c]["avg_us"], "share": kt[c]["share"]}
           for c in ("mg_coarse", "small") if c in kt}
    return roof, lat


def _r(x, d=4):
    """Round floats for the compact line."""
    if isinstance(x, float):
        return float(f"{x:.{d}g}")
    if isinstance(x, dict):
        return {kk: _r(v, d) for kk, v in x.items()}
    if isinstance(x, list):
        return [_r(v, d) for v in x]
    return x


def compact_line(out, full_path):
    """The one JSON line the driver reads: the contract's fields plus the headline's roofline, the
    CPU baseline, the error against the oracle and one figure per leg; the full record is written
    to `full_path`."""
    roof = out["roofline"]
    keep_roof = None if roof is None else {kk: roof[kk] for kk in (
        "bound", "achieved", "peak", "unit", "frac", "traffic", "kernel", "category", "avg_launch_us",
        "algorithmic_bytes_per_launch", "share_of_kernel_time")}
    sw = out.get("spmm_sweep") or {}
    spmm = {kk: {"us": v["avg_us"], "frac": v["frac"], "kernel": v["kernel"], "traffic": v.get("traffic")}
            for kk, v in sw.items()
            if kk.endswith("k=16") or kk.endswith("k=4")}
    if "copy" in sw:
        spmm["copy_256MiB"] = {"us": sw["copy"]["avg_us"], "frac": sw["copy"]["frac"]}
    cpu = out["cpu_baseline"]
    legs = {}
    if out.get("nonlinear"):
        nl = out["nonlinear"]
        legs["nonlinear_1024sq_k16"] = {"value": nl["value"], "k4": nl["k4"]["value"], "plain": nl["plain"]["value"],
                                        "oracle_err_256sq": nl["oracle_max_rel_err_256"]}
        if "multigrid" in nl:
            legs["nonlinear_1024sq_k16"].update(k4_mg=nl["multigrid"]["k4"], plain_mg=nl["multigrid"]["plain"])
    if out.get("richards"):
        ri = out["richards"]
        legs["richards_96cubed_k16"] = {f: v["value"] for f, v in ri["forms"].items()}
        legs["richards_96cubed_k16"]["oracle_err_16x16x20"] = ri["oracle_max_rel_err_16x16x20"]
    if out.get("fully_implicit"):
        fi = out["fully_implicit"]
        legs["radau2_128cubed"] = {"best": fi["best"], "value": fi["forms"][fi["best"]]["value"],
                                   "oracle_err_16cubed": fi["oracle_max_rel_err_16cubed"]}
    if out.get("window_acceleration"):
        wa = out["window_acceleration"]["forms"]
        legs["window_solve_128cubed"] = {kk: {"fgmres": v["fgmres"]["value"], "splitting": v["splitting"]["value"]}
                                         for kk, v in wa.items()}
    if out.get("serving"):
        sv = out["serving"]
        legs["serving"] = {"requests": sv["requests"], "mode": sv.get("mode"),
                           "throughput": sv["throughput_dof_timesteps_per_s"],
                           "p50_ms": sv["latency_p50_ms"], "p99_ms": sv["latency_p99_ms"],
                           "failed": sv["failed"], "oracle_err_sampled": sv["oracle_max_rel_err_sampled"],
                           "fifo_plain": None if not sv["plain_fifo"] else {
                               "throughput": sv["plain_fifo"]["throughput_dof_timesteps_per_s"],
                               "p50_ms": sv["plain_fifo"]["latency_p50_ms"],
                               "p99_ms": sv["plain_fifo"]["latency_p99_ms"]}}
    line = {kk: out[kk] for kk in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
                                   "higher_is_better", "scaling", "vs_baseline", "dtype", "data")}
    line["config"] = {kk: out["config"][kk] for kk in ("workload", "N", "k", "format", "precond", "inner_rtol")}
    line.update({
        "runs": out["runs"], "plain": out["plain"] and {"value": out["plain"]["value"],
                                                      "ms_per_step": out["plain"]["ms_per_step"]},
        "speedup_vs_plain": out["speedup_vs_plain"], "oracle_rel_error": out["oracle_rel_error"] and {
            "max": out["oracle_rel_error"]["max"], "steps": out["oracle_rel_error"]["steps"]},
        "roofline": keep_roof, "latency_bound": out["latency_bound"], "spmm_roofline": spmm or None,
        "cpu_baseline": cpu and {kk: cpu[kk] for kk in ("value", "unit", "cores", "kind", "sample")} | {
            "one_core": cpu["one_core"]["value"], "cpu_model": cpu["cpu_model"]},
        "legs": legs or None, "full_record": os.path.relpath(full_path, ROOT)})
    return json.dumps(_r(line), separators=(",", ":"))


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "bench.py runs on one GPU only: the sharded path (halo exchange over RCCL, "
                                   "k x k all-reduce) is designed but not built; run with --gpus 1"}))
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2504_02117_amd import bkts, inputs

    n = (a.n, a.n, a.n)
    N = a.n ** 3
    if a.calibrate_copy:
        calibrate_copy(torch)
    log(f"inputs {n}")
    kap = inputs.lognormal_field(n, 0.0, 2.0, 8.0, 0)
    u0 = inputs.sin_product(n)
    ctx = bkts.bkts_ctx_create(0, torch.cuda.current_stream())
    kd = torch.from_numpy(kap).cuda()
    y0 = torch.from_numpy(u0).cuda()
    torch.cuda.synchronize()
    t = time.perf_counter()
    fcode = {"stencil": bkts.BKTS_FMT_STENCIL, "sell": bkts.BKTS_FMT_SELL}
    op = bkts.bkts_fv_assemble(ctx, n, kappa=kd, fmt=fcode[a.format])
    setup_s = time.perf_counter() - t
    _, nnz = bkts.bkts_op_info(op)

    log(f"block form k={a.k} {a.precision}: {a.repeats} runs of warmup {a.warmup} + timed {a.steps}")
    runs = []
    for i in range(a.repeats):
        r = run_form(torch, bkts, ctx, op, y0, a.k, a.precision, a.inner_rtol, a.warmup, a.steps,
                     not a.no_kernel_timers, a.precond)
        log(f"  run {i + 1}: {r['value']:.4g} DOF*steps/s, outer={r['info'].outer_iterations} "
            f"krylov={r['info'].krylov_iterations}")
        if runs:
            r["hist"] = None
        runs.append(r)
    order = sorted(range(len(runs)), key=lambda i: runs[i]["value"])
    blk = runs[order[len(runs) // 2]]
    first_hist = runs[0]["hist"]
    result_hist = first_hist[-2:].double().cpu().numpy() if a.steps >= 2 else None
    del first_hist
    for r in runs:
        r["hist"] = None
    torch.cuda.synchronize()

    plain = None
    if not a.no_plain:
        log(f"plain form k=1 f64: timed {a.plain_steps}")
        pl = run_form(torch, bkts, ctx, op, y0, 1, "f64", 1e-8, 1, a.plain_steps, False, a.precond)
        plain = {"value": pl["value"], "ms_per_step": 1e3 * pl["seconds"] / a.plain_steps,
                 "krylov_iterations_per_step": pl["info"].krylov_iterations / a.plain_steps,
                 "config": f"k=1, FP64 block CG (= CG) + {a.precond}, inner = outer = 1e-8"}
        log(f"  {pl['value']:.4g} DOF*steps/s")

    sweep = {}
    for item in [v.strip() for v in a.sweep.split(",") if v.strip()]:
        prec, tol = a.precision, a.inner_rtol
        if "@" in item:
            item, t = item.split("@")
            tol = float(t)
        if item.endswith("f32") or item.endswith("f64"):
            prec, item = item[-3:], item[:-3]
        ks = int(item)
        r = run_form(torch, bkts, ctx, op, y0, ks, prec, tol, a.warmup, a.steps, True, a.precond)
        r["hist"] = None
        sp = r["kernels"].get("spmm", {})
        sv = 4 if prec == "f32" else 8
        bpl = (4 * N * sv if a.format == "stencil" else nnz * (sv + 4) + 4 * (N + 1)) + 2 * N * ks * sv
        dom = max(r["kernels"].items(), key=lambda kv: kv[1]["total_ms"])[0] if r["kernels"] else None
        sweep[f"k={ks} {prec} inner={tol:g}"] = {
            "value": r["value"], "outer": r["info"].outer_iterations, "krylov": r["info"].krylov_iterations,
            "spmm_avg_us": sp.get("avg_us"),
            "spmm_GBps": (bpl / (sp["avg_us"] * 1e-6) / 1e9) if sp else None,
            "spmm_frac": (bpl / (sp["avg_us"] * 1e-6) / 1e9 / HBM_PEAK_GBS) if sp else None,
            "spmm_kernel": kernel_name("spmm", ks, a.format), "spmm_flop_per_byte": 2.0 * nnz * ks / bpl,
            "dominant_kernel": dom,
            "kernels": {kk: {"avg_us": vv["avg_us"], "GBps": vv["GBps"]} for kk, vv in r["kernels"].items()}}
        log(f"  sweep k={ks} {prec} inner={tol:g}: {r['value']:.4g} DOF*steps/s (spmm {sp.get('avg_us', 0):.1f} us)")

    roof, lat = pick_roofline(blk["kernels"], a.k, a.precision, a.format, a.precond)
    spmm_roof = roofline_of(blk["kernels"], "spmm", a.k, a.precision, a.format) if "spmm" in blk["kernels"] else None

    formats = None
    if a.format_compare:
        # the headline's block and plain forms with the other operator storage and preconditioner
        formats = {f"{a.format}+{a.precond}": {"block": blk["value"], "plain": plain["value"] if plain else None,
                                              "krylov_iterations": blk["info"].krylov_iterations,
                                              "spmm_avg_us": blk["kernels"].get("spmm", {}).get("avg_us")}}
        for fmt, pc in (("stencil", "jacobi"), ("sell", "jacobi"), ("stencil", "mg")):
            key = f"{fmt}+{pc}"
            if key in formats:
                continue
            log(f"{key}: block form k={a.k} {a.precision} and plain k=1 f64 beside the headline's")
            op2 = bkts.bkts_fv_assemble(ctx, n, kappa=kd, fmt=fcode[fmt])
            try:
                b2 = run_form(torch, bkts, ctx, op2, y0, a.k, a.precision, a.inner_rtol, a.warmup, a.steps, True, pc)
                b2["hist"] = None
                p2 = None if a.no_plain else run_form(torch, bkts, ctx, op2, y0, 1, "f64", 1e-8, 1, a.plain_steps,
                                                      False, pc)
            finally:
                bkts.bkts_op_destroy(op2)
            sp2 = b2["kernels"].get("spmm", {})
            formats[key] = {"block": b2["value"], "plain": p2["value"] if p2 else None,
                            "krylov_iterations": b2["info"].krylov_iterations, "spmm_avg_us": sp2.get("avg_us")}
            log(f"  {key}: block {b2['value']:.4g}" + (f", plain {p2['value']:.4g}" if p2 else "") +
                f" DOF*steps/s, krylov {b2['info'].krylov_iterations} (spmm {sp2.get('avg_us', 0):.1f} us)")

    spmm_sweep = None
    if a.spmm_ks.strip():
        log(f"block-operator sweep: k in {a.spmm_ks}, FP64 and FP32, 3 rotating copies")
        spmm_sweep = run_spmm_sweep(torch, bkts, ctx, a, kd, n)

    accel, accel_keep = None, None
    if a.accel.strip():
        log(f"window-solve leg (outer acceleration): k in {a.accel}")
        accel, accel_keep = run_accel(torch, bkts, ctx, a, op, y0)

    firk = None
    if a.firk_ks.strip():
        log(f"fully implicit leg (Radau IIA): windows {a.firk_ks}")
        firk = run_firk(torch, bkts, ctx, a, op, y0, kd, n)
        log(f"  Radau IIA: oracle rel. error at 16^3 {firk['oracle_max_rel_err_16cubed']:.2e}")

    nonlinear = None
    if a.nl_n > 0:
        nonlinear = run_nonlinear(torch, bkts, ctx, a)
        log(f"  nonlinear: oracle rel. error at 256^2 {nonlinear['oracle_max_rel_err_256']:.2e}")

    richards = None
    if a.ri_n > 0:
        richards = run_richards(torch, bkts, ctx, a)
        log(f"  Richards: oracle rel. error at 16x16x20 {richards['oracle_max_rel_err_16x16x20']:.2e}")

    serving = None
    if a.serve_requests > 0:
        serving = run_serving(torch, bkts, ctx, a)
        log(f"  serving: {serving['throughput_dof_timesteps_per_s']:.4g} DOF*steps/s, p50 "
            f"{serving['latency_p50_ms']:.1f} ms, p99 {serving['latency_p99_ms']:.1f} ms, "
            f"makespan {serving['makespan_s']:.1f} s")

    cpu = None
    err = None
    oerr = None
    if not a.no_cpu or result_hist is not None or accel_keep is not None or a.err_steps > 0:
        from oracle import fv
        log("oracle assembly (CPU)")
        K, b = fv.assemble_linear(n, kappa=kap)
        if accel_keep is not None:
            # FP64 oracle residual of the first FGMRES window: Y A1^T + (K Y) A2^T - B0 (IE, b = 0)
            kk, Yw = accel_keep
            Rw = (Yw - np.concatenate([u0[:, None], Yw[:, :-1]], axis=1)) / 1e-3 + K @ Yw
            accel["oracle_rel_residual_first_window"] = float(np.linalg.norm(Rw) /
                                                              np.linalg.norm(u0 / 1e-3))
            log(f"  window k={kk}: oracle rel. residual {accel['oracle_rel_residual_first_window']:.2e}")
        if result_hist is not None:
            # FP64 oracle residual of the last accepted step of the first timed block run
            import scipy.sparse as sp
            J = (sp.identity(N) / 1e-3 + K).tocsr()
            r = J @ result_hist[1] - result_hist[0] / 1e-3 - b
            err = float(np.linalg.norm(r) / np.linalg.norm(result_hist[0] / 1e-3 + b))
        if a.err_steps > 0:
            log(f"error against the oracle: {a.err_steps} untimed steps of the headline configuration from u0")
            oerr = headline_error(torch, bkts, ctx, op, y0, a, K, b, u0)
            log(f"  relative errors {['%.2e' % e for e in oerr['per_step']]}")
        if not a.no_cpu:
            cpu = cpu_baselines(a, K, b, u0, N)

    vals = [r["value"] for r in runs]
    out = {
        "metric": "DOF·timesteps/s to 1e-8 residual (block vs plain); SpMM HBM GB/s; p50/p99",
        "value": blk["value"], "unit": "DOF*timesteps/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": 1e3 * blk["seconds"] / a.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32 inner / f64 outer" if a.precision == "f32" else "f64",
        "data": "synthetic (seeded lognormal field, sin-product initial state)",
        "config": {"workload": f"heterogeneous diffusion {a.n}^3 FV 7-point, lognormal kappa (log-std 2, corr. 8 "
                               f"cells), implicit Euler tau=1e-3, block width k={a.k}, {a.format} operator, "
                               f"block CG + {'multigrid V-cycle' if a.precond == 'mg' else 'Jacobi'}, "
                               f"{'FP32-inner + FP64 refinement' if a.precision == 'f32' else 'FP64'} to 1e-8",
                   "N": N, "nnz": nnz, "k": a.k, "inner_rtol": a.inner_rtol, "format": a.format,
                   "precond": a.precond,
                   "setup_s": setup_s},
        "runs": vals, "value_is": f"median of {len(vals)} runs of {a.steps} timed steps",
        "outer_iterations": blk["info"].outer_iterations, "krylov_iterations": blk["info"].krylov_iterations,
        "oracle_rel_error": oerr,
        "oracle_rel_residual_last_step": err,
        "plain": plain,
        "speedup_vs_plain": (blk["value"] / plain["value"]) if plain else None,
        "sweep": sweep or None,
        "formats": formats,
        "roofline": roof,
        "latency_bound": lat,
        "spmm_roofline": spmm_roof,
        "spmm_sweep": spmm_sweep,
        "kernels": blk["kernels"],
        "cpu_baseline": cpu,
        "window_acceleration": accel,
        "fully_implicit": firk,
        "nonlinear": nonlinear,
        "richards": richards,
        "serving": serving,
    }
    full_path = a.full_out if os.path.isabs(a.full_out) else os.path.join(ROOT, a.full_out)
    try:
        os.makedirs(os.path.dirname(full_path), exist_ok=True)
        with open(full_path, "w") as f:
            json.dump(out, f, indent=1)
    except OSError as e:
        log(f"could not write the full record to {full_path}: {e}")
    log(f"full record: {full_path}")
    bkts.bkts_op_destroy(op)
    torch.cuda.synchronize()
    bkts.bkts_ctx_destroy(ctx)
    print(compact_line(out, full_path), flush=True)


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


if __name__ == "__main__":
    main()
