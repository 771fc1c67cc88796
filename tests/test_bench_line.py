"""The benchmark's stdout line: the fields the contract names, every leg present, under 4 KB (the
record is read from the tail of the output), and valid JSON.  Host logic only (no GPU)."""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _kern(avg, share):
    return {"launches": 50, "avg_us": avg, "total_ms": 50 * avg / 1e3, "bytes_per_launch": 1e8, "GBps": 2e3,
            "share": share}


def _record():
    kt = {"spmm": _kern(30.1234567, 0.1), "cg_update": _kern(40.0, 0.2), "mg_coarse": _kern(7.0, 0.25),
          "small": _kern(4.5, 0.08)}
    roof, lat = bench.pick_roofline(kt, 4, "f32", "stencil")
    forms = {f"k={k}": {"fgmres": {"value": 1.23456789e8}, "splitting": {"value": 2.3456789e8}} for k in (4, 8, 16)}
    return {
        "metric": "DOF·timesteps/s to 1e-8 residual (block vs plain); SpMM HBM GB/s; p50/p99",
        "value": 6.5123456789e8, "unit": "DOF*timesteps/s", "n_gpus": 1, "steps": 20, "warmup": 5,
        "ms_per_step": 3.2123456, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 inner / f64 outer", "data": "synthetic (seeded lognormal field, sin-product initial state)",
        "config": {"workload": "heterogeneous diffusion 128^3 FV 7-point, lognormal kappa (log-std 2, corr. 8 "
                               "cells), implicit Euler tau=1e-3, block width k=4, stencil operator, block CG + "
                               "multigrid V-cycle, FP32-inner + FP64 refinement to 1e-8",
                   "N": 2097152, "nnz": 14581760, "k": 4, "inner_rtol": 0.1, "format": "stencil", "precond": "mg",
                   "setup_s": 0.1},
        "runs": [6.4e8, 6.5e8, 6.6e8, 6.55e8, 6.45e8],
        "oracle_rel_error": {"max": 1.1e-9, "per_step": [1e-10, 5e-10, 1.1e-9], "steps": 3, "reference": "x"},
        "plain": {"value": 2.5e8, "ms_per_step": 8.4, "krylov_iterations_per_step": 10, "config": "x"},
        "speedup_vs_plain": 2.6, "roofline": roof, "latency_bound": lat,
        "spmm_sweep": {f"{fmt}{p} k={k}": {"avg_us": 100.0, "frac": 0.5, "kernel": "st_spmm_kernel", "GBps": 4e3}
                       for fmt in ("", "stencil ") for p in ("f64", "f32") for k in (1, 4, 8, 16, 32)},
        "cpu_baseline": {"value": 2e6, "unit": "DOF*timesteps/s", "cores": 16, "kind": "oracle",
                         "sample": "3 implicit-Euler steps of the 128^3 workload, Jacobi-PCG to a 1e-8 relative "
                                   "residual per step, 5.0 s (plain C oracle, OpenMP, 16 threads)",
                         "one_core": {"value": 4e5}, "cpu_model": "AMD EPYC 9575F 64-Core Processor"},
        "nonlinear": {"value": 4e7, "k4": {"value": 1.1e8}, "plain": {"value": 5e7}, "oracle_max_rel_err_256": 7e-9,
                      "multigrid": {"k4": 2.6e8, "plain": 7.6e7}},
        "richards": {"forms": {f: {"value": 1e6} for f in ("block_gmres", "block_bicgstab", "plain_gmres",
                                                            "plain_bicgstab")},
                     "oracle_max_rel_err_16x16x20": 5e-9},
        "fully_implicit": {"best": "pipelined k=4 (2 steps)", "forms": {"pipelined k=4 (2 steps)": {"value": 8e7}},
                           "oracle_max_rel_err_16cubed": 5e-10},
        "window_acceleration": {"forms": forms},
        "serving": {"requests": 512, "throughput_dof_timesteps_per_s": 5e6, "latency_p50_ms": 1234.5,
                    "latency_p99_ms": 5678.9, "failed": 0, "oracle_max_rel_err_sampled": 3e-9,
                    "plain_fifo": {"throughput_dof_timesteps_per_s": 3e6, "latency_p50_ms": 2e4,
                                   "latency_p99_ms": 5e4}},
    }


def test_compact_line_fields_and_size():
    out = _record()
    line = bench.compact_line(out, os.path.join(ROOT, "bench_out", "bench_full.json"))
    assert "\n" not in line
    assert len(line.encode()) < 4096, len(line.encode())
    d = json.loads(line)
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
                "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline",
                "oracle_rel_error", "legs", "runs"):
        assert key in d, key
    assert d["config"]["workload"].startswith("heterogeneous diffusion 128^3")
    for key in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert key in d["roofline"]
    assert d["cpu_baseline"]["cores"] == 16 and d["cpu_baseline"]["kind"] == "oracle"
    assert set(d["legs"]) == {"nonlinear_1024sq_k16", "richards_96cubed_k16", "radau2_128cubed",
                              "window_solve_128cubed", "serving"}


def test_roofline_takes_the_largest_share_without_exclusions():
    kt = {"spmm": _kern(30.0, 0.2), "mg_coarse": _kern(7.0, 0.8)}
    kt["mg_coarse"]["launches"] = 500
    kt["mg_coarse"]["total_ms"] = 3.5
    roof, lat = bench.pick_roofline(kt, 4, "f32", "stencil")
    assert roof["category"] == "mg_coarse"
    assert lat["mg_coarse"]["launches"] == 500
