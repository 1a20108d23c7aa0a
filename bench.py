#!/usr/bin/env python3
"""Benchmark of the DD-PMA hot path on one MI355X.

Workload (one "step" = one pseudo-time step of the whole hot path over every subdomain):
513 x 513 grid on [0,1]^2, 4 x 4 overlapping subdomains (overlap 8 cells, 133/137 nodes per
side), sine-layer monitor rho = 1 + 20 sech^2(40 (y - 1/2 - sin(2 pi x)/4)), gamma = 4 h^2,
dt = gamma / 5.  State stays resident in HBM; exactly --steps steps are timed.

value = global grid nodes x steps / wall time of the timed steps (grid-point updates/s) for the
batched FP32 form (FP32 stencils, fp16-split matrix-core DCT products, graph-replayed shared
launches).  The plain FP64 form (one subdomain per launch, FP64 everywhere, no graph) and the
FP32 form with FP32 matrix-core products are timed beside it on the same workload.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"hbm_GBs": 8000.0, "fp16_TF": 2500.0, "fp32_TF": 157.3, "fp64_TF": 78.6}
MFMA_PEAK = {"split16": PEAK["fp16_TF"], "fp32": PEAK["fp32_TF"], "fp64": PEAK["fp64_TF"]}


def timed_form(ctx, binding, w, prec, exec_, steps, warmup, phase_steps):
    import torch
    plan = binding.Plan(ctx, [w], prec, exec_)
    try:
        plan.step(warmup)
        plan.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.step(steps)
        plan.sync()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        phases = plan.phase_times(phase_steps) if phase_steps > 0 else None
        mesh, st = plan.mesh(0)
    finally:
        plan.close()
    nodes = math.prod(w["grid"]["n"])
    return {"updates_per_s": nodes * steps / dt, "ms_per_step": 1e3 * dt / steps, "seconds": dt,
            "steps": steps, "min_det": st["min_det"], "min_cell": st["min_cell"], "phases": phases}


def roofline_of(phases, prec):
    name, ph = max(((k, v) for k, v in phases.items()), key=lambda kv: kv[1]["ms"])
    sec = ph["ms"] * 1e-3
    kern = {"fwd_last": "fwd_last_kernel", "fwd_mid": "strip_kernel (single)", "pair0": "strip_kernel (pair)",
            "inv_mid": "strip_kernel (single)", "inv_last": "inv_last_kernel", "transmit": "transmit_kernel",
            "stencil": "stencil_kernel", "euler": "euler_kernel"}[name]
    if ph["flops"] > 0:
        ach = ph["flops"] / sec / 1e12
        peak = MFMA_PEAK[prec]
        return {"kernel": f"{kern} ({name})", "bound": "mfma", "achieved": ach, "peak": peak,
                "unit": "TFLOP/s", "frac": ach / peak, "traffic": None,
                "algorithmic_per_launch": ph["flops"], "avg_ms": ph["ms"]}
    ach = ph["bytes"] / sec / 1e9
    return {"kernel": f"{kern} ({name})", "bound": "hbm", "achieved": ach, "peak": PEAK["hbm_GBs"], "unit": "GB/s",
            "frac": ach / PEAK["hbm_GBs"], "traffic": None, "algorithmic_per_launch": ph["bytes"],
            "avg_ms": ph["ms"]}


def cpu_baseline(w, steps):
    import oracle as O
    g = w["grid"]
    gs = O.GridSpec(tuple(g["n"]), tuple(g["lo"]), tuple(g["hi"]))
    t = w["time"]
    t0 = time.perf_counter()
    O.solve_dd(gs, w["dd"]["parts"], w["dd"]["overlap"], w["monitor"], t["dt"], t["gamma"], steps)
    dt = time.perf_counter() - t0
    return {"value": math.prod(g["n"]) * steps / dt, "unit": "grid-point updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{steps} steps of the same 513^2 4x4 DD workload (FP64 NumPy oracle, one thread), "
                      f"{dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cpu-steps", type=int, default=150)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--only", choices=["split16", "fp32", "fp64plain"], default=None,
                    help="time one form only (for profiler runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU layout is design-only.",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2006_14602_amd import binding, workloads
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    w = workloads.sine_dd()
    ctx = binding.Context(0, budget_bytes=4 << 30)
    forms = {}
    todo = [args.only] if args.only else ["split16", "fp32", "fp64plain"]
    for f in todo:
        prec, ex = ("fp64", "plain") if f == "fp64plain" else (f, "batched")
        steps = args.steps if f != "fp64plain" else max(1, min(args.steps, 100))
        forms[f] = timed_form(ctx, binding, w, prec, ex, steps, min(args.warmup, steps), 20)
        print(f"# {f}: {forms[f]['updates_per_s']:.4e} updates/s, {forms[f]['ms_per_step']:.4f} ms/step",
              file=sys.stderr, flush=True)
    ctx.close()
    main_form = args.only or "split16"
    m = forms[main_form]
    prec = "fp64" if main_form == "fp64plain" else main_form
    out = {
        "metric": "PMA grid-point updates/s, batched FP32 vs plain FP64, p50/p99 mesh latency",
        "value": m["updates_per_s"], "unit": "grid-point updates/s", "n_gpus": 1, "steps": m["steps"],
        "warmup": args.warmup, "ms_per_step": m["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "fp64" if prec == "fp64" else "fp32", "data": "synthetic",
        "config": {"workload": "sine-layer DD 513x513, 4x4 subdomains, overlap 8 cells", "grid": w["grid"]["n"],
                   "parts": w["dd"]["parts"], "overlap_cells": w["dd"]["overlap"][0],
                   "gamma": w["time"]["gamma"], "dt": w["time"]["dt"],
                   "precision": {"split16": "fp32 state/stencil, fp16 hi+lo matrix-core DCT, fp32 accumulate",
                                 "fp32": "fp32 everywhere", "fp64": "fp64 everywhere"}[prec],
                   "exec": "plain" if main_form == "fp64plain" else "batched (graph replay)"},
        "roofline": roofline_of(m["phases"], prec),
        "forms": {k: {kk: vv for kk, vv in v.items() if kk != "phases"} for k, v in forms.items()},
        "phases_ms": {k: {p: round(v["ms"], 5) for p, v in f["phases"].items()} for k, f in forms.items()},
    }
    if "fp64plain" in forms and main_form != "fp64plain":
        out["batched_fp32_over_plain_fp64"] = m["updates_per_s"] / forms["fp64plain"]["updates_per_s"]
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_steps)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
