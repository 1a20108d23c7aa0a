#!/usr/bin/env python3
"""Benchmark of the DD-PMA hot path on one MI355X.

Headline workload (one "step" = one pseudo-time step of the whole hot path over every subdomain):
513 x 513 grid on [0,1]^2, 4 x 4 overlapping subdomains (overlap 8 cells, 133/137 nodes per
side), sine-layer monitor rho = 1 + 20 sech^2(40 (y - 1/2 - sin(2 pi x)/4)), gamma = 4 h^2,
dt = gamma / 5.  State stays resident in HBM; exactly --steps steps are timed.

value = global grid nodes x steps / wall time of the timed steps (grid-point updates/s) for the
batched FP32 form (FP32 stencils, fp16-split matrix-core DCT products, graph-replayed shared
launches).  Beside it, on the same MI355X: the same workload in FP32 matrix-core products and in
the plain FP64 form (one subdomain per launch, FP64 everywhere, no graph); the 65^2 ring
(FP64), the 129^3 shell DD, the 256-instance batch (batched FP32 vs plain FP64), a Poisson
serving stream (meshes/s, p50/p99 latency), and the stencil at a >= 1 GB working set.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import threading
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"hbm_GBs": 8000.0, "fp16_TF": 2500.0, "fp32_TF": 157.3, "fp64_TF": 78.6}
MFMA_PEAK = {"split16": PEAK["fp16_TF"], "fp32": PEAK["fp32_TF"], "fp64": PEAK["fp64_TF"]}
ROOT = os.path.dirname(os.path.abspath(__file__))


def profile_entry(workload, key):
    """An entry of the committed rocprofv3 summary (profiles/traffic.json), or None when the
    kernel source has changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    with open(os.path.join(ROOT, "paper_2006_14602_amd", "csrc", "kernels.hip"), "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != rec.get("kernels_hip_sha256"):
            return None
    return rec.get("entries", {}).get(workload, {}).get(key)


def traffic_of(workload, phase):
    """HBM bytes per launch of a step phase's kernel on `workload` from the committed rocprofv3 counters
    (FETCH_SIZE and WRITE_SIZE per dispatch, scaled by the copy calibration), or None."""
    e = profile_entry(workload, phase)
    return None if e is None else e["fetch_bytes"] + e["write_bytes"]


# vector-ALU issue: a wave64 FP32 instruction holds a 16-lane SIMD for 4 cycles (transcendentals 16),
# 256 CUs x 4 SIMDs at 2.4 GHz
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4.0   # full-rate wave instructions per second
KERNEL = {"transmit": "transmit_kernel", "stencil": "stencil_fwd2_kernel / stencil2_kernel / stencil3_kernel",
          "euler": "euler_kernel",
          "fwd_last": "fwd_last_kernel", "fwd_mid": "strip_kernel<single>",
          "pair0": "strip_kernel<pair> (16-column strips) / strip4_kernel<pair> (64-column strips)",
          "inv_mid": "strip_kernel<single>", "inv_last": "inv_last_kernel"}


def log(*a):
    print("#", *a, file=sys.stderr, flush=True)


def nodes_of(ws):
    return sum(math.prod(w["grid"]["n"]) for w in ws)


def timed_plan(ctx, binding, ws, prec, exec_, steps, warmup, phase_reps=0, tune=False):
    """Resident plan: warmup steps, then exactly `steps` timed steps bracketed by synchronize.
    tune: pick the stencil's launch shape with the plan's autotuner first (outside the timing)."""
    import torch
    plan = binding.Plan(ctx, ws, prec, exec_)
    march = None
    try:
        if tune:
            march, _ = plan.autotune(10)
        plan.step(warmup)
        plan.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.step(steps)
        plan.sync()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        phases = plan.phase_times(phase_reps) if phase_reps > 0 else None
        try:
            mesh, st = plan.mesh(0)
        except binding.PmaError as e:  # a folded mesh still has a measured step rate
            st = {"min_det": float("nan"), "min_cell": float("nan"), "quality_e2": float("nan"),
                  "quality_emax": float("nan"), "error": str(e)}
    finally:
        plan.close()
    out = {"updates_per_s": nodes_of(ws) * steps / dt, "ms_per_step": 1e3 * dt / steps, "seconds": dt,
           "steps": steps, "min_det": st["min_det"], "min_cell": st["min_cell"],
           "quality_e2": st["quality_e2"], "quality_emax": st["quality_emax"], "stencil_march": march,
           "phases": phases}
    if "error" in st:
        out["error"] = st["error"]
    return out


def glued_vs_single(ctx, binding, w, prec):
    """The glued DD mesh against the whole-domain mesh of the same problem (same gamma, dt and
    steps): the decomposition error at the headline size (Sec. 4.4)."""
    import numpy as np
    meshes = []
    for ww in (w, dict(w, dd=None)):
        plan = binding.Plan(ctx, [ww], prec, "batched")
        try:
            plan.step(ww["time"]["steps"])
            plan.sync()
            meshes.append(plan.mesh(0)[0])
        finally:
            plan.close()
    d = np.abs(meshes[0] - meshes[1])
    return {"max_mesh_diff": float(d.max()), "rms_mesh_diff": float(np.sqrt(np.mean(d * d))),
            "steps": w["time"]["steps"], "precision": prec}


def paper_workloads(ctx, binding, workloads):
    """The paper's own examples (Sec. 4): arc-length monitors of its test functions, alternating
    sweeps (Algorithm 1) as the paper ran them, and the alternating form of the headline case.
    Step rate from a resident plan; mesh statistics (min det, min cell, quality E_2 / E_max of the
    glued mesh) after the timed steps."""
    sd = workloads.sine_dd(steps=200)
    sd["dd"]["mode"] = "alternating"
    cases = [
        ("burgers_front_65_slabs4_alternating", workloads.burgers_front(parts=(4, 1), steps=300), 300),
        ("burgers_front_65_blocks2x2_alternating", workloads.burgers_front(parts=(2, 2), steps=300), 300),
        ("spiral_257_4x4_parallel", workloads.spiral(steps=300), 300),
        ("sphere_81_blocks8_alternating", workloads.sphere_3d(n=81, steps=150), 150),
        ("spheres9_81_blocks8_alternating", workloads.spheres9_3d(n=81, steps=150), 150),
        ("sine_dd_513_4x4_alternating", sd, 200),
    ]
    out = {}
    for name, w, steps in cases:
        r = timed_plan(ctx, binding, [w], "split16", "batched", steps, 5, tune=True)
        e = {k: r[k] for k in ("updates_per_s", "ms_per_step", "steps", "min_det", "min_cell", "quality_e2",
                               "quality_emax", "stencil_march")}
        if "error" in r:
            e["error"] = r["error"]
        if name.startswith("burgers_front_65_slabs4"):
            p = timed_plan(ctx, binding, [w], "fp64", "plain", 100, 2)
            e["plain_fp64_updates_per_s"] = p["updates_per_s"]
            e["speedup_over_plain_fp64"] = r["updates_per_s"] / p["updates_per_s"]
        if w.get("dd") and w["dd"].get("mode", "parallel") != "parallel":
            e["sweep_levels"] = int(max(binding.sweep_levels(w["grid"], w["dd"])) + 1)
        out[name] = e
        log(f"{name}: {r['updates_per_s']:.3e} updates/s, {r['ms_per_step']:.4f} ms/step, "
            f"E2 {r['quality_e2']:.4f}")
    return out


def roofline_of(phases, prec, workload=None):
    """Dominant kernel of a step: algorithmic work per launch / mean launch duration; traffic from
    the committed counters of `workload` when they are current."""
    name, ph = max(((k, v) for k, v in phases.items() if v["flops"] > 0 or v["bytes"] > 0),
                   key=lambda kv: kv[1]["ms"])
    sec = ph["ms"] * 1e-3
    if ph["flops"] > 0:
        ach = ph["flops"] / sec / 1e12
        peak = MFMA_PEAK[prec]
        return {"kernel": KERNEL[name], "phase": name, "bound": "mfma", "achieved": ach, "peak": peak,
                "unit": "TFLOP/s", "frac": ach / peak, "traffic": traffic_of(workload, name),
                "algorithmic_per_launch": ph["flops"], "avg_launch_ms": ph["ms"]}
    ach = ph["bytes"] / sec / 1e9
    return {"kernel": KERNEL[name], "phase": name, "bound": "hbm", "achieved": ach, "peak": PEAK["hbm_GBs"],
            "unit": "GB/s", "frac": ach / PEAK["hbm_GBs"], "traffic": traffic_of(workload, name),
            "algorithmic_per_launch": ph["bytes"], "avg_launch_ms": ph["ms"]}


def shell_bench(ctx, binding, workloads, steps, warmup):
    """129^3 spherical shell, 2x2x2 subdomains, overlap 6 cells, batched split form."""
    r = timed_plan(ctx, binding, [workloads.shell_dd()], "split16", "batched", steps, warmup, phase_reps=10,
                   tune=True)
    log(f"shell 129^3 split16: {r['updates_per_s']:.3e}")
    return {"updates_per_s": r["updates_per_s"], "ms_per_step": r["ms_per_step"], "stencil_march": r["stencil_march"],
            "roofline": roofline_of(r["phases"], "split16", "shell_dd_129_split16"),
            "phases_ms_per_launch": {p: round(v["ms"], 5) for p, v in r["phases"].items()}}


def batch_bench(ctx, binding, workloads, steps, warmup, plain):
    """256 single-domain instances of uneven sides (33..257) with Gaussian-bump monitors, batched
    split form; plain: also the plain FP64 method on the same instances."""
    batch = workloads.bumps_batch()
    rb = timed_plan(ctx, binding, batch, "split16", "batched", steps, warmup, phase_reps=10, tune=True)
    out = {"batched_split16_updates_per_s": rb["updates_per_s"], "batched_ms_per_step": rb["ms_per_step"],
           "stencil_march": rb["stencil_march"],
           "roofline": roofline_of(rb["phases"], "split16", "bumps_batch_256_split16"),
           "phases_ms_per_launch": {p: round(v["ms"], 5) for p, v in rb["phases"].items()}}
    if plain:
        rp = timed_plan(ctx, binding, batch, "fp64", "plain", 10, 1)
        out.update({"plain_fp64_updates_per_s": rp["updates_per_s"], "plain_ms_per_step": rp["ms_per_step"],
                    "speedup": rb["updates_per_s"] / rp["updates_per_s"]})
        log(f"batch 256: {rb['updates_per_s']:.3e} vs plain fp64 {rp['updates_per_s']:.3e}")
    return out


def stencil_roofline(ctx, binding, workloads):
    """Stencil phase alone over two 8193^2 DD requests (32 x 32 parts): 134 M nodes, 1.07 GB of
    compulsory FP32 traffic per launch, far beyond the 256 MB last-level cache."""
    w = workloads.sine_dd(n=8193, parts=(32, 32), overlap=8, steps=1)
    plan = binding.Plan(ctx, [w, w], "split16", "batched")
    try:
        plan.set_fusion(False)  # the stencil alone (phi -> F), not fused with the first product
        march, cand = plan.autotune(5)
        ph = plan.phase_times(10)
    finally:
        plan.close()
    st = ph["stencil"]
    gbs = st["bytes"] / (st["ms"] * 1e-3) / 1e9
    out = {"kernel": "stencil2_kernel", "bound": "hbm", "achieved": gbs, "peak": PEAK["hbm_GBs"], "unit": "GB/s",
           "frac": gbs / PEAK["hbm_GBs"], "traffic": traffic_of("stencil_large", f"stencil@march={march}"),
           "bytes_per_launch": st["bytes"], "avg_launch_ms": st["ms"],
           "stencil_march": march, "autotune_ms": [round(t, 4) for t in cand],
           "workload": "2 x 8193^2 sine layer, 32x32 parts, FP32 (8 B per node)"}
    # the vector-ALU view of the same launch: issue cycles per node from the committed SQ counters
    a = profile_entry("stencil_large_alu", f"stencil@march={march}")
    if a is not None:
        nodes_s = st["bytes"] / 8.0 / (st["ms"] * 1e-3)
        issued = nodes_s * (a["valu_wave_insts_per_node"] + 3.0 * a["trans_wave_insts_per_node"])
        out["alu"] = {"bound": "alu", "achieved": issued, "peak": VALU_ISSUE_PEAK,
                      "unit": "full-rate wave instructions/s", "frac": issued / VALU_ISSUE_PEAK,
                      "valu_wave_insts_per_node": a["valu_wave_insts_per_node"],
                      "trans_wave_insts_per_node": a["trans_wave_insts_per_node"],
                      "node_rate_ceiling_per_s": a["node_rate_ceiling"],
                      "hbm_equivalent_of_ceiling_GBs": a["node_rate_ceiling"] * 8 / 1e9}
    return out


def serve_stream(binding, workloads, count, budget):
    """Open-loop Poisson stream (mean 200 req/s) through pma_submit / pma_poll.  Latency is taken
    on the client: from the request's scheduled arrival to the poll that sees it DONE."""
    ws = workloads.stream(count=count)
    ctx = binding.Context(0, budget_bytes=budget)
    tickets = [None] * len(ws)
    late = [0.0] * len(ws)
    t_start = time.perf_counter()

    def producer():
        for i, w in enumerate(ws):
            d = w["arrival_s"] - (time.perf_counter() - t_start)
            if d > 0:
                time.sleep(d)
            tickets[i] = ctx.submit(w, "split16")
            late[i] = (time.perf_counter() - t_start) - w["arrival_s"]

    th = threading.Thread(target=producer)
    th.start()
    done = {}
    last_note = time.perf_counter()
    while len(done) < len(ws):
        if time.perf_counter() - last_note > 5.0:
            last_note = time.perf_counter()
            log(f"serving: {len(done)}/{len(ws)} finished, {sum(t is not None for t in tickets)} submitted")
        for i in range(len(ws)):
            if i in done or tickets[i] is None:
                continue
            state, _, st = ctx.poll(tickets[i])
            if state in (2, 3):
                done[i] = (state, st, time.perf_counter() - t_start)
        time.sleep(0.0005)
        if time.perf_counter() - t_start > 300:
            raise RuntimeError("serving stream did not drain")
    th.join()
    wall = max(v[2] for v in done.values())
    ctx.close()
    ok = [i for i, v in done.items() if v[0] == 2]
    lat = sorted(1e3 * (done[i][2] - ws[i]["arrival_s"]) for i in ok)
    upd = sum(math.prod(ws[i]["grid"]["n"]) * ws[i]["time"]["steps"] for i in ok)
    pct = lambda p: lat[min(len(lat) - 1, int(round(p / 100 * (len(lat) - 1))))]
    return {"requests": len(ws), "done": len(ok), "failed": len(ws) - len(ok), "wall_s": wall,
            "meshes_per_s": len(ok) / wall, "updates_per_s": upd / wall, "p50_ms": pct(50), "p99_ms": pct(99),
            "max_submit_lag_ms": 1e3 * max(late),
            "mean_server_queue_ms": sum(v[1]["ms_queue"] for v in done.values()) / len(done),
            "budget_bytes": budget, "offered_rate_per_s": 200.0,
            "arrival_window_s": ws[-1]["arrival_s"]}


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
    ap.add_argument("--cpu-steps", type=int, default=1000)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--serve", type=int, default=600, help="requests in the serving stream (0: skip)")
    ap.add_argument("--quick", action="store_true", help="headline workload only")
    ap.add_argument("--only", choices=["split16", "fp32", "fp64plain", "stencil_large", "paper", "shell", "batch"], default=None,
                    help="one form of the headline workload, or one other workload, only (profiler runs)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-sized float32 buffer 10 times (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.copy_probe:
        import torch
        a = torch.ones(args.copy_probe << 18, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(10):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": a.numel() * 4, "copy_probe_bytes_written": b.numel() * 4}))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU layout is design-only.",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2006_14602_amd import binding, workloads
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.only == "paper":
        ctx = binding.Context(0, budget_bytes=12 << 30)
        print(json.dumps({"paper_workloads": paper_workloads(ctx, binding, workloads)}))
        ctx.close()
        return
    if args.only in ("shell", "batch"):
        ctx = binding.Context(0, budget_bytes=12 << 30)
        if args.only == "shell":
            r = {"shell_dd_129_split16": shell_bench(ctx, binding, workloads, args.steps, args.warmup)}
        else:
            r = {"bumps_batch_256": batch_bench(ctx, binding, workloads, args.steps, args.warmup, plain=False)}
        print(json.dumps(r))
        ctx.close()
        return
    if args.only == "stencil_large":
        ctx = binding.Context(0, budget_bytes=12 << 30)
        print(json.dumps({"stencil_hbm_large": stencil_roofline(ctx, binding, workloads)}))
        ctx.close()
        return
    w = workloads.sine_dd()
    ctx = binding.Context(0, budget_bytes=12 << 30)
    forms = {}
    todo = [args.only] if args.only else ["split16", "fp32", "fp64plain"]
    for f in todo:
        prec, ex = ("fp64", "plain") if f == "fp64plain" else (f, "batched")
        steps = args.steps if f != "fp64plain" else max(1, min(args.steps, 100))
        forms[f] = timed_plan(ctx, binding, [w], prec, ex, steps, min(args.warmup, steps), phase_reps=50,
                              tune=ex == "batched")
        log(f"{f}: {forms[f]['updates_per_s']:.4e} updates/s, {forms[f]['ms_per_step']:.4f} ms/step")
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
        "roofline": roofline_of(m["phases"], prec, "sine_dd_513_" + main_form),
        "forms": {k: {kk: vv for kk, vv in v.items() if kk != "phases"} for k, v in forms.items()},
        "phases_ms_per_launch": {k: {p: round(v["ms"], 5) for p, v in f["phases"].items()}
                                 for k, f in forms.items()},
    }
    if "fp64plain" in forms and main_form != "fp64plain":
        out["batched_fp32_over_plain_fp64"] = m["updates_per_s"] / forms["fp64plain"]["updates_per_s"]
    if not args.only:
        out["glued_vs_single_domain"] = glued_vs_single(ctx, binding, w, prec)
    if not args.quick and not args.only:
        extra = {}
        ring = workloads.ring()
        r = timed_plan(ctx, binding, [ring], "fp64", "batched", 200, 10)
        extra["ring_65_fp64"] = {k: r[k] for k in ("updates_per_s", "ms_per_step")}
        log(f"ring 65^2 fp64: {r['updates_per_s']:.3e}")
        extra["shell_dd_129_split16"] = shell_bench(ctx, binding, workloads, 200, 5)
        extra["bumps_batch_256"] = batch_bench(ctx, binding, workloads, 200, 5, plain=True)
        extra["stencil_hbm_large"] = stencil_roofline(ctx, binding, workloads)
        log(f"stencil large: {extra['stencil_hbm_large']['achieved']:.0f} GB/s")
        out["other_workloads"] = extra
        out["paper_workloads"] = paper_workloads(ctx, binding, workloads)
    ctx.close()
    if args.serve > 0 and not args.quick and not args.only:
        s8 = serve_stream(binding, workloads, args.serve, 8 << 30)
        log(f"serve 8GB: {s8}")
        s512 = serve_stream(binding, workloads, max(50, args.serve // 4), 512 << 20)
        log(f"serve 512MB: {s512}")
        out["serving"] = {"budget_8GiB": s8, "budget_512MiB": s512}
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_steps)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
