#!/usr/bin/env python3
"""Benchmark of the DD-PMA hot path on one MI355X.

Headline workload (one "step" = one pseudo-time step of the whole hot path over every instance):
256 independent single-domain 2D meshes of uneven sides (U{33..257}, PCG64 seed 20060146),
monitors 1 + a sum of 1-4 Gaussian bumps, gamma = 1, dt = 1e-3, 200 steps (6.46 M nodes per
step).  State stays resident in HBM; exactly --steps steps are timed.

value = grid nodes x steps / wall time of the timed steps (grid-point updates/s) for the batched
FP64 form (the paper's precision: FP64 stencils, FP64 matrix-core DCT products, every instance
in the same launches, graph-replayed steps).  Beside it, on the same MI355X and workload: the
batched FP32 form with fp16-split DCT products, the batched FP32 form, and the plain FP64 method
(one instance per launch, no graph); the max mesh error against the FP64 oracle and the FP64
final residual of every instance; the oracle itself timed on the host's cores.  Other lines: the
513^2 4x4 sine-layer DD (all forms), the 65^2 ring, the 129^3 shell DD, the stencil at a >= 1 GB
working set, the paper's own workloads, and a Poisson serving stream (continuous batching
against the plain method serving the same stream).
"""
import argparse
import hashlib
import json
import math
import os
import sys
import threading
import time

if __name__ == "__mp_main__":  # the oracle's worker processes: one thread each
    for _v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[_v] = "1"
import numpy as np  # noqa: E402

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


# the launch-configuration tuner's cache (pma_plan_tune): choices keyed by device, precision and
# shape bucket, reused by later runs on the same machine
TUNE_CACHE = os.path.join(os.environ.get("TMPDIR", "/tmp"), "pma_tune_cache.txt")


def persistent_vs_phases(ctx, binding, w, prec, steps=200):
    """The same workload stepped with one persistent launch per step and with phase launches."""
    import torch
    out = {}
    for pers in (False, True):
        p = binding.Plan(ctx, [w], prec, "batched")
        try:
            p.autotune(5)
            if pers:
                p.set_persistent(True)
            p.step(10)
            p.sync()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            p.step(steps)
            p.sync()
            torch.cuda.synchronize()
            out["persistent" if pers else "phase_launches"] = 1e3 * (time.perf_counter() - t0) / steps
        finally:
            p.close()
    out["unit"] = "ms per step"
    return out


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
    tuning = None
    try:
        if tune:
            tuning = plan.tune(5, TUNE_CACHE)
            march = tuning["march"]
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
           "tuning": tuning, "phases": phases}
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


# Sec. 4.3, tables ddpma_efficiency2D / ddpma_efficiency3D: MATLAB FP64 CPU seconds for one complete
# mesh (single domain; 4- or 8-block DD solved in turn; the same in parallel on 4 or 8 cores), step
# counts not stated; quoted as context only
PAPER_SECONDS = {
    2: {65: (0.2, 0.31, 0.53), 129: (0.38, 0.51, 0.66), 257: (0.8, 1.0, 0.76), 513: (3.53, 2.7, 1.6),
        1025: (13.51, 10.94, 7.09)},
    3: {65: (20.0, 18.0, 4.0), 81: (30.0, 29.0, 8.0), 101: (62.0, 58.0, 16.0), 121: (104.0, 94.0, 37.0)},
}


def efficiency_ladder(ctx, binding, workloads, prec="fp64", steps2=200, steps3=100):
    """The paper's grid ladder (Sec. 4.3): the spiral (Sec. 4.1) at 65^2 .. 1025^2 and the sphere
    (Sec. 4.2) at 65^3 .. 121^3, each on the whole domain, as 2x2 (2x2x2) blocks swept in turn
    (Algorithm 1) and as 2x2 (2x2x2) blocks in parallel; the same number of steps at every size."""
    out = {}
    for dim, sizes, steps in ((2, (65, 129, 257, 513, 1025), steps2), (3, (65, 81, 101, 121), steps3)):
        for n in sizes:
            row = {}
            for form, parts, mode in (("single", None, None), ("blocks_alternating", (2,) * dim, "alternating"),
                                      ("blocks_parallel", (2,) * dim, "parallel")):
                if dim == 2:
                    w = workloads.spiral(n=n, parts=parts, overlap=4, mode=mode or "parallel", steps=steps)
                else:
                    w = workloads.sphere_3d(n=n, parts=parts, overlap=2, mode=mode or "alternating", steps=steps)
                r = timed_plan(ctx, binding, [w], prec, "batched", steps, 3)
                e = {"ms_per_step": r["ms_per_step"], "seconds": r["seconds"], "updates_per_s": r["updates_per_s"],
                     "min_det": r["min_det"], "min_cell": r["min_cell"]}
                if "error" in r:
                    e["error"] = r["error"]
                row[form] = e
            row["paper_matlab_seconds_single_serialdd_paralleldd"] = PAPER_SECONDS[dim][n]
            out[f"{'spiral' if dim == 2 else 'sphere'}_{n}{'^2' if dim == 2 else '^3'}"] = row
            log(f"ladder {dim}D {n}: " + ", ".join(f"{k} {v['ms_per_step']:.3f} ms/step" for k, v in row.items()
                                                   if isinstance(v, dict)))
    return {"precision": prec, "steps_2d": steps2, "steps_3d": steps3, "rows": out,
            "note": "GPU seconds are for the stated step counts; the paper's MATLAB seconds (ode113, CPU) state "
                    "no step counts and are context only"}


# ---- the convergence studies of Sec. 4.4 and the quality table of Sec. 4.5, on the GPU ----------

def _trap_weights(shape, h):
    w = np.ones(shape)
    for k, n in enumerate(shape):
        wk = np.ones(n)
        wk[0] = wk[-1] = 0.5
        sh = [1] * len(shape)
        sh[k] = -1
        w = w * wk.reshape(sh)
    return w * float(np.prod(h))


def rel_errs(ref, approx, h):
    """Sec. 4.4 eqs. rel_errlp / rel_errlinf (integrals by the trapezoid rule) of one field."""
    w = _trap_weights(ref.shape, h)
    d = np.abs(ref - approx)
    out = {p: float((np.sum(w * d ** p) ** (1.0 / p)) / (np.sum(w * np.abs(ref) ** p) ** (1.0 / p))) for p in (1, 2)}
    out["inf"] = float(d.max() / np.abs(ref).max())
    return out


def mesh_rel_errs(ref, approx, h):
    """The relative errors of a mesh: the larger over its coordinate fields."""
    es = [rel_errs(ref[k], approx[k], h) for k in range(ref.shape[0])]
    return {p: max(e[p] for e in es) for p in (1, 2, "inf")}


def _slope(hs, es):
    return float(np.polyfit(np.log(hs), np.log(es), 1)[0])


def smooth_monitor():
    """A smooth ring (amplitude 5, sharpness 10 about |x - c| = 1/4): resolved at 21^2 already, so
    the steady states the studies compare are in the asymptotic range."""
    return {"kind": "sech2_radial", "amp": 5.0, "k": 10.0, "r0": 0.25, "c": [0.5, 0.5]}


def steady_single(ctx, workloads, n, mon, prec="fp64", dt=0.05, steps=1500):
    """Whole-domain steady state (gamma = 1): the mesh, and c, the value F settles to (the uniform
    drift of Psi per unit pseudo time, measured over 100 more steps)."""
    w = {"name": f"single_{n}", "grid": workloads.grid([n, n]), "dd": None, "monitor": dict(mon),
         "time": {"dt": dt, "gamma": 1.0, "steps": steps}}
    m, p1, _ = ctx.dd_mesh(w, precision=prec, want_psi=True)
    _, p2, _ = ctx.dd_mesh(dict(w, time=dict(w["time"], steps=100)), precision=prec, psi0=p1, want_psi=True)
    drift = (p2 - p1) / (100 * dt)
    return m, float(np.mean(drift)), float(drift.max() - drift.min())


def dd_history(ctx, binding, workloads, n, mon, theta, parts=(2, 2), ov=4, dt_frac=0.2, marks=(1000,), prec="fp64"):
    """A decomposed solve (gamma = 4 h^2, dt = dt_frac gamma) stepped resident on the device; the
    glued mesh at each step count in marks."""
    g = workloads.grid([n, n])
    t = workloads.dd_defaults(g)
    t["dt"] = dt_frac * t["gamma"]
    t["steps"] = max(marks)
    w = {"name": f"dd_{n}", "grid": g, "dd": {"parts": list(parts), "overlap": [ov, ov]},
         "monitor": dict(mon, theta=theta), "time": t}
    out = []
    with binding.Plan(ctx, [w], prec, "batched") as p:
        done = 0
        for k in marks:
            p.step(k - done)
            p.sync()
            done = k
            out.append(p.mesh(0)[0])
    return out, t


def studies(ctx, binding, workloads):
    """E4 (space convergence of the DD solution to the fine single-domain one), E6 (history), E7
    (overlap), E8 (the DD steady state against the pseudo-time step) of Sec. 4.4 and the quality
    table of Sec. 4.5, as steady-state comparisons on the smooth ring monitor (the paper's spiral
    has no reachable steady state under the explicit preconditioned step), FP64."""
    mon0 = smooth_monitor()
    res = {"monitor": mon0}
    # whole-domain steady states and their F value c; theta e^c makes the steady state F = 0, the
    # fixed point the decomposed iteration then reaches exactly (no drift)
    ns = (33, 65, 129, 257)
    sd, theta0 = {}, {}
    th = binding.theta(workloads.grid([33, 33]), mon0)
    for n in ns + (1025,):
        m, c, spread = steady_single(ctx, workloads, n, mon0, steps=1500 if n < 1025 else 1200)
        sd[n] = m
        theta0[n] = th * math.exp(c)
        log(f"steady single {n}: c {c:.4e} (spread {spread:.1e})")
    # E4: decomposed (2x2, overlap 4 cells) steady meshes at N against the 1025^2 whole-domain mesh
    e4 = {}
    for n in ns:
        tau = 3.0
        steps = int(math.ceil(tau / (0.2 * 4.0 / (n - 1) ** 2)))
        (m,), _ = dd_history(ctx, binding, workloads, n, mon0, theta0[n], marks=(steps,))
        s = 1024 // (n - 1)
        ref = sd[1025][:, ::s, ::s]
        h = (1.0 / (n - 1),) * 2
        e4[n] = {"steps": steps, "dd_vs_single_same_n": float(np.abs(m - sd[n]).max()),
                 "rel_vs_1025": mesh_rel_errs(ref, m, h)}
        log(f"E4 n {n}: {e4[n]}")
    hs = [1.0 / (n - 1) for n in ns]
    res["E4_space"] = {"rows": {str(n): v for n, v in e4.items()},
                       "slopes": {str(p): _slope(hs, [e4[n]["rel_vs_1025"][p] for n in ns]) for p in (1, 2, "inf")},
                       "paper_slopes": {"1": 2.01, "2": 1.99, "inf": 1.85}}
    # E6 / E7: history of the DD mesh against the whole-domain steady mesh at 129^2, overlaps of
    # 5, 9, 11 and 15 points (4, 8, 10, 14 cells)
    n = 129
    marks = (1000, 2000, 4000, 8000, 16000, 32000, 64000)
    hist = {}
    for ov in (4, 8, 10, 14):
        ms, _ = dd_history(ctx, binding, workloads, n, mon0, theta0[n], ov=ov, marks=marks)
        hist[f"{ov + 1}_points"] = [mesh_rel_errs(sd[n], m, (1.0 / (n - 1),) * 2)["inf"] for m in ms]
        log(f"E6/E7 overlap {ov}: {hist[f'{ov + 1}_points']}")
    res["E6_E7_history"] = {"n": n, "steps": list(marks), "linf_rel_by_overlap": hist}
    # E8: with the exact theta the decomposed iteration settles into a uniform drift; its mesh
    # against the whole-domain steady mesh (65^2, tau = 2) for pseudo-time steps 1, 2, 4, 8 e-5 at
    # gamma = 4 h^2, and for gamma = h^2, 2 h^2, 4 h^2 at dt = gamma / 5
    n = 65
    h2 = 1.0 / (n - 1) ** 2
    e8, e8g = {}, {}
    for mult in (1, 2, 4, 8):
        dt = mult * 1e-5
        steps = int(math.ceil(2.0 / dt))
        (m,), _ = dd_history(ctx, binding, workloads, n, mon0, th, dt_frac=dt / (4.0 * h2), marks=(steps,))
        e8[f"{mult}e-5"] = {"steps": steps, "rel_vs_single": mesh_rel_errs(sd[n], m, (1.0 / (n - 1),) * 2)}
        log(f"E8 dt {dt}: {e8[f'{mult}e-5']}")
    for cg in (1.0, 2.0, 4.0):
        g = workloads.grid([n, n])
        t = {"gamma": cg * h2, "dt": 0.2 * cg * h2}
        t["steps"] = int(math.ceil(2.0 / t["dt"]))
        w = {"grid": g, "dd": {"parts": [2, 2], "overlap": [4, 4]}, "monitor": dict(mon0, theta=th), "time": t}
        m, _, _ = ctx.dd_mesh(w, precision="fp64")
        e8g[f"{cg:g}h^2"] = {"steps": t["steps"], "rel_vs_single": mesh_rel_errs(sd[n], m, (1.0 / (n - 1),) * 2)}
        log(f"E8 gamma {cg} h^2: {e8g[f'{cg:g}h^2']}")
    res["E8_dt"] = {"n": n, "tau": 2.0, "by_dt_gamma_4h2": e8, "by_gamma_dt_gamma_over_5": e8g}
    # quality table (Sec. 4.5): 21^2 and 41^2; 4 slabs, 2x2 blocks, whole domain
    qt = {}
    for n in (21, 41):
        m, c, _ = steady_single(ctx, workloads, n, mon0, steps=1500)
        thn = th * math.exp(c)
        row = {}
        for form, parts in (("slabs4", (4, 1)), ("blocks2x2", (2, 2)), ("whole", None)):
            g = workloads.grid([n, n])
            if parts:
                t = workloads.dd_defaults(g)
                t["steps"] = int(math.ceil(3.0 / t["dt"]))
                w = {"grid": g, "dd": {"parts": list(parts), "overlap": [2, 2]}, "monitor": dict(mon0, theta=thn),
                     "time": t}
            else:
                w = {"grid": g, "dd": None, "monitor": dict(mon0, theta=thn),
                     "time": {"dt": 0.05, "gamma": 1.0, "steps": 1500}}
            _, _, st = ctx.dd_mesh(w, precision="fp64")
            # E is reported with theta = int rho (the run used theta e^c): E scales by e^c
            row[form] = {"E2": st["quality_e2"] * math.exp(c), "Emax": st["quality_emax"] * math.exp(c)}
        qt[f"{n}^2"] = row
        log(f"quality {n}: {row}")
    res["quality_table"] = {"rows": qt, "paper": {"21^2": {"slabs4": (1.0198, 1.1546), "blocks2x2": (1.0194, 1.1590),
                                                          "whole": (1.0194, 1.1609)},
                                                 "41^2": {"slabs4": (1.0053, 1.0997), "blocks2x2": (1.0052, 1.0994),
                                                          "whole": (1.0042, 1.0980)}}}
    return res


def roofline_of(phases, prec, workload=None):
    """Dominant kernel of a step: algorithmic work per launch / mean launch duration; traffic from
    the committed counters of `workload` when they are current."""
    name, ph = max(((k, v) for k, v in phases.items() if k != "resid" and (v["flops"] > 0 or v["bytes"] > 0)),
                   key=lambda kv: kv[1]["ms"])
    sec = ph["ms"] * 1e-3
    if ph["flops"] > 0:
        ach = ph["flops"] / sec / 1e12
        peak = MFMA_PEAK[prec]
        out = {"kernel": KERNEL[name], "phase": name, "bound": "mfma", "achieved": ach, "peak": peak,
               "unit": "TFLOP/s", "frac": ach / peak, "traffic": traffic_of(workload, name),
               "algorithmic_per_launch": ph["flops"], "avg_launch_ms": ph["ms"]}
        if prec == "split16":  # three fp16 products per useful one (hi*hi, hi*lo, lo*hi)
            out["raw_mfma_flops_per_launch"] = 3 * ph["flops"]
            out["raw_mfma_TFLOPs"] = 3 * ach
        return out
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


def copy_bandwidth(mib=1024, reps=20):
    """Device-to-device copy of a MIB-sized float32 buffer (torch's copy kernel), HIP events around
    REPS copies: the read + write bandwidth a plain streaming kernel reaches on this GPU, the
    practical ceiling beside the 8 TB/s peak for a kernel that reads and writes equal amounts."""
    import torch
    a = torch.ones(mib << 18, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    e1.synchronize()
    sec = e0.elapsed_time(e1) * 1e-3 / reps
    del a, b
    torch.cuda.empty_cache()
    return 2.0 * (mib << 20) / sec / 1e9


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
    # the same bytes against what a plain 1 GiB copy reaches on this GPU (read + write, 1:1)
    cp = copy_bandwidth()
    out["copy_GBs"] = cp
    out["frac_of_copy"] = gbs / cp
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


def _pct(lat, p):
    return lat[min(len(lat) - 1, int(round(p / 100 * (len(lat) - 1))))]


def serve_stream(binding, workloads, count, budget):
    """Open-loop Poisson stream (mean 200 req/s) through pma_submit / pma_poll (continuous
    batching, batched split form).  Latency is taken on the client: from the request's scheduled
    arrival to the poll that sees it DONE."""
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
        if time.perf_counter() - t_start > 600:
            raise RuntimeError("serving stream did not drain")
    th.join()
    wall = max(v[2] for v in done.values())
    ctx.close()
    ok = [i for i, v in done.items() if v[0] == 2]
    lat = sorted(1e3 * (done[i][2] - ws[i]["arrival_s"]) for i in ok)
    upd = sum(math.prod(ws[i]["grid"]["n"]) * ws[i]["time"]["steps"] for i in ok)
    return {"requests": len(ws), "done": len(ok), "failed": len(ws) - len(ok), "wall_s": wall,
            "meshes_per_s": len(ok) / wall, "updates_per_s": upd / wall, "p50_ms": _pct(lat, 50),
            "p99_ms": _pct(lat, 99), "max_submit_lag_ms": 1e3 * max(late),
            "mean_server_queue_ms": sum(v[1]["ms_queue"] for v in done.values()) / len(done),
            "budget_bytes": budget, "offered_rate_per_s": 200.0, "arrival_window_s": ws[-1]["arrival_s"],
            "form": "continuous batching, batched split16, graph-replayed ticks"}


def serve_plain(binding, workloads, count, prec="fp64"):
    """The plain per-subdomain method serving the same stream: requests taken one at a time in
    arrival order (FIFO), each solved alone by pma_dd_mesh in the plain form (one subdomain per
    launch, no graph), waiting for its arrival time when the queue is empty.  Latency from the
    scheduled arrival to the end of its solve."""
    ws = workloads.stream(count=count)
    ctx = binding.Context(0, budget_bytes=8 << 30)
    lat, upd = [], 0
    t_start = time.perf_counter()
    for w in ws:
        d = w["arrival_s"] - (time.perf_counter() - t_start)
        if d > 0:
            time.sleep(d)
        ctx.dd_mesh(w, precision=prec, exec_="plain")
        lat.append(1e3 * (time.perf_counter() - t_start - w["arrival_s"]))
        upd += math.prod(w["grid"]["n"]) * w["time"]["steps"]
    wall = time.perf_counter() - t_start
    ctx.close()
    lat.sort()
    return {"requests": len(ws), "wall_s": wall, "meshes_per_s": len(ws) / wall, "updates_per_s": upd / wall,
            "p50_ms": _pct(lat, 50), "p99_ms": _pct(lat, 99), "offered_rate_per_s": 200.0,
            "form": f"plain {prec}: one request at a time, one subdomain per launch, no graph"}


# ---- the oracle on the host's cores ----------------------------------------------------------

def _oracle_worker_init():
    # one thread per worker process: the pool supplies the parallelism
    for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[v] = "1"
    import oracle  # noqa: F401  (imported once per worker, outside the timed tasks)


def _oracle_instance(w):
    import oracle as O
    g = w["grid"]
    gs = O.GridSpec(tuple(g["n"]), tuple(g["lo"]), tuple(g["hi"]))
    t = w["time"]
    t0 = time.perf_counter()
    r = O.solve_single(gs, w["monitor"], t["dt"], t["gamma"], t["steps"])
    return r.mesh, r.min_det, r.min_cell, (r.res_hist[-1] if r.res_hist else 0.0), time.perf_counter() - t0


def _noop(_):
    return os.getpid()


def host_cores():
    """Logical CPUs visible to this process (capped at the 16 a one-GPU share of the box has)
    and the CPU model from lscpu."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    model = None
    try:
        import subprocess
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name"):
                model = line.split(":", 1)[1].strip()
    except Exception:
        pass
    return min(n, 16), os.cpu_count(), model


def cpu_baseline_batch(ws):
    """The FP64 oracle on every instance of the batch workload, one single-threaded process per
    host core (multiprocessing, spawn: the workers import only the oracle), all 200 steps of all
    256 instances; the pool is started and warmed before the clock.  Returns the baseline and the
    oracle's meshes (the reference for the per-result errors)."""
    import multiprocessing as mp
    cores, ncpu, model = host_cores()
    ctxm = mp.get_context("spawn")
    with ctxm.Pool(cores, initializer=_oracle_worker_init) as pool:
        pool.map(_noop, range(4 * cores))
        order = sorted(range(len(ws)), key=lambda i: -math.prod(ws[i]["grid"]["n"]))  # largest first
        t0 = time.perf_counter()
        res = pool.map(_oracle_instance, [ws[i] for i in order], chunksize=1)
        dt = time.perf_counter() - t0
    out = [None] * len(ws)
    for k, i in enumerate(order):
        out[i] = res[k]
    upd = sum(math.prod(w["grid"]["n"]) * w["time"]["steps"] for w in ws)
    base = {"value": upd / dt, "unit": "grid-point updates/s", "cores": cores, "kind": "oracle",
            "sample": f"the whole workload: all {len(ws)} instances x {ws[0]['time']['steps']} steps, "
                      f"FP64 NumPy/SciPy oracle, {cores} single-threaded processes (largest instances first), "
                      f"{dt:.1f} s wall, {sum(r[4] for r in res):.1f} s of CPU",
            "os_cpu_count": ncpu, "cpu_model": model}
    return base, out


def batch_accuracy(ctx, binding, ws, ref, prec):
    """Every instance solved by pma_dd_mesh_batch in `prec`, against the oracle's meshes: max node
    error / domain size per result, FP64 final residual, min det and min cell."""
    import numpy as np
    outs, stats = ctx.dd_mesh_batch(ws, precision=prec)
    err, res, dets, cells, cell_rel = [], [], [], [], []
    for i, w in enumerate(ws):
        ext = max(b - a for a, b in zip(w["grid"]["lo"], w["grid"]["hi"]))
        err.append(float(np.max(np.abs(outs[i] - ref[i][0]))) / ext)
        res.append(stats[i]["final_resid"])
        dets.append(stats[i]["min_det"])
        cells.append(stats[i]["min_cell"])
        cell_rel.append(abs(stats[i]["min_cell"] - ref[i][2]) / abs(ref[i][2]))
    r3 = lambda v: [float(f"{x:.3g}") for x in v]
    return {"precision": prec, "max_mesh_err_over_results": max(err), "median_mesh_err": float(np.median(err)),
            "tolerance": 1e-10 if prec == "fp64" else 1e-5,
            "max_min_cell_rel_diff": max(cell_rel),
            "max_final_resid_rel_diff": max(abs(a - b[3]) / b[3] for a, b in zip(res, ref)),
            "per_result": {"mesh_err": r3(err), "final_resid": r3(res), "min_det": r3(dets)}}


def cpu_baseline_sine(w, steps):
    """The oracle on the 513^2 4x4 DD workload, one process, scipy.fft over all cores."""
    import oracle as O
    import scipy.fft
    cores, _, _ = host_cores()
    g = w["grid"]
    gs = O.GridSpec(tuple(g["n"]), tuple(g["lo"]), tuple(g["hi"]))
    t = w["time"]
    with scipy.fft.set_workers(cores):
        t0 = time.perf_counter()
        O.solve_dd(gs, w["dd"]["parts"], w["dd"]["overlap"], w["monitor"], t["dt"], t["gamma"], steps)
        dt = time.perf_counter() - t0
    return {"value": math.prod(g["n"]) * steps / dt, "unit": "grid-point updates/s", "cores": cores,
            "sample": f"{steps} steps of the 513^2 4x4 DD workload, scipy.fft workers = {cores}, {dt:.1f} s"}


def sine_forms(ctx, binding, workloads, steps, warmup):
    w = workloads.sine_dd()
    forms = {}
    for f in ["split16", "fp32", "fp64plain", "fp64"]:
        prec, ex = ("fp64", "plain") if f == "fp64plain" else (f, "batched")
        st = steps if f != "fp64plain" else max(1, min(steps, 100))
        forms[f] = timed_plan(ctx, binding, [w], prec, ex, st, min(warmup, st), phase_reps=50, tune=ex == "batched")
        log(f"sine 513 {f}: {forms[f]['updates_per_s']:.4e} updates/s, {forms[f]['ms_per_step']:.4f} ms/step")
    out = {"workload": "sine-layer DD 513x513, 4x4 subdomains, overlap 8 cells, gamma = 4 h^2, dt = gamma / 5",
           "forms": {k: {kk: vv for kk, vv in v.items() if kk != "phases"} for k, v in forms.items()},
           "phases_ms_per_launch": {k: {p: round(v["ms"], 5) for p, v in f["phases"].items()}
                                    for k, f in forms.items()},
           "roofline_split16": roofline_of(forms["split16"]["phases"], "split16", "sine_dd_513_split16"),
           "batched_split16_over_plain_fp64": forms["split16"]["updates_per_s"] / forms["fp64plain"]["updates_per_s"],
           "glued_vs_single_domain": glued_vs_single(ctx, binding, w, "split16"),
           "persistent_step_split16": persistent_vs_phases(ctx, binding, w, "split16")}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--serve", type=int, default=2000, help="requests in the serving stream (0: skip)")
    ap.add_argument("--serve-small", type=int, default=500, help="requests in the 512 MiB serving stream")
    ap.add_argument("--serve-plain", type=int, default=40, help="requests of the stream served by the plain method")
    ap.add_argument("--quick", action="store_true", help="headline workload only")
    ap.add_argument("--only", choices=["fp64", "split16", "fp32", "fp64plain", "sine", "stencil_large", "paper",
                                       "shell", "serve", "ladder", "studies"], default=None,
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
    if args.only in ("paper", "shell", "stencil_large", "sine", "ladder", "studies"):
        ctx = binding.Context(0, budget_bytes=12 << 30)
        if args.only == "studies":
            r = {"studies": studies(ctx, binding, workloads)}
        elif args.only == "paper":
            r = {"paper_workloads": paper_workloads(ctx, binding, workloads)}
        elif args.only == "ladder":
            r = {"efficiency_ladder": efficiency_ladder(ctx, binding, workloads)}
        elif args.only == "shell":
            r = {"shell_dd_129_split16": shell_bench(ctx, binding, workloads, args.steps, args.warmup)}
        elif args.only == "sine":
            r = {"sine_dd_513": sine_forms(ctx, binding, workloads, args.steps, args.warmup)}
        else:
            r = {"stencil_hbm_large": stencil_roofline(ctx, binding, workloads)}
        print(json.dumps(r))
        ctx.close()
        return
    if args.only == "serve":
        r = {"budget_8GiB": serve_stream(binding, workloads, args.serve, 8 << 30)}
        if args.serve_small > 0:
            r["budget_512MiB"] = serve_stream(binding, workloads, args.serve_small, 512 << 20)
        if args.serve_plain > 0:
            r["plain_fp64_same_stream"] = serve_plain(binding, workloads, args.serve_plain)
            r["batched_same_prefix"] = serve_stream(binding, workloads, args.serve_plain, 8 << 30)
        print(json.dumps({"serving": r}))
        return

    batch = workloads.bumps_batch()
    ctx = binding.Context(0, budget_bytes=12 << 30)
    forms = {}
    todo = [args.only] if args.only else ["fp64", "split16", "fp32", "fp64plain"]
    for f in todo:
        prec, ex = ("fp64", "plain") if f == "fp64plain" else (f, "batched")
        steps = args.steps if f != "fp64plain" else max(1, min(args.steps, 10))
        forms[f] = timed_plan(ctx, binding, batch, prec, ex, steps, min(args.warmup, steps) if ex == "batched" else 1,
                              phase_reps=10 if ex == "batched" else 0, tune=ex == "batched")
        log(f"batch {f}: {forms[f]['updates_per_s']:.4e} updates/s, {forms[f]['ms_per_step']:.4f} ms/step")
    main_form = args.only or "fp64"
    m = forms[main_form]
    prec = "fp64" if main_form == "fp64plain" else main_form
    out = {
        "metric": "PMA grid-point updates/s, batched FP32 vs plain FP64, p50/p99 mesh latency",
        "value": m["updates_per_s"], "unit": "grid-point updates/s", "n_gpus": 1, "steps": m["steps"],
        "warmup": args.warmup, "ms_per_step": m["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": {"fp64": "f64", "split16": "f32", "fp32": "f32"}[prec], "data": "synthetic",
        "config": {"workload": "256 single-domain 2D meshes, sides U{33..257} (seed 20060146), 1-4 Gaussian bumps, "
                               "gamma = 1, dt = 1e-3, 200 steps",
                   "instances": len(batch), "nodes_per_step": nodes_of(batch),
                   "precision": {"split16": "fp32 state/stencil, fp16 hi+lo matrix-core DCT, fp32 accumulate",
                                 "fp32": "fp32 everywhere", "fp64": "fp64 everywhere (the paper's precision)"}[prec],
                   "exec": "plain" if main_form == "fp64plain" else "batched (graph replay)"},
        "forms": {k: {kk: vv for kk, vv in v.items() if kk != "phases"} for k, v in forms.items()},
        "phases_ms_per_launch": {k: {p: round(v["ms"], 5) for p, v in f["phases"].items()}
                                 for k, f in forms.items() if f["phases"]},
    }
    if m["phases"]:
        out["roofline"] = roofline_of(m["phases"], prec, "bumps_batch_256_" + prec)
        ksum = sum(v["ms"] for k, v in m["phases"].items() if k != "resid")
        out["kernel_ms_per_step"] = ksum
    if "split16" in forms and forms["split16"]["phases"]:
        out["roofline_split16"] = roofline_of(forms["split16"]["phases"], "split16", "bumps_batch_256_split16")
    if "fp64plain" in forms:
        for f in ("fp64", "split16", "fp32"):
            if f in forms:
                out[f"batched_{f}_over_plain_fp64"] = forms[f]["updates_per_s"] / forms["fp64plain"]["updates_per_s"]
    if not args.no_cpu and not args.only:
        base, ref = cpu_baseline_batch(batch)
        out["cpu_baseline"] = base
        log(f"oracle on {base['cores']} cores: {base['value']:.3e} updates/s")
        out["accuracy_vs_oracle"] = {p: batch_accuracy(ctx, binding, batch, ref, p) for p in ("fp64", "split16")}
    if not args.quick and not args.only:
        extra = {}
        extra["sine_dd_513"] = sine_forms(ctx, binding, workloads, 500, 20)
        ring = workloads.ring()
        r = timed_plan(ctx, binding, [ring], "fp64", "batched", 200, 10)
        extra["ring_65_fp64"] = {k: r[k] for k in ("updates_per_s", "ms_per_step")}
        log(f"ring 65^2 fp64: {r['updates_per_s']:.3e}")
        extra["shell_dd_129_split16"] = shell_bench(ctx, binding, workloads, 200, 5)
        extra["stencil_hbm_large"] = stencil_roofline(ctx, binding, workloads)
        log(f"stencil large: {extra['stencil_hbm_large']['achieved']:.0f} GB/s")
        if not args.no_cpu:
            extra["sine_dd_513"]["cpu_baseline"] = cpu_baseline_sine(workloads.sine_dd(), 300)
        out["other_workloads"] = extra
        out["paper_workloads"] = paper_workloads(ctx, binding, workloads)
        out["efficiency_ladder"] = efficiency_ladder(ctx, binding, workloads)
    ctx.close()
    if args.serve > 0 and not args.quick and not args.only:
        sv = {"budget_8GiB": serve_stream(binding, workloads, args.serve, 8 << 30)}
        log(f"serve 8GB: {sv['budget_8GiB']}")
        if args.serve_small > 0:
            sv["budget_512MiB"] = serve_stream(binding, workloads, args.serve_small, 512 << 20)
            log(f"serve 512MB: {sv['budget_512MiB']}")
        if args.serve_plain > 0:
            sv["plain_fp64_same_stream"] = serve_plain(binding, workloads, args.serve_plain)
            sv["batched_same_prefix"] = serve_stream(binding, workloads, args.serve_plain, 8 << 30)
            log(f"serve plain: {sv['plain_fp64_same_stream']}")
        out["serving"] = sv
    print(json.dumps(out))


if __name__ == "__main__":
    main()
