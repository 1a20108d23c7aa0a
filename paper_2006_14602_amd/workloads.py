"""Seeded synthetic workloads for the DD-PMA mesh generator.

This module only draws and names inputs (grids, decompositions, monitor parameters, step
parameters, arrival times).  It evaluates nothing of the method itself, so both the GPU path
and the FP64 oracle can be fed from it without sharing solver code.

Workloads follow the paper's experiments in kind (analytic monitors on box domains, Sec. 4):
  ring        2D 65^2 single domain, rho = 1 + 10 sech^2(50(|x - (1/2,1/2)|^2 - 1/16)),
              200 steps, dt = 1e-3, gamma = 1
  sine_dd     2D 513^2, 4x4 subdomains, overlap 8 cells,
              rho = 1 + 20 sech^2(40(y - 1/2 - sin(2 pi x)/4)), 500 steps
  shell_dd    3D 129^3, 2x2x2 subdomains, overlap 6 cells,
              rho = 1 + 15 sech^2(30(|x - c|^2 - 0.09)), c = (1/2,1/2,1/2), 200 steps
  bumps_batch 256 single-domain 2D instances, sides U{33..257}, 1..4 Gaussian bumps
  stream      Poisson request stream, 70% 2D (65..1025 per side), 30% 3D (33..193 per side)
The paper's own examples use the arc-length monitor rho = sqrt(1 + |grad u|^2) of given
functions u (Sec. 4): burgers_front (Sec. 4.1, 65^2, 4 slabs / 2 x 2 blocks, overlap 3 points),
spiral (Sec. 4.1), sphere_3d and spheres9_3d (Sec. 4.2, eight blocks).

Subdomain runs use gamma = 4 h^2 and dt = gamma / 5 (the largest h over axes); single-domain runs
use gamma = 1 and dt = 1e-3.
"""
from __future__ import annotations

import math

import numpy as np

CFG4_SEED = 20060146
CFG5_SEED = 20060147


def grid(n, lo=None, hi=None):
    d = len(n)
    return {"dim": d, "n": list(n), "lo": list(lo or [0.0] * d), "hi": list(hi or [1.0] * d)}


def dd_defaults(g: dict) -> dict:
    """gamma = 4 h^2, dt = gamma / 5 for decomposed runs."""
    h = max((b - a) / (n - 1) for a, b, n in zip(g["lo"], g["hi"], g["n"]))
    gamma = 4.0 * h * h
    return {"gamma": gamma, "dt": 0.2 * gamma}


def ring_monitor(d=2, amp=10.0, k=50.0, r0=0.25, c=0.5):
    return {"kind": "sech2_radial", "amp": amp, "k": k, "r0": r0, "c": [c] * d}


def sine_monitor(amp=20.0, k=40.0, r0=0.25, c1=0.5):
    return {"kind": "sech2_sine", "amp": amp, "k": k, "r0": r0, "c": [0.0, c1]}


def shell_monitor(amp=15.0, k=30.0, r0=0.3, c=0.5):
    return {"kind": "sech2_radial", "amp": amp, "k": k, "r0": r0, "c": [c, c, c]}


def const_monitor(amp=1.0):
    return {"kind": "const", "amp": amp}


def separable_monitor(amps, ks, cs):
    return {"kind": "separable_sech2", "amp_axes": list(amps), "k_axes": list(ks), "c": list(cs)}


def front_monitor(eps=0.01, offset=1.0):
    """Arc-length monitor of the 2D Burgers front u = 1 / (1 + exp((x + y - offset) / (2 eps)))
    (Sec. 4.1, first example)."""
    return {"kind": "arclen_front", "eps": eps, "offset": offset}


def spiral_monitor(amp=9.0, k=100.0, twist=20.0, c=(0.7, 0.5)):
    """Arc-length monitor of u = 1 + amp / (1 + k r^2 cos^2(theta - twist r^2)), polar
    coordinates about c (Sec. 4.1, second example)."""
    return {"kind": "arclen_spiral", "amp": amp, "k": k, "twist": twist, "c": list(c)}


def spheres_monitor(k, r0, centres):
    """Arc-length monitor of u = sum_b tanh(k (|x - c_b|^2 - r0^2)) (Sec. 4.2)."""
    return {"kind": "arclen_spheres", "k": k, "r0": r0, "bc": [list(map(float, c)) for c in centres]}


# Sec. 4.2, second example: nine spheres of radius^2 0.1875
NINE_CENTRES = [(0.0, 0.0, 0.0), (0.5, 0.5, 0.5), (0.5, -0.5, 0.5), (-0.5, 0.5, 0.5), (-0.5, -0.5, 0.5),
                (0.5, 0.5, -0.5), (0.5, -0.5, -0.5), (-0.5, 0.5, -0.5), (-0.5, -0.5, -0.5)]


def _arclen_time(g: dict, dd, dt_frac: float, steps: int) -> dict:
    if dd:
        t = dd_defaults(g)
        t["dt"] = dt_frac * t["gamma"]
    else:
        t = {"dt": 1e-3, "gamma": 1.0}
    t["steps"] = steps
    return t


def burgers_front(n=65, parts=(4, 1), overlap=2, mode="alternating", steps=300):
    """Sec. 4.1, first example: 65^2 on the unit square, 4 slabs or 2 x 2 blocks overlapping by
    three grid points (2 cells), alternating sweeps."""
    g = grid([n, n])
    dd = {"parts": list(parts), "overlap": [overlap] * 2, "mode": mode} if parts and max(parts) > 1 else None
    return {"name": f"burgers_front_{n}", "grid": g, "dd": dd, "monitor": front_monitor(),
            "time": _arclen_time(g, dd, 0.2, steps)}


def spiral(n=257, parts=(4, 4), overlap=4, mode="parallel", steps=300):
    """Sec. 4.1, second example.  Its ridges need dt = gamma / 50 on decomposed runs."""
    g = grid([n, n])
    dd = {"parts": list(parts), "overlap": [overlap] * 2, "mode": mode} if parts and max(parts) > 1 else None
    return {"name": f"spiral_{n}", "grid": g, "dd": dd, "monitor": spiral_monitor(),
            "time": _arclen_time(g, dd, 0.02, steps)}


def sphere_3d(n=81, parts=(2, 2, 2), overlap=2, mode="alternating", steps=150):
    """Sec. 4.2, first example: u = tanh(100(|x|^2 - 0.125)) on (-1,1)^3, eight blocks."""
    g = grid([n] * 3, [-1.0] * 3, [1.0] * 3)
    dd = {"parts": list(parts), "overlap": [overlap] * 3, "mode": mode} if parts and max(parts) > 1 else None
    return {"name": f"sphere_{n}", "grid": g, "dd": dd,
            "monitor": spheres_monitor(100.0, math.sqrt(0.125), [(0.0, 0.0, 0.0)]),
            "time": _arclen_time(g, dd, 0.02, steps)}


def spheres9_3d(n=81, parts=(2, 2, 2), overlap=2, mode="alternating", steps=150):
    """Sec. 4.2, second example: nine tanh spheres on (-2,2)^3, eight blocks."""
    g = grid([n] * 3, [-2.0] * 3, [2.0] * 3)
    dd = {"parts": list(parts), "overlap": [overlap] * 3, "mode": mode} if parts and max(parts) > 1 else None
    return {"name": f"spheres9_{n}", "grid": g, "dd": dd,
            "monitor": spheres_monitor(50.0, math.sqrt(0.1875), NINE_CENTRES),
            "time": _arclen_time(g, dd, 0.02, steps)}


def ring(steps=200):
    return {"name": "ring_65", "grid": grid([65, 65]), "dd": None, "monitor": ring_monitor(),
            "time": {"dt": 1e-3, "gamma": 1.0, "steps": steps}}


def sine_dd(n=513, parts=(4, 4), overlap=8, steps=500):
    g = grid([n, n])
    t = dd_defaults(g)
    t["steps"] = steps
    return {"name": f"sine_dd_{n}", "grid": g, "dd": {"parts": list(parts), "overlap": [overlap] * 2},
            "monitor": sine_monitor(), "time": t}


def shell_dd(n=129, parts=(2, 2, 2), overlap=6, steps=200):
    g = grid([n, n, n])
    t = dd_defaults(g)
    t["steps"] = steps
    return {"name": f"shell_dd_{n}", "grid": g, "dd": {"parts": list(parts), "overlap": [overlap] * 3},
            "monitor": shell_monitor(), "time": t}


def _bumps(rng, d):
    K = int(rng.integers(1, 5))
    amps = [float(v) for v in rng.uniform(5.0, 30.0, K)]
    ws = [float(v) for v in rng.uniform(0.02, 0.15, K)]
    cs = [[float(v) for v in rng.uniform(0.0, 1.0, d)] for _ in range(K)]
    return {"kind": "gauss_sum", "bamp": amps, "bw": ws, "bc": cs}


def bumps_batch(count=256, seed=CFG4_SEED, steps=200, n_lo=33, n_hi=257):
    """Independent single-domain 2D instances of uneven size."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(rng.integers(n_lo, n_hi + 1))
        mon = _bumps(rng, 2)
        out.append({"name": f"bump_{i}", "grid": grid([n, n]), "dd": None, "monitor": mon,
                    "time": {"dt": 1e-3, "gamma": 1.0, "steps": steps}})
    return out


def stream(count=2000, seed=CFG5_SEED, rate=200.0, steps=200):
    """Open-loop Poisson stream of mesh requests; decomposition chosen per size:
    M = ceil((n-1)/256) parts per axis in 2D, ceil((n-1)/64) in 3D, overlap 8 / 6 cells."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(count):
        t += float(rng.exponential(1.0 / rate))
        if rng.uniform() < 0.7:
            d = 2
            n = int(rng.integers(65, 1026))
            M = math.ceil((n - 1) / 256)
            ov = 8
        else:
            d = 3
            n = int(rng.integers(33, 194))
            M = math.ceil((n - 1) / 64)
            ov = 6
        g = grid([n] * d)
        mon = _bumps(rng, d)
        if M > 1:
            tm = dd_defaults(g)
            dd = {"parts": [M] * d, "overlap": [ov] * d}
        else:
            tm = {"dt": 1e-3, "gamma": 1.0}
            dd = None
        tm["steps"] = steps
        out.append({"name": f"req_{i}", "arrival_s": t, "grid": g, "dd": dd, "monitor": mon, "time": tm})
    return out


def global_nodes(w: dict) -> int:
    return int(np.prod(w["grid"]["n"]))
