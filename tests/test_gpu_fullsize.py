"""Parity at the full workload sizes, in the launch configuration the benchmark times (resident
plan, all subdomains per launch, graph replay).

Expected values: tests/golden/*.npz, written by tests/golden/make_golden.py from the FP64 oracle
alone (strided + seeded random node samples of the glued mesh).  The 256-instance batch is
checked against live oracle runs of sampled instances.
"""
import os

import numpy as np
import pytest

import oracle as O
from paper_2006_14602_amd import workloads as W
from parity_checks import check_min_cell

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
TOL = {"fp64": 1e-10, "fp32": 1e-5, "split16": 1e-5}


@pytest.fixture(scope="module")
def ctx(lib):
    from paper_2006_14602_amd import binding
    c = binding.Context(0, budget_bytes=8 << 30)
    yield c
    c.close()


def gspec(w):
    g = w["grid"]
    return O.GridSpec(tuple(g["n"]), tuple(g["lo"]), tuple(g["hi"]))


def golden(name):
    return np.load(os.path.join(HERE, "golden", name + ".npz"))


def plan_mesh(ctx, w, prec, exec_="batched"):
    from paper_2006_14602_amd import binding
    with binding.Plan(ctx, [w], prec, exec_) as p:
        p.step(w["time"]["steps"])
        p.sync()
        return p.mesh(0)


@pytest.mark.parametrize("prec", ["split16", "fp32", "fp64"])
def test_sine_dd_513_full(ctx, prec):
    w = W.sine_dd()
    gd = golden("sine_dd_513")
    mesh, st = plan_mesh(ctx, w, prec, "plain" if prec == "fp64" else "batched")
    idx = gd["idx"]
    got = np.stack([mesh[k][tuple(idx.T)] for k in range(2)], -1)
    err = float(np.max(np.abs(got - gd["mesh"])))
    print(f"sine_dd_513 {prec}: max err over {len(idx)} sampled nodes {err:.3e}, min det {st['min_det']:.6f}")
    assert err <= TOL[prec]
    assert abs(st["min_det"] - float(gd["min_det"])) <= (1e-9 if prec == "fp64" else 1e-3)
    check_min_cell(st["min_cell"], float(gd["min_cell"]), prec, "sine_dd_513")
    # faces stay put (Sec. 2, eq. nbd)
    assert np.all(mesh[0][0, :] == 0.0) and np.all(mesh[0][-1, :] == 1.0)
    assert np.all(mesh[1][:, 0] == 0.0) and np.all(mesh[1][:, -1] == 1.0)


@pytest.mark.parametrize("prec", ["split16", "fp64"])
def test_shell_dd_129_full(ctx, prec):
    w = W.shell_dd()
    gd = golden("shell_dd_129")
    mesh, st = plan_mesh(ctx, w, prec)
    idx = gd["idx"]
    got = np.stack([mesh[k][tuple(idx.T)] for k in range(3)], -1)
    err = float(np.max(np.abs(got - gd["mesh"])))
    print(f"shell_dd_129 {prec}: max err {err:.3e}, min det {st['min_det']:.6f}")
    assert err <= TOL[prec]
    assert st["min_det"] > 0
    check_min_cell(st["min_cell"], float(gd["min_cell"]), prec, "shell_dd_129")
    for k in range(3):
        sl0 = [slice(None)] * 3
        sl0[k] = 0
        sl1 = [slice(None)] * 3
        sl1[k] = -1
        assert np.all(mesh[k][tuple(sl0)] == 0.0) and np.all(mesh[k][tuple(sl1)] == 1.0)


def test_bumps_batch_256_full(ctx):
    ws = W.bumps_batch()
    outs, stats = ctx.dd_mesh_batch(ws, precision="split16")
    assert all(s["min_det"] > 0 and s["min_cell"] > 0 and s["steps_done"] == 200 for s in stats)
    rng = np.random.default_rng(5)
    pick = sorted(set([int(np.argmin([w["grid"]["n"][0] for w in ws])), int(np.argmax([w["grid"]["n"][0] for w in ws]))]
                      + list(rng.choice(len(ws), 2, replace=False))))
    for i in pick:
        w = ws[i]
        g = w["grid"]
        ref = O.solve_single(O.GridSpec(tuple(g["n"]), tuple(g["lo"]), tuple(g["hi"])), w["monitor"],
                             w["time"]["dt"], w["time"]["gamma"], w["time"]["steps"])
        err = float(np.max(np.abs(outs[i] - ref.mesh)))
        print(f"bump {i} n={g['n'][0]}: err {err:.3e}")
        assert err <= TOL["split16"]
        check_min_cell(stats[i]["min_cell"], ref.min_cell, "split16", f"bump {i}")


PAPER = {
    "sine_dd_513_alt": lambda: dict(W.sine_dd(steps=200), dd={"parts": [4, 4], "overlap": [8, 8],
                                                               "mode": "alternating"}),
    "burgers_front_65": lambda: W.burgers_front(parts=(4, 1), steps=300),
    "spiral_257": lambda: W.spiral(steps=300),
    "sphere_81": lambda: W.sphere_3d(n=81, steps=150),
    "spheres9_81": lambda: W.spheres9_3d(n=81, steps=150),
}


@pytest.mark.parametrize("prec", ["split16", "fp64"])
@pytest.mark.parametrize("name", list(PAPER))
def test_paper_workload_full(ctx, name, prec):
    # the paper's examples and the alternating headline split, at the benchmarked sizes and launch
    # configuration, against oracle samples; the oracle's theta is handed to the library
    w = PAPER[name]()
    gd = golden(name)
    w["monitor"] = dict(w["monitor"], theta=float(gd["theta"]))
    print(f"case {name} {prec}", flush=True)
    mesh, st = plan_mesh(ctx, w, prec)
    d = w["grid"]["dim"]
    idx = gd["idx"]
    got = np.stack([mesh[k][tuple(idx.T)] for k in range(d)], -1)
    ext = max(b - a for a, b in zip(w["grid"]["lo"], w["grid"]["hi"]))
    err = float(np.max(np.abs(got - gd["mesh"]))) / ext
    print(f"{name} {prec}: max err over {len(idx)} sampled nodes {err:.3e}, min det {st['min_det']:.6f} "
          f"(oracle {float(gd['min_det']):.6f}), E2 {st['quality_e2']:.4f}")
    assert err <= TOL[prec]
    assert abs(st["min_det"] - float(gd["min_det"])) <= (1e-9 if prec == "fp64" else 2e-3)
    check_min_cell(st["min_cell"], float(gd["min_cell"]), prec, name)


@pytest.mark.parametrize("prec", ["split16", "fp64"])
def test_sine_513_glued_dd_vs_single_domain(ctx, prec):
    # the glued 4 x 4 mesh against the whole-domain mesh of the same problem (same gamma, dt and
    # steps): the GPU's whole-domain mesh matches the oracle's, and the gap between the two meshes
    # on the GPU is the oracle's gap (the decomposition error of Sec. 4.4, not a GPU artefact)
    w = W.sine_dd()
    ws = dict(w, dd=None)
    gd, gs = golden("sine_dd_513"), golden("sine_single_513")
    idx = gs["idx"]
    assert np.array_equal(idx, gd["idx"])
    single, st = plan_mesh(ctx, ws, prec)
    dd, _ = plan_mesh(ctx, w, prec)
    pick = lambda m: np.stack([m[k][tuple(idx.T)] for k in range(2)], -1)
    err = float(np.max(np.abs(pick(single) - gs["mesh"])))
    gap_gpu = float(np.max(np.abs(pick(dd) - pick(single))))
    gap_oracle = float(np.max(np.abs(gd["mesh"] - gs["mesh"])))
    print(f"sine 513 {prec}: single-domain err {err:.3e}; glued DD - single: GPU {gap_gpu:.4e}, oracle {gap_oracle:.4e}")
    assert err <= TOL[prec]
    assert abs(gap_gpu - gap_oracle) <= 2 * TOL[prec]
    assert st["min_det"] > 0
    check_min_cell(st["min_cell"], float(gs["min_cell"]), prec, "sine_single_513")


def test_serving_stream_requests_full_size(ctx):
    # requests of the Poisson stream itself, at their own sizes, served in a mix with their stream
    # neighbours: the smallest 2D and 3D ones of each kind (single domain and decomposed) against
    # the oracle; every request of the mix completes with a valid mesh
    from paper_2006_14602_amd import binding
    import time
    ws = W.stream(count=2000)
    picks = [747, 887, 1062, 1687]          # 65^2 single, 33^3 single, 258^2 2x2, 66^3 2x2x2
    mix = picks + list(range(10))           # plus the first arrivals of the stream
    with binding.Context(0, budget_bytes=4 << 30) as c:
        tickets = [c.submit(ws[i], "split16") for i in mix]
        res = {}
        t0 = time.time()
        while len(res) < len(mix):
            for i, t in zip(mix, tickets):
                if i in res:
                    continue
                shape = (ws[i]["grid"]["dim"],) + tuple(ws[i]["grid"]["n"])
                state, mesh, st = c.poll(t, shape=shape)
                if state in (binding.DONE, binding.FAILED):
                    res[i] = (state, mesh, st)
            assert time.time() - t0 < 240, "serving did not finish"
            time.sleep(0.002)
    for i in mix:
        assert res[i][0] == binding.DONE, (i, res[i][2])
        assert res[i][2]["min_det"] > 0 and res[i][2]["min_cell"] > 0
    for i in picks:
        w = ws[i]
        t = w["time"]
        g = gspec(w)
        print(f"case stream request {i} n={w['grid']['n'][0]} dd={w['dd']}", flush=True)
        if w["dd"]:
            ref = O.solve_dd(g, w["dd"]["parts"], w["dd"]["overlap"], w["monitor"], t["dt"], t["gamma"], t["steps"])
        else:
            ref = O.solve_single(g, w["monitor"], t["dt"], t["gamma"], t["steps"])
        err = float(np.max(np.abs(res[i][1] - ref.mesh)))
        print(f"stream request {i}: max mesh err {err:.3e}")
        assert err <= TOL["split16"]
        check_min_cell(res[i][2]["min_cell"], ref.min_cell, "split16", f"stream {i}")


@pytest.mark.parametrize("name,prec", [("sphere_81", "fp64"), ("spiral_257", "split16"), ("burgers_front_65", "fp64")])
def test_paper_workload_full_library_theta(ctx, name, prec):
    # the same runs with the library computing theta itself (its reduced integrals or quadrature)
    w = PAPER[name]()
    assert not w["monitor"].get("theta")
    gd = golden(name)
    print(f"case {name} {prec} own theta", flush=True)
    mesh, st = plan_mesh(ctx, w, prec)
    d = w["grid"]["dim"]
    idx = gd["idx"]
    got = np.stack([mesh[k][tuple(idx.T)] for k in range(d)], -1)
    ext = max(b - a for a, b in zip(w["grid"]["lo"], w["grid"]["hi"]))
    err = float(np.max(np.abs(got - gd["mesh"]))) / ext
    print(f"{name} {prec} own theta {st['theta']:.12g} (oracle {float(gd['theta']):.12g}): max err {err:.3e}")
    assert err <= TOL[prec]
    check_min_cell(st["min_cell"], float(gd["min_cell"]), prec, name + " own theta")
