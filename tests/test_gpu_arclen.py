"""GPU parity on the paper's own workloads: arc-length monitors rho = sqrt(1 + |grad u|^2) of the
test functions of Sec. 4 (Burgers front, spiral, one sphere, nine spheres), single domain and
decomposed (slabs / blocks, alternating and parallel), against the FP64 oracle.

Where the oracle's tensor quadrature of theta = int rho is only accurate to ~1e-7 (spiral) or
too slow at the paper's sharpness (nine spheres), the oracle's theta is handed to both sides, so
both solve the same discrete problem.  Tolerances as for the other parity tests, on the mesh
relative to the box size.
"""
import copy
import functools
import math

import numpy as np
import pytest

import oracle as O
from paper_2006_14602_amd import workloads as W
from parity_checks import check_min_cell

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32": 1e-5, "split16": 1e-5}


@pytest.fixture(scope="module")
def ctx(lib):
    from paper_2006_14602_amd import binding
    c = binding.Context(0, budget_bytes=2 << 30)
    yield c
    c.close()


def gspec(w):
    g = w["grid"]
    return O.GridSpec(tuple(g["n"]), tuple(g["lo"]), tuple(g["hi"]))


def steps(w, n):
    w["time"]["steps"] = n
    return w


def with_theta(w, panels=None):
    g = w["grid"]
    th = O.theta_quadrature(w["monitor"], g["lo"], g["hi"], panels=panels) if panels else \
        O.theta(w["monitor"], g["lo"], g["hi"])
    w["monitor"] = dict(w["monitor"], theta=th)
    return w


CASES = {
    "front65_single": lambda: steps(W.burgers_front(parts=None), 100),
    "front65_slabs4_alternating": lambda: steps(W.burgers_front(parts=(4, 1)), 100),
    "front65_blocks2x2_alternating": lambda: steps(W.burgers_front(parts=(2, 2)), 100),
    "spiral129_single": lambda: with_theta(steps(W.spiral(n=129, parts=None), 60)),
    "spiral129_blocks2x2_parallel": lambda: with_theta(steps(W.spiral(n=129, parts=(2, 2)), 80)),
    # 33^3 leaves the shell unresolved (h = 1/16 against a width ~ 1/70): by step 40 a corner
    # Jacobian of the mesh turns negative (oracle and GPU agree), so stop at 20
    "sphere33_blocks8_alternating": lambda: steps(W.sphere_3d(n=33), 20),
    "sphere25_single": lambda: steps(W.sphere_3d(n=25, parts=None), 30),
    "spheres9_33_blocks8_alternating": lambda: with_theta(steps(W.spheres9_3d(n=33), 30), panels=24),
}


@functools.lru_cache(maxsize=None)
def oracle_of(name):
    w = CASES[name]()
    t = w["time"]
    if w.get("dd"):
        return O.solve_dd(gspec(w), w["dd"]["parts"], w["dd"]["overlap"], w["monitor"], t["dt"], t["gamma"],
                          t["steps"], mode=w["dd"].get("mode", "parallel"))
    return O.solve_single(gspec(w), w["monitor"], t["dt"], t["gamma"], t["steps"])


def extent(w):
    g = w["grid"]
    return max(b - a for a, b in zip(g["lo"], g["hi"]))


@pytest.mark.parametrize("prec", ["fp64", "fp32", "split16"])
@pytest.mark.parametrize("name", list(CASES))
def test_arclen_workload_vs_oracle(ctx, name, prec):
    w = CASES[name]()
    print(f"case {name} {prec}", flush=True)
    mesh, _, st = ctx.dd_mesh(w, precision=prec)
    ref = oracle_of(name)
    err = float(np.max(np.abs(mesh - ref.mesh))) / extent(w)
    print(f"{name} {prec}: max mesh err {err:.3e}, min det {st['min_det']:.4f} (oracle {ref.min_det:.4f})")
    assert err <= TOL[prec], err
    assert st["min_det"] > 0
    assert abs(st["min_det"] - ref.min_det) < (1e-8 if prec == "fp64" else 1e-3)
    check_min_cell(st["min_cell"], ref.min_cell, prec, name)


def test_arclen_front_mesh_symmetric_on_gpu(ctx):
    # rho of the front is invariant under the swap of axes: so is the GPU mesh, bit for bit in the
    # single-domain FP64 form up to the rounding of mirrored operations
    w = CASES["front65_single"]()
    mesh, _, _ = ctx.dd_mesh(w, precision="fp64")
    assert np.max(np.abs(mesh[0] - mesh[1].T)) < 1e-12


def test_folded_mesh_reported_like_the_oracle(ctx, lib):
    # the same unresolved sphere, run on: the oracle's final mesh has a cell of negative measure
    # and the library reports the request as folded
    from paper_2006_14602_amd import binding as B
    w = steps(W.sphere_3d(n=33), 40)
    t = w["time"]
    ref = O.solve_dd(gspec(w), w["dd"]["parts"], w["dd"]["overlap"], w["monitor"], t["dt"], t["gamma"],
                     t["steps"], mode="alternating")
    assert ref.min_cell < 0 < ref.min_det
    with pytest.raises(B.PmaError) as e:
        ctx.dd_mesh(w, precision="fp64")
    assert e.value.code == B.PMA_E_TANGLED
