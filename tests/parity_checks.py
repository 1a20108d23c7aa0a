"""Comparison of the GPU's FP64 Jacobian check with the oracle's (shared by the GPU tests).

The minimum signed cell measure (2D: quadrilateral area by the shoelace formula; 3D: minimum
corner Jacobian of each hexahedron) is computed in FP64 on the GPU from the glued mesh, and by
the oracle from its own mesh.  Its difference follows from the mesh difference: each edge of a
cell moves by at most twice the mesh error, so the relative change of the measure is bounded by
about 2 d (mesh error) / h.  The bounds below hold that with margin: FP64 meshes agree to
~1e-13, the FP32 forms to ~1e-7 at h >= 1/512.  A wrong corner, orientation or index changes the
measure by O(1) relative and fails them.
"""

CELL_RTOL = {"fp64": 1e-8, "fp32": 2e-3, "split16": 2e-3}


def check_min_cell(got: float, ref: float, prec: str, label: str = "") -> float:
    rel = abs(got - ref) / abs(ref)
    print(f"min cell {label} {prec}: gpu {got:.12e} oracle {ref:.12e} rel {rel:.2e}", flush=True)
    assert got > 0 and ref > 0, (got, ref)
    assert rel <= CELL_RTOL[prec], (got, ref, rel)
    return rel
