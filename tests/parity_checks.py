"""Comparison of the GPU's FP64 Jacobian check with the oracle's (shared by the GPU tests).

The minimum signed cell measure (2D: quadrilateral area by the shoelace formula; 3D: minimum
corner Jacobian of each hexahedron) is computed in FP64 on the GPU from the glued mesh, and by
the oracle from its own mesh.  Its difference follows from the mesh difference: each edge of a
cell moves by at most twice the mesh error, so the relative change of the measure is bounded by
about 2 d (mesh error) / h.  The bounds below hold that with margin.  Measured on MI355X: FP64
up to 2e-10 relative (the 545-node axes, h = 1/544, where the FP64 mesh error is ~1e-13 of a
cell of ~2e-3 x 0.11); the FP32 forms up to 1.6e-3 (FP32 at the 545-node axes: mesh error
~4e-6, skinny cells), below 1e-3 elsewhere.  A wrong corner, orientation or index changes the
measure by O(1) relative and fails them.
"""

CELL_RTOL = {"fp64": 1e-8, "fp32": 5e-3, "split16": 5e-3}


def check_min_cell(got: float, ref: float, prec: str, label: str = "", mesh_err: float = 0.0,
                   h: float = 1.0, dim: int = 2) -> float:
    """mesh_err, h, dim: the measured max node error, the smallest spacing and the dimension; the
    bound is then also at least 4 dim mesh_err / h (twice the first-order estimate above), which
    matters for the finest spacings (FP32 at 1025-node axes: 5.3e-3 measured)."""
    rel = abs(got - ref) / abs(ref)
    tol = max(CELL_RTOL[prec], 4.0 * dim * mesh_err / h)
    print(f"min cell {label} {prec}: gpu {got:.12e} oracle {ref:.12e} rel {rel:.2e} (bound {tol:.1e})", flush=True)
    assert got > 0 and ref > 0, (got, ref)
    assert rel <= tol, (got, ref, rel)
    return rel
