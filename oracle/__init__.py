"""FP64 CPU oracle for the DD-PMA mesh method (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this package.  The
product library never imports it and shares no code with it.
"""
from .pma_oracle import (  # noqa: F401
    Box, Decomposition, GridSpec, NonFiniteError, Result, TangledError, assemble_neumann_laplacian_1d,
    derivatives, det_sym, equidistribution_exact_sech2, ghost_pad, initial_psi, mesh_from_psi,
    min_cell_measure, min_det_hessian, neumann_mu, owner_axis, partition_axis, precondition,
    grad_u, quality, quality_of_mesh, rel_errors, rhs_F, rho, solve_dd, solve_single, step_box, sweep_order, theta,
    theta_closed_form, theta_quadrature, theta_reduced,
)
