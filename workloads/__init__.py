"""Seeded, synthetic inputs for the anisotropic-conduction LBM solver.

This package builds what the solver consumes -- a uint8 phase (material-id)
grid in ``[nz][ny][nx]`` order (x fastest) and a per-phase table of symmetric
3x3 conductivity tensors stored as ``(kxx, kyy, kzz, kxy, kxz, kyz)`` -- plus
the geometric/material calculators of the paper's braided unit cell.

It holds none of the lattice Boltzmann arithmetic (no relaxation times, no
collision, streaming, boundaries or flux evaluation).  Both the CPU oracle's
tests and the GPU path's tests/benchmarks draw their inputs from here, so the
two sides see identical media without sharing any solver code.
"""

from .media import (  # noqa: F401
    Medium,
    sym6,
    full3,
    rot_x,
    rot_y,
    rot_z,
    rotate_tensor,
    slab_tensor_eq26,
    transversely_isotropic,
    layered,
    c1_layered,
    table1_slabs,
    dual_component_cube,
    braid,
    braid_family_axes,
    random_medium,
    random_spd,
    sweep_cells,
    warmstart_cells,
    warmstart_cells_mixed,
)
from .unitcell import (  # noqa: F401
    PHI_Y_EXACT,
    PHI_Y_ROUNDED,
    paper_unit_cell,
    unit_cell_geometry,
    yarn_conductivities,
)
