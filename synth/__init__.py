"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This package only builds inputs: rest meshes (structured hex grids split into
tetrahedra), per-element material weights, lumped nodal masses, pinned sets and
initial states.  It holds none of the simulation method's arithmetic (no
deformation gradients, projections, matrices or solves), so that the oracle and
the HIP path share nothing beyond their inputs.
"""

from .meshes import (  # noqa: F401
    Problem,
    box_grid,
    cylinder_shell,
    make_box_problem,
    make_shell_problem,
    problem_by_name,
    serving_garment_sizes,
    serving_shell_problem,
)
from .yarn import yarn_points  # noqa: F401
