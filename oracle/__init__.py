"""FP64 CPU oracle for the domain-decomposed projective-dynamics step.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and its
Python binding) may import, call or link anything here; only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` use it.
It shares no code with the HIP path: its only common ground is the seeded input
generator package ``synth``.
"""

from .pd import (  # noqa: F401
    OracleSim,
    assemble_L,
    element_geometry,
    deformation_gradient,
    signed_svd,
    proj_sl3,
    local_step,
    pd_energy,
)
from .dd import bisect_elements, DDSolver  # noqa: F401
