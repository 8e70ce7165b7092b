"""FP64 CPU oracle for the D3Q19 adaptive volumetric-flux LBM step.

TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` may import this package. It shares no code with
the HIP library (``paper_1806_10589_amd``) and never imports it.
"""
from .oracle import (  # noqa: F401
    OracleColour,
    OracleLattice,
    mrt_collide_site,
    mrt_collide_site_rates,
    mrt_matrix,
    build,
    equilibrium,
    inlet_bc_site,
    outlet_bc_site,
    velocity_set,
    Z_FLUX,
    Z_PERIODIC,
    Z_WALL,
)
