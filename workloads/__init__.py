"""Seeded synthetic problem instances for the stochastic Helmholtz solver.

This package only *describes problems*: grids, the wavenumber fields
k_0..k_s at the nodes, the source f and the solver settings.  It holds none of
the method's arithmetic (no basis, no Galerkin projection, no finite
differences, no solver), so both the CPU oracle and the GPU path may import it.
"""
from .configs import (  # noqa: F401
    Instance,
    grid_rule_q,
    sine_mode_fields,
    gaussian_source,
    point_source,
    config1,
    config2,
    config3,
    config4_instances,
    config5_instance,
    small_2d,
    degree_sweep_instance,
    one_d_paper,
    wedge_instance,
    MODES,
)
