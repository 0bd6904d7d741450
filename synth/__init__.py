"""Seeded synthetic inputs for the transit search (light curves, grids,
single-event shapes in ``synth.templates``).

Serves the oracle, the tests and the benchmark alike. Holds none of the
search's arithmetic; see ``synth.lightcurve`` for how curves are drawn.
"""
from .lightcurve import (  # noqa: F401
    Workload,
    config1,
    config2,
    config3,
    two_sectors,
    principle_e1,
    make_workload,
    lattice_box_mask,
    sample_sho_state_space,
    sho_omega_from_rotation,
    linspace_periods,
    quadratic_trend,
)
