"""Seeded synthetic scenario generators shared by the oracle tests and the GPU harness.

This package draws random numbers and returns plain parameter dictionaries.  It holds
none of the value-iteration arithmetic: no demand PMFs, no transitions, no rewards,
no state counts.  Each side (oracle and library) builds its own tables from these
parameters.
"""
from .scenarios import (  # noqa: F401
    scenario_a,
    scenario_b,
    scenario_c,
    scenario_a_paper,
    PAPER_A_EXPERIMENTS,
    scenario_c_paper,
    PAPER_C_EXPERIMENTS,
    PAPER_C_RUL_LARGE,
    scenario_b1,
    scenario_b_paper,
    PAPER_B_EXPERIMENTS,
    config0,
    config1,
    config2,
    config3,
    config_by_index,
    serving_mix,
    random_values,
    sample_indices,
)
