"""Seeded synthetic inputs shared by the CPU oracle and the HIP path.

This package holds parameter draws and random test states only.  It contains
none of the method's arithmetic (no Hamiltonians, bath terms or propagation):
both sides read the same plain dictionaries and arrays produced here.
"""

from .configs import (  # noqa: F401
    FS_PER_TIME_UNIT,
    FS_PER_TIME_UNIT_WATER,
    WATER_OMEGA0_CM,
    cfg1,
    cfg2,
    cfg3,
    cfg3_brownian,
    cfg4_instances,
    cfg5,
    cfg5_small,
    apply_theta,
    theta_directions,
    theta_size,
    harmonic_pin,
    paper_scale,
    fs_to_steps,
    response_grid,
    with_brownian_baths,
    water_beta,
    water_three_mode,
    water_two_mode,
)
from .states import random_hierarchy  # noqa: F401
