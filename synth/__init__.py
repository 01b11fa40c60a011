"""Seeded synthetic inputs for the GCB greedy RBF workloads.

This module produces coordinates, displacement fields, volume point clouds,
deformation modes and request streams only.  It holds none of the method's
arithmetic (no basis function, no interpolant, no solve), so that the CPU
oracle and the HIP library can both be fed from it without sharing code.

Every draw comes from ``numpy.random.PCG64`` seeded with
``SeedSequence([base, stream])``; streams: 1 surface, 2 volume, 4 modes,
5 arrivals (stream 3 is the partition seed, consumed by splitmix64 inside the
library and the oracle themselves).
"""
from .geometry import (  # noqa: F401
    rng, ellipsoid_surface, ellipsoid_field, ellipsoid_volume,
    wing_surface, wing_field, wing_volume, wing_mode_basis, random_modes,
    WING_HALF_SPAN, WING_ROOT_CHORD, WING_TAPER, WING_SWEEP_DEG,
)
from .configs import (  # noqa: F401
    Problem, config_small_ellipsoid, config_wing, config_wing_large,
    config_modes, config_multi_surface, multi_surface_problem, config_requests, request_mesh, request_field, tiny_problem,
    partition_seed,
)
