"""Workload recipes.  Each returns plain arrays plus scalar parameters.

Sizes follow the five workloads the hot path is measured on: a small
ellipsoid (Nb = 2,000, Nv = 50,000), the 80,000-node wing with 3,000,000
volume points, a 300,000-node wing with 20,000,000 volume points, 64 wing
modes as multiple right-hand sides, 32 uneven independent surfaces, and a
Poisson request stream.  These synthetic surfaces stand in for the paper's
ONERA M6 and DLR-F6 meshes (Sections 4.1 and 4.2), which are not available.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from . import geometry as g

# base seeds per workload; stream ids: 1 surface, 2 volume, 3 partition, 4 modes, 5 arrivals
SEED_SMALL, SEED_WING, SEED_WING_LARGE, SEED_MODES, SEED_MULTI, SEED_REQUESTS = 1, 2, 3, 41, 42, 5


def partition_seed(base: int) -> int:
    """64-bit seed handed to the splitmix64 partition of the boundary nodes."""
    return int(np.random.SeedSequence([int(base), 3]).generate_state(1, dtype=np.uint64)[0])


@dataclasses.dataclass
class Problem:
    name: str
    xyz: np.ndarray          # (nb, 3) float64 boundary coordinates
    disp: np.ndarray         # (nb, 3) float64 prescribed boundary displacements
    radius: float            # Wendland support radius R
    m: int                   # number of groups
    tol_rel: float           # tolerance relative to max_j |disp_j|
    seed: int                # partition seed (splitmix64)
    nc_max: int
    volume: np.ndarray | None = None   # (nv, 3) float64

    @property
    def nb(self) -> int:
        return self.xyz.shape[0]

    @property
    def max_disp(self) -> float:
        return float(np.sqrt((self.disp * self.disp).sum(axis=1)).max())

    @property
    def tol_abs(self) -> float:
        return self.tol_rel * self.max_disp


def config_small_ellipsoid(nv: int = 50_000, nb: int = 2_000, with_volume: bool = True) -> Problem:
    """Ellipsoid (1, 0.3, 0.1), Nb = 2,000, field (0, 0.05x^2, 0.02 sin(pi x)), R = 2, m = 10, tol 1e-4."""
    s = SEED_SMALL
    xyz = g.ellipsoid_surface(nb, gen=g.rng(s, 1))
    disp = g.ellipsoid_field(xyz)
    vol = g.ellipsoid_volume(nv, gen=g.rng(s, 2)) if with_volume else None
    return Problem("ellipsoid-nb2000", xyz, disp, 2.0, 10, 1e-4, partition_seed(s), nb, vol)


WING_RADIUS = 1.5 * g.WING_ROOT_CHORD


def config_wing(nv: int = 3_000_000, with_volume: bool = True, m: int = 107, n_chord: int = 201,
                n_span: int = 200, seed: int = SEED_WING) -> Problem:
    """Swept tapered wing, Nb = (2*201-2)*200 = 80,000, Nv = 3,000,000, R = 1.5 c_r, tol 1e-5.

    m defaults to the value chosen by the pilot rule m = round(1.5 Nb / Nc0)
    with Nc0 = 1,120 from a pilot run at m0 = 40 (1.5 * 80000 / 1120 = 107;
    the final Nc = 1,135 keeps m inside the paper's recommended range
    [Nb/Nc, 2 Nb/Nc] = [70, 141], Section 4.1).
    """
    xyz = g.wing_surface(n_chord, n_span)
    disp = g.wing_field(xyz)
    vol = g.wing_volume(nv, n_chord, n_span, gen=g.rng(seed, 2)) if with_volume else None
    return Problem(f"wing-nb{xyz.shape[0]}", xyz, disp, WING_RADIUS, m, 1e-5, partition_seed(seed),
                   xyz.shape[0], vol)


def config_wing_large(nv: int = 20_000_000, with_volume: bool = True, m: int = 399) -> Problem:
    """Wing at Nb = (2*301-2)*500 = 300,000, Nv = 20,000,000, R = 1.5 c_r, tol 1e-5.

    m comes from the same pilot rule as the 80,000-node wing: a pilot run at
    m0 = 40 gives Nc0 = 1,129, so m = round(1.5 * 300000 / 1129) = 399; the
    final Nc = 1,176 keeps m inside [Nb/Nc, 2 Nb/Nc] = [255, 510] (Section 4.1).
    """
    return config_wing(nv=nv, with_volume=with_volume, m=m, n_chord=301, n_span=500, seed=SEED_WING_LARGE)


def config_modes(base: Problem, k_modes: int = 64) -> np.ndarray:
    """64 seeded random combinations of bending, twist and sin(k pi y/b) modes: (nb, 3K)."""
    return g.random_modes(base.xyz, k_modes, g.rng(SEED_MODES, 4))


def _surface_sizes(count: int, gen: np.random.Generator) -> np.ndarray:
    return np.rint(np.exp(gen.uniform(math.log(1e3), math.log(5e4), count))).astype(np.int64)


NC_REF = {"ellipsoid": 400, "wing": 2000}


def multi_surface_problem(j: int, nb_target: int, seed: int) -> Problem:
    """One surface of the uneven batch: even j ellipsoid, odd j wing; Nv = 25 Nb."""
    if j % 2 == 0:
        xyz = g.ellipsoid_surface(int(nb_target), gen=g.rng(seed, 1))
        disp = g.ellipsoid_field(xyz)
        radius, kind = 2.0, "ellipsoid"
    else:
        n_span = max(2, int(round(math.sqrt(nb_target / 2.0))))
        n_chord = max(3, int(round(nb_target / (2.0 * n_span))) + 1)
        xyz = g.wing_surface(n_chord, n_span)
        disp = g.wing_field(xyz)
        radius, kind = WING_RADIUS, "wing"
    nb = xyz.shape[0]
    m = int(min(max(round(1.5 * nb / NC_REF[kind]), 1), 80))
    return Problem(f"{kind}-{j}-nb{nb}", xyz, disp, radius, m, 1e-5, partition_seed(seed), nb, None)


def config_multi_surface(count: int = 32, with_volume: bool = True, nv_per_nb: int = 25,
                         size_scale: float = 1.0) -> list[Problem]:
    """32 independent surfaces, Nb log-uniform in [1e3, 5e4], Nv = 25 Nb."""
    gen = g.rng(SEED_MULTI, 1)
    sizes = _surface_sizes(count, gen)
    out = []
    for j, nbt in enumerate(sizes):
        nbt = max(16, int(nbt * size_scale))
        p = multi_surface_problem(j, nbt, SEED_MULTI * 1000 + j)
        if with_volume:
            nv = nv_per_nb * p.nb
            if j % 2 == 0:
                p.volume = g.ellipsoid_volume(nv, gen=g.rng(SEED_MULTI * 1000 + j, 2))
            else:
                p.volume = g.wing_volume(nv, 3, 3, gen=g.rng(SEED_MULTI * 1000 + j, 2))
        out.append(p)
    return out


def config_requests(n_requests: int = 650, rate: float = 20.0, repeat_p: float = 0.2,
                    size_scale: float = 1.0):
    """Poisson arrival stream: list of (arrival_time_s, mesh_key, nb_target, field_seed).

    Sizes follow the uneven-batch distribution; with probability ``repeat_p`` a
    request reuses an earlier mesh (same key) with a fresh field seed.
    """
    gen = g.rng(SEED_REQUESTS, 5)
    t = np.cumsum(gen.exponential(1.0 / rate, n_requests))
    sizes = _surface_sizes(n_requests, gen)
    reqs = []
    keys = []
    for r in range(n_requests):
        if keys and gen.random() < repeat_p:
            key = keys[int(gen.integers(len(keys)))]
            nbt = key[1]
        else:
            key = (len(keys), max(16, int(sizes[r] * size_scale)))
            keys.append(key)
            nbt = key[1]
        reqs.append((float(t[r]), key[0], int(nbt), int(gen.integers(1 << 62))))
    return reqs


def request_mesh(key: int, nb_target: int) -> Problem:
    """The boundary of mesh `key` of a request stream (ellipsoid for even keys, wing for odd)."""
    return multi_surface_problem(key, nb_target, SEED_REQUESTS * 1000 + key)


def request_field(base: Problem, field_seed: int) -> np.ndarray:
    """A new smooth displacement field on a resident mesh: a seeded random mix of
    the base field's components plus a small chordwise tilt."""
    gen = g.rng(field_seed & 0x7FFFFFFF, 5)
    A = np.eye(3) + 0.6 * gen.standard_normal((3, 3))
    d = base.disp @ A.T
    x = base.xyz[:, 0]
    d[:, 2] += 0.02 * base.max_disp * (x - x.min()) / max(float(np.ptp(x)), 1e-12)
    return np.ascontiguousarray(d)


def tiny_problem(nb: int = 12, seed: int = 7, m: int = 3, radius: float = 1.5, tol_rel: float = 0.0,
                 nc_max: int | None = None) -> Problem:
    """Small random point set on a unit sphere with a smooth field (for brute force)."""
    gen = g.rng(seed, 1)
    u = gen.standard_normal((nb, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    disp = np.stack([0.1 * u[:, 0] * u[:, 1], 0.05 * np.sin(2 * u[:, 2]), 0.02 * u[:, 0]], axis=1)
    return Problem(f"tiny-{nb}", np.ascontiguousarray(u), np.ascontiguousarray(disp), radius, m, tol_rel,
                   partition_seed(seed), nb if nc_max is None else nc_max, None)
