"""Geometry and field generators (inputs only; no method arithmetic).

Coordinates are float64 arrays of shape (n, 3), row-major (x, y, z).
Wing convention: y is spanwise (root at y = 0, tip at y = b), z is vertical.
"""
from __future__ import annotations

import math

import numpy as np

WING_HALF_SPAN = 1.2        # b
WING_ROOT_CHORD = 0.805     # c_r (the root chord of the ONERA M6 class)
WING_TAPER = 0.56           # tip chord / root chord
WING_SWEEP_DEG = 30.0       # leading-edge sweep
WING_THICKNESS = 0.10       # symmetric four-digit section, t/c


def rng(base: int, stream: int) -> np.random.Generator:
    """Independent generator for (workload seed, stream id)."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(base), int(stream)])))


# --------------------------------------------------------------------- ellipsoid
def ellipsoid_surface(n: int, axes=(1.0, 0.3, 0.1), gen: np.random.Generator | None = None) -> np.ndarray:
    """Area-uniform samples on an ellipsoid surface.

    A point u uniform on the unit sphere maps to p = (a u1, b u2, c u3); it is
    accepted with probability min(a,b,c)*sqrt((u1/a)^2+(u2/b)^2+(u3/c)^2), the
    ratio of the surface element of the ellipsoid to its largest value.
    """
    a, b, c = axes
    gen = gen if gen is not None else rng(0, 1)
    out = np.empty((0, 3))
    lo = min(axes)
    while out.shape[0] < n:
        k = max(2 * (n - out.shape[0]), 1024)
        u = gen.standard_normal((k, 3))
        u /= np.linalg.norm(u, axis=1, keepdims=True)
        p = u * np.array([a, b, c])
        acc = lo * np.sqrt((u[:, 0] / a) ** 2 + (u[:, 1] / b) ** 2 + (u[:, 2] / c) ** 2)
        keep = gen.random(k) < acc
        out = np.concatenate([out, p[keep]], axis=0)
    return np.ascontiguousarray(out[:n])


def ellipsoid_field(xyz: np.ndarray) -> np.ndarray:
    """Smooth analytic displacement d = (0, 0.05 x^2, 0.02 sin(pi x))."""
    x = xyz[:, 0]
    d = np.zeros_like(xyz)
    d[:, 1] = 0.05 * x * x
    d[:, 2] = 0.02 * np.sin(np.pi * x)
    return d


def ellipsoid_volume(n: int, axes=(1.0, 0.3, 0.1), box=((-2, 2), (-1, 1), (-1, 1)),
                     gen: np.random.Generator | None = None) -> np.ndarray:
    """Uniform points in a box, rejecting the ellipsoid interior."""
    gen = gen if gen is not None else rng(0, 2)
    a, b, c = axes
    lo = np.array([bx[0] for bx in box], dtype=np.float64)
    hi = np.array([bx[1] for bx in box], dtype=np.float64)
    out = []
    got = 0
    while got < n:
        k = max(int(1.2 * (n - got)) + 64, 1024)
        p = lo + (hi - lo) * gen.random((k, 3))
        inside = (p[:, 0] / a) ** 2 + (p[:, 1] / b) ** 2 + (p[:, 2] / c) ** 2 < 1.0
        p = p[~inside]
        out.append(p)
        got += p.shape[0]
    return np.ascontiguousarray(np.concatenate(out, axis=0)[:n])


# --------------------------------------------------------------------- wing
def _thickness(xi: np.ndarray, chord: np.ndarray) -> np.ndarray:
    """Half-thickness of the symmetric four-digit section, closed trailing edge."""
    t = WING_THICKNESS
    return 5.0 * t * chord * (0.2969 * np.sqrt(xi) - 0.1260 * xi - 0.3516 * xi ** 2
                              + 0.2843 * xi ** 3 - 0.1036 * xi ** 4)


def _thickness_slope(xi: np.ndarray) -> np.ndarray:
    """d(half-thickness / chord)/d(xi); finite at xi > 0."""
    t = WING_THICKNESS
    xi = np.maximum(xi, 1e-12)
    return 5.0 * t * (0.5 * 0.2969 / np.sqrt(xi) - 0.1260 - 2 * 0.3516 * xi
                      + 3 * 0.2843 * xi ** 2 - 4 * 0.1036 * xi ** 3)


def _chord(y: np.ndarray) -> np.ndarray:
    b = WING_HALF_SPAN
    return WING_ROOT_CHORD * (1.0 - (1.0 - WING_TAPER) * y / b)


def _x_le(y: np.ndarray) -> np.ndarray:
    return y * math.tan(math.radians(WING_SWEEP_DEG))


def wing_surface(n_chord: int, n_span: int) -> np.ndarray:
    """Structured swept, tapered wing surface.

    Chordwise cosine spacing xi_i = (1 - cos(pi i/(n_chord-1)))/2, spanwise
    uniform y_j = b j/(n_span-1).  The upper surface uses all n_chord stations,
    the lower surface the n_chord-2 interior ones (no duplicate leading or
    trailing edge points), so Nb = (2 n_chord - 2) n_span.
    """
    b = WING_HALF_SPAN
    i = np.arange(n_chord, dtype=np.float64)
    xi = 0.5 * (1.0 - np.cos(np.pi * i / (n_chord - 1)))
    y = b * np.arange(n_span, dtype=np.float64) / (n_span - 1)
    pts = []
    for j in range(n_span):
        c = _chord(np.array([y[j]]))[0]
        xle = _x_le(np.array([y[j]]))[0]
        zt = _thickness(xi, np.full_like(xi, c))
        up = np.stack([xle + xi * c, np.full_like(xi, y[j]), zt], axis=1)
        lo = np.stack([xle + xi[1:-1] * c, np.full(n_chord - 2, y[j]), -zt[1:-1]], axis=1)
        pts.append(up)
        pts.append(lo)
    return np.ascontiguousarray(np.concatenate(pts, axis=0))


def wing_twist_field(xyz: np.ndarray, tip_deg: float = 5.0) -> np.ndarray:
    """Linear twist theta(y) = tip_deg * y/b, nose up, about the local quarter chord."""
    b = WING_HALF_SPAN
    y = xyz[:, 1]
    th = np.radians(tip_deg) * y / b
    qx = _x_le(y) + 0.25 * _chord(y)
    dx = xyz[:, 0] - qx
    dz = xyz[:, 2]
    c, s = np.cos(th), np.sin(th)
    d = np.zeros_like(xyz)
    d[:, 0] = dx * (c - 1.0) + dz * s
    d[:, 2] = -dx * s + dz * (c - 1.0)
    return d


def wing_field(xyz: np.ndarray) -> np.ndarray:
    """Bending d_z = 0.1 (y/b)^2 plus a linear twist up to 5 degrees."""
    b = WING_HALF_SPAN
    d = wing_twist_field(xyz)
    d[:, 2] += 0.1 * (xyz[:, 1] / b) ** 2
    return d


def _inside_wing(p: np.ndarray) -> np.ndarray:
    b = WING_HALF_SPAN
    y = p[:, 1]
    ok = (y >= 0.0) & (y <= b)
    yc = np.clip(y, 0.0, b)
    c = _chord(yc)
    xi = (p[:, 0] - _x_le(yc)) / c
    ok &= (xi >= 0.0) & (xi <= 1.0)
    zt = _thickness(np.clip(xi, 0.0, 1.0), c)
    return ok & (np.abs(p[:, 2]) < zt)


def wing_volume(n: int, surface_n_chord: int, surface_n_span: int,
                gen: np.random.Generator | None = None,
                frac_graded: float = 0.9) -> np.ndarray:
    """Volume cloud graded toward the wing surface.

    A fraction ``frac_graded`` of the points are offsets along the outward
    normal of a uniformly chosen point of the parametric surface, at distance
    h = h0 (H/h0)^U with h0 = 1e-5 c_r, H = 3 c_r (log-uniform, so dense near
    the wall); the rest are uniform in [-1.5,3.5]x[0,2.5]x[-2,2] outside the wing.
    """
    gen = gen if gen is not None else rng(0, 2)
    b = WING_HALF_SPAN
    ng = int(round(frac_graded * n))
    nu = n - ng
    # graded part: continuous parametric surface points (not only the nodes)
    xi = 0.5 * (1.0 - np.cos(np.pi * gen.random(ng)))
    y = b * gen.random(ng)
    upper = gen.random(ng) < 0.5
    c = _chord(y)
    zt = _thickness(xi, c)
    sgn = np.where(upper, 1.0, -1.0)
    px = _x_le(y) + xi * c
    pz = sgn * zt
    slope = _thickness_slope(np.maximum(xi, 1e-6))
    # outward normal of z = +-c T(xi) in the x-z plane: (-T'(xi), 0, +-1)
    nx = -slope
    nz = sgn.copy()
    nrm = np.sqrt(nx * nx + nz * nz)
    nx /= nrm
    nz /= nrm
    h0 = 1e-5 * WING_ROOT_CHORD
    H = 3.0 * WING_ROOT_CHORD
    h = h0 * (H / h0) ** gen.random(ng)
    graded = np.stack([px + h * nx, y, pz + h * nz], axis=1)
    # uniform far field
    lo = np.array([-1.5, 0.0, -2.0])
    hi = np.array([3.5, 2.5, 2.0])
    far = []
    got = 0
    while got < nu:
        k = max(int(1.2 * (nu - got)) + 64, 1024)
        p = lo + (hi - lo) * gen.random((k, 3))
        p = p[~_inside_wing(p)]
        far.append(p)
        got += p.shape[0]
    far = np.concatenate(far, axis=0)[:nu] if nu > 0 else np.zeros((0, 3))
    out = np.concatenate([graded, far], axis=0)
    return np.ascontiguousarray(out[gen.permutation(n)])


def wing_mode_basis(xyz: np.ndarray) -> list[np.ndarray]:
    """Ten basis fields: bending (y/b)^2, the 5-degree twist, sin(k pi y/b), k=1..8 (z)."""
    b = WING_HALF_SPAN
    y = xyz[:, 1]
    out = []
    d = np.zeros_like(xyz)
    d[:, 2] = (y / b) ** 2
    out.append(d)
    out.append(wing_twist_field(xyz))
    for k in range(1, 9):
        d = np.zeros_like(xyz)
        d[:, 2] = np.sin(k * np.pi * y / b)
        out.append(d)
    return out


def random_modes(xyz: np.ndarray, k_modes: int, gen: np.random.Generator, peak: float = 0.1) -> np.ndarray:
    """k_modes random combinations of the basis, each scaled so max_j |D_q(j)| = peak.

    Returns an array of shape (nb, 3 * k_modes): columns (x, y, z) of mode 0,
    then mode 1, and so on.
    """
    basis = wing_mode_basis(xyz)
    a = gen.standard_normal((k_modes, len(basis)))
    out = np.empty((xyz.shape[0], 3 * k_modes))
    for q in range(k_modes):
        d = sum(a[q, t] * basis[t] for t in range(len(basis)))
        mx = np.sqrt((d * d).sum(axis=1)).max()
        out[:, 3 * q:3 * q + 3] = d * (peak / mx)
    return out
