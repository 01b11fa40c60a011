"""Compact-support culling of Eq. (6) (params.cull_volume): phi is exactly zero
beyond R (Eq. 2), so the culled sweep sums the same non-zero terms as the plain
sweep, in another order (supports in Morton order, in tiles).

Bar: within 1e-12 max|d| of the plain FP64 sweep and within 1e-11 max|d| of
the oracle (the plain sweep's own bar); points beyond R of every support give
exactly 0; the evaluated pair count lies between the pairs within R (brute
force) and the dense count nv x nc."""
import numpy as np
import pytest

import oracle
import paper_2004_04817_amd as gcb
import synth
from tests.gpu_util import oracle_select

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def _select(p, cull):
    ctx = gcb.Context(0)
    ctx.set_boundary(p.xyz, p.disp)
    ctx.set_params(p.radius, p.m, p.tol_abs, seed=p.seed, cull_volume=cull)
    info = ctx.select()
    return ctx, info


def test_cull_small_ellipsoid_all_points():
    torch = _torch()
    p = synth.config_small_ellipsoid()
    ctx, info = _select(p, True)
    plain, _ = _select(p, False)
    x = torch.from_numpy(p.volume).cuda()
    got = ctx.deform(x).cpu().numpy()
    ref = plain.deform(x).cpu().numpy()
    md = p.max_disp
    assert np.abs(got - ref).max() <= 1e-12 * md
    S, W = ctx.get_support()
    r = oracle_select(p)
    assert list(S) == list(r.S)
    want = oracle.interpolate(p.xyz[r.S], r.W, p.radius, p.volume)
    assert np.abs(got - want).max() <= 1e-11 * md
    ev, dense = ctx.deform_pairs()
    assert dense == p.volume.shape[0] * info["nc"]
    # at least every pair within R, at most all of them
    sub = p.volume[::25]
    d = np.sqrt(((sub[:, None, :] - p.xyz[S][None]) ** 2).sum(-1))
    within = (d < p.radius).mean()
    print(f"ellipsoid: evaluated {ev / dense:.3f} of the dense pairs; {within:.3f} lie within R", flush=True)
    assert ev <= dense and ev >= 0.98 * within * dense
    ctx.close()
    plain.close()


def test_cull_far_points_are_exactly_zero_and_skipped():
    torch = _torch()
    p = synth.config_small_ellipsoid(nv=10_007)
    ctx, info = _select(p, True)
    far = p.volume + np.array([10.0, 0.0, 0.0]) * p.radius
    out = ctx.deform(torch.from_numpy(far).cuda()).cpu().numpy()
    assert np.all(out == 0.0)
    ev, dense = ctx.deform_pairs()
    assert ev == 0 and dense == far.shape[0] * info["nc"]
    # a point just beyond R of the only nearby support, and one just inside
    S, W = ctx.get_support()
    s0 = p.xyz[S[0]]
    dirn = np.array([0.0, 0.0, 1.0])
    pts = np.stack([s0 + dirn * p.radius * (1 + 1e-6), s0 + dirn * p.radius * (1 - 1e-3)])
    got = ctx.deform(pts)
    plain, _ = _select(p, False)
    ref = plain.deform(pts)
    assert np.abs(got - ref).max() <= 1e-12 * p.max_disp
    ctx.close()
    plain.close()


@pytest.mark.parametrize("in_dt,out_dt", [("f64", "f32"), ("f32", "f64"), ("f32", "f32")])
def test_cull_dtypes_and_ragged_count(in_dt, out_dt):
    torch = _torch()
    p = synth.config_small_ellipsoid(nv=20_011)
    ctx, info = _select(p, True)
    plain, _ = _select(p, False)
    tin = torch.float64 if in_dt == "f64" else torch.float32
    tout = torch.float64 if out_dt == "f64" else torch.float32
    x = torch.from_numpy(p.volume).cuda().to(tin)
    got = ctx.deform(x, out_dtype=tout).double().cpu().numpy()
    ref = plain.deform(x, out_dtype=tout).double().cpu().numpy()
    tol = 1e-12 if out_dt == "f64" else 1e-6
    assert np.abs(got - ref).max() <= tol * p.max_disp
    ctx.close()
    plain.close()


def test_cull_wing_full_size():
    """The 80,000-node wing's 3,000,000 points: culled against plain at every point, against the oracle on
    20,000 sampled points; the share of pairs evaluated."""
    torch = _torch()
    p = synth.config_wing()
    ctx, info = _select(p, True)
    x = torch.from_numpy(p.volume).cuda()
    got = ctx.deform(x)
    ev, dense = ctx.deform_pairs()
    ctx.set_params(p.radius, p.m, p.tol_abs, seed=p.seed, cull_volume=False)
    ctx.select()
    ref = ctx.deform(x)
    md = p.max_disp
    assert float((got - ref).abs().max()) <= 1e-12 * md
    S, W = ctx.get_support()
    idx = np.random.default_rng(5).choice(p.volume.shape[0], 20_000, replace=False)
    want = oracle.interpolate(p.xyz[S], W, p.radius, p.volume[idx])
    assert np.abs(got.cpu().numpy()[idx] - want).max() <= 1e-9 * md
    print(f"wing: evaluated {ev / dense:.3f} of {dense} pairs", flush=True)
    assert ev < dense
    ctx.close()


def test_cull_needs_a_culled_deformation():
    p = synth.config_small_ellipsoid(nv=100)
    ctx, info = _select(p, False)
    ctx.deform(p.volume)
    with pytest.raises(gcb.GcbError) as e:
        ctx.deform_pairs()
    assert e.value.code == gcb.GCB_E_STATE
    ctx.close()
