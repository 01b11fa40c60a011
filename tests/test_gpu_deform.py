"""GPU parity of the volume deformation (Eq. 6) against the FP64 oracle.

Bar: displacements within 1e-6 * max|d| of the oracle (the stated target);
the FP64 path is in fact checked at 1e-11 * max|d|."""
import numpy as np
import pytest

import oracle
import paper_2004_04817_amd as gcb
import synth
from tests.gpu_util import gpu_select, oracle_select

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def test_small_ellipsoid_volume_all_points():
    p = synth.config_small_ellipsoid()
    ctx, info, S, W, log = gpu_select(p)
    r = oracle_select(p)
    assert list(S) == list(r.S)
    ref = oracle.interpolate(p.xyz[r.S], r.W, p.radius, p.volume)
    out = ctx.deform(p.volume)
    md = p.max_disp
    err = np.abs(out - ref).max()
    print("ellipsoid volume max err / max|d|:", err / md)
    assert err <= 1e-11 * md
    # boundary nodes reproduce their prescribed displacement within E*
    ob = ctx.deform(p.xyz)
    assert np.sqrt(((ob - p.disp) ** 2).sum(1)).max() <= p.tol_abs * (1 + 1e-9)
    ctx.close()


def test_device_tensors_and_dtypes():
    torch = _torch()
    p = synth.config_small_ellipsoid(nv=20011)   # ragged: not a multiple of the block size
    ctx, info, S, W, log = gpu_select(p)
    r = oracle_select(p)
    ref = oracle.interpolate(p.xyz[r.S], r.W, p.radius, p.volume)
    md = p.max_disp
    x64 = torch.from_numpy(p.volume).cuda()
    o64 = ctx.deform(x64)
    torch.cuda.synchronize()
    assert np.abs(o64.cpu().numpy() - ref).max() <= 1e-11 * md
    o32 = ctx.deform(x64, out_dtype=torch.float32)
    torch.cuda.synchronize()
    assert np.abs(o32.cpu().numpy().astype(np.float64) - ref).max() <= 1e-6 * md
    x32 = x64.float()
    ref32 = oracle.interpolate(p.xyz[r.S], r.W, p.radius, x32.cpu().numpy().astype(np.float64))
    o = ctx.deform(x32, out_dtype=torch.float64)
    torch.cuda.synchronize()
    assert np.abs(o.cpu().numpy() - ref32).max() <= 1e-11 * md
    # host numpy path equals the device path bit for bit
    oh = ctx.deform(p.volume)
    assert np.array_equal(oh, o64.cpu().numpy())
    # host path with FP32 input and FP64 output at an odd point count (output buffer after the input)
    oh32 = ctx.deform(x32.cpu().numpy())
    assert oh32.dtype == np.float64 and np.array_equal(oh32, o.cpu().numpy())
    ctx.close()


def test_compact_support_exact_zero_and_empty():
    p = synth.config_small_ellipsoid(with_volume=False)
    ctx, info, S, W, log = gpu_select(p)
    far = np.array([[10.0, 0, 0], [0, 5.0, 0], [-9, -9, -9]])
    out = ctx.deform(far)
    assert np.all(out == 0.0)
    assert ctx.deform(np.zeros((0, 3))).shape == (0, 3)
    ctx.close()


def test_wing_volume_sampled_full_size():
    """3,000,000 graded volume points in the launch the benchmark times;
    20,000 sampled outputs checked one by one against the oracle."""
    torch = _torch()
    p = synth.config_wing()
    ctx, info, S, W, log = gpu_select(p)
    r = oracle_select(p)
    x = torch.from_numpy(p.volume).cuda()
    out = ctx.deform(x)
    torch.cuda.synchronize()
    out = out.cpu().numpy()
    idx = np.random.default_rng(0).choice(p.volume.shape[0], 20000, replace=False)
    md = p.max_disp
    if list(S) == list(r.S):
        ref = oracle.interpolate(p.xyz[r.S], r.W, p.radius, p.volume[idx])
        err = np.abs(out[idx] - ref).max()
        print("wing volume max err / max|d|:", err / md)
        assert err <= 1e-9 * md
    else:
        # the selections legitimately differ after a near tie: both must meet E*
        ref = oracle.interpolate(p.xyz[r.S], r.W, p.radius, p.volume[idx])
        assert np.abs(out[idx] - ref).max() <= 10 * p.tol_abs
    ctx.close()


def test_wing_large_full_size():
    """Precision-scaling case: 300,000-node wing (m = 399, R = 1.5 root chord, E* = 1e-5 max|d|)
    and 20,000,000 volume points: selection against the oracle (identical or certified by
    replay), Eq. (6) on 20,000 sampled points against the oracle's FP64 sum."""
    torch = _torch()
    from tests.test_gpu_select import assert_same_run
    p = synth.config_wing_large()
    ctx, info, S, W, log = gpu_select(p)
    r = oracle_select(p)
    print("wing-large: nc", info["nc"], "iters", info["iterations"], "ms", info["ms_select"], "oracle nc", r.nc,
          flush=True)
    assert info["converged"] and info["final_max_err"] <= p.tol_abs
    assert_same_run(p, info, S, W, log, r, p.tol_abs, p.m)
    x = torch.from_numpy(p.volume).cuda()
    out = ctx.deform(x)
    torch.cuda.synchronize()
    idx = np.random.default_rng(3).choice(p.volume.shape[0], 20000, replace=False)
    o = out[torch.from_numpy(idx).cuda()].cpu().numpy()
    md = p.max_disp
    ref = oracle.interpolate(p.xyz[S], W, p.radius, p.volume[idx])
    err = np.abs(o - ref).max()
    print("wing-large volume max err / max|d| (same supports and weights):", err / md, flush=True)
    assert err <= 1e-9 * md
    if list(S) == list(r.S):
        ref_o = oracle.interpolate(p.xyz[r.S], r.W, p.radius, p.volume[idx])
        assert np.abs(o - ref_o).max() <= 1e-6 * md
    ctx.close()


def test_fp32_evaluation_accuracy_and_dtypes():
    """GCB_PREC_FP32_EVAL: Eq. (6) in FP32 with FP64 chunk sums.  Its error is that
    of phi and the coordinates in FP32, amplified by the weights of the
    ill-conditioned support system (sum condition about 195 here): measured at
    1.2e-5 max|d| against the oracle's own selection and weights, bounded here
    by 5e-5 max|d| (max) and 1e-5 max|d| (RMS), so that a regression shows; the
    FP64 path meets 1e-11.  FP32 in / FP64 out does not change it."""
    torch = _torch()
    p = synth.config_small_ellipsoid(nv=20000)
    c = gcb.Context(0)
    c.set_boundary(p.xyz, p.disp)
    c.set_params(p.radius, p.m, p.tol_abs, seed=p.seed)
    c.select()
    S, W = c.get_support()
    r = oracle.select(p.xyz, p.disp, p.radius, p.m, p.tol_abs, seed=p.seed)
    assert np.array_equal(S, r.S)
    ref = oracle.interpolate(p.xyz[r.S], r.W, p.radius, p.volume)
    x = torch.from_numpy(p.volume).cuda()
    o64 = c.deform(x).cpu().numpy()
    c.set_params(p.radius, p.m, p.tol_abs, seed=p.seed, precision=gcb.GCB_PREC_FP32_EVAL)
    c.select()
    o32 = c.deform(x).cpu().numpy()
    o32f = c.deform(x.float(), out_dtype=torch.float32).cpu().numpy().astype(np.float64)
    md = p.max_disp
    e64 = np.abs(o64 - ref).max() / md
    e32 = np.abs(o32 - ref).max() / md
    r32 = float(np.sqrt(((o32 - ref) ** 2).sum(axis=1).mean())) / md
    print("FP64 eval err / max|d|:", e64, " FP32 eval err / max|d|: max", e32, "RMS", r32, flush=True)
    assert e64 <= 1e-11
    assert e32 <= 5e-5 and r32 <= 1e-5
    assert np.abs(o32f - ref).max() / md <= 5e-5
    # support nodes: the FP32 interpolant still reproduces the field to FP32 accuracy
    o_s = c.deform(np.ascontiguousarray(p.xyz[S]))
    assert np.abs(o_s - p.disp[S]).max() / md <= 5e-5
    c.close()


def test_volume_far_points_and_translation():
    """Eq. 6 is exactly zero beyond the radius of every support, and the volume
    sweep's centred distances keep the parity bar when the whole problem sits
    far from the origin (the centring removes the offset before any square)."""
    import dataclasses
    p = synth.config_small_ellipsoid(nv=5003)
    ctx, info, S, W, log = gpu_select(p)
    md = p.max_disp
    far = p.volume + np.array([10.0, 0.0, 0.0]) * p.radius + 3.0
    assert np.all(ctx.deform(far) == 0.0)
    ctx.close()
    off = np.array([1.0e3, -2.0e3, 5.0e2]) * p.radius
    q = dataclasses.replace(p, xyz=p.xyz + off, volume=p.volume + off)
    ctx, info, S, W, log = gpu_select(q)
    ref = oracle.interpolate(q.xyz[S], W, q.radius, q.volume)
    err = np.abs(ctx.deform(q.volume) - ref).max()
    print("translated volume max err / max|d|:", err / md)
    assert err <= 1e-11 * md
    # the supports themselves: the interpolation condition of Eq. 3
    osup = ctx.deform(q.xyz[S])
    assert np.abs(osup - q.disp[S]).max() <= 1e-9 * md
    ctx.close()


def test_deform_time_reports_the_kernels():
    p = synth.config_small_ellipsoid(nv=20000)
    ctx, info, S, W, log = gpu_select(p)
    with pytest.raises(gcb.GcbError) as e:
        ctx.deform_time()              # nothing timed yet
    assert e.value.code == gcb.GCB_E_STATE
    ctx.deform(p.volume)
    ms = ctx.deform_time()
    assert 0.0 < ms < 1000.0
    ctx.close()
