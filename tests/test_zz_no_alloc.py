"""The allocation-free deformation entry point (gcb_deform_noalloc) against gcb_deform.

Both run the same kernels on the same support set, so the bar is bitwise
equality with gcb_deform (device buffers), on two calls in a row, the second
with a smaller support set and a smaller, ragged point count (stale table
entries of the first call must not be read); the first call is also held to
the FP64 oracle at 1e-11 max|d|.  A selection with more supports than the
static table holds is rejected, and the context stays usable."""
import numpy as np
import pytest

import oracle
import paper_2004_04817_amd as gcb
import synth
from tests.gpu_util import gpu_select, oracle_select

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _pair(ctx, x, out_dtype):
    """(gcb_deform result, gcb_deform_noalloc result) for device points x."""
    import torch
    ref = ctx.deform(x, out_dtype=out_dtype)
    out = torch.full(x.shape, float("nan"), dtype=out_dtype, device=x.device)
    got = ctx.deform_noalloc(x, out)
    torch.cuda.synchronize()
    return ref, got


def test_noalloc_equals_deform_two_calls():
    import torch
    # first call: the ellipsoid's 282 supports, 50,000 points
    p = synth.config_small_ellipsoid()
    ctx, info, S, W, _ = gpu_select(p)
    assert info["nc"] > 200
    x = _dev(p.volume)
    ref, got = _pair(ctx, x, torch.float64)
    assert torch.equal(ref, got)
    r = oracle_select(p)
    assert list(S) == list(r.S)
    want = oracle.interpolate(p.xyz[r.S], r.W, p.radius, p.volume)
    assert np.abs(got.cpu().numpy() - want).max() <= 1e-11 * p.max_disp
    # FP32 points and FP32 output through the same table
    ref, got = _pair(ctx, x.float(), torch.float32)
    assert torch.equal(ref, got)

    # second call, smaller: 58 supports of a 300-node sphere, 1,001 points (ragged)
    q = synth.tiny_problem(nb=300, seed=11, m=4, radius=1.5, tol_rel=3e-2)
    ctx2, info2, S2, W2, _ = gpu_select(q)
    assert 3 <= info2["nc"] < info["nc"]
    pts = synth.geometry.rng(11, 2).uniform(-1.2, 1.2, size=(1001, 3))
    x2 = _dev(pts)
    ref2, got2 = _pair(ctx2, x2, torch.float64)
    assert torch.equal(ref2, got2)
    w2 = oracle.solve_on_support(q.xyz, S2, q.radius, q.disp)   # the oracle's weights on this support set
    want2 = oracle.interpolate(q.xyz[S2], w2, q.radius, pts)
    assert np.abs(got2.cpu().numpy() - want2).max() <= 1e-11 * q.max_disp
    # and the first context again, after the second one overwrote part of the table
    ref, got = _pair(ctx, x[:777], torch.float64)
    assert torch.equal(ref, got)
    ctx2.close()
    ctx.close()


def test_noalloc_fp32_evaluation_equals_deform():
    import torch
    p = synth.config_small_ellipsoid(nv=30_001)
    ctx, info, S, W, _ = gpu_select(p, precision=gcb.GCB_PREC_FP32_EVAL)
    x = _dev(p.volume)
    for n in (30_001, 4_097):
        ref, got = _pair(ctx, x[:n], torch.float64)
        assert torch.equal(ref, got)
    ctx.close()


def test_noalloc_errors_and_the_support_limit():
    import torch
    ctx = gcb.Context(0)
    x = torch.zeros((5, 3), dtype=torch.float64, device="cuda")
    out = torch.zeros_like(x)
    with pytest.raises(gcb.GcbError) as e:   # no selection yet
        ctx.deform_noalloc(x, out)
    assert e.value.code == gcb.GCB_E_STATE
    ctx.close()

    # 8,193 supports: sparse random points with a small radius keep Phi_S well conditioned
    nb = gcb.GCB_NOALLOC_MAX_SUPPORTS + 400
    gen = synth.geometry.rng(23, 1)
    xyz = gen.uniform(0.0, 1.0, size=(nb, 3))
    disp = gen.uniform(0.5, 1.0, size=(nb, 3))
    ctx = gcb.Context(0)
    ctx.set_boundary(xyz, disp)
    ctx.set_params(0.02, 4, 0.0, nc_max=gcb.GCB_NOALLOC_MAX_SUPPORTS + 1, seed=5)
    info = ctx.select()
    assert info["nc"] == gcb.GCB_NOALLOC_MAX_SUPPORTS + 1
    x = _dev(xyz[:100])
    out = torch.zeros_like(x)
    with pytest.raises(gcb.GcbError) as e:
        ctx.deform_noalloc(x, out)
    assert e.value.code == gcb.GCB_E_INVALID
    assert "allocation-free maximum" in str(e.value)
    # gcb_deform has no such limit: the supports reproduce their displacements
    sel, _ = ctx.get_support()
    got = ctx.deform(_dev(xyz[sel[:100]]))
    torch.cuda.synchronize()
    assert np.abs(got.cpu().numpy() - disp[sel[:100]]).max() <= 1e-9
    # an empty call is a no-op
    e0 = torch.zeros((0, 3), dtype=torch.float64, device="cuda")
    assert ctx.deform_noalloc(e0, torch.zeros_like(e0)).shape == (0, 3)
    ctx.close()
