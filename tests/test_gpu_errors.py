"""Error paths of the C ABI on the GPU (all forced from the host)."""
import numpy as np
import pytest

import paper_2004_04817_amd as gcb
import synth
from tests.gpu_util import gpu_select, oracle_select

pytestmark = pytest.mark.gpu


def test_state_and_argument_errors():
    p = synth.tiny_problem(nb=20)
    ctx = gcb.Context(0)
    with pytest.raises(gcb.GcbError) as e:
        ctx.select()
    assert e.value.code == gcb.GCB_E_STATE
    ctx.set_boundary(p.xyz, p.disp)
    with pytest.raises(gcb.GcbError) as e:
        ctx.deform(p.xyz)
    assert e.value.code == gcb.GCB_E_STATE
    for kw in (dict(radius=-1.0, m=2, tol_abs=0.0), dict(radius=1.0, m=0, tol_abs=0.0),
               dict(radius=1.0, m=21, tol_abs=0.0), dict(radius=1.0, m=2, tol_abs=-1.0),
               dict(radius=1.0, m=2, tol_abs=0.0, nc_max=2), dict(radius=1.0, m=2, tol_abs=0.0, init_idx=[1, 1, 2])):
        ctx.set_params(**kw)
        with pytest.raises(gcb.GcbError) as e:
            ctx.select()
        assert e.value.code == gcb.GCB_E_INVALID, kw
    bad = p.xyz.copy()
    bad[4, 2] = np.inf
    with pytest.raises(gcb.GcbError) as e:
        ctx.set_boundary(bad, p.disp)
    assert e.value.code == gcb.GCB_E_INVALID
    ctx.close()


def test_device_nan_rejected():
    import torch
    p = synth.tiny_problem(nb=20)
    x = torch.from_numpy(p.xyz).cuda()
    d = torch.from_numpy(p.disp).cuda()
    d[3, 1] = float("nan")
    ctx = gcb.Context(0)
    with pytest.raises(gcb.GcbError) as e:
        ctx.set_boundary(x, d)
    assert e.value.code == gcb.GCB_E_INVALID
    ctx.close()


def test_duplicate_node_is_singular():
    """Phi_S is SPD only for distinct nodes (Section 2): a duplicate forced into
    the starting set gives GCB_E_SINGULAR, as in the oracle."""
    p = synth.tiny_problem(nb=20)
    xyz = p.xyz.copy()
    xyz[7] = xyz[3]
    p.xyz = xyz
    ctx = gcb.Context(0)
    ctx.set_boundary(p.xyz, p.disp)
    ctx.set_params(p.radius, 2, 0.0, init_idx=[3, 7, 9])
    with pytest.raises(gcb.GcbError) as e:
        ctx.select()
    assert e.value.code == gcb.GCB_E_SINGULAR
    r = oracle_select(p, tol_abs=0.0, m=2, init_idx=[3, 7, 9])
    assert r.status == -4
    ctx.close()


def test_device_boundary_input_equals_host_input():
    import torch
    p = synth.config_small_ellipsoid(with_volume=False)
    ctx, info, S, W, log = gpu_select(p)
    c2 = gcb.Context(0)
    c2.set_boundary(torch.from_numpy(p.xyz).cuda(), torch.from_numpy(p.disp).cuda())
    c2.set_params(p.radius, p.m, p.tol_abs, seed=p.seed)
    info2 = c2.select()
    S2, W2 = c2.get_support()
    assert np.array_equal(S, S2) and np.array_equal(W, W2)
    ctx.close()
    c2.close()


def test_run_to_run_bitwise_determinism():
    p = synth.config_small_ellipsoid(with_volume=False)
    a = gpu_select(p)
    b = gpu_select(p)
    assert np.array_equal(a[2], b[2]) and np.array_equal(a[3], b[3])
    assert np.array_equal(a[4].err, b[4].err)
    a[0].close()
    b[0].close()


def test_contexts_return_their_device_memory():
    """Creating, using (selection, FP64 and FP32 deformation, refactorisation) and destroying
    contexts leaves the device's free memory where it was: nothing a context allocates outlives it."""
    import torch
    p = synth.config_small_ellipsoid(nv=20000)
    vol = torch.from_numpy(p.volume).cuda()
    torch.cuda.synchronize()

    def cycle():
        c = gcb.Context(0)
        c.set_boundary(p.xyz, p.disp)
        c.set_params(p.radius, p.m, p.tol_abs, seed=p.seed, monitor_every=p.m)
        c.select()
        c.deform(vol)
        c.set_params(p.radius, p.m, p.tol_abs, seed=p.seed, precision=gcb.GCB_PREC_FP32_EVAL)
        c.select()
        c.deform(vol)
        c.refactor()
        torch.cuda.synchronize()
        c.close()

    cycle()   # first use: runtime and module set-up
    free0 = torch.cuda.mem_get_info()[0]
    for _ in range(12):
        cycle()
    free1 = torch.cuda.mem_get_info()[0]
    print("free device bytes before / after 12 context cycles:", free0, free1)
    assert free0 - free1 < (4 << 20)
