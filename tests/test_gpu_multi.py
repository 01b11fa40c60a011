"""Several right-hand sides on one support set (deformation modes): GPU
weights W = M^T (M D_S) and the FP64-MFMA volume sweep against the oracle,
which re-factors the same support set with its RC scheme and evaluates Eq. 6."""
import numpy as np
import pytest

import oracle
import synth
from synth import geometry as g
from tests.gpu_util import gpu_select, oracle_select

pytestmark = pytest.mark.gpu


def _modes(xyz, k, seed):
    return g.random_modes(xyz, k, g.rng(seed, 4))


@pytest.mark.parametrize("k_modes,nv", [(1, 1000), (5, 4099), (64, 20000)])
def test_modes_small_ellipsoid(k_modes, nv):
    p = synth.config_small_ellipsoid(nv=nv)
    ctx, info, S, W, log = gpu_select(p)
    r = oracle_select(p)
    assert list(S) == list(r.S)
    D = _modes(p.xyz, k_modes, 100 + k_modes)
    out = ctx.deform_multi(D, p.volume)
    Wo = oracle.solve_on_support(p.xyz, r.S, p.radius, D)
    ref = oracle.interpolate(p.xyz[r.S], Wo, p.radius, p.volume)
    scale = np.abs(D).max()
    err = np.abs(out - ref).max()
    print(f"K={k_modes} nv={nv}: max err / max|D| = {err / scale:.2e}")
    assert err <= 1e-9 * scale
    ctx.close()


def test_mode_equal_to_the_selection_field():
    """Linearity: a mode equal to the field the selection used reproduces gcb_deform."""
    p = synth.config_small_ellipsoid(nv=3000)
    ctx, info, S, W, log = gpu_select(p)
    D = np.concatenate([p.disp, 2.0 * p.disp, _modes(p.xyz, 1, 7)], axis=1)
    out = ctx.deform_multi(D, p.volume)
    single = ctx.deform(p.volume)
    md = p.max_disp
    assert np.abs(out[:, :3] - single).max() <= 1e-11 * md
    assert np.abs(out[:, 3:6] - 2.0 * single).max() <= 2e-11 * md
    ctx.close()


def test_wing_64_modes_full_launch():
    """The wing support set with 64 seeded modes (192 right-hand sides) over
    all 3,000,000 volume points in one launch; 2,000 sampled outputs checked."""
    import torch
    p = synth.config_wing()
    ctx, info, S, W, log = gpu_select(p)
    r = oracle_select(p)
    D = synth.config_modes(p)
    dev = torch.device("cuda:0")
    out = ctx.deform_multi(torch.from_numpy(D).to(dev), torch.from_numpy(p.volume).to(dev))
    torch.cuda.synchronize()
    idx = np.random.default_rng(1).choice(p.volume.shape[0], 2000, replace=False)
    got = out[torch.from_numpy(idx).to(dev)].cpu().numpy()
    assert list(S) == list(r.S)
    Wo = oracle.solve_on_support(p.xyz, r.S, p.radius, D)
    ref = oracle.interpolate(p.xyz[r.S], Wo, p.radius, p.volume[idx])
    scale = np.abs(D).max()
    err = np.abs(got - ref).max()
    print(f"wing 64 modes: max err / max|D| = {err / scale:.2e}")
    assert err <= 1e-9 * scale
    del out
    ctx.close()
