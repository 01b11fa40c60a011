"""GPU warm start (kept support set, new displacement field) against the FP64 oracle.

The oracle starts from the same kept set (the GPU's own selection), rebuilds
its factor by the RC recurrence, certifies, and resumes Algorithm 1 at
k = |S0|; the GPU recomputes W = M^T (M Delta_S0) from the kept inverse
factor.  Bar as for a fresh selection: the index sequence is identical
unless a near tie (TAU_FP64 * max|d|) is certified by the follow-mode replay.
"""
import numpy as np
import pytest

import oracle
import synth
import paper_2004_04817_amd as gcb
from tests.gpu_util import first_divergence

pytestmark = pytest.mark.gpu

TAU_FP64 = 1e-9


def new_field(p, seed):
    """A different smooth field on the same boundary: rotated components, scaled, plus a tilt."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((3, 3)) * 0.6 + np.eye(3)
    d = p.disp @ A.T
    d[:, 2] += 0.02 * p.max_disp * p.xyz[:, 0] / np.abs(p.xyz[:, 0]).max()
    return np.ascontiguousarray(d)


def fresh(p):
    c = gcb.Context(0)
    c.set_boundary(p.xyz, p.disp)
    c.set_params(p.radius, p.m, p.tol_abs, seed=p.seed)
    info = c.select()
    S, W = c.get_support()
    return c, info, S, W


def warm(c, p, disp2, tol_abs):
    c.set_displacement(disp2)
    c.set_params(p.radius, p.m, tol_abs, seed=p.seed, warm_start=True)
    info = c.select()
    S, W = c.get_support()
    return info, S, W, c.get_log()


def check_against_oracle(p, disp2, tol, S0, info, S, W, log):
    r = oracle.select(p.xyz, disp2, p.radius, p.m, tol, seed=p.seed, warm_S=S0)
    md = float(np.sqrt((disp2 ** 2).sum(axis=1)).max())
    assert np.array_equal(S[: len(S0)], S0)
    if first_divergence(S, r.S) == -1:
        assert info["iterations"] == r.iterations
        assert np.array_equal(log.node, r.log_node) and np.array_equal(log.group, r.log_group)
        assert np.abs(log.err - r.log_err).max(initial=0.0) <= 1e-10 * md
        assert np.abs(W - r.W).max() <= 1e-7 * max(1.0, np.abs(r.W).max())
    else:
        bad, reason, _ = oracle.validate(p.xyz, disp2, p.radius, p.m, tol, S0, log.group, log.node, log.appended,
                                         TAU_FP64 * md, seed=p.seed, warm_S=S0)
        assert bad == -1, f"warm run fails replay at {bad} (reason {reason})"
    assert info["final_max_err"] == pytest.approx(r.final_max_err, rel=1e-6, abs=1e-12 * md)
    return r


def test_warm_same_field_needs_no_iteration():
    p = synth.config_small_ellipsoid(with_volume=False)
    c, info0, S0, W0 = fresh(p)
    info, S, W, log = warm(c, p, p.disp, p.tol_abs)
    assert info["iterations"] == 0 and info["converged"] and info["nc"] == info0["nc"]
    assert np.array_equal(S, S0)
    # recomputed from the inverse factor: equal to the incremental weights up to rounding
    assert np.abs(W - W0).max() <= 1e-8 * max(1.0, np.abs(W0).max())
    c.close()


@pytest.mark.parametrize("seed", [0, 1])
def test_warm_new_field_small_ellipsoid(seed):
    p = synth.config_small_ellipsoid(with_volume=False)
    c, info0, S0, _ = fresh(p)
    d2 = new_field(p, seed)
    tol = 1e-4 * float(np.sqrt((d2 ** 2).sum(axis=1)).max())
    info, S, W, log = warm(c, p, d2, tol)
    assert info["iterations"] > 0
    check_against_oracle(p, d2, tol, S0, info, S, W, log)
    # a second warm start chains from the grown set
    d3 = new_field(p, seed + 10)
    tol3 = 1e-4 * float(np.sqrt((d3 ** 2).sum(axis=1)).max())
    info3, S3, W3, log3 = warm(c, p, d3, tol3)
    check_against_oracle(p, d3, tol3, S, info3, S3, W3, log3)
    c.close()


def test_warm_wing_full_size():
    p = synth.config_wing(with_volume=False)
    c, info0, S0, _ = fresh(p)
    d2 = np.ascontiguousarray(1.25 * p.disp + 0.3 * new_field(p, 5))
    tol = 1e-5 * float(np.sqrt((d2 ** 2).sum(axis=1)).max())
    info, S, W, log = warm(c, p, d2, tol)
    check_against_oracle(p, d2, tol, S0, info, S, W, log)
    assert info["converged"]
    c.close()


def test_warm_start_errors():
    p = synth.tiny_problem(nb=40, seed=2, m=3)
    c = gcb.Context(0)
    c.set_boundary(p.xyz, p.disp)
    c.set_params(p.radius, 3, 0.01 * p.max_disp, seed=p.seed, warm_start=True)
    with pytest.raises(gcb.GcbError) as e:       # nothing kept yet
        c.select()
    assert e.value.code == gcb.GCB_E_STATE
    c.set_params(p.radius, 3, 0.01 * p.max_disp, seed=p.seed)
    c.select()
    c.set_params(p.radius, 2, 0.01 * p.max_disp, seed=p.seed, warm_start=True)
    with pytest.raises(gcb.GcbError) as e:       # another partition
        c.select()
    assert e.value.code == gcb.GCB_E_STATE
    c.set_params(p.radius, 3, 0.01 * p.max_disp, seed=p.seed, nc_max=3, warm_start=True)
    with pytest.raises(gcb.GcbError) as e:       # cap below the kept count
        c.select()
    assert e.value.code == gcb.GCB_E_INVALID
    c.set_boundary(p.xyz, p.disp)                # a new boundary drops the kept set
    c.set_params(p.radius, 3, 0.01 * p.max_disp, seed=p.seed, warm_start=True)
    with pytest.raises(gcb.GcbError) as e:
        c.select()
    assert e.value.code == gcb.GCB_E_STATE
    c.close()
