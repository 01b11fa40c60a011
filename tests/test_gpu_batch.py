"""Batched selection and deformation of several surfaces (shared launches).

Every context of a batch runs the same kernels with the same arguments as a
single selection, so its support sequence, log and weights must equal those
of gcb_select on the same problem; one scaled-down uneven batch is also
checked against the FP64 oracle directly.
"""
import numpy as np
import pytest
import torch

import synth
import paper_2004_04817_amd as gcb
from tests.gpu_util import gpu_select, oracle_select
from tests.test_gpu_select import assert_same_run

pytestmark = pytest.mark.gpu


def make_ctx(p, m=None):
    c = gcb.Context(0)
    c.set_boundary(p.xyz, p.disp)
    c.set_params(p.radius, p.m if m is None else m, p.tol_abs, nc_max=p.nc_max, seed=p.seed)
    return c


def assert_equal_runs(c, single):
    _, info1, S1, W1, log1 = single
    S, W = c.get_support()
    log = c.get_log()
    assert np.array_equal(S, S1)
    assert np.array_equal(log.group, log1.group)
    assert np.array_equal(log.node, log1.node)
    assert np.array_equal(log.appended, log1.appended)
    assert np.abs(log.err - log1.err).max(initial=0.0) <= 1e-12 * max(1.0, np.abs(log1.err).max(initial=0.0))
    assert np.abs(W - W1).max() <= 1e-12 * max(1.0, np.abs(W1).max())


def test_multi_surface_batch_equals_single():
    """32 uneven surfaces (Nb log-uniform in [1e3, 5e4], ellipsoids and wings)."""
    probs = synth.config_multi_surface(32, with_volume=False)
    singles = [gpu_select(p) for p in probs]
    ctxs = [make_ctx(p) for p in probs]
    with gcb.Batch(0) as b:
        infos = b.select(ctxs)
    for p, c, s, inf in zip(probs, ctxs, singles, infos):
        assert inf["nc"] == s[1]["nc"] and inf["iterations"] == s[1]["iterations"], p.name
        assert inf["status"] == s[1]["status"]
        assert inf["final_max_err"] == pytest.approx(s[1]["final_max_err"], rel=1e-9, abs=1e-15)
        assert_equal_runs(c, s)
    for c, s in zip(ctxs, singles):
        c.close()
        s[0].close()


def test_scaled_batch_matches_oracle():
    probs = synth.config_multi_surface(32, with_volume=False, size_scale=0.08)
    ctxs = [make_ctx(p) for p in probs]
    with gcb.Batch(0) as b:
        infos = b.select(ctxs)
    for p, c, inf in zip(probs, ctxs, infos):
        S, W = c.get_support()
        r = oracle_select(p)
        assert_same_run(p, inf, S, W, c.get_log(), r, p.tol_abs, p.m)
        c.close()


def test_step_api_small_steps():
    """begin / step(5) / end with contexts that finish at different steps."""
    probs = [synth.config_small_ellipsoid(with_volume=False), synth.tiny_problem(nb=70, seed=3, m=3),
             synth.multi_surface_problem(1, 3000, 77)]
    singles = [gpu_select(p) for p in probs]
    ctxs = [make_ctx(p) for p in probs]
    with gcb.Batch(0) as b:
        for c in ctxs:
            b.begin(c)
        seen_partial = False
        while True:
            run = b.step(ctxs, 5)
            if run.sum() == 0:
                break
            seen_partial |= 0 < run.sum() < len(ctxs)
        assert seen_partial
        infos = [b.end(c) for c in ctxs]
    for c, s, inf in zip(ctxs, singles, infos):
        assert inf["nc"] == s[1]["nc"]
        assert_equal_runs(c, s)
        c.close()


def test_batch_probe_completes_the_same_run(monkeypatch):
    """Batch steps of 8 iterations poll often enough for the convergence probe to end the 80,000-node wing's
    final quiet run (m = 107) inside the batch: the run equals a single selection with the probe off (support
    sequence, iteration count, groups, appended flags and argmax nodes; weights within 1e-12 relative, errors
    within 1e-12 max|d|, the certificate within 1e-9 relative) and the oracle's."""
    probs = [synth.config_wing(with_volume=False), synth.config_small_ellipsoid(with_volume=False)]
    monkeypatch.setenv("GCB_PROBE", "0")
    refs = [gpu_select(p) for p in probs]
    monkeypatch.setenv("GCB_PROBE", "1")
    ctxs = [make_ctx(p) for p in probs]
    with gcb.Batch(0) as b:
        for c in ctxs:
            b.begin(c)
        while b.step(ctxs, 8).sum() > 0:
            pass
        infos = [b.end(c) for c in ctxs]
    assert infos[0]["probed_iterations"] > 0
    for p, c, inf, (c0, i0, S0, W0, l0) in zip(probs, ctxs, infos, refs):
        assert i0["probed_iterations"] == 0
        S, W = c.get_support()
        log = c.get_log()
        assert np.array_equal(S, S0)
        assert np.abs(W - W0).max() <= 1e-12 * max(1.0, np.abs(W0).max())
        assert inf["iterations"] == i0["iterations"] and inf["nc"] == i0["nc"]
        assert np.array_equal(log.group, l0.group) and np.array_equal(log.appended, l0.appended)
        assert np.array_equal(log.node, l0.node)
        assert np.abs(log.err - l0.err).max() <= 1e-12 * p.max_disp
        assert inf["final_max_err"] == pytest.approx(i0["final_max_err"], rel=1e-9)
        assert_same_run(p, inf, S, W, log, oracle_select(p), p.tol_abs, p.m)
        c.close()
        c0.close()


def test_more_than_64_contexts():
    probs = [synth.tiny_problem(nb=16 + (j % 9), seed=100 + j, m=1 + j % 4, tol_rel=0.01) for j in range(70)]
    ctxs = [make_ctx(p) for p in probs]
    with gcb.Batch(0) as b:
        infos = b.select(ctxs)
    for p, c, inf in zip(probs, ctxs, infos):
        S, W = c.get_support()
        r = oracle_select(p)
        assert list(S) == list(r.S)
        assert_same_run(p, inf, S, W, c.get_log(), r, p.tol_abs, p.m)
        c.close()


@pytest.mark.parametrize("in_dt,out_dt", [(torch.float64, torch.float64), (torch.float32, torch.float32),
                                          (torch.float64, torch.float32)])
def test_deform_batch_equals_single(in_dt, out_dt):
    probs = synth.config_multi_surface(12, with_volume=True, nv_per_nb=3, size_scale=0.3)
    probs.append(synth.tiny_problem(nb=20, seed=5, m=2))
    probs[-1].volume = np.zeros((0, 3))            # an empty point set in the batch
    ctxs = [make_ctx(p) for p in probs]
    with gcb.Batch(0) as b:
        b.select(ctxs)
        xs = [torch.from_numpy(p.volume).to(device="cuda", dtype=in_dt).contiguous() for p in probs]
        outs = b.deform(ctxs, xs, out_dtype=out_dt)
        torch.cuda.synchronize()
    for p, c, x, o in zip(probs, ctxs, xs, outs):
        ref = c.deform(x, out_dtype=out_dt)
        torch.cuda.synchronize()
        if out_dt == torch.float64:
            assert torch.equal(o, ref), p.name
        else:
            assert torch.allclose(o, ref, rtol=0, atol=1e-7 * p.max_disp), p.name
        c.close()


def test_batch_errors():
    p = synth.config_small_ellipsoid(with_volume=False)
    c = make_ctx(p)
    fresh = make_ctx(synth.tiny_problem(nb=20, seed=9, m=2))
    with gcb.Batch(0) as b:
        with pytest.raises(gcb.GcbError) as e:
            b.step([c], 0)
        assert e.value.code == gcb.GCB_E_INVALID
        with pytest.raises(gcb.GcbError) as e:
            b.deform([fresh], [torch.zeros((4, 3), dtype=torch.float64, device="cuda")])
        assert e.value.code == gcb.GCB_E_STATE
        b.begin(c)
        with pytest.raises(gcb.GcbError) as e:
            b.end(c)
        assert e.value.code == gcb.GCB_E_STATE
        while b.step([c], 64).sum():
            pass
        info = b.end(c)
        assert info["converged"]
    c.close()
    fresh.close()


@pytest.mark.parametrize("layout", [(1, 1), (2, 4), (4, 4), (4, 1)])
def test_every_layout_gives_the_same_selection(layout):
    """The autotuner's candidates: the factor's sums do not depend on the layout and the
    sweep layout changes only rounding, so each candidate reproduces the single selections."""
    probs = synth.config_multi_surface(8, with_volume=False, size_scale=0.3)
    singles = [gpu_select(p) for p in probs]
    ctxs = [make_ctx(p) for p in probs]
    with gcb.Batch(0) as b:
        b.set_layout(*layout)
        b.select(ctxs)
    for c, s in zip(ctxs, singles):
        assert_equal_runs(c, s)
        c.close()


def test_autotune_picks_a_candidate():
    from paper_2004_04817_amd import autotune
    probs = synth.config_multi_surface(6, with_volume=False, size_scale=0.2)
    ctxs = [make_ctx(p) for p in probs]
    best, times = autotune.tune_batch(ctxs, repeats=1)
    assert best in autotune.CANDIDATES and set(times) == set(autotune.CANDIDATES)
    assert all(t > 0 for t in times.values())
    for c in ctxs:
        c.close()


def test_lone_context_uses_its_graph_and_matches():
    """A batch with one running context replays that context's captured chunk."""
    p = synth.config_small_ellipsoid(with_volume=False)
    single = gpu_select(p)
    c = make_ctx(p)
    with gcb.Batch(0) as b:
        b.select([c])
    assert_equal_runs(c, single)
    c.close()
