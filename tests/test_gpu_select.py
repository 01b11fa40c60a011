"""GPU parity of the greedy selection (Algorithm 1) against the FP64 oracle.

Bar: the selected index sequence is bit-exact, except after an iteration
whose top two errors differ by less than TAU_FP64 * max|d| (then the GPU run
must be certified step by step by the oracle's follow-mode replay).
Weights and errors agree to FP64 rounding of the different factor algorithm
(inverse factor M = L^-1 on the GPU, forward/back substitution in the oracle).
"""
import numpy as np
import pytest

import oracle
import paper_2004_04817_amd as gcb
import synth
from oracle import brute
from tests.gpu_util import first_divergence, gpu_select, oracle_select

pytestmark = pytest.mark.gpu

TAU_FP64 = 1e-9   # near-tie tolerance, relative to max|d|


def assert_same_run(p, g_info, g_S, g_W, g_log, r, tol_abs, m, tau=TAU_FP64, nc_max=None):
    md = p.max_disp
    div = first_divergence(g_S, r.S)
    if div == -1:
        assert g_info["iterations"] == r.iterations
        assert np.array_equal(g_log.group, r.log_group)
        assert np.array_equal(g_log.node, r.log_node)
        assert np.array_equal(g_log.appended, r.log_appended)
        assert np.abs(g_log.err - r.log_err).max() <= 1e-10 * md
        Wscale = max(1.0, np.abs(r.W).max())
        assert np.abs(g_W - r.W).max() <= 1e-7 * Wscale
    else:
        bad, reason, gap = oracle.validate(p.xyz, p.disp, p.radius, m, tol_abs, g_S, g_log.group, g_log.node,
                                           g_log.appended, tau * md, nc_max=nc_max, seed=p.seed)
        assert bad == -1, f"GPU sequence diverges at {div} and fails replay at {bad} (reason {reason})"
    assert g_info["nc"] == len(g_S)
    assert g_info["pairs_cert"] == p.nb * g_info["nc"]


@pytest.mark.parametrize("nb", [8, 13, 16, 70])
@pytest.mark.parametrize("mm", ["1", "2", "3", "nb"])
def test_tiny_brute_force(nb, mm):
    m = nb if mm == "nb" else int(mm)
    p = synth.tiny_problem(nb=nb, seed=nb, m=m)
    for tol_rel in (0.0, 0.05):
        tol = tol_rel * p.max_disp
        ctx, info, S, W, log = gpu_select(p, tol_abs=tol, m=m)
        r = oracle_select(p, tol_abs=tol, m=m)
        g = oracle.partition(p.nb, m, p.seed)
        Sb, _ = brute.gcb_brute(p.xyz, p.disp, p.radius, g, m, tol)
        assert list(S) == list(r.S) == Sb
        assert_same_run(p, info, S, W, log, r, tol, m)
        ctx.close()


def test_small_ellipsoid_matches_oracle():
    """Nb = 2,000 ellipsoid, m = 10, E* = 1e-4 max|d| (Nc of a few hundred)."""
    p = synth.config_small_ellipsoid(with_volume=False)
    ctx, info, S, W, log = gpu_select(p)
    r = oracle_select(p)
    assert info["status"] == 0 and info["converged"]
    assert_same_run(p, info, S, W, log, r, p.tol_abs, p.m)
    assert abs(info["final_max_err"] - r.final_max_err) <= 1e-10 * p.max_disp
    assert abs(info["final_rms_err"] - r.final_rms_err) <= 1e-10 * p.max_disp
    assert info["pairs_group"] == r.pairs_group and info["pairs_append"] == r.pairs_append
    ctx.close()


def test_traditional_greedy_m1():
    """m = 1 is the traditional greedy: GPU sequence equals the oracle's and
    the independent NumPy Rendall-Allen implementation."""
    p = synth.config_small_ellipsoid(with_volume=False)
    ctx, info, S, W, log = gpu_select(p, m=1)
    r = oracle_select(p, m=1)
    assert_same_run(p, info, S, W, log, r, p.tol_abs, 1)
    assert list(S) == brute.traditional_greedy(p.xyz, p.disp, p.radius, p.tol_abs)
    ctx.close()


def test_capacity_growth_and_cap():
    """E* = 0 with Nc^max = 1,100 forces |S| past the initial device capacity
    (1,024) and ends at the cap with GCB_NOT_CONVERGED, like the oracle."""
    p = synth.config_small_ellipsoid(with_volume=False)
    ctx, info, S, W, log = gpu_select(p, tol_abs=0.0, nc_max=1100)
    r = oracle_select(p, tol_abs=0.0, nc_max=1100)
    assert info["status"] == 1 and r.status == oracle.ORC_NOT_CONVERGED
    assert len(S) == 1100
    assert_same_run(p, info, S, W, log, r, 0.0, p.m, nc_max=1100)
    ctx.close()



def test_selection_past_one_staging_window():
    """E* = 0 with Nc^max = 2,000 on the 80,000-node wing: |S| passes the group sweep's 1,280-support staging
    window (the next window is loaded into registers while one is evaluated), the factor kernels' 1,024-entry
    prefetch of a row or column of M, and a capacity growth past 1,024; ends at the cap like the oracle."""
    p = synth.config_wing(with_volume=False)
    ctx, info, S, W, log = gpu_select(p, tol_abs=0.0, nc_max=2000)
    r = oracle_select(p, tol_abs=0.0, nc_max=2000)
    assert info["status"] == 1 and r.status == oracle.ORC_NOT_CONVERGED
    assert len(S) == 2000 == r.nc
    assert_same_run(p, info, S, W, log, r, 0.0, p.m, nc_max=2000)
    ctx.close()


def test_explicit_partition_and_start():
    p = synth.config_small_ellipsoid(nb=1500, with_volume=False)
    g = np.random.default_rng(3).integers(0, 7, p.nb).astype(np.int32)
    init = [5, 700, 1400]
    ctx, info, S, W, log = gpu_select(p, m=7, group_of=g, init_idx=init)
    r = oracle_select(p, m=7, group_of=g, init_idx=init)
    assert list(S[:3]) == init
    assert_same_run(p, info, S, W, log, r, p.tol_abs, 7)
    ctx.close()


def test_wing_full_size_selection():
    """80,000-node wing at m = 107, E* = 1e-5 max|d|: the full workload."""
    p = synth.config_wing(with_volume=False)
    ctx, info, S, W, log = gpu_select(p)
    r = oracle_select(p)
    print("wing: nc", info["nc"], "iters", info["iterations"], "ms", info["ms_select"], "oracle nc", r.nc, flush=True)
    assert info["converged"] and info["final_max_err"] <= p.tol_abs
    assert_same_run(p, info, S, W, log, r, p.tol_abs, p.m)
    ctx.close()


def test_monitor_samples_match_oracle():
    """Monitor every m iterations (Section 3: all nodes checked once per m iterations):
    the selection is unchanged and every sample equals the oracle's."""
    p = synth.config_small_ellipsoid(with_volume=False)
    _, info0, S0, _, _ = gpu_select(p)
    c = gcb.Context(0)
    c.set_boundary(p.xyz, p.disp)
    c.set_params(p.radius, p.m, p.tol_abs, seed=p.seed, monitor_every=p.m)
    info = c.select()
    S, _ = c.get_support()
    assert np.array_equal(S, S0) and info["iterations"] == info0["iterations"]
    it, mx, rm = c.get_monitor()
    r = oracle.select(p.xyz, p.disp, p.radius, p.m, p.tol_abs, seed=p.seed, monitor_every=p.m)
    assert len(mx) == len(r.mon_max) == info["iterations"] // p.m
    assert np.array_equal(it, p.m * np.arange(1, len(mx) + 1))
    assert np.abs(mx - r.mon_max).max() <= 1e-10 * p.max_disp
    assert np.abs(rm - r.mon_rms).max() <= 1e-10 * p.max_disp
    # m = 1 with a sample every iteration
    c.set_params(p.radius, 1, p.tol_abs, seed=p.seed, monitor_every=1)
    info1 = c.select()
    it1, mx1, _ = c.get_monitor()
    log = c.get_log()
    assert len(mx1) == info1["iterations"]
    assert np.abs(mx1[:-1] - log.err[1:]).max() <= 1e-12 * p.max_disp
    with gcb.Batch(0) as b:
        with pytest.raises(gcb.GcbError):
            b.begin(c)
    c.close()


def test_empty_and_uneven_groups_single_and_batched():
    """An explicit partition with empty groups (their iterations find nothing: E = 0, quiet)
    and very uneven sizes, single and in a batch, against the oracle."""
    p = synth.config_small_ellipsoid(nb=1200, with_volume=False)
    m = 9
    rng = np.random.default_rng(5)
    g = rng.choice([0, 2, 3, 7], size=p.nb, p=[0.55, 0.3, 0.1, 0.05]).astype(np.int32)   # groups 1,4,5,6,8 empty
    r = oracle_select(p, m=m, group_of=g)
    ctx, info, S, W, log = gpu_select(p, m=m, group_of=g)
    assert_same_run(p, info, S, W, log, r, p.tol_abs, m)
    assert np.all(log.node[np.isin(log.group, [1, 4, 5, 6, 8])] == -1)
    c2 = gcb.Context(0)
    c2.set_boundary(p.xyz, p.disp)
    c2.set_params(p.radius, m, p.tol_abs, seed=p.seed)
    c2.set_groups(g)
    other = [gcb.Context(0) for _ in range(4)]
    for j, c in enumerate(other):
        q = synth.tiny_problem(nb=60 + j, seed=40 + j, m=2)
        c.set_boundary(q.xyz, q.disp)
        c.set_params(q.radius, 2, 0.01 * q.max_disp, seed=q.seed)
    with gcb.Batch(0) as b:
        b.select([c2] + other)
    S2, W2 = c2.get_support()
    assert np.array_equal(S2, S)
    assert np.abs(W2 - W).max() <= 1e-12 * max(1.0, np.abs(W).max())
    for c in [ctx, c2] + other:
        c.close()


def test_randomised_small_problems_against_the_oracle():
    """40 seeded random problems: Nb from 5 to 600, any m in [1, Nb], radius from 0.3 to 3 (sparse
    to dense Phi), tolerance from 0 to 10 % of max|d|, sometimes a cap on Nc: the same run as the
    oracle (or a run the oracle's replay certifies after a near-tie)."""
    g = np.random.default_rng(2004)
    for case in range(40):
        nb = int(g.integers(5, 601))
        m = int(g.integers(1, nb + 1))
        radius = float(g.uniform(0.3, 3.0))
        p = synth.tiny_problem(nb=nb, seed=1000 + case, m=m, radius=radius)
        tol = float(g.choice([0.0, 1e-4, 1e-3, 1e-2, 0.1])) * p.max_disp
        nc_max = int(g.integers(3, nb + 1)) if g.random() < 0.3 else None
        print(f"case {case}: nb={nb} m={m} R={radius:.3f} tol={tol:.3e} nc_max={nc_max}", flush=True)
        r = oracle_select(p, tol_abs=tol, m=m, nc_max=nc_max)
        if r.status < 0:
            # the oracle found the support matrix singular (close nodes at a large radius): the library
            # must report the same condition, not a result
            assert r.status == oracle.ORC_E_SINGULAR
            with pytest.raises(gcb.GcbError) as e:
                gpu_select(p, tol_abs=tol, m=m, nc_max=nc_max)
            assert e.value.code == gcb.GCB_E_SINGULAR
            continue
        ctx, info, S, W, log = gpu_select(p, tol_abs=tol, m=m, nc_max=nc_max)
        assert_same_run(p, info, S, W, log, r, tol, m, nc_max=nc_max)
        ctx.close()


@pytest.mark.parametrize("m", [1, 2])
def test_large_groups_against_the_oracle(m):
    """Groups of 10,000 nodes (one target per lane, supports split over the block's waves) and 5,000 nodes (two
    targets per lane, small staging windows)."""
    p = synth.config_small_ellipsoid(nb=10_000, with_volume=False)
    ctx, info, S, W, log = gpu_select(p, m=m)
    r = oracle_select(p, m=m)
    assert_same_run(p, info, S, W, log, r, p.tol_abs, m)
    ctx.close()


@pytest.mark.parametrize("m", [300, 263])
def test_group_counts_above_256(m):
    """m = 300 replays captured chunks of 60 iterations in five phases of k mod m; m = 263 (prime, no
    divisor in [32, 128]) launches its iterations uncaptured.  Both against the oracle."""
    p = synth.config_wing(with_volume=False, m=m)
    ctx, info, S, W, log = gpu_select(p)
    r = oracle_select(p)
    assert_same_run(p, info, S, W, log, r, p.tol_abs, m)
    ctx.close()


def test_kernel_timing_keeps_the_selection():
    """With kernel timing on, the selection runs uncaptured with events between its launches: the same
    support sequence and weights, bitwise; one launch of each factor kernel per iteration (iterations past the
    stop included), one certificate."""
    p = synth.config_small_ellipsoid(with_volume=False)
    ctx, info, S, W, log = gpu_select(p)
    ctx.set_kernel_timing(True)
    info2 = ctx.select()
    S2, W2 = ctx.get_support()
    kt = ctx.kernel_times()
    ctx.set_kernel_timing(False)
    assert np.array_equal(S, S2) and np.array_equal(W, W2) and info2["iterations"] == info["iterations"]
    assert kt["k_factor_l"]["launches"] == kt["k_factor_u"]["launches"] >= info2["iterations"]
    assert 0 < kt["sweep"]["launches"] <= kt["k_factor_l"]["launches"]
    assert kt["certificate"]["launches"] == 1
    assert all(v["ms"] > 0 for v in kt.values())
    info3 = ctx.select()
    S3, W3 = ctx.get_support()
    assert np.array_equal(S, S3) and np.array_equal(W, W3)
    fresh = gcb.Context(0)
    with pytest.raises(gcb.GcbError):   # no selection ran with kernel timing on
        fresh.kernel_times()
    fresh.close()
    ctx.close()


@pytest.mark.parametrize("case", ["wing80k", "ellipsoid", "wing_m300"])
def test_convergence_probe_completes_the_same_run(case, monkeypatch):
    """The convergence probe ends the final run of quiet iterations early, writing the log entries those
    iterations would write: the same support sequence, weights and iteration count as with the probe off, the
    same groups, appended flags and argmax nodes, errors within 1e-12 max|d|; and against the oracle."""
    if case == "wing80k":
        p = synth.config_wing(with_volume=False)
    elif case == "ellipsoid":
        p = synth.config_small_ellipsoid(with_volume=False)
    else:
        p = synth.config_wing(with_volume=False, m=300)
    ctx, info, S, W, log = gpu_select(p)
    monkeypatch.setenv("GCB_PROBE", "0")
    c0, i0, S0, W0, l0 = gpu_select(p)
    monkeypatch.setenv("GCB_PROBE", "1")
    print(f"{case}: iterations {info['iterations']}, probe completed {info['probed_iterations']}; "
          f"select {info['ms_select']:.2f} ms vs {i0['ms_select']:.2f} ms without", flush=True)
    assert i0["probed_iterations"] == 0
    assert np.array_equal(S, S0) and np.array_equal(W, W0)
    assert info["iterations"] == i0["iterations"] and info["nc"] == i0["nc"]
    assert np.array_equal(log.group, l0.group) and np.array_equal(log.appended, l0.appended)
    assert np.array_equal(log.node, l0.node)
    assert np.abs(log.err - l0.err).max() <= 1e-12 * p.max_disp
    assert info["pairs_group"] == i0["pairs_group"] and info["pairs_append"] == i0["pairs_append"]
    assert info["final_max_err"] == i0["final_max_err"]
    r = oracle_select(p)
    assert_same_run(p, info, S, W, log, r, p.tol_abs, p.m)
    ctx.close()
    c0.close()
