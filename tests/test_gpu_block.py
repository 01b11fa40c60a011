"""GPU parity of the several-nodes-per-iteration variant (per_iter = p > 1; the
block form of the peak-selection idea cited in Section 1) against the oracle's
block rule.

Bar: the support sequence equal to oracle.select(per_iter = p), with equal
per-iteration groups, group maxima and appended counts, errors within 1e-10
max|d|, the interpolant (Eq. 1) at up to 2,000 boundary nodes within 1e-9
max|d| of the oracle's, and weights within kappa(Phi_S) u relative (at least
1e-7); or, after a near tie, a sequence the oracle's block replay certifies at
tau = 1e-9 max|d|.  Two FP64 solves of Phi_S W = D_S differ by about
kappa(Phi_S) u relative whatever their order (the oracle's own recurrence and a
LU solve differ by 1.6e-6 relative on the 10,000-node ellipsoid, where
kappa = 3.4e11 and kappa u = 3.8e-5), and the block append rounds differently
from q single appends, so the weights are held to the conditioning of the
support system, kappa computed from the oracle's support set.  Counters equal
the oracle's sums (an append of q nodes at |S| = n counts n + (n + 1) + ... +
(n + q - 1) pairs, as q single appends would)."""
import numpy as np
import pytest

import oracle
import paper_2004_04817_amd as gcb
import synth
from oracle import brute
from tests.gpu_util import first_divergence

pytestmark = pytest.mark.gpu

TAU = 1e-9


def gpu_block(p, per_iter, m=None, tol_abs=None, nc_max=None, init_idx=None):
    ctx = gcb.Context(0)
    ctx.set_boundary(p.xyz, p.disp)
    ctx.set_params(p.radius, p.m if m is None else m, p.tol_abs if tol_abs is None else tol_abs, nc_max=nc_max,
                   seed=p.seed, per_iter=per_iter, init_idx=init_idx)
    info = ctx.select()
    S, W = ctx.get_support()
    return ctx, info, S, W, ctx.get_log()


def oracle_block(p, per_iter, m=None, tol_abs=None, nc_max=None, init_idx=None):
    return oracle.select(p.xyz, p.disp, p.radius, p.m if m is None else m, p.tol_abs if tol_abs is None else tol_abs,
                         nc_max=nc_max, seed=p.seed, per_iter=per_iter, init_idx=init_idx, nthreads=0)


def assert_same_block_run(p, ctx, info, S, W, log, r, per_iter, m, tol, nc_max=None):
    md = p.max_disp
    div = first_divergence(S, r.S)
    if div == -1:
        assert info["iterations"] == r.iterations
        assert np.array_equal(log.group, r.log_group)
        assert np.array_equal(log.node, r.log_node)
        assert np.array_equal(log.appended, r.log_appended)
        assert np.abs(log.err - r.log_err).max(initial=0.0) <= 1e-10 * md
        phi_s = brute.rbf_matrix(p.xyz[r.S], p.xyz[r.S], p.radius)
        bar = max(1e-7, float(np.linalg.cond(phi_s)) * np.finfo(np.float64).eps / 2)
        assert np.abs(W - r.W).max() <= bar * max(1.0, np.abs(r.W).max())
        idx = np.unique(np.linspace(0, p.nb - 1, min(p.nb, 2000)).astype(np.int64))
        got = ctx.deform(np.ascontiguousarray(p.xyz[idx]))
        want = oracle.interpolate(p.xyz[r.S], r.W, p.radius, p.xyz[idx])
        assert np.abs(got - want).max() <= 1e-9 * md
        assert info["pairs_group"] == r.pairs_group and info["pairs_append"] == r.pairs_append
        assert abs(info["final_max_err"] - r.final_max_err) <= 1e-10 * md
    else:
        bad, reason, gap = oracle.validate_block(p.xyz, p.disp, p.radius, m, tol, S, log.group, log.appended,
                                                 TAU * md, per_iter, nc_max=nc_max, seed=p.seed)
        assert bad == -1, f"GPU sequence diverges at {div} and fails the block replay at {bad} (reason {reason})"
    assert info["nc"] == len(S) == 3 + int(np.sum(log.appended))
    assert info["pairs_cert"] == p.nb * info["nc"]


@pytest.mark.parametrize("nb", [8, 13, 16, 70])
@pytest.mark.parametrize("mm", ["1", "2", "3", "nb"])
@pytest.mark.parametrize("per_iter", [2, 3, 16])
def test_tiny_block_brute_force(nb, mm, per_iter):
    m = nb if mm == "nb" else int(mm)
    p = synth.tiny_problem(nb=nb, seed=nb, m=m)
    for tol_rel in (0.0, 0.05):
        tol = tol_rel * p.max_disp
        ctx, info, S, W, log = gpu_block(p, per_iter, m=m, tol_abs=tol)
        r = oracle_block(p, per_iter, m=m, tol_abs=tol)
        g = oracle.partition(p.nb, m, p.seed)
        Sb, _ = brute.gcb_brute(p.xyz, p.disp, p.radius, g, m, tol, per_iter=per_iter)
        assert list(S) == list(r.S) == Sb
        assert_same_block_run(p, ctx, info, S, W, log, r, per_iter, m, tol)
        ctx.close()


@pytest.mark.parametrize("per_iter", [2, 4, 8, 16])
def test_block_small_ellipsoid(per_iter):
    p = synth.config_small_ellipsoid(with_volume=False)
    ctx, info, S, W, log = gpu_block(p, per_iter)
    r = oracle_block(p, per_iter)
    print(f"p={per_iter}: nc={info['nc']} iterations={info['iterations']} (oracle {r.nc}, {r.iterations})",
          flush=True)
    assert_same_block_run(p, ctx, info, S, W, log, r, per_iter, p.m, p.tol_abs)
    assert info["converged"] and info["final_max_err"] <= p.tol_abs
    assert int(np.max(log.appended)) <= per_iter
    ctx.close()


def test_block_p1_is_algorithm1():
    """per_iter = 1 runs Algorithm 1's own kernels: the same run as per_iter = 0."""
    p = synth.config_small_ellipsoid(with_volume=False)
    c0, i0, S0, W0, l0 = gpu_block(p, 0)
    c1, i1, S1, W1, l1 = gpu_block(p, 1)
    assert np.array_equal(S0, S1) and np.array_equal(W0, W1) and i0["iterations"] == i1["iterations"]
    c0.close()
    c1.close()


@pytest.mark.parametrize("per_iter", [4, 8])
def test_block_wing_full_size(per_iter):
    """The 80,000-node wing (m = 107): the variant against the oracle's block rule."""
    p = synth.config_wing(with_volume=False)
    ctx, info, S, W, log = gpu_block(p, per_iter)
    r = oracle_block(p, per_iter)
    print(f"wing p={per_iter}: nc={info['nc']} iterations={info['iterations']} ms={info['ms_select']:.2f} "
          f"(oracle nc={r.nc}, iterations={r.iterations})", flush=True)
    assert info["converged"]
    assert_same_block_run(p, ctx, info, S, W, log, r, per_iter, p.m, p.tol_abs)
    ctx.close()


@pytest.mark.parametrize("m", [1, 2])
def test_block_large_groups(m):
    """Groups of 10,000 nodes (one target per lane: 64 candidates per block, several selection tiles) and
    5,000 nodes (two targets per lane)."""
    p = synth.config_small_ellipsoid(nb=10_000, with_volume=False)
    ctx, info, S, W, log = gpu_block(p, 4, m=m)
    r = oracle_block(p, 4, m=m)
    assert_same_block_run(p, ctx, info, S, W, log, r, 4, m, p.tol_abs)
    ctx.close()


def test_block_cap_inside_a_block():
    """Nc^max reached inside an iteration's block: fewer than p appended, then NOT_CONVERGED."""
    p = synth.config_small_ellipsoid(with_volume=False)
    for nc_max in (50, 51, 53):
        ctx, info, S, W, log = gpu_block(p, 4, nc_max=nc_max)
        r = oracle_block(p, 4, nc_max=nc_max)
        assert info["nc"] == nc_max == r.nc
        assert info["status"] == gcb.GCB_NOT_CONVERGED
        assert_same_block_run(p, ctx, info, S, W, log, r, 4, p.m, p.tol_abs, nc_max=nc_max)
        ctx.close()


def test_block_randomised_problems():
    """20 seeded random problems (Nb 5-600, any m, radius 0.3-3, tolerance 0-10 % max|d|, sometimes a cap),
    p from 2 to 16: the oracle's run, or a run its block replay certifies; GCB_E_SINGULAR where the oracle
    finds the support matrix singular."""
    g = np.random.default_rng(4817)
    for case in range(20):
        nb = int(g.integers(5, 601))
        m = int(g.integers(1, nb + 1))
        radius = float(g.uniform(0.3, 3.0))
        per_iter = int(g.integers(2, 17))
        p = synth.tiny_problem(nb=nb, seed=2000 + case, m=m, radius=radius)
        tol = float(g.choice([0.0, 1e-4, 1e-3, 1e-2, 0.1])) * p.max_disp
        nc_max = int(g.integers(3, nb + 1)) if g.random() < 0.3 else None
        print(f"case {case}: nb={nb} m={m} p={per_iter} R={radius:.3f} tol={tol:.3e} nc_max={nc_max}", flush=True)
        r = oracle_block(p, per_iter, m=m, tol_abs=tol, nc_max=nc_max)
        if r.status < 0:
            assert r.status == oracle.ORC_E_SINGULAR
            with pytest.raises(gcb.GcbError) as e:
                gpu_block(p, per_iter, m=m, tol_abs=tol, nc_max=nc_max)
            assert e.value.code == gcb.GCB_E_SINGULAR
            continue
        ctx, info, S, W, log = gpu_block(p, per_iter, m=m, tol_abs=tol, nc_max=nc_max)
        assert_same_block_run(p, ctx, info, S, W, log, r, per_iter, m, tol, nc_max=nc_max)
        ctx.close()


def test_block_duplicate_node_is_singular():
    """Two copies of one node ranked into the same block: the Schur complement's pivot is zero."""
    p = synth.tiny_problem(nb=40, seed=5, m=1)
    xyz, disp = p.xyz.copy(), p.disp.copy()
    r0 = oracle_block(p, 8, m=1, tol_abs=0.0)
    first = int(r0.S[3])      # the first node the loop appends
    xyz[first ^ 1] = xyz[first]
    disp[first ^ 1] = disp[first] * 1.5   # a different value, so both keep a large error
    p.xyz, p.disp = xyz, disp
    r = oracle_block(p, 8, m=1, tol_abs=0.0)
    assert r.status == oracle.ORC_E_SINGULAR
    with pytest.raises(gcb.GcbError) as e:
        gpu_block(p, 8, m=1, tol_abs=0.0)
    assert e.value.code == gcb.GCB_E_SINGULAR


def test_block_argument_errors():
    p = synth.tiny_problem(nb=30)
    ctx = gcb.Context(0)
    ctx.set_boundary(p.xyz, p.disp)
    with pytest.raises(gcb.GcbError) as e:
        ctx.set_params(p.radius, 3, 0.0, per_iter=gcb.GCB_MAX_PER_ITER + 1)
    assert e.value.code == gcb.GCB_E_INVALID
    with pytest.raises(gcb.GcbError) as e:
        ctx.set_params(p.radius, 3, 0.0, per_iter=-1)
    assert e.value.code == gcb.GCB_E_INVALID
    with pytest.raises(gcb.GcbError) as e:
        ctx.set_params(p.radius, 3, 0.0, per_iter=4, warm_start=True)
    assert e.value.code == gcb.GCB_E_INVALID
    ctx.set_params(p.radius, 3, 0.0, per_iter=4)
    b = gcb.Batch(0)
    with pytest.raises(gcb.GcbError) as e:
        b.select([ctx])
    assert e.value.code == gcb.GCB_E_INVALID
    b.close()
    ctx.close()
