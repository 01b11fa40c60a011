"""Pins of the oracle's several-nodes-per-iteration variant (per_iter = p > 1):
in every iteration the nodes of the active group whose error exceeds E* are
ranked by (error descending, index ascending) on one sweep's errors and the
first p are appended (the peak-selection idea cited in Section 1, in block
form); p = 1 is Algorithm 1.

Pinned against an independent NumPy brute force that re-solves Phi_S with a
library solver every iteration, the full-system special case, the cap, an
independent ranking check on the 2,000-node ellipsoid, and planted deviations
that the block replay must reject."""
import numpy as np
import pytest

import oracle
import synth
from oracle import brute


def _tiny(nb, m, tol_rel, seed=7):
    p = synth.tiny_problem(nb=nb, m=m, seed=seed, radius=1.5)
    return p, tol_rel * p.max_disp


@pytest.mark.parametrize("nb", [8, 12, 16])
@pytest.mark.parametrize("m", [1, 2, 3])
@pytest.mark.parametrize("per_iter", [2, 3, 16])
@pytest.mark.parametrize("tol_rel", [0.0, 1e-3, 0.05])
def test_block_select_matches_brute_force_tiny(nb, m, per_iter, tol_rel):
    p, tol = _tiny(nb, m, tol_rel)
    g = oracle.partition(p.nb, m, p.seed)
    r = oracle.select(p.xyz, p.disp, p.radius, m, tol, seed=p.seed, per_iter=per_iter)
    S, log = brute.gcb_brute(p.xyz, p.disp, p.radius, g, m, tol, per_iter=per_iter)
    assert r.status >= 0
    assert list(r.S) == S
    assert len(r.log_group) == len(log)
    for it, (k, gg, n, E, cnt) in enumerate(log):
        assert r.log_group[it] == gg and r.log_node[it] == n and r.log_appended[it] == cnt
        assert abs(r.log_err[it] - E) <= 1e-9 * max(1.0, E)
    W = brute.solve_weights(p.xyz[r.S], p.disp[r.S], p.radius)
    assert np.abs(r.W - W).max() <= 1e-8 * max(1.0, np.abs(W).max())


def test_per_iter_one_is_algorithm_1():
    """p = 1 is Algorithm 1: the same run as the default selection on the ellipsoid."""
    p = synth.config_small_ellipsoid(with_volume=False)
    a = oracle.select(p.xyz, p.disp, p.radius, p.m, p.tol_abs, seed=p.seed)
    b = oracle.select(p.xyz, p.disp, p.radius, p.m, p.tol_abs, seed=p.seed, per_iter=1)
    assert np.array_equal(a.S, b.S) and np.array_equal(a.W, b.W) and a.iterations == b.iterations


def test_full_system_in_one_block():
    """E* = 0, m = 1, p >= Nb: the first iteration appends every remaining node, ranked by
    error; then Eq. 3 holds at every node and W solves the full system."""
    p, _ = _tiny(12, 1, 0.0)
    r = oracle.select(p.xyz, p.disp, p.radius, 1, 0.0, seed=p.seed, per_iter=64)
    assert r.nc == p.nb and r.log_appended[0] == p.nb - 3 and r.log_appended[1:].sum() == 0
    S0 = list(r.S[:3])
    W0 = brute.solve_weights(p.xyz[S0], p.disp[S0], p.radius)
    rest = [j for j in range(p.nb) if j not in S0]
    e = np.sqrt(((brute.rbf_matrix(p.xyz[rest], p.xyz[S0], p.radius) @ W0 - p.disp[rest]) ** 2).sum(1))
    order = [rest[t] for t in np.lexsort((rest, -e))]
    assert list(r.S[3:]) == order
    Wf = np.linalg.solve(brute.rbf_matrix(p.xyz, p.xyz, p.radius), p.disp)
    F = brute.rbf_matrix(p.xyz, p.xyz[r.S], p.radius) @ r.W
    assert np.abs(F - p.disp).max() <= 1e-9 * p.max_disp
    assert np.abs(r.W - Wf[r.S]).max() <= 1e-7 * np.abs(Wf).max()


def test_block_cap():
    """Nc^max bounds |S| inside a block: the block is cut at the cap and the next iteration
    that finds a node over E* ends the run as not converged."""
    p = synth.config_small_ellipsoid(with_volume=False)
    r = oracle.select(p.xyz, p.disp, p.radius, p.m, p.tol_abs, seed=p.seed, nc_max=50, per_iter=4)
    assert r.status == oracle.ORC_NOT_CONVERGED and r.nc == 50
    assert 3 + int(r.log_appended.sum()) == 50


def test_block_ranking_on_the_ellipsoid():
    """Every iteration of a p = 4 run on the ellipsoid appended the top of its group: checked at
    sampled iterations with a from-scratch dense solve on the support prefix."""
    p = synth.config_small_ellipsoid(with_volume=False)
    per = 4
    r = oracle.select(p.xyz, p.disp, p.radius, p.m, p.tol_abs, seed=p.seed, per_iter=per)
    assert r.converged and r.final_max_err <= p.tol_abs
    g = oracle.partition(p.nb, p.m, p.seed)
    n_before = 3 + np.concatenate([[0], np.cumsum(r.log_appended.astype(int))[:-1]])
    checked = 0
    for it in range(0, len(r.log_group), 3):
        n0, q = int(n_before[it]), int(r.log_appended[it])
        S = list(r.S[:n0])
        cand = np.array([j for j in np.flatnonzero(g == r.log_group[it]) if j not in S])
        W = brute.solve_weights(p.xyz[S], p.disp[S], p.radius)
        e = np.sqrt(((brute.rbf_matrix(p.xyz[cand], p.xyz[S], p.radius) @ W - p.disp[cand]) ** 2).sum(1))
        order = cand[np.lexsort((cand, -e))]
        over = int((e > p.tol_abs).sum())
        assert q == min(per, over), it
        assert list(r.S[n0:n0 + q]) == list(order[:q]), it
        checked += 1
    assert checked > 20 and r.log_appended.max() == per
    # fewer iterations than Algorithm 1 for about the same support count
    a = oracle.select(p.xyz, p.disp, p.radius, p.m, p.tol_abs, seed=p.seed)
    assert r.iterations < a.iterations


def test_block_replay_accepts_own_run_and_rejects_planted_deviations():
    p = synth.config_small_ellipsoid(with_volume=False)
    per = 4
    r = oracle.select(p.xyz, p.disp, p.radius, p.m, p.tol_abs, seed=p.seed, per_iter=per)
    args = (p.xyz, p.disp, p.radius, p.m, p.tol_abs)
    bad, reason, gap = oracle.validate_block(*args, r.S, r.log_group, r.log_appended, 0.0, per, seed=p.seed)
    assert bad == -1 and gap == 0.0
    n_before = 3 + np.concatenate([[0], np.cumsum(r.log_appended.astype(int))[:-1]])
    it = int(np.flatnonzero(r.log_appended == per)[2])
    n0 = int(n_before[it])
    # two nodes of a block swapped: the factor order no longer follows the ranking
    S = r.S.copy()
    S[n0], S[n0 + 1] = S[n0 + 1], S[n0]
    bad, reason, _ = oracle.validate_block(*args, S, r.log_group, r.log_appended, 1e-12 * p.max_disp, per,
                                           seed=p.seed)
    assert bad == it and reason == 3
    # a block cut short: one node over E* left out
    app = r.log_appended.copy()
    app[it] -= 1
    S = np.delete(r.S, n0 + per - 1)
    bad, reason, _ = oracle.validate_block(*args, S, r.log_group, app, 1e-12 * p.max_disp, per, seed=p.seed)
    assert bad == it and reason == 4
    # a node from outside the top of the group
    g = oracle.partition(p.nb, p.m, p.seed)
    others = [j for j in np.flatnonzero(g == r.log_group[it]) if j not in r.S]
    S = r.S.copy()
    S[n0 + per - 1] = others[0]
    bad, reason, _ = oracle.validate_block(*args, S, r.log_group, r.log_appended, 1e-12 * p.max_disp, per,
                                           seed=p.seed)
    assert bad == it and reason in (3, 4)
    # Algorithm 1's own run is a valid p = 1 block run
    a = oracle.select(*args, seed=p.seed)
    bad, reason, _ = oracle.validate_block(*args, a.S, a.log_group, a.log_appended, 0.0, 1, seed=p.seed)
    assert bad == -1, reason


def test_invalid_per_iter_rejected():
    p, tol = _tiny(10, 2, 0.0)
    assert oracle.select(p.xyz, p.disp, p.radius, 2, tol, per_iter=65).status == oracle.ORC_E_INVALID
