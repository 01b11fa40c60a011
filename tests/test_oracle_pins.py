"""Pins of the CPU FP64 oracle against what the paper and mathematics fix.

Each test cites the passage it checks.  None compares the oracle with a
retyped copy of its own formula: the references are closed forms, library
routines (Cholesky, LU solve), an independently written brute force, the
paper's printed Table 1, and invariants.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import synth
from oracle import brute

HERE = os.path.dirname(os.path.abspath(__file__))


# ------------------------------------------------------------------ Eq. (2)
def test_phi_closed_form_values():
    """Eq. (2): phi(0) = 1, phi(1/2) = (1/2)^4 * 3 = 3/16, phi(1) = 0, zero beyond."""
    assert oracle.phi(0.0) == 1.0
    assert oracle.phi(0.5) == 0.1875
    assert oracle.phi(1.0) == 0.0
    for eta in (1.0 + 1e-12, 1.5, 2.0, 1e6):
        assert oracle.phi(eta) == 0.0


def test_phi_expanded_polynomial_and_derivatives():
    """Eq. (2) expands to 1 - 10 e^2 + 20 e^3 - 15 e^4 + 4 e^5 on [0, 1]; its
    derivative -20 e (1 - e)^3 vanishes at 0 and 1, and phi''(1) = 0 (C2)."""
    for eta in np.linspace(0.0, 1.0, 41):
        poly = 1 - 10 * eta ** 2 + 20 * eta ** 3 - 15 * eta ** 4 + 4 * eta ** 5
        assert abs(oracle.phi(eta) - poly) < 1e-13
    h = 1e-6
    for eta in (0.1, 0.3, 0.55, 0.8, 0.95):
        fd = (oracle.phi(eta + h) - oracle.phi(eta - h)) / (2 * h)
        assert abs(fd - (-20 * eta * (1 - eta) ** 3)) < 1e-8
    h2 = 1e-4
    d2_right = (oracle.phi(1 + h2) - 2 * oracle.phi(1.0) + oracle.phi(1 - h2)) / h2 ** 2
    assert abs(d2_right) < 1e-5
    assert abs((oracle.phi(h) - oracle.phi(0.0)) / h) < 1e-4


def test_phi_matrix_is_positive_definite():
    """Section 2: with Eq. (2) the RBF matrix Phi of Eq. (5) is SPD."""
    p = synth.tiny_problem(nb=40, seed=3)
    Phi = brute.rbf_matrix(p.xyz, p.xyz, p.radius)
    assert np.allclose(Phi, Phi.T)
    assert np.linalg.eigvalsh(Phi).min() > 0


# ------------------------------------------------------------------ splitmix64 / partition
def test_splitmix64_published_vector():
    """splitmix64 seeded with 0 yields the published first outputs."""
    out = oracle.splitmix64(0, 3)
    assert [int(x) for x in out] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


@pytest.mark.parametrize("nb,m", [(2000, 10), (80000, 107), (17, 5), (10, 10), (9, 1)])
def test_partition_conditions(nb, m):
    """Section 3: G = union of G_0..G_{m-1}, pairwise disjoint, |card(G_i) - card(G_j)| <= 1."""
    g = oracle.partition(nb, m, 12345)
    assert g.shape == (nb,) and g.min() >= 0 and g.max() < m
    counts = np.bincount(g, minlength=m)
    assert counts.sum() == nb
    assert counts.max() - counts.min() <= 1
    assert np.array_equal(g, oracle.partition(nb, m, 12345))
    if m > 1 and nb > 2 * m:
        assert not np.array_equal(g, oracle.partition(nb, m, 12346))


def test_partition_is_a_uniform_shuffle():
    """Section 3 asks for a stochastic division: with m = nb = 4 every one of the
    24 orders is equally likely (catches e.g. the cyclic-only Sattolo variant)."""
    counts = {}
    n = 24000
    for s in range(n):
        key = tuple(oracle.partition(4, 4, s * 0x9E3779B97F4A7C15 + 1))
        counts[key] = counts.get(key, 0) + 1
    assert len(counts) == 24
    exp = n / 24
    chi2 = sum((c - exp) ** 2 / exp for c in counts.values())
    assert chi2 < 60.0  # 23 degrees of freedom; p ~ 5e-5


def test_partition_node_marginal_is_uniform():
    """Each node lands in each group with probability 1/m."""
    nb, m, reps = 12, 3, 6000
    hits = np.zeros((nb, m))
    for s in range(reps):
        g = oracle.partition(nb, m, 1000003 * s + 7)
        hits[np.arange(nb), g] += 1
    assert np.abs(hits / reps - 1.0 / m).max() < 0.04


# ------------------------------------------------------------------ starting nodes
def test_initial_nodes_rule_brute_force():
    """Algorithm 1 starts from 3 nodes; the farthest-point reading, checked
    against an independent NumPy evaluation, ties to the lowest index."""
    for seed in range(5):
        p = synth.tiny_problem(nb=50, seed=seed)
        assert list(oracle.initial_nodes(p.xyz, p.disp)) == brute.start_nodes(p.xyz, p.disp)
    xyz = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, 0, 1.0]])
    disp = np.array([[0.1, 0, 0]] * 5)
    n = oracle.initial_nodes(xyz, disp)
    assert n[0] == 0
    assert n[1] == 1      # nodes 1..4 all at distance 1 from node 0 -> lowest index
    assert n[2] == 2      # node 2 is 2 away from node 1, farther than 3 and 4


# ------------------------------------------------------------------ Eq. (1) / Eq. (6)
def test_interpolate_matches_dense_matrix_product():
    """Eq. (6) is the product of the RBF matrix with W (NumPy matmul)."""
    gen = np.random.default_rng(0)
    S = gen.uniform(-1, 1, (37, 3))
    T = gen.uniform(-1.5, 1.5, (101, 3))
    W = gen.standard_normal((37, 5))
    out = oracle.interpolate(S, W, 0.9, T)
    ref = brute.rbf_matrix(T, S, 0.9) @ W
    assert np.abs(out - ref).max() < 1e-13 * max(1.0, np.abs(ref).max())


def test_interpolate_compact_support_exact_zero():
    """Eq. (2) is exactly zero for eta > 1: targets farther than R from every support get 0."""
    S = np.array([[0, 0, 0], [0.5, 0, 0]], float)
    W = np.ones((2, 3))
    T = np.array([[3.0, 0, 0], [0, 2.1, 0], [1.5 + 1e-9, 0, 0]])
    assert np.all(oracle.interpolate(S, W, 1.0, T) == 0.0)


def test_interpolate_translation_scale_invariance_and_linearity():
    """Eq. (1) depends on |r - r_i| / R only, and is linear in W."""
    gen = np.random.default_rng(1)
    S = gen.uniform(-1, 1, (20, 3))
    T = gen.uniform(-1, 1, (30, 3))
    W = gen.standard_normal((20, 3))
    a = oracle.interpolate(S, W, 1.3, T)
    b = oracle.interpolate(S * 2.0 + 5.0, W, 2.6, T * 2.0 + 5.0)
    assert np.abs(a - b).max() < 1e-12
    W2 = gen.standard_normal((20, 3))
    c = oracle.interpolate(S, 2.0 * W - 3.0 * W2, 1.3, T)
    d = 2.0 * a - 3.0 * oracle.interpolate(S, W2, 1.3, T)
    assert np.abs(c - d).max() < 1e-12


# ------------------------------------------------------------------ RC factor
def test_rc_factor_equals_cholesky_at_every_step():
    """Section 1, RC scheme: the incrementally grown L is the Cholesky factor
    of Phi_S at every step (numpy.linalg.cholesky), and W solves Phi_S W = Delta_S
    (numpy.linalg.solve)."""
    p = synth.tiny_problem(nb=30, seed=11, radius=1.2)
    rc = oracle.RC(3)
    order = np.random.default_rng(2).permutation(30)
    for t, n in enumerate(order):
        b = brute.rbf_matrix(p.xyz[order[:t]], p.xyz[[n]], p.radius)[:, 0]
        assert rc.append(b, p.disp[n]) == oracle.ORC_OK
        S = order[: t + 1]
        Phi = brute.rbf_matrix(p.xyz[S], p.xyz[S], p.radius)
        L = rc.factor()
        Lref = np.linalg.cholesky(Phi)
        assert np.abs(L - Lref).max() < 1e-10
        W = rc.weights()
        Wref = np.linalg.solve(Phi, p.disp[S])
        assert np.abs(W - Wref).max() < 1e-8 * max(1.0, np.abs(Wref).max())
        # interpolation condition at the supports (Eq. 3 restricted to S)
        assert np.abs(Phi @ W - p.disp[S]).max() < 1e-10


def test_rc_detects_singular_append():
    """Phi_S is SPD only for distinct nodes: a duplicate makes phi0 - l.l = 0."""
    rc = oracle.RC(3)
    assert rc.append([], [0.1, 0, 0]) == oracle.ORC_OK
    assert rc.append([1.0], [0.1, 0, 0]) == oracle.ORC_E_SINGULAR
    assert rc.n == 1


# ------------------------------------------------------------------ Algorithm 1
@pytest.mark.parametrize("nb", [8, 12, 16])
@pytest.mark.parametrize("mm", ["1", "2", "3", "nb"])
def test_select_matches_brute_force_tiny(nb, mm):
    """Algorithm 1 on tiny inputs against an independent NumPy brute force that
    re-solves Phi_S from scratch every iteration: identical sequence and log."""
    m = nb if mm == "nb" else int(mm)
    for seed, tol_rel in ((nb, 0.0), (nb + 100, 0.05)):
        p = synth.tiny_problem(nb=nb, seed=seed, m=m)
        tol = tol_rel * p.max_disp
        g = oracle.partition(p.nb, m, p.seed)
        r = oracle.select(p.xyz, p.disp, p.radius, m, tol, seed=p.seed)
        S, log = brute.gcb_brute(p.xyz, p.disp, p.radius, g, m, tol)
        assert list(r.S) == S
        assert r.iterations == len(log)
        assert list(r.log_group) == [e[1] for e in log]
        assert list(r.log_node) == [e[2] for e in log]
        assert list(r.log_appended.astype(bool)) == [e[4] for e in log]
        assert np.allclose(r.log_err, [e[3] for e in log], rtol=1e-9, atol=1e-13)


def test_full_system_special_case():
    """E* = 0, Nc_max = Nb: every node becomes a support, and the interpolant
    satisfies Eq. (3) at all boundary nodes; W solves Eqs. (4)-(5) over all of G."""
    p = synth.tiny_problem(nb=15, seed=5, m=4)
    r = oracle.select(p.xyz, p.disp, p.radius, p.m, 0.0, seed=p.seed)
    assert r.status == oracle.ORC_OK
    assert sorted(r.S.tolist()) == list(range(15))
    F = oracle.interpolate(p.xyz[r.S], r.W, p.radius, p.xyz)
    assert np.abs(F - p.disp).max() < 1e-12
    Wfull = np.linalg.solve(brute.rbf_matrix(p.xyz, p.xyz, p.radius), p.disp)
    assert np.abs(r.W - Wfull[r.S]).max() < 1e-9 * np.abs(Wfull).max()


def test_m1_is_the_traditional_greedy():
    """Section 4.1: the traditional greedy is GCB with m = 1; the selected index
    sequence equals that of an independent Rendall-Allen implementation."""
    p = synth.config_small_ellipsoid(with_volume=False)
    r = oracle.select(p.xyz, p.disp, p.radius, 1, p.tol_abs, seed=p.seed)
    St = brute.traditional_greedy(p.xyz, p.disp, p.radius, p.tol_abs)
    assert r.status == oracle.ORC_OK
    assert list(r.S) == St


def test_replay_invariants_small_ellipsoid():
    """Algorithm 1: iteration k evaluates G_{k mod m}; every append is that
    group's maximum-error node (checked by brute force at sampled iterations);
    the run ends after m quiet iterations; the all-node FP64 max <= E*."""
    p = synth.config_small_ellipsoid(with_volume=False)
    r = oracle.select(p.xyz, p.disp, p.radius, p.m, p.tol_abs, seed=p.seed)
    assert r.status == oracle.ORC_OK and r.converged
    k = np.arange(3, 3 + r.iterations)
    assert np.array_equal(r.log_group, k % p.m)
    assert not r.log_appended[-p.m:].any()
    assert r.log_appended[:-p.m].sum() == r.nc - 3
    assert r.final_max_err <= p.tol_abs
    g = oracle.partition(p.nb, p.m, p.seed)
    S = list(r.S[:3])
    checked = 0
    for it in range(r.iterations):
        if it % 37 == 0:
            cand = [j for j in np.flatnonzero(g == r.log_group[it]) if j not in S]
            W = brute.solve_weights(p.xyz[S], p.disp[S], p.radius)
            e = np.sqrt(((brute.rbf_matrix(p.xyz[cand], p.xyz[S], p.radius) @ W - p.disp[cand]) ** 2).sum(1))
            assert cand[int(np.argmax(e))] == r.log_node[it]
            assert abs(e.max() - r.log_err[it]) < 1e-9 * p.max_disp
            checked += 1
        if r.log_appended[it]:
            S.append(int(r.log_node[it]))
    assert checked > 5 and S == list(r.S)
    # Eq. 3 on S: the interpolant reproduces the prescribed displacement at every support
    F = oracle.interpolate(p.xyz[r.S], r.W, p.radius, p.xyz[r.S])
    assert np.abs(F - p.disp[r.S]).max() < 1e-9 * p.max_disp


def test_work_counters_match_the_log():
    """Pair-evaluation counters equal the closed-form sums over the recorded run."""
    p = synth.config_small_ellipsoid(with_volume=False)
    r = oracle.select(p.xyz, p.disp, p.radius, p.m, p.tol_abs, seed=p.seed)
    g = oracle.partition(p.nb, p.m, p.seed)
    sizes = np.bincount(g, minlength=p.m)
    inS = np.zeros(p.nb, bool)
    inS[r.S[:3]] = True
    nS, pg, pa = 3, 0, 0
    for it in range(r.iterations):
        grp = r.log_group[it]
        pg += (sizes[grp] - inS[g == grp].sum()) * nS
        if r.log_appended[it]:
            pa += nS
            inS[r.log_node[it]] = True
            nS += 1
    assert r.pairs_group == pg and r.pairs_append == pa and r.pairs_cert == p.nb * r.nc


def test_cap_gives_not_converged():
    """Nc^max bounds |S| (Algorithm 1 input); hitting it with E > E* is reported."""
    p = synth.config_small_ellipsoid(with_volume=False)
    r = oracle.select(p.xyz, p.disp, p.radius, p.m, p.tol_abs, nc_max=50, seed=p.seed)
    assert r.status == oracle.ORC_NOT_CONVERGED and r.nc == 50 and not r.converged


def test_invalid_inputs_rejected():
    p = synth.tiny_problem(nb=10)
    assert oracle.select(p.xyz, p.disp, -1.0, 2, 0.0).status == oracle.ORC_E_INVALID
    assert oracle.select(p.xyz, p.disp, 1.0, 11, 0.0).status == oracle.ORC_E_INVALID
    bad = p.xyz.copy()
    bad[3, 1] = np.nan
    assert oracle.select(bad, p.disp, 1.0, 2, 0.0).status == oracle.ORC_E_INVALID


def test_validate_accepts_own_run_and_flags_planted_deviation():
    """Follow-mode replay accepts the oracle's own sequence (tau = 0) and
    rejects a sequence whose appended node is not the group maximum."""
    p = synth.config_small_ellipsoid(with_volume=False)
    r = oracle.select(p.xyz, p.disp, p.radius, p.m, p.tol_abs, seed=p.seed)
    bad, reason, gap = oracle.validate(p.xyz, p.disp, p.radius, p.m, p.tol_abs, r.S, r.log_group, r.log_node,
                                       r.log_appended, 0.0, seed=p.seed)
    assert bad == -1 and gap == 0.0
    g = oracle.partition(p.nb, p.m, p.seed)
    node = r.log_node.copy()
    it = 40
    assert r.log_appended[it]
    others = [j for j in np.flatnonzero(g == r.log_group[it]) if j != node[it] and j not in r.S[:40]]
    node[it] = others[0]
    bad, reason, gap = oracle.validate(p.xyz, p.disp, p.radius, p.m, p.tol_abs, r.S, r.log_group, node,
                                       r.log_appended, 1e-12, seed=p.seed)
    assert bad == it and reason in (3, 4)
    grp = r.log_group.copy()
    grp[5] = (grp[5] + 1) % p.m
    bad, reason, _ = oracle.validate(p.xyz, p.disp, p.radius, p.m, p.tol_abs, r.S, grp, r.log_node,
                                     r.log_appended, 0.0, seed=p.seed)
    assert bad == 5 and reason == 1


def test_validate_rejects_false_skip():
    """Algorithm 1 appends whenever the group maximum exceeds E* and |S| <
    Nc^max: a replayed sequence that marks such an iteration as skipped is
    rejected there (reason 4), even with a generous tau below the margin."""
    p = synth.config_small_ellipsoid(with_volume=False)
    r = oracle.select(p.xyz, p.disp, p.radius, p.m, p.tol_abs, seed=p.seed)
    app = r.log_appended.copy()
    # an append whose error clears E* by a wide margin (the starting iterations have E >> E*)
    it = next(i for i in range(len(app)) if app[i] and r.log_err[i] > 10.0 * p.tol_abs)
    app[it] = 0
    tau = 1e-3 * p.tol_abs
    bad, reason, _ = oracle.validate(p.xyz, p.disp, p.radius, p.m, p.tol_abs, r.S, r.log_group, r.log_node,
                                     app, tau, seed=p.seed)
    assert bad == it and reason == 4
    # the same skip late in the run, where the error is only a few E*
    late = [i for i in range(len(app)) if r.log_appended[i] and r.log_err[i] > p.tol_abs + 10 * tau]
    it2 = late[-1]
    app = r.log_appended.copy()
    app[it2] = 0
    bad, reason, _ = oracle.validate(p.xyz, p.disp, p.radius, p.m, p.tol_abs, r.S, r.log_group, r.log_node,
                                     app, tau, seed=p.seed)
    assert bad == it2 and reason == 4


def test_validate_rejects_truncated_fresh_run():
    """A fresh run ends only after m consecutive iterations without an append
    (every group checked with one W) or at the cap: the oracle's own sequence
    cut before its last quiet iteration is rejected at its end (reason 6),
    and so is one cut right after an append; the whole sequence passes."""
    p = synth.config_small_ellipsoid(with_volume=False)
    r = oracle.select(p.xyz, p.disp, p.radius, p.m, p.tol_abs, seed=p.seed)
    n = len(r.log_group)
    assert not r.log_appended[n - p.m:].any() and r.log_appended[n - p.m - 1]
    for cut in (n - 1, n - p.m):
        bad, reason, _ = oracle.validate(p.xyz, p.disp, p.radius, p.m, p.tol_abs, r.S, r.log_group[:cut],
                                         r.log_node[:cut], r.log_appended[:cut], 0.0, seed=p.seed)
        assert bad == cut and reason == 6, (cut, bad, reason)
    bad, reason, _ = oracle.validate(p.xyz, p.disp, p.radius, p.m, p.tol_abs, r.S, r.log_group, r.log_node,
                                     r.log_appended, 0.0, seed=p.seed)
    assert bad == -1 and reason == 0
    # at the cap the run may end right after an append
    rc = oracle.select(p.xyz, p.disp, p.radius, p.m, p.tol_abs, nc_max=50, seed=p.seed)
    nz = len(rc.log_group)
    bad, reason, _ = oracle.validate(p.xyz, p.disp, p.radius, p.m, p.tol_abs, rc.S, rc.log_group, rc.log_node,
                                     rc.log_appended, 0.0, nc_max=50, seed=p.seed)
    assert bad == -1, (bad, reason)
    last_app = int(np.flatnonzero(rc.log_appended)[-1])
    cut = last_app   # one append short of the cap
    bad, reason, _ = oracle.validate(p.xyz, p.disp, p.radius, p.m, p.tol_abs, rc.S, rc.log_group[:cut],
                                     rc.log_node[:cut], rc.log_appended[:cut], 0.0, nc_max=50, seed=p.seed)
    assert bad == cut and reason == 6 and nz > cut


# ------------------------------------------------------------------ Table 1
def test_table1_cost_model():
    """Table 1 (Nv = 4e6, Nb = 8e4, Nc = 2000): 5.3e9, 4.8e11, 8.0e10 and the
    printed percentages (to the table's rounding, with 'others' = 0.29 %);
    Section 3: the GCB error cost equals the RC cost when m = 9 Nb / (4 Nc)."""
    gold = json.load(open(os.path.join(HERE, "golden", "table1_cost_model.json")))
    pr = gold["problem"]
    c = oracle.cost_model(pr["nc"], pr["nb"], pr["nv"])
    for k, v in gold["amounts"].items():
        assert abs(c[k] - v) / v < 0.01
    total = sum(c.values()) / (1.0 - gold["percent"]["others"] / 100.0)
    for k in ("solve", "errors", "volume"):
        assert abs(100.0 * c[k] / total - gold["percent"][k]) <= 0.011
    nc, nb = 1234.0, 56789.0
    m = 9 * nb / (4 * nc)
    c2 = oracle.cost_model(nc, nb, 0, m)
    assert math.isclose(c2["errors"], c2["solve"], rel_tol=1e-12)


def test_solve_on_support_matches_library_solve():
    """Eqs. 4-5 restricted to S with several right-hand sides: RC forward/back
    substitution equals numpy.linalg.solve for every column."""
    p = synth.tiny_problem(nb=40, seed=9, radius=1.3)
    S = np.array([3, 17, 8, 31, 0, 22, 39, 11])
    D = np.random.default_rng(5).standard_normal((40, 7))
    W = oracle.solve_on_support(p.xyz, S, p.radius, D)
    Wr = np.linalg.solve(brute.rbf_matrix(p.xyz[S], p.xyz[S], p.radius), D[S])
    assert np.abs(W - Wr).max() < 1e-10 * np.abs(Wr).max()


def test_warm_start_from_the_starting_nodes_is_algorithm1():
    """A warm start from the three starting nodes fails the certificate and then
    runs the loop from k = 3: exactly Algorithm 1."""
    p = synth.config_small_ellipsoid(with_volume=False)
    r = oracle.select(p.xyz, p.disp, p.radius, p.m, p.tol_abs, seed=p.seed)
    w = oracle.select(p.xyz, p.disp, p.radius, p.m, p.tol_abs, seed=p.seed, warm_S=r.S[:3])
    assert np.array_equal(w.S, r.S) and np.array_equal(w.W, r.W)
    assert w.iterations == r.iterations
    assert np.array_equal(w.log_node, r.log_node) and np.array_equal(w.log_group, r.log_group)


@pytest.mark.parametrize("nb,m", [(13, 1), (16, 2), (40, 3), (70, 3)])
def test_warm_start_brute_force(nb, m):
    """Kept support set, new displacement field: brute force (dense solves) from the same set."""
    p = synth.tiny_problem(nb=nb, seed=nb + 5, m=m)
    tol = 0.02 * p.max_disp
    r = oracle.select(p.xyz, p.disp, p.radius, m, tol, seed=p.seed)
    g = oracle.partition(p.nb, m, p.seed)
    rot = np.array([[0.0, 1.0, 0.0], [0.0, 0.0, 1.0], [1.0, 0.0, 0.0]])
    for disp2, expect_iters in ((p.disp, False), (1.7 * p.disp @ rot + 0.01, True)):
        w = oracle.select(p.xyz, disp2, p.radius, m, tol, seed=p.seed, warm_S=r.S)
        Sb, logb = brute.gcb_brute(p.xyz, disp2, p.radius, g, m, tol, warm=r.S)
        assert list(w.S) == Sb
        assert w.iterations == len(logb)
        assert [e[2] for e in logb] == list(w.log_node)
        assert [e[1] for e in logb] == list(w.log_group)
        if not expect_iters:
            assert w.iterations == 0 and w.converged
        # the weights interpolate the new field at every support node
        F = oracle.interpolate(p.xyz[w.S], w.W, p.radius, p.xyz[w.S])
        assert np.abs(F - disp2[w.S]).max() <= 1e-9 * np.abs(disp2).max()


def test_warm_start_validation_and_replay():
    p = synth.tiny_problem(nb=40, seed=3, m=3)
    tol = 0.02 * p.max_disp
    r = oracle.select(p.xyz, p.disp, p.radius, 3, tol, seed=p.seed)
    bad = oracle.select(p.xyz, p.disp, p.radius, 3, tol, seed=p.seed, warm_S=[r.S[0], r.S[1], r.S[0]])
    assert bad.status == oracle.ORC_E_INVALID
    d2 = 1.5 * p.disp[:, ::-1].copy()
    w = oracle.select(p.xyz, d2, p.radius, 3, tol, seed=p.seed, warm_S=r.S)
    assert w.iterations > 0
    ok = oracle.validate(p.xyz, d2, p.radius, 3, tol, r.S, w.log_group, w.log_node, w.log_appended, 1e-12,
                         seed=p.seed, warm_S=r.S)
    assert ok[0] == -1
    # claiming that the kept set already meets E* is rejected (reason 6)
    none = oracle.validate(p.xyz, d2, p.radius, 3, tol, r.S, [], [], [], 1e-12, seed=p.seed, warm_S=r.S)
    assert none[0] == 0 and none[1] == 6


@pytest.mark.parametrize("n", [3, 17, 120])
def test_inverse_factor_against_library_cholesky(n):
    """M = L^-1: M L = I and L L^T = Phi_S, checked with numpy's Cholesky and inverse
    (an independent factorisation, not the oracle's recurrence)."""
    p = synth.config_small_ellipsoid(with_volume=False)
    r = oracle.select(p.xyz, p.disp, p.radius, p.m, p.tol_abs, seed=p.seed)
    S = r.S[:n]
    M = oracle.inverse_factor(p.xyz, S, p.radius)
    Phi = brute.rbf_matrix(p.xyz[S], p.xyz[S], p.radius)
    L = np.linalg.cholesky(Phi)
    assert np.allclose(np.triu(M, 1), 0.0)
    assert np.abs(M @ L - np.eye(n)).max() <= 1e-10
    Minv = np.linalg.inv(L)
    assert np.abs(M - Minv).max() <= 1e-9 * np.abs(Minv).max()
    # the weights M^T M d equal the oracle's RC solve on S
    W = M.T @ (M @ p.disp[S])
    assert np.abs(W - oracle.solve_on_support(p.xyz, S, p.radius, p.disp)).max() <= 1e-8 * np.abs(W).max()


def test_inverse_factor_singular():
    p = synth.tiny_problem(nb=12, seed=1)
    xyz = np.concatenate([p.xyz, p.xyz[:1]])
    with pytest.raises(RuntimeError):
        oracle.inverse_factor(xyz, [0, 3, 12], p.radius)


def test_monitor_is_passive_and_agrees_with_the_greedy():
    """The monitor never alters the selection; with m = 1 its all-node maximum after
    iteration i is the maximum error the next iteration finds (nodes in S have zero error)."""
    p = synth.config_small_ellipsoid(with_volume=False)
    r0 = oracle.select(p.xyz, p.disp, p.radius, 1, p.tol_abs, seed=p.seed)
    r1 = oracle.select(p.xyz, p.disp, p.radius, 1, p.tol_abs, seed=p.seed, monitor_every=1)
    assert np.array_equal(r0.S, r1.S) and np.array_equal(r0.log_err, r1.log_err)
    assert len(r1.mon_max) == r1.iterations
    assert np.array_equal(r1.mon_max[:-1], r1.log_err[1:])
    assert r1.mon_max[-1] == r1.final_max_err
    rm = oracle.select(p.xyz, p.disp, p.radius, p.m, p.tol_abs, seed=p.seed, monitor_every=p.m)
    assert len(rm.mon_max) == rm.iterations // p.m
    assert np.all(rm.mon_rms <= rm.mon_max)


def test_monitor_brute_force():
    """Monitor samples against dense solves on the support prefix of each sample."""
    p = synth.tiny_problem(nb=40, seed=11, m=3)
    tol = 0.01 * p.max_disp
    every = 2
    r = oracle.select(p.xyz, p.disp, p.radius, 3, tol, seed=p.seed, monitor_every=every)
    for s in range(len(r.mon_max)):
        it = (s + 1) * every                         # iterations done
        nS = 3 + int(r.log_appended[:it].sum())
        S = r.S[:nS]
        W = brute.solve_weights(p.xyz[S], p.disp[S], p.radius)
        F = brute.rbf_matrix(p.xyz, p.xyz[S], p.radius) @ W
        e = np.sqrt(((F - p.disp) ** 2).sum(axis=1))
        assert abs(r.mon_max[s] - e.max()) <= 1e-10 * p.max_disp
        assert abs(r.mon_rms[s] - np.sqrt((e ** 2).mean())) <= 1e-10 * p.max_disp
