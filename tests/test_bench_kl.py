"""The KL divergence of support-node distributions (Section 4.1, the KL equation)
used by the benchmark's fixed-Nc m-sweep, against a brute-force evaluation."""
import math

import numpy as np

import bench


def _brute(xyz, s1, s2):
    total = 0.0
    for i in range(len(xyz)):
        d1 = min(math.dist(xyz[i], xyz[j]) for j in s1)
        d2 = min(math.dist(xyz[i], xyz[j]) for j in s2)
        if d1 > 0.0 and d2 > 0.0:
            total += d1 * math.log(d1 / d2)
    return total


def test_kl_matches_brute_force_and_vanishes_for_equal_sets():
    g = np.random.default_rng(7)
    xyz = g.uniform(-1.0, 1.0, (60, 3))
    s1 = g.choice(60, 9, replace=False)
    s2 = g.choice(60, 9, replace=False)
    assert abs(bench.kl_divergence(xyz, s1, s2) - _brute(xyz, s1, s2)) < 1e-12
    assert abs(bench.kl_divergence(xyz, s2, s1) - _brute(xyz, s2, s1)) < 1e-12
    assert bench.kl_divergence(xyz, s1, s1[::-1]) == 0.0


def test_kl_sign_follows_the_nearest_distances():
    # nodes on a line; S1 spread evenly, S2 bunched at one end: every node farther from S2
    xyz = np.zeros((41, 3))
    xyz[:, 0] = np.linspace(0.0, 1.0, 41)
    s1 = np.arange(0, 41, 8)
    far = np.array([0, 1, 2, 3, 4])
    # with S2 bunched, d2 >= d1 at every kept node, so every kept term is <= 0 (the sum is not normalised)
    assert bench.kl_divergence(xyz, s1, far) < 0.0
    # and swapping the roles gives a positive sum (most nodes are far from the bunched set)
    assert bench.kl_divergence(xyz, far, s1) > 0.0
