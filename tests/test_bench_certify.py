"""The bench's certification of a selection sequence by the oracle's follow-mode replay (CPU): the oracle's
own sequence is certified, and a sequence with one appended node replaced is rejected at that iteration."""
import os
import sys
from types import SimpleNamespace

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
import oracle  # noqa: E402
import synth  # noqa: E402


class _Log:
    """Stands in for a context: get_log() returns a recorded sequence."""

    def __init__(self, group, node, appended):
        self.log = SimpleNamespace(group=group, node=node, appended=appended)

    def get_log(self):
        return self.log


def test_oracle_sequence_is_certified_and_a_planted_change_is_not():
    p = synth.config_small_ellipsoid(with_volume=False)
    r = oracle.select(p.xyz, p.disp, p.radius, p.m, p.tol_abs, seed=p.seed)
    ok = bench.certify_sequence(_Log(r.log_group, r.log_node, r.log_appended), p, np.asarray(r.S))
    assert ok["certified"] and ok["first_bad_iteration"] == -1 and ok["iterations"] == len(r.log_group)
    # replace the node of the sixth append by another node: the replay must stop there
    k = int(np.nonzero(r.log_appended)[0][5])
    node = r.log_node.copy()
    node[k] = (node[k] + 1) % p.nb
    bad = bench.certify_sequence(_Log(r.log_group, node, r.log_appended), p, np.asarray(r.S))
    assert not bad["certified"] and bad["first_bad_iteration"] == k
