"""Host-side checks of the C ABI library (no GPU needed): it loads, exports
every function include/gcb.h declares, and its host logic (the seeded
partition) equals the oracle's bit for bit."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle
import paper_2004_04817_amd as gcb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "gcb.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gcb_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert len(names) >= 15
    L = C.CDLL(gcb.LIB_PATH)
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(gcb.EXPORTS)


def test_version_string():
    assert "gfx950" in gcb.version()


@pytest.mark.parametrize("nb,m,seed", [(2000, 10, 1), (80000, 107, 2), (300000, 160, 3), (3, 1, 0), (17, 17, 9),
                                       (1001, 7, 0xFFFFFFFFFFFFFFFF)])
def test_partition_bit_exact_with_oracle(nb, m, seed):
    """Section 3 partition: identical group of every node for the same seed."""
    assert np.array_equal(gcb.partition(nb, m, seed), oracle.partition(nb, m, seed))


def test_partition_rejects_bad_arguments():
    L = gcb.lib()
    g = np.empty(4, np.int32)
    assert L.gcb_partition(4, 0, 1, g.ctypes.data) == gcb.GCB_E_INVALID
    assert L.gcb_partition(4, 5, 1, g.ctypes.data) == gcb.GCB_E_INVALID
    assert L.gcb_partition(0, 1, 1, g.ctypes.data) == gcb.GCB_E_INVALID
    assert L.gcb_partition(4, 2, 1, None) == gcb.GCB_E_INVALID


def test_null_context_calls_are_rejected():
    L = gcb.lib()
    assert L.gcb_select(None, None) == gcb.GCB_E_INVALID
    assert L.gcb_set_params(None, None) == gcb.GCB_E_INVALID
    assert L.gcb_deform(None, 0, None, 1, None, 1, 0) == gcb.GCB_E_INVALID
    L.gcb_destroy(None)
    assert L.gcb_create(None, 0, None) == gcb.GCB_E_INVALID


def test_header_documents_every_call():
    """Every declaration in include/gcb.h carries a comment (argument meaning,
    layout, ownership, errors) right above it."""
    lines = open(os.path.join(ROOT, "include", "gcb.h")).read().splitlines()
    for name in declared_functions():
        i = next(k for k, l in enumerate(lines) if re.search(rf"\b{name}\s*\(", l) and not l.strip().startswith("*"))
        above = "\n".join(lines[max(0, i - 3):i])
        assert "*/" in above or "/*" in above, name
