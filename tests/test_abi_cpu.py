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


@pytest.mark.parametrize("nb,m,seed", [(2000, 10, 1), (80000, 107, 2), (300000, 399, 3), (3, 1, 0), (17, 17, 9),
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


def test_null_and_invalid_arguments_of_the_batch_server_and_factor_calls():
    """Argument checks that return before any device work (no GPU needed)."""
    L = gcb.lib()
    assert L.gcb_batch_create(None, 0, None) == gcb.GCB_E_INVALID
    assert L.gcb_batch_step(None, None, 0, 1, None) == gcb.GCB_E_INVALID
    assert L.gcb_batch_begin(None, None) == gcb.GCB_E_INVALID
    assert L.gcb_batch_end(None, None, None) == gcb.GCB_E_INVALID
    assert L.gcb_select_batch(None, None, 0, None) == gcb.GCB_E_INVALID
    assert L.gcb_deform_batch(None, None, 0, None, None, 1, None, 1) == gcb.GCB_E_INVALID
    assert L.gcb_batch_set_layout(None, 0, 0, 1) == gcb.GCB_E_INVALID
    L.gcb_batch_destroy(None)
    h = C.c_void_p()
    assert L.gcb_server_create(None, 0, None, 1 << 30, 4, 3) == gcb.GCB_E_INVALID
    assert L.gcb_server_create(C.byref(h), 0, None, 1 << 30, 0, 3) == gcb.GCB_E_INVALID     # no slot
    assert L.gcb_server_create(C.byref(h), 0, None, 1 << 30, 65, 3) == gcb.GCB_E_INVALID    # > 64 slots
    assert L.gcb_server_create(C.byref(h), 0, None, 1 << 30, 4, 8) == gcb.GCB_E_INVALID     # unknown flag
    assert L.gcb_server_submit(None, None, None) == gcb.GCB_E_INVALID
    assert L.gcb_server_progress(None, 1, None) == gcb.GCB_E_INVALID
    assert L.gcb_server_result(None, 1, None) == gcb.GCB_E_INVALID
    assert L.gcb_server_memory(None, None, None) == gcb.GCB_E_INVALID
    L.gcb_server_destroy(None)
    assert L.gcb_server_clock() > 0.0
    assert L.gcb_set_support(None, None, 0, 0, None) == gcb.GCB_E_INVALID
    assert L.gcb_refactor(None, None, None) == gcb.GCB_E_INVALID
    assert L.gcb_get_factor(None, None, 0) == gcb.GCB_E_INVALID
    assert L.gcb_get_monitor(None, None, None, None, 0) == gcb.GCB_E_INVALID


def test_struct_layouts_match_the_header(tmp_path):
    """The binding's ctypes layouts equal the C compiler's for every ABI struct."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    src = tmp_path / "sizes.c"
    fields = {"gcb_params": gcb.Params, "gcb_select_info": gcb.SelectInfo, "gcb_request": gcb.Request,
              "gcb_result": gcb.Result, "gcb_record": gcb.Record}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "gcb.h"', "int main(void) {"]
    for cname, cls in fields.items():
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'printf("{cname}.{fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0; }")
    src.write_text("\n".join(lines))
    exe = tmp_path / "sizes"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = dict(l.rsplit(" ", 1) for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                          check=True).stdout.splitlines())
    for cname, cls in fields.items():
        assert int(out[cname]) == C.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert int(out[f"{cname}.{fname}"]) == getattr(cls, fname).offset, (cname, fname)
