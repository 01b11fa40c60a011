"""Each pin must catch a plausible mistake: a copy of the oracle source with
one planted mistake (a dropped term, a wrong sign, a wrong index or bound) is
compiled on the CPU, and at least one pin must fail against it.  The planted
copies live in a temporary directory; the real oracle is never modified."""
import os
import subprocess

import pytest

import oracle
from tests import test_oracle_block as blk
from tests import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "gcb_oracle.c")

MUTANTS = [
    ("phi-sign", "return a * a * a * a * (4.0 * eta + 1.0);", "return a * a * a * a * (4.0 * eta - 1.0);",
     [pins.test_phi_closed_form_values]),
    ("phi-dropped-factor", "return a * a * a * a * (4.0 * eta + 1.0);", "return a * a * a * (4.0 * eta + 1.0);",
     [pins.test_phi_closed_form_values]),
    ("phi-support-bound", "if (eta > 1.0) return 0.0;", "if (eta > 2.0) return 0.0;",
     [pins.test_phi_closed_form_values]),
    ("splitmix-shift", "z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;", "z = (z ^ (z >> 31)) * 0xBF58476D1CE4E5B9ull;",
     [pins.test_splitmix64_published_vector]),
    ("shuffle-sattolo", "% (uint64_t)(i + 1);", "% (uint64_t)(i);", [pins.test_partition_is_a_uniform_shuffle]),
    ("distance-dropped-z", "return sqrt(dx * dx + dy * dy + dz * dz);", "return sqrt(dx * dx + dy * dy);",
     [pins.test_interpolate_matches_dense_matrix_product]),
    ("rc-forward-sign", "for (int64_t j = 0; j < i; ++j) acc -= Li[j] * rc->l[j];",
     "for (int64_t j = 0; j < i; ++j) acc += Li[j] * rc->l[j];", [pins.test_rc_factor_equals_cholesky_at_every_step]),
    ("rc-schur-sign", "double s = phi0 - ll;", "double s = phi0 + ll;",
     [pins.test_rc_factor_equals_cholesky_at_every_step]),
    ("rc-y-transposed", "acc -= rc->l[j] * rc->y[(size_t)j * (size_t)rc->K + (size_t)c];",
     "acc -= rc->l[j] * rc->y[(size_t)c * (size_t)rc->K + (size_t)j];",
     [pins.test_rc_factor_equals_cholesky_at_every_step]),
    ("backsub-sign", "w[(size_t)i * (size_t)K + (size_t)c] -= Lj[i] * w[(size_t)j * (size_t)K + (size_t)c];",
     "w[(size_t)i * (size_t)K + (size_t)c] += Lj[i] * w[(size_t)j * (size_t)K + (size_t)c];",
     [pins.test_rc_factor_equals_cholesky_at_every_step]),
    ("schedule-offset", "int32_t g = (int32_t)(k % p->m);\n        int64_t gsize",
     "int32_t g = (int32_t)((k + 1) % p->m);\n        int64_t gsize", [lambda: pins.test_select_matches_brute_force_tiny(12, "3")]),
    ("error-dropped-z", "st->e[t - lo] = sqrt(ex * ex + ey * ey + ez * ez);", "st->e[t - lo] = sqrt(ex * ex + ey * ey);",
     [lambda: pins.test_select_matches_brute_force_tiny(16, "2")]),
    ("stop-after-one-quiet", "if (quiet >= p->m) break;", "if (quiet >= 1) break;",
     [lambda: pins.test_select_matches_brute_force_tiny(12, "3")]),
    ("support-not-excluded", "if (st->in_S[j]) { st->e[t - lo] = -1.0; continue; }", "(void)0;",
     [lambda: pins.test_select_matches_brute_force_tiny(8, "2"), pins.test_full_system_special_case]),
    ("argmax-direction", "if (v > best || (v == best && j < arg)) { best = v; arg = j; }",
     "if (v < best || (v == best && j < arg)) { best = v; arg = j; }",
     [lambda: pins.test_select_matches_brute_force_tiny(12, "2")]),
    ("start-rule-min", "double v = a < b ? a : b;", "double v = a < b ? b : a;", [pins.test_initial_nodes_rule_brute_force]),
    ("block-rank-ascending", "if (x->e > y->e) return -1;\n    if (x->e < y->e) return 1;",
     "if (x->e > y->e) return 1;\n    if (x->e < y->e) return -1;",
     [lambda: blk.test_block_select_matches_brute_force_tiny(12, 2, 3, 0.0)]),
    ("block-count-uncapped", "int64_t q = over < p->per_iter ? over : p->per_iter;", "int64_t q = over;",
     [lambda: blk.test_block_select_matches_brute_force_tiny(12, 2, 2, 0.0)]),
    ("block-candidates-below-tolerance", "if (v < 0.0 || !(v > tol)) continue;", "if (v < 0.0) continue;",
     [lambda: blk.test_block_select_matches_brute_force_tiny(16, 2, 3, 0.05)]),
    ("validate-skip-check-dropped",
     "if (n >= 0 && E > p->tol_abs + tau && st.nS < p->nc_max) { bad = it; r = 4; break; }", "(void)0;",
     [pins.test_validate_rejects_false_skip]),
    ("validate-termination-check-dropped",
     "if (!(quiet == p->m || st.nS == p->nc_max)) { bad = n_iter; r = 6; }", "(void)0;",
     [pins.test_validate_rejects_truncated_fresh_run]),
]


@pytest.mark.parametrize("name,old,new,checks", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_is_caught(tmp_path, name, old, new, checks):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not unique"
    mutated = src.replace(old, new)
    csrc = tmp_path / "gcb_oracle.c"
    csrc.write_text(mutated)
    hdr = os.path.join(os.path.dirname(SRC), "gcb_oracle.h")
    (tmp_path / "gcb_oracle.h").write_text(open(hdr).read())
    so = tmp_path / "liboracle_mut.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-o", str(so),
                    str(csrc), "-lm"], check=True)
    caught = False
    with oracle.use_library(str(so)):
        for chk in checks:
            try:
                chk()
            except (AssertionError, ValueError, IndexError, np_linalg_error()):
                caught = True
                break
    assert caught, f"planted mistake {name} passed every pin"


def np_linalg_error():
    import numpy as np
    return np.linalg.LinAlgError
