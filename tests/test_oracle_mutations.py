"""The oracle's pins catch plausible mistakes in its decision rules.

Each case copies the oracle's source, plants one mistake (a textual edit of one
rule), compiles the copy and runs the pin that should catch it in a child
pytest process that loads the copy (ORACLE_LIBRARY).  The case passes when that
pin fails.  The mistakes are the ones a reader could plausibly make in the
aFSAI growth rule, its eps_g stop and outer loop (Section 3.1, Algorithm "aFSAI
Smoother Set-up"), the start of the SRQCG test-space iteration (Section 3.3),
the theta filter (Section 3.4) and the interpolation candidates (Section 3.5)."""
import os
import subprocess
import sys

import pytest

import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(ROOT, "oracle", "aspamg_oracle.c")

ASC = """static int cmp_qcand_asc(const void *a, const void *b) { return -cmp_qcand(a, b); }
"""

# (id, [(old, new), ...], pin selector in test_oracle_replays.py)
MUTATIONS = [
    ("growth_score_from_g_not_unit_last",
     [("double gp = R->g[d][k] / glast;", "double gp = R->g[d][k];")],
     "test_growth_steps_replay"),
    ("growth_candidates_adjacent_to_I_only",
     [("for (int p = 0; p <= nb; p++) {\n    int32_t K = p < nb ? R->nodes[p] : I;",
       "for (int p = nb; p <= nb; p++) {\n    int32_t K = p < nb ? R->nodes[p] : I;")],
     "test_growth_steps_replay"),
    ("growth_keeps_smallest_scores",
     [("static int fsai_grow_row(", ASC + "static int fsai_grow_row("),
      ("qsort(qc, nq, sizeof(qcand), cmp_qcand);\n  int add", "qsort(qc, nq, sizeof(qcand), cmp_qcand_asc);\n  int add")],
     "test_growth_steps_replay"),
    ("eps_stop_reversed",
     [("if (dec <= thr) break;", "if (dec >= thr) break;")],
     "test_eps_stop_fires_exactly_at_threshold"),
    ("eps_stop_strict",
     [("if (dec <= thr) break;", "if (dec < thr) break;")],
     "test_eps_stop_fires_exactly_at_threshold"),
    ("eps_stop_unquantised",
     [("double dec = qz(psi_prev - R->psi_sum), thr = qz(p->eps_g * psi_prev);",
       "double dec = psi_prev - R->psi_sum, thr = p->eps_g * psi_prev;")],
     "test_eps_stop_fires_exactly_at_threshold"),
    ("outer_loop_omega_test_reversed",
     [("if (!(qz(L->omega_q) < qz(p->omega_bar))) break;", "if (qz(L->omega_q) < qz(p->omega_bar)) break;")],
     "test_outer_loop_replay"),
    ("outer_loop_without_density_stop",
     [("if (!(L->G.nnzb < A->nnzb)) break;", "")],
     "test_outer_loop_replay"),
    ("theta_filter_keeps_weakest",
     [("static int coarsen(", ASC + "static int coarsen("),
      ("qsort(qc, nq, sizeof(qcand), cmp_qcand);\n    int kk", "qsort(qc, nq, sizeof(qcand), cmp_qcand_asc);\n    int kk")],
     "test_theta_filter_replay"),
    ("theta_filter_intersection_not_union",
     [("if (dup && j < i) continue;", "if (!dup || j < i) continue;")],
     "test_theta_filter_replay"),
    ("candidates_depth_one_short",
     [("if (dist[u] >= d_p) continue;", "if (dist[u] >= d_p - 1) continue;")],
     "test_interpolation_candidates_replay"),
    ("candidates_depth_one_long",
     [("if (dist[u] >= d_p) continue;", "if (dist[u] > d_p) continue;")],
     "test_interpolation_candidates_replay"),
    ("srqcg_start_not_in_the_variable_of_S",
     [("    gt_solve(G, x);\n    apply_gagt", "    apply_gagt")],
     "test_oracle_srqcg.py::test_srqcg_keeps_the_rigid_body_modes_of_a_free_body"),
]


@pytest.mark.parametrize("name,edits,pin", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pin_catches_planted_mistake(name, edits, pin, tmp_path, oracle_lib):
    src = open(SRC).read()
    for old, new in edits:
        n = src.count(old)
        assert n >= 1, f"{name}: the text to mutate is gone from the oracle: {old!r}"
        src = src.replace(old, new)
    path = tmp_path / "mutant.c"
    path.write_text(src)
    lib = O.compile_source(str(path), str(tmp_path / "libmutant.so"))
    env = dict(os.environ, ORACLE_LIBRARY=lib)
    fname, _, sel = pin.rpartition("::")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(HERE, fname or "test_oracle_replays.py"), "-k", sel],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 1, f"{name}: pin {pin} did not fail (rc {r.returncode})\n{r.stdout[-2000:]}"
