"""Planted-mistake check of the oracle's pins (CPU only).

Each mutant is a copy of oracle.c with one plausible mistake -- a reversed
tie-break, an off-by-one staleness, a dropped visited mark, a dropped
dimension or neighbour, a short candidate list, a wrong sign, and in the PQ
navigation a dropped subspace, a reversed code tie-break, a shifted centroid,
an exact entry key or a missing re-rank, and in the beam-width schedule a
drain of all or of one in-flight node when nothing was selected and a
processing threshold of delay instead of delay*W -- compiled into a
temporary library.  The pin battery (tests/oracle_battery.py) must fail on
every mutant and pass on the unmodified source.
"""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(os.path.dirname(HERE), "oracle", "oracle.c")

MUTANTS = {
    "tie_break_reversed": ("if (a->id < b->id) return -1;\n  if (a->id > b->id) return 1;",
                           "if (a->id > b->id) return -1;\n  if (a->id < b->id) return 1;"),
    "staleness_off_by_one": ("if (f_len > J->delay * W) to_process = f_len - J->delay * W;",
                             "if (f_len > (J->delay + 1) * W) to_process = f_len - (J->delay + 1) * W;"),
    "neighbour_not_marked_visited": ("visited[x] = 1;\n        merged[m].dist",
                                     "merged[m].dist"),
    "entry_not_marked_visited": ("visited[J->entry] = 1;", ""),
    "last_dimension_dropped": ("for (int32_t j = 0; j < d; j++) {\n      int64_t t = (int64_t)a[j] - (int64_t)b[j];",
                               "for (int32_t j = 0; j < d - 1; j++) {\n      int64_t t = (int64_t)a[j] - (int64_t)b[j];"),
    "last_neighbour_dropped": ("for (int32_t j = 0; j < J->R; j++) {",
                               "for (int32_t j = 0; j + 1 < J->R; j++) {"),
    "list_one_short": ("nc = m < L ? m : L;", "nc = m < L - 1 ? m : (L > 1 ? L - 1 : 1);"),
    "f32_sign_error": ("double t = (double)a[j] - (double)b[j];\n      s += t * t;",
                       "double t = (double)a[j] + (double)b[j];\n      s += t * t;"),
    "pq_sum_skips_last_subspace": ("for (int32_t m = 0; m < M; m++) s += tab[",
                                   "for (int32_t m = 0; m + 1 < M; m++) s += tab["),
    "pq_code_ties_to_highest": ("if (c == 0 || s < bd) {", "if (c == 0 || s <= bd) {"),
    "pq_sub_distance_sign": ("const float t = x[j] - c[j];", "const float t = x[j] + c[j];"),
    "pq_table_shifted_centroid": (
        "orc_pq_sub(x + m * dsub, codebooks + ((int64_t)m * ORC_KSUB + c) * dsub, dsub);\n  free(x);\n  return 0;\n}\n\nstatic float",
        "orc_pq_sub(x + m * dsub, codebooks + ((int64_t)m * ORC_KSUB + (c ^ 1)) * dsub, dsub);\n  free(x);\n  return 0;\n}\n\nstatic float"),
    "pq_entry_keyed_exactly": ("cand[0].dist = orc_nav_dist(J, w, q, J->entry);",
                               "cand[0].dist = orc_dist(J->base, J->entry, J->d, J->dtype, q);"),
    "pq_answer_not_reranked": ("out = res;\n    nout = nres;", "out = cand;\n    nout = nc;"),
    "pq_encode_slices_leave_a_gap": ("orc_enc_job j = {base, n * t / threads, n * (t + 1) / threads,",
                                     "orc_enc_job j = {base, n * t / threads + (t > 0), n * (t + 1) / threads,"),
    "drain_all_in_flight_when_idle": ("if (nsel == 0 && to_process == 0) to_process = f_len < W ? f_len : W;",
                                      "if (nsel == 0 && to_process == 0) to_process = f_len;"),
    "drain_one_when_idle": ("if (nsel == 0 && to_process == 0) to_process = f_len < W ? f_len : W;",
                            "if (nsel == 0 && to_process == 0) to_process = 1;"),
    "threshold_ignores_beam": ("if (f_len > J->delay * W) to_process = f_len - J->delay * W;",
                               "if (f_len > J->delay) to_process = f_len - J->delay;"),
    "selects_second_unexpanded": ("if (cand[i].expanded) continue;",
                                  "if (cand[i].expanded || (nsel == 0 && i == 0 && nc > 1 && !cand[1].expanded)) continue;"),
}


def _build(tmp_path, name, text):
    c = tmp_path / (name + ".c")
    c.write_text(text)
    so = tmp_path / ("lib" + name + ".so")
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-shared", "-fPIC", "-pthread", str(c),
                           "-o", str(so), "-lm"])
    return str(so)


def _battery(so):
    return subprocess.run([sys.executable, os.path.join(HERE, "oracle_battery.py"), so],
                          capture_output=True, text=True, timeout=300)


def test_battery_passes_on_oracle(tmp_path):
    src = open(SRC).read()
    r = _battery(_build(tmp_path, "orig", src))
    assert r.returncode == 0, r.stdout + r.stderr


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_battery_catches_mutant(tmp_path, name):
    src = open(SRC).read()
    old, new = MUTANTS[name]
    assert src.count(old) >= 1, "mutation anchor not found: " + name
    r = _battery(_build(tmp_path, name, src.replace(old, new, 1)))
    assert r.returncode != 0, "pins did not catch mutant " + name
