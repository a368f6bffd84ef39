"""Mutation test of the oracle's pins (CPU only).

Each mutant is a copy of ``oracle/mst_oracle.c`` with one plausible mistake
planted (a flipped comparison, a dropped term, a transposed operand, an
off-by-one).  Every mutant must fail at least one pin of ``mst_pins``; a
mutant that survives would mean the pins cannot tell that mistake from the
correct oracle.  Mutants run in a subprocess so a crash or a hang counts as
caught without taking the test runner down.
"""

import os
import subprocess
import sys

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "mst_oracle.c")

# (name, original text, replacement)
MUTANTS = [
    ("sort_descending", "return (x > y) - (x < y);", "return (x < y) - (x > y);"),
    ("key_drops_index", "return ((uint64_t)w[e] << 32) | (uint64_t)e;", "return ((uint64_t)w[e] << 32);"),
    ("key_drops_weight", "return ((uint64_t)w[e] << 32) | (uint64_t)e;", "return (uint64_t)e;"),
    ("kruskal_no_cycle_check", "if (ra == rb) continue; /* would close", "if (ra == rb && 0) continue; /* would close"),
    ("kruskal_stops_early", "taken + 1 < (int64_t)n", "taken + 2 < (int64_t)n"),
    ("kruskal_total_dropped", "in_mst[e] = 1;\n        *total += w[e];\n        ++taken;",
     "in_mst[e] = 1;\n        ++taken;"),
    ("boruvka_min_flipped", "order_key(w, minimum[c1]) > k", "order_key(w, minimum[c1]) < k"),
    ("boruvka_drops_second_end",
     "if (minimum[c2] == -1 || order_key(w, minimum[c2]) > k) minimum[c2] = e;", ""),
    ("boruvka_transposed_end", "int32_t c2 = uf_find(&comp, dst[e]);\n            if (c1 == c2) {",
     "int32_t c2 = uf_find(&comp, src[e]);\n            if (c1 == c2) {"),
    ("boruvka_no_reset", "for (int32_t v = 0; v < n; ++v) minimum[v] = -1;", ""),
    ("boruvka_no_recheck", "if (c1 == c2) continue;\n            in_mst[e] = 1;",
     "in_mst[e] = 1;"),
    ("boruvka_count_off_by_one", "components -= added;", "components -= added + 1;"),
    ("boruvka_live_counts_internal", "            ++live;\n", ""),
    ("checker_cycle_flipped", "if (order_key(w, e) < pmax) bad", "if (order_key(w, e) > pmax) bad"),
    ("checker_lca_last_step_dropped", "uint64_t x = upmax[a], y = upmax[b];", "uint64_t x = 0, y = 0;"),
    ("checker_no_span_check", "if (marked != (int64_t)n - comps) return CHECK_NOT_SPANNING;", ""),
    ("checker_no_total_check", "if (sum != total) return CHECK_TOTAL;", ""),
    ("min_edges_drops_second_end", "if (k < keys[dst[e]]) keys[dst[e]] = k;", ""),
    ("min_edges_keeps_loops", "if (src[e] == dst[e]) continue;\n        uint64_t k = order_key(w, e);",
     "uint64_t k = order_key(w, e);"),
    ("range_check_off_by_one", "src[e] >= n || dst[e] < 0 || dst[e] >= n) return ORACLE_ERR_RANGE",
     "src[e] > n || dst[e] < 0 || dst[e] >= n) return ORACLE_ERR_RANGE"),
]

RUNNER = r"""
import sys
sys.path.insert(0, {root!r}); sys.path.insert(0, {tests!r})
import oracle, mst_pins
orc = oracle.Oracle({lib!r})
for name, fn in mst_pins.PINS.items():
    try:
        fn(orc)
    except Exception as exc:
        print("CAUGHT", name, type(exc).__name__, str(exc)[:200])
        sys.exit(0)
print("SURVIVED")
sys.exit(3)
"""


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(tmp_path, name, old, new):
    text = open(SRC).read()
    assert text.count(old) == 1, f"mutation site for {name} must occur exactly once"
    mut_src = tmp_path / "mutant.c"
    mut_src.write_text(text.replace(old, new))
    lib = oracle.build(force=True, src=str(mut_src), out=str(tmp_path / "libmutant.so"))
    code = RUNNER.format(root=ROOT, tests=os.path.join(ROOT, "tests"), lib=lib)
    try:
        p = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120)
    except subprocess.TimeoutExpired:
        return  # a hang is a caught mistake
    assert "SURVIVED" not in p.stdout, f"mutant {name} passed every pin"
