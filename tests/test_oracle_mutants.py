"""Planted mistakes in copies of the oracle must each fail at least one pin.

Every mutant is a single textual change to a copy of oracle/pirrt_oracle.c (the
kind of slip a hand-written Replan can carry: a dropped term, a wrong comparison,
a wrong index, a transposed operand).  The copy is compiled on the CPU into a
temporary directory and run through the pins of oracle_pins.py.
"""
import os
import subprocess

import pytest

import oracle as O
from oracle_pins import PINS

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "pirrt_oracle.c")

MUTANTS = {
    "improve_non_strict": ("if (best_u >= 0 && best < G->g[v] && (", "if (best_u >= 0 && best <= G->g[v] && ("),
    "improve_tie_highest": ("(u < best_u || (u == best_u && G->cst[v][j] < best_c))",
                            "(u > best_u || (u == best_u && G->cst[v][j] < best_c))"),
    "improve_tie_first_seen": ("(u < best_u || (u == best_u && G->cst[v][j] < best_c))", "0"),
    "improve_cost_tie_ignored": ("(u < best_u || (u == best_u && G->cst[v][j] < best_c))", "(u < best_u)"),
    "improve_max": (
        "float cand = G->g[u] + G->cst[v][j];\n        if (cand < best ||",
        "float cand = G->g[u] + G->cst[v][j];\n        if (cand > best ||"),
    "improve_drops_cost": ("float cand = G->g[u] + G->cst[v][j];", "float cand = G->g[u];"),
    "improve_keeps_old_pcost": ("newpc[v] = best_c;", "newpc[v] = G->pcost[v];"),
    "improve_gauss_seidel": ("newpar[v] = best_u;", "newpar[v] = best_u;\n        G->g[v] = best;"),
    "insert_tie_highest": ("(u < best_u || (u == best_u && cost[j] < best_c))",
                           "(u > best_u || (u == best_u && cost[j] < best_c))"),
    "insert_cost_tie_ignored": ("(u < best_u || (u == best_u && cost[j] < best_c))", "(u < best_u)"),
    "insert_orphan_zero": ("    G->g[v] = best;\n", "    G->g[v] = best_u >= 0 ? best : 0.0f;\n"),
    "evaluate_wrong_index": ("G->g[c] = G->g[v] + G->pcost[c];\n      depth[c]", "G->g[c] = G->g[v] + G->pcost[v];\n      depth[c]"),
    "evaluate_no_reset": ("for (int64_t v = 0; v < n; ++v) G->g[v] = INFINITY;", ""),
    "domain_without_neighbours": ("        inD[w] = 1;\n", ""),
    "lookahead_drops_heuristic": ("float f = offer + (h ? h[w] : 0.0f);", "float f = offer;"),
    "lookahead_target_g": ("float offer = G->g[v] + G->cst[v][j];", "float offer = G->g[w] + G->cst[v][j];"),
    "lookahead_ignored": ("        if (lookahead) {", "        if (0) {"),
    "domain_keeps_root": ("inD[root] = 0;", ""),
    "promising_non_strict": ("inP[v] = f < thr;", "inP[v] = f <= thr;"),
    "threshold_wrong_vertex": ("float thr = prune ? G->g[goal] : INFINITY;", "float thr = prune ? G->g[root] : INFINITY;"),
    "heuristic_dropped": ("float hv = h ? h[v] : 0.0f;", "float hv = 0.0f;"),
    "single_iteration": ("if (nchg == 0) break;", "break;"),
    "edges_stat_per_vertex": ("ex += G->deg[v];", "ex += 1;"),
    "trunc_wrong_index": ("G->g[c] = G->g[v] + G->pcost[c];\n      float f", "G->g[c] = G->g[v] + G->pcost[v];\n      float f"),
    "trunc_counts_own_parent": ("best < G->g[v] && (!truncated || best_u != G->parent[v] || best_c != G->pcost[v])",
                                "best < G->g[v]"),
    "trunc_tests_parent": ("float f = G->g[c] + (h ? h[c] : 0.0f);", "float f = G->g[v] + (h ? h[v] : 0.0f);"),
    "trunc_non_strict": ("      if (f < G0) {", "      if (f <= G0) {"),
    "trunc_resets_unvisited": ("  G->g[root] = 0.0f;\n  queue[tail++] = root;",
                               "  for (int64_t v = 0; v < n; ++v) G->g[v] = INFINITY;\n  G->g[root] = 0.0f;\n  queue[tail++] = root;"),
    "trunc_root_in_b": ("  return nb;\n}", "  inB[root] = 1;\n  return nb + 1;\n}"),
    "trunc_full_promising_test": ("    if (truncated) {\n      np = nb;", "    if (0) {\n      np = nb;"),
    "mirror_wrong_endpoint": ("push_adj(G, col[j], (int32_t)v, cost[j])", "push_adj(G, col[j], col[j], cost[j])"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, "mutation site of %s not unique/present" % name
    mutated = tmp_path / "mutant.c"
    mutated.write_text(src.replace(old, new))
    so = tmp_path / "libmutant.so"
    subprocess.run(["gcc"] + O.CFLAGS + [str(mutated), "-o", str(so), "-lm"], check=True)
    lib = O.load(str(so))
    caught = []
    for pin in PINS:
        try:
            pin(lib)
        except AssertionError as e:
            caught.append("%s: %s" % (pin.__name__, str(e).splitlines()[0] if str(e) else ""))
            break
    assert caught, "mutant %s passed every pin" % name
