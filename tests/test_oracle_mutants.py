"""The oracle's pins must catch plausible mistakes.

Each case plants one mistake in a temporary copy of oracle.c (never in the
file itself), builds it with gcc, and checks that at least one pin - brute
force, closed form, a golden fixture or an exact-limit case - rejects it.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import synth
from oracle import INF, SRC_PATH, Oracle
from tests import golden_io
from tests.test_oracle_pins import as_u64, bellman_ford, definition_edges, polygon_pins_pass

MUTANTS = {
    "strict_stop": ("if (ws->heap[0].key > tau) break;", "if (ws->heap[0].key >= tau) break;"),
    "no_incoming_rule": ("            if (!is_settled(ws, g->in_tail[e]))\n"
                         "                buf = push_key(buf, &cnt, &cap, g->in_tail[e], u);",
                         "            ;"),
    "swapped_incoming_pair": ("buf = push_key(buf, &cnt, &cap, g->in_tail[e], u);",
                              "buf = push_key(buf, &cnt, &cap, u, g->in_tail[e]);"),
    "heap_wrong_child": ("if (c + 1 < len && ws->heap[c + 1].key < ws->heap[c].key) c++;",
                         "if (c + 1 < len && ws->heap[c + 1].key > ws->heap[c].key) c++;"),
    "definition_one_way": ("if (u_in != v_in) buf", "if (u_in && !v_in) buf"),
    "definition_strict": ("int v_in = dist[g->out_head[e]] <= tau;",
                          "int v_in = dist[g->out_head[e]] < tau;"),
    "isodij_no_inf_keys": ("                heap_push(ws, ORC_INF, v);          /* key infinity */\n", ""),
    "isodij_no_out_sweep": ("            if (is_settled(ws, g->out_head[e]))\n"
                            "                buf = push_key(buf, &cnt, &cap, v, g->out_head[e]);",
                            "            ;"),
    "in_range_drops_one": ("for (uint64_t i = 0; i < settled; ++i) buf[i] = ws->order[i];\n"
                           "    qsort(buf, settled, sizeof(uint32_t), cmp_u32);\n    *verts_out = buf;\n"
                           "    return settled;",
                           "for (uint64_t i = 0; i < settled; ++i) buf[i] = ws->order[i];\n"
                           "    qsort(buf, settled, sizeof(uint32_t), cmp_u32);\n    *verts_out = buf;\n"
                           "    return settled ? settled - 1 : 0;"),
    "polygon_ccw_walk": ("uint64_t kc = ka == off[b] ? off[b + 1] - 1 : ka - 1;",
                         "uint64_t kc = ka + 1 == off[b + 1] ? off[b] : ka + 1;"),
    "polygon_no_twin": ("uint64_t key = ((uint64_t)b << 32) | a, lo = 0, hi = nd;",
                        "uint64_t key = ((uint64_t)a << 32) | b, lo = 0, hi = nd;"),
    "polygon_exit_test": ("if (!in_range[a] && in_range[b]) break;", "if (in_range[a] && !in_range[b]) break;"),
    "relax_wrong_weight": ("uint64_t nd = it.key + g->out_w[e];\n            if (nd < get_dist(ws, v)) {\n"
                           "                set_dist(ws, v, nd);\n                heap_push(ws, nd, v);\n            }\n        }\n    }\n    return",
                           "uint64_t nd = it.key + g->out_w[e] / 2;\n            if (nd < get_dist(ws, v)) {\n"
                           "                set_dist(ws, v, nd);\n                heap_push(ws, nd, v);\n            }\n        }\n    }\n    return"),
}


def _pins_pass(libpath) -> bool:
    """Run a compact set of pins against the library at libpath; False on the first failure."""
    # brute force
    for seed in range(12):
        g = synth.random_digraph(18, 50, seed=500 + seed, wmax=9, zero_frac=0.2)
        arcs = list(zip(g.tail.tolist(), g.head.tolist(), g.w.tolist()))
        orc = Oracle.from_graph(g, libpath)
        bf = bellman_ford(g.n, arcs, 0)
        if not np.array_equal(orc.distances(0), as_u64(bf)):
            return False
        for tau in sorted({x for x in bf if x is not None}):
            want = definition_edges(arcs, bf, tau)
            if not np.array_equal(orc.isochrone(0, tau)[0], want):
                return False
            if not np.array_equal(orc.iso_dijkstra(0, tau)[0], want):
                return False
            if not np.array_equal(orc.edges_by_definition(as_u64(bf), tau), want):
                return False
            inr = [v for v in range(g.n) if bf[v] is not None and bf[v] <= tau]
            if not np.array_equal(orc.in_range(0, tau), np.array(inr, dtype=np.uint32)):
                return False
    # closed form
    g = synth.uniform_grid(21, 3)
    orc = Oracle.from_graph(g, libpath)
    for r in range(0, 9):
        if len(orc.isochrone(10 * 21 + 10, 3 * r)[0]) != 8 * (2 * r + 1):
            return False
    # golden reconstruction
    for name in ("fig2_right.txt", "fig2_left_mountain.txt"):
        f = golden_io.load(name)
        orc = Oracle(f["n"], f["tail"], f["head"], f["w"], libpath)
        if not np.array_equal(orc.isochrone(f["source"], f["tau"])[0], f["expect"]):
            return False
        if not np.array_equal(orc.distances(f["source"]), f["dist"]):
            return False
    try:
        return polygon_pins_pass(libpath)
    except ValueError:   # a face walk that never closes
        return False


def test_unmodified_oracle_passes(tmp_path):
    out = str(tmp_path / "liboracle_ref.so")
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-shared", "-fPIC", "-o", out, SRC_PATH, "-lm"])
    assert _pins_pass(out)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc missing")
@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC_PATH).read()
    assert src.count(old) == 1, f"mutation site for {name} not found exactly once"
    mpath = tmp_path / f"oracle_{name}.c"
    mpath.write_text(src.replace(old, new))
    out = str(tmp_path / f"liboracle_{name}.so")
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-shared", "-fPIC", "-o", out, str(mpath), "-lm"])
    assert not _pins_pass(out), f"mutant {name} survived every pin"
    os.remove(out)
