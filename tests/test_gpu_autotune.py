"""The autotuner on a road graph with a reduced search space (needs an MI355X): the knobs it
chooses are the ones applied to the graph, a saved result re-applies them, and the answers
under the chosen knobs equal those under the defaults."""
import sys

import numpy as np
import pytest

import paper_1512_09090_amd as iso
import synth
from paper_1512_09090_amd import autotune

pytestmark = pytest.mark.gpu


def test_autotune_reduced_space(tmp_path):
    g = synth.road_graph(50_000, 31)
    G = iso.Graph.from_synth(g, num_cells=256, device=0)
    src, tau = synth.batch_queries(g.n, 192, seed=17, lo_min=1, hi_min=120)
    ref = G.query_batch(src, tau, iso.MODE_CELLS)
    space = {"lanes_per_launch": [32, 64], "cell_lds_kb": [40, 64], "use_graph": [0, 1], "overlap_cells": [0, 2]}
    res = autotune.tune(G, src, tau, space=space,
                        log=lambda m: print(m, file=sys.stderr, flush=True))
    best = res["best"]
    # every value of every knob was measured at least once (a knob's earlier best is measured again
    # once another value has replaced it)
    assert res["qps"] > 0
    for k, vals in space.items():
        assert set(vals) <= {t["knobs"][k] for t in res["trials"]}, k
    applied = G.get_tuning()
    for k, v in best.items():
        assert applied[k] == v, f"knob {k}: chosen {v}, applied {applied[k]}"
    out = G.query_batch(src, tau, iso.MODE_CELLS)
    for j in range(len(src)):
        np.testing.assert_array_equal(out[j], ref[j], err_msg=f"lane {j} under {best}")
    path = tmp_path / "tuning.json"
    autotune.save(res, str(path))
    G.set_tuning()
    assert autotune.apply(G, str(path)) == best
    assert {k: G.get_tuning()[k] for k in best} == best
    G.set_tuning()
