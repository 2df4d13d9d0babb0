"""Autotuner for the device sweep: queries per launch, core-kernel block size, LDS budget per
cell workgroup, the cell-kernel variant (one workgroup per active cell, or work items of a
cell and some of its queries with a level pipeline or the whole cell in LDS), resident cell
workgroups per compute unit while two sweeps overlap, hipGraph replay and the level-merge
threshold (how many vertices of the top core levels are merged into one distance-table
product instead of one launch per level).

Coordinate search: starting from the defaults, each knob in turn is set to every candidate
value while the others stay fixed; the best throughput (queries/s of iso_query_batch on a
sample of the caller's queries) is kept.  Every call returns identical results whatever the
knobs, so the search only measures time.  The result is applied to the graph and can be
written to a JSON file and re-applied later with `apply`.
"""
from __future__ import annotations

import json
import time

import numpy as np

from .binding import MODE_CELLS, Graph

SPACE = {
    "cell_stage": [2, 0, 1],
    "overlap_cells": [0, 1, 2],
    "lanes_per_launch": [16, 32, 64],
    "block": [128, 256, 512],
    "cell_lds_kb": [40, 64, 96],
    "use_graph": [0, 1],
    "table_max": [0, 4096, 8192],
}
# the library's defaults (include/iso.h), the search's starting point
DEFAULT = {"lanes_per_launch": 64, "block": 256, "cell_lds_kb": 64, "use_graph": 1, "core_mode": 0, "cell_stage": 2,
           "cell_block": 0, "table_max": 0, "stall": 1, "edge_cap": 0, "overlap_cells": 0, "plain_sweep": 0}


def measure(G: Graph, sources, taus, mode=MODE_CELLS, repeats: int = 2) -> float:
    """Queries per second of iso_query_batch over the whole sample (best of `repeats`)."""
    best = 0.0
    for _ in range(repeats):
        t0 = time.perf_counter()
        G.query_batch(sources, taus, mode)
        best = max(best, len(sources) / (time.perf_counter() - t0))
    return best


def tune(G: Graph, sources, taus, mode=MODE_CELLS, space=None, log=None) -> dict:
    space = space or SPACE
    cur = dict(DEFAULT)
    G.set_tuning(**cur)
    measure(G, sources[:64], taus[:64], mode, repeats=1)          # warm the buffers
    best_qps = measure(G, sources, taus, mode)
    trials = [{"knobs": dict(cur), "qps": best_qps}]
    for knob, values in space.items():
        for v in values:
            if v == cur[knob]:
                continue
            cand = dict(cur, **{knob: v})
            G.set_tuning(**cand)
            qps = measure(G, sources, taus, mode)
            trials.append({"knobs": cand, "qps": qps})
            if log:
                log(f"autotune {cand} -> {qps:.1f} q/s")
            if qps > best_qps:
                best_qps, cur = qps, cand
        G.set_tuning(**cur)
    return {"best": cur, "qps": best_qps, "trials": trials}


def save(result: dict, path: str):
    with open(path, "w") as f:
        json.dump(result, f, indent=1)


def apply(G: Graph, path: str) -> dict:
    with open(path) as f:
        best = json.load(f)["best"]
    G.set_tuning(**best)
    return best


def sample(n_queries: int, sources, taus, seed: int = 0):
    rng = np.random.default_rng(seed)
    idx = rng.choice(len(sources), size=min(n_queries, len(sources)), replace=False)
    return np.asarray(sources)[idx], np.asarray(taus)[idx]
