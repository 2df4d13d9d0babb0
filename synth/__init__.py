"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This package only draws graphs and query lists.  It contains no shortest-path,
hierarchy or isochrone arithmetic, so that the oracle and the HIP path can both
consume its output without sharing any of the method's code.
"""
from .roadgen import (  # noqa: F401
    Graph,
    grid_graph,
    road_graph,
    random_digraph,
    uniform_grid,
    config_graph,
    config_queries,
    CONFIGS,
    batch_queries,
    serving_trace,
    target_ball,
)
