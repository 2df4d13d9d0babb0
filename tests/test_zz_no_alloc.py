"""The no-allocation entry point (iso_query_batch_device_noalloc) against iso_query_batch_device,
called through the C ABI on the same queries: edges and offsets equal, two calls in a row with
the second one smaller, and two graphs sharing the GPU's static scratch in turn."""
import sys

import numpy as np
import pytest

import paper_1512_09090_amd as iso
import synth
from oracle import Oracle

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def run(G, src, tau, mode, noalloc, cap=None):
    import torch

    k = len(src)
    pairs = torch.full((cap if cap is not None else 80_000 * max(1, k), 2), -1, dtype=torch.int32, device="cuda:0")
    offsets = torch.full((k + 1,), -1, dtype=torch.int32, device="cuda:0")
    fn = G.query_batch_device_noalloc if noalloc else G.query_batch_device
    total = fn(src, tau, mode, pairs, offsets)
    off = offsets.cpu().numpy().view(np.uint32).astype(np.int64)
    flat = pairs[:total].cpu().numpy().view(np.uint32)
    return total, off, flat


def same(G, src, tau, mode):
    want = run(G, src, tau, mode, False)
    got = run(G, src, tau, mode, True)
    assert got[0] == want[0]
    np.testing.assert_array_equal(got[1], want[1])
    np.testing.assert_array_equal(got[2], want[2])
    return got


@pytest.fixture(scope="module")
def graphs():
    import torch

    torch.cuda.init()
    g1 = synth.road_graph(40_000, 37)
    g2 = synth.config_graph("grid64")
    say("road40k / 128 cells, grid64 / 16 cells")
    return ((g1, iso.Graph.from_synth(g1, num_cells=128, device=0)),
            (g2, iso.Graph.from_synth(g2, num_cells=16, device=0)))


def test_noalloc_equals_device_output(graphs):
    (g1, G1), (g2, G2) = graphs
    for mode in (iso.MODE_CELLS, iso.MODE_PLAIN, iso.MODE_CD):
        src, tau = synth.batch_queries(g1.n, 70, seed=40 + mode, lo_min=1, hi_min=90)
        say(f"mode {mode}: 70 queries (two sweeps), then 5")
        total, off, flat = same(G1, src, tau, mode)
        same(G1, src[:5], tau[:5], mode)            # a second, smaller call
    orc = Oracle.from_graph(g1)
    for j in (0, 33, 69):
        want, _, _ = orc.isochrone(int(src[j]), int(tau[j]))
        np.testing.assert_array_equal(flat[off[j]:off[j + 1]], want)


def test_noalloc_graphs_share_the_scratch(graphs):
    (g1, G1), (g2, G2) = graphs
    s1, t1 = synth.batch_queries(g1.n, 20, seed=50, lo_min=1, hi_min=90)
    s2, t2 = synth.config_queries("grid64", 12)
    for rep in range(2):
        say(f"alternating graphs, round {rep}")
        same(G1, s1, t1, iso.MODE_CELLS)
        same(G2, s2, t2, iso.MODE_CELLS)
        same(G1, s1[:3], t1[:3], iso.MODE_PLAIN)


def test_noalloc_small_output_buffer(graphs):
    (g1, G1), _ = graphs
    src, tau = synth.batch_queries(g1.n, 10, seed=60, lo_min=30, hi_min=90)
    total, _, _ = run(G1, src, tau, iso.MODE_CELLS, False)
    with pytest.raises(iso.IsoError) as e:
        run(G1, src, tau, iso.MODE_CELLS, True, cap=max(1, total // 2))
    assert e.value.code == iso.ISO_ESPACE and e.value.total == total
    got = run(G1, src, tau, iso.MODE_CELLS, True, cap=total)
    assert got[0] == total
