"""Isochrone polygons on the device (iso_query_polygon_batch, Section 7) against the oracle's
face traversal, on planar jittered grids, on a uniform grid with a hole, and on a non-planar
road-like graph (where both still trace the faces of the same rotation system).  Needs an
MI355X."""
import sys

import numpy as np
import pytest

import paper_1512_09090_amd as iso
import synth
from oracle import Oracle

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def same_polygon(got, want, what):
    assert len(got) == len(want), f"{what}: {len(got)} cycles, oracle {len(want)}"
    for c, (x, y) in enumerate(zip(got, want)):
        np.testing.assert_array_equal(x, y, err_msg=f"{what}: cycle {c}")


def check_batch(G, orc, xy, src, tau, mode, what):
    out = G.polygon_batch(src, tau, mode)
    assert len(out) == len(src)
    for j in range(len(src)):
        want = orc.polygon(xy, orc.in_range(int(src[j]), int(tau[j])))
        same_polygon(out[j], want, f"{what} mode {mode} lane {j} (source {src[j]}, tau {tau[j]})")
    return out


@pytest.fixture(scope="module")
def grid64():
    g = synth.config_graph("grid64")
    say(f"grid64: n={g.n}")
    G = iso.Graph(g.n, g.tail, g.head, g.w, xy=g.xy, num_cells=16, device=0)
    return g, Oracle.from_graph(g), G


@pytest.mark.parametrize("mode", [iso.MODE_PLAIN, iso.MODE_CELLS, iso.MODE_CD])
def test_grid64_batch_of_64(grid64, mode):
    g, orc, G = grid64
    rng = np.random.default_rng(20 + mode)
    src = rng.integers(0, g.n, size=64).astype(np.uint32)
    tau = rng.integers(0, 12000, size=64).astype(np.uint32)
    tau[:4] = [0, 1, 4_000_000, 2_000]   # the source alone, tiny, everything (no border), mid
    out = check_batch(G, orc, g.xy, src, tau, mode, "grid64")
    assert out[2] == []
    assert sum(len(c) for c in out) > 64


def test_grid64_single_and_small_batches(grid64):
    g, orc, G = grid64
    s, tau = 1234, 3000
    want = orc.polygon(g.xy, orc.in_range(s, tau))
    same_polygon(G.polygon(s, tau, iso.MODE_CELLS), want, "single query")
    for k in (1, 3, 17):
        rng = np.random.default_rng(k)
        src = rng.integers(0, g.n, size=k).astype(np.uint32)
        tau = rng.integers(500, 9000, size=k).astype(np.uint32)
        check_batch(G, orc, g.xy, src, tau, iso.MODE_CELLS, f"k={k}")


def test_larger_jittered_grid():
    g = synth.grid_graph(300, 200, seed=5)
    say(f"grid300x200: n={g.n}")
    G = iso.Graph(g.n, g.tail, g.head, g.w, xy=g.xy, num_cells=64, device=0)
    orc = Oracle.from_graph(g)
    rng = np.random.default_rng(6)
    src = rng.integers(0, g.n, size=40).astype(np.uint32)
    tau = rng.integers(1000, 40000, size=40).astype(np.uint32)
    check_batch(G, orc, g.xy, src, tau, iso.MODE_CELLS, "grid300x200")


def test_uniform_grid_diamond_and_hole():
    """Closed forms on the device: an L1 ball of radius r is one cycle of 4(2r + 1) darts; slow
    vertices inside it add a clockwise hole cycle."""
    W, c = 25, 10
    s = 12 * W + 12
    g = synth.uniform_grid(W, c)
    G = iso.Graph(g.n, g.tail, g.head, g.w, xy=g.xy, device=0)
    for r in range(0, 9):
        cyc = G.polygon(s, c * r, iso.MODE_PLAIN)
        assert len(cyc) == 1 and len(cyc[0]) == 4 * (2 * r + 1)
    block = (np.arange(15, 18)[:, None] * W + np.arange(14, 16)[None, :]).ravel()
    slow = np.zeros(g.n, dtype=bool)
    slow[block] = True
    w = g.w.astype(np.uint64)
    w[slow[g.tail] | slow[g.head]] *= 1_000_000
    w = w.astype(np.uint32)
    Gb = iso.Graph(g.n, g.tail, g.head, w, xy=g.xy, device=0)
    ob = Oracle(g.n, g.tail, g.head, w)
    cyc = Gb.polygon(s, c * 9, iso.MODE_PLAIN)
    assert sorted(len(x) for x in cyc) == [10, 4 * 19]
    same_polygon(cyc, ob.polygon(g.xy, ob.in_range(s, c * 9)), "grid with a hole")


def test_non_planar_graph_follows_the_rotation_system():
    g = synth.road_graph(20_000, 41)
    G = iso.Graph(g.n, g.tail, g.head, g.w, xy=g.xy, num_cells=32, device=0)
    orc = Oracle.from_graph(g)
    src, tau = synth.batch_queries(g.n, 24, seed=9, lo_min=1, hi_min=30)
    check_batch(G, orc, g.xy, src, tau, iso.MODE_CELLS, "road20k")


def test_without_coordinates_is_a_state_error():
    g = synth.config_graph("grid64")
    G = iso.Graph(g.n, g.tail, g.head, g.w, device=0)
    with pytest.raises(iso.IsoError) as e:
        G.polygon(0, 1000)
    assert e.value.code == iso.ISO_ESTATE
    # the handle stays usable
    assert len(G.query(0, 1000)) > 0
