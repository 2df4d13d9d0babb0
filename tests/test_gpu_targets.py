"""One-to-many distances (RPHAST: target selection, then a sweep restricted to the selected
vertices) on the GPU against the oracle's exact distances, element by element: grids with and
without a partition, random digraphs with unreachable targets and zero-length arcs, target sets
that include the top of the hierarchy, several sweeps per call, every top-table prefix
(including none), and the device-memory form."""
import sys

import numpy as np
import pytest

import paper_1512_09090_amd as iso
import synth
from oracle import Oracle, clamp_u32

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def expected(orc, sources, targets):
    return np.stack([clamp_u32(orc.distances(int(s)))[targets] for s in sources])


@pytest.fixture(scope="module")
def grid():
    import torch
    torch.cuda.init()
    g = synth.config_graph("grid64")
    return g, Oracle.from_graph(g)


@pytest.mark.parametrize("cells", [16, 0])
def test_grid64_ball(grid, cells):
    g, orc = grid
    G = iso.Graph.from_synth(g, num_cells=cells, device=0)
    top = int(G.layout()["perm"][0])                     # the top of the hierarchy as a target too
    _, ball = synth.target_ball(g, 300, seed=3)
    targets = np.concatenate([ball, [top, ball[0]]]).astype(np.uint32)   # with a duplicate
    T = G.select_targets(targets)
    say(f"grid64 cells={cells}: {T.info()}")
    sources = np.array([int(ball[5]), 0, 4095, top], dtype=np.uint32)
    np.testing.assert_array_equal(T.query(sources), expected(orc, sources, targets))
    T.close()


@pytest.mark.parametrize("seed", range(4))
def test_random_digraph_unreachable(seed):
    g = synth.random_digraph(300, 700, seed=1300 + seed, wmax=30, zero_frac=0.15)
    rng = np.random.default_rng(seed)
    k = int(rng.integers(1, 7))
    cells = rng.integers(0, k, size=g.n).astype(np.uint32)
    G = iso.Graph(g.n, g.tail, g.head, g.w, cell_of=cells, num_cells=k, device=0)
    orc = Oracle.from_graph(g)
    targets = rng.choice(g.n, size=60, replace=False).astype(np.uint32)
    sources = rng.integers(0, g.n, size=9).astype(np.uint32)
    T = G.select_targets(targets)
    got = T.query(sources)
    np.testing.assert_array_equal(got, expected(orc, sources, targets))   # INF where unreachable


@pytest.fixture(scope="module")
def road():
    import torch
    torch.cuda.init()
    g = synth.road_graph(40_000, 31)
    say("road40k / 128 cells")
    return g, Oracle.from_graph(g), iso.Graph.from_synth(g, num_cells=128, device=0)


@pytest.mark.parametrize("table_max", [0, 1, 64, 16384])
def test_road_ball_many_sources(road, table_max):
    """70 sources at 64 per sweep (two sweeps), for every top-table prefix."""
    g, orc, G = road
    G.set_tuning(table_max=table_max)
    try:
        _, targets = synth.target_ball(g, 1024, seed=7)
        T = G.select_targets(targets)
        info = T.info()
        say(f"road40k table_max={table_max}: {info}")
        assert 0 < info["vertices"] < g.n
        sources = synth.batch_queries(g.n, 70, seed=9)[0]
        got = T.query(sources)
        want = expected(orc, sources[::7], targets)
        np.testing.assert_array_equal(got[::7], want)
        # the other rows against single-source calls of the same target set
        for j in (1, 64, 69):
            np.testing.assert_array_equal(T.query(sources[j:j + 1])[0], got[j])
        if table_max != 1:
            G.set_tuning(table_max=1)                 # another table prefix than at selection
            with pytest.raises(iso.IsoError) as e:
                T.query(sources[:2])
            assert e.value.code == iso.ISO_ESTATE
    finally:
        G.set_tuning()


def test_road_device_output(road):
    import torch
    g, orc, G = road
    _, targets = synth.target_ball(g, 2000, seed=11)
    T = G.select_targets(targets)
    sources = synth.batch_queries(g.n, 40, seed=12)[0]
    dist = torch.full((40, len(targets)), -1, dtype=torch.int32, device="cuda:0")
    T.query_device(sources, dist)
    got = dist.cpu().numpy().view(np.uint32)
    np.testing.assert_array_equal(got, T.query(sources))
    np.testing.assert_array_equal(got[:3], expected(orc, sources[:3], targets))
    small = torch.zeros(10, dtype=torch.int32, device="cuda:0")
    with pytest.raises(iso.IsoError):
        T.query_device(sources, small)
    # isochrones on the same handle afterwards
    s, tau = int(sources[0]), 600_000
    np.testing.assert_array_equal(G.query(s, tau, iso.MODE_CELLS), orc.isochrone(s, tau)[0])
