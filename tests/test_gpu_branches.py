"""Rare paths of the device sweep, forced on small hand-built graphs (needs an MI355X).

Each test builds an input that drives one path the benchmark graph reaches only at full
size, checks with the branch counters (iso_debug_read) that the path ran, and compares every
result with the oracle or with the same query on the common path.
"""
import sys

import numpy as np
import pytest

import paper_1512_09090_amd as iso
import synth
from oracle import Oracle

pytestmark = pytest.mark.gpu

CAND_FULL, WIDE_LEVEL, CORE_WALK, CORE_KEYS_FULL, RESWEEP = range(5)


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def arcs_both_ways(a, b, w):
    a, b, w = (np.asarray(x, dtype=np.int64) for x in (a, b, w))
    return (np.concatenate([a, b]).astype(np.uint32), np.concatenate([b, a]).astype(np.uint32),
            np.concatenate([w, w]).astype(np.uint32))


def star_cell_graph(leaves=1200, path=50):
    """A hub with `leaves` leaves (one cell, all leaves on one level) and a path in a second
    cell, so that the hub is a core vertex."""
    hub = 0
    lv = np.arange(1, leaves + 1)
    p = np.arange(leaves + 1, leaves + 1 + path)
    a = np.concatenate([np.zeros(leaves, np.int64), [hub], p[:-1]])
    b = np.concatenate([lv, [p[0]], p[1:]])
    w = np.concatenate([np.full(leaves, 100), [10], np.full(path - 1, 10)])
    t, h, ww = arcs_both_ways(a, b, w)
    n = leaves + 1 + path
    cells = np.zeros(n, np.uint32)
    cells[p] = 1
    return n, t, h, ww, cells


def check_all(G, orc, src, tau, modes):
    for mode in modes:
        out = G.query_batch(src, tau, mode)
        for j in range(len(src)):
            want, _, _ = orc.isochrone(int(src[j]), int(tau[j]))
            np.testing.assert_array_equal(out[j], want, err_msg=f"mode {mode} lane {j}")


def test_cell_level_wider_than_workgroup_and_full_edge_list():
    """1200 leaves on the one level of a cell (more than a cell workgroup's 512 threads), all
    straddling the limit (2400 isochrone edges in one cell, more than the 512-key list)."""
    n, t, h, w, cells = star_cell_graph()
    G = iso.Graph(n, t, h, w, cell_of=cells, num_cells=2, device=0)
    orc = Oracle(n, t, h, w)
    G.debug_enable(True)
    src = np.array([0, 0, 5, 1230, 0], np.uint32)
    tau = np.array([50, 150, 120, 500, 99], np.uint32)
    check_all(G, orc, src, tau, (iso.MODE_CELLS, iso.MODE_PLAIN))
    cnt = G.debug_read()
    say(f"counters {cnt}")
    assert cnt[WIDE_LEVEL] > 0 and cnt[CAND_FULL] > 0
    assert len(orc.isochrone(0, 50)[0]) >= 2400   # every leaf arc, and one path arc
    # the per-item cell kernels (level buffers of 512 entries, 512-word candidate lists) agree
    for stage in (0, 1):
        G.set_tuning(cell_stage=stage)
        check_all(G, orc, src, tau, (iso.MODE_CELLS,))
    G.set_tuning()
    G.debug_enable(False)


def test_core_key_list_full():
    """2000 degree-one vertices on the bottom core level, each straddling the limit: with one
    query and 1024-thread core workgroups a workgroup finds 2048 keys (list of 1024)."""
    N = 2000
    u, x = np.arange(1, N + 1), np.arange(N + 1, 2 * N + 1)
    t, h, w = arcs_both_ways(np.concatenate([np.zeros(N, np.int64), u]), np.concatenate([u, x]),
                             np.concatenate([np.ones(N), np.full(N, 100)]))
    n = 2 * N + 1
    G = iso.Graph(n, t, h, w, device=0)
    orc = Oracle(n, t, h, w)
    G.set_tuning(block=1024, table_max=1, lanes_per_launch=1)
    G.debug_enable(True)
    check_all(G, orc, np.array([0, 3], np.uint32), np.array([50, 101], np.uint32), (iso.MODE_PLAIN,))
    cnt = G.debug_read()
    say(f"counters {cnt}")
    assert cnt[CORE_KEYS_FULL] > 0
    G.set_tuning()
    G.debug_enable(False)


def test_core_vertex_with_many_entries():
    """A vertex joined to a 40-clique by long arcs is contracted first and keeps 40 downward
    entries; with 64 queries per sweep each (vertex, query) thread walks them again for the
    straddling ones."""
    k = 40
    v = 0
    ys = np.arange(1, k + 1)
    ia, ib = np.triu_indices(k, 1)
    a = np.concatenate([np.zeros(k, np.int64), ys[ia]])
    b = np.concatenate([ys, ys[ib]])
    w = np.concatenate([np.full(k, 10), np.ones(ia.size)])
    t, h, ww = arcs_both_ways(a, b, w)
    n = k + 1
    G = iso.Graph(n, t, h, ww, device=0)
    L = G.layout()
    pos_v = int(np.flatnonzero(L["perm"] == v)[0])
    assert L["down_off"][pos_v + 1] - L["down_off"][pos_v] > 32
    orc = Oracle(n, t, h, ww)
    rng = np.random.default_rng(3)
    src = rng.integers(0, n, size=64).astype(np.uint32)
    tau = rng.integers(0, 30, size=64).astype(np.uint32)
    src[0], tau[0] = v, 5
    G.set_tuning(table_max=1)
    G.debug_enable(True)
    check_all(G, orc, src, tau, (iso.MODE_PLAIN,))
    cnt = G.debug_read()
    say(f"counters {cnt}")
    assert cnt[CORE_WALK] > 0
    G.set_tuning()
    G.debug_enable(False)


@pytest.fixture(scope="module")
def road():
    g = synth.road_graph(40_000, 37)
    say("road40k / 128 cells")
    return g, Oracle.from_graph(g), iso.Graph.from_synth(g, num_cells=128, device=0)


def test_edge_buffer_resweep(road):
    """A 16-edge key buffer: every sweep overflows and is run again with a larger one."""
    g, orc, G = road
    src, tau = synth.batch_queries(g.n, 70, seed=5, lo_min=1, hi_min=60)
    ref = G.query_batch(src, tau, iso.MODE_CELLS)
    G.debug_enable(True)
    G.set_tuning(edge_cap=16)
    out = G.query_batch(src, tau, iso.MODE_CELLS)
    one = G.query(int(src[3]), int(tau[3]), iso.MODE_PLAIN)
    cnt = G.debug_read()
    say(f"counters {cnt}")
    assert cnt[RESWEEP] >= 2
    G.set_tuning()
    G.debug_enable(False)
    for j in range(len(src)):
        np.testing.assert_array_equal(out[j], ref[j])
    np.testing.assert_array_equal(one, ref[3])
    for j in (0, 3, 69):
        np.testing.assert_array_equal(ref[j], orc.isochrone(int(src[j]), int(tau[j]))[0])


def test_server_regrows_edge_buffer(road):
    """The serving loop starting from a 16-edge buffer grows it and answers every request as a
    single query does."""
    g, orc, G = road
    src, tau = synth.batch_queries(g.n, 40, seed=6, lo_min=1, hi_min=60)
    singles = [G.query(int(s), int(t), iso.MODE_CELLS) for s, t in zip(src, tau)]
    G.set_tuning(edge_cap=16)
    srv = iso.Server(G, max_lanes=8, max_inflight=2, mode=iso.MODE_CELLS)
    try:
        tickets = [srv.submit(int(s), int(t)) for s, t in zip(src, tau)]
        for i, tk in enumerate(tickets):
            got, _ = srv.wait(tk)
            np.testing.assert_array_equal(got, singles[i], err_msg=f"request {i}")
        st = srv.stats()
        say(f"server stats {st}")
        assert st["regrown"] >= 1
    finally:
        srv.close()
        G.set_tuning()


def test_wide_entries():
    """Lengths too large for the packed one-word entries: the cell data keep two-word entries
    (same answers)."""
    g = synth.road_graph(30_000, 38)
    w64 = g.w.astype(np.uint64) * 256
    assert int(w64.max()) < 0xFFFFFFFF and int(w64.max()) >= 1 << 24
    w = w64.astype(np.uint32)
    G = iso.Graph(g.n, g.tail, g.head, w, xy=g.xy, num_cells=64, device=0)
    orc = Oracle(g.n, g.tail, g.head, w)
    rng = np.random.default_rng(8)
    src = rng.integers(0, g.n, size=20).astype(np.uint32)
    tau = rng.integers(60_000 * 256, 3_600_000 * 256, size=20).astype(np.uint32)
    check_all(G, orc, src, tau, (iso.MODE_CELLS, iso.MODE_PLAIN))
    d, sw = G.distances(int(src[0]), int(tau[0]), iso.MODE_PLAIN)
    from oracle import clamp_u32
    np.testing.assert_array_equal(d, clamp_u32(orc.distances(int(src[0]))))
