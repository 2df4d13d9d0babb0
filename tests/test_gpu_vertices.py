"""Vertices in range (the alternative output of Section 3) on the GPU against the oracle, set for
set: single queries through iso_query_vertices and batches through the device bitmaps of
iso_query_batch_vertices_device, in both sweep modes and both cell-kernel variants, on graphs
with uncovered cells, zero-length arcs, unreachable parts and no partition."""
import ctypes as C
import sys

import numpy as np
import pytest

import paper_1512_09090_amd as iso
import synth
from oracle import Oracle

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def bitmap_rows(bits, n):
    """(k, W) uint64 rows -> list of sorted uint32 vertex arrays."""
    b = np.ascontiguousarray(bits.view(np.uint64))
    out = []
    for row in b:
        flags = np.unpackbits(row.view(np.uint8), bitorder="little")[:n]
        out.append(np.flatnonzero(flags).astype(np.uint32))
    return out


def device_vertices(G, src, tau, mode):
    import torch
    W = (G.n + 63) // 64
    bits = torch.full((len(src), W), -1, dtype=torch.int64, device="cuda:0")   # every bit must be written
    G.query_batch_vertices_device(src, tau, mode, bits)
    return bitmap_rows(bits.cpu().numpy(), G.n)


@pytest.fixture(scope="module")
def grid():
    import torch
    torch.cuda.init()
    g = synth.config_graph("grid64")
    return g, Oracle.from_graph(g)


def test_grid64_single_queries(grid):
    g, orc = grid
    G = iso.Graph.from_synth(g, num_cells=16, device=0)
    src, _ = synth.config_queries("grid64", 4)
    for s in src.tolist():
        for tau in (0, 150, 2000, 7000, 40000, iso.TAU_MAX):
            want = orc.in_range(s, tau)
            for mode in (iso.MODE_CELLS, iso.MODE_PLAIN):
                say(f"grid64 vertices s={s} tau={tau} mode={mode}")
                np.testing.assert_array_equal(G.query_vertices(s, tau, mode), want)
    # the edge output of the same handle is unchanged by vertex calls
    s = int(src[0])
    np.testing.assert_array_equal(G.query(s, 2000, iso.MODE_CELLS), orc.isochrone(s, 2000)[0])


def test_plain_hierarchy(grid):
    g, orc = grid
    G = iso.Graph.from_synth(g, num_cells=0, device=0)
    for s in (0, 2080, 4095):
        for tau in (0, 2000, 9000):
            say(f"no partition: vertices s={s} tau={tau}")
            np.testing.assert_array_equal(G.query_vertices(s, tau, iso.MODE_PLAIN), orc.in_range(s, tau))
    out = device_vertices(G, np.array([0, 2080, 4095], np.uint32), np.array([0, 2000, 9000], np.uint32),
                          iso.MODE_PLAIN)
    for got, s, tau in zip(out, (0, 2080, 4095), (0, 2000, 9000)):
        np.testing.assert_array_equal(got, orc.in_range(s, tau))


@pytest.mark.parametrize("seed", range(6))
def test_random_digraph_random_cells(seed):
    """Random cells: uncovered cells, cells without core vertices, unreachable parts, zero arcs."""
    g = synth.random_digraph(300, 900, seed=900 + seed, wmax=40, zero_frac=0.1)
    rng = np.random.default_rng(seed)
    k = int(rng.integers(1, 9))
    cells = rng.integers(0, k, size=g.n).astype(np.uint32)
    say(f"random digraph seed={seed} cells={k}")
    G = iso.Graph(g.n, g.tail, g.head, g.w, cell_of=cells, num_cells=k, device=0)
    orc = Oracle.from_graph(g)
    srcs, taus = [], []
    for s in rng.integers(0, g.n, size=4).tolist():
        d = orc.distances(s)
        fin = d[d != np.uint64(0xFFFFFFFFFFFFFFFF)]
        for tau in sorted({0, int(fin.max()), int(np.median(fin)), int(fin.max()) + 1}):
            srcs.append(s)
            taus.append(tau)
            want = orc.in_range(s, tau)
            for mode in (iso.MODE_CELLS, iso.MODE_PLAIN):
                np.testing.assert_array_equal(G.query_vertices(s, tau, mode), want, err_msg=f"s={s} tau={tau}")
    for mode in (iso.MODE_CELLS, iso.MODE_PLAIN):
        out = device_vertices(G, np.array(srcs, np.uint32), np.array(taus, np.uint32), mode)
        for got, s, tau in zip(out, srcs, taus):
            np.testing.assert_array_equal(got, orc.in_range(s, tau), err_msg=f"batch s={s} tau={tau} mode={mode}")


@pytest.fixture(scope="module")
def road():
    import torch
    torch.cuda.init()
    g = synth.road_graph(40_000, 29)
    say("road40k / 128 cells")
    return g, Oracle.from_graph(g), iso.Graph.from_synth(g, num_cells=128, device=0)


@pytest.mark.parametrize("knobs", [dict(), dict(cell_stage=1), dict(table_max=1, use_graph=0),
                                   dict(cell_lds_kb=16, cell_block=256)])
def test_road_batches(road, knobs):
    g, orc, G = road
    G.set_tuning(**knobs)
    try:
        src, tau = synth.batch_queries(g.n, 64, seed=41, lo_min=1, hi_min=150)
        for mode in (iso.MODE_CELLS, iso.MODE_PLAIN):
            say(f"road40k vertex bitmaps, 64 queries, mode {mode}, {knobs}")
            out = device_vertices(G, src, tau, mode)
            for j in range(0, 64, 3):
                np.testing.assert_array_equal(out[j], orc.in_range(int(src[j]), int(tau[j])), err_msg=f"lane {j}")
        out = device_vertices(G, src[:5], tau[:5], iso.MODE_CELLS)      # fewer lanes than a power of two
        for j in range(5):
            np.testing.assert_array_equal(out[j], orc.in_range(int(src[j]), int(tau[j])))
    finally:
        G.set_tuning()
    # edges of the same handle afterwards
    np.testing.assert_array_equal(G.query(int(src[0]), int(tau[0]), iso.MODE_CELLS),
                                  orc.isochrone(int(src[0]), int(tau[0]))[0])


def test_vertex_output_bad_arguments(road):
    import torch
    g, orc, G = road
    W = (G.n + 63) // 64
    bits = torch.zeros((65, W), dtype=torch.int64, device="cuda:0")
    src = np.zeros(65, np.uint32)
    tau = np.full(65, 1000, np.uint32)
    L = iso.lib()
    sp = src.ctypes.data_as(C.POINTER(C.c_uint32))
    tp = tau.ctypes.data_as(C.POINTER(C.c_uint32))
    for k in (0, 65):
        rc = L.iso_query_batch_vertices_device(G._h, k, sp, tp, iso.MODE_CELLS, C.c_void_p(bits.data_ptr()), None)
        assert rc == iso.ISO_EINVAL
    host = np.zeros((2, W), np.uint64)
    rc = L.iso_query_batch_vertices_device(G._h, 2, sp, tp, iso.MODE_CELLS, C.c_void_p(host.ctypes.data), None)
    assert rc == iso.ISO_EINVAL
    small = torch.zeros(W, dtype=torch.int64, device="cuda:0")      # one row where two are needed
    with pytest.raises(iso.IsoError):
        G.query_batch_vertices_device(src[:2], tau[:2], iso.MODE_CELLS, small)
    np.testing.assert_array_equal(G.query_vertices(0, 1000, iso.MODE_CELLS), orc.in_range(0, 1000))
