"""Host preprocessing (partition, hierarchy, sweep layout) checked on the CPU.

These tests load graphs with device = -1 and inspect the layout arrays through
iso_graph_get_layout.  The numpy sweep below is a checker of the hierarchy (it
reads the library's layout), not the oracle; its distances are compared with
the oracle's.
"""
import heapq
import os

import numpy as np
import pytest

import paper_1512_09090_amd as iso
import synth
from oracle import INF as OINF
from oracle import Oracle, clamp_u32
from tests import golden_io

MASK = 0x3FFFFFFF
FWD, REV = 0x80000000, 0x40000000
U32INF = 0xFFFFFFFF


def load(g, **kw):
    kw.setdefault("device", -1)
    if "cell_of" in kw:
        return iso.Graph(g.n, g.tail, g.head, g.w, **kw)
    return iso.Graph.from_synth(g, **kw)


def segment_index(L):
    """Per position: a sweep-step index that every downward arc must strictly increase."""
    n, nc = L["n"], L["n_core"]
    seg = np.zeros(n, dtype=np.int64)
    cl = L["core_lvl"]
    for i in range(len(cl) - 1):
        seg[cl[i]:cl[i + 1]] = i
    base = len(cl)
    for c in range(L["num_cells"]):
        starts = list(L["cell_lvl"][L["cell_lvl_ptr"][c]:L["cell_lvl_ptr"][c + 1]]) + [L["cell_off"][c + 1]]
        for i in range(len(starts) - 1):
            seg[starts[i]:starts[i + 1]] = base + i
    return seg


def cell_of_position(L):
    n = L["n"]
    cp = np.full(n, -1, dtype=np.int64)
    for c in range(L["num_cells"]):
        cp[L["cell_off"][c]:L["cell_off"][c + 1]] = c
    return cp


def check_structure(g, L):
    n, nc = L["n"], L["n_core"]
    perm = L["perm"]
    assert np.array_equal(np.sort(perm), np.arange(n))
    pos = np.empty(n, dtype=np.int64)
    pos[perm] = np.arange(n)
    off, arc = L["down_off"], L["down_arc"]
    heads = np.repeat(np.arange(n), np.diff(off))
    tails = (arc[:, 0] & MASK).astype(np.int64)
    seg = segment_index(L)
    # I6: every downward arc goes from an earlier sweep step to a later one
    assert np.all(tails < heads)
    cpos = cell_of_position(L)
    internal = heads >= nc
    assert np.all(seg[tails[~internal]] < seg[heads[~internal]])
    # internal heads: tails are core, or in the same cell on an earlier cell level
    t_in = tails[internal] >= nc
    hh, tt = heads[internal], tails[internal]
    assert np.all(cpos[tt[t_in]] == cpos[hh[t_in]])
    assert np.all(seg[tt[t_in]] < seg[hh[t_in]])
    # I9: each original arc exactly once, FWD at its head position or REV at its tail position
    fwd = (arc[:, 0] & FWD) != 0
    rev = (arc[:, 0] & REV) != 0
    got = np.concatenate([perm[tails[fwd]].astype(np.uint64) << np.uint64(32) | perm[heads[fwd]].astype(np.uint64),
                          perm[heads[rev]].astype(np.uint64) << np.uint64(32) | perm[tails[rev]].astype(np.uint64)])
    t, h = g.tail.astype(np.uint64), g.head.astype(np.uint64)
    keep = t != h
    want = np.unique((t[keep] << np.uint64(32)) | h[keep])
    assert got.size == want.size, "an original arc is missing or duplicated in the downward graph"
    assert np.array_equal(np.sort(got), want)
    # dummy entries (length INF) carry REV only
    dummy = arc[:, 1] == U32INF
    assert np.all(rev[dummy] & ~fwd[dummy])
    return pos


def layout_sweep(L, pos, s):
    """Upward search + level-ordered downward sweep over the layout (numpy)."""
    n = L["n"]
    d = np.full(n, U32INF, dtype=np.uint64)
    uo, uh, uw = L["up_off"], L["up_head"], L["up_w"]
    ps = int(pos[s])
    d[ps] = 0
    heap = [(0, ps)]
    while heap:
        k, u = heapq.heappop(heap)
        if k != d[u]:
            continue
        for e in range(uo[u], uo[u + 1]):
            x, nd = int(uh[e]), min(k + int(uw[e]), U32INF)
            if nd < d[x]:
                d[x] = nd
                heapq.heappush(heap, (nd, x))
    off, arc = L["down_off"], L["down_arc"]
    tails = (arc[:, 0] & MASK).astype(np.int64)
    w = arc[:, 1].astype(np.uint64)

    def relax(a, b):
        eb, ee = off[a], off[b]
        if ee == eb:
            return
        cand = np.minimum(d[tails[eb:ee]] + w[eb:ee], U32INF)
        heads = np.repeat(np.arange(a, b), np.diff(off[a:b + 1]))
        np.minimum.at(d, heads, cand)

    cl = L["core_lvl"]
    for i in range(len(cl) - 1):
        relax(cl[i], cl[i + 1])
    for c in range(L["num_cells"]):
        starts = list(L["cell_lvl"][L["cell_lvl_ptr"][c]:L["cell_lvl_ptr"][c + 1]]) + [L["cell_off"][c + 1]]
        for i in range(len(starts) - 1):
            relax(starts[i], starts[i + 1])
    out = np.empty(n, dtype=np.uint32)
    out[L["perm"]] = d.astype(np.uint32)
    return out


CASES = [
    ("grid64-plain", lambda: synth.config_graph("grid64"), dict(num_cells=0)),
    ("grid64-16", lambda: synth.config_graph("grid64"), dict(num_cells=16)),
    ("road20k-64", lambda: synth.road_graph(20_000, 21), dict(num_cells=64)),
    ("road20k-oneway-64", lambda: synth.road_graph(20_000, 22, oneway_frac=0.25), dict(num_cells=64)),
    ("road20k-plain", lambda: synth.road_graph(20_000, 23), dict(num_cells=0)),
]


@pytest.mark.parametrize("name,make,kw", CASES, ids=[c[0] for c in CASES])
def test_layout_structure_and_sweep(name, make, kw):
    g = make()
    G = load(g, **kw)
    L = G.layout()
    pos = check_structure(g, L)
    orc = Oracle.from_graph(g)
    rng = np.random.default_rng(len(name))
    for s in rng.integers(0, g.n, size=4).tolist():
        np.testing.assert_array_equal(layout_sweep(L, pos, s), clamp_u32(orc.distances(s)))


@pytest.mark.parametrize("seed", range(6))
def test_random_digraph_random_cells(seed):
    g = synth.random_digraph(60, 200, seed=300 + seed, zero_frac=0.2)
    rng = np.random.default_rng(seed)
    cells = rng.integers(0, 5, size=g.n).astype(np.uint32)
    G = load(g, cell_of=cells, num_cells=5)
    L = G.layout()
    pos = check_structure(g, L)
    orc = Oracle.from_graph(g)
    for s in range(0, 60, 7):
        np.testing.assert_array_equal(layout_sweep(L, pos, s), clamp_u32(orc.distances(s)))


def test_eccentricity_and_uncovered():
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import dijkstra

    g = synth.road_graph(20_000, 22, oneway_frac=0.25)
    G = load(g, num_cells=64)
    L = G.layout()
    perm, nc, cell_of = L["perm"], L["n_core"], L["cell_of"]
    rng = np.random.default_rng(3)
    checked_unc = 0
    for c in rng.choice(64, size=10, replace=False).tolist():
        verts = np.flatnonzero(cell_of == c)
        local = -np.ones(g.n, dtype=np.int64)
        local[verts] = np.arange(verts.size)
        inside = (cell_of[g.tail] == c) & (cell_of[g.head] == c)
        A = csr_matrix((g.w[inside].astype(np.float64),
                        (local[g.tail[inside]], local[g.head[inside]])), shape=(verts.size, verts.size))
        core_here = [p for p in range(nc) if L["core_cell"][p] == c]
        for p in core_here:
            dd = dijkstra(A, indices=int(local[perm[p]]))
            assert L["core_ecc"][p] == int(dd[np.isfinite(dd)].max())
        # boundary vertices: an arc to or from another cell
        out_cut = cell_of[g.head] != cell_of[g.tail]
        bset = set(g.tail[out_cut & (cell_of[g.tail] == c)].tolist()) | set(g.head[out_cut & (cell_of[g.head] == c)].tolist())
        if bset:
            dd = dijkstra(A, indices=[int(local[b]) for b in bset], min_only=True)
            uncovered = not np.all(np.isfinite(dd))
        else:
            uncovered = verts.size > 0
        assert bool(L["uncovered"][c]) == uncovered
        checked_unc += uncovered
    # the one-way graph is built so that some cells are uncovered; make sure the case is exercised overall
    assert L["uncovered"].sum() > 0


def test_uncovered_hand_built():
    # cell 0 = {0, 1}: boundary vertex 1 reaches 0 (1->0), so the cell is covered.
    # cell 1 = {2, 3}: boundary vertex 2 (arc 1->2 from cell 0); vertex 3 only reaches 2 (3->2), is never reached
    tail = np.array([0, 1, 1, 3], dtype=np.uint32)
    head = np.array([1, 0, 2, 2], dtype=np.uint32)
    w = np.array([1, 1, 1, 1], dtype=np.uint32)
    G = iso.Graph(4, tail, head, w, cell_of=np.array([0, 0, 1, 1], dtype=np.uint32), num_cells=2, device=-1)
    L = G.layout()
    assert list(L["uncovered"]) == [0, 1]


def test_golden_fixtures_layout():
    for name in ("fig2_right.txt", "fig2_left_mountain.txt"):
        f = golden_io.load(name)
        g = synth.Graph(f["n"], f["tail"], f["head"], f["w"])
        G = iso.Graph(f["n"], f["tail"], f["head"], f["w"], cell_of=f["cells"],
                      num_cells=int(f["cells"].max()) + 1, device=-1)
        L = G.layout()
        pos = check_structure(g, L)
        np.testing.assert_array_equal(layout_sweep(L, pos, f["source"]), f["dist"].astype(np.uint32))


def test_prep_file_roundtrip(tmp_path):
    g = synth.road_graph(20_000, 21)
    path = str(tmp_path / "g.prep")
    G1 = load(g, num_cells=64, prep_path=path)
    assert os.path.exists(path)
    G2 = load(g, num_cells=64, prep_path=path)
    assert G2.info()["prep_seconds"] == 0.0
    L1, L2 = G1.layout(), G2.layout()
    for k in ("perm", "down_off", "down_arc", "up_off", "up_head", "up_w", "core_lvl", "cell_off",
              "cell_lvl", "core_ecc", "uncovered"):
        np.testing.assert_array_equal(L1[k], L2[k])
    # a corrupted file is refused, not silently used
    raw = bytearray(open(path, "rb").read())
    raw[len(raw) // 2] ^= 0xFF
    open(path, "wb").write(bytes(raw))
    with pytest.raises(iso.IsoError) as e:
        load(g, num_cells=64, prep_path=path)
    assert e.value.code == iso.ISO_EFORMAT


def test_abi_exports_every_declared_symbol():
    L = iso.lib()
    names = iso.header_functions()
    assert len(names) >= 12
    for name in names:
        assert hasattr(L, name), name


def test_abi_error_paths():
    g = synth.config_graph("grid64")
    with pytest.raises(iso.IsoError) as e:
        iso.Graph(0, g.tail, g.head, g.w, device=-1)
    assert e.value.code == iso.ISO_EINVAL
    bad = g.head.copy()
    bad[3] = g.n
    with pytest.raises(iso.IsoError) as e:
        iso.Graph(g.n, g.tail, bad, g.w, device=-1)
    assert e.value.code == iso.ISO_EINVAL
    w = g.w.copy()
    w[0] = 0xFFFFFFFF
    with pytest.raises(iso.IsoError) as e:
        iso.Graph(g.n, g.tail, g.head, w, device=-1)
    assert e.value.code == iso.ISO_EINVAL
    with pytest.raises(iso.IsoError) as e:
        iso.Graph(g.n, g.tail, g.head, g.w, cell_of=np.full(g.n, 9, dtype=np.uint32), num_cells=4, device=-1)
    assert e.value.code == iso.ISO_EINVAL
    with pytest.raises(iso.IsoError) as e:   # a cell larger than max_cell_size
        iso.Graph(g.n, g.tail, g.head, g.w, cell_of=np.zeros(g.n, dtype=np.uint32), num_cells=1,
                  max_cell_size=1024, device=-1)
    assert e.value.code == iso.ISO_EINVAL
    G = iso.Graph(g.n, g.tail, g.head, g.w, device=-1)
    with pytest.raises(iso.IsoError) as e:
        G.query(0, 10)
    assert e.value.code == iso.ISO_EDEVICE
    with pytest.raises(iso.IsoError) as e:
        G.query(g.n, 10)
    assert e.value.code == iso.ISO_EINVAL
    with pytest.raises(iso.IsoError) as e:
        G.query(0, 0xFFFFFFFF)
    assert e.value.code == iso.ISO_EINVAL
    for mode in (iso.MODE_CELLS, iso.MODE_CD, 3, -1):   # no partition; unknown modes
        with pytest.raises(iso.IsoError) as e:
            G.query(0, 10, mode)
        assert e.value.code == iso.ISO_EINVAL, mode
    Gc = iso.Graph.from_synth(g, num_cells=16, device=-1)
    with pytest.raises(iso.IsoError) as e:      # the core-search mode needs the device as well
        Gc.query(0, 10, iso.MODE_CD)
    assert e.value.code == iso.ISO_EDEVICE
    with pytest.raises(iso.IsoError) as e:
        G.set_tuning(lanes_per_launch=65)
    assert e.value.code == iso.ISO_EINVAL
    for bad in (dict(block=96), dict(cell_lds_kb=8), dict(use_graph=2), dict(core_mode=1), dict(core_mode=3),
                dict(cell_stage=3),
                dict(cell_block=128), dict(table_max=16385), dict(stall=2)):
        with pytest.raises(iso.IsoError) as e:
            G.set_tuning(**bad)
        assert e.value.code == iso.ISO_EINVAL, bad


@pytest.mark.parametrize("kind", ["grid_cells", "random_cells", "oneway_cells", "oneway_plain"])
def test_every_arc_flagged_on_exactly_one_entry(kind):
    """The downward entries' arc flags (Section 5: original-arc flags, dummy entries) name every
    arc of the input exactly once, forward or reverse; isochrone-edge keys rank arcs through
    these flags, so a missing or repeated arc would drop or duplicate an output edge."""
    if kind == "grid_cells":
        g = synth.config_graph("grid64")
        G = iso.Graph.from_synth(g, num_cells=16, device=-1)
    elif kind == "random_cells":
        g = synth.random_digraph(300, 900, seed=701, wmax=40, zero_frac=0.1)
        cells = np.random.default_rng(1).integers(0, 5, size=g.n).astype(np.uint32)
        G = iso.Graph(g.n, g.tail, g.head, g.w, cell_of=cells, num_cells=5, device=-1)
    else:
        g = synth.road_graph(20_000, 32, oneway_frac=0.3)
        G = iso.Graph.from_synth(g, num_cells=64 if kind == "oneway_cells" else 0, device=-1)
    L = G.layout()
    perm = L["perm"].astype(np.int64)
    off = L["down_off"].astype(np.int64)
    x = L["down_arc"][:, 0].astype(np.int64)
    v = np.repeat(np.arange(len(off) - 1), np.diff(off))
    t = x & 0x3FFFFFFF
    f, r = (x & 0x80000000) != 0, (x & 0x40000000) != 0
    flagged = np.concatenate([perm[t[f]] << 32 | perm[v[f]], perm[v[r]] << 32 | perm[t[r]]])
    loops = g.tail == g.head
    want = np.unique(g.tail[~loops].astype(np.int64) << 32 | g.head[~loops].astype(np.int64))
    assert len(flagged) == len(want)
    np.testing.assert_array_equal(np.sort(flagged), want)


def _core_search(L, s_pos, tau):
    """The isoPHAST-CD reading, written out plainly on the layout: an upward search from s that does
    not expand core vertices, then a tau-bounded Dijkstra over the core hierarchy (upward arcs and
    finite downward entries turned around) from the core vertices it reached."""
    import heapq
    nc, INF = int(L["n_core"]), 0xFFFFFFFF
    up_off, up_head, up_w = L["up_off"], L["up_head"], L["up_w"]
    d, pq, done = {s_pos: 0}, [(0, s_pos)], set()
    while pq:
        du, u = heapq.heappop(pq)
        if u in done or du != d[u]:
            continue
        done.add(u)
        if u < nc:
            continue
        for e in range(int(up_off[u]), int(up_off[u + 1])):
            x, nd = int(up_head[e]), min(INF, du + int(up_w[e]))
            if nd < d.get(x, INF):
                d[x] = nd
                heapq.heappush(pq, (nd, x))
    adj = {}
    for x in range(nc):
        for e in range(int(up_off[x]), int(up_off[x + 1])):
            adj.setdefault(x, []).append((int(up_head[e]), int(up_w[e])))
    off, arc = L["down_off"], L["down_arc"]
    for v in range(nc):
        for e in range(int(off[v]), int(off[v + 1])):
            t, w = int(arc[e, 0]) & 0x3FFFFFFF, int(arc[e, 1])
            if w != INF:
                adj.setdefault(t, []).append((v, w))
    lab = {u: du for u, du in d.items() if u < nc}
    pq, settled = [(du, u) for u, du in lab.items()], {}
    heapq.heapify(pq)
    while pq and pq[0][0] <= tau:
        du, u = heapq.heappop(pq)
        if u in settled or du != lab[u]:
            continue
        settled[u] = du
        for x, w in adj.get(u, ()):
            nd = min(INF, du + w)
            if nd < lab.get(x, INF):
                lab[x] = nd
                heapq.heappush(pq, (nd, x))
    return settled


@pytest.mark.parametrize("kind", ["grid", "random"])
def test_core_hierarchy_search_settles_the_core_in_range(kind):
    """isoPHAST-CD runs isoDijkstra on the core (Section 5); here the core is itself contracted, and a
    search on its hierarchy must settle exactly the core vertices the oracle puts in range, with the
    oracle's distances (the reading the GPU mode relies on)."""
    from oracle import Oracle
    if kind == "grid":
        g = synth.config_graph("grid64")
        G = iso.Graph.from_synth(g, num_cells=16, device=-1)
        sources, taus = [0, 2080, 4095], [0, 150, 2000, 7000]
    else:
        g = synth.random_digraph(300, 900, seed=1701, wmax=40, zero_frac=0.1)
        cells = np.random.default_rng(3).integers(0, 6, size=g.n).astype(np.uint32)
        G = iso.Graph(g.n, g.tail, g.head, g.w, cell_of=cells, num_cells=6, device=-1)
        sources, taus = [0, 77, 299], [0, 20, 60, 10_000]
    L = G.layout()
    perm = L["perm"]
    pos = np.empty_like(perm)
    pos[perm] = np.arange(len(perm), dtype=perm.dtype)
    orc = Oracle.from_graph(g)
    for s in sources:
        full = orc.distances(s)
        for tau in taus:
            got = _core_search(L, int(pos[s]), tau)
            want = {p: int(full[perm[p]]) for p in range(int(L["n_core"])) if full[perm[p]] <= tau}
            assert got == want, (s, tau)


def test_parallel_arcs_and_self_loops_are_merged():
    tail = np.array([0, 0, 0, 1, 1, 2], dtype=np.uint32)
    head = np.array([1, 1, 0, 2, 2, 0], dtype=np.uint32)
    w = np.array([5, 3, 1, 7, 2, 4], dtype=np.uint32)
    G = iso.Graph(3, tail, head, w, device=-1)
    assert G.info()["m"] == 3
    L = G.layout()
    pos = np.empty(3, dtype=np.int64)
    pos[L["perm"]] = np.arange(3)
    np.testing.assert_array_equal(layout_sweep(L, pos, 0), np.array([0, 3, 5], dtype=np.uint32))


def test_result_buffer_views_own_library_memory():
    """Edge arrays wrap the library's result buffer without a copy; slices keep it alive and
    the last view releases it with iso_free."""
    import ctypes
    import gc

    from paper_1512_09090_amd import binding

    libc = ctypes.CDLL(None)
    libc.malloc.restype = ctypes.c_void_p
    libc.malloc.argtypes = [ctypes.c_size_t]
    freed = []
    real_free = binding.lib().iso_free

    class Spy:
        def __getattr__(self, name):
            return getattr(binding.lib(), name)

        def iso_free(self, p):
            freed.append(p.value)
            real_free(p)

    addr = libc.malloc(6 * 4)
    ctypes.memmove(addr, np.arange(6, dtype=np.uint32).ctypes.data, 24)
    saved = binding._lib
    binding._lib = Spy()
    try:
        arr = binding._edges_to_numpy(ctypes.cast(addr, ctypes.POINTER(binding.Edge)), 3)
        assert arr.shape == (3, 2) and arr.dtype == np.uint32
        tail = arr[1:]
        del arr
        gc.collect()
        assert freed == []
        np.testing.assert_array_equal(tail, [[2, 3], [4, 5]])
        del tail
        gc.collect()
        assert freed == [addr]
        empty = binding._edges_to_numpy(ctypes.cast(libc.malloc(8), ctypes.POINTER(binding.Edge)), 0)
        assert empty.shape == (0, 2) and len(freed) == 2
    finally:
        binding._lib = saved


def test_device_only_entry_points_refuse_hostless_graphs():
    """The device-output, vertex-output and one-to-many entry points on a graph loaded without a
    device, and their argument checks, fail with status codes before any device work."""
    import ctypes

    g = synth.config_graph("grid64")
    G = iso.Graph.from_synth(g, num_cells=16, device=-1)
    L = iso.lib()
    src = np.array([1, 2], dtype=np.uint32)
    tau = np.array([100, 200], dtype=np.uint32)
    sp = src.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))
    tp = tau.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))
    with pytest.raises(iso.IsoError) as e:
        G.query_vertices(1, 100, iso.MODE_CELLS)
    assert e.value.code == iso.ISO_EDEVICE
    words = np.zeros(2 * 64, dtype=np.uint64)
    rc = L.iso_query_batch_vertices_device(G._h, 2, sp, tp, iso.MODE_CELLS, ctypes.c_void_p(words.ctypes.data), None)
    assert rc == iso.ISO_EDEVICE
    total = ctypes.c_uint64()
    offs = np.zeros(3, dtype=np.uint32)
    rc = L.iso_query_batch_device(G._h, 2, sp, tp, iso.MODE_CELLS, ctypes.c_void_p(words.ctypes.data), 10,
                                  ctypes.c_void_p(offs.ctypes.data), ctypes.byref(total), None)
    assert rc == iso.ISO_EDEVICE
    rc = L.iso_query_batch_device(G._h, 2, sp, tp, iso.MODE_CELLS, None, 10, None, ctypes.byref(total), None)
    assert rc == iso.ISO_EINVAL                  # NULL offsets
    with pytest.raises(iso.IsoError) as e:
        G.select_targets(np.array([1, 2, 3], dtype=np.uint32))
    assert e.value.code == iso.ISO_EDEVICE
    h = ctypes.c_void_p()
    rc = L.iso_targets_select(G._h, None, 3, ctypes.byref(h))
    assert rc == iso.ISO_EINVAL and not h.value  # NULL targets with a count
    L.iso_targets_free(None)                     # freeing nothing is a no-op
    rc = L.iso_targets_get_info(None, None, None, None, None)
    assert rc == iso.ISO_EINVAL
