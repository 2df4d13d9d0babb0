"""Pins for the CPU oracle against things other than itself.

* brute force: Bellman-Ford in pure Python plus the Section 3 definition of
  isochrone edges written as a full scan over the arcs (tiny random digraphs with
  zero weights, one-way arcs, self-loops, parallel arcs and several components);
* a library routine: scipy's Dijkstra with a distance limit;
* a closed form: the uniform 4-neighbour grid (d = c * L1, 8(2r+1) isochrone arcs);
* special limits: tau = 0, tau = d(s,v) exactly, tau beyond every finite distance;
* the reconstructed Figure 2 instances (tests/golden);
* invariants: d(s) = 0, triangle inequality on every arc, tight predecessors,
  reversal closure, monotonicity in tau.
"""
import numpy as np
import pytest

import synth
from oracle import INF, Oracle
from tests import golden_io


# ---------------------------------------------------------------- helpers
def bellman_ford(n, arcs, s):
    """Pure-Python Bellman-Ford; None marks unreachable."""
    d = [None] * n
    d[s] = 0
    for _ in range(n):
        changed = False
        for t, h, w in arcs:
            if d[t] is not None and (d[h] is None or d[t] + w < d[h]):
                d[h] = d[t] + w
                changed = True
        if not changed:
            break
    return d


def definition_edges(arcs, d, tau):
    """Section 3: arcs with exactly one endpoint u having d(s,u) <= tau."""
    inr = lambda x: d[x] is not None and d[x] <= tau  # noqa: E731
    out = sorted({(t, h) for t, h, _ in arcs if inr(t) != inr(h)})
    return np.array(out, dtype=np.uint32).reshape(-1, 2)


def as_u64(d):
    return np.array([INF if x is None else x for x in d], dtype=np.uint64)


def arcs_of(g):
    return list(zip(g.tail.tolist(), g.head.tolist(), g.w.tolist()))


# ---------------------------------------------------------------- brute force
@pytest.mark.parametrize("seed", range(60))
def test_bellman_ford_random_digraphs(seed):
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(1, 40))
    m = int(rng.integers(0, 4 * n + 1))
    g = synth.random_digraph(n, m, seed=seed, wmax=int(rng.integers(1, 30)), zero_frac=0.15)
    arcs = arcs_of(g)
    orc = Oracle.from_graph(g)
    for s in rng.integers(0, n, size=min(n, 4)).tolist():
        bf = bellman_ford(n, arcs, s)
        np.testing.assert_array_equal(orc.distances(s), as_u64(bf))
        finite = sorted({x for x in bf if x is not None})
        taus = {0, finite[-1], finite[-1] + 1, int(rng.integers(0, finite[-1] + 2))}
        taus |= set(finite[: 6])                        # exact hits tau = d(s, v)
        taus |= {max(0, x - 1) for x in finite[: 6]}
        for tau in sorted(taus):
            want = definition_edges(arcs, bf, tau)
            edges, dist, settled = orc.isochrone(s, tau, want_dist=True)
            np.testing.assert_array_equal(edges, want)
            exp_d = as_u64([x if (x is not None and x <= tau) else None for x in bf])
            np.testing.assert_array_equal(dist, exp_d)
            assert settled == sum(1 for x in bf if x is not None and x <= tau)
            e2, settled2 = orc.iso_dijkstra(s, tau)
            np.testing.assert_array_equal(e2, want)
            assert settled2 == settled
            np.testing.assert_array_equal(orc.edges_by_definition(as_u64(bf), tau), want)
            # the vertices in range (Section 3), against the brute-force distances
            inr = [v for v in range(n) if bf[v] is not None and bf[v] <= tau]
            np.testing.assert_array_equal(orc.in_range(s, tau), np.array(inr, dtype=np.uint32))


# ---------------------------------------------------------------- library routine
@pytest.mark.parametrize("name,nsrc", [("grid64", 6), ("road1m", 2)])
def test_scipy_dijkstra_with_limit(name, nsrc):
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import dijkstra

    g = synth.config_graph(name)
    A = csr_matrix((g.w.astype(np.float64), (g.tail.astype(np.int64), g.head.astype(np.int64))),
                   shape=(g.n, g.n))
    assert A.nnz == g.m                      # arcs are simple: nothing summed or dropped
    orc = Oracle.from_graph(g)
    srcs, taus = synth.config_queries(name, nsrc)
    for s, tau in zip(srcs.tolist(), taus.tolist()):
        ref = dijkstra(A, directed=True, indices=s, limit=float(tau))
        _, dist, _ = orc.isochrone(s, tau, want_dist=True)
        fin = np.isfinite(ref)
        assert np.all(ref[fin] <= tau)
        np.testing.assert_array_equal(dist != INF, fin)
        np.testing.assert_array_equal(dist[fin], ref[fin].astype(np.uint64))
        # unbounded distances against scipy without a limit (small graph only)
        if g.n <= 10_000:
            full = dijkstra(A, directed=True, indices=s)
            d = orc.distances(s)
            ff = np.isfinite(full)
            np.testing.assert_array_equal(d != INF, ff)
            np.testing.assert_array_equal(d[ff], full[ff].astype(np.uint64))


# ---------------------------------------------------------------- closed form
@pytest.mark.parametrize("c", [1, 7])
def test_uniform_grid_closed_form(c):
    W, cx = 41, 20
    g = synth.uniform_grid(W, c)
    orc = Oracle.from_graph(g)
    s = cx * W + cx
    ys, xs = np.divmod(np.arange(W * W), W)
    l1 = np.abs(xs - cx) + np.abs(ys - cx)
    np.testing.assert_array_equal(orc.distances(s), (c * l1).astype(np.uint64))
    for r in range(0, 20):
        for tau in (c * r, c * r + c - 1):
            edges, _, settled = orc.isochrone(s, tau)
            assert len(edges) == 8 * (2 * r + 1), (r, tau)
            assert settled == 2 * r * (r + 1) + 1          # |{L1 <= r}| in Z^2
            np.testing.assert_array_equal(orc.in_range(s, tau), np.flatnonzero(l1 <= r).astype(np.uint32))
            lt, lh = l1[edges[:, 0]], l1[edges[:, 1]]
            assert np.all(np.minimum(lt, lh) == r) and np.all(np.maximum(lt, lh) == r + 1)


# ---------------------------------------------------------------- special limits
@pytest.mark.parametrize("name", ["grid64"])
def test_tau_zero_is_star_of_source(name):
    g = synth.config_graph(name)
    assert g.w.min() >= 1
    orc = Oracle.from_graph(g)
    for s in [0, 1, 63, 2080, 4095]:
        edges, _, settled = orc.isochrone(s, 0)
        assert settled == 1
        np.testing.assert_array_equal(orc.in_range(s, 0), [s])
        star = {(s, int(h)) for h in g.head[g.tail == s]} | {(int(t), s) for t in g.tail[g.head == s]}
        assert set(map(tuple, edges.tolist())) == star


def test_random_simple_tau_zero():
    for seed in range(10):
        g = synth.random_digraph(30, 90, seed=seed, zero_frac=0.0, simple=True)
        orc = Oracle.from_graph(g)
        s = seed % 30
        edges, _, _ = orc.isochrone(s, 0)
        star = {(s, int(h)) for h in g.head[g.tail == s]} | {(int(t), s) for t in g.tail[g.head == s]}
        assert set(map(tuple, edges.tolist())) == star


def test_tau_exact_hit_is_in_range():
    g = synth.config_graph("grid64")
    orc = Oracle.from_graph(g)
    s = 1234
    d = orc.distances(s)
    rng = np.random.default_rng(5)
    for v in rng.integers(0, g.n, size=20).tolist():
        dv = int(d[v])
        _, dist, _ = orc.isochrone(s, dv, want_dist=True)
        assert dist[v] == dv
        if dv > 0:
            _, dist, _ = orc.isochrone(s, dv - 1, want_dist=True)
            assert dist[v] == INF


def test_tau_beyond_every_distance():
    g = synth.config_graph("grid64")        # strongly connected
    orc = Oracle.from_graph(g)
    d = orc.distances(7)
    assert np.all(d != INF)
    edges, _, settled = orc.isochrone(7, int(d.max()))
    assert settled == g.n and len(edges) == 0
    np.testing.assert_array_equal(orc.in_range(7, int(d.max())), np.arange(g.n, dtype=np.uint32))
    # with unreachable vertices the only survivors are arcs entering the reachable part
    for seed in range(8):
        rg = synth.random_digraph(25, 40, seed=100 + seed, zero_frac=0.0, simple=True)
        o2 = Oracle.from_graph(rg)
        dd = o2.distances(0)
        top = int(dd[dd != INF].max())
        edges, _, _ = o2.isochrone(0, top + 5)
        reach = dd != INF
        want = sorted((int(t), int(h)) for t, h in zip(rg.tail, rg.head) if reach[h] and not reach[t])
        assert [tuple(e) for e in edges.tolist()] == want


# ---------------------------------------------------------------- paper examples
def test_fig2_right_reconstruction():
    f = golden_io.load("fig2_right.txt")
    orc = Oracle(f["n"], f["tail"], f["head"], f["w"])
    edges, dist, _ = orc.isochrone(f["source"], f["tau"], want_dist=True)
    np.testing.assert_array_equal(edges, f["expect"])
    np.testing.assert_array_equal(orc.distances(f["source"]), f["dist"])
    assert (2, 3) not in set(map(tuple, edges.tolist()))      # (v, w) lies inside the range


def test_fig2_left_mountain_reconstruction():
    f = golden_io.load("fig2_left_mountain.txt")
    orc = Oracle(f["n"], f["tail"], f["head"], f["w"])
    edges, _, _ = orc.isochrone(f["source"], f["tau"])
    np.testing.assert_array_equal(edges, f["expect"])
    np.testing.assert_array_equal(orc.distances(f["source"]), f["dist"])
    e2, _ = orc.iso_dijkstra(f["source"], f["tau"])
    np.testing.assert_array_equal(e2, f["expect"])


# ---------------------------------------------------------------- invariants
@pytest.mark.parametrize("name,nq", [("grid64", 8), ("road1m", 2)])
def test_invariants(name, nq):
    g = synth.config_graph(name)
    orc = Oracle.from_graph(g)
    srcs, taus = synth.config_queries(name, nq)
    t64, h64, w64 = g.tail.astype(np.int64), g.head.astype(np.int64), g.w.astype(np.uint64)
    for s, tau in zip(srcs.tolist(), taus.tolist()):
        edges, dist, _ = orc.isochrone(s, tau, want_dist=True)
        inr = dist != INF
        assert dist[s] == 0                                           # I1
        # I2: no arc leaves the settled set with d(u) + w <= tau, and labels are consistent
        u_in = inr[t64]
        reach = dist[t64[u_in]] + w64[u_in]
        hv = dist[h64[u_in]]
        assert np.all((hv == INF) & (reach > tau) | (hv != INF) & (hv <= reach))
        # I3: every settled v != s has an in-arc with d(v) = d(u) + w
        tight = np.zeros(g.n, dtype=bool)
        both = inr[t64] & inr[h64]
        ok = both & (dist[h64] == dist[t64] + w64)
        tight[h64[ok]] = True
        tight[s] = True
        assert np.all(tight[inr])
        # I4: output = exactly the straddling arcs
        strad = inr[t64] != inr[h64]
        want = np.stack([g.tail[strad], g.head[strad]], axis=1)
        np.testing.assert_array_equal(edges, want)      # arcs are sorted by (tail, head)
        # I5: reversal closure
        eset = set(map(tuple, edges.tolist()))
        arcset = set(zip(g.tail.tolist(), g.head.tolist()))
        for (a, b) in list(eset)[:5000]:
            if (b, a) in arcset:
                assert (b, a) in eset
        # I7: monotone in tau
        _, d_lo, _ = orc.isochrone(s, tau // 2, want_dist=True)
        assert np.all(inr[d_lo != INF])


# ------------------------------------------------------------------ isochrone polygon (Section 7)

def signed_area(g, cycle):
    """Shoelace area of the polygon through the midpoints of a cycle's boundary edges."""
    p = 0.5 * (g.xy[cycle[:, 0]] + g.xy[cycle[:, 1]])
    x, y = p[:, 0], p[:, 1]
    return 0.5 * float(np.sum(x * np.roll(y, -1) - np.roll(x, -1) * y))


def grid_with_slow_block(W, c, block):
    """Uniform W x W grid (weight c) whose arcs touching the `block` vertices weigh c * 10^6."""
    g = synth.uniform_grid(W, c)
    slow = np.zeros(g.n, dtype=bool)
    slow[block] = True
    w = g.w.astype(np.uint64)
    w[slow[g.tail] | slow[g.head]] *= 1_000_000
    return synth.Graph(g.n, g.tail, g.head, w.astype(np.uint32), g.xy)


def polygon_pins_pass(libpath=None) -> bool:
    """Closed forms of the polygon on a uniform grid: the in-range set of a source far from the
    border is an L1 ball of radius r, bounded by one cycle of 4(2r+1) darts; a block of slow
    vertices strictly inside the ball and off both axes through the source (so that no other
    distance changes: an L-shaped path avoids it) adds a second cycle of 2(k + l) darts around a
    k x l block.  The walk keeps the region on its left, so the outer cycle runs counterclockwise
    (positive area in x-right, y-up coordinates) and a hole's cycle clockwise."""
    W, c = 25, 10
    s = 12 * W + 12
    g = synth.uniform_grid(W, c)
    orc = Oracle.from_graph(g, libpath)
    for r in range(0, 9):
        cyc = orc.polygon(g.xy, orc.in_range(s, c * r))
        if len(cyc) != 1 or len(cyc[0]) != 4 * (2 * r + 1):
            return False
        if r > 0 and signed_area(g, cyc[0]) <= 0:
            return False
    bx, by = np.meshgrid(np.arange(14, 16), np.arange(15, 18))   # a 2 x 3 block at offsets (2..3, 3..5)
    block = (by * W + bx).ravel()
    gb = grid_with_slow_block(W, c, block)
    ob = Oracle.from_graph(gb, libpath)
    r = 9
    inr = ob.in_range(s, c * r)
    if not np.array_equal(np.sort(inr), np.sort(np.setdiff1d(orc.in_range(s, c * r), block))):
        return False
    cyc = ob.polygon(gb.xy, inr)
    if sorted(len(x) for x in cyc) != [2 * (2 + 3), 4 * (2 * r + 1)]:
        return False
    outer, hole = sorted(cyc, key=len, reverse=True)
    return signed_area(gb, outer) > 0 > signed_area(gb, hole)


def test_polygon_closed_forms():
    assert polygon_pins_pass()


@pytest.mark.parametrize("seed", range(4))
def test_polygon_partitions_the_boundary(seed):
    """On the jittered planar grid: the cycles hold every dart (u in range, v not, u and v
    neighbours in either direction) exactly once, so the polygon covers the isochrone edges."""
    g = synth.config_graph("grid64")
    orc = Oracle.from_graph(g)
    rng = np.random.default_rng(seed)
    for s, tau in zip(rng.integers(0, g.n, size=5), rng.integers(0, 9000, size=5)):
        inr = orc.in_range(int(s), int(tau))
        cyc = orc.polygon(g.xy, inr)
        got = np.concatenate(cyc) if cyc else np.zeros((0, 2), np.uint32)
        key = got[:, 0].astype(np.int64) << 32 | got[:, 1].astype(np.int64)
        assert len(np.unique(key)) == len(key)
        mark = np.zeros(g.n, dtype=bool)
        mark[inr] = True
        u = np.concatenate([g.tail, g.head]).astype(np.int64)
        v = np.concatenate([g.head, g.tail]).astype(np.int64)
        want = np.unique((u << 32 | v)[mark[u] & ~mark[v]])
        np.testing.assert_array_equal(np.sort(key), want)
        for cy in cyc:   # each cycle starts at its smallest dart; cycles ordered by it
            k = cy[:, 0].astype(np.int64) << 32 | cy[:, 1].astype(np.int64)
            assert k[0] == k.min()
        firsts = [int(cy[0, 0]) << 32 | int(cy[0, 1]) for cy in cyc]
        assert firsts == sorted(firsts)
        # the isochrone edges are exactly the arcs of these darts, in either direction
        edges, _, _ = orc.isochrone(int(s), int(tau))
        ek = edges[:, 0].astype(np.int64) << 32 | edges[:, 1].astype(np.int64)
        und = np.unique(np.concatenate([key, (key & 0xFFFFFFFF) << 32 | key >> 32]))
        assert np.isin(ek, und).all()
