"""Seeded generators for road-like test graphs and isochrone query lists.

Every graph is returned as a plain directed arc list (tail, head, weight) of
uint32 values over vertex ids 0..n-1, sorted by (tail, head), with self-loops
dropped and parallel arcs merged to their minimum weight.  Weights are integer
travel times: grid units for the small jittered grid, milliseconds for the
road-like kNN graphs.  The generators draw numbers only; they compute no
distances.

Workload recipes (sizes and distributions of the road networks the method is
evaluated on, Section 6; the continental graph itself is not available, so the
kNN generator stands in for it at the same vertex count):

* ``grid64``  - 64x64 grid, coordinates jittered by U(-0.3, 0.3) per axis,
  4-neighbour arcs in both directions, weight = round(100 * euclidean length)
  times a road-class factor in {1, 2, 4} (probabilities 0.2 / 0.5 / 0.3) drawn
  independently for every directed arc.
* ``road1m`` / ``road18m`` - points uniform in a 1000 km x 1000 km square; each
  point linked both ways to its 3 nearest neighbours (local roads, 30 km/h);
  every 16th point linked to its 4 nearest points of that subset (arterials,
  80 km/h); every 256th point linked to its 4 nearest of that subset (highways,
  120 km/h); weight = max(1, round(length_m * 3600 / speed_kmh)) milliseconds.
"""
from __future__ import annotations

import os
from dataclasses import dataclass, field

import numpy as np

U32_MAX = np.uint64(0xFFFFFFFF)


@dataclass
class Graph:
    n: int
    tail: np.ndarray
    head: np.ndarray
    w: np.ndarray
    xy: np.ndarray | None = None
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return int(self.tail.shape[0])


def _round_half_away(x: np.ndarray) -> np.ndarray:
    """Round non-negative float64 values half away from zero (C ``llround``)."""
    f = np.floor(x)
    return np.where(x - f >= 0.5, f + 1.0, f)


def _simplify(n, tail, head, w):
    """Drop self-loops; merge parallel arcs keeping the minimum weight; sort by (tail, head)."""
    tail = np.asarray(tail, dtype=np.uint64)
    head = np.asarray(head, dtype=np.uint64)
    w = np.asarray(w, dtype=np.uint64)
    keep = tail != head
    tail, head, w = tail[keep], head[keep], w[keep]
    key = (tail << np.uint64(32)) | head
    order = np.argsort(key, kind="stable")
    key = key[order]
    w = w[order]
    if key.size == 0:
        z = np.zeros(0, dtype=np.uint32)
        return z, z.copy(), z.copy()
    starts = np.flatnonzero(np.concatenate(([True], key[1:] != key[:-1])))
    wmin = np.minimum.reduceat(w, starts)
    key = key[starts]
    return ((key >> np.uint64(32)).astype(np.uint32),
            (key & U32_MAX).astype(np.uint32),
            wmin.astype(np.uint32))


def _undirected_to_arcs(n, a, b, w):
    """Emit both directions of undirected links and simplify."""
    return _simplify(n, np.concatenate([a, b]), np.concatenate([b, a]), np.concatenate([w, w]))


def grid_graph(W: int = 64, H: int = 64, seed: int = 1) -> Graph:
    """Jittered 4-neighbour grid with per-directed-arc road-class factors (vertex id = y*W + x)."""
    rng = np.random.default_rng(seed)
    gx, gy = np.meshgrid(np.arange(W, dtype=np.float64), np.arange(H, dtype=np.float64))
    x = gx.ravel() + rng.uniform(-0.3, 0.3, size=W * H)
    y = gy.ravel() + rng.uniform(-0.3, 0.3, size=W * H)
    ids = np.arange(W * H, dtype=np.int64).reshape(H, W)
    # horizontal and vertical neighbour pairs, each as two directed arcs
    a = np.concatenate([ids[:, :-1].ravel(), ids[:-1, :].ravel()])
    b = np.concatenate([ids[:, 1:].ravel(), ids[1:, :].ravel()])
    tail = np.concatenate([a, b])
    head = np.concatenate([b, a])
    length = np.hypot(x[tail] - x[head], y[tail] - y[head])
    factor = rng.choice(np.array([1, 2, 4], dtype=np.int64), size=tail.size, p=[0.2, 0.5, 0.3])
    w = _round_half_away(100.0 * length).astype(np.int64) * factor
    t, h, ww = _simplify(W * H, tail, head, w)
    return Graph(W * H, t, h, ww, np.stack([x, y], axis=1), name=f"grid{W}x{H}-s{seed}")


def uniform_grid(W: int, c: int) -> Graph:
    """Un-jittered W x W 4-neighbour grid, every arc of weight c (vertex id = y*W + x)."""
    ids = np.arange(W * W, dtype=np.int64).reshape(W, W)
    a = np.concatenate([ids[:, :-1].ravel(), ids[:-1, :].ravel()])
    b = np.concatenate([ids[:, 1:].ravel(), ids[1:, :].ravel()])
    t, h, w = _undirected_to_arcs(W * W, a, b, np.full(a.size, c, dtype=np.int64))
    gx, gy = np.meshgrid(np.arange(W, dtype=np.float64), np.arange(W, dtype=np.float64))
    return Graph(W * W, t, h, w, np.stack([gx.ravel(), gy.ravel()], axis=1), name=f"ugrid{W}-c{c}")


def _knn_pairs(xy: np.ndarray, k: int):
    """Undirected (i, j, euclidean length) links from every point to its k nearest other points."""
    from scipy.spatial import cKDTree

    tree = cKDTree(xy)
    dist, idx = tree.query(xy, k=k + 1, workers=-1)
    n = xy.shape[0]
    src = np.repeat(np.arange(n, dtype=np.int64), k + 1).reshape(n, k + 1)
    notself = idx != src
    # keep the first k non-self neighbours of each row (a coincident twin may precede self)
    rank = np.cumsum(notself, axis=1)
    sel = notself & (rank <= k)
    return src[sel], idx[sel].astype(np.int64), dist[sel]


def road_graph(n: int, seed: int, side_m: float = 1.0e6, oneway_frac: float = 0.0) -> Graph:
    """Road-like kNN graph with local / arterial / highway classes (weights in ms).

    ``oneway_frac`` > 0 removes that fraction of directed arcs at random after the
    build (used only by robustness tests to create one-way roads).
    """
    rng = np.random.default_rng(seed)
    xy = rng.uniform(0.0, side_m, size=(n, 2))
    links_a, links_b, links_w = [], [], []
    for stride, k, speed in ((1, 3, 30.0), (16, 4, 80.0), (256, 4, 120.0)):
        sub = np.arange(0, n, stride, dtype=np.int64)
        if sub.size < k + 1:
            continue
        i, j, length = _knn_pairs(xy[sub], k)
        ms = np.maximum(1.0, _round_half_away(length * 3600.0 / speed))
        links_a.append(sub[i])
        links_b.append(sub[j])
        links_w.append(ms.astype(np.int64))
    a = np.concatenate(links_a)
    b = np.concatenate(links_b)
    w = np.concatenate(links_w)
    t, h, ww = _undirected_to_arcs(n, a, b, w)
    if oneway_frac > 0.0:
        keep = rng.uniform(size=t.size) >= oneway_frac
        t, h, ww = t[keep], h[keep], ww[keep]
    return Graph(n, t, h, ww, xy, name=f"road{n}-s{seed}" + (f"-ow{oneway_frac}" if oneway_frac else ""))


def random_digraph(n: int, m: int, seed: int, wmax: int = 20, zero_frac: float = 0.1,
                   simple: bool = False) -> Graph:
    """Uniform random directed multigraph (self-loops and parallel arcs kept unless ``simple``)."""
    rng = np.random.default_rng(seed)
    tail = rng.integers(0, n, size=m, dtype=np.int64)
    head = rng.integers(0, n, size=m, dtype=np.int64)
    w = rng.integers(1, wmax + 1, size=m, dtype=np.int64)
    w[rng.uniform(size=m) < zero_frac] = 0
    if simple:
        t, h, ww = _simplify(n, tail, head, w)
    else:
        t, h, ww = tail.astype(np.uint32), head.astype(np.uint32), w.astype(np.uint32)
    xy = rng.uniform(0.0, 1.0, size=(n, 2))
    return Graph(n, t, h, ww, xy, name=f"rand{n}x{m}-s{seed}")


# ---------------------------------------------------------------------------
# named workloads
# ---------------------------------------------------------------------------
CONFIGS = {
    # tiny plain query: one seeded source, tau = 2000 grid units
    "grid64": dict(kind="grid", W=64, graph_seed=1, query_seed=11, cells=16,
                   tau_fixed=[2000]),
    # 1M-vertex plain query, tau in {10, 30, 60} min, 2^12 cells
    "road1m": dict(kind="road", n=1_000_000, graph_seed=2, query_seed=12, cells=1 << 12,
                   tau_fixed=[600_000, 1_800_000, 3_600_000]),
    # continental scale: 18M vertices, 2^14 cells, tau uniform in [10, 240] min
    "road18m": dict(kind="road", n=18_000_000, graph_seed=3, query_seed=13, cells=1 << 14,
                    tau_range=(600_000, 14_400_000)),
}


def _cache_dir() -> str:
    d = os.environ.get("ISO_SYNTH_CACHE", "/tmp/iso_synth_cache")
    os.makedirs(d, exist_ok=True)
    return d


def config_graph(name: str, cache: bool = True) -> Graph:
    cfg = CONFIGS[name]
    path = os.path.join(_cache_dir(), f"{name}-v1.npz")
    if cache and os.path.exists(path):
        z = np.load(path, allow_pickle=False)
        return Graph(int(z["n"]), z["tail"], z["head"], z["w"], z["xy"], name=name)
    if cfg["kind"] == "grid":
        g = grid_graph(cfg["W"], cfg["W"], cfg["graph_seed"])
    else:
        g = road_graph(cfg["n"], cfg["graph_seed"])
    g.name = name
    if cache:
        tmp = path + f".tmp{os.getpid()}.npz"
        np.savez(tmp, n=g.n, tail=g.tail, head=g.head, w=g.w, xy=g.xy)
        os.replace(tmp, path)
    return g


def config_queries(name: str, count: int, seed: int | None = None):
    """(sources uint32[count], taus uint32[count]) for a named workload."""
    cfg = CONFIGS[name]
    n = cfg["n"] if cfg["kind"] == "road" else cfg["W"] * cfg["W"]
    rng = np.random.default_rng(cfg["query_seed"] if seed is None else seed)
    src = rng.integers(0, n, size=count, dtype=np.int64).astype(np.uint32)
    if "tau_range" in cfg:
        lo, hi = cfg["tau_range"]
        tau = rng.integers(lo, hi + 1, size=count, dtype=np.int64).astype(np.uint32)
    else:
        fixed = np.asarray(cfg["tau_fixed"], dtype=np.uint32)
        tau = fixed[np.arange(count) % fixed.size]
    return src, tau


def batch_queries(n: int, count: int, seed: int = 14, lo_min: int = 10, hi_min: int = 240):
    """Batched form: sources uniform over V, tau uniform integer ms in [lo_min, hi_min] minutes."""
    rng = np.random.default_rng(seed)
    src = rng.integers(0, n, size=count, dtype=np.int64).astype(np.uint32)
    tau = rng.integers(lo_min * 60_000, hi_min * 60_000 + 1, size=count, dtype=np.int64)
    return src, tau.astype(np.uint32)


def serving_trace(n: int, rate_hz: float, duration_s: float, seed: int = 15,
                  lo_min: float = 5.0, hi_min: float = 300.0):
    """Poisson arrival times (s), uniform sources and log-uniform tau (ms) for the serving loop."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, size=int(rate_hz * duration_s * 1.5) + 16)
    t = np.cumsum(gaps)
    t = t[t < duration_s]
    cnt = t.size
    src = rng.integers(0, n, size=cnt, dtype=np.int64).astype(np.uint32)
    tau = _round_half_away(np.exp(rng.uniform(np.log(lo_min), np.log(hi_min), size=cnt)) * 60_000.0)
    return t, src, tau.astype(np.uint32)


def target_ball(g: Graph, size: int, seed: int = 16):
    """A compact target set for one-to-many queries: a random centre c and the first `size`
    vertices of a breadth-first traversal from c over the outgoing arcs (hop count, no
    lengths).  Stands in for the paper's forward Dijkstra ball of the same size.  Returns
    (c, targets) with the targets in traversal order (c first); fewer than `size` if c reaches
    fewer vertices."""
    rng = np.random.default_rng(seed)
    n = g.n
    tail, head = g.tail, g.head
    if tail.size and np.any(tail[1:] < tail[:-1]):
        order = np.argsort(tail, kind="stable")
        tail, head = tail[order], head[order]
    off = np.searchsorted(tail, np.arange(n + 1, dtype=np.int64)).astype(np.int64)
    c = int(rng.integers(0, n))
    seen = {c}
    out = [c]
    frontier = [c]
    while len(out) < size and frontier:
        nxt = []
        for v in frontier:
            for x in head[off[v]:off[v + 1]].tolist():
                if x not in seen:
                    seen.add(x)
                    nxt.append(x)
        out.extend(nxt)
        frontier = nxt
    return c, np.array(out[:size], dtype=np.uint32)
