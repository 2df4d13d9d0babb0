"""ctypes binding of libiso.so (include/iso.h).  Argument marshalling only:
every step of a query runs inside the native library and its HIP kernels.
"""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libiso.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "iso.h")

ISO_OK, ISO_EINVAL, ISO_ENOMEM, ISO_EDEVICE, ISO_EFORMAT, ISO_EBUSY, ISO_ESTATE, ISO_EAGAIN, ISO_ESPACE = \
    0, -1, -2, -3, -4, -6, -7, -8, -9
MODE_PLAIN, MODE_CELLS, MODE_CD = 0, 1, 2
INF = 0xFFFFFFFF
TAU_MAX = 0xFFFFFFFE


class IsoError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (status {code})")
        self.code = code


class GraphDesc(C.Structure):
    _fields_ = [("n", C.c_uint32), ("m", C.c_uint64),
                ("tail", C.POINTER(C.c_uint32)), ("head", C.POINTER(C.c_uint32)),
                ("weight", C.POINTER(C.c_uint32)), ("xy", C.POINTER(C.c_double)),
                ("cell_of", C.POINTER(C.c_uint32)), ("num_cells", C.c_uint32),
                ("max_cell_size", C.c_uint32), ("prep_path", C.c_char_p),
                ("device", C.c_int), ("threads", C.c_int), ("verbose", C.c_int)]


class GraphInfo(C.Structure):
    _fields_ = [("n", C.c_uint32), ("n_core", C.c_uint32), ("num_cells", C.c_uint32),
                ("core_levels", C.c_uint32), ("max_cell_levels", C.c_uint32),
                ("max_cell_internal", C.c_uint32), ("m", C.c_uint64), ("down_arcs", C.c_uint64),
                ("up_arcs", C.c_uint64), ("shortcuts", C.c_uint64), ("device_bytes", C.c_uint64),
                ("prep_seconds", C.c_double), ("host_threads", C.c_uint32), ("top_table", C.c_uint32)]


class QueryStats(C.Structure):
    _fields_ = [("lanes", C.c_uint32), ("active_cells", C.c_uint32), ("swept_vertices", C.c_uint64),
                ("edges", C.c_uint64), ("upward_settled", C.c_uint64), ("t_upward_ms", C.c_double),
                ("t_device_ms", C.c_double), ("t_sort_ms", C.c_double), ("t_total_ms", C.c_double)]


class Tuning(C.Structure):
    _fields_ = [("lanes_per_launch", C.c_uint32), ("block", C.c_uint32), ("cell_lds_kb", C.c_uint32),
                ("use_graph", C.c_uint32), ("core_mode", C.c_uint32), ("cell_stage", C.c_uint32),
                ("cell_block", C.c_uint32), ("table_max", C.c_uint32), ("stall", C.c_uint32),
                ("edge_cap", C.c_uint32), ("overlap_cells", C.c_uint32), ("plain_sweep", C.c_uint32)]


_U32P = C.POINTER(C.c_uint32)
_U64P = C.POINTER(C.c_uint64)


class Layout(C.Structure):
    _fields_ = [("perm", _U32P), ("cell_of", _U32P), ("down_off", _U32P), ("down_arc", _U32P),
                ("up_off", _U32P), ("up_head", _U32P), ("up_w", _U32P), ("core_lvl", _U32P),
                ("core_lvl_len", C.c_uint32), ("cell_off", _U32P), ("cell_lvl_ptr", _U32P),
                ("cell_lvl", _U32P), ("cell_lvl_len", C.c_uint32), ("core_cell", _U32P),
                ("core_ecc", _U32P), ("uncovered", C.POINTER(C.c_uint8))]


class Profile(C.Structure):
    _fields_ = [("core_ms", C.c_double), ("active_ms", C.c_double), ("cell_ms", C.c_double),
                ("sort_ms", C.c_double), ("core_launches", C.c_uint64), ("cell_launches", C.c_uint64),
                ("calls", C.c_uint64), ("core_bytes", C.c_uint64), ("cell_bytes", C.c_uint64),
                ("core_entries", C.c_uint64), ("cell_entries", C.c_uint64), ("cell_vertices", C.c_uint64),
                ("cells_swept", C.c_uint64), ("cell_lanes", C.c_uint64), ("cell_items", C.c_uint64),
                ("cell_bytes_survey", C.c_uint64), ("level_ms", C.c_double), ("level_launches", C.c_uint64),
                ("level_bytes", C.c_uint64)]


class Edge(C.Structure):
    _fields_ = [("tail", C.c_uint32), ("head", C.c_uint32)]


class ServerConfig(C.Structure):
    _fields_ = [("max_lanes", C.c_uint32), ("max_inflight", C.c_uint32), ("device_budget", C.c_uint64),
                ("mode", C.c_int)]


class RequestStats(C.Structure):
    _fields_ = [("t_queue_ms", C.c_double), ("t_total_ms", C.c_double), ("batch_lanes", C.c_uint32)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_uint64), ("completed", C.c_uint64), ("sweeps", C.c_uint64),
                ("lanes_total", C.c_uint64), ("contexts", C.c_uint32), ("lanes_cap", C.c_uint32),
                ("queue_depth", C.c_uint32), ("inflight", C.c_uint32), ("ctx_bytes", C.c_uint64),
                ("regrown", C.c_uint64)]


_lib = None


def header_functions(path: str = HEADER) -> list[str]:
    """Names of the functions declared in include/iso.h."""
    src = open(path).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|void|const char \*)\s*\*?\s*(iso_\w+)\s*\(", src, flags=re.M)))


def lib():
    """Load libiso.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
    # PyTorch ships its own HIP runtime (same soname as ROCm's).  Loading it first makes the
    # library bind to that copy, so the process holds one HIP runtime and torch tensors can be
    # handed to the library; a second runtime loaded after ours cannot open the GPU.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(LIB_PATH)
    L.iso_load_graph.argtypes = [C.POINTER(GraphDesc), C.POINTER(C.c_void_p)]
    L.iso_free_graph.argtypes = [C.c_void_p]
    L.iso_free_graph.restype = None
    L.iso_graph_get_info.argtypes = [C.c_void_p, C.POINTER(GraphInfo)]
    L.iso_graph_get_layout.argtypes = [C.c_void_p, C.POINTER(Layout)]
    L.iso_query.argtypes = [C.c_void_p, C.c_uint32, C.c_uint32, C.c_int, C.POINTER(C.POINTER(Edge)),
                            C.POINTER(C.c_size_t)]
    L.iso_query_batch.argtypes = [C.c_void_p, C.c_size_t, _U32P, _U32P, C.c_int, C.POINTER(C.POINTER(Edge)),
                                  C.POINTER(C.c_size_t)]
    L.iso_query_batch_device.argtypes = [C.c_void_p, C.c_size_t, _U32P, _U32P, C.c_int, C.c_void_p, C.c_uint64,
                                         C.c_void_p, C.POINTER(C.c_uint64), C.c_void_p]
    L.iso_query_batch_device_noalloc.argtypes = L.iso_query_batch_device.argtypes
    L.iso_query_batch_vertices_device.argtypes = [C.c_void_p, C.c_size_t, _U32P, _U32P, C.c_int, C.c_void_p,
                                                  C.c_void_p]
    L.iso_query_vertices.argtypes = [C.c_void_p, C.c_uint32, C.c_uint32, C.c_int, C.POINTER(_U32P),
                                     C.POINTER(C.c_size_t)]
    L.iso_query_polygon_batch.argtypes = [C.c_void_p, C.c_size_t, _U32P, _U32P, C.c_int, C.POINTER(C.POINTER(Edge)),
                                          C.POINTER(C.c_size_t), C.POINTER(_U64P), C.POINTER(C.c_size_t)]
    L.iso_query_polygon.argtypes = [C.c_void_p, C.c_uint32, C.c_uint32, C.c_int, C.POINTER(C.POINTER(Edge)),
                                    C.POINTER(C.c_size_t), C.POINTER(_U64P), C.POINTER(C.c_size_t)]
    L.iso_targets_select.argtypes = [C.c_void_p, _U32P, C.c_size_t, C.POINTER(C.c_void_p)]
    L.iso_targets_query.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, _U32P, _U32P]
    L.iso_targets_query_device.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, _U32P, C.c_void_p, C.c_void_p]
    L.iso_targets_get_info.argtypes = [C.c_void_p, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64),
                                       C.POINTER(C.c_uint32), C.POINTER(C.c_double)]
    L.iso_targets_free.argtypes = [C.c_void_p]
    L.iso_targets_free.restype = None
    L.iso_query_distances.argtypes = [C.c_void_p, C.c_uint32, C.c_uint32, C.c_int, _U32P, C.POINTER(C.c_uint8)]
    L.iso_last_query_stats.argtypes = [C.c_void_p, C.POINTER(QueryStats)]
    L.iso_debug_enable.argtypes = [C.c_void_p, C.c_int]
    L.iso_debug_read.argtypes = [C.c_void_p, C.POINTER(C.c_uint64)]
    L.iso_set_tuning.argtypes = [C.c_void_p, C.POINTER(Tuning)]
    L.iso_get_tuning.argtypes = [C.c_void_p, C.POINTER(Tuning)]
    L.iso_profile_enable.argtypes = [C.c_void_p, C.c_int]
    L.iso_profile_read.argtypes = [C.c_void_p, C.POINTER(Profile)]
    L.iso_server_start.argtypes = [C.c_void_p, C.POINTER(ServerConfig), C.POINTER(C.c_void_p)]
    L.iso_server_submit.argtypes = [C.c_void_p, C.c_uint32, C.c_uint32, C.POINTER(C.c_uint64)]
    L.iso_server_wait.argtypes = [C.c_void_p, C.c_uint64, C.c_int, C.POINTER(C.POINTER(Edge)),
                                  C.POINTER(C.c_size_t), C.POINTER(RequestStats)]
    L.iso_server_get_stats.argtypes = [C.c_void_p, C.POINTER(ServerStats)]
    L.iso_server_stop.argtypes = [C.c_void_p]
    L.iso_server_free.argtypes = [C.c_void_p]
    L.iso_server_free.restype = None
    L.iso_free.argtypes = [C.c_void_p]
    L.iso_free.restype = None
    L.iso_last_error.restype = C.c_char_p
    _lib = L
    return L


def _check(rc):
    if rc != ISO_OK:
        raise IsoError(rc, lib().iso_last_error().decode(errors="replace"))


def _u32(a):
    a = np.ascontiguousarray(a, dtype=np.uint32)
    return a, a.ctypes.data_as(_U32P)


class _LibBuffer:
    """Owner of an edge array returned by the library: numpy views keep it alive, and it is
    released with iso_free when the last view goes away (no copy of the result)."""

    def __init__(self, addr: int, count: int):
        self._addr = addr
        self.__array_interface__ = {"data": (addr, False), "shape": (count, 2), "typestr": "<u4",
                                    "version": 3}

    def __del__(self):
        if self._addr:
            lib().iso_free(C.c_void_p(self._addr))
            self._addr = 0


def _edges_to_numpy(ptr, count) -> np.ndarray:
    addr = C.cast(ptr, C.c_void_p).value
    if count == 0:
        if addr:
            lib().iso_free(C.c_void_p(addr))
        return np.zeros((0, 2), dtype=np.uint32)
    return np.asarray(_LibBuffer(addr, count))


class Graph:
    """A preprocessed graph resident on one device (or host-only with device=-1)."""

    def __init__(self, n, tail, head, weight, *, xy=None, cell_of=None, num_cells=0, max_cell_size=0,
                 prep_path=None, device=0, threads=0, verbose=False):
        L = lib()
        t, tp = _u32(tail)
        h, hp = _u32(head)
        w, wp = _u32(weight)
        d = GraphDesc()
        d.n, d.m = int(n), int(t.size)
        d.tail, d.head, d.weight = tp, hp, wp
        keep = [t, h, w]
        if xy is not None:
            xyc = np.ascontiguousarray(xy, dtype=np.float64).reshape(-1)
            keep.append(xyc)
            d.xy = xyc.ctypes.data_as(C.POINTER(C.c_double))
        if cell_of is not None:
            co, cp = _u32(cell_of)
            keep.append(co)
            d.cell_of = cp
        d.num_cells = int(num_cells)
        d.max_cell_size = int(max_cell_size)
        d.prep_path = prep_path.encode() if prep_path else None
        d.device, d.threads, d.verbose = int(device), int(threads), int(bool(verbose))
        h_out = C.c_void_p()
        _check(L.iso_load_graph(C.byref(d), C.byref(h_out)))
        self._h = h_out
        self.n = int(n)

    @classmethod
    def from_synth(cls, g, num_cells=0, **kw):
        return cls(g.n, g.tail, g.head, g.w, xy=g.xy if num_cells else None, num_cells=num_cells, **kw)

    def close(self):
        if getattr(self, "_h", None):
            lib().iso_free_graph(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> dict:
        i = GraphInfo()
        _check(lib().iso_graph_get_info(self._h, C.byref(i)))
        return {f: getattr(i, f) for f, _ in GraphInfo._fields_}

    def layout(self) -> dict:
        """Copies of the preprocessed arrays (see iso_layout in include/iso.h)."""
        Lr = Layout()
        _check(lib().iso_graph_get_layout(self._h, C.byref(Lr)))
        info = self.info()
        n, nc, cells = info["n"], info["n_core"], info["num_cells"]

        def arr(p, k, dt=np.uint32):
            if k == 0 or not p:
                return np.zeros(0, dtype=dt)
            return np.ctypeslib.as_array(p, shape=(k,)).copy()

        down_off = arr(Lr.down_off, n + 1)
        up_off = arr(Lr.up_off, n + 1)
        return dict(perm=arr(Lr.perm, n), cell_of=arr(Lr.cell_of, n), down_off=down_off,
                    down_arc=arr(Lr.down_arc, 2 * int(down_off[-1])).reshape(-1, 2), up_off=up_off,
                    up_head=arr(Lr.up_head, int(up_off[-1])), up_w=arr(Lr.up_w, int(up_off[-1])),
                    core_lvl=arr(Lr.core_lvl, Lr.core_lvl_len),
                    cell_off=arr(Lr.cell_off, cells + 1 if cells else 0),
                    cell_lvl_ptr=arr(Lr.cell_lvl_ptr, cells + 1 if cells else 0),
                    cell_lvl=arr(Lr.cell_lvl, Lr.cell_lvl_len), core_cell=arr(Lr.core_cell, nc),
                    core_ecc=arr(Lr.core_ecc, nc), uncovered=arr(Lr.uncovered, cells, np.uint8),
                    n=n, n_core=nc, num_cells=cells)

    def query(self, source: int, tau: int, mode: int = MODE_PLAIN) -> np.ndarray:
        """Isochrone edges as an (count, 2) uint32 array sorted by (tail, head)."""
        ptr = C.POINTER(Edge)()
        cnt = C.c_size_t()
        _check(lib().iso_query(self._h, int(source), int(tau), int(mode), C.byref(ptr), C.byref(cnt)))
        return _edges_to_numpy(ptr, cnt.value)

    def query_batch(self, sources, taus, mode: int = MODE_PLAIN) -> list[np.ndarray]:
        s, sp = _u32(sources)
        t, tp = _u32(taus)
        k = s.size
        offsets = (C.c_size_t * (k + 1))()
        ptr = C.POINTER(Edge)()
        _check(lib().iso_query_batch(self._h, k, sp, tp, int(mode), C.byref(ptr), offsets))
        total = offsets[k]
        flat = _edges_to_numpy(ptr, total)
        return [flat[offsets[j]:offsets[j + 1]] for j in range(k)]

    def query_batch_device_noalloc(self, sources, taus, mode, pairs, offsets, stream=None) -> int:
        """query_batch_device through iso_query_batch_device_noalloc (no allocation in the call)."""
        return self.query_batch_device(sources, taus, mode, pairs, offsets, stream, noalloc=True)

    def query_batch_device(self, sources, taus, mode, pairs, offsets, stream=None, noalloc=False) -> int:
        """Edges of k queries written to device memory: `pairs` (cap x 2, 32-bit integers) and
        `offsets` (k + 1, 32-bit integers) are contiguous torch tensors on the graph's device;
        `stream` (default: torch's current stream) is waited for before they are written.
        Returns the edge count; raises IsoError with code ISO_ESPACE and `.total` (the count
        needed) when `pairs` is too small."""
        if stream is None:
            import torch
            stream = torch.cuda.current_stream(pairs.device).cuda_stream
        s, sp = _u32(sources)
        t, tp = _u32(taus)
        k = s.size
        for name, x, need in (("pairs", pairs, None), ("offsets", offsets, k + 1)):
            if x.element_size() != 4 or not x.is_contiguous() or x.device.type != "cuda":
                raise IsoError(ISO_EINVAL, f"{name} must be a contiguous 32-bit tensor in device memory")
            if need is not None and x.numel() < need:
                raise IsoError(ISO_EINVAL, f"{name} needs {need} entries")
        total = C.c_uint64()
        fn = lib().iso_query_batch_device_noalloc if noalloc else lib().iso_query_batch_device
        st = fn(self._h, k, sp, tp, int(mode), C.c_void_p(pairs.data_ptr()), pairs.numel() // 2,
                C.c_void_p(offsets.data_ptr()), C.byref(total), C.c_void_p(stream))
        if st == ISO_ESPACE:
            e = IsoError(st, lib().iso_last_error().decode(errors="replace"))
            e.total = total.value
            raise e
        _check(st)
        return total.value

    def query_vertices(self, source: int, tau: int, mode: int = MODE_PLAIN) -> np.ndarray:
        """Vertices with d(source, v) <= tau, sorted original ids (uint32)."""
        ptr = _U32P()
        cnt = C.c_size_t()
        _check(lib().iso_query_vertices(self._h, int(source), int(tau), int(mode), C.byref(ptr), C.byref(cnt)))
        try:
            n = cnt.value
            return np.ctypeslib.as_array(ptr, shape=(n,)).copy() if n else np.zeros(0, dtype=np.uint32)
        finally:
            lib().iso_free(ptr)

    def query_batch_vertices_device(self, sources, taus, mode, bits, stream=None):
        """Vertices in range of k <= 64 queries as bitmaps in `bits`, a contiguous 64-bit torch
        tensor of shape (k, ceil(n / 64)) on the graph's device: bit v % 64 of bits[j, v // 64]
        is set iff vertex v is in range of query j."""
        if stream is None:
            import torch
            stream = torch.cuda.current_stream(bits.device).cuda_stream
        s, sp = _u32(sources)
        t, tp = _u32(taus)
        k, W = s.size, (self.n + 63) // 64
        if bits.element_size() != 8 or not bits.is_contiguous() or bits.device.type != "cuda" or \
                bits.numel() < k * W:
            raise IsoError(ISO_EINVAL, f"bits must be a contiguous 64-bit device tensor of {k} x {W} words")
        _check(lib().iso_query_batch_vertices_device(self._h, k, sp, tp, int(mode), C.c_void_p(bits.data_ptr()),
                                                     C.c_void_p(stream)))

    def polygon_batch_raw(self, sources, taus, mode: int = MODE_PLAIN):
        """iso_query_polygon_batch as flat arrays: darts (total, 2) uint32 in cycle order, dart_off
        (k + 1), cycles (cycle starts into darts, then the total) and cycle_off (k + 1)."""
        s, sp = _u32(sources)
        t, tp = _u32(taus)
        k = s.size
        doff = (C.c_size_t * (k + 1))()
        coff = (C.c_size_t * (k + 1))()
        dp = C.POINTER(Edge)()
        cp = _U64P()
        _check(lib().iso_query_polygon_batch(self._h, k, sp, tp, int(mode), C.byref(dp), doff, C.byref(cp), coff))
        try:
            cyc = np.ctypeslib.as_array(cp, shape=(coff[k] + 1,)).copy()
        finally:
            lib().iso_free(cp)
        darts = _edges_to_numpy(dp, doff[k])
        return darts, np.array(doff[:], dtype=np.int64), cyc.astype(np.int64), np.array(coff[:], dtype=np.int64)

    def polygon_batch(self, sources, taus, mode: int = MODE_PLAIN) -> list[list[np.ndarray]]:
        """Isochrone polygons of k <= 64 queries (iso_query_polygon_batch): per query a list of
        cycles, each an (len, 2) uint32 array of boundary darts (tail in range, head not) in
        cycle order from its smallest dart, the cycles ordered by that dart."""
        darts, doff, cyc, coff = self.polygon_batch_raw(sources, taus, mode)
        return [[darts[cyc[c]:cyc[c + 1]] for c in range(coff[j], coff[j + 1])] for j in range(len(coff) - 1)]

    def polygon(self, source: int, tau: int, mode: int = MODE_PLAIN) -> list[np.ndarray]:
        """The isochrone polygon of one query (iso_query_polygon), as polygon_batch's lists."""
        dp = C.POINTER(Edge)()
        cp = _U64P()
        cnt, nc = C.c_size_t(), C.c_size_t()
        _check(lib().iso_query_polygon(self._h, int(source), int(tau), int(mode), C.byref(dp), C.byref(cnt),
                                       C.byref(cp), C.byref(nc)))
        try:
            cyc = np.ctypeslib.as_array(cp, shape=(nc.value + 1,)).copy()
        finally:
            lib().iso_free(cp)
        flat = _edges_to_numpy(dp, cnt.value)
        return [flat[int(cyc[c]):int(cyc[c + 1])] for c in range(nc.value)]

    def select_targets(self, targets) -> "Targets":
        """RPHAST target selection for a one-to-many target set (original ids)."""
        return Targets(self, targets)

    def distances(self, source: int, tau: int, mode: int = MODE_PLAIN):
        """(dist uint32[n] with 2^32-1 where not labelled, swept bool[n])."""
        dist = np.empty(self.n, dtype=np.uint32)
        swept = np.empty(self.n, dtype=np.uint8)
        _check(lib().iso_query_distances(self._h, int(source), int(tau), int(mode),
                                         dist.ctypes.data_as(_U32P), swept.ctypes.data_as(C.POINTER(C.c_uint8))))
        return dist, swept.astype(bool)

    def debug_enable(self, enable: bool = True):
        _check(lib().iso_debug_enable(self._h, int(bool(enable))))

    def debug_read(self) -> list[int]:
        """Branch counters (iso_debug_read in include/iso.h)."""
        out = (C.c_uint64 * 8)()
        _check(lib().iso_debug_read(self._h, out))
        return list(out)

    def last_stats(self) -> dict:
        s = QueryStats()
        _check(lib().iso_last_query_stats(self._h, C.byref(s)))
        return {f: getattr(s, f) for f, _ in QueryStats._fields_}

    def set_tuning(self, lanes_per_launch=64, block=256, cell_lds_kb=64, use_graph=1, core_mode=0, cell_stage=2,
                   cell_block=0, table_max=0, stall=1, edge_cap=0, overlap_cells=0, plain_sweep=0):
        t = Tuning(lanes_per_launch, block, cell_lds_kb, use_graph, core_mode, cell_stage, cell_block, table_max,
                   stall, edge_cap, overlap_cells, plain_sweep)
        _check(lib().iso_set_tuning(self._h, C.byref(t)))

    def profile_enable(self, enable: bool = True):
        _check(lib().iso_profile_enable(self._h, int(bool(enable))))

    def profile_read(self) -> dict:
        p = Profile()
        _check(lib().iso_profile_read(self._h, C.byref(p)))
        return {f: getattr(p, f) for f, _ in Profile._fields_}

    def get_tuning(self) -> dict:
        t = Tuning()
        _check(lib().iso_get_tuning(self._h, C.byref(t)))
        return {f: getattr(t, f) for f, _ in Tuning._fields_}


class Targets:
    """A selected target set (iso_targets): distances from any sources to its targets."""

    def __init__(self, graph: "Graph", targets):
        t, tp = _u32(targets)
        self.graph, self.count, self._h = graph, int(t.size), C.c_void_p()
        _check(lib().iso_targets_select(graph._h, tp, t.size, C.byref(self._h)))

    def info(self) -> dict:
        v, a, g, ms = C.c_uint64(), C.c_uint64(), C.c_uint32(), C.c_double()
        _check(lib().iso_targets_get_info(self._h, C.byref(v), C.byref(a), C.byref(g), C.byref(ms)))
        return {"vertices": v.value, "arcs": a.value, "groups": g.value, "select_ms": ms.value}

    def query(self, sources) -> np.ndarray:
        """(k, count) uint32: d(sources[j], targets[i]), 2^32-1 where unreachable."""
        s, sp = _u32(sources)
        out = np.empty((s.size, self.count), dtype=np.uint32)
        _check(lib().iso_targets_query(self.graph._h, self._h, s.size, sp, out.ctypes.data_as(_U32P)))
        return out

    def query_device(self, sources, dist, stream=None):
        """The same into `dist`, a contiguous 32-bit torch tensor of k * count entries on the device."""
        if stream is None:
            import torch
            stream = torch.cuda.current_stream(dist.device).cuda_stream
        s, sp = _u32(sources)
        if dist.element_size() != 4 or not dist.is_contiguous() or dist.device.type != "cuda" or \
                dist.numel() < s.size * self.count:
            raise IsoError(ISO_EINVAL, f"dist must be a contiguous 32-bit device tensor of {s.size * self.count} entries")
        _check(lib().iso_targets_query_device(self.graph._h, self._h, s.size, sp, C.c_void_p(dist.data_ptr()),
                                              C.c_void_p(stream)))

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().iso_targets_free(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Serving loop with continuous batching on a resident graph (iso_server_* in include/iso.h)."""

    def __init__(self, graph: Graph, max_lanes=64, max_inflight=2, device_budget=0, mode=MODE_CELLS):
        cfg = ServerConfig(int(max_lanes), int(max_inflight), int(device_budget), int(mode))
        h = C.c_void_p()
        _check(lib().iso_server_start(graph._h, C.byref(cfg), C.byref(h)))
        self._h = h
        self._graph = graph

    def submit(self, source: int, tau: int) -> int:
        t = C.c_uint64()
        _check(lib().iso_server_submit(self._h, int(source), int(tau), C.byref(t)))
        return t.value

    def wait(self, ticket: int, timeout_ms: int = -1):
        """(edges (count, 2) uint32, stats dict); raises IsoError (code ISO_EAGAIN if not ready)."""
        ptr = C.POINTER(Edge)()
        cnt = C.c_size_t()
        st = RequestStats()
        _check(lib().iso_server_wait(self._h, int(ticket), int(timeout_ms), C.byref(ptr), C.byref(cnt),
                                     C.byref(st)))
        return _edges_to_numpy(ptr, cnt.value), {f: getattr(st, f) for f, _ in RequestStats._fields_}

    def stats(self) -> dict:
        s = ServerStats()
        _check(lib().iso_server_get_stats(self._h, C.byref(s)))
        return {f: getattr(s, f) for f, _ in ServerStats._fields_}

    def stop(self):
        if getattr(self, "_h", None):
            _check(lib().iso_server_stop(self._h))

    def close(self):
        if getattr(self, "_h", None):
            lib().iso_server_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
