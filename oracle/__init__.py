"""CPU oracle for isochrone queries - TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  The product library never loads it.  The C source
(``oracle.c``) is a plain transcription of the paper's definitions (Dijkstra,
Section 2; problem statement and isoDijkstra, Section 3) in 64-bit integer
arithmetic; this module only marshals arguments.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC_PATH = os.path.join(_HERE, "oracle.c")
INF = np.uint64(0xFFFFFFFFFFFFFFFF)


def build(force: bool = False, src: str = SRC_PATH, out: str = LIB_PATH) -> str:
    """Compile oracle.c with gcc into a shared library (plain -O2, no vectorisation tricks)."""
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(src):
        tmp = out + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-shared", "-fPIC", "-o", tmp, src, "-lm"])
        os.replace(tmp, out)
    return out


_P = C.c_void_p
_U32P = C.POINTER(C.c_uint32)
_U64P = C.POINTER(C.c_uint64)


def _load(path: str):
    lib = C.CDLL(path)
    lib.orc_graph_new.restype = _P
    lib.orc_graph_new.argtypes = [C.c_uint32, C.c_uint64, _U32P, _U32P, _U32P]
    lib.orc_graph_free.argtypes = [_P]
    lib.orc_ws_new.restype = _P
    lib.orc_ws_new.argtypes = [C.c_uint32]
    lib.orc_ws_free.argtypes = [_P]
    lib.orc_isochrone.restype = C.c_uint64
    lib.orc_isochrone.argtypes = [_P, _P, C.c_uint32, C.c_uint64, _U64P, C.POINTER(_U64P), _U64P]
    lib.orc_distances.restype = C.c_uint64
    lib.orc_distances.argtypes = [_P, _P, C.c_uint32, _U64P]
    lib.orc_edges_by_definition.argtypes = [_P, _U64P, C.c_uint64, C.POINTER(_U64P), _U64P]
    lib.orc_iso_dijkstra.restype = C.c_uint64
    lib.orc_iso_dijkstra.argtypes = [_P, _P, C.c_uint32, C.c_uint64, C.POINTER(_U64P), _U64P]
    lib.orc_in_range.restype = C.c_uint64
    lib.orc_in_range.argtypes = [_P, _P, C.c_uint32, C.c_uint64, C.POINTER(_U32P)]
    lib.orc_polygon.restype = C.c_uint64
    lib.orc_polygon.argtypes = [_P, C.POINTER(C.c_double), C.POINTER(C.c_uint8), C.POINTER(_U64P),
                                C.POINTER(_U64P), _U64P]
    lib.orc_free.argtypes = [_P]
    return lib


_LIB = None


def lib(path: str | None = None):
    global _LIB
    if path is not None:
        return _load(path)
    if _LIB is None:
        _LIB = _load(build())
    return _LIB


def _u32(a):
    a = np.ascontiguousarray(a, dtype=np.uint32)
    return a, a.ctypes.data_as(_U32P)


def _take_edges(L, ptr, cnt) -> np.ndarray:
    """Copy the oracle's malloc'ed (tail << 32 | head) keys into an (cnt, 2) uint32 array."""
    n = int(cnt.value)
    if n == 0:
        L.orc_free(ptr)
        return np.zeros((0, 2), dtype=np.uint32)
    keys = np.ctypeslib.as_array(ptr, shape=(n,)).copy()
    L.orc_free(ptr)
    return np.stack([(keys >> np.uint64(32)).astype(np.uint32),
                     (keys & np.uint64(0xFFFFFFFF)).astype(np.uint32)], axis=1)


class Oracle:
    """One graph (original arc list) plus a reusable workspace."""

    def __init__(self, n, tail, head, w, libpath: str | None = None):
        self._L = lib(libpath)
        self.n = int(n)
        t, tp = _u32(tail)
        h, hp = _u32(head)
        ww, wp = _u32(w)
        self._g = self._L.orc_graph_new(self.n, t.size, tp, hp, wp)
        self._ws = self._L.orc_ws_new(self.n)
        if not self._g or not self._ws:
            raise MemoryError("oracle allocation failed")

    @classmethod
    def from_graph(cls, g, libpath: str | None = None):
        return cls(g.n, g.tail, g.head, g.w, libpath)

    def close(self):
        if getattr(self, "_g", None):
            self._L.orc_graph_free(self._g)
            self._L.orc_ws_free(self._ws)
            self._g = self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def isochrone(self, s: int, tau: int, want_dist: bool = False):
        """(edges (k,2) uint32 sorted, dist uint64[n] or None, settled count)."""
        _check_source(s, self.n)
        ptr, cnt = _U64P(), C.c_uint64()
        dist = np.empty(self.n, dtype=np.uint64) if want_dist else None
        dptr = dist.ctypes.data_as(_U64P) if want_dist else None
        settled = self._L.orc_isochrone(self._g, self._ws, int(s), int(tau), dptr,
                                        C.byref(ptr), C.byref(cnt))
        return _take_edges(self._L, ptr, cnt), dist, int(settled)

    def distances(self, s: int) -> np.ndarray:
        """d(s, .) for all vertices; INF (2^64-1) where unreachable."""
        _check_source(s, self.n)
        dist = np.empty(self.n, dtype=np.uint64)
        self._L.orc_distances(self._g, self._ws, int(s), dist.ctypes.data_as(_U64P))
        return dist

    def edges_by_definition(self, dist: np.ndarray, tau: int) -> np.ndarray:
        d = np.ascontiguousarray(dist, dtype=np.uint64)
        ptr, cnt = _U64P(), C.c_uint64()
        self._L.orc_edges_by_definition(self._g, d.ctypes.data_as(_U64P), int(tau),
                                        C.byref(ptr), C.byref(cnt))
        return _take_edges(self._L, ptr, cnt)

    def in_range(self, s: int, tau: int) -> np.ndarray:
        """The vertices with d(s, v) <= tau (Section 3), sorted, as uint32."""
        _check_source(s, self.n)
        ptr = _U32P()
        cnt = int(self._L.orc_in_range(self._g, self._ws, int(s), int(tau), C.byref(ptr)))
        try:
            return np.ctypeslib.as_array(ptr, shape=(cnt,)).copy() if cnt else np.zeros(0, dtype=np.uint32)
        finally:
            self._L.orc_free(ptr)

    def polygon(self, xy, in_range):
        """The isochrone polygon of a vertex set in range (Section 7, face traversal on the planar
        embedding xy): a list of cycles, each an (k, 2) uint32 array of boundary darts (u in range,
        v not), each cycle from its smallest dart, the cycles ordered by it."""
        xyc = np.ascontiguousarray(xy, dtype=np.float64).reshape(-1)
        inr = np.zeros(self.n, dtype=np.uint8)
        inr[np.asarray(in_range, dtype=np.int64)] = 1
        dp, cp, nc = _U64P(), _U64P(), C.c_uint64()
        nd = self._L.orc_polygon(self._g, xyc.ctypes.data_as(C.POINTER(C.c_double)),
                                 inr.ctypes.data_as(C.POINTER(C.c_uint8)), C.byref(dp), C.byref(cp), C.byref(nc))
        if nd == 0xFFFFFFFFFFFFFFFF:
            raise ValueError("a face walk did not close: the embedding is not planar")
        try:
            d = np.ctypeslib.as_array(dp, shape=(nd,)).copy() if nd else np.zeros(0, dtype=np.uint64)
            c = np.ctypeslib.as_array(cp, shape=(nc.value + 1,)).copy()
        finally:
            self._L.orc_free(dp)
            self._L.orc_free(cp)
        pairs = np.stack([(d >> np.uint64(32)).astype(np.uint32), (d & np.uint64(0xFFFFFFFF)).astype(np.uint32)],
                         axis=1)
        return [pairs[c[i]:c[i + 1]] for i in range(int(nc.value))]

    def iso_dijkstra(self, s: int, tau: int):
        """The paper's isoDijkstra: (edges, settled count).  Requires tau < 2^64-1."""
        _check_source(s, self.n)
        ptr, cnt = _U64P(), C.c_uint64()
        settled = self._L.orc_iso_dijkstra(self._g, self._ws, int(s), int(tau),
                                           C.byref(ptr), C.byref(cnt))
        return _take_edges(self._L, ptr, cnt), int(settled)


class OracleWorker:
    """A second workspace over an existing Oracle's graph (one per host thread)."""

    def __init__(self, parent: "Oracle"):
        self._parent = parent
        self._L = parent._L
        self._g = parent._g
        self._ws = self._L.orc_ws_new(parent.n)
        if not self._ws:
            raise MemoryError("oracle workspace allocation failed")

    def isochrone(self, s: int, tau: int):
        _check_source(s, self._parent.n)
        ptr, cnt = _U64P(), C.c_uint64()
        settled = self._L.orc_isochrone(self._g, self._ws, int(s), int(tau), None, C.byref(ptr), C.byref(cnt))
        return _take_edges(self._L, ptr, cnt), int(settled)

    def iso_dijkstra(self, s: int, tau: int):
        _check_source(s, self._parent.n)
        ptr, cnt = _U64P(), C.c_uint64()
        settled = self._L.orc_iso_dijkstra(self._g, self._ws, int(s), int(tau), C.byref(ptr), C.byref(cnt))
        return _take_edges(self._L, ptr, cnt), int(settled)

    def __del__(self):
        try:
            self._L.orc_ws_free(self._ws)
        except Exception:
            pass


def _check_source(s: int, n: int):
    if not 0 <= int(s) < n:
        raise ValueError(f"source {s} out of range [0, {n})")


def clamp_u32(dist: np.ndarray) -> np.ndarray:
    """Distances as the 32-bit interface reports them: min(d, 2^32 - 1)."""
    return np.minimum(dist, np.uint64(0xFFFFFFFF)).astype(np.uint32)
