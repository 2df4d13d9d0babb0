"""iso_query_batch_device: the edges of a batch written to caller-owned device memory (torch
tensors) are the same, lane by lane, as iso_query_batch's host result and the oracle's; a
buffer that is too small gives ISO_ESPACE with the exact count; pointers that are not device
memory of the right size are refused before any work."""
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


@pytest.fixture(scope="module")
def road():
    import torch
    torch.cuda.init()
    g = synth.road_graph(40_000, 23)
    say("road40k / 128 cells")
    G = iso.Graph.from_synth(g, num_cells=128, device=0)
    return g, G


def _device_batch(G, src, tau, mode, cap):
    import torch
    pairs = torch.empty((max(cap, 1), 2), dtype=torch.int32, device="cuda:0")
    offsets = torch.full((len(src) + 1,), -1, dtype=torch.int32, device="cuda:0")
    total = G.query_batch_device(src, tau, mode, pairs[:cap] if cap else pairs[:0], offsets)
    off = offsets.cpu().numpy().view(np.uint32).astype(np.int64)
    flat = pairs[:total].cpu().numpy().view(np.uint32)
    return total, off, flat


@pytest.mark.parametrize("mode", [iso.MODE_CELLS, iso.MODE_PLAIN])
def test_device_output_equals_host_batch(road, mode):
    g, G = road
    src, tau = synth.batch_queries(g.n, 150, seed=31 + mode, lo_min=1, hi_min=90)   # 3 sweeps of <= 64
    host = G.query_batch(src, tau, mode)
    need = sum(len(h) for h in host)
    say(f"device output: 150 queries, mode {mode}, {need} edges")
    total, off, flat = _device_batch(G, src, tau, mode, need + 100)
    assert total == need and off[0] == 0 and off[-1] == total
    for j in range(len(src)):
        np.testing.assert_array_equal(flat[off[j]:off[j + 1]], host[j], err_msg=f"lane {j}")
    orc = Oracle.from_graph(g)
    for j in (0, 63, 64, 127, 128, 149):   # first and last lanes of each sweep
        want, _, _ = orc.isochrone(int(src[j]), int(tau[j]))
        np.testing.assert_array_equal(flat[off[j]:off[j + 1]], want, err_msg=f"oracle lane {j}")


def test_device_output_too_small(road):
    g, G = road
    src, tau = synth.batch_queries(g.n, 100, seed=8, lo_min=1, hi_min=60)
    need = sum(len(h) for h in G.query_batch(src, tau, iso.MODE_CELLS))
    assert need > 10
    for cap in (0, 10, need - 1):
        say(f"device output: capacity {cap} of {need}")
        with pytest.raises(iso.IsoError) as e:
            _device_batch(G, src, tau, iso.MODE_CELLS, cap)
        assert e.value.code == iso.ISO_ESPACE and e.value.total == need
    total, off, flat = _device_batch(G, src, tau, iso.MODE_CELLS, need)   # exact fit after the failures
    assert total == need and off[-1] == need
    np.testing.assert_array_equal(flat[off[5]:off[6]], G.query(int(src[5]), int(tau[5]), iso.MODE_CELLS))


def test_device_output_empty_batch(road):
    import torch
    g, G = road
    offsets = torch.full((1,), -1, dtype=torch.int32, device="cuda:0")
    pairs = torch.empty((4, 2), dtype=torch.int32, device="cuda:0")
    assert G.query_batch_device([], [], iso.MODE_CELLS, pairs, offsets) == 0
    assert int(offsets.cpu()[0]) == 0


def test_device_output_rejects_bad_pointers(road):
    import torch
    g, G = road
    src = np.array([5, 17], dtype=np.uint32)
    tau = np.array([60_000, 120_000], dtype=np.uint32)
    L = iso.lib()
    sp = src.ctypes.data_as(C.POINTER(C.c_uint32))
    tp = tau.ctypes.data_as(C.POINTER(C.c_uint32))
    total = C.c_uint64()
    host_pairs = np.zeros((1000, 2), dtype=np.uint32)
    dev_off = torch.zeros(3, dtype=torch.int32, device="cuda:0")
    say("device output: host pointer as pairs")
    rc = L.iso_query_batch_device(G._h, 2, sp, tp, iso.MODE_CELLS, C.c_void_p(host_pairs.ctypes.data), 1000,
                                  C.c_void_p(dev_off.data_ptr()), C.byref(total), None)
    assert rc == iso.ISO_EINVAL
    # a capacity far beyond the tensor's allocation (the real tensor holds the whole result,
    # so nothing could be written out of bounds even if the check did not catch it)
    need = sum(len(h) for h in G.query_batch(src, tau, iso.MODE_CELLS))
    dev_pairs = torch.zeros((need + 16, 2), dtype=torch.int32, device="cuda:0")
    say("device output: capacity beyond the allocation")
    rc = L.iso_query_batch_device(G._h, 2, sp, tp, iso.MODE_CELLS, C.c_void_p(dev_pairs.data_ptr()), 1 << 40,
                                  C.c_void_p(dev_off.data_ptr()), C.byref(total), None)
    assert rc == iso.ISO_EINVAL
    # the handle stays usable
    total = G.query_batch_device(src, tau, iso.MODE_CELLS, dev_pairs, dev_off)
    assert total == need
