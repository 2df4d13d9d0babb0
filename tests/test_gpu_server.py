"""Serving loop (continuous batching) on the GPU: a request's result is the same alone and
in a mix of concurrent requests, admission by device memory, state errors."""
import sys
import threading

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
    g = synth.road_graph(60_000, 41)
    say("road60k / 256 cells")
    G = iso.Graph.from_synth(g, num_cells=256, device=0)
    return g, G


def test_alone_equals_in_mix(road):
    g, G = road
    src, tau = synth.serving_trace(g.n, 2000.0, 0.1, seed=15)[1:]
    src, tau = src[:150], tau[:150]
    singles = [G.query(int(s), int(t), iso.MODE_CELLS) for s, t in zip(src, tau)]
    srv = iso.Server(G, max_lanes=16, max_inflight=3, mode=iso.MODE_CELLS)
    try:
        with pytest.raises(iso.IsoError) as e:        # the graph belongs to the server now
            G.query(0, 1000)
        assert e.value.code == iso.ISO_EBUSY
        say("server: one request alone")
        t0 = srv.submit(int(src[7]), int(tau[7]))
        alone, st = srv.wait(t0)
        assert st["batch_lanes"] == 1
        np.testing.assert_array_equal(alone, singles[7])
        say("server: burst of 150 from 3 submitting threads")
        tickets = [None] * len(src)

        def submit(lo, hi):
            for i in range(lo, hi):
                tickets[i] = srv.submit(int(src[i]), int(tau[i]))

        ths = [threading.Thread(target=submit, args=(k * 50, (k + 1) * 50)) for k in range(3)]
        for t in ths:
            t.start()
        for t in ths:
            t.join()
        lanes = []
        for i, tk in enumerate(tickets):
            got, st = srv.wait(tk)
            lanes.append(st["batch_lanes"])
            np.testing.assert_array_equal(got, singles[i], err_msg=f"request {i}")
        stats = srv.stats()
        assert stats["completed"] == stats["submitted"] == len(src) + 1
        assert max(lanes) > 1, "requests that arrive together must share sweeps"
        say(f"server stats {stats}, max batch {max(lanes)}")
    finally:
        srv.close()
    np.testing.assert_array_equal(G.query(int(src[7]), int(tau[7]), iso.MODE_CELLS), alone)
    orc = Oracle.from_graph(g)
    for i in range(0, len(src), 30):
        want, _, _ = orc.isochrone(int(src[i]), int(tau[i]))
        np.testing.assert_array_equal(singles[i], want)


def test_admission_by_device_memory(road):
    g, G = road
    probe = iso.Server(G, max_lanes=64, max_inflight=2)
    per_ctx = probe.stats()["ctx_bytes"]
    probe.close()
    # room for one context of fewer lanes only
    srv = iso.Server(G, max_lanes=64, max_inflight=4, device_budget=per_ctx // 3)
    try:
        st = srv.stats()
        assert st["contexts"] == 1 and st["lanes_cap"] < 64
        src, tau = synth.batch_queries(g.n, 40, seed=3, lo_min=1, hi_min=120)
        tk = [srv.submit(int(s), int(t)) for s, t in zip(src, tau)]
        out = [srv.wait(t) for t in tk]
        res = [o[0] for o in out]
        assert all(o[1]["batch_lanes"] <= st["lanes_cap"] for o in out)
    finally:
        srv.close()
    for i in range(0, 40, 7):
        np.testing.assert_array_equal(res[i], G.query(int(src[i]), int(tau[i]), iso.MODE_CELLS))
    with pytest.raises(iso.IsoError) as e:
        iso.Server(G, max_lanes=8, device_budget=1024)
    assert e.value.code == iso.ISO_ENOMEM


def test_stop_completes_and_refuses(road):
    g, G = road
    srv = iso.Server(G, max_lanes=8, max_inflight=2, mode=iso.MODE_PLAIN)
    src, tau = synth.batch_queries(g.n, 30, seed=5, lo_min=1, hi_min=60)
    tk = [srv.submit(int(s), int(t)) for s, t in zip(src, tau)]
    srv.stop()                                      # completes everything already submitted
    with pytest.raises(iso.IsoError) as e:
        srv.submit(0, 10)
    assert e.value.code == iso.ISO_ESTATE
    res = [srv.wait(t, timeout_ms=0)[0] for t in tk]
    with pytest.raises(iso.IsoError) as e:
        srv.wait(tk[0], timeout_ms=0)               # already collected
    assert e.value.code == iso.ISO_EINVAL
    srv.close()
    for i in range(0, 30, 6):
        np.testing.assert_array_equal(res[i], G.query(int(src[i]), int(tau[i]), iso.MODE_PLAIN))
