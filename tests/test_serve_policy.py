"""CPU tests of the step server's scheduling policy (serve_policy.h) through
the test shim in tests/host: FIFO admission under an HBM budget, request
ordering, multi-frame requests, and a synthetic-clock continuous-batching
timeline with a fake in-order device."""

import ctypes

import numpy as np
import pytest

from tests.host import build as host_build

_lib = None


def lib():
    global _lib
    if _lib is None:
        L = ctypes.CDLL(host_build.ensure())
        vp, i, d, sz, u64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t, ctypes.c_uint64
        P = ctypes.POINTER
        sig = {
            "vhp_pol_new": (vp, []), "vhp_pol_free": (None, [vp]), "vhp_pol_add": (i, [vp, sz]),
            "vhp_pol_state": (i, [vp, i]), "vhp_pol_to_admit": (i, [vp, sz, sz, P(i), i]),
            "vhp_pol_admit": (None, [vp, i]), "vhp_pol_release": (None, [vp, i]),
            "vhp_pol_submit": (u64, [vp, i, i, d]), "vhp_pol_pick": (i, [vp, i, P(i), i]),
            "vhp_pol_launch": (None, [vp, P(i), i]), "vhp_pol_complete": (None, [vp, P(i), i, d]),
            "vhp_pol_idle": (i, [vp, i]), "vhp_pol_in_flight": (i, [vp, i]), "vhp_pol_any_pending": (i, [vp]),
            "vhp_pol_request": (i, [vp, u64, P(i), P(i), P(i), P(d)]),
            "vhp_pol_percentile": (d, [vp, d]), "vhp_pol_span": (d, [vp]),
            "vhp_pol_frames_done": (ctypes.c_int64, [vp]), "vhp_pol_requests_done": (ctypes.c_int64, [vp]),
        }
        for k, (r, a) in sig.items():
            getattr(L, k).restype = r
            getattr(L, k).argtypes = a
        _lib = L
    return _lib


class Pol:
    QUEUED, RESIDENT, RELEASED = 0, 1, 2

    def __init__(self):
        self.L = lib()
        self.h = self.L.vhp_pol_new()

    def __del__(self):
        self.L.vhp_pol_free(self.h)

    def add(self, need=0):
        return self.L.vhp_pol_add(self.h, need)

    def state(self, g):
        return self.L.vhp_pol_state(self.h, g)

    def _ids(self, f, *args):
        out = (ctypes.c_int * 4096)()
        n = f(self.h, *args, out, 4096)
        return [out[k] for k in range(n)]

    def to_admit(self, in_use, budget):
        return self._ids(self.L.vhp_pol_to_admit, in_use, budget)

    def admit(self, g):
        self.L.vhp_pol_admit(self.h, g)

    def release(self, g):
        self.L.vhp_pol_release(self.h, g)

    def submit(self, g, frames, t):
        return self.L.vhp_pol_submit(self.h, g, frames, t)

    def pick(self, m):
        return self._ids(self.L.vhp_pol_pick, m)

    def launch(self, ids):
        a = (ctypes.c_int * len(ids))(*ids)
        self.L.vhp_pol_launch(self.h, a, len(ids))

    def complete(self, ids, t):
        a = (ctypes.c_int * len(ids))(*ids)
        self.L.vhp_pol_complete(self.h, a, len(ids), t)

    def idle(self, g):
        return bool(self.L.vhp_pol_idle(self.h, g))

    def in_flight(self, g):
        return self.L.vhp_pol_in_flight(self.h, g)

    def any_pending(self):
        return bool(self.L.vhp_pol_any_pending(self.h))

    def request(self, ticket):
        la, do, g, td = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
        ok = self.L.vhp_pol_request(self.h, ticket, ctypes.byref(la), ctypes.byref(do), ctypes.byref(g),
                                    ctypes.byref(td))
        assert ok
        return la.value, do.value, g.value, td.value

    def percentile(self, q):
        return self.L.vhp_pol_percentile(self.h, q)


def test_fifo_admission_under_budget():
    p = Pol()
    need = [5, 3, 4, 1]
    ids = [p.add(n) for n in need]
    assert ids == [0, 1, 2, 3]
    assert p.to_admit(0, 0) == [0, 1, 2, 3]          # unlimited budget
    # budget 8: 5 + 3 fits; 4 does not, and the 1 behind it waits (strict FIFO)
    assert p.to_admit(0, 8) == [0, 1]
    p.admit(0)
    p.admit(1)
    assert p.state(0) == Pol.RESIDENT and p.state(2) == Pol.QUEUED
    assert p.to_admit(8, 8) == []
    p.release(0)                                       # 5 bytes free again
    assert p.to_admit(3, 8) == [2, 3]
    assert p.to_admit(3, 7) == [2]


def test_pick_orders_by_oldest_request_and_skips_queued():
    p = Pol()
    for _ in range(4):
        p.add(1)
    for g in (0, 1, 2):
        p.admit(g)
    p.submit(1, 1, 0.10)
    p.submit(0, 1, 0.20)
    p.submit(2, 1, 0.05)
    p.submit(3, 1, 0.00)                               # garment 3 is not admitted
    assert p.pick(8) == [2, 1, 0]
    assert p.pick(2) == [2, 1]
    p.launch([2, 1])
    assert p.pick(8) == [0]                            # their only frames are launched
    p.complete([2, 1], 0.5)
    assert p.idle(2) and p.idle(1) and not p.idle(0)
    assert p.any_pending()


def test_multi_frame_request_pipelines_and_completes_in_order():
    p = Pol()
    g = p.add(1)
    p.admit(g)
    t1 = p.submit(g, 3, 0.0)
    t2 = p.submit(g, 1, 0.1)
    order = []
    for k in range(4):
        ids = p.pick(1)
        assert ids == [g]
        p.launch(ids)
        order.append(p.in_flight(g))
    assert order == [1, 2, 3, 4]                       # frames queue back to back
    assert p.pick(1) == []
    assert p.request(t1)[:2] == (3, 0) and p.request(t2)[:2] == (1, 0)
    for k in range(4):
        p.complete([g], 1.0 + k)
    la, do, _, td1 = p.request(t1)
    assert (la, do) == (3, 3) and td1 == 3.0           # done with its third frame
    assert p.request(t2)[3] == 4.0
    assert p.idle(g) and not p.any_pending()
    assert p.L.vhp_pol_frames_done(p.h) == 4 and p.L.vhp_pol_requests_done(p.h) == 2


def _simulate(p, arrivals, depth, max_batch, cost):
    """Drive the policy as the server does, with a fake device that runs
    launches in order; cost(batch) is a launch's duration.  Returns the
    launches as (start, end, ids)."""
    t = 0.0
    i = 0
    inflight = []          # (end, ids)
    launches = []
    gpu_free = 0.0
    while i < len(arrivals) or p.any_pending():
        # retire what has finished by now
        while inflight and inflight[0][0] <= t:
            end, ids = inflight.pop(0)
            p.complete(ids, end)
        while i < len(arrivals) and arrivals[i][0] <= t:
            ta, g, n = arrivals[i]
            p.submit(g, n, ta)
            i += 1
        launched = False
        while len(inflight) < depth:
            ids = p.pick(max_batch)
            if not ids:
                break
            p.launch(ids)
            start = max(t, gpu_free)
            gpu_free = start + cost(ids)
            inflight.append((gpu_free, ids))
            launches.append((start, gpu_free, ids))
            launched = True
        if not launched:
            nxt = [inflight[0][0]] if inflight else []
            if i < len(arrivals):
                nxt.append(arrivals[i][0])
            if not nxt:
                break
            t = max(t, min(nxt))
    return launches


@pytest.mark.parametrize("depth,max_batch", [(1, 64), (2, 64), (2, 3), (3, 1)])
def test_continuous_batching_timeline(depth, max_batch):
    rng = np.random.default_rng(11)
    p = Pol()
    ng = 6
    for _ in range(ng):
        p.admit(p.add(1))
    # Poisson arrivals, one frame each, assigned uniformly to garments
    n_req = 300
    ta = np.cumsum(rng.exponential(1.0 / 2.0, n_req))
    garments = rng.integers(0, ng, n_req)
    arrivals = [(float(a), int(g), 1) for a, g in zip(ta, garments)]
    cost = lambda ids: 0.2 + 0.05 * len(ids)
    tickets = list(range(1, n_req + 1))
    launches = _simulate(p, arrivals, depth, max_batch, cost)
    assert not p.any_pending()
    done_t = {}
    for tk, (a, g, _) in zip(tickets, arrivals):
        la, do, gg, td = p.request(tk)
        assert (la, do, gg) == (1, 1, g)
        assert td >= a
        done_t[tk] = (g, td, a)
    # per-garment order is preserved: completion times follow submission order
    for g in range(ng):
        ts = [done_t[k][1] for k in tickets if done_t[k][0] == g]
        assert all(x <= y for x, y in zip(ts, ts[1:]))
    # a launch never holds one garment twice, nor more than max_batch garments
    for _, _, ids in launches:
        assert len(ids) == len(set(ids)) <= max_batch
    # launches run back to back in order on the fake device
    assert all(l1[1] <= l2[0] + 1e-12 for l1, l2 in zip(launches, launches[1:]))
    # latency percentiles: nearest rank over the completed requests
    lat = np.sort([td - a for (_, td, a) in done_t.values()])
    for q in (0.5, 0.99, 1.0):
        k = max(0, int(np.ceil(q * len(lat))) - 1)
        assert p.percentile(q) == pytest.approx(lat[k], abs=1e-12)
    if max_batch > 1:
        # batching: fewer launches than frames
        assert len(launches) < n_req


def test_requests_arriving_mid_launch_join_the_next_launch():
    p = Pol()
    for _ in range(3):
        p.admit(p.add(1))
    # garment 0 starts alone at t=0; 1 and 2 arrive while it runs
    arrivals = [(0.0, 0, 1), (0.1, 1, 1), (0.2, 2, 1)]
    launches = _simulate(p, arrivals, depth=1, max_batch=64, cost=lambda ids: 1.0)
    assert [sorted(ids) for _, _, ids in launches] == [[0], [1, 2]]
    assert launches[1][0] == pytest.approx(1.0)
