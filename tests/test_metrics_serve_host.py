"""Host-side logic: the waste metric (Eq. waste) and the serving slot bookkeeping."""
import numpy as np

from paper_1608_05794_amd import metrics


def test_waste_closed_forms():
    # equal step counts waste nothing
    assert np.all(metrics.waste([7] * 64, 4) == 0.0)
    # one busy lane among P idle-ish lanes: W = 1 - (N + (P-1) M) / (P N)
    s = [100, 1, 1, 1]
    assert np.isclose(metrics.waste(s, 4)[0], 1 - 103 / 400)
    # groups are consecutive and a trailing partial group is dropped
    w = metrics.waste([1, 3, 2, 2, 5], 2)
    assert np.allclose(w, [1 - 4 / 6, 0.0])
    # wider groups never waste less on the same data (max over a superset)
    rng = np.random.default_rng(0)
    st = rng.integers(1, 1000, size=4096)
    means = [metrics.waste(st, p).mean() for p in (4, 8, 16, 32, 64)]
    assert all(a <= b + 1e-12 for a, b in zip(means, means[1:]))
    # lane efficiency is one minus the max-weighted mean waste
    g = st.reshape(-1, 64).astype(float)
    W = metrics.waste(st, 64)
    assert np.isclose(metrics.lane_efficiency(st, 64), 1 - np.sum(W * g.max(1)) / g.max(1).sum())


def test_slot_bookkeeping():
    from paper_1608_05794_amd import serve
    p = serve.Pool.__new__(serve.Pool)
    p.cap, p.free, p.active, p.hwm = 100, [(0, 100)], {}, 0
    a = p.alloc(30)
    b = p.alloc(50)
    assert a == (0, 30) and b == (30, 80) and p.alloc(30) is None
    p.release(*a)
    assert p.free == [(0, 30), (80, 100)]
    p.release(*b)
    assert p.free == [(0, 100)]


def test_tuner_candidates():
    from paper_1608_05794_amd import tune
    c53 = tune.candidates(54)
    assert {"kernel": "wave", "blocks_per_cu": 8} in c53 and {"kernel": "lane", "blocks_per_cu": 0} in c53
    c112 = tune.candidates(112)
    assert all(c["kernel"] != "wave" for c in c112) and any(c["kernel"] == "group" for c in c112)
    assert all(c["kernel"] == "wave" for c in tune.candidates(54, precision="fp32_refine"))
    assert tune.candidates(200) == [{"kernel": "lane", "blocks_per_cu": 0}]


class _FakePool:
    """Host stand-in for a device pool: admits while slots are free; every launch finishes at once
    (or never, with stuck=True)."""

    def __init__(self, cap, stuck=False):
        self.cap, self.free_slots, self.active, self.stuck = cap, cap, {}, stuck
        self._inflight = False

    def admit(self, req):
        if req.n > self.free_slots:
            return False
        self.free_slots -= req.n
        self.active[req.rid] = req
        return True

    def in_flight(self):
        return self._inflight

    def launch(self):
        self._inflight = True

    def finished(self):
        return self._inflight and not self.stuck

    def harvest(self, now):
        self._inflight = False
        done = list(self.active.values())
        for r in done:
            r.completed = now
            self.free_slots += r.n
        self.active.clear()
        return done


def _server(pools):
    from paper_1608_05794_amd import serve
    s = serve.Server.__new__(serve.Server)
    s.pools, s.budget, s.allocated = pools, 1.0, 0.0
    s.waiting = {k: [] for k in pools}
    s.done, s.rejected, s.iterations, s.max_backlog = [], [], 0, 0
    return s


def _req(rid, mech, n, arrival=0.0):
    from paper_1608_05794_amd import serve
    return serve.Request(rid, mech, np.zeros((3, n)), np.zeros(n), 1e-6, arrival)


def test_oversized_request_is_rejected_and_does_not_block():
    s = _server({"A": _FakePool(100), "B": _FakePool(100)})
    reqs = [_req(0, "A", 500), _req(1, "A", 10), _req(2, "B", 20), _req(3, "C", 5)]
    done = s.run(reqs, time_limit=5.0)
    assert sorted(r.rid for r in done) == [1, 2]
    assert sorted(r.rid for r in s.rejected) == [0, 3]
    assert all(r.error for r in s.rejected) and s.backlog() == 0


def test_blocked_queue_holds_only_its_own_mechanism():
    # A's pool is busy forever (its launch never finishes): B's requests are still served
    s = _server({"A": _FakePool(10, stuck=True), "B": _FakePool(100)})
    reqs = [_req(0, "A", 10), _req(1, "A", 5), _req(2, "B", 30), _req(3, "B", 30)]
    done = s.run(reqs, time_limit=0.5)
    assert sorted(r.rid for r in done) == [2, 3]
    assert s.backlog() == 2          # one A request on the device, one waiting for slots


def test_time_limit_ends_an_idle_wait():
    import time
    # nothing is ever admitted (the only request's pool is stuck with an earlier one) and future
    # arrivals are far away: the loop must still return at the time limit
    s = _server({"A": _FakePool(10, stuck=True)})
    reqs = [_req(0, "A", 10), _req(1, "A", 10, arrival=1e6)]
    t0 = time.perf_counter()
    s.run(reqs, time_limit=0.3)
    assert time.perf_counter() - t0 < 5.0
