"""Continuous-batching solve service on one GPU.

Requests (a mechanism, a batch of reactor states, pressures and an end time)
are admitted into device-resident slot pools, one pool per mechanism, under
an HBM budget.  Each pool with active slots runs bounded launches of the
persistent work-queue integrator (at most `launch_steps` attempted steps per
reactor) on its own stream, so the mechanisms' work overlaps on the device,
and each pool is harvested and relaunched as soon as its own launch ends
(a completion event per launch), not at the pace of the slowest pool.
Reactors resume from their (t, h) in the next launch, so a request's result
does not depend on how its work was split into launches or what else was in
the pool.  A request completes when none of its reactors still has steps
left; its slots are freed and waiting requests are admitted.

HBM budget: the pools are the serving state's device memory.  Unless capacities
are given, each pool's capacity is its share of the budget divided by the bytes
one reactor slot holds (state, pressure, end time, t, h, step counters, and
its share of the integrator workspace), capped at `max_capacity` slots so a
launch never sweeps an unbounded grid; the pools' real allocations are checked
against the budget at construction.  A request is admitted when its pool has
a free range of slots for all its reactors; one that is larger than its
pool's capacity can never be admitted and is rejected on arrival.  Each
mechanism has its own FIFO queue, so a request that waits for slots holds up
only later requests of the same mechanism.

Only the control plane is here (admission, slot bookkeeping, timing); every
state update runs in the library's kernels.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import ck

ST_MAX_STEPS = 1


@dataclass
class Request:
    rid: int
    mech: str
    y0: np.ndarray            # [N, n] float64
    P: np.ndarray             # [n] Pa
    t_end: float
    arrival: float            # seconds after the stream started
    admitted: float = -1.0
    completed: float = -1.0
    slots: tuple = ()         # (start, stop) in its pool
    launched: bool = False    # part of a launch whose statuses have not been read yet
    result: dict = field(default_factory=dict)
    error: str = ""           # set when the request was rejected (never admitted)

    @property
    def n(self):
        return self.y0.shape[1]


class Pool:
    """Device-resident state of one mechanism: fixed-capacity slot arrays."""

    def __init__(self, mech: ck.Mechanism, capacity: int, method="ros4", launch_steps=500, **opts):
        dev = mech.device
        self.mech = mech
        self.cap = capacity
        self.method = method
        self.launch_steps = launch_steps
        self.opts = opts
        N = mech.N
        f64 = dict(dtype=torch.float64, device=dev)
        self.y = torch.zeros((N, capacity), **f64)
        self.y[0].fill_(1000.0)
        self.y[1].fill_(1.0)
        self.P = torch.full((capacity,), 101325.0, **f64)
        self.te = torch.zeros(capacity, **f64)       # empty slots: t = t_end = 0, nothing to do
        self.t = torch.zeros(capacity, **f64)
        self.h = torch.zeros(capacity, **f64)
        self.steps = torch.zeros(capacity, dtype=torch.int64, device=dev)
        self.ws = torch.empty(mech.workspace_bytes(capacity, **opts), dtype=torch.uint8, device=dev)
        self.stream = torch.cuda.Stream(device=dev)          # default priority
        self.free = [(0, capacity)]                          # sorted free ranges
        self.active = {}                                     # rid -> Request
        self.hwm = 0                                         # slots beyond it are empty
        self.last = None
        self.event = None

    # --- slot bookkeeping ----------------------------------------------------------------
    @staticmethod
    def slot_bytes(N):
        """Device bytes of one reactor slot: state [N], P, t_end, t, h (float64) and the step counter."""
        return (N + 4) * 8 + 8

    def device_bytes(self):
        """Device memory this pool holds (its arrays and the integrator workspace)."""
        ts = (self.y, self.P, self.te, self.t, self.h, self.steps, self.ws)
        return sum(t.numel() * t.element_size() for t in ts)

    def bytes_per_reactor(self):
        return self.device_bytes() / max(self.cap, 1)

    def alloc(self, n):
        for i, (a, b) in enumerate(self.free):
            if b - a >= n:
                self.free[i] = (a + n, b)
                if a + n == b:
                    self.free.pop(i)
                return a, a + n
        return None

    def release(self, a, b):
        self.free.append((a, b))
        self.free.sort()
        merged = []
        for x, y in self.free:
            if merged and merged[-1][1] == x:
                merged[-1] = (merged[-1][0], y)
            else:
                merged.append((x, y))
        self.free = merged
        self.hwm = max((r.slots[1] for r in self.active.values()), default=0)

    def admit(self, req: Request):
        rng = self.alloc(req.n)
        if rng is None:
            return False
        a, b = rng
        req.slots = rng
        with torch.cuda.stream(self.stream):
            self.y[:, a:b].copy_(torch.as_tensor(req.y0), non_blocking=False)
            self.P[a:b].copy_(torch.as_tensor(req.P))
            self.te[a:b].fill_(req.t_end)
            self.t[a:b].zero_()
            self.h[a:b].zero_()
            self.steps[a:b].zero_()
        self.active[req.rid] = req
        self.hwm = max(self.hwm, b)
        return True

    # --- one iteration ---------------------------------------------------------------------
    def launch(self):
        if not self.active or self.hwm == 0:
            self.last = None
            self.event = None
            return
        n = self.hwm
        for req in self.active.values():
            req.launched = True
        with torch.cuda.stream(self.stream):
            r = ck.integrate(self.mech, self.y[:, :n], self.P[:n], self.te[:n], method=self.method,
                             t=self.t[:n], h=self.h[:n], workspace=self.ws, stream=self.stream, inplace=True,
                             max_steps=self.launch_steps, **self.opts)
            self.steps[:n].add_(r["n_accept"] + r["n_reject"])
            self.last = r["status"]
            self.event = torch.cuda.Event()
            self.event.record(self.stream)

    def in_flight(self):
        return self.event is not None

    def finished(self):
        """The last launch (and the bookkeeping queued behind it) has completed on the device."""
        return self.event is not None and self.event.query()

    def harvest(self, now):
        """Requests of the last launch whose reactors all finished; frees their slots.  Requests
        admitted while that launch ran were not part of it and wait for the next one."""
        done = []
        self.event = None
        if self.last is None:
            return done
        last, self.last = self.last, None
        unfinished = (last == ST_MAX_STEPS).cpu().numpy()
        for rid, req in list(self.active.items()):
            if not req.launched:
                continue
            req.launched = False
            a, b = req.slots
            if not unfinished[a:b].any():
                req.completed = now
                req.result = dict(y=self.y[:, a:b].cpu().numpy(), status=last[a:b].cpu().numpy(),
                                  steps=self.steps[a:b].cpu().numpy())
                del self.active[rid]
                self.release(a, b)
                done.append(req)
        return done


class Server:
    """Admission by HBM budget and continuous batching over per-mechanism pools.

    mechs: name -> ck.Mechanism.  capacity: name -> slots (default: the budget split evenly over
    the mechanisms, capped at max_capacity).  pool_opts: name -> extra integrator options for that
    pool (for example {"precision": "fp32_refine"}); opts apply to every pool."""

    def __init__(self, mechs: dict, capacity: dict = None, hbm_budget=200e9, launch_steps=500,
                 max_capacity=262144, pool_opts: dict = None, **opts):
        self.budget = float(hbm_budget)
        pool_opts = pool_opts or {}
        if capacity is None:
            share = self.budget / max(len(mechs), 1)
            capacity = {}
            for k, m in mechs.items():
                o = dict(opts, **pool_opts.get(k, {}))
                fixed = m.workspace_bytes(1, **o)
                slots = int((share - fixed) // Pool.slot_bytes(m.N))
                capacity[k] = max(0, min(max_capacity, slots)) // 64 * 64
        self.pools = {k: Pool(m, capacity[k], launch_steps=launch_steps, **dict(opts, **pool_opts.get(k, {})))
                      for k, m in mechs.items()}
        self.allocated = sum(p.device_bytes() for p in self.pools.values())
        if self.allocated > self.budget:
            raise ValueError(f"pools need {self.allocated:.3e} B of device memory, over the {self.budget:.3e} B budget")
        self.waiting = {k: [] for k in mechs}     # per-mechanism FIFO queues
        self.done = []
        self.rejected = []
        self.iterations = 0
        self.max_backlog = 0

    def backlog(self):
        """Requests that arrived and are not finished: waiting for slots or on the device."""
        return sum(len(q) for q in self.waiting.values()) + sum(len(p.active) for p in self.pools.values())

    def _arrive(self, req, now):
        pool = self.pools.get(req.mech)
        if pool is None or req.n > pool.cap or req.n < 1:
            req.error = "unknown mechanism" if pool is None else f"{req.n} reactors do not fit a pool of {pool.cap}"
            req.completed = now
            self.rejected.append(req)
        else:
            self.waiting[req.mech].append(req)

    def run(self, requests, time_limit=None, log=None):
        """Serve `requests` (sorted by arrival) against the wall clock; returns completed requests.
        Stops early once `time_limit` seconds have passed (requests still waiting or on the device
        are then counted in `backlog()`)."""
        pending = list(requests)
        t0 = time.perf_counter()
        next_log = 0
        while pending or self.backlog() or any(p.in_flight() for p in self.pools.values()):
            now = time.perf_counter() - t0
            if time_limit is not None and now > time_limit:
                break
            while pending and pending[0].arrival <= now:
                self._arrive(pending.pop(0), now)
            # admission: each mechanism's queue in arrival order, while its pool has room
            for k, q in self.waiting.items():
                while q and self.pools[k].admit(q[0]):
                    q[0].admitted = time.perf_counter() - t0
                    q.pop(0)
            self.max_backlog = max(self.max_backlog, self.backlog())
            if not any(p.active or p.in_flight() for p in self.pools.values()):
                if pending:
                    time.sleep(max(0.0, min(pending[0].arrival - now, 0.01)))
                continue
            for p in self.pools.values():
                if p.active and not p.in_flight():
                    p.launch()
            harvested = False
            for p in self.pools.values():
                if p.finished():
                    self.iterations += 1
                    harvested = True
                    now = time.perf_counter() - t0
                    self.done.extend(p.harvest(now))
            if not harvested:
                time.sleep(0.0002)
            if log and self.iterations >= next_log:
                next_log = self.iterations + 20
                log(f"iteration {self.iterations}: t={now:.1f}s done {len(self.done)} "
                    f"waiting {sum(len(q) for q in self.waiting.values())} "
                    f"active {sum(len(p.active) for p in self.pools.values())} rejected {len(self.rejected)}")
        return self.done


def poisson_requests(n_requests, rate, seed=5000, mech_weights=(("M13", 0.3), ("M53", 0.5), ("M111", 0.2)),
                     n_range=(1, 65536), t_range=(1e-6, 1e-3), species=None):
    """Seeded request stream: Poisson arrivals, mechanism by weight, log-uniform size and end time.

    species: dict name -> number of species (to draw states); states follow the configurations
    (13 species: 1 atm 'small'; 53: 'mid'; 111: 'divergent')."""
    from . import synth
    rng = np.random.default_rng(seed)
    names = [m for m, _ in mech_weights]
    w = np.array([p for _, p in mech_weights], dtype=float)
    w /= w.sum()
    recipe = {"M13": "small", "M53": "mid", "M111": "divergent"}
    t = 0.0
    out = []
    for i in range(n_requests):
        t += rng.exponential(1.0 / rate)
        m = names[rng.choice(len(names), p=w)]
        n = int(np.floor(np.exp(rng.uniform(np.log(n_range[0]), np.log(n_range[1] + 1)))))
        n = max(n_range[0], min(n, n_range[1]))
        te = float(np.exp(rng.uniform(np.log(t_range[0]), np.log(t_range[1]))))
        y0, P = synth.reactor_states(species[m], n, recipe[m], seed=int(rng.integers(1 << 31)))
        out.append(Request(i, m, y0, P, te, t))
    return out


def latency_summary(done, offered_rate, elapsed, arrived=None):
    """Completed-request latency (arrival to completion) and served load over `elapsed` seconds."""
    lat = np.array([r.completed - r.arrival for r in done]) if done else np.zeros(0)
    reactors = sum(r.n for r in done)
    out = dict(completed=len(done), offered_rate=offered_rate,
               served_rate=len(done) / elapsed if elapsed > 0 else 0.0,
               reactors_per_s=reactors / elapsed if elapsed > 0 else 0.0,
               p50_s=float(np.percentile(lat, 50)) if len(lat) else None,
               p99_s=float(np.percentile(lat, 99)) if len(lat) else None)
    if arrived is not None:
        out["arrived"] = len(arrived)
        out["offered_reactors_per_s"] = (sum(r.n for r in arrived) / (max(r.arrival for r in arrived) or 1e-9)
                                         if arrived else 0.0)
    return out
