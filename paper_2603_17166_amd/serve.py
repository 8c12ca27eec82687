"""Serving form: continuous batching of synthesis / adjoint requests.

Requests name a registered point set ("patch"), a band limit, a spin, an
accuracy and an operation; their data (coefficients or a map) is already on
the device.  The scheduler keeps plans resident on the device (sorted
points, ring tables, kernel tables; the Legendre recurrence tables are
shared by every plan of the same (lmax, spin) inside the library) and, on
every step:

  1. retires finished batches (their HIP event has completed), which frees
     their slot and their memory;
  2. takes the oldest waiting request, gathers the waiting requests with the
     same plan and operation (up to `max_batch`), and admits them as one
     multi-map call if a slot is free and the memory budget (resident plans
     + in-flight workspaces, inputs and outputs) has room; idle plans are
     evicted least-recently-used first to make room.  A table that several
     plans share (the library's Legendre table of one (lmax, spin)) is
     counted once, and the budget is checked again once a plan exists (its
     size before creation is an estimate);
  3. launches the batch on its slot's HIP stream, so batches on different
     slots overlap on the device.

With policy="sjf" step 2 takes, instead of the oldest request, the waiting
request whose plan has the smallest estimated GPU time (the executor's
`cost_estimate`, from the resident plan's Legendre work and point count; a
plan that does not exist yet counts as free, so that it gets created), unless
some request has waited longer than `max_wait` seconds: those go first, oldest
first, so that large requests are not starved.

Requests that arrive while others run are admitted as soon as a slot and
memory free up: the queue is drained continuously, not in rounds.  The
device side is behind a small executor interface so that the scheduling
logic runs on the CPU in tests with a simulated executor.
"""
from __future__ import annotations

import collections
import dataclasses
import math
import random
import time
from typing import Callable

OPS = ("synth", "adjoint")


@dataclasses.dataclass(frozen=True)
class PlanKey:
    patch: str
    lmax: int
    spin: int
    epsilon: float
    precision: str = "auto"


@dataclasses.dataclass(eq=False)
class Request:
    rid: int
    key: PlanKey
    op: str
    data: object
    t_arrival: float
    t_admit: float = math.nan
    t_done: float = math.nan
    batch_size: int = 0
    result: object = None
    error: str | None = None

    @property
    def done(self) -> bool:
        return not math.isnan(self.t_done)

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival


@dataclasses.dataclass(eq=False)
class _PlanEntry:
    key: PlanKey
    handle: object
    resident: int          # bytes the plan holds alone
    busy: int = 0
    last_use: float = 0.0
    shared: object = None  # key of a table shared with other plans, or None


@dataclasses.dataclass(eq=False)
class _Batch:
    entry: _PlanEntry
    op: str
    reqs: list
    slot: int
    footprint: int
    token: object


class Server:
    """Continuous-batching scheduler over an executor (see TorchExecutor)."""

    def __init__(self, executor, memory_budget: int, n_slots: int = 4, max_batch: int = 8,
                 clock: Callable[[], float] = time.perf_counter, policy: str = "fifo", max_wait: float = 0.01):
        if n_slots < 1 or max_batch < 1 or memory_budget <= 0:
            raise ValueError("n_slots, max_batch and memory_budget must be positive")
        if policy not in ("fifo", "sjf"):
            raise ValueError("policy must be 'fifo' or 'sjf'")
        if not max_wait > 0:
            raise ValueError("max_wait must be positive")
        self.policy = policy
        self.max_wait = float(max_wait)
        self.costs: dict = {}  # (plan key, op) -> estimated seconds (policy "sjf")
        self.ex = executor
        self.budget = int(memory_budget)
        self.n_slots = n_slots
        self.max_batch = max_batch
        self.clock = clock
        self.pending: collections.deque = collections.deque()
        self.inflight: list = []
        self.free_slots = list(range(n_slots))
        self.plans: dict = {}
        self.shared: dict = {}  # shared-table key -> [bytes, plans holding it]
        self.resident = 0
        self.inflight_bytes = 0
        self.completed: list = []
        self._next_id = 0
        # counters
        self.n_batches = 0
        self.max_concurrent = 0
        self.plans_created = 0
        self.plans_evicted = 0
        self.peak_bytes = 0

    # -- client side -------------------------------------------------------
    def submit(self, key: PlanKey, op: str, data, t_arrival: float | None = None) -> Request:
        if op not in OPS:
            raise ValueError("op must be one of %s" % (OPS,))
        r = Request(self._next_id, key, op, data, self.clock() if t_arrival is None else t_arrival)
        self._next_id += 1
        self.pending.append(r)
        return r

    def idle(self) -> bool:
        return not self.pending and not self.inflight

    # -- scheduler ---------------------------------------------------------
    def step(self) -> int:
        """Retire finished batches, then admit and launch what fits.  Returns the number of batches launched."""
        self._retire()
        launched = 0
        while self.pending and self.free_slots:
            if not self._admit_head(self._next()):
                break
            launched += 1
        return launched

    def _next(self) -> Request:
        """The request to admit next: the oldest (FIFO), or under "sjf" the
        cheapest by estimated GPU time unless one has waited past max_wait."""
        head = self.pending[0]
        if self.policy == "fifo" or self.clock() - head.t_arrival > self.max_wait:
            return head
        best, best_cost = head, self.costs.get((head.key, head.op), 0.0)
        for r in self.pending:
            c = self.costs.get((r.key, r.op), 0.0)
            if c < best_cost:
                best, best_cost = r, c
        return best

    def run_until_idle(self, poll: float = 2e-5) -> None:
        while not self.idle():
            if self.step() == 0 and self.inflight:
                self._wait(poll)

    def _wait(self, poll: float) -> None:
        w = getattr(self.ex, "wait", None)
        if w is not None:
            w([b.token for b in self.inflight], poll)
        elif poll > 0:
            time.sleep(poll)

    def _retire(self) -> None:
        still = []
        for b in self.inflight:
            if not self.ex.ready(b.token):
                still.append(b)
                continue
            now = self.clock()
            outs = self.ex.results(b.token)
            for r, o in zip(b.reqs, outs):
                r.result = o
                r.t_done = now
                self.completed.append(r)
            self.ex.release(b.token)
            b.entry.busy -= 1
            b.entry.last_use = now
            self.inflight_bytes -= b.footprint
            self.free_slots.append(b.slot)
        self.inflight = still

    def _fail(self, reqs, msg: str) -> None:
        now = self.clock()
        for r in reqs:
            r.error = msg
            r.t_done = now
            self.completed.append(r)

    def _used(self) -> int:
        return self.resident + self.inflight_bytes

    def _evict_for(self, need: int, keep: _PlanEntry | None) -> bool:
        """Evict idle plans, least recently used first, until `need` more bytes fit."""
        while self._used() + need > self.budget:
            idle = [e for e in self.plans.values() if e.busy == 0 and e is not keep]
            if not idle:
                return False
            e = min(idle, key=lambda x: x.last_use)
            self.ex.drop_plan(e.handle)
            del self.plans[e.key]
            self._release(e)
            self.plans_evicted += 1
        return True

    def _release(self, e: _PlanEntry) -> None:
        self.resident -= e.resident
        if e.shared is not None:
            ent = self.shared[e.shared]
            ent[1] -= 1
            if ent[1] == 0:
                self.resident -= ent[0]
                del self.shared[e.shared]

    def _plan(self, key: PlanKey):
        e = self.plans.get(key)
        if e is not None:
            return e
        est = self.ex.plan_bytes_estimate(key)
        shared_of = getattr(self.ex, "shared_of", None)
        if shared_of is not None:
            skey, sbytes = shared_of(key)
            if skey in self.shared:
                est = max(0, est - sbytes)  # already resident
        if not self._evict_for(est, None):
            return None
        try:
            res = self.ex.create_plan(key)
        except Exception as exc:  # invalid request (bad arguments, unknown patch)
            return exc
        # (handle, bytes) or (handle, own bytes, shared-table key, shared bytes)
        skey, sbytes = (res[2], int(res[3])) if len(res) > 2 else (None, 0)
        e = _PlanEntry(key, res[0], int(res[1]), last_use=self.clock(), shared=skey)
        self.plans[key] = e
        self.resident += e.resident
        if skey is not None:
            ent = self.shared.setdefault(skey, [sbytes, 0])
            if ent[1] == 0:
                self.resident += sbytes
            ent[1] += 1
        self.plans_created += 1
        est = getattr(self.ex, "cost_estimate", None)
        if est is not None:
            for op in OPS:
                self.costs[(key, op)] = float(est(e.handle, op))
        # the estimate may have been low: make room now if other plans are idle
        self._evict_for(0, e)
        self.peak_bytes = max(self.peak_bytes, self._used())
        return e

    def _admit_head(self, head: Request) -> bool:
        batch = [r for r in self.pending if r.key == head.key and r.op == head.op][: self.max_batch]
        e = self._plan(head.key)
        if e is None:
            if not self.inflight and not any(p.busy for p in self.plans.values()):
                self._drop_pending(batch, "plan does not fit in the memory budget")
                return True
            return False
        if isinstance(e, Exception):
            self._drop_pending(batch, "plan creation failed: %s" % e)
            return True
        while batch:
            fp = self.ex.footprint(e.handle, head.op, len(batch))
            if self._used() + fp <= self.budget or self._evict_for(fp, e):
                break
            batch = batch[:-1]
        if not batch:
            if not self.inflight:
                self._drop_pending([head], "request does not fit in the memory budget")
                return True
            return False
        for r in batch:
            self.pending.remove(r)
        slot = self.free_slots.pop(0)
        now = self.clock()
        for r in batch:
            r.t_admit = now
            r.batch_size = len(batch)
        try:
            token = self.ex.launch(e.handle, head.op, [r.data for r in batch], slot)
        except Exception as exc:
            self.free_slots.append(slot)
            self._fail(batch, "launch failed: %s" % exc)
            return True
        e.busy += 1
        e.last_use = now
        self.inflight_bytes += fp
        self.inflight.append(_Batch(e, head.op, batch, slot, fp, token))
        self.n_batches += 1
        self.max_concurrent = max(self.max_concurrent, len(self.inflight))
        self.peak_bytes = max(self.peak_bytes, self._used())
        return True

    def _drop_pending(self, reqs, msg: str) -> None:
        for r in reqs:
            self.pending.remove(r)
        self._fail(reqs, msg)

    def close(self) -> None:
        self.run_until_idle()
        for e in list(self.plans.values()):
            self.ex.drop_plan(e.handle)
        self.plans.clear()
        self.shared.clear()
        self.resident = 0


# -- load generation and statistics -----------------------------------------

def poisson_arrivals(n: int, rate: float, seed: int) -> list:
    """Arrival offsets (s) of a Poisson process of `rate` requests/s."""
    r = random.Random(seed)
    t, out = 0.0, []
    for _ in range(n):
        t += r.expovariate(rate)
        out.append(t)
    return out


def run_open_loop(server: Server, specs: list, offsets: list, poll: float = 2e-5) -> list:
    """Submit specs[i] = (key, op, data) at offsets[i] seconds after the start
    (requests arriving while earlier ones run join the queue at once) and
    serve until all are done.  Returns the requests in submission order."""
    t0 = server.clock()
    reqs, i, n = [], 0, len(specs)
    while i < n or not server.idle():
        now = server.clock()
        while i < n and t0 + offsets[i] <= now:
            key, op, data = specs[i]
            reqs.append(server.submit(key, op, data, t_arrival=t0 + offsets[i]))
            i += 1
        if server.step() == 0:
            if server.inflight:
                server._wait(poll)
            elif i < n:
                dt = t0 + offsets[i] - server.clock()
                if dt > 0:
                    time.sleep(min(dt, 1e-3))
    return reqs


def run_closed_loop(server: Server, specs: list) -> tuple:
    """Submit every spec at once and serve them; returns (requests, seconds)."""
    t0 = server.clock()
    reqs = [server.submit(k, op, d, t_arrival=t0) for k, op, d in specs]
    server.run_until_idle()
    return reqs, server.clock() - t0


def percentile(xs: list, q: float) -> float:
    """Nearest-rank percentile (q in [0, 100])."""
    if not xs:
        return math.nan
    s = sorted(xs)
    k = max(0, min(len(s) - 1, math.ceil(q / 100.0 * len(s)) - 1))
    return s[k]


def latency_stats(reqs: list, skip: int = 0) -> dict:
    ok = [r for r in reqs[skip:] if r.done and r.error is None]
    lat = [r.latency for r in ok]
    if not ok:
        return {"n": 0}
    span = max(r.t_done for r in ok) - min(r.t_arrival for r in ok)
    return {"n": len(ok), "p50_ms": 1e3 * percentile(lat, 50), "p99_ms": 1e3 * percentile(lat, 99),
            "mean_ms": 1e3 * sum(lat) / len(lat), "requests_per_s": len(ok) / span if span > 0 else math.nan,
            "mean_batch": sum(r.batch_size for r in ok) / len(ok)}


# -- device executor ----------------------------------------------------------

class TorchExecutor:
    """Runs batches through the library on `n_slots` HIP streams of `device`
    (default priority).  Patches are registered as host or device coordinate
    arrays; each request's data must be a device tensor of the plan's layout:
    alm (2, nalm) complex128 for synthesis, a map (npoints,) of the plan's
    map dtype for the adjoint."""

    def __init__(self, device=None, n_slots: int = 4):
        import torch

        self.torch = torch
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.streams = [torch.cuda.Stream(self.device) for _ in range(n_slots)]
        self.patches: dict = {}

    def add_patch(self, name: str, theta, phi) -> None:
        self.patches[name] = (theta, phi)

    def shared_of(self, key: PlanKey):
        """The Legendre recurrence table every plan of (lmax, spin) shares:
        32 bytes per (l, m) and a seed per m."""
        nalm = (key.lmax + 1) * (key.lmax + 2) // 2
        return ("legendre", key.lmax, key.spin), nalm * 32 + (key.lmax + 1) * 16

    def plan_bytes_estimate(self, key: PlanKey) -> int:
        """Bytes a plan will hold, from the host-side parameters: per point the
        sorted coordinates and permutation (20 B) and the creation scratch
        (24 B); the adjoint's recurrence states (40 B per ring and segment, at
        most one segment per 64 degrees); the shared Legendre table; 1 MiB of
        ring and FFT tables."""
        from .plan import plan_geometry

        th, _ = self.patches[key.patch]
        n = int(len(th))
        ts = float(th.max()) if n else 0.0
        info = plan_geometry(key.lmax, key.spin, ts, key.epsilon, key.precision, rings=False)[0]
        states = (info["Lmax"] + 1) * ((key.lmax + 64) // 64) * 40
        return n * 44 + states + self.shared_of(key)[1] + (1 << 20)

    def create_plan(self, key: PlanKey):
        from .plan import Plan

        th, ph = self.patches[key.patch]
        p = Plan(th, ph, key.lmax, key.spin, key.epsilon, key.precision, device=self.device)
        sb = int(p.info["shared_bytes"])
        return p, p.info["resident_bytes"] - sb, self.shared_of(key)[0], sb

    def drop_plan(self, plan) -> None:
        # the server drops only idle plans, whose batches have all retired:
        # no device synchronisation is needed
        plan.close(sync=False)

    def cost_estimate(self, plan, op: str) -> float:
        """Seconds of GPU time of one request on `plan`: its Legendre work at
        about 25 TFLOP/s (18 FLOP per ring, order and degree) and its NUFFT at
        about 15 ps (FP32) or 40 ps (FP64) per point, as measured on the served
        discs; both operations alike."""
        per_point = 1.5e-11 if plan.info["map_is_fp32"] else 4e-11
        return plan.info["legendre_triples"] * 18 / 25e12 + plan.npoints * per_point

    def footprint(self, plan, op: str, n: int) -> int:
        from .plan import nalm

        alm = 2 * nalm(plan.lmax) * 16
        mp = plan.npoints * (8 if plan.info["map_is_fp32"] else 16)
        return n * (plan.info["workspace_bytes_per_map"] + alm + mp)

    def launch(self, plan, op: str, inputs: list, slot: int):
        torch = self.torch
        s = self.streams[slot]
        s.wait_stream(torch.cuda.current_stream(self.device))
        with torch.cuda.device(self.device), torch.cuda.stream(s):
            x = torch.stack(inputs) if len(inputs) > 1 else inputs[0].unsqueeze(0)
            ws = torch.empty(max(1, len(inputs) * plan.info["workspace_bytes_per_map"]), dtype=torch.uint8,
                             device=self.device)
            out = plan.synth(x, stream=s, workspace=ws) if op == "synth" else plan.adjoint(x, stream=s, workspace=ws)
            ev = torch.cuda.Event()
            ev.record(s)
        return (ev, out, ws, x)

    def ready(self, token) -> bool:
        return token[0].query()

    def results(self, token) -> list:
        out = token[1]
        return [out[i] for i in range(out.shape[0])]

    def release(self, token) -> None:
        pass

    def wait(self, tokens: list, poll: float) -> None:
        # a short sleep keeps the polling host thread from spinning
        if poll > 0:
            time.sleep(poll)
