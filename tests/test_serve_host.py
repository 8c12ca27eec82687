"""Scheduling logic of the serving form, on the CPU with a simulated executor:
continuous admission, batching by (plan, operation), slot and memory limits,
LRU plan eviction, error paths and latency statistics."""
import math

import pytest

from paper_2603_17166_amd.serve import (PlanKey, Server, latency_stats, percentile, poisson_arrivals,
                                        run_closed_loop, run_open_loop)


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeExecutor:
    """Batches take `cost(key, op, n)` seconds of simulated time; the result of
    each request is (rid tag, op, plan key) so routing can be checked."""

    def __init__(self, clock, plan_bytes=100, per_map=10, cost=None, fail_patch=None):
        self.clock = clock
        self.plan_bytes = plan_bytes
        self.per_map = per_map
        self.cost = cost or (lambda key, op, n: 1.0 + 0.1 * n)
        self.fail_patch = fail_patch
        self.live_plans = set()
        self.created = []
        self.launches = []
        self.running = []

    def plan_bytes_estimate(self, key):
        return self.plan_bytes

    def create_plan(self, key):
        if key.patch == self.fail_patch:
            raise ValueError("bad patch")
        self.created.append(key)
        self.live_plans.add(key)
        return key, self.plan_bytes

    def drop_plan(self, h):
        self.live_plans.remove(h)

    def footprint(self, h, op, n):
        return n * self.per_map

    def launch(self, h, op, inputs, slot):
        assert h in self.live_plans
        tok = {"end": self.clock() + self.cost(h, op, len(inputs)), "out": [(x, op, h) for x in inputs], "slot": slot}
        self.launches.append((h, op, len(inputs), slot, self.clock()))
        self.running.append(tok)
        return tok

    def ready(self, tok):
        return self.clock() >= tok["end"]

    def results(self, tok):
        return tok["out"]

    def release(self, tok):
        self.running.remove(tok)

    def wait(self, toks, poll):
        # advance simulated time to the next completion
        self.clock.t = max(self.clock.t, min(t["end"] for t in toks))


def K(p="a", l=64, s=0):
    return PlanKey(p, l, s, 1e-5, "fp32")


def test_results_routed_and_batched():
    c = Clock()
    ex = FakeExecutor(c)
    srv = Server(ex, memory_budget=10_000, n_slots=2, max_batch=3, clock=c)
    reqs = [srv.submit(K("a"), "synth", i) for i in range(5)] + [srv.submit(K("b"), "adjoint", 10 + i) for i in range(2)]
    srv.run_until_idle()
    for r in reqs:
        assert r.result == (r.data, r.op, r.key)
        assert r.error is None and r.done
    sizes = sorted(n for _, _, n, _, _ in ex.launches)
    assert sizes == [2, 2, 3]  # a:3 + a:2 (head first, FIFO), b:2
    assert srv.max_concurrent == 2


def test_fifo_head_first_and_slot_limit():
    c = Clock()
    ex = FakeExecutor(c)
    srv = Server(ex, memory_budget=10_000, n_slots=1, max_batch=4, clock=c)
    r1 = srv.submit(K("a"), "synth", 1)
    r2 = srv.submit(K("b"), "synth", 2)
    r3 = srv.submit(K("a"), "synth", 3)
    srv.step()
    assert len(srv.inflight) == 1 and r1.batch_size == 2 and r3.batch_size == 2  # same plan/op joins the head
    assert math.isnan(r2.t_admit)
    srv.run_until_idle()
    assert r2.t_admit >= r1.t_done
    assert max(len(ex.running), 0) == 0


def test_continuous_admission_while_running():
    """A request that arrives while a batch runs starts as soon as a slot is free,
    without waiting for the running batch."""
    c = Clock()
    ex = FakeExecutor(c, cost=lambda k, op, n: 10.0 if k.patch == "big" else 1.0)
    srv = Server(ex, memory_budget=10_000, n_slots=2, max_batch=4, clock=c)
    big = srv.submit(K("big"), "synth", 0)
    srv.step()
    c.t = 2.0
    small = srv.submit(K("small"), "adjoint", 1)
    srv.step()
    assert small.t_admit == 2.0
    srv.run_until_idle()
    assert small.t_done == 3.0 and big.t_done == 10.0
    assert small.latency == pytest.approx(1.0)


def test_memory_budget_never_exceeded_and_lru_eviction():
    c = Clock()
    ex = FakeExecutor(c, plan_bytes=100, per_map=30)
    # room for two plans plus one batch of 3 maps at most
    srv = Server(ex, memory_budget=290, n_slots=4, max_batch=8, clock=c)
    seen = []
    orig = srv._admit_head

    def admit(head):
        ok = orig(head)
        seen.append(srv._used())
        return ok
    srv._admit_head = admit
    keys = [K(p) for p in "abcab"]
    reqs = [srv.submit(k, "synth", i) for i, k in enumerate(keys) for _ in range(4)]
    srv.run_until_idle()
    assert all(r.error is None for r in reqs)
    assert max(seen) <= 290 and srv.peak_bytes <= 290
    assert srv.plans_evicted >= 1
    assert len(ex.live_plans) <= 2


def test_request_too_large_fails_cleanly():
    c = Clock()
    ex = FakeExecutor(c, plan_bytes=100, per_map=1000)
    srv = Server(ex, memory_budget=500, n_slots=2, clock=c)
    r = srv.submit(K("a"), "synth", 0)
    ok = srv.submit(K("b"), "synth", 1)
    ex.per_map = 1000
    srv.run_until_idle()
    assert r.error is not None and "memory budget" in r.error
    assert ok.error is not None  # same footprint rule
    ex2 = FakeExecutor(c, plan_bytes=600)
    srv2 = Server(ex2, memory_budget=500, n_slots=2, clock=c)
    r2 = srv2.submit(K("a"), "synth", 0)
    srv2.run_until_idle()
    assert "memory budget" in r2.error


def test_plan_creation_error_fails_only_that_request():
    c = Clock()
    ex = FakeExecutor(c, fail_patch="bad")
    srv = Server(ex, memory_budget=10_000, clock=c)
    bad = srv.submit(K("bad"), "synth", 0)
    good = srv.submit(K("a"), "synth", 1)
    srv.run_until_idle()
    assert "plan creation failed" in bad.error
    assert good.error is None and good.result[0] == 1


def test_invalid_op_rejected():
    srv = Server(FakeExecutor(Clock()), memory_budget=100)
    with pytest.raises(ValueError):
        srv.submit(K(), "inverse", 0)
    with pytest.raises(ValueError):
        Server(FakeExecutor(Clock()), memory_budget=0)


def test_open_loop_poisson_stats():
    c = Clock()
    ex = FakeExecutor(c, cost=lambda k, op, n: 0.01 * n)
    srv = Server(ex, memory_budget=1 << 30, n_slots=2, max_batch=4, clock=c)
    offs = poisson_arrivals(400, 50.0, 7)
    assert all(b > a for a, b in zip(offs, offs[1:]))
    assert abs(len(offs) / offs[-1] - 50.0) < 10.0
    specs = [(K("ab"[i % 2]), "synth" if i % 3 else "adjoint", i) for i in range(400)]

    # the simulated clock moves only through executor waits; advance it to the next arrival too
    import paper_2603_17166_amd.serve as sv
    real_sleep = sv.time.sleep
    sv.time.sleep = lambda dt: setattr(c, "t", c.t + dt)
    try:
        reqs = run_open_loop(srv, specs, offs)
    finally:
        sv.time.sleep = real_sleep
    st = latency_stats(reqs, skip=20)
    assert st["n"] == 380
    assert st["p50_ms"] <= st["p99_ms"]
    assert all(r.result[0] == r.data for r in reqs)
    assert all(r.latency >= 0.0 for r in reqs)


def test_closed_loop_and_percentiles():
    c = Clock()
    ex = FakeExecutor(c, cost=lambda k, op, n: 1.0)
    srv = Server(ex, memory_budget=1 << 30, n_slots=2, max_batch=2, clock=c)
    reqs, secs = run_closed_loop(srv, [(K(), "synth", i) for i in range(8)])
    assert secs == pytest.approx(2.0)  # 4 batches of 2 on 2 slots
    assert percentile([3, 1, 2, 4], 50) == 2 and percentile([3, 1, 2, 4], 100) == 4
    assert percentile(list(range(1, 101)), 99) == 99


class SharedExecutor(FakeExecutor):
    """Plans of the same lmax share a table of `shared` bytes; the created
    plans hold `actual` bytes of their own (more than the estimate)."""

    def __init__(self, clock, shared=50, actual=None, **kw):
        super().__init__(clock, **kw)
        self.shared = shared
        self.actual = actual if actual is not None else self.plan_bytes

    def shared_of(self, key):
        return ("tab", key.lmax), self.shared

    def plan_bytes_estimate(self, key):
        return self.plan_bytes + self.shared

    def create_plan(self, key):
        h, _ = super().create_plan(key)
        return h, self.actual, ("tab", key.lmax), self.shared


def test_shared_table_counted_once():
    c = Clock()
    ex = SharedExecutor(c, shared=50, plan_bytes=100)
    srv = Server(ex, memory_budget=10_000, n_slots=1, max_batch=1, clock=c)
    for p in ("a", "b", "c"):
        srv.submit(K(p, l=64), "synth", 0)
    srv.submit(K("a", l=128), "synth", 0)
    srv.run_until_idle()
    assert srv.resident == 4 * 100 + 2 * 50   # two tables (lmax 64 and 128), each once
    assert srv.shared == {("tab", 64): [50, 3], ("tab", 128): [50, 1]}
    # evicting plans releases a table with the last plan that holds it
    assert srv._evict_for(10_000 - srv._used() + 150, None)   # the two least recently used plans go
    assert srv.shared == {("tab", 64): [50, 1], ("tab", 128): [50, 1]} and srv.resident == 300
    assert srv._evict_for(10**9, None) is False                # every plan goes, then nothing is left
    assert srv.plans == {} and srv.shared == {} and srv.resident == 0


def test_budget_rechecked_after_creation():
    """The estimate (100 own bytes) is below what a plan holds (600): once the
    second plan exists the budget is exceeded, and the idle first plan is
    evicted (the shared table stays: the new plan holds it)."""
    c = Clock()
    ex = SharedExecutor(c, shared=50, plan_bytes=100, actual=600, per_map=0)
    srv = Server(ex, memory_budget=1000, n_slots=1, max_batch=1, clock=c)
    srv.submit(K("a"), "synth", 0)
    srv.run_until_idle()
    assert srv._used() == 650
    srv.submit(K("b"), "synth", 0)
    srv.run_until_idle()
    assert srv.plans_evicted == 1 and set(ex.live_plans) == {K("b")}
    assert srv._used() == 650 and srv.shared == {("tab", 64): [50, 1]}


class CostExecutor(FakeExecutor):
    """FakeExecutor that also reports each plan's cost, as the device executor does."""

    def cost_estimate(self, h, op):
        return self.cost(h, op, 1)


def test_sjf_admits_cheapest_first():
    """One slot: after the first batch, the cheap plan's request goes before
    the older expensive ones (their plans are known from earlier requests)."""
    c = Clock()
    ex = CostExecutor(c, cost=lambda k, op, n: 10.0 if k.patch == "big" else 1.0)
    srv = Server(ex, memory_budget=10_000, n_slots=1, max_batch=1, clock=c, policy="sjf", max_wait=100.0)
    warm = [srv.submit(K("big"), "synth", 0), srv.submit(K("small"), "synth", 1)]
    srv.run_until_idle()
    assert all(r.done for r in warm)
    t0 = c.t
    b1 = srv.submit(K("big"), "synth", 2, t_arrival=t0)
    b2 = srv.submit(K("big"), "synth", 3, t_arrival=t0)
    s1 = srv.submit(K("small"), "synth", 4, t_arrival=t0)
    srv.run_until_idle()
    assert s1.t_admit < b1.t_admit < b2.t_admit  # cheapest first, then in arrival order
    fifo = Server(CostExecutor(c), memory_budget=10_000, n_slots=1, max_batch=1, clock=c)
    assert fifo.policy == "fifo"


def test_sjf_starvation_guard():
    """A request that waited past max_wait is admitted before cheaper ones."""
    c = Clock()
    ex = CostExecutor(c, cost=lambda k, op, n: 10.0 if k.patch == "big" else 1.0)
    srv = Server(ex, memory_budget=10_000, n_slots=1, max_batch=1, clock=c, policy="sjf", max_wait=5.0)
    for p in ("big", "small"):
        srv.submit(K(p), "synth", 0)
    srv.run_until_idle()
    t0 = c.t
    big = srv.submit(K("big"), "synth", 1, t_arrival=t0)
    smalls = [srv.submit(K("small"), "synth", 10 + i, t_arrival=t0 + 0.5 * i) for i in range(20)]
    srv.run_until_idle()
    # the big request waits at most about max_wait plus one running batch, not for all 20 small ones
    assert big.t_admit - t0 <= 5.0 + 1.0 + 1e-9
    assert sum(1 for r in smalls if r.t_admit < big.t_admit) < 20


def test_policy_arguments_checked():
    with pytest.raises(ValueError):
        Server(FakeExecutor(Clock()), memory_budget=10, policy="lifo")
    with pytest.raises(ValueError):
        Server(FakeExecutor(Clock()), memory_budget=10, policy="sjf", max_wait=0.0)
