"""The continuous-batching scheduler on the CPU, against a simulated device:
admission in arrival order within the HBM budget and the launch slots,
overlap of batches, retries of sets that outgrew their reservation, and the
latency / throughput accounting."""
import math

import numpy as np
import pytest

from paper_2307_06345_amd import serving as sv  # host-only module (no device needed)


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def idle(self, dt):
        self.t += max(dt, 1e-6)


class SimDevice:
    """Batches run one after another on a device of `rate` particles/s with a
    fixed launch overhead; completion is seen once the clock passes it."""

    def __init__(self, clock, rate=1e9, overhead=2e-4, budget=None, max_inflight=None, fail_first=()):
        self.clock, self.rate, self.overhead = clock, rate, overhead
        self.busy_until = 0.0
        self.budget, self.max_inflight = budget, max_inflight
        self.inflight = []
        self.fail_first = set(fail_first)
        self.launch_log = []

    def launch(self, group):
        now = self.clock()
        start = max(now, self.busy_until)
        done = start + self.overhead + sum(r.n for r in group) / self.rate
        self.busy_until = done
        nbytes = sum(sv.request_bytes(r.n, sv.leaf_reservation(r.n, r.n_crit, r.full)) for r in group)
        h = {"done": done, "group": list(group), "bytes": nbytes}
        self.inflight.append(h)
        if self.budget is not None:
            assert sum(x["bytes"] for x in self.inflight) <= self.budget
        if self.max_inflight is not None:
            assert len(self.inflight) <= self.max_inflight
        self.launch_log.append((now, [r.rid for r in group], [r.full for r in group]))
        return h

    def poll(self, h):
        return self.clock() >= h["done"]

    def finish(self, h):
        self.inflight.remove(h)
        out = []
        for r in h["group"]:
            if r.rid in self.fail_first and not r.full:
                out.append(("CAPACITY", 0, 0))
            else:
                out.append(("OK", 7 * r.rid + 1, 3))
        return out


def make_requests(count, rate, seed=0, n_lo=12, n_hi=18):
    g = np.random.default_rng(seed)
    sizes = (2.0 ** g.uniform(n_lo, n_hi, count)).astype(int)
    gaps = g.exponential(1.0, count)
    specs = [("uniform" if i % 2 else "plummer", int(sizes[i]), 16 if i % 3 else 64, i + 1, float(gaps[i]))
             for i in range(count)]
    return sv.poisson_requests(specs, rate)


def run(reqs, clock, dev, **kw):
    loop = sv.ServingLoop(dev, clock=clock, idle=clock.idle, **kw)
    return loop.run(reqs)


def test_every_request_completes_once_in_arrival_order():
    clock = Clock()
    dev = SimDevice(clock, max_inflight=3, budget=64 * 10**9)
    reqs = make_requests(300, rate=2000.0)
    done, st = run(reqs, clock, dev, max_inflight=3)
    assert [r.rid for r in done] == list(range(300))
    assert all(r.status == "OK" and r.attempts == 1 for r in done)
    # admission is first come, first served
    order = [rid for _, rids, _ in dev.launch_log for rid in rids]
    assert order == sorted(order)
    for r in done:
        assert r.launched >= r.arrival and r.done > r.launched
    assert st.batches == len(dev.launch_log) and st.max_inflight <= 3
    assert st.requests == 300 and st.particles == sum(r.n for r in reqs)
    lat = np.array([r.latency for r in done]) * 1e3
    assert st.latency_p50_ms == pytest.approx(np.percentile(lat, 50))
    assert st.latency_p99_ms == pytest.approx(np.percentile(lat, 99))
    assert st.particles_per_s == pytest.approx(st.particles / (max(r.done for r in done) - reqs[0].arrival))


def test_requests_arriving_meanwhile_join_the_next_batch():
    """Under load the device is busy; requests that arrived meanwhile are
    launched together as soon as a slot frees (batches grow with the load)."""
    clock = Clock()
    dev = SimDevice(clock, rate=2e8, max_inflight=2)
    reqs = make_requests(400, rate=5000.0)
    done, st = run(reqs, clock, dev, max_inflight=2)
    assert st.mean_batch_requests > 2.0
    assert st.max_inflight == 2
    # the device never idles while requests wait: each batch starts when the previous ends or at launch
    light = make_requests(400, rate=50.0, seed=1)
    clock2 = Clock()
    _, st2 = run(light, clock2, SimDevice(clock2, rate=2e8), max_inflight=2)
    assert st2.mean_batch_requests < st.mean_batch_requests


def test_budget_limits_what_is_in_flight():
    clock = Clock()
    reqs = make_requests(60, rate=1e5, n_lo=16, n_hi=17)
    one = max(sv.request_bytes(r.n, sv.leaf_reservation(r.n, r.n_crit)) for r in reqs)
    budget = int(2.5 * one)
    dev = SimDevice(clock, budget=budget, max_inflight=8)
    done, st = run(reqs, clock, dev, budget_bytes=budget, max_inflight=8)
    assert len(done) == 60 and st.peak_reserved_bytes <= budget  # SimDevice also checks every launch
    assert st.peak_reserved_bytes > budget // 2  # the budget, not the slots, was binding
    assert st.max_inflight < 8
    # everything arrived at once, yet admission waited for memory to be released
    assert max(r.launched - r.arrival for r in done) > 0.0


def test_oversized_request_is_refused():
    clock = Clock()
    reqs = make_requests(3, rate=10.0, n_lo=20, n_hi=20.5)
    with pytest.raises(RuntimeError):
        run(reqs, clock, SimDevice(clock), budget_bytes=1 << 20)


def test_sets_over_their_reservation_are_rebuilt_with_the_full_bound():
    clock = Clock()
    reqs = make_requests(50, rate=3000.0)
    dev = SimDevice(clock, fail_first={3, 17, 40})
    done, st = run(reqs, clock, dev, max_inflight=3)
    assert st.retries == 3 and len(done) == 50
    for r in done:
        assert r.status == "OK"
        assert r.attempts == (2 if r.rid in (3, 17, 40) else 1)
        assert r.full == (r.rid in (3, 17, 40))
    # the second attempt reserved the full leaf bound
    assert any(all(f) and set(rids) & {3, 17, 40} for _, rids, f in dev.launch_log)


def test_reservations_and_rounds():
    assert sv.leaf_bound(1000, 15) == 7 * 21 * (1000 // 16) + 1
    assert sv.leaf_reservation(1 << 20, 16) == 8 * (1 << 20) // 17 + 64
    assert sv.leaf_reservation(1 << 20, 16, full=True) == sv.leaf_bound(1 << 20, 16)
    assert sv.leaf_reservation(10, 64) == sv.leaf_bound(10, 64) == 1  # never above the bound
    r = sv.Request(0, 0.0, 1 << 22, "plummer", 16, 5, 1)
    # log8(2^22 / 17) = 5.96 -> 6 levels, + 2 + slack 5
    assert sv.rounds_for([r]) == 13
    r.full = True
    assert sv.rounds_for([r]) == 22
    assert sv.request_bytes(100, 1) > 64 * 100
    assert math.isnan(sv.Request(1, 0.0, 5, "uniform", 8, 5, 2).done)


def test_request_bytes_cover_the_batch_buffers():
    """The reservation model is an upper bound of what a group's batched build
    holds on the device (its workspace and output buffers, from the plan's own
    layout, plus the coordinates), for single requests over the serving sizes
    (up to 2^22, both N_crit, the full leaf bound of a retry) and for groups."""
    cs = pytest.importorskip("paper_2307_06345_amd")

    def actual(reqs, full=False):
        sets = [(n, sv.BOXES[k], 1, nc, sv.leaf_reservation(n, nc, full)) for k, n, nc in reqs]
        lay = cs.batch_layout(sets)
        return cs.BatchArena.bytes_of(cs.BatchArena.need(lay)) + 24 * sum(n for _, n, _ in reqs)

    for n in (1, 4096, 65537, 1 << 20, 3_000_001, 1 << 22):
        for nc in (16, 64):
            for full in (False, True):
                if full and n > (1 << 20):
                    continue  # the full bound of the largest sizes is plan-only arithmetic, same formula
                model = sv.request_bytes(n, sv.leaf_reservation(n, nc, full))
                assert model >= actual([("plummer", n, nc)], full), (n, nc, full)
    import workloads as wl

    rng = np.random.default_rng(3)
    specs = wl.serving_specs(count=400, seed=11)
    for _ in range(20):
        idx = rng.choice(len(specs), size=int(rng.integers(1, 40)), replace=False)
        grp = [(specs[i][0], specs[i][1], specs[i][2]) for i in idx]
        model = sum(sv.request_bytes(n, sv.leaf_reservation(n, nc)) for _, n, nc in grp)
        assert model >= actual(grp), len(grp)
