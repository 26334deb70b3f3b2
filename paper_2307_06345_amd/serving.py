"""Continuous-batching serving loop for octree-build requests on one GPU.

Requests arrive over time, each a particle set (size, kind, N_crit, seed
stream). The loop
  * admits arrived requests in arrival order while their memory reservation
    fits the HBM budget and a launch slot is free,
  * builds every admitted group as one batched build (all its sets in one
    launch sequence) on a HIP stream of its own, so up to `max_inflight`
    batches run on the device at once and requests that arrive meanwhile join
    the next group as slots and memory free up,
  * retires a batch when its completion event has fired, releasing its
    memory; a set that outgrew its leaf reservation, or needed more rebalance
    rounds than were enqueued, is built again with the full leaf bound and
    L + 1 rounds.
Latency of a request = completion time - arrival time.

The scheduler is independent of the device: an executor launches groups and
reports completion. GpuExecutor draws each request's coordinates on the device
(standing for the request payload arriving in HBM) and runs the batched build
of libcstone; tests drive the scheduler with a simulated executor too.
"""
from __future__ import annotations

import collections
import math
import time
from dataclasses import dataclass, field

import numpy as np

L = 21

UNIT_BOX = ((0.0, 0.0, 0.0), (1.0, 1.0, 1.0))
PLUMMER_BOX = ((-20.0,) * 3, (20.0,) * 3)
BOXES = {"uniform": UNIT_BOX, "plummer": PLUMMER_BOX}


@dataclass
class Request:
    rid: int
    arrival: float  # seconds from the start of the run
    n: int
    kind: str
    n_crit: int
    seed: int
    stream: int
    curve: int = 1  # Hilbert
    full: bool = False  # reserve the full leaf bound (retries)
    # outcome
    launched: float = math.nan
    done: float = math.nan
    status: str = ""
    n_leaves: int = 0
    rounds: int = 0
    attempts: int = 0

    @property
    def box(self):
        return BOXES[self.kind]

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def leaf_bound(n: int, n_crit: int) -> int:
    """Leaves a from-root build can reach: at most n / (n_crit + 1) internal
    nodes per level, L levels, 7 leaves added per internal node."""
    return 7 * L * (n // (n_crit + 1)) + 1


def leaf_reservation(n: int, n_crit: int, full: bool = False) -> int:
    """Leaf capacity reserved for a request: 8 n / (n_crit + 1) + 64 (above
    every leaf count seen on uniform and Plummer sets), or the full bound."""
    b = leaf_bound(n, n_crit)
    return b if full else min(b, 8 * n // (n_crit + 1) + 64)


def request_bytes(n: int, cap: int) -> int:
    """HBM reserved for one request: coordinates 24 n, sorted keys and
    permutation 12 n, unsorted keys and sort buffers 28 n (plus look-back rows
    and digit counts), leaves and counts 12 (cap + 1), nodes 12 node slots,
    rebalance arrays 32 (cap + 1) and split list, and a fixed 128 KiB (the
    set's digit counts of every sort pass, its tables and level offsets). A
    test checks it against the plan's own layout."""
    node_cap = cap + (cap - 1) // 7
    return 64 * n + 12 * (cap + 1) + 12 * node_cap + 48 * (cap + 1) + 131072


def rounds_for(reqs) -> int:
    """Rebalance rounds to enqueue: from the root a build takes depth + 1
    rounds; log8(n / (n_crit + 1)) + 2 for an even set, plus slack for
    clustered ones (a set that needs more is built again with L + 1)."""
    r = 1
    for q in reqs:
        if q.full:
            return L + 1
        ratio = q.n / (q.n_crit + 1)
        d = 0
        while ratio > 1.0:
            ratio /= 8.0
            d += 1
        r = max(r, d + 2 + 5)
    return min(r, L + 1)


@dataclass
class Stats:
    requests: int = 0
    particles: int = 0
    makespan_s: float = 0.0
    particles_per_s: float = 0.0
    latency_p50_ms: float = 0.0
    latency_p99_ms: float = 0.0
    latency_mean_ms: float = 0.0
    batches: int = 0
    mean_batch_requests: float = 0.0
    max_inflight: int = 0
    peak_reserved_bytes: int = 0
    retries: int = 0
    statuses: dict = field(default_factory=dict)


class ServingLoop:
    def __init__(self, executor, budget_bytes: int = 64 * 10**9, max_inflight: int = 3,
                 max_batch_particles: int = 1 << 27, max_batch_requests: int = 1024,
                 clock=time.perf_counter, idle=None):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.max_inflight = int(max_inflight)
        self.max_batch_particles = int(max_batch_particles)
        self.max_batch_requests = int(max_batch_requests)
        self.clock = clock
        self.idle = idle  # idle(seconds): wait for at most that long (default: sleep / spin)

    def _wait(self, dt: float):
        if self.idle is not None:
            self.idle(dt)
        elif dt > 2e-4:
            time.sleep(min(dt, 1e-3) - 1e-4)

    def run(self, requests) -> tuple:
        reqs = sorted(requests, key=lambda r: (r.arrival, r.rid))
        pending = collections.deque(reqs)  # not yet arrived
        queue = collections.deque()  # arrived, waiting for admission
        inflight = []  # (handle, group, bytes)
        reserved = 0
        st = Stats(requests=len(reqs), particles=sum(r.n for r in reqs))
        done = []
        sizes = []
        t0 = self.clock()
        while pending or queue or inflight:
            now = self.clock() - t0
            progressed = False
            while pending and pending[0].arrival <= now:
                queue.append(pending.popleft())
                progressed = True
            # retire finished batches
            for item in list(inflight):
                h, group, nbytes = item
                if not self.ex.poll(h):
                    continue
                t_done = self.clock() - t0
                outcome = self.ex.finish(h)
                inflight.remove(item)
                reserved -= nbytes
                retry = []
                for r, (status, nl, rounds) in zip(group, outcome):
                    r.attempts += 1
                    if status in ("CAPACITY", "NOT_CONVERGED") and not r.full:
                        r.full = True
                        retry.append(r)
                        st.retries += 1
                        continue
                    r.done, r.status, r.n_leaves, r.rounds = t_done, status, nl, rounds
                    done.append(r)
                queue.extendleft(reversed(retry))  # retried requests go first
                progressed = True
            # admit one group into a free slot
            if queue and len(inflight) < self.max_inflight:
                group, parts, nbytes = [], 0, 0
                while queue and len(group) < self.max_batch_requests:
                    r = queue[0]
                    b = request_bytes(r.n, leaf_reservation(r.n, r.n_crit, r.full))
                    if group and parts + r.n > self.max_batch_particles:
                        break
                    if reserved + nbytes + b > self.budget:
                        if not group and not inflight:
                            raise RuntimeError(f"request {r.rid} needs {b} bytes, above the budget")
                        break
                    group.append(queue.popleft())
                    parts += r.n
                    nbytes += b
                if group:
                    t_l = self.clock() - t0
                    for r in group:
                        r.launched = t_l
                    inflight.append((self.ex.launch(group), group, nbytes))
                    reserved += nbytes
                    st.batches += 1
                    sizes.append(len(group))
                    st.max_inflight = max(st.max_inflight, len(inflight))
                    st.peak_reserved_bytes = max(st.peak_reserved_bytes, reserved)
                    progressed = True
            if not progressed:
                nxt = pending[0].arrival - (self.clock() - t0) if pending else 0.0
                self._wait(nxt if (not inflight and not queue) else min(nxt, 5e-5) if pending else 5e-5)
        lat = np.array([r.latency for r in done]) * 1e3
        first = min(r.arrival for r in reqs) if reqs else 0.0
        last = max(r.done for r in done) if done else 0.0
        st.makespan_s = last - first
        st.particles_per_s = st.particles / st.makespan_s if st.makespan_s > 0 else 0.0
        if lat.size:
            st.latency_p50_ms = float(np.percentile(lat, 50))
            st.latency_p99_ms = float(np.percentile(lat, 99))
            st.latency_mean_ms = float(lat.mean())
        st.mean_batch_requests = float(np.mean(sizes)) if sizes else 0.0
        st.statuses = dict(collections.Counter(r.status for r in done))
        return sorted(done, key=lambda r: r.rid), st


class _Slot:
    """A launch slot: a stream and the device buffers its batches reuse."""

    def __init__(self, stream):
        self.stream = stream
        self.arena = None
        self.coords = None  # x, y, z, each of the capacity below
        self.coord_cap = 0
        self.host_results = None  # pinned copy of the last batch's per-set results
        self.host_stage = None  # pinned staging of the last batch's plan tables

    @property
    def nbytes(self) -> int:
        return (self.arena.nbytes if self.arena is not None else 0) + 24 * self.coord_cap

    def drop(self):
        self.arena, self.coords, self.coord_cap = None, None, 0


class GpuExecutor:
    """Runs each admitted group as one batched build on a slot of its own.

    A slot keeps its device buffers (coordinates, the batch's outputs and
    workspace) from one group to the next and grows them only when a group
    needs more, so a launch allocates nothing in the common case; the plan of
    each group is made on the host. With `budget_bytes`, the slots' buffers
    together stay within it: before a slot grows, idle slots give theirs
    back."""

    def __init__(self, max_inflight: int = 3, device="cuda", keep=(), reserve=None, sink=None,
                 budget_bytes: int | None = None):
        import torch

        import workloads

        from . import Batch  # noqa: F401  (fails loudly without libcstone)

        self.torch = torch
        self.wl = workloads
        self.device = torch.device(device)
        self.free = [_Slot(torch.cuda.Stream(self.device)) for _ in range(max_inflight)]
        self.slots = list(self.free)
        self.budget = budget_bytes
        self.peak_buffer_bytes = 0
        self.grows = 0
        self.keep = set(keep)
        self.kept = {}  # rid -> dict of host outputs
        self.sink = sink  # sink(rid, outputs): takes the kept outputs instead of self.kept
        # leaf capacity of a request (default: leaf_reservation)
        self.reserve = reserve or (lambda r: leaf_reservation(r.n, r.n_crit, r.full))

    def _buffers(self, slot, need, total):
        """Make the slot's buffers large enough for a group with these plan
        needs and particles. Only the buffers that are too small grow, with
        25% headroom unless that would not fit the budget. Returns the slot's
        batch buffers."""
        from . import BatchArena

        if slot.arena is not None and slot.arena.fits(need) and total <= slot.coord_cap:
            return slot.arena
        have = slot.arena.cap if slot.arena is not None else (0,) * len(need)
        exact = tuple(max(int(v), c) for v, c in zip(need, have))
        roomy = tuple(c if int(v) <= c else max(int(v * 1.25), 1) for v, c in zip(need, have))
        exact_cap = max(total, slot.coord_cap, 1)
        roomy_cap = slot.coord_cap if total <= slot.coord_cap else max(int(total * 1.25), 1)
        grown, cap = roomy, roomy_cap
        if self.budget is not None:
            busy = sum(s.nbytes for s in self.slots if s is not slot and s not in self.free)
            idle = [s for s in self.free if s is not slot]
            if busy + BatchArena.bytes_of(roomy) + 24 * roomy_cap > self.budget:
                grown, cap = exact, exact_cap
            new_bytes = BatchArena.bytes_of(grown) + 24 * cap
            for s in idle:  # idle slots give their buffers back first
                if busy + sum(o.nbytes for o in idle) + new_bytes <= self.budget:
                    break
                s.drop()
        # the slot is idle (its last batch has completed), so its buffers can be replaced
        if slot.arena is None:
            slot.arena = BatchArena(self.device, grown)
        else:
            slot.arena.grow(grown)
        if cap > slot.coord_cap:
            slot.coords = None
            slot.coords = tuple(self.torch.empty(cap, dtype=self.torch.float64, device=self.device) for _ in range(3))
            slot.coord_cap = cap
        self.grows += 1
        self.peak_buffer_bytes = max(self.peak_buffer_bytes, sum(s.nbytes for s in self.slots))
        return slot.arena

    def _stage(self, slot, nbytes):
        """The slot's pinned staging buffer for plan tables (grown as needed;
        its last upload has completed, since the slot is idle)."""
        if slot.host_stage is None or slot.host_stage.numel() < nbytes:
            slot.host_stage = None
            slot.host_stage = self.torch.empty(max(int(nbytes * 1.25), 1 << 16), dtype=self.torch.uint8,
                                               pin_memory=True)
        return slot.host_stage

    def launch(self, group):
        from . import Batch

        torch = self.torch
        slot = self.free.pop()
        stream = slot.stream
        sets = [(r.n, r.box, r.curve, r.n_crit, self.reserve(r)) for r in group]
        total = sum(r.n for r in group)
        with torch.cuda.stream(stream):  # buffers made and used in the slot's stream order
            b = Batch(sets, device=self.device, arena=lambda need: self._buffers(slot, need, total),
                      stage=lambda nbytes: self._stage(slot, nbytes))
            b.set_rounds(rounds_for(group))
            x, y, z = (c[:max(total, 1)] for c in slot.coords)
            self.wl.device_generate([(r.kind, r.n, r.seed, r.stream) for r in group], x, y, z, stream=stream)
            b.build(x, y, z, stream=stream)
            # the per-set results come back on the slot's own stream, so that
            # finishing a group needs no device call (a copy on the default
            # stream would wait behind whatever shares its hardware queue)
            k = 4 * len(group)
            if slot.host_results is None or slot.host_results.numel() < k:
                slot.host_results = torch.empty(max(k, 4096), dtype=torch.int32, pin_memory=True)
            slot.host_results[:k].copy_(b.results[:k], non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(stream)
        return {"slot": slot, "stream": stream, "event": ev, "batch": b, "coords": (x, y, z), "group": group}

    def poll(self, h) -> bool:
        return h["event"].query()

    def finish(self, h):
        from . import STATUS

        b = h["batch"]
        group = h["group"]
        res = h["slot"].host_results[:4 * len(group)].numpy().view(np.uint32).reshape(len(group), 4)
        out = []
        for s, r in enumerate(group):
            status = STATUS.get(int(res[s, 3]), str(int(res[s, 3])))
            out.append((status, int(res[s, 0]), int(res[s, 2])))
            if r.rid in self.keep and status == "OK":
                with self.torch.cuda.stream(h["stream"]):  # the copies below wait on the slot's stream only
                    rec = self._outputs(b, s, res[s], h["coords"])
                if self.sink is not None:
                    self.sink(r.rid, rec)
                else:
                    self.kept[r.rid] = rec
        self.free.append(h["slot"])
        return out

    @staticmethod
    def _outputs(b, s, res, coords):
        from . import to_numpy

        v = b.set_view(s, res)
        p0, p1 = int(b.particle_offsets[s]), int(b.particle_offsets[s + 1])
        rec = {k: to_numpy(v[k]).copy() for k in
               ("sorted_keys", "perm", "leaves", "counts", "node_keys", "child", "level_offsets")}
        rec.update({a: coords[i][p0:p1].cpu().numpy() for i, a in enumerate("xyz")})
        return rec


def poisson_requests(specs, rate_per_s: float):
    """Requests from (kind, n, n_crit, stream, unit gap) specs with exponential
    inter-arrival gaps scaled to `rate_per_s` arrivals per second."""
    t = 0.0
    out = []
    for i, (kind, n, n_crit, stream, gap) in enumerate(specs):
        t += gap / rate_per_s
        out.append(Request(rid=i, arrival=t, n=int(n), kind=kind, n_crit=int(n_crit), seed=5, stream=int(stream)))
    return out
