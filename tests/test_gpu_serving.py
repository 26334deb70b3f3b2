"""GPU checks of the serving path: the device input generator (Philox
known answers, determinism, a set drawn alone equals the same set drawn in a
group), and continuous batching: every request's tree built in the mix of a
serving run is bit-identical to the same request built alone (plain build and
batch of one), and to the oracle on a sample."""
import concurrent.futures as cf

import numpy as np
import pytest
import torch

import oracle
import workloads as wl

pytestmark = pytest.mark.gpu

cs = pytest.importorskip("paper_2307_06345_amd")
from paper_2307_06345_amd import serving as sv  # noqa: E402


def say(*a):
    print("[case]", *a, flush=True)


def host(t):
    return cs.to_numpy(t)


def eq(a, b, what):
    a = np.asarray(a)
    b = np.asarray(b)
    assert a.shape == b.shape, (what, a.shape, b.shape)
    bad = np.nonzero(a != b)[0]
    assert bad.size == 0, f"{what}: {bad.size} mismatches, first at {bad[:5]}"


def test_device_philox_known_answers():
    """Philox4x32-10 known-answer vectors (Salmon et al., SC'11 reference set)."""
    say("philox KAT")
    got = wl.device_philox(np.array([[0, 0, 0, 0]], dtype=np.uint32), (0, 0))
    assert [hex(v) for v in got[0]] == ["0x6627e8d5", "0xe169c58d", "0xbc57ac4c", "0x9b00dbd8"]
    got = wl.device_philox(np.array([[0xffffffff] * 4], dtype=np.uint32), (0xffffffff, 0xffffffff))
    assert [hex(v) for v in got[0]] == ["0x408f276d", "0x41c83b0e", "0xa20bc7c6", "0x6d5451fd"]
    got = wl.device_philox(np.array([[0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344]], dtype=np.uint32),
                           (0xa4093822, 0x299f31d0))
    assert [hex(v) for v in got[0]] == ["0xd16cfe09", "0x94fdcceb", "0x5001e420", "0x24126ea1"]


def test_device_sets_are_keyed_per_set():
    specs = [("uniform", 5000, 5, 11), ("plummer", 7001, 5, 12), ("uniform", 1, 5, 13), ("plummer", 40000, 5, 14)]
    say("device generator", specs)
    x, y, z, offs = wl.device_sets(specs)
    torch.cuda.synchronize()
    X, Y, Z = (host(t) for t in (x, y, z))
    for k, spec in enumerate(specs):
        a, b = offs[k], offs[k + 1]
        xa, ya, za, oa = wl.device_sets([spec])  # the same set alone
        eq(host(xa)[:spec[1]], X[a:b], f"set {k} x alone vs group")
        eq(host(za)[:spec[1]], Z[a:b], f"set {k} z alone vs group")
        if spec[0] == "uniform":
            assert X[a:b].min() >= 0.0 and X[a:b].max() < 1.0
        else:
            r = np.sqrt(X[a:b] ** 2 + Y[a:b] ** 2 + Z[a:b] ** 2)
            assert r.max() <= 20.0 + 1e-9
            if spec[1] > 10000:  # Plummer half-mass radius (a = 1): (2^(2/3) - 1)^(-1/2) = 1.305
                assert abs(np.median(r) - 1.305) < 0.05
    x2, _, _, _ = wl.device_sets(specs)
    eq(host(x2), X, "second draw")


def _alone(rec, kind, n, n_crit):
    box = sv.BOXES[kind]
    x, y, z = (cs.from_numpy(rec[a], "cuda") for a in "xyz")
    r = cs.build(x, y, z, box, cs.HILBERT, n_crit)
    b = cs.Batch([(n, box, cs.HILBERT, n_crit)])
    b.build(x, y, z)
    torch.cuda.synchronize()
    return r, b.set_view(0)


def _serve(reqs, keep, reserve=None, **kw):
    ex = sv.GpuExecutor(max_inflight=3, keep=keep, reserve=reserve)
    loop = sv.ServingLoop(ex, **kw)
    done, st = loop.run(reqs)
    torch.cuda.synchronize()
    return ex, done, st


def test_serving_results_equal_alone():
    specs = wl.serving_specs(count=160, seed=7, log2_min=12.0, log2_max=16.5)
    reqs = sv.poisson_requests(specs, rate_per_s=20000.0)
    keep = set(range(0, 160, 9))
    say("serving 160 requests, kept", sorted(keep))
    ex, done, st = _serve(reqs, keep)
    assert len(done) == 160 and all(r.status == "OK" for r in done), st.statuses
    assert st.batches < 160  # requests shared batches
    say("batches", st.batches, "mean", st.mean_batch_requests, "max in flight", st.max_inflight)
    for rid in sorted(keep):
        r, rec = done[rid], ex.kept[rid]
        xa, ya, za, _ = wl.device_sets([(r.kind, r.n, r.seed, r.stream)])
        eq(host(xa)[:r.n], rec["x"], f"request {rid} coordinates")
        plain, one = _alone(rec, r.kind, r.n, r.n_crit)
        for name, a, b in (("sorted_keys", plain.sorted_keys, one["sorted_keys"]), ("perm", plain.perm, one["perm"]),
                           ("leaves", plain.leaves, one["leaves"]), ("counts", plain.counts, one["counts"]),
                           ("node_keys", plain.node_keys, one["node_keys"]), ("child", plain.child, one["child"]),
                           ("level_offsets", plain.level_offsets, one["level_offsets"])):
            eq(rec[name], host(a), f"request {rid} {name}: mix vs plain alone")
            eq(rec[name], host(b), f"request {rid} {name}: mix vs batch of one")
        assert r.n_leaves == plain.leaves.numel() - 1 and r.rounds == plain.rounds
    for rid in sorted(keep)[:4]:
        r, rec = done[rid], ex.kept[rid]
        o = oracle.build_tree(rec["x"], rec["y"], rec["z"], sv.BOXES[r.kind], cs.HILBERT, r.n_crit)
        eq(rec["leaves"], o["K"], f"request {rid} leaves vs oracle")
        eq(rec["perm"], o["perm"], f"request {rid} perm vs oracle")
        eq(rec["node_keys"], o["NK"], f"request {rid} NK vs oracle")


def test_serving_retries_sets_over_their_reservation():
    specs = wl.serving_specs(count=24, seed=8, log2_min=12.0, log2_max=14.0)
    reqs = sv.poisson_requests(specs, rate_per_s=50000.0)
    keep = set(range(24))
    tiny = {2, 5, 11}  # first attempt with room for one leaf only

    def reserve(r):
        return 1 if (r.rid in tiny and not r.full) else sv.leaf_reservation(r.n, r.n_crit, r.full)

    say("serving with forced capacity overflow", sorted(tiny))
    ex, done, st = _serve(reqs, keep, reserve=reserve)
    assert all(r.status == "OK" for r in done), st.statuses
    assert st.retries >= len(tiny)
    for rid in tiny:
        assert done[rid].attempts == 2 and done[rid].full
    for rid in sorted(keep)[:8] + sorted(tiny):
        r, rec = done[rid], ex.kept[rid]
        plain, _ = _alone(rec, r.kind, r.n, r.n_crit)
        eq(rec["leaves"], host(plain.leaves), f"request {rid} leaves vs alone")
        eq(rec["node_keys"], host(plain.node_keys), f"request {rid} NK vs alone")


def _digest(rec, names):
    import hashlib

    return {k: hashlib.blake2b(np.ascontiguousarray(rec[k]).tobytes(), digest_size=20).hexdigest() for k in names}


OUT_NAMES = ("sorted_keys", "perm", "leaves", "counts", "node_keys", "child", "level_offsets")


def stratified_sample(specs, per_stratum=50):
    """Request indices of the serving workload, `per_stratum` from every unit
    interval of log2(size) in [12, 22) (in arrival order), plus the largest."""
    sizes = np.array([s[1] for s in specs], dtype=np.float64)
    lg = np.log2(sizes)
    pick = set()
    for k in range(12, 22):
        pick.update(int(i) for i in np.flatnonzero((lg >= k) & (lg < k + 1))[:per_stratum])
    pick.add(int(np.argmax(sizes)))
    return sorted(pick)


def test_serving_stratified_sample_equals_alone_and_oracle():
    """Requests of the serving workload itself (same payload streams), 50 from
    every octave of size up to 2^22 plus the largest, served together with
    continuous batching: every one equals the oracle in every output (checked
    on host threads as requests complete, then dropped) and the same request
    built alone, as a plain build and (every 5th) as a batch of one."""
    import threading

    from tests import oracle_pool as pool

    specs = wl.serving_specs()
    pick = stratified_sample(specs)
    sample = [specs[i] for i in pick]
    assert len(sample) >= 500 and max(s[1] for s in sample) >= 1 << 21
    assert {s[2] for s in sample} == {16, 64} and {s[0] for s in sample} == {"uniform", "plummer"}
    reqs = sv.poisson_requests(sample, rate_per_s=5000.0)
    say("serving", len(reqs), "sampled requests,", sum(r.n for r in reqs), "particles")
    gate = threading.BoundedSemaphore(24)  # records waiting for the oracle (bounds host memory)
    jobs = {}
    ex_pool = cf.ThreadPoolExecutor(max_workers=pool.workers())
    by_rid = {r.rid: r for r in reqs}

    def check(rid, rec):
        try:
            r = by_rid[rid]
            msgs = pool.compare_build(rec, rec["x"], rec["y"], rec["z"], sv.BOXES[r.kind], cs.HILBERT, r.n_crit,
                                      f"request {rid} (n={r.n}, {r.kind}, n_crit={r.n_crit})")
            return msgs, _digest(rec, OUT_NAMES + tuple("xyz"))
        finally:
            gate.release()

    def sink(rid, rec):
        gate.acquire()
        jobs[rid] = ex_pool.submit(check, rid, rec)

    try:
        ex = sv.GpuExecutor(max_inflight=3, keep={r.rid for r in reqs}, sink=sink)
        done, st = sv.ServingLoop(ex).run(reqs)
        torch.cuda.synchronize()
        say("batches", st.batches, "mean", st.mean_batch_requests, "max in flight", st.max_inflight)
        assert len(done) == len(reqs) and all(r.status == "OK" for r in done), st.statuses
        assert st.batches < len(reqs) and st.max_inflight > 1
        results = {rid: f.result() for rid, f in jobs.items()}
    finally:
        ex_pool.shutdown(wait=True)
    assert sorted(results) == sorted(by_rid)
    msgs = [m for ms, _ in results.values() for m in ms]
    assert not msgs, "\n".join(msgs[:20])
    say("all", len(results), "requests equal the oracle; now alone")
    cap = max(sv.leaf_bound(r.n, r.n_crit) for r in reqs)
    builder = cs.Builder(max(r.n for r in reqs), 16, leaf_capacity=min(cap, 8 * (1 << 22) // 17 + 64))
    for j, r in enumerate(done):
        x, y, z, _ = wl.device_sets([(r.kind, r.n, r.seed, r.stream)])
        x, y, z = x[:r.n], y[:r.n], z[:r.n]
        mix = results[r.rid][1]
        alone = builder.build(x, y, z, sv.BOXES[r.kind], cs.HILBERT, r.n_crit)
        rec = {k: cs.to_numpy(getattr(alone, k)) for k in OUT_NAMES}
        rec.update({a: host(t) for a, t in zip("xyz", (x, y, z))})
        got = _digest(rec, OUT_NAMES + tuple("xyz"))
        assert got == mix, f"request {r.rid} (n={r.n}): plain build alone differs from the mix"
        if j % 5 == 0:
            b = cs.Batch([(r.n, sv.BOXES[r.kind], cs.HILBERT, r.n_crit)])
            b.build(x, y, z)
            v = b.set_view(0)
            got = _digest({k: host(v[k]) for k in OUT_NAMES}, OUT_NAMES)
            assert got == {k: mix[k] for k in OUT_NAMES}, f"request {r.rid}: batch of one differs from the mix"
            del b


def test_serving_admission_limited_by_the_hbm_budget():
    """A budget that holds two of these requests at a time: all arrive at
    once, yet the reserved bytes and the slots' resident buffers never exceed
    the budget, fewer requests than the slots allow run together, and every
    result equals the oracle on a sample."""
    n = 1 << 20
    specs = [("plummer" if i % 2 else "uniform", n, 16 if i % 3 else 64, 900 + i, 1.0) for i in range(8)]
    reqs = sv.poisson_requests(specs, rate_per_s=1e12)
    per = max(sv.request_bytes(r.n, sv.leaf_reservation(r.n, r.n_crit)) for r in reqs)
    budget = int(2.2 * per)
    say("serving with budget", budget, "bytes,", per, "per request")
    keep = {0, 5}
    ex = sv.GpuExecutor(max_inflight=3, keep=keep, budget_bytes=budget)
    loop = sv.ServingLoop(ex, budget_bytes=budget, max_inflight=3)
    done, st = loop.run(reqs)
    torch.cuda.synchronize()
    assert all(r.status == "OK" for r in done) and len(done) == len(reqs)
    assert st.peak_reserved_bytes <= budget
    assert ex.peak_buffer_bytes <= budget
    # two requests fit at a time: at least four groups, never three requests in flight
    assert st.batches >= 4 and st.mean_batch_requests <= 2.0
    for rid in keep:
        r = reqs[rid]
        rec = ex.kept[rid]
        ref = oracle.build_tree(rec["x"], rec["y"], rec["z"], r.box, cs.HILBERT, r.n_crit)
        for k, kk in (("sorted_keys", "P"), ("perm", "perm"), ("leaves", "K"), ("counts", "counts"),
                      ("node_keys", "NK"), ("child", "CO"), ("level_offsets", "LO")):
            eq(rec[k], ref[kk], f"request {rid} {k}")


def test_serving_slots_reuse_their_buffers():
    """After the first groups the slots' buffers are large enough: later
    launches allocate nothing (no slot grows), and results stay exact."""
    specs = wl.serving_specs(count=120, seed=9, log2_min=12.0, log2_max=18.0)
    reqs = sv.poisson_requests(specs, rate_per_s=2000.0)
    ex = sv.GpuExecutor(max_inflight=3, keep={7, 100})
    loop = sv.ServingLoop(ex, budget_bytes=64 * 10**9, max_inflight=3)
    done, st = loop.run(reqs)
    torch.cuda.synchronize()
    say("groups", st.batches, "slot growths", ex.grows)
    assert all(r.status == "OK" for r in done)
    assert ex.grows < st.batches / 2  # most launches reuse their slot's buffers
    for rid in (7, 100):
        r = reqs[rid]
        rec = ex.kept[rid]
        ref = oracle.build_tree(rec["x"], rec["y"], rec["z"], r.box, cs.HILBERT, r.n_crit)
        eq(rec["leaves"], ref["K"], f"request {rid} leaves")
        eq(rec["perm"], ref["perm"], f"request {rid} perm")


def test_three_large_groups_at_once_equal_each_alone():
    """Three groups of 40 requests (about 2.4e7 particles each) in flight on
    three streams at once, so that their look-back passes share the GPU and
    its XCDs: every request's arrays equal those of its group built alone, and
    no set reports a device-side wait that gave up."""
    reqs = sv.poisson_requests(wl.serving_specs(120), rate_per_s=1e12)
    groups = [reqs[k * 40:(k + 1) * 40] for k in range(3)]
    keep = {r.rid for r in reqs}
    together = sv.GpuExecutor(max_inflight=3, keep=keep)
    say("three groups at once", [sum(r.n for r in g) for g in groups])
    handles = [together.launch(g) for g in groups]
    status_together = {}
    for h in handles:
        while not together.poll(h):
            pass
        for r, (st, nl, rounds) in zip(h["group"], together.finish(h)):
            status_together[r.rid] = (st, nl, rounds)
    alone = sv.GpuExecutor(max_inflight=1, keep=keep)
    status_alone = {}
    for g in groups:
        say("group alone", len(g))
        h = alone.launch(g)
        torch.cuda.synchronize()
        for r, res in zip(g, alone.finish(h)):
            status_alone[r.rid] = res
    assert status_together == status_alone
    assert all(st != "DEVICE" for st, _, _ in status_together.values())
    for rid in sorted(together.kept):
        a, b = together.kept[rid], alone.kept[rid]
        assert a.keys() == b.keys()
        for k in a:
            eq(a[k], b[k], f"request {rid} {k}")
