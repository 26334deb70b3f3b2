"""Benchmark: the whole Cornerstone octree build (keys -> sort -> rebalance loop
-> link) on one MI355X, on 2^24 uniform particles with Hilbert keys and
N_crit = 64, inputs resident in HBM.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Prints one JSON line: particles/s over K timed builds, the HBM roofline of the
dominant kernel (a radix-sort digit pass) from HIP events recorded around every
pass during the timed builds, the byte-model fraction of the whole build, the
batched-vs-plain ratio on 512 independent sets, the 2^27 Plummer build with
its incremental rebuilds, the latency of a continuous-batching serving run,
and the CPU oracle timed on a bounded sample of the
same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s


_T0 = time.perf_counter()


def progress(*a):
    """A progress line on stderr (the JSON result goes to stdout)."""
    print(f"[bench {time.perf_counter() - _T0:7.1f} s]", *a, file=sys.stderr, flush=True)
# Compulsory bytes per particle of a build: coordinates read once (24), keys
# written and read once (16), P and perm written once (12), and the leaf /
# node arrays (about 10 per particle at N_crit 64).
FLOOR_BYTES_PER_PARTICLE = 62


def byte_model(n: int, leaves_per_round: list, n_leaves: int) -> dict:
    """Algorithmic bytes of one build (fixed model, independent of the code):
    keys 32 N; sort 196 N (8 passes of 8-bit digits: 8 N histogram read, 20 N
    first pass with implicit values, 24 N per later pass); per rebalance round
    with n_l(t) leaves: 12 n_l + min(8 N, 64 (n_l + 1)) for f, 16 n_l for g1,
    8 n_l for g2, 16 n_l + 8 n_l(t+1) for g3; link with n = n_l + n_i nodes:
    8 n_l + 8 n + 136 n + 8 n + 4 n + 64 n_i."""
    keys = 32 * n
    sort = 196 * n
    reb = 0
    for t, nl in enumerate(leaves_per_round[:-1]):
        nxt = leaves_per_round[t + 1]
        reb += 12 * nl + min(8 * n, 64 * (nl + 1)) + 16 * nl + 8 * nl + 16 * nl + 8 * nxt
    ni = (n_leaves - 1) // 7
    nn = n_leaves + ni
    link = 8 * n_leaves + 8 * nn + 136 * nn + 8 * nn + 4 * nn + 64 * ni
    return dict(keys=keys, sort=sort, rebalance=reb, link=link, total=keys + sort + reb + link)


def path_bytes(model: dict, n: int) -> dict:
    """Algorithmic bytes of the path as built here: the fixed model's keys,
    rebalance and link, and the split sort of particle keys: 20 N for the
    first top pass (its histogram comes with the keys, its values are the
    indices), 24 N for each of the two later top passes, 8 N for the bucket
    pass (every key read once; keys that move are data-dependent and not
    counted), and nothing for the low passes when no bucket is listed."""
    sort = 20 * n + 2 * 24 * n + 8 * n
    out = dict(model)
    out["sort"] = sort
    out["total"] = model["keys"] + sort + model["rebalance"] + model["link"]
    return out


def leaves_per_round(leaves, level_offsets) -> list:
    """Leaves entering every round of a build from the root, from the final
    tree: from the root the loop only splits (a split parent's children sum to
    more than N_crit, so nothing merges), so after t rounds the leaves are the
    final tree cut at level t: its leaves on levels <= t plus its internal
    nodes on level t. Ends with the final count twice (the check round)."""
    import paper_2307_06345_amd as cs

    K = cs.to_numpy(leaves).astype(np.uint64)
    LO = cs.to_numpy(level_offsets).astype(np.int64)
    delta = K[1:] - K[:-1]
    lev = 21 - (np.floor(np.log2(delta.astype(np.float64)) + 0.5).astype(np.int64) // 3)
    hist = np.bincount(lev, minlength=22)
    nodes = LO[1:23] - LO[0:22]  # nodes per level
    depth = int(lev.max())
    out = [1]
    for t in range(1, depth + 1):
        out.append(int(hist[:t + 1].sum() + (nodes[t] - hist[t]) if t < depth else hist.sum()))
    out.append(int(hist.sum()))
    return out


def lsd_sort_bytes(n: int, passes: int) -> int:
    """A plain LSD sort with the permutation: 20 N for the first pass (values
    implicit), 24 N for every other."""
    return 20 * n + 24 * n * (passes - 1)


def kernel_source_digest() -> str:
    h = hashlib.sha256()
    for name in ("sort.hip", "common.hpp"):
        with open(os.path.join(ROOT, "paper_2307_06345_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(digest: str):
    """HBM bytes per launch of the digit pass from the committed rocprofv3 PMC
    summary, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "onesweep_pass_uniform_2_24_traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_digest") != digest:
        return None
    return rec.get("hbm_bytes_per_launch")


def cpu_baseline(sample_n: int) -> dict:
    import oracle
    import workloads as wl

    s = wl.config_uniform_2_24(n=sample_n)
    t0 = time.perf_counter()
    ref = oracle.build_tree(s.x, s.y, s.z, s.box, s.curve, s.n_crit)
    dt = time.perf_counter() - t0
    return {"value": sample_n / dt, "unit": "particles/s", "cores": 1, "kind": "oracle",
            "sample": f"single-threaded oracle, whole build (keys, sort, leaves, counts, links) of {sample_n} "
                      f"uniform particles, Hilbert, N_crit 64 ({ref['K'].size - 1} leaves) in {dt:.2f} s"}


def cpu_baseline_small() -> dict:
    """The oracle on the whole 65,536-particle Morton configuration."""
    import oracle
    import workloads as wl

    s = wl.config_small()
    t0 = time.perf_counter()
    oracle.build_tree(s.x, s.y, s.z, s.box, s.curve, s.n_crit)
    dt = time.perf_counter() - t0
    return {"value": s.n / dt, "unit": "particles/s", "cores": 1, "kind": "oracle", "ms": dt * 1e3,
            "sample": f"the whole configuration: {s.n} uniform particles, Morton, N_crit 64"}


def cpu_baseline_plummer(sample_n: int) -> dict:
    """The oracle on a bounded sample of the 2^27 Plummer configuration: the
    first sample_n particles of the same seeded stream (the oracle builds
    every tree from scratch, so a rebuild costs it a whole build)."""
    import oracle
    import workloads as wl

    s = wl.make_set("plummer", sample_n, 3, 0, wl.HILBERT, 16)
    t0 = time.perf_counter()
    ref = oracle.build_tree(s.x, s.y, s.z, s.box, s.curve, s.n_crit)
    dt = time.perf_counter() - t0
    return {"value": sample_n / dt, "unit": "particles/s", "cores": 1, "kind": "oracle",
            "sample": f"single-threaded oracle, whole build of {sample_n} Plummer particles (a = 1, r_t = 20), "
                      f"Hilbert, N_crit 16 ({ref['K'].size - 1} leaves) in {dt:.2f} s"}


def copy_bandwidth(nbytes: int, reps: int = 10) -> dict:
    """Device-to-device copy of nbytes (read + write), for context beside the
    8 TB/s peak: GB/s of (2 nbytes) per copy, median over reps."""
    import torch

    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda").fill_(1)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ts = []
    for _ in range(reps):
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    ms = float(np.median(ts))
    del src, dst
    return {"bytes_moved": 2 * nbytes, "ms": ms, "gbs": 2 * nbytes / (ms * 1e-3) / 1e9}


def event_ms(fn, reps: int):
    """Median and minimum ms of fn() between two events on the current stream."""
    import torch

    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        e0.record()
        fn()
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    return float(np.median(ts)), float(np.min(ts))


def bench_small(steps: int) -> dict:
    """Latency of the 65,536-particle Morton build (N_crit 64, from the root):
    wall time of each synchronous build, median and minimum."""
    import torch

    import paper_2307_06345_amd as cs
    import workloads as wl

    s = wl.config_small()
    x, y, z = (cs.from_numpy(a, "cuda") for a in (s.x, s.y, s.z))
    b = cs.Builder(s.n, s.n_crit)
    for _ in range(5):
        b.build(x, y, z, s.box, s.curve, s.n_crit)
    torch.cuda.synchronize()
    ts = []
    for _ in range(steps):
        t0 = time.perf_counter()
        r = b.build(x, y, z, s.box, s.curve, s.n_crit)
        ts.append((time.perf_counter() - t0) * 1e3)
    return {"workload": "plain build, 65,536 uniform particles, Morton, N_crit 64, from the root",
            "latency_ms_median": float(np.median(ts)), "latency_ms_min": float(np.min(ts)),
            "leaves": r.n_leaves, "rounds": r.rounds}


def bench_beyond(b, x, y, z, s, r, reps: int) -> dict:
    """The steps around the build and its alternatives, on the 2^24 tree just
    built (each timed with events, median of reps):
      node counts of the linked octree: 8 n (NK) + 4 n (out) + 4 n_l (leaf
        counts) + 8 n_l (S written and read) algorithmic bytes;
      gather of x, y, z by perm: 4 N + 24 N + 24 N = 52 N (one array per pass,
        or one fused pass);
      the link through the binary radix tree against the default link;
      the compact octree (empty buckets removed);
      the sharded build with 8 shards (keys, 8 shard sorts, rounds with summed
        counts and a host synchronisation each) against the plain build;
      the tree focused on 1/64 of the curve, theta 0.5, from the root."""
    import torch

    import paper_2307_06345_amd as cs

    n, nl = s.n, r.n_leaves
    nn = cs.node_count(nl)
    out = {}
    leaves, counts, nk = r.leaves.clone(), r.counts.clone(), r.node_keys.clone()
    P, perm = r.sorted_keys.clone(), r.perm.clone()
    cnt = torch.empty(nn, dtype=torch.int32, device="cuda")
    ws = cs._workspace(cs._lib.cstone_octree_node_counts_workspace_bytes(nl), "cuda")
    med, mn = event_ms(lambda: cs.octree_node_counts(leaves, counts, nk, out=cnt, ws=ws), reps)
    byt = 8 * nn + 4 * nn + 4 * nl + 8 * nl
    out["node_counts"] = {"ms": med, "ms_min": mn, "nodes": nn, "bytes": byt, "gbs": byt / (med * 1e-3) / 1e9}
    gx = tuple(torch.empty(n, dtype=torch.float64, device="cuda") for _ in range(3))
    byt = 52 * n
    med, mn = event_ms(lambda: cs.gather_xyz(x, y, z, perm, out=gx), reps)
    medf, mnf = event_ms(lambda: cs.gather_xyz(x, y, z, perm, out=gx, fused=True), reps)
    out["gather_xyz"] = {"ms_per_array_passes": med, "ms_fused": medf, "bytes": byt,
                         "gbs_per_array_passes": byt / (med * 1e-3) / 1e9, "gbs_fused": byt / (medf * 1e-3) / 1e9}
    NK = torch.empty(nn, dtype=torch.int64, device="cuda")
    CO = torch.empty(nn, dtype=torch.int32, device="cuda")
    LO = torch.empty(cs.LEVEL_OFFSETS, dtype=torch.int32, device="cuda")
    wl_ = cs._workspace(cs._lib.cstone_link_workspace_bytes(nl), "cuda")
    wr = cs._workspace(cs._lib.cstone_link_octree_radix_workspace_bytes(nl), "cuda")
    d_med, _ = event_ms(lambda: cs.link_octree(leaves, NK, CO, LO, ws=wl_), reps)
    s_med, _ = event_ms(lambda: cs.link_octree(leaves, NK, CO, LO, ws=wl_, by_sort=True), reps)
    r_med, _ = event_ms(lambda: cs.link_octree_radix(leaves, NK, CO, LO, ws=wr), reps)
    same = bool(torch.equal(NK, nk))
    t0 = time.perf_counter()
    for _ in range(reps):
        ck, cp, _ = cs.compact_octree(leaves, counts)
    c_ms = (time.perf_counter() - t0) * 1e3 / reps
    out["link"] = {"breadth_first_ms": d_med, "five_steps_by_sort_ms": s_med, "radix_tree_ms": r_med,
                   "radix_equals_default": same, "compact_octree_ms_wall": c_ms,
                   "compact_nodes": int(ck.numel()), "linked_nodes": nn}
    G = 8
    off = np.linspace(0, n, G + 1).astype(np.uint64)
    cs.build_sharded(x, y, z, off, s.box, s.curve, s.n_crit)
    torch.cuda.synchronize()
    ts = []
    for _ in range(max(1, reps // 2)):
        t0 = time.perf_counter()
        _, _, Kg, Ng, rg = cs.build_sharded(x, y, z, off, s.box, s.curve, s.n_crit)
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - t0) * 1e3)
    out["sharded_8"] = {"ms_wall": float(np.median(ts)), "rounds": rg, "equals_plain": bool(torch.equal(Kg, leaves)),
                        "particles_per_s": n / (float(np.median(ts)) * 1e-3)}
    Ph = P[int(n * 0.5)].item() & ((1 << 64) - 1)
    fa = (Ph >> 45) << 45
    fb = min(fa + (1 << 57), 1 << 63)
    cs.focus_rebalance(P, s.n_crit, s.curve, fa, fb, 0.5)
    torch.cuda.synchronize()
    ts = []
    for _ in range(max(1, reps // 2)):
        t0 = time.perf_counter()
        Kf, _, rf = cs.focus_rebalance(P, s.n_crit, s.curve, fa, fb, 0.5)
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - t0) * 1e3)
    out["focus"] = {"ms_wall": float(np.median(ts)), "rounds": rf, "leaves": int(Kf.numel() - 1),
                    "range": [fa, fb], "theta": 0.5}
    return out


def bench_batched(steps: int) -> dict:
    """512 independent sets (sizes log-uniform in [2^10, 2^20], uniform or
    Plummer, Morton or Hilbert, N_crit in {8..128}): one captured hipGraph
    launch per step, against plain per-set cstone_build calls (each
    synchronous, as a caller without batching would issue them). The sort shape
    is autotuned and the graph captured before timing; both are excluded."""
    import torch

    import paper_2307_06345_amd as cs
    import workloads as wl

    sets = wl.batched_sets()
    total = sum(p.n for p in sets)
    x, y, z = (cs.from_numpy(np.concatenate([getattr(p, a) for p in sets]), "cuda") for a in "xyz")
    b = cs.Batch([(p.n, p.box, p.curve, p.n_crit) for p in sets])
    t0 = time.perf_counter()
    tune_ms = b.autotune(x, y, z, reps=1)
    side = torch.cuda.Stream()
    b.capture(x, y, z, side)
    setup_s = time.perf_counter() - t0
    for _ in range(2):
        b.launch(side)
    side.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    times = []
    for _ in range(steps):
        e0.record(side)
        b.launch(side)
        e1.record(side)
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    res = b.set_results()
    ok = bool(all(int(r) == 0 for r in res[:, 3]))
    t_batched = float(np.median(times))

    # plain: every set alone through cstone_build, one after another
    big = max(p.n for p in sets)
    builder = cs.Builder(big, n_crit_min=min(p.n_crit for p in sets))
    po = b.particle_offsets
    views = [(x[po[i]:po[i + 1]], y[po[i]:po[i + 1]], z[po[i]:po[i + 1]]) for i in range(len(sets))]

    def plain_pass():
        for (vx, vy, vz), p in zip(views, sets):
            builder.build(vx, vy, vz, p.box, p.curve, p.n_crit)
        torch.cuda.synchronize()

    plain_pass()  # warm-up
    plain = []
    for _ in range(max(1, min(steps, 3))):
        t1 = time.perf_counter()
        plain_pass()
        plain.append((time.perf_counter() - t1) * 1e3)
    t_plain = float(np.median(plain))
    return {"workload": "512 independent sets, sizes floor(2^U), U ~ U[10, 20], uniform/Plummer, Morton/Hilbert, "
                        "N_crit in {8,16,32,64,128}, seed 4",
            "sets": len(sets), "particles": total, "all_sets_ok": ok,
            "batched_ms": t_batched, "batched_ms_all": times,
            "batched_particles_per_s": total / (t_batched * 1e-3),
            "plain_ms": t_plain, "plain_particles_per_s": total / (t_plain * 1e-3),
            "ratio": t_plain / t_batched,
            "sort_variant": b.sort_variant, "sort_shapes": cs.sort_variants(), "autotune_ms": tune_ms,
            "setup_s_excluded": setup_s, "max_rounds": int(res[:, 2].max())}


def bench_serving(count: int, rhos=(0.5, 0.7, 0.9)) -> dict:
    """Continuous batching of `count` build requests (sizes floor(2^U), U ~
    U[12, 22], uniform/Plummer, Hilbert, N_crit in {16, 64}) arriving as a
    Poisson stream, HBM budget 64 GB, coordinates drawn on the device as each
    group is launched. Each launch slot keeps its device buffers between
    groups (they grow only when a group needs more). Capacity is measured
    first with every request of a 2000-request prefix available at once; the
    arrival rate is then rho * capacity / E[N] for each rho."""
    import torch

    from paper_2307_06345_amd import serving as sv
    import workloads as wl

    specs = wl.serving_specs(count)
    mean_n = float(np.mean([s[1] for s in specs]))

    ex = sv.GpuExecutor(max_inflight=3, budget_bytes=64 * 10**9)  # slots keep their buffers across runs

    def run(reqs):
        loop = sv.ServingLoop(ex, budget_bytes=64 * 10**9, max_inflight=3)
        done, st = loop.run(reqs)
        torch.cuda.synchronize()
        return done, st

    # warm-up: the capacity workload itself, so that every slot has grown its
    # buffers to the largest group before anything is timed
    run(sv.poisson_requests(specs[:min(count, 2000)], rate_per_s=1e12))
    progress("serving warm-up done")
    _, cal = run(sv.poisson_requests(specs[:min(count, 2000)], rate_per_s=1e12))
    progress("serving capacity run done")
    capacity = cal.particles_per_s
    runs = {}
    for rho in rhos:
        rate = rho * capacity / mean_n
        done, st = run(sv.poisson_requests(specs, rate_per_s=rate))
        progress(f"serving run at rho {rho} done")
        runs[str(rho)] = {"arrival_rate_per_s": rate, "particles_per_s": st.particles_per_s,
                          "latency_p50_ms": st.latency_p50_ms, "latency_p99_ms": st.latency_p99_ms,
                          "latency_mean_ms": st.latency_mean_ms, "makespan_s": st.makespan_s,
                          "batches": st.batches, "mean_batch_requests": st.mean_batch_requests,
                          "max_inflight": st.max_inflight, "peak_reserved_gb": st.peak_reserved_bytes / 1e9,
                          "retries": st.retries, "statuses": st.statuses}
    out_buffers = {"slot_buffer_peak_gb": ex.peak_buffer_bytes / 1e9, "slot_buffer_growths": ex.grows}
    main_run = runs[str(0.7)] if str(0.7) in runs else next(iter(runs.values()))
    return {"workload": f"{count} requests, sizes floor(2^U), U ~ U[12, 22], uniform/Plummer, Hilbert, "
                        "N_crit in {16, 64}, Poisson arrivals, HBM budget 64 GB, seed 5",
            "requests": count, "particles": int(sum(s[1] for s in specs)), "mean_n": mean_n,
            "capacity_particles_per_s": capacity, "capacity_batches": cal.batches,
            "rho": 0.7, "latency_p50_ms": main_run["latency_p50_ms"],
            "latency_p99_ms": main_run["latency_p99_ms"], "particles_per_s": main_run["particles_per_s"],
            "runs": runs, "resident_buffers": out_buffers}


def bench_plummer(reps: int = 3, rebuilds: int = 10) -> dict:
    """2^27 Plummer particles (a = 1, r_t = 20), Hilbert, N_crit 16: build from
    the root (median of `reps`), then `rebuilds` incremental rebuilds from the
    previous leaves after cumulative N(0, 1e-3^2) displacements (each timed;
    the displacement itself is outside the timed region)."""
    import torch

    import paper_2307_06345_amd as cs
    import workloads as wl

    n, n_crit = 1 << 27, 16
    x, y, z, _ = wl.device_sets([("plummer", n, 3, 0)])
    # the sort shape for this size class, tuned on these keys (excluded from the timing)
    keys = cs.compute_keys(x, y, z, wl.PLUMMER_BOX, wl.HILBERT)
    chosen, tune_ms = cs.sort_autotune(keys, reps=2)
    del keys
    b = cs.Builder(n, n_crit, leaf_capacity=8 * n // (n_crit + 1) + 64)
    b.build(x, y, z, wl.PLUMMER_BOX, wl.HILBERT, n_crit)  # warm-up
    torch.cuda.synchronize()
    root_ms = []
    for _ in range(reps):
        t0 = time.perf_counter()
        r = b.build(x, y, z, wl.PLUMMER_BOX, wl.HILBERT, n_crit)
        torch.cuda.synchronize()
        root_ms.append((time.perf_counter() - t0) * 1e3)
    leaves, rounds = r.leaves.numel() - 1, r.rounds
    reb_ms, reb_rounds = [], []
    for k in range(1, rebuilds + 1):
        wl.device_displace(x, y, z, 1e-3, 3, k)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = b.build(x, y, z, wl.PLUMMER_BOX, wl.HILBERT, n_crit, incremental=True)
        torch.cuda.synchronize()
        reb_ms.append((time.perf_counter() - t0) * 1e3)
        reb_rounds.append(r.rounds)
    t_root = float(np.median(root_ms))
    r0 = b.build(x, y, z, wl.PLUMMER_BOX, wl.HILBERT, n_crit)  # from the root again, for its tree
    hist = leaves_per_round(r0.leaves, r0.level_offsets)
    model = byte_model(n, hist, r0.n_leaves)
    bits, _, _ = cs.sort_variants()[chosen]
    split = bool(cs.sort_variant_splits()[chosen])
    path = dict(model)
    # the split sort's low passes over listed buckets are data-dependent: its path bytes count the top passes
    # and the bucket pass only (a lower bound); an LSD shape's are exact
    path["sort"] = (20 * n + 2 * 24 * n + 8 * n) if split else lsd_sort_bytes(n, (63 + bits - 1) // bits)
    path["total"] = model["keys"] + path["sort"] + model["rebalance"] + model["link"]
    peak = HBM_PEAK_GBS * 1e9
    return {"workload": "2^27 Plummer particles (a = 1, r_t = 20, box [-20, 20]^3), Hilbert, N_crit 16; "
                        "then 10 incremental rebuilds after cumulative N(0, 1e-3^2) displacements",
            "leaves_per_round": hist, "model_bytes": model, "model_fraction": model["total"] / (t_root * 1e-3) / peak,
            "path_bytes": path, "path_fraction": path["total"] / (t_root * 1e-3) / peak,
            "n": n, "leaves": leaves, "rounds_from_root": rounds,
            "from_root_ms": t_root, "from_root_particles_per_s": n / (t_root * 1e-3),
            "rebuild_ms": reb_ms, "rebuild_rounds": reb_rounds,
            "rebuild_particles_per_s": n / (float(np.mean(reb_ms)) * 1e-3),
            "sort_shape": {"chosen": chosen, "shape": cs.sort_variants()[chosen],
                           "split": cs.sort_variant_splits()[chosen], "sort_ms_per_shape": tune_ms}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=1 << 24)
    ap.add_argument("--cpu-sample", type=int, default=1 << 24)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batch-steps", type=int, default=5)
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-plummer", action="store_true")
    ap.add_argument("--no-beyond", action="store_true")
    ap.add_argument("--no-small", action="store_true")
    ap.add_argument("--calibration-copy", action="store_true",
                    help="also copy 24 N bytes device to device once (the same bytes as a digit pass), "
                         "to scale hardware traffic counters")
    ap.add_argument("--serving-requests", type=int, default=10000)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs the single-GPU octree build only; --gpus {args.gpus} is not supported "
              f"(one tree per GPU; see the design notes on sharding)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2307_06345_amd as cs
    import workloads as wl

    torch.cuda.set_device(0)
    s = wl.config_uniform_2_24(n=args.n)
    x, y, z = (cs.from_numpy(a, "cuda") for a in (s.x, s.y, s.z))
    b = cs.Builder(s.n, s.n_crit)

    for _ in range(args.warmup):
        b.build(x, y, z, s.box, s.curve, s.n_crit)
    torch.cuda.synchronize()

    # throughput: K whole builds (each synchronises once, as cstone_build does)
    t0 = time.perf_counter()
    build_ms = []
    for _ in range(args.steps):
        t1 = time.perf_counter()
        r = b.build(x, y, z, s.box, s.curve, s.n_crit)  # synchronises once (the leaf count)
        build_ms.append((time.perf_counter() - t1) * 1e3)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0

    # breakdown: K more builds with HIP events on the build stream around every
    # stage and every sort pass (events add gaps between kernels, so these
    # builds are kept out of the throughput figure)
    stage = [0.0] * 4
    passes = None
    for _ in range(args.steps):
        r = b.build(x, y, z, s.box, s.curve, s.n_crit, timed=True)
        stage = [a + v for a, v in zip(stage, r.stage_ms)]
        passes = list(r.sort_pass_ms) if passes is None else [a + v for a, v in zip(passes, r.sort_pass_ms)]
    torch.cuda.synchronize()

    copy = copy_bandwidth(24 * s.n)

    if args.calibration_copy:
        src = torch.empty(24 * s.n, dtype=torch.uint8, device="cuda").fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    n = s.n
    ms_per_step = dt * 1e3 / args.steps
    value = n * args.steps / dt
    stage = [v / args.steps for v in stage]
    passes = [v / args.steps for v in passes]

    # leaves per round from the root, for the byte model
    nl_final = r.leaves.numel() - 1
    leaves_hist = leaves_per_round(r.leaves, r.level_offsets)
    model = byte_model(n, leaves_hist, nl_final)

    # dominant kernel: a later top digit pass (keys + permutation in and out).
    # Sort intervals: the first top pass, the two later top passes (one
    # interval: no event between their launches), the bucket pass, the low passes
    split = len(passes) == 4
    if split:
        pass_ms = passes[1] / 2
    else:
        mid = passes[1:] if len(passes) > 1 else passes
        pass_ms = sum(mid) / len(mid)
    path = path_bytes(model, n)
    pass_bytes = 24 * n
    achieved = pass_bytes / (pass_ms * 1e-3) / 1e9
    digest = kernel_source_digest()
    traffic = measured_traffic(digest)

    out = {
        "metric": "octree-build particles/s at 2^24",
        "value": value,
        "unit": "particles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "plain build, one tree: 2^24 uniform particles in [0,1)^3 (float64), 3D Hilbert "
                               "keys (21 bits/dim), N_crit 64, keys -> sort -> counts -> rebalance -> links",
                   "n": n, "n_crit": s.n_crit, "curve": "hilbert", "leaves": nl_final,
                   "rounds": r.rounds, "leaves_per_round": leaves_hist},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "onesweep_kernel<false,true> (top digit passes 2 and 3 of the split particle sort)",
                     "bytes_per_launch": pass_bytes, "avg_launch_ms": pass_ms,
                     "kernel_source_digest": digest},
        "build": {"stage_ms": {"keys": stage[0], "sort": stage[1], "rebalance": stage[2], "link": stage[3]},
                  "sort_pass_ms": passes,
                  "sort_pass_names": (["top pass 1 (bits 36-44)", "top passes 2 and 3 (bits 45-62)", "buckets",
                                       "low passes"] if split else [f"digit {i}" for i in range(len(passes))]),
                  "model_bytes": model,
                  "model_fraction": model["total"] / (ms_per_step * 1e-3) / (HBM_PEAK_GBS * 1e9),
                  "path_bytes": path,
                  "path_fraction": path["total"] / (ms_per_step * 1e-3) / (HBM_PEAK_GBS * 1e9),
                  "floor_bytes": FLOOR_BYTES_PER_PARTICLE * n,
                  "floor_fraction": FLOOR_BYTES_PER_PARTICLE * n / (ms_per_step * 1e-3) / (HBM_PEAK_GBS * 1e9),
                  "build_ms_median": float(np.median(build_ms)), "build_ms_min": float(np.min(build_ms)),
                  "build_ms_all": build_ms},
        "copy_bandwidth": copy,
    }
    progress("2^24 builds done:", f"{ms_per_step:.4f} ms per build")
    if not args.no_small:
        out["small_65536"] = bench_small(args.steps)
        progress("65,536-particle latency done")
    if not args.no_beyond:
        out["beyond_the_build"] = bench_beyond(b, x, y, z, s, r, 10)
        progress("steps beyond the build done")
    if not args.no_batched:
        out["batched"] = bench_batched(args.batch_steps)
        progress("batched builds done")
    if not args.no_plummer:
        out["plummer_2_27"] = bench_plummer()
        progress("2^27 Plummer builds done")
    if not args.no_serving:
        out["serving"] = bench_serving(args.serving_requests)
        progress("serving done")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(min(args.cpu_sample, n))
        out["cpu_baseline"]["host_cpus"] = os.cpu_count()
        out["cpu_baseline"]["small_65536"] = cpu_baseline_small()
        out["cpu_baseline"]["plummer_sample"] = cpu_baseline_plummer(1 << 23)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
