"""The deep, unbalanced configuration at full size: 2^27 Plummer particles
(scale radius 1, truncated at r_t = 20, box [-20, 20]^3), Hilbert keys,
N_crit 16, built from the root, then 10 incremental rebuilds from the previous
leaves after cumulative N(0, (1e-3)^2) displacements of every coordinate.

At this size the oracle cannot rebuild the whole tree inside a test, so every
output is checked through properties that hold at any size and fix it
uniquely (sorted keys with a stable permutation; Eq. cstone with counts by
binary search, every leaf within N_crit and no 8 mergeable siblings, which by
the uniqueness of the fixed point is exactly the oracle's top-down tree; the
full Sec. 5 link structure), plus the oracle itself on samples: keys of
sampled particles, and the leaves inside sampled subtrees, which depend only on
the particles inside them."""
import numpy as np
import pytest
import torch

import oracle
import workloads as wl
from tests import device_checks as dc

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

cs = pytest.importorskip("paper_2307_06345_amd")

N = 1 << 27
N_CRIT = 16
SIGMA = 1e-3
SEED = 3
REBUILDS = 10


def say(*a):
    print("[case]", *a, flush=True)


def sampled_keys(P, perm, x, y, z, count, rng):
    i = torch.from_numpy(rng.integers(0, N, count)).cuda()
    src = perm.long()[i]
    cx, cy, cz = (t[src].cpu().numpy() for t in (x, y, z))
    keys, bad = oracle.compute_keys(cx, cy, cz, wl.PLUMMER_BOX, wl.HILBERT)
    assert not bad
    assert np.array_equal(cs.to_numpy(P[i]), keys), "sorted keys differ from the oracle's keys of their particles"


def sampled_subtrees(P, K, count, rng, lo=2000, hi=300000):
    """Leaves of the built tree inside a node equal the oracle's top-down
    leaves of the particles inside that node."""
    Kh = cs.to_numpy(K)
    picks = rng.integers(0, Kh.size - 1, 64)
    done = 0
    for j in picks:
        for lev in range(12, 0, -1):
            span = 1 << (3 * (21 - lev))
            start = int(Kh[j]) & ~(span - 1)
            end = start + span
            a = int(torch.searchsorted(P, torch.tensor([start], dtype=torch.int64, device=P.device)))
            b = int(torch.searchsorted(P, torch.tensor([min(end, (1 << 63) - 1)], dtype=torch.int64,
                                                         device=P.device))) if end < (1 << 63) else N
            if lo <= b - a <= hi:
                sub = cs.to_numpy(P[a:b])
                ref = oracle.build_leaves(sub, N_CRIT)
                ref_in = ref[(ref >= start) & (ref < end)]
                got_in = Kh[(Kh >= np.uint64(start)) & (Kh < np.uint64(end))]
                assert np.array_equal(ref_in, got_in), f"subtree at level {lev} start {start:#x}"
                done += 1
                break
        if done >= count:
            break
    assert done >= 1


def check_build(r, x, y, z, rng, links):
    dc.check_sorted_perm(r.sorted_keys, r.perm, N)
    sampled_keys(r.sorted_keys, r.perm, x, y, z, 200000, rng)
    dc.check_balanced(r.sorted_keys, r.leaves, r.counts, N_CRIT)
    sampled_subtrees(r.sorted_keys, r.leaves, 4, rng)
    if links:
        dc.check_linked(r.leaves, r.node_keys, r.child, r.level_offsets)
    torch.cuda.synchronize()


def test_config3_plummer_2_27_and_incremental_rebuilds():
    rng = np.random.default_rng(33)
    say("config 3: generate 2^27 Plummer particles on the device")
    x, y, z, _ = wl.device_sets([("plummer", N, SEED, 0)])
    cap = 8 * N // (N_CRIT + 1) + 64
    b = cs.Builder(N, N_CRIT, leaf_capacity=cap)
    say("build from the root")
    r = b.build(x, y, z, wl.PLUMMER_BOX, wl.HILBERT, N_CRIT)
    lev, _ = dc.leaf_levels(r.leaves)
    depth = int(lev.max())
    say("leaves", r.leaves.numel() - 1, "depth", depth, "rounds", r.rounds)
    assert r.rounds == depth + 1
    check_build(r, x, y, z, rng, links=True)
    for k in range(1, REBUILDS + 1):
        wl.device_displace(x, y, z, SIGMA, SEED, k)
        r = b.build(x, y, z, wl.PLUMMER_BOX, wl.HILBERT, N_CRIT, incremental=True)
        say("rebuild", k, "leaves", r.leaves.numel() - 1, "rounds", r.rounds)
        assert 1 <= r.rounds < depth + 1  # a few local splits and merges, fewer rounds than from the root
        check_build(r, x, y, z, rng, links=(k == REBUILDS))
    # the incremental result is the tree a build from the root gives
    inc = cs.to_numpy(r.leaves).copy()
    root = b.build(x, y, z, wl.PLUMMER_BOX, wl.HILBERT, N_CRIT)
    assert np.array_equal(cs.to_numpy(root.leaves), inc)
