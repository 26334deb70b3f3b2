"""The deep, unbalanced configuration at full size: 2^27 Plummer particles
(scale radius 1, truncated at r_t = 20, box [-20, 20]^3), Hilbert keys,
N_crit 16, built from the root, then 10 incremental rebuilds from the previous
leaves after cumulative N(0, (1e-3)^2) displacements of every coordinate.

Every build's keys come from the oracle for all 2^27 particles (host threads),
and P must equal them taken through perm, with P sorted and ties in ascending
index: that is the oracle's stable sort exactly. The two builds from the root
(first, and after the last rebuild) are compared with the oracle in every
output at full size: P, perm, the top-down leaves and counts (computed node by
node on host threads), NK, CO and LO. The incremental rebuilds' trees are
checked through properties that fix them uniquely (Eq. cstone with counts by
binary search, every leaf within N_crit and no 8 mergeable siblings, which by
the uniqueness of the fixed point is the oracle's top-down tree; the Sec. 5
link structure), and the last one must equal the build from the root."""
import numpy as np
import pytest
import torch

import oracle
import workloads as wl
from tests import device_checks as dc
from tests import oracle_pool as pool

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

cs = pytest.importorskip("paper_2307_06345_amd")

N = 1 << 27
N_CRIT = 16
SIGMA = 1e-3
SEED = 3
REBUILDS = 10


def say(*a):
    print("[case]", *a, flush=True)


def host_coords(x, y, z):
    return tuple(t.cpu().numpy() for t in (x, y, z))


def check_keys_and_sort(r, x, y, z):
    """Every particle's key from the oracle (host threads), uploaded: P must be
    the oracle keys taken through perm, which with P sorted and ties in
    ascending index is exactly the oracle's stable sort."""
    hx, hy, hz = host_coords(x, y, z)
    ref = pool.keys(hx, hy, hz, wl.PLUMMER_BOX, wl.HILBERT)
    keys = cs.from_numpy(ref, "cuda")
    dc.check_sorted_perm(r.sorted_keys, r.perm, N, keys=keys)
    del keys
    return ref


def check_against_oracle(r, ref_keys):
    """Every output of a build from the root against the oracle at full size:
    P and perm (oracle sort of the oracle keys), the top-down leaves and their
    counts (host threads, node by node), and the linked octree."""
    P, perm = oracle.sort(ref_keys)
    msgs = pool.mismatch(cs.to_numpy(r.sorted_keys), P, "P") + pool.mismatch(cs.to_numpy(r.perm), perm, "perm")
    assert not msgs, msgs
    del perm
    K = pool.leaves(P, N_CRIT)
    msgs = pool.mismatch(cs.to_numpy(r.leaves), K, "leaves")
    assert not msgs, msgs
    msgs = pool.mismatch(cs.to_numpy(r.counts), pool.counts(P, K), "counts")
    NK, CO, LO = oracle.link_octree(K)
    msgs += pool.mismatch(cs.to_numpy(r.node_keys), NK, "NK") + pool.mismatch(cs.to_numpy(r.child), CO, "CO")
    msgs += pool.mismatch(cs.to_numpy(r.level_offsets), LO, "LO")
    assert not msgs, msgs


def test_plummer_2_27_and_incremental_rebuilds():
    say("2^27 Plummer particles, generated on the device")
    x, y, z, _ = wl.device_sets([("plummer", N, SEED, 0)])
    cap = 8 * N // (N_CRIT + 1) + 64
    b = cs.Builder(N, N_CRIT, leaf_capacity=cap)
    say("build from the root")
    r = b.build(x, y, z, wl.PLUMMER_BOX, wl.HILBERT, N_CRIT)
    lev, _ = dc.leaf_levels(r.leaves)
    depth = int(lev.max())
    say("leaves", r.leaves.numel() - 1, "depth", depth, "rounds", r.rounds)
    assert r.rounds == depth + 1
    say("oracle keys of all particles, P == keys[perm]")
    ref = check_keys_and_sort(r, x, y, z)
    say("oracle sort, leaves, counts and links at full size")
    check_against_oracle(r, ref)
    del ref
    for k in range(1, REBUILDS + 1):
        wl.device_displace(x, y, z, SIGMA, SEED, k)
        r = b.build(x, y, z, wl.PLUMMER_BOX, wl.HILBERT, N_CRIT, incremental=True)
        say("rebuild", k, "leaves", r.leaves.numel() - 1, "rounds", r.rounds)
        assert 1 <= r.rounds < depth + 1  # a few local splits and merges, fewer rounds than from the root
        check_keys_and_sort(r, x, y, z)
        dc.check_balanced(r.sorted_keys, r.leaves, r.counts, N_CRIT)
        if k == REBUILDS:
            dc.check_linked(r.leaves, r.node_keys, r.child, r.level_offsets)
        torch.cuda.synchronize()
    # the incremental result is the tree a build from the root gives, and that
    # build equals the oracle in every output
    inc = {k: cs.to_numpy(getattr(r, k)).copy() for k in ("leaves", "counts", "node_keys", "child")}
    say("build from the root after the last rebuild")
    root = b.build(x, y, z, wl.PLUMMER_BOX, wl.HILBERT, N_CRIT)
    for k, v in inc.items():
        assert np.array_equal(cs.to_numpy(getattr(root, k)), v), f"incremental {k} differs from the root build"
    ref = check_keys_and_sort(root, x, y, z)
    check_against_oracle(root, ref)
