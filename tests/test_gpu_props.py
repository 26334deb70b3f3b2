"""Node counts of the linked octree and the particle gather against the
oracle, element by element (Sec. 5 node properties; Sec. 4 permutation)."""
import numpy as np
import pytest
import torch

import oracle
import workloads as wl

pytestmark = pytest.mark.gpu

cs = pytest.importorskip("paper_2307_06345_amd")


def say(*a):
    print("[case]", *a, flush=True)


def coords(s):
    return tuple(cs.from_numpy(a, "cuda") for a in (s.x, s.y, s.z))


CASES = [("uniform", 0, 64, wl.MORTON), ("uniform", 1, 1, wl.HILBERT), ("uniform", 65536, 64, wl.MORTON),
         ("plummer", 300001, 16, wl.HILBERT), ("plummer", 20000, 1, wl.HILBERT), ("uniform", 200003, 3, wl.MORTON)]


@pytest.mark.parametrize("kind,n,n_crit,curve", CASES)
def test_octree_node_counts_parity(kind, n, n_crit, curve):
    s = wl.make_set(kind, n, 17 + n, 0, curve, n_crit)
    say("node counts", kind, n, n_crit, curve)
    r = cs.build(*coords(s), s.box, s.curve, s.n_crit)
    got = cs.octree_node_counts(r.leaves, r.counts, r.node_keys)
    torch.cuda.synchronize()
    P = cs.to_numpy(r.sorted_keys)
    NK = cs.to_numpy(r.node_keys)
    ref = oracle.octree_node_counts(P, NK)
    assert np.array_equal(cs.to_numpy(got), ref)
    assert int(ref[0]) == n


def test_octree_node_counts_full_size_2_24():
    s = wl.config_uniform_2_24()
    say("node counts 2^24")
    b = cs.Builder(s.n, s.n_crit)
    r = b.build(*coords(s), s.box, s.curve, s.n_crit)
    got = cs.to_numpy(cs.octree_node_counts(r.leaves, r.counts, r.node_keys))
    ref = oracle.octree_node_counts(cs.to_numpy(r.sorted_keys), cs.to_numpy(r.node_keys))
    assert np.array_equal(got, ref)


def test_octree_node_counts_of_another_tree_are_marked():
    s = wl.make_set("uniform", 5000, 3, 0, wl.HILBERT, 8)
    r = cs.build(*coords(s), s.box, s.curve, s.n_crit)
    other = cs.from_numpy(np.array([(1 << 63) | 12345], np.uint64), "cuda")  # a level-21 node no leaf starts
    got = cs.to_numpy(cs.octree_node_counts(r.leaves, r.counts, other))
    assert got[0] == 0xFFFFFFFF


@pytest.mark.parametrize("n,fused", [(0, False), (1, True), (4099, False), (300001, True), (300001, False)])
def test_gather_parity(n, fused):
    s = wl.make_set("plummer", n, 5 + n, 0, wl.HILBERT, 16)
    say("gather", n, fused)
    x, y, z = coords(s)
    r = cs.build(x, y, z, s.box, s.curve, s.n_crit)
    out = cs.gather_xyz(x, y, z, r.perm, fused=fused)
    single = cs.gather(y, r.perm)
    torch.cuda.synchronize()
    perm = cs.to_numpy(r.perm)
    for got, a in zip(out, (s.x, s.y, s.z)):
        assert np.array_equal(cs.to_numpy(got).view(np.uint64), oracle.gather(a, perm).view(np.uint64))
    assert np.array_equal(cs.to_numpy(single).view(np.uint64), oracle.gather(s.y, perm).view(np.uint64))
