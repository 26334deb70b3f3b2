"""The binary radix tree (after Karras), the linked octree through it, and
the compact octree without empty buckets (Sec. 5), against the oracle."""
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


CASES = [("uniform", 0, 64, wl.MORTON), ("uniform", 100, 64, wl.HILBERT), ("uniform", 65536, 64, wl.MORTON),
         ("plummer", 300001, 16, wl.HILBERT), ("plummer", 20000, 1, wl.HILBERT), ("uniform", 200003, 3, wl.MORTON)]


@pytest.mark.parametrize("kind,n,n_crit,curve", CASES)
def test_radix_tree_and_links(kind, n, n_crit, curve):
    s = wl.make_set(kind, n, 70 + n_crit, 0, curve, n_crit)
    say("radix", kind, n, n_crit)
    r = cs.build(*coords(s), s.box, s.curve, s.n_crit)
    K = cs.to_numpy(r.leaves)
    m = K.size - 1
    first, last, split, plen = (cs.to_numpy(t) for t in cs.radix_tree(r.leaves[:m]))
    pl, fi, la = oracle.radix_nodes(K[:m])
    # node i is the one that splits after key split[i]: the same prefix and range as the oracle's pair
    assert np.array_equal(np.sort(split), np.arange(m - 1, dtype=np.uint32))
    assert np.array_equal(plen, pl[split]) and np.array_equal(first, fi[split]) and np.array_equal(last, la[split])
    if m > 1:
        assert first[0] == 0 and last[0] == m - 1  # node 0 is the root
    NK, CO, LO = cs.link_octree_radix(r.leaves)
    rNK, rCO, rLO = oracle.link_octree(K)
    assert np.array_equal(cs.to_numpy(NK), rNK) and np.array_equal(cs.to_numpy(CO), rCO)
    assert np.array_equal(cs.to_numpy(LO), rLO)
    nk, par, lo = cs.compact_octree(r.leaves, r.counts)
    cNK, cpar = oracle.compact_octree(K, cs.to_numpy(r.counts))
    assert np.array_equal(cs.to_numpy(nk), cNK) and np.array_equal(cs.to_numpy(par), cpar)
    assert cs.to_numpy(lo)[22] == cNK.size


def test_compact_octree_degenerate():
    K = cs.from_numpy(np.array([0, 1 << 63], np.uint64), "cuda")
    for c in (0, 5):
        nk, par, lo = cs.compact_octree(K, cs.from_numpy(np.array([c], np.uint32), "cuda"))
        assert list(cs.to_numpy(nk)) == [1] and list(cs.to_numpy(par)) == [0xFFFFFFFF]
    K8 = np.array([0] + [j << 60 for j in range(1, 8)] + [1 << 63], np.uint64)
    cnt = np.array([0, 0, 3, 0, 0, 0, 0, 0], np.uint32)
    nk, par, lo = cs.compact_octree(cs.from_numpy(K8, "cuda"), cs.from_numpy(cnt, "cuda"))
    assert list(cs.to_numpy(nk)) == [1, 0o12] and list(cs.to_numpy(par)) == [0xFFFFFFFF, 0]


def test_radix_links_2_24():
    s = wl.config_uniform_2_24()
    say("radix 2^24")
    b = cs.Builder(s.n, s.n_crit)
    r = b.build(*coords(s), s.box, s.curve, s.n_crit)
    NK, CO, LO = cs.link_octree_radix(r.leaves)
    assert torch.equal(NK, r.node_keys) and torch.equal(CO, r.child) and torch.equal(LO, r.level_offsets)
    nk, par, lo = cs.compact_octree(r.leaves, r.counts)
    cNK, cpar = oracle.compact_octree(cs.to_numpy(r.leaves), cs.to_numpy(r.counts))
    assert np.array_equal(cs.to_numpy(nk), cNK) and np.array_equal(cs.to_numpy(par), cpar)
