"""Pins for the oracle's functions beyond the build itself: node counts of the
linked octree (Sec. 5 node properties), the particle gather by the sort
permutation (Sec. 4), the replicated tree of sharded particles and the SFC
partition (Sec. 6), the minimum-distance MAC and the focused tree (Sec. 7),
and the binary radix tree over the leaf keys (Sec. 5, after Karras).

Each pin checks the oracle against something other than itself: brute force
on small inputs computed another way, closed forms, special cases that reduce
to the already pinned balanced tree, and structural characterisations.
"""
import numpy as np
import pytest

import oracle
from tests import invariants as inv

L = 21
END = 1 << 63


def placeholder_range(key: int):
    """(start, end, level) of a node key in placeholder-bit format."""
    level = (int(key).bit_length() - 1) // 3
    prefix = int(key) - (1 << (3 * level))
    start = prefix << (3 * (L - level))
    return start, start + (1 << (3 * (L - level))), level


def random_P(rng, n, spread_bits=63):
    P = rng.integers(0, 1 << 62, n, dtype=np.int64).astype(np.uint64) * np.uint64(2)
    if spread_bits < 63:
        P >>= np.uint64(63 - spread_bits)
    return np.sort(P)


def clustered_P(rng, n):
    """Keys concentrated in a few regions of the curve (a deep, uneven tree)."""
    centres = rng.integers(0, 1 << 62, 4, dtype=np.int64).astype(np.uint64)
    widths = np.array([1 << 30, 1 << 40, 1 << 50, 1 << 58], np.uint64)
    c = rng.integers(0, 4, n)
    off = rng.integers(0, 1 << 62, n, dtype=np.int64).astype(np.uint64) % widths[c]
    return np.sort((centres[c] + off) % np.uint64(END))


# ---- node counts of the linked octree ------------------------------------------

@pytest.mark.parametrize("seed", range(6))
def test_octree_node_counts_brute_force(seed):
    rng = np.random.default_rng(seed)
    P = np.sort(rng.integers(0, 512, int(rng.integers(0, 60))).astype(np.uint64) << np.uint64(54))
    K = oracle.build_leaves(P, int(rng.integers(1, 6)))
    NK, CO, LO = oracle.link_octree(K)
    got = oracle.octree_node_counts(P, NK)
    for p, key in enumerate(NK):
        a, b, _ = placeholder_range(int(key))
        assert got[p] == sum(1 for q in P if a <= int(q) < b), (p, oct(int(key)))


@pytest.mark.parametrize("seed,n_crit", [(1, 1), (2, 8), (3, 64)])
def test_octree_node_counts_sum_over_children(seed, n_crit):
    rng = np.random.default_rng(seed)
    P = clustered_P(rng, 20000)
    K = oracle.build_leaves(P, n_crit)
    NK, CO, LO = oracle.link_octree(K)
    cnt = oracle.octree_node_counts(P, NK).astype(np.int64)
    assert cnt[0] == P.size  # the root holds every particle
    internal = np.flatnonzero(CO)
    for p in internal:
        assert cnt[p] == cnt[CO[p]:CO[p] + 8].sum(), p
    # the leaves, in SFC order, hold Eq. histogram's counts
    leaves = np.flatnonzero(CO == 0)
    order = np.argsort([placeholder_range(int(k))[0] for k in NK[leaves]], kind="stable")
    assert np.array_equal(cnt[leaves[order]], oracle.node_counts(P, K).astype(np.int64))


def test_octree_node_counts_paper_example(golden_fig):
    """Fig. 1's refined array with one particle per leaf and two more in leaf
    "21": the root holds 17 particles and node "2" (index 3 in Fig. 2) 10."""
    K = np.array([int(p, 8) << (3 * (L - len(p))) for p in golden_fig["fig1_bottom_octal_prefixes"]] + [END],
                 np.uint64)
    P = np.sort(np.concatenate([K[:-1], np.full(2, K[3] + np.uint64(5), np.uint64)]))
    NK, CO, LO = oracle.link_octree(K)
    cnt = oracle.octree_node_counts(P, NK)
    assert cnt[0] == 17 and cnt[3] == 10
    assert list(cnt[9:17]) == [1, 3, 1, 1, 1, 1, 1, 1]


# ---- gather ------------------------------------------------------------------

def test_gather_puts_particles_in_key_order():
    rng = np.random.default_rng(7)
    n = 5000
    x, y, z = (rng.random(n) for _ in range(3))
    box = ((0.0, 0.0, 0.0), (1.0, 1.0, 1.0))
    keys, _ = oracle.compute_keys(x, y, z, box, oracle.HILBERT)
    P, perm = oracle.sort(keys)
    gx, gy, gz = (oracle.gather(a, perm) for a in (x, y, z))
    # the gathered particles have the sorted keys, and the same multiset of coordinates
    k2, _ = oracle.compute_keys(gx, gy, gz, box, oracle.HILBERT)
    assert np.array_equal(k2, P)
    assert np.array_equal(np.sort(gx), np.sort(x))
    assert [gx[i] for i in range(5)] == [x[int(perm[i])] for i in range(5)]


# ---- replicated tree of sharded particles (Sec. 6) ----------------------------

@pytest.mark.parametrize("G,n_crit,seed", [(1, 16, 1), (2, 16, 2), (4, 8, 3), (8, 64, 4), (3, 1, 5)])
def test_global_tree_equals_the_tree_of_all_particles(G, n_crit, seed):
    rng = np.random.default_rng(seed)
    keys = clustered_P(rng, 30000)
    rng.shuffle(keys)
    cuts = np.sort(rng.integers(0, keys.size + 1, G - 1))
    parts = [np.sort(p) for p in np.split(keys, cuts)]
    K, N, rounds, conv = oracle.global_rebalance(parts, n_crit)
    P = np.sort(keys)
    assert conv
    assert np.array_equal(K, oracle.build_leaves(P, n_crit))
    assert np.array_equal(N, oracle.node_counts(P, K))
    if G == 1:
        K1, N1, r1, _, _ = oracle.rebalance_iterate(P, np.array([0, END], np.uint64), n_crit)
        assert np.array_equal(K1, K) and r1 == rounds


# ---- SFC partition (Sec. 6) ----------------------------------------------------

@pytest.mark.parametrize("seed", range(8))
def test_partition_brute_force(seed):
    rng = np.random.default_rng(seed)
    nl = int(rng.integers(1, 300))
    counts = rng.integers(0, 50, nl).astype(np.uint32)
    if seed == 0:
        counts[:] = 0  # no particles: every bin starts at leaf 0 but the last
    R = int(rng.integers(1, 40))
    b = oracle.sfc_partition(counts, R)
    N = int(counts.sum())
    C = [0]
    for c in counts:
        C.append(C[-1] + int(c))
    for r in range(R):
        # the first leaf boundary i with C_i >= r N / R, found by scanning the fractions
        want = next(i for i in range(nl + 1) if C[i] * R >= r * N)
        assert b[r] == want, (r, b[r], want)
    assert b[R] == nl
    assert np.all(np.diff(b.astype(np.int64)) >= 0)
    mx = int(counts.max())
    for r in range(R):
        got = C[b[r + 1]] - C[b[r]]
        assert abs(got * R - N) <= mx * R, (r, got, N / R, mx)


def test_partition_equal_counts():
    b = oracle.sfc_partition(np.full(64, 10, np.uint32), 8)
    assert list(b) == list(range(0, 65, 8))
    b = oracle.sfc_partition(np.full(10, 3, np.uint32), 1)
    assert list(b) == [0, 10]


# ---- MAC and node boxes (Sec. 7.1) -------------------------------------------------

def test_node_box_morton_closed_form():
    # Morton digits carry x, y, z bits as 4, 2, 1: octant 5 = x high, z high
    assert oracle.node_box(5 << 60, 1, oracle.MORTON) == ((1 << 20, 0, 1 << 20), 1 << 20)
    assert oracle.node_box(0, 0, oracle.MORTON) == ((0, 0, 0), 1 << 21)
    key = int("3726", 8) << (3 * (L - 4))  # digits 011 111 010 110: x 0101, y 1111, z 1100
    lo, e = oracle.node_box(key, 4, oracle.MORTON)
    assert e == 1 << 17 and lo == (0b0101 << 17, 0b1111 << 17, 0b1100 << 17)


@pytest.mark.parametrize("curve", [oracle.MORTON, oracle.HILBERT])
def test_node_box_contains_its_keys(curve):
    rng = np.random.default_rng(3 + curve)
    for _ in range(200):
        level = int(rng.integers(0, 22))
        start = (int(rng.integers(0, 1 << 62)) * 2) >> (3 * (L - level)) << (3 * (L - level)) if level else 0
        lo, e = oracle.node_box(start, level, curve)
        assert e == 1 << (L - level)
        span = 1 << (3 * (L - level))
        for k in (start, start + span - 1, start + int(rng.integers(0, span))):
            c = oracle.hilbert_decode(k) if curve == oracle.HILBERT else _morton_decode(k)
            assert all(lo[d] <= c[d] < lo[d] + e for d in range(3)), (level, oct(start), oct(k))


def _morton_decode(key):
    x = y = z = 0
    for b in range(L):
        x |= ((key >> (3 * b + 2)) & 1) << b
        y |= ((key >> (3 * b + 1)) & 1) << b
        z |= ((key >> (3 * b)) & 1) << b
    return x, y, z


def _brute_mac_fails(start, level, curve, fa, fb, theta, m):
    """MAC by enumeration: every level-m cell of F (F aligned to level m), the
    squared distance from the node's box to the nearest one."""
    lo, e = oracle.node_box(start, level, curve)
    step = 1 << (3 * (L - m))
    best = None
    for k in range(fa, fb, step):
        clo, ce = oracle.node_box(k, m, curve)
        r2 = 0
        for d in range(3):
            gap = max(0, clo[d] - (lo[d] + e), lo[d] - (clo[d] + ce))
            r2 += gap * gap
        best = r2 if best is None else min(best, r2)
    if best is None:
        return False
    return not (float(best) * (theta * theta) > float(e) * float(e))


@pytest.mark.parametrize("curve", [oracle.MORTON, oracle.HILBERT])
@pytest.mark.parametrize("theta", [0.3, 0.5, 1.0])
def test_mac_matches_enumeration_of_the_focus_cells(curve, theta):
    rng = np.random.default_rng(int(theta * 10) + 7 * curve)
    m = 3
    step = 1 << (3 * (L - m))
    for trial in range(40):
        a = int(rng.integers(0, 512))
        b = int(rng.integers(a, min(512, a + 40) + 1))
        fa, fb = a * step, b * step
        for _ in range(6):
            level = int(rng.integers(1, 8))
            start = int(rng.integers(0, 1 << (3 * level))) << (3 * (L - level))
            want = _brute_mac_fails(start, level, curve, fa, fb, theta, m)
            assert oracle.mac_fails(start, level, curve, fa, fb, theta) == want, (trial, level, oct(start), a, b)


def test_mac_special_cases():
    H = oracle.HILBERT
    fa, fb = 5 << 57, 9 << 57
    # a node overlapping F always fails (r_min = 0), whatever theta
    assert oracle.mac_fails(0, 0, H, fa, fb, 1e9)
    assert oracle.mac_fails(fa, 3, H, fa, fb, 1e9)
    # theta = 0: l / theta is infinite, the MAC never passes
    assert oracle.mac_fails(7 << 60, 1, H, fa, fb, 0.0)
    # an empty F: nothing to fail against
    assert not oracle.mac_fails(0, 0, H, fa, fa, 0.5)
    # far from F with a large theta: passes
    assert not oracle.mac_fails((7 << 60) + (7 << 57), 2, oracle.MORTON, 0, 1 << 57, 5.0)


# ---- focused tree (Sec. 7) ---------------------------------------------------------

def _focus_case(seed, n=20000):
    rng = np.random.default_rng(seed)
    P = clustered_P(rng, n) if seed % 2 else random_P(rng, n)
    i, j = sorted(rng.integers(0, n, 2))
    fa, fb = int(P[i]) >> 48 << 48, (int(P[j]) >> 48 << 48) + (1 << 48)
    return P, fa, min(fb, END)


@pytest.mark.parametrize("curve", [oracle.MORTON, oracle.HILBERT])
def test_focus_reduces_to_the_balanced_tree(curve):
    P, fa, fb = _focus_case(11)
    ref = oracle.build_leaves(P, 16)
    assert np.array_equal(oracle.focus_leaves(P, 16, curve, fa, fb, 0.0), ref)  # theta 0: every MAC fails
    assert np.array_equal(oracle.focus_leaves(P, 16, curve, 0, END, 0.7), ref)  # F is the whole domain
    K = oracle.focus_leaves(P, 16, curve, fa, fb, 0.7)
    assert K.size < ref.size  # far from F, nodes that pass the MAC stay coarse


@pytest.mark.parametrize("seed,curve,theta,n_crit", [(1, 1, 0.5, 16), (2, 0, 0.5, 8), (3, 1, 1.0, 1),
                                                     (4, 1, 0.25, 64)])
def test_focus_tree_meets_its_definition(seed, curve, theta, n_crit):
    """Sec. 7.1: leaves within N_crit or passing the MAC; internal nodes over
    N_crit and failing it; the array is a cornerstone array."""
    P, fa, fb = _focus_case(seed)
    K = oracle.focus_leaves(P, n_crit, curve, fa, fb, theta)
    inv.check_cornerstone(K)
    N = oracle.node_counts(P, K)
    NK, CO, LO = oracle.link_octree(K)
    cnt = oracle.octree_node_counts(P, NK)
    for p in range(NK.size):
        a, b, level = placeholder_range(int(NK[p]))
        m = oracle.mac_fails(a, level, curve, fa, fb, theta)
        if CO[p]:
            assert cnt[p] > n_crit and m, (p, level)
        else:
            assert cnt[p] <= n_crit or not m or level == L, (p, level)
        if a < fb and b > fa:
            assert m  # nodes overlapping F always fail
    assert int(N.sum()) == P.size


@pytest.mark.parametrize("seed,curve,theta,n_crit", [(5, 1, 0.5, 16), (6, 0, 0.8, 4), (7, 1, 0.4, 32)])
def test_focus_literal_iteration_reaches_the_top_down_tree(seed, curve, theta, n_crit):
    P, fa, fb = _focus_case(seed)
    ref = oracle.focus_leaves(P, n_crit, curve, fa, fb, theta)
    K, N, rounds, conv, hist = oracle.focus_iterate(P, n_crit, curve, fa, fb, theta)
    assert conv and np.array_equal(K, ref)
    # from an unrelated start (the plain balanced tree): the same fixed point
    K0 = oracle.build_leaves(P, n_crit)
    K2, _, _, conv2, _ = oracle.focus_iterate(P, n_crit, curve, fa, fb, theta, K=K0)
    assert conv2 and np.array_equal(K2, ref)
    # with F moved: the old focused tree converges to the new one
    fa2 = fb
    fb2 = min(END, fb + (fb - fa))
    ref2 = oracle.focus_leaves(P, n_crit, curve, fa2, fb2, theta)
    K3, _, _, conv3, _ = oracle.focus_iterate(P, n_crit, curve, fa2, fb2, theta, K=ref)
    assert conv3 and np.array_equal(K3, ref2)


def test_focus_step_merges_siblings_that_pass_the_mac():
    """A complete group of 8 sibling leaves far from F whose parent passes the
    MAC is merged even though it holds more than N_crit particles."""
    M = oracle.MORTON
    K = np.array([0] + [(7 << 60) + (j << 57) for j in range(8)] + [END], np.uint64)
    K = np.concatenate([[0], [(d << 60) for d in range(1, 7)], K[1:]]).astype(np.uint64)
    K = np.unique(K)
    N = np.full(K.size - 1, 100, np.uint32)
    K2, changed = oracle.focus_rebalance_step(K, N, 16, M, 0, 1 << 54, 2.0)
    assert changed
    # octant 0 holds F and splits; octants 1-6 pass the MAC and stay; the
    # children of octant 7 merge
    assert list(K2) == [j << 57 for j in range(8)] + [d << 60 for d in range(1, 8)] + [END]
    # with theta = 0 the MAC never passes: the group stays, the leaves split
    K3, _ = oracle.focus_rebalance_step(K, N, 16, M, 0, 1 << 54, 0.0)
    assert K3.size - 1 == 8 * (K.size - 1)


# ---- binary radix tree (Sec. 5) --------------------------------------------------------

@pytest.mark.parametrize("seed,n_crit", [(1, 1), (2, 16), (3, 4)])
def test_radix_nodes_structure(seed, n_crit):
    rng = np.random.default_rng(seed)
    P = clustered_P(rng, 5000)
    K = oracle.build_leaves(P, n_crit)
    keys = K[:-1]
    m = keys.size
    pl, fi, la = oracle.radix_nodes(keys)
    assert pl.size == m - 1
    ranges = {}
    for i in range(m - 1):
        d = int(pl[i])
        # range of the prefix by binary search of its key bounds (not by scanning)
        pre = int(keys[i]) >> (63 - d)
        a = int(np.searchsorted(keys, np.uint64(pre << (63 - d))))
        b = int(np.searchsorted(keys, np.uint64((pre + 1) << (63 - d)))) - 1 if (pre + 1) << (63 - d) < END else m - 1
        assert (fi[i], la[i]) == (a, b), i
        assert fi[i] <= i < la[i]
        # the two keys at the split differ in the bit right after the prefix
        assert (int(keys[i]) >> (62 - d)) & 1 == 0 and (int(keys[i + 1]) >> (62 - d)) & 1 == 1
        ranges[(int(fi[i]), int(la[i]))] = i
    assert len(ranges) == m - 1  # one node per range
    assert (0, m - 1) in ranges  # the root covers every key
    # every node but the root is exactly one child: left [first, i], right [i + 1, last]
    parents = {}
    for (a, b), i in ranges.items():
        for child in ((a, i), (i + 1, b)):
            if child[0] < child[1]:
                assert child in ranges
                assert child not in parents
                parents[child] = i
    assert len(parents) == m - 2


def test_radix_nodes_with_prefix_length_3l_are_the_octree_nodes():
    rng = np.random.default_rng(9)
    for n_crit in (1, 8, 64):
        P = clustered_P(rng, 20000)
        K = oracle.build_leaves(P, n_crit)
        keys = K[:-1]
        pl, fi, la = oracle.radix_nodes(keys)
        sel = np.flatnonzero(pl % 3 == 0)
        got = sorted((1 << int(pl[i])) | (int(keys[i]) >> (63 - int(pl[i]))) for i in sel)
        NK, CO, LO = oracle.link_octree(K)
        internal = sorted(int(k) for k in NK[CO != 0])
        assert got == internal


# ---- compact octree (Sec. 5, empty buckets removed) ---------------------------------------


def test_compact_octree_without_empty_leaves_is_the_linked_octree():
    rng = np.random.default_rng(21)
    for n_crit in (1, 4, 16):
        P = clustered_P(rng, 8000)
        K = oracle.build_leaves(P, n_crit)
        ones = np.ones(K.size - 1, np.uint32)  # every leaf counted as non-empty
        NKc, par = oracle.compact_octree(K, ones)
        NK, CO, LO = oracle.link_octree(K)
        assert np.array_equal(NKc, NK)
        for p in np.flatnonzero(CO):
            assert all(par[c] == p for c in range(CO[p], CO[p] + 8))
        assert par[0] == 0xFFFFFFFF


@pytest.mark.parametrize("seed", range(5))
def test_compact_octree_structure(seed):
    rng = np.random.default_rng(seed)
    P = clustered_P(rng, 3000)
    K = oracle.build_leaves(P, int(rng.integers(1, 9)))
    N = oracle.node_counts(P, K)
    NKc, par = oracle.compact_octree(K, N)
    ranges = [placeholder_range(int(k)) for k in NKc]
    # every non-empty leaf is a node, no empty one is
    leaf_keys = {(int(K[i]), int(K[i + 1])) for i in range(K.size - 1) if N[i]}
    present = {(a, b) for a, b, _ in ranges}
    assert leaf_keys <= present
    assert not {(int(K[i]), int(K[i + 1])) for i in range(K.size - 1) if not N[i]} & present
    # parents contain their children; at most one node has no parent
    children = {}
    for p, q in enumerate(par):
        if q == 0xFFFFFFFF:
            continue
        a, b, lv = ranges[p]
        pa, pb, plv = ranges[q]
        assert pa <= a and b <= pb and plv < lv
        children.setdefault(int(q), []).append(p)
    assert int(np.sum(par == 0xFFFFFFFF)) == 1 and par[0] == 0xFFFFFFFF and NKc[0] == 1  # the root
    # internal nodes but the root have 2 or more children
    internal = set(range(NKc.size)) - {i for i, r in enumerate(ranges) if (r[0], r[1]) in leaf_keys}
    for q in internal:
        assert q == 0 or len(children.get(q, [])) >= 2, q
    assert len(children.get(0, [])) >= 1
    # brute force: a node is internal iff two adjacent non-empty leaves split exactly at its digit boundary
    lk = sorted(a for a, b in leaf_keys)
    want = set()
    for x, y in zip(lk[:-1], lk[1:]):
        d = 63 - (x ^ y).bit_length()
        if d % 3 == 0:
            want.add((1 << d) | (x >> (63 - d) if d else 0))
    assert {int(NKc[q]) for q in internal} == want | {1}


def test_compact_octree_degenerate():
    K = np.array([0, END], np.uint64)
    NKc, par = oracle.compact_octree(K, np.array([5], np.uint32))  # the root is the only leaf
    assert list(NKc) == [1] and list(par) == [0xFFFFFFFF]
    NKc, par = oracle.compact_octree(K, np.array([0], np.uint32))  # no particles: the root alone
    assert list(NKc) == [1] and list(par) == [0xFFFFFFFF]
    K = np.array([0] + [j << 60 for j in range(1, 8)] + [END], np.uint64)
    NKc, par = oracle.compact_octree(K, np.array([0, 0, 3, 0, 0, 0, 0, 0], np.uint32))  # one non-empty octant
    assert list(NKc) == [1, 0o12] and list(par) == [0xFFFFFFFF, 0]
