"""Pins for the oracle's sort, counts, leaves, rebalance step and links
(Secs. 4-5): brute force on tiny inputs, the paper's worked examples
(Figs. 1 and 2), and the balance / linked-format invariants, which determine
the outputs uniquely.
"""
import numpy as np
import pytest

import oracle
from tests import invariants as inv

L = 21
END = 1 << 63


def octal_prefix_key(prefix: str) -> int:
    """Key whose leading octal digits are `prefix`, padded with zeros to L digits."""
    return int(prefix, 8) << (3 * (L - len(prefix)))


def fig_array(prefixes):
    return np.array([octal_prefix_key(p) for p in prefixes] + [END], dtype=np.uint64)


def point_in(prefix: str):
    """Grid point inside the Morton cell of the given octal prefix (Morton digits
    carry x, y, z bits as 4, 2, 1)."""
    x = y = z = 0
    for d in prefix:
        d = int(d)
        x = (x << 1) | (d >> 2)
        y = (y << 1) | ((d >> 1) & 1)
        z = (z << 1) | (d & 1)
    sh = L - len(prefix)
    return x << sh, y << sh, z << sh


def keys_for(prefixes):
    return np.sort(np.array([oracle.morton_key(*point_in(p)) for p in prefixes], dtype=np.uint64))


# ---- sort ------------------------------------------------------------------

@pytest.mark.parametrize("n,distinct", [(0, 1), (1, 1), (2, 1), (1000, 7), (5000, 1 << 40)])
def test_sort_is_stable_sort(n, distinct):
    rng = np.random.default_rng(n)
    keys = (rng.integers(0, distinct, n, dtype=np.int64).astype(np.uint64) * np.uint64(977)) % np.uint64(END)
    P, perm = oracle.sort(keys)
    inv.check_sorted_perm(keys, P, perm)


# ---- counts ----------------------------------------------------------------

def test_counts_brute_force():
    rng = np.random.default_rng(1)
    for trial in range(30):
        P = np.sort(rng.integers(0, 64, rng.integers(0, 40)).astype(np.uint64) << np.uint64(57))
        K = oracle.build_leaves(P, int(rng.integers(1, 5)))
        N = oracle.node_counts(P, K)
        brute = [sum(1 for p in P if K[i] <= p < K[i + 1]) for i in range(K.size - 1)]
        assert list(N) == brute
        assert N.sum() == P.size


# ---- leaves ----------------------------------------------------------------

def test_fig1_refined_array(golden_fig):
    # Fig. 1: N_crit = 1, two particles in different children of octant 2 and at
    # most one particle in every other octant give the bottom panel.
    P = keys_for(["0", "1", "21", "26", "3", "5", "7"])
    K = oracle.build_leaves(P, 1)
    assert np.array_equal(K, fig_array(golden_fig["fig1_bottom_octal_prefixes"]))
    assert K.size - 1 == 15


def test_fig1_one_step_split_and_reverse_merge(golden_fig):
    top = fig_array(golden_fig["fig1_top_octal_prefixes"])
    bottom = fig_array(golden_fig["fig1_bottom_octal_prefixes"])
    # split: only octant 2 exceeds N_crit = 1
    P = keys_for(["0", "1", "21", "26", "3", "5", "7"])
    K2, changed = oracle.rebalance_step(top, oracle.node_counts(P, top), 1)
    assert changed and np.array_equal(K2, bottom)
    # reverse: octant 2's children now hold one particle in total -> merge
    P = keys_for(["0", "1", "24", "3", "5", "7"])
    K3, changed = oracle.rebalance_step(bottom, oracle.node_counts(P, bottom), 1)
    assert changed and np.array_equal(K3, top)
    # fixed point: top with these particles is balanced, nothing changes
    K4, changed = oracle.rebalance_step(top, oracle.node_counts(P, top), 1)
    assert not changed and np.array_equal(K4, top)


def test_step_split_and_merge_in_one_update():
    # octant 2's children merge while octant 5 splits, in the same application of g
    bottom = fig_array(["0", "1", "20", "21", "22", "23", "24", "25", "26", "27", "3", "4", "5", "6", "7"])
    P = keys_for(["0", "1", "23", "3", "51", "53", "7"])
    K2, changed = oracle.rebalance_step(bottom, oracle.node_counts(P, bottom), 1)
    expect = fig_array(["0", "1", "2", "3", "4"] + [f"5{c}" for c in range(8)] + ["6", "7"])
    assert changed and np.array_equal(K2, expect)
    assert K2.size == bottom.size  # +7 and -7: a leaf-count comparison would miss the change


def test_root_only_cases():
    root = np.array([0, END], np.uint64)
    for P in (np.zeros(0, np.uint64), np.array([5], np.uint64), np.arange(64, dtype=np.uint64)):
        K = oracle.build_leaves(P, 64)
        assert np.array_equal(K, root)
        K2, changed = oracle.rebalance_step(root, oracle.node_counts(P, root), 64)
        assert not changed and np.array_equal(K2, root)


def test_duplicates_stop_at_level_21():
    # 10 particles on one grid point: the leaf holding them reaches span 1 and
    # cannot be split further (reading R6).
    P = np.full(10, 12345, np.uint64)
    K = oracle.build_leaves(P, 4)
    inv.check_balanced(P, K, 4)
    assert 12345 in K and 12346 in K
    K_it, N, rounds, conv, _ = oracle.rebalance_iterate(P, np.array([0, END], np.uint64), 4)
    assert conv and np.array_equal(K_it, K) and rounds <= L + 1


def _random_keys(rng, n, kind):
    if kind == "uniform":
        return rng.integers(0, END, n, dtype=np.uint64)
    if kind == "clustered":
        c = rng.integers(0, END, 4, dtype=np.uint64)
        return (c[rng.integers(0, 4, n)] + rng.integers(0, 1 << 30, n).astype(np.uint64)) % np.uint64(END)
    if kind == "coarse":  # many duplicates
        return rng.integers(0, 512, n).astype(np.uint64) << np.uint64(54)
    raise ValueError(kind)


@pytest.mark.parametrize("kind", ["uniform", "clustered", "coarse"])
@pytest.mark.parametrize("n_crit", [1, 3, 16, 64])
def test_leaves_balanced_and_iteration_reaches_them(kind, n_crit):
    rng = np.random.default_rng(hash((kind, n_crit)) & 0xFFFF)
    for n in (0, 1, n_crit, n_crit + 1, 700, 3000):
        P = np.sort(_random_keys(rng, n, kind))
        K = oracle.build_leaves(P, n_crit)
        inv.check_balanced(P, K, n_crit, oracle.node_counts(P, K))
        # from the root: the fixed point of f and g is the top-down tree, reached
        # in depth + 1 rounds (at most L + 1)
        K_it, N, rounds, conv, hist = oracle.rebalance_iterate(P, np.array([0, END], np.uint64), n_crit)
        assert conv and np.array_equal(K_it, K)
        depth = int(L - np.log2(np.diff(K).min().astype(float)) // 3) if K.size > 2 else 0
        assert rounds == depth + 1 and rounds <= L + 1
        # from an unrelated previous tree (another particle set) as in a later time-step
        P_old = np.sort(_random_keys(rng, 500, "uniform"))
        K_old = oracle.build_leaves(P_old, 2)
        K_inc, _, rounds_inc, conv, _ = oracle.rebalance_iterate(P, K_old, n_crit)
        assert conv and np.array_equal(K_inc, K) and rounds_inc <= L + 1


# ---- links -----------------------------------------------------------------

def test_fig2_linked_octree(golden_fig):
    K = fig_array(golden_fig["fig1_bottom_octal_prefixes"])
    NK, CO, LO = oracle.link_octree(K)
    expect_lo = golden_fig["fig2_LO_prefix"] + [golden_fig["fig2_LO_tail_value"]] * (L + 2 - 3)
    assert list(LO) == expect_lo
    assert [int(v) for v in NK] == [int(s, 8) for s in golden_fig["fig2_NK_octal"]]
    assert list(CO) == golden_fig["fig2_CO"]
    assert NK.size == 15 + (15 - 1) // 7


def test_link_root_only():
    NK, CO, LO = oracle.link_octree(np.array([0, END], np.uint64))
    assert list(NK) == [1] and list(CO) == [0] and list(LO) == [0] + [1] * (L + 1)


def _prefix_set_brute_force(K):
    nodes = set()
    for i in range(K.size - 1):
        d = int(K[i + 1] - K[i])
        lv = L - (d.bit_length() - 1) // 3
        for l in range(lv + 1):
            nodes.add((l, int(K[i]) >> (3 * (L - l))))
    return sorted((1 << (3 * l)) | pre for l, pre in nodes)


@pytest.mark.parametrize("n_crit", [1, 4, 32])
def test_link_structure_random_trees(n_crit):
    rng = np.random.default_rng(n_crit)
    for trial in range(12):
        kind = ["uniform", "clustered", "coarse"][trial % 3]
        P = np.sort(_random_keys(rng, int(rng.integers(0, 2000)), kind))
        K = oracle.build_leaves(P, n_crit)
        NK, CO, LO = oracle.link_octree(K)
        inv.check_linked(K, NK, CO, LO)
        if K.size < 400:
            assert [int(v) for v in NK] == _prefix_set_brute_force(K)
