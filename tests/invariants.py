"""Property checks for the octree build, written independently of both the
oracle and the HIP path (numpy only). They hold at any size, so the full-size
GPU runs use them where the oracle would be too slow, and the oracle tests use
them as pins.

Every check follows a statement of the paper:
  * Eq. cstone (Sec. 4): K_0 = 0, K_{n_l} = 8^L, increasing, gaps powers of 8;
    plus alignment K_i mod delta_i = 0 (Sec. 3: a level-i node covers
    [k, k + 8^(L-i)) with k mod 8^(L-i) = 0);
  * balance (Sec. 4): leaf counts <= N_crit, internal node counts > N_crit
    (a leaf of span 1 cannot be divided and is exempt);
  * linked format (Sec. 5): n_i = (n_l - 1) / 7, placeholder-bit node keys,
    breadth-first order, CO = first child (0 for leaves), LO = level offsets.
"""
from __future__ import annotations

import numpy as np

L = 21
ROOT_END = np.uint64(1 << 63)


def is_pow8(d: np.ndarray) -> np.ndarray:
    d = d.astype(np.uint64)
    pow2 = (d != 0) & ((d & (d - np.uint64(1))) == 0)
    # log2 divisible by 3: the single set bit sits at a position 0, 3, 6, ...
    return pow2 & ((d & np.uint64(0x9249249249249249)) != 0)


def span_level(d: np.ndarray) -> np.ndarray:
    """Division level L - log8(delta) of spans that are powers of 8."""
    lg = np.zeros(d.shape, np.int64)
    dd = d.astype(np.uint64).copy()
    for s in (32, 16, 8, 4, 2, 1):
        big = dd >= (np.uint64(1) << np.uint64(s))
        lg[big] += s
        dd[big] >>= np.uint64(s)
    return L - lg // 3


def check_cornerstone(K: np.ndarray):
    K = K.astype(np.uint64)
    assert K.size >= 2, "a cornerstone array has at least 2 keys"
    assert K[0] == 0, "K_0 must be 0"
    assert K[-1] == ROOT_END, "K_{n_l} must be 8^L"
    d = np.diff(K)
    assert np.all(K[1:] > K[:-1]), "keys must increase"
    assert np.all(is_pow8(d)), "every gap must be a power of 8"
    assert np.all(K[:-1] % d == 0), "every leaf must be aligned to its span"
    assert (K.size - 2) % 7 == 0, "(n_l - 1) must be a multiple of 7"


def counts_by_search(P: np.ndarray, K: np.ndarray) -> np.ndarray:
    pos = np.searchsorted(P.astype(np.uint64), K.astype(np.uint64), side="left")
    return np.diff(pos).astype(np.int64)


def internal_nodes(K: np.ndarray):
    """(start, level) of every internal node, found as the distinct proper
    ancestors of the leaves."""
    K = K.astype(np.uint64)
    lev = span_level(np.diff(K))
    starts, levels = [], []
    for l in range(0, L):
        sel = lev > l
        if not np.any(sel):
            break
        span = np.uint64(1) << np.uint64(3 * (L - l))
        st = np.unique((K[:-1][sel] // span) * span)
        starts.append(st)
        levels.append(np.full(st.size, l))
    if not starts:
        return np.zeros(0, np.uint64), np.zeros(0, np.int64)
    return np.concatenate(starts), np.concatenate(levels)


def check_balanced(P: np.ndarray, K: np.ndarray, n_crit: int, counts: np.ndarray | None = None):
    """Leaf counts <= n_crit (span-1 leaves exempt), every internal node count
    > n_crit, counts sum to N. Together with Eq. cstone these fix K uniquely."""
    P = P.astype(np.uint64)
    K = K.astype(np.uint64)
    check_cornerstone(K)
    N = counts_by_search(P, K)
    if counts is not None:
        assert np.array_equal(N, counts.astype(np.int64)), "counts differ from binary-search counts"
    assert N.sum() == P.size, "leaf counts must sum to the particle count"
    d = np.diff(K)
    over = (N > n_crit) & (d > 1)
    assert not np.any(over), f"{int(over.sum())} leaves hold more than N_crit particles"
    st, lv = internal_nodes(K)
    if st.size:
        span = np.left_shift(np.uint64(1), (3 * (L - lv)).astype(np.uint64))
        end = st + span
        cnt = np.searchsorted(P, end, side="left") - np.searchsorted(P, st, side="left")
        assert np.all(cnt > n_crit), "an internal node holds <= N_crit particles (8 mergeable siblings)"


def check_sorted_perm(keys: np.ndarray, P: np.ndarray, perm: np.ndarray):
    """Full characterisation of a stable sort by key."""
    keys = keys.astype(np.uint64)
    n = keys.size
    assert P.size == n and perm.size == n
    if n == 0:
        return
    perm = perm.astype(np.int64)
    assert np.all(P[1:] >= P[:-1]), "sorted keys must be non-decreasing"
    seen = np.zeros(n, bool)
    assert perm.min() >= 0 and perm.max() < n
    seen[perm] = True
    assert seen.all(), "perm must be a permutation"
    assert np.array_equal(keys[perm], P), "P[i] must equal keys[perm[i]]"
    tie = P[1:] == P[:-1]
    assert np.all(perm[1:][tie] > perm[:-1][tie]), "equal keys must keep ascending original index"


def placeholder(start: np.ndarray, level: np.ndarray) -> np.ndarray:
    start = start.astype(np.uint64)
    level = np.asarray(level, np.int64)
    sh = (3 * (L - level)).astype(np.uint64)
    return (np.left_shift(np.uint64(1), (3 * level).astype(np.uint64))) | np.right_shift(start, sh)


def node_level(nk: np.ndarray) -> np.ndarray:
    """Level of placeholder-bit keys: (position of the leading 1) / 3."""
    nk = nk.astype(np.uint64)
    lg = np.zeros(nk.shape, np.int64)
    dd = nk.copy()
    for s in (32, 16, 8, 4, 2, 1):
        big = dd >= (np.uint64(1) << np.uint64(s))
        lg[big] += s
        dd[big] >>= np.uint64(s)
    return lg // 3


def check_linked(K: np.ndarray, NK: np.ndarray, CO: np.ndarray, LO: np.ndarray):
    """NK / CO / LO against the structural definition of Sec. 5."""
    K = K.astype(np.uint64)
    nl = K.size - 1
    ni = (nl - 1) // 7
    n = nl + ni
    assert NK.size == n and CO.size == n and LO.size == L + 2
    NK = NK.astype(np.uint64)
    CO = CO.astype(np.int64)
    LO = LO.astype(np.int64)
    assert np.all(NK[1:] > NK[:-1]), "NK must be strictly increasing (breadth-first, unique)"
    lev = node_level(NK)
    assert np.all(NK >= np.left_shift(np.uint64(1), (3 * lev).astype(np.uint64)))
    # the expected node set: leaves plus their distinct ancestors
    leaf_lv = span_level(np.diff(K))
    st, lv = internal_nodes(K)
    expect = np.sort(np.concatenate([placeholder(K[:-1], leaf_lv), placeholder(st, lv)]))
    assert np.array_equal(expect, NK), "NK must hold exactly the leaves and their ancestors"
    # level offsets: LO[l] = first node of level >= l, LO[L+1] = n
    for l in range(L + 1):
        assert LO[l] == np.searchsorted(NK, np.uint64(1) << np.uint64(3 * l), side="left")
    assert LO[L + 1] == n
    # CO: first child; the 8 children are contiguous with keys (NK[p] << 3) | c
    internal = CO != 0
    assert internal.sum() == ni, "exactly n_i nodes have children"
    p = np.nonzero(internal)[0]
    for c in range(8):
        assert np.array_equal(NK[CO[p] + c], (NK[p] << np.uint64(3)) | np.uint64(c))
    # every non-root node has exactly one parent
    parent_of = np.zeros(n, np.int64)
    for c in range(8):
        np.add.at(parent_of, CO[p] + c, 1)
    assert parent_of[0] == 0 and np.all(parent_of[1:] == 1)
    # the leaves (CO = 0), read in SFC order, are K in placeholder form
    leaves = NK[~internal]
    llev = node_level(leaves)
    start = np.left_shift(leaves ^ np.left_shift(np.uint64(1), (3 * llev).astype(np.uint64)),
                          (3 * (L - llev)).astype(np.uint64))
    assert np.array_equal(np.sort(start), K[:-1]), "leaf nodes must be the cornerstone leaves"
