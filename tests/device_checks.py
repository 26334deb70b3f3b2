"""Structural checks of large build outputs, run as plain torch operations on
the device (test infrastructure; none of the library's kernels is used).
They are the same properties tests/invariants.py checks on the host, written
for arrays too large to check there quickly. uint64 values sit in int64
containers; XOR with the sign bit maps them to an order-preserving int64."""
import torch

L = 21
SIGN = -(1 << 63)  # the bit pattern of 2^63 (the closing key 8^21)


def ordered(t):
    return torch.bitwise_xor(t, torch.tensor(SIGN, dtype=torch.int64, device=t.device))


def check_sorted_perm(P, perm, n, keys=None):
    """P non-decreasing (keys < 2^63), perm a permutation, ties ascending, and
    (if the unsorted keys are given) P[i] = keys[perm[i]]: together these fix
    the stable sort's output exactly."""
    assert P.numel() == n and perm.numel() == n
    if keys is not None and n:
        assert torch.equal(P, keys[perm.long()]), "P must be the keys taken through perm"
    if n < 2:
        return
    assert bool((P[1:] >= P[:-1]).all()), "sorted keys must be non-decreasing"
    p = perm.long()
    assert int(p.min()) >= 0 and int(p.max()) < n
    assert bool((torch.bincount(p, minlength=n) == 1).all()), "perm must be a permutation"
    tie = P[1:] == P[:-1]
    assert bool((p[1:][tie] > p[:-1][tie]).all()), "equal keys must keep ascending original index"


def leaf_levels(K):
    """Levels of the leaves of a cornerstone array (K int64 view, closing 2^63)."""
    delta = K[1:] - K[:-1]  # wraps to the right bit pattern for the last leaf
    if delta.numel() == 1:
        return torch.zeros(1, dtype=torch.int64, device=K.device), delta
    assert bool((delta > 0).all()), "K must be strictly increasing"
    assert bool(((delta & (delta - 1)) == 0).all()), "every span must be a power of two"
    lg = torch.log2(delta.double()).round().long()  # exact for powers of two
    assert bool((lg % 3 == 0).all()), "every span must be a power of 8"
    return L - lg // 3, delta


def check_balanced(P, K, counts, n_crit):
    """Eq. cstone, counts by binary search, every leaf within N_crit (spans
    of 1 exempt) and no 8 sibling leaves with at most N_crit together: by the
    uniqueness of the fixed point this is exactly the top-down tree."""
    n = P.numel()
    nl = K.numel() - 1
    assert int(K[0]) == 0 and int(K[-1]) == SIGN, "K must run from 0 to 8^21"
    lev, delta = leaf_levels(K)
    Kl = K[:-1]
    if nl > 1:
        assert bool((Kl % delta == 0).all()), "leaves must be aligned to their span"
    pos = torch.searchsorted(P, Kl)
    end = torch.full((1,), n, dtype=pos.dtype, device=pos.device)
    N = torch.diff(torch.cat([pos, end]))
    assert bool((N == counts.long()).all()), "counts differ from binary-search counts"
    assert int(N.sum()) == n
    over = (N > n_crit) & (delta != 1)
    assert not bool(over.any()), f"{int(over.sum())} leaves hold more than N_crit particles"
    if nl >= 8:
        m = nl - 7
        d = delta[:m]
        first = (Kl[:m] // d) % 8 == 0  # first of 8 siblings (d > 0 except the root)
        same = (K[8:8 + m] - K[:m]) == 8 * d  # 8 leaves of span d (wrapping arithmetic, exact mod 2^64)
        S = torch.cat([torch.zeros(1, dtype=torch.int64, device=N.device), torch.cumsum(N, 0)])
        group = S[8:8 + m] - S[:m]
        bad = first & same & (group <= n_crit) & (lev[:m] > 0)
        assert not bool(bad.any()), f"{int(bad.sum())} groups of 8 sibling leaves could merge"
    return N


def node_levels(NK):
    """Level of placeholder-bit node keys: (index of the leading 1) / 3."""
    x = NK.clone()
    lg = torch.zeros_like(x)
    top = x < 0  # bit 63 set: level 21
    x = torch.where(top, torch.zeros_like(x), x)
    for s in (32, 16, 8, 4, 2, 1):
        big = (x >> s) != 0
        lg = torch.where(big, lg + s, lg)
        x = torch.where(big, x >> s, x)
    lg = torch.where(top, torch.full_like(lg, 63), lg)
    return lg // 3


def check_linked(K, NK, CO, LO):
    """Sec. 5 structure: NK strictly increasing in placeholder form, LO the
    level starts, CO the first of 8 contiguous children (NK << 3) | c, one
    parent per non-root node, and the childless nodes equal to the leaves."""
    nl = K.numel() - 1
    ni = (nl - 1) // 7
    n = nl + ni
    assert NK.numel() == n and CO.numel() == n and LO.numel() == L + 2
    NKo = ordered(NK)
    assert bool((NKo[1:] > NKo[:-1]).all()), "NK must be strictly increasing"
    starts = torch.tensor([(1 << (3 * l)) if l < L else SIGN for l in range(L + 1)], dtype=torch.int64,
                          device=NK.device)
    lo = torch.searchsorted(NKo, ordered(starts))
    assert torch.equal(LO[:L + 1].long(), lo) and int(LO[L + 1]) == n, "level offsets"
    co = CO.long()
    internal = co != 0
    assert int(internal.sum()) == ni, "exactly n_i nodes have children"
    p = torch.nonzero(internal).flatten()
    parents = torch.zeros(n, dtype=torch.int64, device=NK.device)
    for c in range(8):
        ch = co[p] + c
        assert bool((NK[ch] == ((NK[p] << 3) | c)).all()), "children keys"
        parents += torch.bincount(ch, minlength=n)
    assert int(parents[0]) == 0 and bool((parents[1:] == 1).all()), "one parent per non-root node"
    # the childless nodes, read in SFC order (by start key), are the leaves of K
    lev, _ = leaf_levels(K)
    leaf_nk = NK[~internal]
    llev = node_levels(leaf_nk)
    start = (leaf_nk - (torch.ones_like(llev) << (3 * llev))) << (3 * (L - llev))  # drop the placeholder bit
    order = torch.argsort(start)
    assert torch.equal(start[order], K[:-1]), "childless nodes must be the leaves of K"
    assert torch.equal(llev[order], lev), "childless nodes must have the levels of the leaves"
