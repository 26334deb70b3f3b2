"""CPU oracle for the Cornerstone octree build (test infrastructure only).

This package is the plain, slow, single-threaded reference that the HIP
implementation is checked against. Only the test suite, the smoke check and
the benchmark's CPU-baseline leg may import it; the product path never does,
and it imports nothing from the product package.

It wraps ``cstone_oracle.cpp`` (built into ``liboracle.so`` next to this file
by :func:`compile_library`) with numpy-in / numpy-out functions. See the header of the
C++ file for what each function follows in the paper and how it is pinned.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cstone_oracle.cpp")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

L = 21
ROOT_END = 1 << 63
MORTON = 0
HILBERT = 1

_lib = None


def compile_library(verbose: bool = False) -> str:
    """Compile the oracle with g++ (strict IEEE: no fast-math, no contraction)."""
    cmd = ["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-shared", "-fPIC",
           "-Wall", "-Wextra", "-o", _LIB_PATH + ".tmp", _SRC]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        compile_library()
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    u64, u32, i32 = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
    sigs = {
        "oracle_quantize": (i32, [P, P, P, u64, P, P, P, P, P]),
        "oracle_morton_key": (u64, [u32, u32, u32]),
        "oracle_hilbert_key": (u64, [u32, u32, u32, i32]),
        "oracle_hilbert_decode": (None, [u64, i32, P]),
        "oracle_compute_keys": (i32, [P, P, P, u64, P, P, i32, P]),
        "oracle_sort": (None, [P, u64, P, P]),
        "oracle_node_counts": (None, [P, u64, P, u64, P]),
        "oracle_build_leaves": (u64, [P, u64, u32, P, u64]),
        "oracle_rebalance_step": (i32, [P, u64, P, u32, P, u64, P]),
        "oracle_node_count": (u64, [u64]),
        "oracle_link_octree": (u64, [P, u64, P, P, P]),
        "oracle_build": (u64, [P, P, P, u64, P, P, i32, u32, P, P, P, u64, P]),
        "oracle_octree_node_counts": (None, [P, u64, P, u64, P]),
        "oracle_sfc_partition": (None, [P, u64, u32, P]),
        "oracle_mac_fails": (i32, [u64, i32, i32, u64, u64, ctypes.c_double]),
        "oracle_node_box": (None, [u64, i32, i32, P, P]),
        "oracle_focus_leaves": (u64, [P, u64, u32, i32, u64, u64, ctypes.c_double, P, u64]),
        "oracle_focus_rebalance_step": (i32, [P, u64, P, u32, i32, u64, u64, ctypes.c_double, P, u64, P]),
        "oracle_radix_nodes": (None, [P, u64, P, P, P]),
        "oracle_compact_octree": (u64, [P, u64, P, P, P, u64]),
    }
    for name, (res, args) in sigs.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _u64(a):
    return np.ascontiguousarray(a, dtype=np.uint64)


def _box(box):
    lo = np.ascontiguousarray(box[0], dtype=np.float64).reshape(3)
    hi = np.ascontiguousarray(box[1], dtype=np.float64).reshape(3)
    return lo, hi


def quantize(x, y, z, box):
    """Integer grid coordinates (ix, iy, iz) and the non-finite flag."""
    lib = _load()
    x, y, z = _f64(x), _f64(y), _f64(z)
    lo, hi = _box(box)
    n = x.size
    ix, iy, iz = (np.empty(n, np.uint32) for _ in range(3))
    flag = lib.oracle_quantize(_ptr(x), _ptr(y), _ptr(z), n, _ptr(lo), _ptr(hi), _ptr(ix), _ptr(iy), _ptr(iz))
    return ix, iy, iz, bool(flag)


def morton_key(ix: int, iy: int, iz: int) -> int:
    return int(_load().oracle_morton_key(ix, iy, iz))


def hilbert_key(ix: int, iy: int, iz: int, bits: int = L) -> int:
    return int(_load().oracle_hilbert_key(ix, iy, iz, bits))


def hilbert_decode(key: int, bits: int = L):
    out = np.zeros(3, np.uint32)
    _load().oracle_hilbert_decode(key, bits, _ptr(out))
    return int(out[0]), int(out[1]), int(out[2])


def compute_keys(x, y, z, box, curve):
    """SFC keys (uint64) of every particle and the non-finite flag."""
    lib = _load()
    x, y, z = _f64(x), _f64(y), _f64(z)
    lo, hi = _box(box)
    keys = np.empty(x.size, np.uint64)
    flag = lib.oracle_compute_keys(_ptr(x), _ptr(y), _ptr(z), x.size, _ptr(lo), _ptr(hi), int(curve), _ptr(keys))
    return keys, bool(flag)


def sort(keys):
    """Stable sort: (sorted keys P, permutation perm) with P[i] = keys[perm[i]]."""
    keys = _u64(keys)
    P = np.empty_like(keys)
    perm = np.empty(keys.size, np.uint32)
    _load().oracle_sort(_ptr(keys), keys.size, _ptr(P), _ptr(perm))
    return P, perm


def node_counts(P, K):
    P, K = _u64(P), _u64(K)
    counts = np.empty(K.size - 1, np.uint32)
    _load().oracle_node_counts(_ptr(P), P.size, _ptr(K), K.size - 1, _ptr(counts))
    return counts


def build_leaves(P, n_crit: int):
    """Balanced cornerstone array K (n_l + 1 keys) by top-down recursion."""
    P = _u64(P)
    lib = _load()
    cap = 1024
    while True:
        K = np.empty(cap, np.uint64)
        nl = lib.oracle_build_leaves(_ptr(P), P.size, int(n_crit), _ptr(K), cap)
        if nl + 1 <= cap:
            return K[: nl + 1].copy()
        cap = int(nl) + 1


def rebalance_step(K, N, n_crit: int):
    """One literal g3.g2.g1 update. Returns (K', changed)."""
    K = _u64(K)
    N = np.ascontiguousarray(N, dtype=np.uint32)
    nl = K.size - 1
    cap = 8 * nl + 1
    out = np.empty(cap, np.uint64)
    nl_out = ctypes.c_uint64(0)
    changed = _load().oracle_rebalance_step(_ptr(K), nl, _ptr(N), int(n_crit), _ptr(out), cap,
                                            ctypes.byref(nl_out))
    return out[: nl_out.value + 1].copy(), bool(changed)


def rebalance_iterate(P, K, n_crit: int, max_iters: int = L + 1):
    """Alternate f and g from K until no leaf changes (or max_iters rounds).

    Returns (K, counts, rounds, converged, history) where history holds K after
    every round."""
    K = _u64(K)
    history = []
    for r in range(1, max_iters + 1):
        N = node_counts(P, K)
        K2, changed = rebalance_step(K, N, n_crit)
        history.append(K2)
        if not changed:
            return K2, node_counts(P, K2), r, True, history
        K = K2
    return K, node_counts(P, K), max_iters, False, history


def node_count(n_leaves: int) -> int:
    return int(n_leaves + (n_leaves - 1) // 7)


def link_octree(K):
    """Fully linked octree (NK uint64[n], CO uint32[n], LO uint32[23])."""
    K = _u64(K)
    nl = K.size - 1
    n = node_count(nl)
    NK = np.empty(n, np.uint64)
    CO = np.empty(n, np.uint32)
    LO = np.empty(L + 2, np.uint32)
    got = _load().oracle_link_octree(_ptr(K), nl, _ptr(NK), _ptr(CO), _ptr(LO))
    assert got == n, (got, n)
    return NK, CO, LO


def build_tree(x, y, z, box, curve=HILBERT, n_crit=64):
    """The whole pipeline of Secs. 3-5; returns a dict of every output."""
    keys, nonfinite = compute_keys(x, y, z, box, curve)
    P, perm = sort(keys)
    K = build_leaves(P, n_crit)
    counts = node_counts(P, K)
    NK, CO, LO = link_octree(K)
    return dict(keys=keys, nonfinite=nonfinite, P=P, perm=perm, K=K, counts=counts, NK=NK, CO=CO, LO=LO)


# ---- beyond the build: node properties, decomposition, focused tree ---------


def octree_node_counts(P, NK):
    """Particle count of every node of a linked octree (Sec. 5 node
    properties): keys of P inside each node's range, by Eq. histogram."""
    P, NK = _u64(P), _u64(NK)
    out = np.empty(NK.size, np.uint32)
    _load().oracle_octree_node_counts(_ptr(P), P.size, _ptr(NK), NK.size, _ptr(out))
    return out


def gather(a, perm):
    """Particle property in SFC order: out[i] = a[perm[i]] (Sec. 4, the
    permutation that sorts the keys applied to the particle arrays)."""
    return np.ascontiguousarray(a)[np.asarray(perm).astype(np.int64)]


def sfc_partition(counts, n_ranks: int):
    """Sec. 6: bounds (uint32[n_ranks + 1]) of n_ranks bins of consecutive
    leaves, bin r = leaves [bounds[r], bounds[r + 1])."""
    counts = np.ascontiguousarray(counts, dtype=np.uint32)
    out = np.empty(int(n_ranks) + 1, np.uint32)
    _load().oracle_sfc_partition(_ptr(counts), counts.size, int(n_ranks), _ptr(out))
    return out


def global_rebalance(P_parts, n_crit: int, K=None, max_iters: int = L + 1):
    """Sec. 6: the replicated tree of particles spread over several shards,
    each holding its own sorted keys. Every round computes f on every shard,
    sums the count arrays element-wise (f_r, the global reduction) and applies
    g to the summed counts; from the root unless K is given. Returns (K,
    summed counts, rounds, converged)."""
    K = np.array([0, ROOT_END], np.uint64) if K is None else _u64(K)
    for r in range(1, max_iters + 1):
        N = np.zeros(K.size - 1, np.uint64)
        for Pg in P_parts:
            N += node_counts(Pg, K)
        N = N.astype(np.uint32)
        K2, changed = rebalance_step(K, N, n_crit)
        if not changed:
            Nf = np.zeros(K2.size - 1, np.uint64)
            for Pg in P_parts:
                Nf += node_counts(Pg, K2)
            return K2, Nf.astype(np.uint32), r, True
        K = K2
    Nf = np.zeros(K.size - 1, np.uint64)
    for Pg in P_parts:
        Nf += node_counts(Pg, K)
    return K, Nf.astype(np.uint32), max_iters, False


def mac_fails(start: int, level: int, curve: int, fa: int, fb: int, theta: float) -> bool:
    """Sec. 7.1 minimum-distance MAC of node (start, level) against F = [fa, fb)."""
    return bool(_load().oracle_mac_fails(int(start), int(level), int(curve), int(fa), int(fb), float(theta)))


def node_box(start: int, level: int, curve: int):
    """(lower corner (3 ints), edge) of a node in grid cells."""
    lo = np.zeros(3, np.uint32)
    edge = np.zeros(1, np.uint32)
    _load().oracle_node_box(int(start), int(level), int(curve), _ptr(lo), _ptr(edge))
    return tuple(int(v) for v in lo), int(edge[0])


def focus_leaves(P, n_crit: int, curve: int, fa: int, fb: int, theta: float):
    """Sec. 7.1: the cornerstone array focused on F = [fa, fb), top-down."""
    P = _u64(P)
    lib = _load()
    cap = 1024
    while True:
        K = np.empty(cap, np.uint64)
        nl = lib.oracle_focus_leaves(_ptr(P), P.size, int(n_crit), int(curve), int(fa), int(fb), float(theta),
                                     _ptr(K), cap)
        if nl + 1 <= cap:
            return K[: nl + 1].copy()
        cap = int(nl) + 1


def focus_rebalance_step(K, N, n_crit: int, curve: int, fa: int, fb: int, theta: float):
    """One literal g^LE update (Sec. 7.2). Returns (K', changed)."""
    K = _u64(K)
    N = np.ascontiguousarray(N, dtype=np.uint32)
    nl = K.size - 1
    cap = 8 * nl + 1
    out = np.empty(cap, np.uint64)
    nl_out = ctypes.c_uint64(0)
    changed = _load().oracle_focus_rebalance_step(_ptr(K), nl, _ptr(N), int(n_crit), int(curve), int(fa), int(fb),
                                                  float(theta), _ptr(out), cap, ctypes.byref(nl_out))
    return out[: nl_out.value + 1].copy(), bool(changed)


def focus_iterate(P, n_crit: int, curve: int, fa: int, fb: int, theta: float, K=None, max_iters: int = L + 1):
    """Alternate f and g^LE from K (default the root) until no leaf changes.
    Returns (K, counts, rounds, converged, history)."""
    K = np.array([0, ROOT_END], np.uint64) if K is None else _u64(K)
    history = []
    for r in range(1, max_iters + 1):
        K2, changed = focus_rebalance_step(K, node_counts(P, K), n_crit, curve, fa, fb, theta)
        history.append(K2)
        if not changed:
            return K2, node_counts(P, K2), r, True, history
        K = K2
    return K, node_counts(P, K), max_iters, False, history


def radix_nodes(keys):
    """Binary radix tree over sorted unique keys: per adjacent pair i, the
    prefix length and key range [first, last] of the node that splits there."""
    keys = _u64(keys)
    m = keys.size
    k = max(m - 1, 0)
    pl, fi, la = (np.empty(k, np.uint32) for _ in range(3))
    if k:
        _load().oracle_radix_nodes(_ptr(keys), m, _ptr(pl), _ptr(fi), _ptr(la))
    return pl, fi, la


def compact_octree(K, counts):
    """Compact octree over the non-empty leaves (Sec. 5): (NK sorted, parent)."""
    K = _u64(K)
    counts = np.ascontiguousarray(counts, dtype=np.uint32)
    lib = _load()
    cap = max(2 * K.size, 16)
    NK = np.empty(cap, np.uint64)
    par = np.empty(cap, np.uint32)
    n = lib.oracle_compact_octree(_ptr(K), K.size - 1, _ptr(counts), _ptr(NK), _ptr(par), cap)
    assert n <= cap
    return NK[:n].copy(), par[:n].copy()
