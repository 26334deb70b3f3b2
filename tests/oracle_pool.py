"""Runs the CPU oracle over many particle sets, or over one very large set in
slices, on host threads (test infrastructure).

The oracle's work happens in C calls through ctypes, which release the GIL, so
a thread pool runs its builds in parallel inside the test process; no data is
copied to worker processes, and no second process touches the GPU.

Slicing a large set keeps the oracle's own definitions: keys are computed per
particle, so any slicing of the particles gives the same keys; and the
top-down leaves (split a node iff it holds more than N_crit particles) inside
a node that the recursion splits depend only on the sorted keys inside that
node, so the leaves of a large set are gathered node by node (see leaves()).
"""
from __future__ import annotations

import concurrent.futures as cf
import os

import numpy as np

import oracle

L = 21
END = np.uint64(1 << 63)


def workers() -> int:
    """Threads for oracle work: the host's CPUs, at most 16."""
    return max(1, min(16, os.cpu_count() or 1))


def pmap(fn, items, max_workers: int | None = None) -> list:
    """[fn(item) for item in items], run on a thread pool, in item order."""
    items = list(items)
    if not items:
        return []
    with cf.ThreadPoolExecutor(max_workers=max_workers or workers()) as ex:
        return list(ex.map(fn, items))


def mismatch(got, ref, what: str) -> list:
    """[] if the two arrays are equal element by element, else one message."""
    got = np.asarray(got)
    ref = np.asarray(ref)
    if got.shape != ref.shape:
        return [f"{what}: shape {got.shape} vs oracle {ref.shape}"]
    bad = np.flatnonzero(got != ref)
    if bad.size:
        return [f"{what}: {bad.size} mismatches, first at {bad[:5]}: {got[bad[:5]]} vs oracle {ref[bad[:5]]}"]
    return []


OUTPUTS = (("sorted_keys", "P"), ("perm", "perm"), ("leaves", "K"), ("counts", "counts"),
           ("node_keys", "NK"), ("child", "CO"), ("level_offsets", "LO"))


def compare_build(got: dict, x, y, z, box, curve, n_crit, tag: str) -> list:
    """Run the oracle on one set and compare every output of `got` (host
    arrays named as the build's outputs) element by element."""
    ref = oracle.build_tree(x, y, z, box, curve, n_crit)
    msgs = []
    for name, key in OUTPUTS:
        if name in got:
            msgs += mismatch(got[name], ref[key], f"{tag} {name}")
    return msgs


def keys(x, y, z, box, curve, chunk: int = 1 << 22) -> np.ndarray:
    """The oracle's keys of every particle, computed slice by slice on the pool."""
    n = x.size
    out = np.empty(n, np.uint64)

    def run(a):
        b = min(n, a + chunk)
        k, bad = oracle.compute_keys(x[a:b], y[a:b], z[a:b], box, curve)
        assert not bad, "non-finite coordinate"
        out[a:b] = k

    pmap(run, range(0, n, chunk))
    return out


def leaves(P: np.ndarray, n_crit: int, job_keys: int = 1 << 20) -> np.ndarray:
    """The oracle's top-down leaves of a large sorted key array, on the pool.

    The root is expanded by the oracle's own rule (a node holding more than
    n_crit particles, above level L, is split into its 8 children) until every
    node of the frontier holds at most `job_keys` particles. A frontier node
    holding more than n_crit particles is handed whole to the oracle, whose
    leaves inside it are the tree's there; one holding at most n_crit is a leaf
    (its parent was split). The leaves are the frontier's in SFC order."""
    P = np.ascontiguousarray(P, dtype=np.uint64)
    n = P.size
    job_keys = max(int(job_keys), int(n_crit) + 1)
    frontier = []  # (start, level, first, end) in SFC order

    def expand(start, level, a, b):
        if b - a > job_keys and level < L:
            span = 1 << (3 * (L - level - 1))
            bounds = np.searchsorted(P[a:b], np.array([start + c * span for c in range(1, 8)], np.uint64))
            cuts = [a] + [a + int(v) for v in bounds] + [b]
            for c in range(8):
                expand(start + c * span, level + 1, cuts[c], cuts[c + 1])
        else:
            frontier.append((start, level, a, b))

    expand(0, 0, 0, n)

    def run(item):
        start, level, a, b = item
        if b - a <= n_crit or level == L:
            return np.array([start], np.uint64)
        sub = oracle.build_leaves(P[a:b], n_crit)[:-1]
        lo, hi = np.uint64(start), np.uint64(start + (1 << (3 * (L - level))))
        return sub[(sub >= lo) & (sub < hi)]

    parts = pmap(run, frontier)
    return np.concatenate(parts + [np.array([END], np.uint64)])


def counts(P: np.ndarray, K: np.ndarray, chunk: int = 1 << 20) -> np.ndarray:
    """The oracle's leaf counts (Eq. histogram), slice by slice of the leaves."""
    nl = K.size - 1
    out = np.empty(nl, np.uint32)

    def run(a):
        b = min(nl, a + chunk)
        out[a:b] = oracle.node_counts(P, K[a:b + 1])

    pmap(run, range(0, nl, chunk))
    return out
