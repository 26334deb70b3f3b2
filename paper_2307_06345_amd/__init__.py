"""Python binding of libcstone, the MI355X Cornerstone octree build.

Thin ctypes marshalling over the C ABI declared in ``include/cstone.h``: every
function here has the name of the C entry point without the ``cstone_``
prefix, takes torch tensors that live on the GPU (PyTorch provides device
memory and streams only) and passes their pointers straight through. All the
work runs in the HIP kernels of ``libcstone.so``; if the library is missing
the import of this module fails.

Integer arrays are held in signed torch containers with the same bit
patterns: uint64 keys in ``torch.int64``, uint32 counts / permutation / CO / LO
in ``torch.int32``. :func:`to_numpy` returns them as unsigned numpy arrays.
"""
from __future__ import annotations

import ctypes
import os
import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcstone.so")

L = 21
KEY_END = 1 << 63
MORTON, HILBERT = 0, 1
LEVEL_OFFSETS = L + 2
FLAG_NONFINITE = 1

STATUS = {0: "OK", 1: "INVALID_ARG", 2: "NONFINITE", 3: "CAPACITY", 4: "NOT_CONVERGED", 5: "DEVICE"}


class CstoneError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {STATUS.get(status, status)}")
        self.status = status
        self.name = STATUS.get(status, str(status))


class Timings(ctypes.Structure):
    _fields_ = [("stage_ms", ctypes.c_float * 4), ("sort_pass_ms", ctypes.c_float * 8),
                ("sort_passes", ctypes.c_uint32)]


class Box(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3)]

    @classmethod
    def of(cls, box) -> "Box":
        lo, hi = box
        return cls((ctypes.c_double * 3)(*map(float, lo)), (ctypes.c_double * 3)(*map(float, hi)))


class CSet(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint64), ("box", Box), ("curve", ctypes.c_int32), ("n_crit", ctypes.c_uint32),
                ("leaf_capacity", ctypes.c_uint64)]


class BatchLayout(ctypes.Structure):
    _fields_ = [("n_sets", ctypes.c_uint64), ("n_particles", ctypes.c_uint64), ("leaf_slots", ctypes.c_uint64),
                ("node_slots", ctypes.c_uint64), ("workspace_bytes", ctypes.c_uint64), ("n_tiles", ctypes.c_uint64),
                ("sort_variant", ctypes.c_int32), ("rounds", ctypes.c_uint32)]


def _load() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2307_06345_amd.build.build() "
                          "(the octree build has no fallback path)")
    lib = ctypes.CDLL(LIB_PATH)
    P, sz, u32, i32 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_uint32, ctypes.c_int
    pbox = ctypes.POINTER(Box)
    psz = ctypes.POINTER(ctypes.c_size_t)
    pu32 = ctypes.POINTER(ctypes.c_uint32)
    sigs = {
        "cstone_status_string": (ctypes.c_char_p, [i32]),
        "cstone_compute_keys": (i32, [P, P, P, sz, pbox, i32, P, P, P]),
        "cstone_sort_workspace_bytes": (sz, [sz]),
        "cstone_sort": (i32, [P, P, P, sz, P, sz, P]),
        "cstone_node_counts": (i32, [P, sz, P, sz, P, P]),
        "cstone_rebalance_workspace_bytes": (sz, [sz, u32, sz]),
        "cstone_rebalance": (i32, [P, sz, u32, P, psz, sz, P, u32, pu32, P, sz, P]),
        "cstone_leaf_capacity_bound": (sz, [sz, u32, sz]),
        "cstone_node_count": (sz, [sz]),
        "cstone_link_workspace_bytes": (sz, [sz]),
        "cstone_link_octree": (i32, [P, sz, P, P, P, P, sz, P]),
        "cstone_link_octree_by_sort": (i32, [P, sz, P, P, P, P, sz, P]),
        "cstone_sort_variant_count": (i32, []),
        "cstone_sort_variant_info": (i32, [i32, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32)]),
        "cstone_sort_variant_split": (i32, [i32, ctypes.POINTER(i32)]),
        "cstone_set_lookback_patience": (i32, [u32]),
        "cstone_sort_autotune": (i32, [P, sz, P, P, P, sz, i32, ctypes.POINTER(ctypes.c_float),
                                       ctypes.POINTER(i32), P]),
        "cstone_radix_tree": (i32, [P, sz, P, P, P, P, P]),
        "cstone_link_octree_radix_workspace_bytes": (sz, [sz]),
        "cstone_link_octree_radix": (i32, [P, sz, P, P, P, P, sz, P]),
        "cstone_compact_octree_workspace_bytes": (sz, [sz]),
        "cstone_compact_octree": (i32, [P, P, sz, P, P, P, psz, P, sz, P]),
        "cstone_octree_node_counts_workspace_bytes": (sz, [sz]),
        "cstone_octree_node_counts": (i32, [P, P, sz, P, sz, P, P, sz, P]),
        "cstone_gather": (i32, [P, P, sz, P, P]),
        "cstone_gather_xyz": (i32, [P, P, P, P, sz, P, P, P, i32, P]),
        "cstone_global_rebalance_workspace_bytes": (sz, [sz, u32]),
        "cstone_global_rebalance": (i32, [P, P, u32, u32, P, psz, sz, P, u32, pu32, P, sz, P]),
        "cstone_build_sharded_workspace_bytes": (sz, [P, u32, sz]),
        "cstone_build_sharded": (i32, [P, P, P, P, u32, pbox, i32, u32, P, P, P, psz, sz, P, u32, pu32, P, sz, P]),
        "cstone_focus_rebalance_workspace_bytes": (sz, [sz]),
        "cstone_focus_rebalance": (i32, [P, sz, u32, i32, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_double, P, psz, sz,
                                         P, u32, pu32, P, sz, P]),
        "cstone_focus_mac_workspace_bytes": (sz, []),
        "cstone_focus_mac": (i32, [P, sz, i32, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_double, P, P, sz, P]),
        "cstone_sfc_partition_workspace_bytes": (sz, [sz]),
        "cstone_sfc_partition": (i32, [P, sz, u32, P, P, sz, P]),
        "cstone_tune_set": (i32, [i32, sz, i32]),
        "cstone_tune_get": (i32, [i32, sz]),
        "cstone_tune_clear": (None, []),
        "cstone_tune_entries": (sz, []),
        "cstone_tune_save": (i32, [ctypes.c_char_p]),
        "cstone_tune_load": (i32, [ctypes.c_char_p]),
        "cstone_batch_create": (i32, [ctypes.POINTER(CSet), u32, ctypes.POINTER(P)]),
        "cstone_batch_destroy": (None, [P]),
        "cstone_batch_get_layout": (i32, [P, ctypes.POINTER(BatchLayout), P, P, P]),
        "cstone_batch_set_variant": (i32, [P, i32]),
        "cstone_batch_set_rounds": (i32, [P, u32]),
        "cstone_batch_upload": (i32, [P, P, sz, P]),
        "cstone_batch_table_bytes": (sz, [P]),
        "cstone_batch_upload_staged": (i32, [P, P, sz, P, sz, P]),
        "cstone_batch_build": (i32, [P] + [P] * 11 + [P, sz, P]),
        "cstone_batch_capture": (i32, [P] + [P] * 11 + [P, sz, P]),
        "cstone_batch_launch": (i32, [P, P]),
        "cstone_batch_autotune": (i32, [P] + [P] * 11 + [P, sz, i32, ctypes.POINTER(ctypes.c_float), P]),
        "cstone_build_workspace_bytes": (sz, [sz, sz]),
        "cstone_build_static": (i32, [P, P, P, sz, pbox, i32, u32, P, P, P, psz, sz, P, P, P, P, u32, pu32, P]),
        "cstone_build": (i32, [P, P, P, sz, pbox, i32, u32, P, P, P, psz, sz, P, P, P, P, u32, pu32, P, sz,
                               ctypes.POINTER(Timings), P]),
    }
    for name, (res, args) in sigs.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _check(status: int, what: str):
    if status != 0:
        raise CstoneError(status, what)


def _dev(t: torch.Tensor, dtype) -> torch.Tensor:
    assert t.is_cuda, "device tensors expected"
    assert t.dtype == dtype and t.is_contiguous(), (t.dtype, dtype)
    return t


def _workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def to_numpy(t: torch.Tensor) -> np.ndarray:
    a = t.detach().cpu().numpy()
    if a.dtype == np.int64:
        return a.view(np.uint64)
    if a.dtype == np.int32:
        return a.view(np.uint32)
    return a


def from_numpy(a: np.ndarray, device="cuda") -> torch.Tensor:
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint64:
        a = a.view(np.int64)
    elif a.dtype == np.uint32:
        a = a.view(np.int32)
    return torch.from_numpy(a).to(device)


def status_string(status: int) -> str:
    return _lib.cstone_status_string(status).decode()


# ---- the six operations ------------------------------------------------------

def compute_keys(x, y, z, box, curve=HILBERT, keys=None, flags=None, stream=None) -> torch.Tensor:
    """SFC keys (int64 container of uint64) of FP64 device coordinates."""
    n = x.numel()
    for t in (x, y, z):
        _dev(t, torch.float64)
    if keys is None:
        keys = torch.empty(n, dtype=torch.int64, device=x.device)
    b = Box.of(box)
    _check(_lib.cstone_compute_keys(_ptr(x), _ptr(y), _ptr(z), n, ctypes.byref(b), int(curve), _ptr(keys),
                                    _ptr(flags), _stream(stream)), "cstone_compute_keys")
    return keys


def sort(keys, keys_out=None, perm_out=None, ws=None, stream=None):
    """Stable radix sort: (sorted keys, perm) with sorted[i] = keys[perm[i]]."""
    n = keys.numel()
    _dev(keys, torch.int64)
    if keys_out is None:
        keys_out = torch.empty(n, dtype=torch.int64, device=keys.device)
    if perm_out is None:
        perm_out = torch.empty(n, dtype=torch.int32, device=keys.device)
    need = _lib.cstone_sort_workspace_bytes(n)
    if ws is None:
        ws = _workspace(need, keys.device)
    _check(_lib.cstone_sort(_ptr(keys), _ptr(keys_out), _ptr(perm_out), n, _ptr(ws), ws.numel(), _stream(stream)),
           "cstone_sort")
    return keys_out, perm_out


def node_counts(sorted_keys, leaves, counts=None, stream=None) -> torch.Tensor:
    nl = leaves.numel() - 1
    if counts is None:
        counts = torch.empty(max(nl, 1), dtype=torch.int32, device=leaves.device)
    _check(_lib.cstone_node_counts(_ptr(sorted_keys), sorted_keys.numel(), _ptr(leaves), nl, _ptr(counts),
                                   _stream(stream)), "cstone_node_counts")
    return counts[:nl]


def leaf_capacity_bound(n: int, n_crit: int, n_leaves_start: int = 1) -> int:
    return int(_lib.cstone_leaf_capacity_bound(n, n_crit, n_leaves_start))


def node_count(n_leaves: int) -> int:
    return int(_lib.cstone_node_count(n_leaves))


def rebalance(sorted_keys, n_crit: int, leaves=None, capacity=None, max_iters: int = 0, ws=None, stream=None):
    """Iterate f and g from `leaves` (default: the root) to convergence.

    Returns (K, counts, rounds). Raises CstoneError on CAPACITY/NOT_CONVERGED
    (the error carries .leaves / .rounds of the last valid array)."""
    n = sorted_keys.numel()
    dev = sorted_keys.device
    nl0 = 1 if leaves is None else leaves.numel() - 1
    if capacity is None:
        capacity = leaf_capacity_bound(n, n_crit, nl0)
    buf = torch.empty(capacity + 1, dtype=torch.int64, device=dev)
    if leaves is not None:
        buf[: nl0 + 1].copy_(leaves)
    counts = torch.empty(capacity, dtype=torch.int32, device=dev)
    need = _lib.cstone_rebalance_workspace_bytes(n, int(n_crit), capacity)
    if ws is None:
        ws = _workspace(need, dev)
    nl = ctypes.c_size_t(nl0)
    rounds = ctypes.c_uint32(0)
    st = _lib.cstone_rebalance(_ptr(sorted_keys), n, int(n_crit), _ptr(buf), ctypes.byref(nl), capacity, _ptr(counts),
                               int(max_iters), ctypes.byref(rounds), _ptr(ws), ws.numel(), _stream(stream))
    if st != 0:
        err = CstoneError(st, "cstone_rebalance")
        err.n_leaves = nl.value
        err.rounds = rounds.value
        err.buffer = buf
        err.counts = counts
        raise err
    return buf[: nl.value + 1], counts[: nl.value], int(rounds.value)


def link_octree(leaves, node_keys=None, child=None, level_offsets=None, ws=None, stream=None, by_sort=False):
    """Fully linked octree of a cornerstone array: (NK, CO, LO). With
    by_sort=True the paper's literal five steps are used (same outputs)."""
    nl = leaves.numel() - 1
    n = node_count(nl)
    dev = leaves.device
    if node_keys is None:
        node_keys = torch.empty(n, dtype=torch.int64, device=dev)
    if child is None:
        child = torch.empty(n, dtype=torch.int32, device=dev)
    if level_offsets is None:
        level_offsets = torch.empty(LEVEL_OFFSETS, dtype=torch.int32, device=dev)
    need = _lib.cstone_link_workspace_bytes(nl)
    if ws is None:
        ws = _workspace(need, dev)
    fn = _lib.cstone_link_octree_by_sort if by_sort else _lib.cstone_link_octree
    _check(fn(_ptr(leaves), nl, _ptr(node_keys), _ptr(child), _ptr(level_offsets), _ptr(ws), ws.numel(),
              _stream(stream)), "cstone_link_octree")
    return node_keys[:n], child[:n], level_offsets


def radix_tree(keys, stream=None):
    """Binary radix tree over sorted unique keys: (first, last, split, prefix_len) per internal node."""
    m = keys.numel()
    k = max(m - 1, 1)
    out = [torch.empty(k, dtype=torch.int32, device=keys.device) for _ in range(4)]
    _check(_lib.cstone_radix_tree(_ptr(keys), m, *(_ptr(o) for o in out), _stream(stream)), "cstone_radix_tree")
    return tuple(o[: max(m - 1, 0)] for o in out)


def link_octree_radix(leaves, node_keys=None, child=None, level_offsets=None, ws=None, stream=None):
    """Linked octree through the binary radix tree (same outputs as link_octree)."""
    nl = leaves.numel() - 1
    n = node_count(nl)
    dev = leaves.device
    node_keys = torch.empty(n, dtype=torch.int64, device=dev) if node_keys is None else node_keys
    child = torch.empty(n, dtype=torch.int32, device=dev) if child is None else child
    level_offsets = torch.empty(LEVEL_OFFSETS, dtype=torch.int32, device=dev) if level_offsets is None else level_offsets
    if ws is None:
        ws = _workspace(_lib.cstone_link_octree_radix_workspace_bytes(nl), dev)
    _check(_lib.cstone_link_octree_radix(_ptr(leaves), nl, _ptr(node_keys), _ptr(child), _ptr(level_offsets),
                                         _ptr(ws), ws.numel(), _stream(stream)), "cstone_link_octree_radix")
    return node_keys[:n], child[:n], level_offsets


def compact_octree(leaves, counts, stream=None):
    """Octree over the non-empty leaves (empty buckets removed): (NK, parent, LO)."""
    nl = leaves.numel() - 1
    dev = leaves.device
    cap = 2 * nl + 1
    nk = torch.empty(cap, dtype=torch.int64, device=dev)
    par = torch.empty(cap, dtype=torch.int32, device=dev)
    lo = torch.empty(LEVEL_OFFSETS, dtype=torch.int32, device=dev)
    ws = _workspace(_lib.cstone_compact_octree_workspace_bytes(nl), dev)
    n = ctypes.c_size_t(0)
    _check(_lib.cstone_compact_octree(_ptr(leaves), _ptr(counts), nl, _ptr(nk), _ptr(par), _ptr(lo),
                                      ctypes.byref(n), _ptr(ws), ws.numel(), _stream(stream)), "cstone_compact_octree")
    return nk[: n.value], par[: n.value], lo


def octree_node_counts(leaves, counts, node_keys, out=None, ws=None, stream=None) -> torch.Tensor:
    """Particle count of every node of the linked octree over `leaves` (same
    order as node_keys)."""
    nl = leaves.numel() - 1
    n = node_keys.numel()
    if out is None:
        out = torch.empty(max(n, 1), dtype=torch.int32, device=leaves.device)
    if ws is None:
        ws = _workspace(_lib.cstone_octree_node_counts_workspace_bytes(nl), leaves.device)
    _check(_lib.cstone_octree_node_counts(_ptr(leaves), _ptr(counts), nl, _ptr(node_keys), n, _ptr(out), _ptr(ws),
                                          ws.numel(), _stream(stream)), "cstone_octree_node_counts")
    return out[:n]


def gather(src, perm, out=None, stream=None) -> torch.Tensor:
    """out[i] = src[perm[i]] (float64 device arrays)."""
    n = perm.numel()
    _dev(src, torch.float64)
    if out is None:
        out = torch.empty(n, dtype=torch.float64, device=src.device)
    _check(_lib.cstone_gather(_ptr(src), _ptr(perm), n, _ptr(out), _stream(stream)), "cstone_gather")
    return out


def gather_xyz(x, y, z, perm, out=None, fused: bool = False, stream=None):
    """(x, y, z) in curve order: each taken through perm."""
    n = perm.numel()
    for t in (x, y, z):
        _dev(t, torch.float64)
    if out is None:
        out = tuple(torch.empty(n, dtype=torch.float64, device=x.device) for _ in range(3))
    _check(_lib.cstone_gather_xyz(_ptr(x), _ptr(y), _ptr(z), _ptr(perm), n, *(_ptr(o) for o in out), int(fused),
                                  _stream(stream)), "cstone_gather_xyz")
    return out


def _offsets(shard_offsets):
    off = np.ascontiguousarray(shard_offsets, dtype=np.uint64)
    return off, off.ctypes.data_as(ctypes.c_void_p), off.size - 1


def build_sharded(x, y, z, shard_offsets, box, curve, n_crit: int, capacity=None, max_iters: int = 0, stream=None):
    """Sec. 6 on one device: particles split into shards at `shard_offsets`
    (n_shards + 1 ints), each shard's keys sorted on their own, the tree of all
    particles from per-shard counts summed every round. Returns (sorted keys
    per shard, perm per shard, K, summed counts, rounds)."""
    n = x.numel()
    for t in (x, y, z):
        _dev(t, torch.float64)
    off, off_p, G = _offsets(shard_offsets)
    dev = x.device
    if capacity is None:
        capacity = leaf_capacity_bound(n, n_crit)
    P = torch.empty(max(n, 1), dtype=torch.int64, device=dev)
    perm = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    K = torch.empty(capacity + 1, dtype=torch.int64, device=dev)
    K[:2].copy_(torch.tensor([0, -(1 << 63)], dtype=torch.int64))  # the root {0, 8^L}
    counts = torch.empty(capacity, dtype=torch.int32, device=dev)
    ws = _workspace(_lib.cstone_build_sharded_workspace_bytes(off_p, G, capacity), dev)
    nl = ctypes.c_size_t(1)
    rounds = ctypes.c_uint32(0)
    b = Box.of(box)
    _check(_lib.cstone_build_sharded(_ptr(x), _ptr(y), _ptr(z), off_p, G, ctypes.byref(b), int(curve), int(n_crit),
                                     _ptr(P), _ptr(perm), _ptr(K), ctypes.byref(nl), capacity, _ptr(counts),
                                     int(max_iters), ctypes.byref(rounds), _ptr(ws), ws.numel(), _stream(stream)),
           "cstone_build_sharded")
    return P[:n], perm[:n], K[: nl.value + 1], counts[: nl.value], int(rounds.value)


def global_rebalance(sorted_keys, shard_offsets, n_crit: int, leaves=None, capacity=None, max_iters: int = 0,
                     stream=None):
    """Tree of all shards' particles from their separately sorted keys (back to
    back at `shard_offsets`), from `leaves` (default the root). Returns (K,
    summed counts, rounds)."""
    n = sorted_keys.numel()
    off, off_p, G = _offsets(shard_offsets)
    dev = sorted_keys.device
    nl0 = 1 if leaves is None else leaves.numel() - 1
    if capacity is None:
        capacity = leaf_capacity_bound(n, n_crit, nl0)
    K = torch.empty(capacity + 1, dtype=torch.int64, device=dev)
    if leaves is None:
        K[:2].copy_(torch.tensor([0, -(1 << 63)], dtype=torch.int64))
    else:
        K[: nl0 + 1].copy_(leaves)
    counts = torch.empty(capacity, dtype=torch.int32, device=dev)
    ws = _workspace(_lib.cstone_global_rebalance_workspace_bytes(capacity, G), dev)
    nl = ctypes.c_size_t(nl0)
    rounds = ctypes.c_uint32(0)
    _check(_lib.cstone_global_rebalance(_ptr(sorted_keys), off_p, G, int(n_crit), _ptr(K), ctypes.byref(nl),
                                        capacity, _ptr(counts), int(max_iters), ctypes.byref(rounds), _ptr(ws),
                                        ws.numel(), _stream(stream)), "cstone_global_rebalance")
    return K[: nl.value + 1], counts[: nl.value], int(rounds.value)


def focus_rebalance(sorted_keys, n_crit: int, curve: int, focus_start: int, focus_end: int, theta: float,
                    leaves=None, capacity=None, max_iters: int = 0, stream=None):
    """Tree focused on the curve range [focus_start, focus_end) (Sec. 7), from
    `leaves` (default the root). Returns (K, counts, rounds)."""
    n = sorted_keys.numel()
    dev = sorted_keys.device
    nl0 = 1 if leaves is None else leaves.numel() - 1
    if capacity is None:
        capacity = leaf_capacity_bound(n, n_crit, nl0)
    K = torch.empty(capacity + 1, dtype=torch.int64, device=dev)
    if leaves is None:
        K[:2].copy_(torch.tensor([0, -(1 << 63)], dtype=torch.int64))
    else:
        K[: nl0 + 1].copy_(leaves)
    counts = torch.empty(capacity, dtype=torch.int32, device=dev)
    ws = _workspace(_lib.cstone_focus_rebalance_workspace_bytes(capacity), dev)
    nl = ctypes.c_size_t(nl0)
    rounds = ctypes.c_uint32(0)
    st = _lib.cstone_focus_rebalance(_ptr(sorted_keys), n, int(n_crit), int(curve), int(focus_start), int(focus_end),
                                     float(theta), _ptr(K), ctypes.byref(nl), capacity, _ptr(counts), int(max_iters),
                                     ctypes.byref(rounds), _ptr(ws), ws.numel(), _stream(stream))
    if st != 0:
        err = CstoneError(st, "cstone_focus_rebalance")
        err.n_leaves = nl.value
        raise err
    return K[: nl.value + 1], counts[: nl.value], int(rounds.value)


def focus_mac(node_keys, curve: int, focus_start: int, focus_end: int, theta: float, stream=None) -> torch.Tensor:
    """f^LE_2: 1 where a node of the linked octree fails the MAC against F (uint8)."""
    n = node_keys.numel()
    out = torch.empty(max(n, 1), dtype=torch.uint8, device=node_keys.device)
    ws = _workspace(_lib.cstone_focus_mac_workspace_bytes(), node_keys.device)
    _check(_lib.cstone_focus_mac(_ptr(node_keys), n, int(curve), int(focus_start), int(focus_end), float(theta),
                                 _ptr(out), _ptr(ws), ws.numel(), _stream(stream)), "cstone_focus_mac")
    return out[:n]


def sfc_partition(counts, n_ranks: int, bounds=None, stream=None) -> torch.Tensor:
    """Bounds (n_ranks + 1) of n_ranks bins of consecutive leaves with about
    N / n_ranks particles each (Sec. 6)."""
    nl = counts.numel()
    if bounds is None:
        bounds = torch.empty(int(n_ranks) + 1, dtype=torch.int32, device=counts.device)
    ws = _workspace(_lib.cstone_sfc_partition_workspace_bytes(nl), counts.device)
    _check(_lib.cstone_sfc_partition(_ptr(counts), nl, int(n_ranks), _ptr(bounds), _ptr(ws), ws.numel(),
                                     _stream(stream)), "cstone_sfc_partition")
    return bounds


# ---- whole build with preallocated buffers ----------------------------------------

class BuildResult:
    """Outputs of one build: views into the Builder's buffers (valid until its
    next build). The views are made on first access, so a caller that only
    needs some of them pays for none of the others."""

    __slots__ = ("_b", "n", "n_leaves", "rounds", "stage_ms", "sort_pass_ms")

    def __init__(self, builder, n, n_leaves, rounds, stage_ms=(), sort_pass_ms=()):
        self._b = builder
        self.n = n
        self.n_leaves = n_leaves
        self.rounds = rounds
        self.stage_ms = stage_ms          # keys, sort, rebalance, link (timed builds only)
        self.sort_pass_ms = sort_pass_ms  # top passes, bucket pass, low passes of the particle sort (timed builds only)

    @property
    def sorted_keys(self):
        return self._b.sorted_keys[: self.n]

    @property
    def perm(self):
        return self._b.perm[: self.n]

    @property
    def leaves(self):
        return self._b.leaves[: self.n_leaves + 1]

    @property
    def counts(self):
        return self._b.counts[: self.n_leaves]

    @property
    def node_keys(self):
        return self._b.node_keys[: node_count(self.n_leaves)] if self._b.link else None

    @property
    def child(self):
        return self._b.child[: node_count(self.n_leaves)] if self._b.link else None

    @property
    def level_offsets(self):
        return self._b.level_offsets if self._b.link else None


class Builder:
    """Holds every buffer of a build of up to `n_max` particles so repeated
    builds allocate nothing (the library itself never allocates)."""

    def __init__(self, n_max: int, n_crit_min: int = 1, leaf_capacity: int | None = None, device="cuda",
                 link: bool = True):
        self.device = torch.device(device)
        self.n_max = int(n_max)
        cap = leaf_capacity or leaf_capacity_bound(self.n_max, n_crit_min)
        self.capacity = int(cap)
        dev = self.device
        self.sorted_keys = torch.empty(max(self.n_max, 1), dtype=torch.int64, device=dev)
        self.perm = torch.empty(max(self.n_max, 1), dtype=torch.int32, device=dev)
        self.leaves = torch.empty(self.capacity + 1, dtype=torch.int64, device=dev)
        self.counts = torch.empty(self.capacity, dtype=torch.int32, device=dev)
        self.link = link
        nn = node_count(self.capacity)
        self.node_keys = torch.empty(nn, dtype=torch.int64, device=dev) if link else None
        self.child = torch.empty(nn, dtype=torch.int32, device=dev) if link else None
        self.level_offsets = torch.empty(LEVEL_OFFSETS, dtype=torch.int32, device=dev) if link else None
        self.ws = _workspace(_lib.cstone_build_workspace_bytes(self.n_max, self.capacity), dev)
        self.n_leaves = 0
        # pointers of the fixed buffers, marshalled once
        self._out = (_ptr(self.sorted_keys), _ptr(self.perm), _ptr(self.leaves))
        self._out2 = (_ptr(self.counts), _ptr(self.node_keys), _ptr(self.child), _ptr(self.level_offsets))
        self._ws = (_ptr(self.ws), self.ws.numel())
        self._boxes = {}
        self._nl = ctypes.c_size_t(0)
        self._rounds = ctypes.c_uint32(0)

    def build(self, x, y, z, box, curve, n_crit: int, incremental: bool = False, max_iters: int = 0,
              timed: bool = False, stream=None) -> BuildResult:
        n = x.numel()
        assert n <= self.n_max
        for t in (x, y, z):
            _dev(t, torch.float64)
        key = (tuple(box[0]), tuple(box[1]))
        b = self._boxes.get(key)
        if b is None:
            b = self._boxes[key] = Box.of(box)
        self._nl.value = self.n_leaves if incremental else 0
        tm = Timings() if timed else None
        st = _lib.cstone_build(x.data_ptr(), y.data_ptr(), z.data_ptr(), n, ctypes.byref(b), int(curve), int(n_crit),
                               *self._out, ctypes.byref(self._nl), self.capacity, *self._out2, int(max_iters),
                               ctypes.byref(self._rounds), *self._ws, ctypes.byref(tm) if timed else None,
                               _stream(stream))
        if st != 0:
            err = CstoneError(st, "cstone_build")
            err.n_leaves = self._nl.value
            raise err
        self.n_leaves = self._nl.value
        return BuildResult(self, n, self._nl.value, int(self._rounds.value),
                           tuple(tm.stage_ms) if timed else (),
                           tuple(tm.sort_pass_ms[: tm.sort_passes]) if timed else ())


def build(x, y, z, box, curve=HILBERT, n_crit: int = 64, link: bool = True) -> BuildResult:
    """One-shot build (allocates a Builder sized for this set)."""
    return Builder(x.numel(), n_crit, device=x.device, link=link).build(x, y, z, box, curve, n_crit)


# ---- sort shapes and their autotuner ------------------------------------------------

def sort_variants() -> list:
    """(digit bits, block, items per thread) of every compiled sort shape."""
    out = []
    for v in range(_lib.cstone_sort_variant_count()):
        b, bl, it = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(_lib.cstone_sort_variant_info(v, ctypes.byref(b), ctypes.byref(bl), ctypes.byref(it)),
               "cstone_sort_variant_info")
        out.append((b.value, bl.value, it.value))
    return out


def set_lookback_patience(waits: int):
    """Look-back waits before a sort block counts a missing predecessor
    tile's digits itself (default 256; 0 sends every wait to that fallback).
    Applies to later launches on the current device."""
    _check(_lib.cstone_set_lookback_patience(int(waits)), "cstone_set_lookback_patience")


def sort_variant_splits() -> list:
    """Whether each compiled sort shape takes the split sort (1) or plain LSD
    passes (0) for particle keys."""
    out = []
    for v in range(_lib.cstone_sort_variant_count()):
        sp = ctypes.c_int()
        _check(_lib.cstone_sort_variant_split(v, ctypes.byref(sp)), "cstone_sort_variant_split")
        out.append(sp.value)
    return out


def sort_autotune(keys, reps: int = 3, stream=None):
    """Time every sort shape on `keys` and record the fastest in the autotune
    table for sorts of this size class on this device. Returns (chosen index,
    ms per shape)."""
    n = keys.numel()
    _dev(keys, torch.int64)
    out = torch.empty_like(keys)
    perm = torch.empty(n, dtype=torch.int32, device=keys.device)
    ws = _workspace(_lib.cstone_sort_workspace_bytes(n), keys.device)
    nv = _lib.cstone_sort_variant_count()
    ms = (ctypes.c_float * nv)()
    chosen = ctypes.c_int(-1)
    _check(_lib.cstone_sort_autotune(_ptr(keys), n, _ptr(out), _ptr(perm), _ptr(ws), ws.numel(), int(reps), ms,
                                     ctypes.byref(chosen), _stream(stream)), "cstone_sort_autotune")
    return chosen.value, list(ms)


TUNE_SORT, TUNE_BATCH_SORT = 0, 1


def tune_set(kernel: int, n: int, variant: int):
    """Record `variant` for (kernel, size class of n, current device); -1 removes the entry."""
    _check(_lib.cstone_tune_set(int(kernel), int(n), int(variant)), "cstone_tune_set")


def tune_get(kernel: int, n: int) -> int:
    return int(_lib.cstone_tune_get(int(kernel), int(n)))


def tune_clear():
    _lib.cstone_tune_clear()


def tune_entries() -> int:
    return int(_lib.cstone_tune_entries())


def tune_save(path: str):
    _check(_lib.cstone_tune_save(os.fsencode(path)), "cstone_tune_save")


def tune_load(path: str):
    _check(_lib.cstone_tune_load(os.fsencode(path)), "cstone_tune_load")


# ---- batched builds -------------------------------------------------------------------

SET_RESULT_FIELDS = ("n_leaves", "n_nodes", "rounds", "status")


class BatchArena:
    """Device buffers for batched builds, reusable across plans: a batch takes
    views of the first elements it needs. `need` gives the element counts of
    a plan: particles, leaf slots, node slots, sets, workspace bytes."""

    _GROUPS = (("sorted_keys", "perm"), ("leaves", "counts"), ("node_keys", "child"), ("level_offsets", "results"),
               ("ws",))

    def __init__(self, device, need):
        self.device = torch.device(device)
        self.cap = (0, 0, 0, 0, 0)
        self.grow(need)

    def _alloc(self, group: int, c: int):
        dev = self.device
        if group == 0:
            self.sorted_keys = torch.empty(c, dtype=torch.int64, device=dev)
            self.perm = torch.empty(c, dtype=torch.int32, device=dev)
        elif group == 1:
            self.leaves = torch.empty(c, dtype=torch.int64, device=dev)
            self.counts = torch.empty(c, dtype=torch.int32, device=dev)
        elif group == 2:
            self.node_keys = torch.empty(c, dtype=torch.int64, device=dev)
            self.child = torch.empty(c, dtype=torch.int32, device=dev)
        elif group == 3:
            self.level_offsets = torch.empty(c * LEVEL_OFFSETS, dtype=torch.int32, device=dev)
            self.results = torch.empty(c * 4, dtype=torch.int32, device=dev)
        else:
            self.ws = _workspace(c, dev)

    def grow(self, want):
        """Make every buffer hold at least `want` (same order as a need):
        only the buffers that are too small are reallocated (their contents
        are not kept)."""
        caps = list(self.cap)
        for g, v in enumerate(want):
            v = max(int(v), 256 if g == 4 else 1)
            if v > caps[g]:
                for name in self._GROUPS[g]:  # free first, so the old and new buffers are not held together
                    setattr(self, name, None)
                self._alloc(g, v)
                caps[g] = v
        self.cap = tuple(caps)

    @staticmethod
    def need(layout) -> tuple:
        return (int(layout.n_particles), int(layout.leaf_slots), int(layout.node_slots), int(layout.n_sets),
                int(layout.workspace_bytes))

    @staticmethod
    def bytes_of(need) -> int:
        n, leaf, node, sets, ws = (max(int(v), 1) for v in need)
        return 12 * n + 12 * leaf + 12 * node + sets * (4 * LEVEL_OFFSETS + 16) + max(ws, 256)

    @property
    def nbytes(self) -> int:
        return self.bytes_of(self.cap)

    def fits(self, need) -> bool:
        return all(max(int(v), 1) <= c for v, c in zip(need, self.cap))

    def views(self, need):
        n, leaf, node, sets, ws = (max(int(v), 1) for v in need)
        return (self.sorted_keys[:n], self.perm[:n], self.leaves[:leaf], self.counts[:leaf], self.node_keys[:node],
                self.child[:node], self.level_offsets[:sets * LEVEL_OFFSETS], self.results[:sets * 4],
                self.ws[:max(ws, 256)])


def batch_layout(sets) -> BatchLayout:
    """The layout a Batch of these sets would have (host-side plan only)."""
    arr = (CSet * max(len(sets), 1))()
    for i, spec in enumerate(sets):
        n, box, curve, n_crit = spec[:4]
        cap = spec[4] if len(spec) > 4 else 0
        arr[i] = CSet(int(n), Box.of(box), int(curve), int(n_crit), int(cap))
    plan = ctypes.c_void_p()
    _check(_lib.cstone_batch_create(arr, len(sets), ctypes.byref(plan)), "cstone_batch_create")
    try:
        lay = BatchLayout()
        _check(_lib.cstone_batch_get_layout(plan, ctypes.byref(lay), None, None, None), "cstone_batch_get_layout")
    finally:
        _lib.cstone_batch_destroy(plan)
    return lay


class Batch:
    """A planned batch of independent particle sets and every device buffer
    its build needs (allocated once here; building allocates nothing).

    `sets` is a sequence of (n, box, curve, n_crit) or (n, box, curve, n_crit,
    leaf_capacity). Particles of set s are x[po[s]:po[s+1]] (po =
    self.particle_offsets); build() enqueues the whole batch, capture() records
    it into a hipGraph that launch() replays."""

    def __init__(self, sets, device="cuda", arena=None, stage=None):
        """arena: optional BatchArena whose buffers this batch uses (views)
        instead of allocating its own, or a callable that takes the plan's
        needs (BatchArena.need) and returns such an arena large enough.
        stage: optional callable that takes the tables' size in bytes and
        returns a pinned uint8 host tensor at least that large; the tables
        then go up asynchronously through it (see upload)."""
        self.device = torch.device(device)
        arr = (CSet * max(len(sets), 1))()
        for i, spec in enumerate(sets):
            n, box, curve, n_crit = spec[:4]
            cap = spec[4] if len(spec) > 4 else 0
            arr[i] = CSet(int(n), Box.of(box), int(curve), int(n_crit), int(cap))
        self.n_sets = len(sets)
        plan = ctypes.c_void_p()
        _check(_lib.cstone_batch_create(arr, self.n_sets, ctypes.byref(plan)), "cstone_batch_create")
        self._plan = plan
        self._refresh_layout()
        lay = self.layout
        dev = self.device
        need = BatchArena.need(lay)
        if callable(arena):
            arena = arena(need)
        if arena is not None:
            assert arena.fits(need), "the arena is smaller than this batch"
            views = arena.views(need)
        else:
            views = BatchArena(dev, need).views(need)
        (self.sorted_keys, self.perm, self.leaves, self.counts, self.node_keys, self.child, self.level_offsets,
         self.results, self.ws) = views
        self.results.zero_()  # (a reused arena holds an earlier batch's results)
        self.upload(stage=stage(self.table_bytes) if stage is not None else None)

    def _refresh_layout(self):
        lay = BatchLayout()
        k = self.n_sets + 1
        po, lo, no = (ctypes.c_uint64 * k)(), (ctypes.c_uint64 * k)(), (ctypes.c_uint64 * k)()
        _check(_lib.cstone_batch_get_layout(self._plan, ctypes.byref(lay), po, lo, no), "cstone_batch_get_layout")
        self.layout = lay
        self.particle_offsets = np.frombuffer(po, dtype=np.uint64).astype(np.int64)
        self.leaf_offsets = np.frombuffer(lo, dtype=np.uint64).astype(np.int64)
        self.node_offsets = np.frombuffer(no, dtype=np.uint64).astype(np.int64)

    def __del__(self):
        plan = getattr(self, "_plan", None)
        if plan is not None and plan.value and _lib is not None:  # (None once the interpreter is shutting down)
            _lib.cstone_batch_destroy(plan)
            self._plan = None

    @property
    def n_particles(self) -> int:
        return int(self.layout.n_particles)

    @property
    def sort_variant(self) -> int:
        return int(self.layout.sort_variant)

    def set_variant(self, variant: int, stream=None):
        _check(_lib.cstone_batch_set_variant(self._plan, int(variant)), "cstone_batch_set_variant")
        self._refresh_layout()
        self.upload(stream)

    def set_rounds(self, rounds: int):
        """Rebalance rounds enqueued per build (1..22; a set that needs more
        reports NOT_CONVERGED)."""
        _check(_lib.cstone_batch_set_rounds(self._plan, int(rounds)), "cstone_batch_set_rounds")
        self._refresh_layout()

    def upload(self, stream=None, stage=None):
        """Copy the plan's tables into the workspace. With `stage` (a pinned
        uint8 host tensor of at least table_bytes) the copy is asynchronous on
        the stream, and the stage must stay unchanged until the stream has
        passed it; without, the call synchronises the stream."""
        if stage is None:
            _check(_lib.cstone_batch_upload(self._plan, _ptr(self.ws), self.ws.numel(), _stream(stream)),
                   "cstone_batch_upload")
            return
        assert stage.is_pinned() and stage.dtype == torch.uint8
        _check(_lib.cstone_batch_upload_staged(self._plan, _ptr(self.ws), self.ws.numel(), _ptr(stage), stage.numel(),
                                               _stream(stream)), "cstone_batch_upload_staged")

    @property
    def table_bytes(self) -> int:
        return int(_lib.cstone_batch_table_bytes(self._plan))

    def _args(self, x, y, z):
        for t in (x, y, z):
            _dev(t, torch.float64)
            assert t.numel() >= self.n_particles
        return [_ptr(x), _ptr(y), _ptr(z), _ptr(self.sorted_keys), _ptr(self.perm), _ptr(self.leaves),
                _ptr(self.counts), _ptr(self.node_keys), _ptr(self.child), _ptr(self.level_offsets),
                _ptr(self.results), _ptr(self.ws), self.ws.numel()]

    def build(self, x, y, z, stream=None):
        """Enqueue the batched build (asynchronous)."""
        _check(_lib.cstone_batch_build(self._plan, *self._args(x, y, z), _stream(stream)), "cstone_batch_build")

    def capture(self, x, y, z, stream):
        """Record the build with these inputs into a hipGraph (stream: a torch.cuda.Stream)."""
        _check(_lib.cstone_batch_capture(self._plan, *self._args(x, y, z), _stream(stream)), "cstone_batch_capture")

    def launch(self, stream=None):
        _check(_lib.cstone_batch_launch(self._plan, _stream(stream)), "cstone_batch_launch")

    def autotune(self, x, y, z, reps: int = 3, stream=None):
        """Time every sort shape on this batch, keep the fastest (also recorded
        in the autotune table for batches of this size); returns ms per shape."""
        nv = _lib.cstone_sort_variant_count()
        ms = (ctypes.c_float * nv)()
        _check(_lib.cstone_batch_autotune(self._plan, *self._args(x, y, z), int(reps), ms, _stream(stream)),
               "cstone_batch_autotune")
        self._refresh_layout()
        return list(ms)

    def set_results(self) -> np.ndarray:
        """(n_sets, 4) uint32: n_leaves, n_nodes, rounds, status of every set (synchronises)."""
        return to_numpy(self.results[: 4 * self.n_sets]).reshape(self.n_sets, 4)

    def set_view(self, s: int, res=None) -> dict:
        """Device views of set s's outputs (after the build has finished)."""
        if res is None:
            res = self.set_results()[s]
        nl, nn = int(res[0]), int(res[1])
        p0, p1 = int(self.particle_offsets[s]), int(self.particle_offsets[s + 1])
        l0, n0 = int(self.leaf_offsets[s]), int(self.node_offsets[s])
        return {
            "sorted_keys": self.sorted_keys[p0:p1], "perm": self.perm[p0:p1],
            "leaves": self.leaves[l0:l0 + nl + 1], "counts": self.counts[l0:l0 + nl],
            "node_keys": self.node_keys[n0:n0 + nn], "child": self.child[n0:n0 + nn],
            "level_offsets": self.level_offsets[s * LEVEL_OFFSETS:(s + 1) * LEVEL_OFFSETS],
            "n_leaves": nl, "n_nodes": nn, "rounds": int(res[2]), "status": STATUS.get(int(res[3]), int(res[3])),
        }
