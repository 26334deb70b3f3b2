"""The C-ABI library loads on the host and exports every entry point that
include/cstone.h declares; host-only queries answer without a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cstone.h")
LIB = os.path.join(ROOT, "paper_2307_06345_amd", "libcstone.so")


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"CSTONE_API\s+[\w\s\*]*?\b(cstone_\w+)\s*\(", text)))


def test_header_declares_the_six_operations():
    names = declared_symbols()
    for op in ("compute_keys", "sort", "node_counts", "rebalance", "link_octree", "build"):
        assert f"cstone_{op}" in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "run __graft_entry__.build() first"
    lib = ctypes.CDLL(LIB)
    for name in declared_symbols():
        assert hasattr(lib, name), name


def test_library_exports_nothing_else():
    import subprocess
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = sorted(l.split()[-1] for l in out.splitlines() if " T " in l)
    assert exported == declared_symbols()


def test_host_queries():
    import paper_2307_06345_amd as cs
    assert cs.status_string(0) == "ok"
    assert cs.node_count(1) == 1 and cs.node_count(15) == 17 and cs.node_count(64) == 73
    # 7 * 21 * floor(n / (n_crit + 1)) + 1
    assert cs.leaf_capacity_bound(1 << 16, 64) == 7 * 21 * ((1 << 16) // 65) + 1
    assert cs.leaf_capacity_bound(10, 64) == 1
    lib = cs._lib
    assert lib.cstone_sort_workspace_bytes(1 << 20) >= 12 * (1 << 20)
    assert lib.cstone_build_workspace_bytes(1000, 100) >= lib.cstone_sort_workspace_bytes(1000)


def test_invalid_arguments_are_rejected_without_a_device():
    import paper_2307_06345_amd as cs
    lib = cs._lib
    box = cs.Box.of(((0, 0, 0), (1, 1, 1)))
    bad = cs.Box.of(((0, 0, 0), (1, 0, 1)))
    # n > 0 with null pointers, a degenerate box, an unknown curve
    assert lib.cstone_compute_keys(None, None, None, 5, ctypes.byref(box), 0, None, None, None) == 1
    assert lib.cstone_compute_keys(None, None, None, 0, ctypes.byref(bad), 0, None, None, None) == 1
    assert lib.cstone_compute_keys(None, None, None, 0, ctypes.byref(box), 7, None, None, None) == 1
    # link: n_leaves - 1 must be a multiple of 7
    assert lib.cstone_link_octree(ctypes.c_void_p(8), 5, ctypes.c_void_p(8), ctypes.c_void_p(8),
                                  ctypes.c_void_p(8), ctypes.c_void_p(8), 1 << 20, None) == 1
    # rebalance: n_crit == 0
    nl = ctypes.c_size_t(1)
    assert lib.cstone_rebalance(ctypes.c_void_p(8), 10, 0, ctypes.c_void_p(8), ctypes.byref(nl), 10, None, 0, None,
                                ctypes.c_void_p(8), 1 << 20, None) == 1


def _plan(cs, specs):
    arr = (cs.CSet * max(len(specs), 1))()
    for i, (n, box, curve, n_crit, cap) in enumerate(specs):
        arr[i] = cs.CSet(n, cs.Box.of(box), curve, n_crit, cap)
    plan = ctypes.c_void_p()
    st = cs._lib.cstone_batch_create(arr, len(specs), ctypes.byref(plan))
    return st, plan


def test_batch_plan_layout_on_the_host():
    """The batch plan is host-only: offsets are prefix sums of the sizes and
    of the per-set capacities, tiles never straddle two sets."""
    import paper_2307_06345_amd as cs
    unit = ((0, 0, 0), (1, 1, 1))
    specs = [(0, unit, 0, 8, 0), (1000, unit, 1, 16, 0), (8192, unit, 0, 64, 500), (8193, unit, 1, 1, 0)]
    st, plan = _plan(cs, specs)
    assert st == 0
    try:
        lay = cs.BatchLayout()
        k = len(specs) + 1
        po, lo, no = (ctypes.c_uint64 * k)(), (ctypes.c_uint64 * k)(), (ctypes.c_uint64 * k)()
        assert cs._lib.cstone_batch_get_layout(plan, ctypes.byref(lay), po, lo, no) == 0
        ns = [s[0] for s in specs]
        caps = [s[4] or cs.leaf_capacity_bound(s[0], s[3]) for s in specs]
        assert list(po) == [0, 0, 1000, 9192, 17385]
        assert list(lo) == [0] + list(__import__("itertools").accumulate(c + 1 for c in caps))
        assert list(no) == [0] + list(__import__("itertools").accumulate(c + (c - 1) // 7 for c in caps))
        assert lay.n_sets == 4 and lay.n_particles == sum(ns)
        assert lay.leaf_slots == lo[-1] and lay.node_slots == no[-1]
        for v in range(cs._lib.cstone_sort_variant_count()):
            bits, block, items = cs.sort_variants()[v]
            assert cs._lib.cstone_batch_set_variant(plan, v) == 0
            assert cs._lib.cstone_batch_get_layout(plan, ctypes.byref(lay), None, None, None) == 0
            tile = block * items
            assert lay.n_tiles == sum((n + tile - 1) // tile for n in ns)
            assert lay.sort_variant == v
            assert lay.workspace_bytes >= 8 * sum(ns)
    finally:
        cs._lib.cstone_batch_destroy(plan)


def test_batch_staged_upload_checks_its_stage_on_the_host():
    """The tables' size is a host query, and a staged upload with no stage, or
    one smaller than the tables, is refused before any device call."""
    import numpy as np

    import paper_2307_06345_amd as cs
    unit = ((0, 0, 0), (1, 1, 1))
    specs = [(1000, unit, 0, 8, 0), (8192, unit, 1, 64, 0), (3, unit, 1, 1, 0)]
    st, plan = _plan(cs, specs)
    assert st == 0
    try:
        need = int(cs._lib.cstone_batch_table_bytes(plan))
        assert need >= 3 * 4  # at least the sets' bases
        lay = cs.BatchLayout()
        assert cs._lib.cstone_batch_get_layout(plan, ctypes.byref(lay), None, None, None) == 0
        assert need <= lay.workspace_bytes
        small = np.zeros(max(need - 1, 1), dtype=np.uint8)
        fake_ws = ctypes.c_void_p(1 << 40)  # never touched: the checks come first
        assert cs._lib.cstone_batch_upload_staged(plan, fake_ws, lay.workspace_bytes, None, need, None) == 1
        assert cs._lib.cstone_batch_upload_staged(plan, fake_ws, lay.workspace_bytes,
                                                  small.ctypes.data_as(ctypes.c_void_p), small.size, None) == 1
        assert cs._lib.cstone_batch_upload_staged(plan, fake_ws, lay.workspace_bytes - 1,
                                                  small.ctypes.data_as(ctypes.c_void_p), need, None) == 1
        assert cs._lib.cstone_batch_table_bytes(None) == 0
    finally:
        cs._lib.cstone_batch_destroy(plan)


def test_batch_plan_rejects_bad_sets():
    import paper_2307_06345_amd as cs
    unit = ((0, 0, 0), (1, 1, 1))
    for bad in [(10, unit, 0, 0, 0),                       # N_crit 0
                (10, ((0, 0, 0), (1, 0, 1)), 0, 8, 0),     # empty box
                (10, unit, 7, 8, 0),                       # unknown curve
                (1 << 32, unit, 0, 8, 0)]:                 # too many particles
        st, plan = _plan(cs, [bad])
        assert st == 1 and not plan.value, bad
    assert cs._lib.cstone_batch_launch(None, None) == 1


def test_tune_table_round_trips_through_its_json_file(tmp_path):
    """The autotune table: set, look up, save as JSON, clear, load back. Host
    only (without a GPU the device key is "unknown", the same on both sides)."""
    import json

    import paper_2307_06345_amd as cs
    nv = len(cs.sort_variants())
    cs.tune_clear()
    try:
        cs.tune_set(cs.TUNE_SORT, 1 << 24, nv - 1)
        cs.tune_set(cs.TUNE_BATCH_SORT, 77_000_000, 1)
        cs.tune_set(cs.TUNE_SORT, (1 << 25) - 1, 2)  # same size class as 2^24: replaces the entry
        assert cs.tune_entries() == 2
        assert cs.tune_get(cs.TUNE_SORT, 1 << 24) == 2
        assert cs.tune_get(cs.TUNE_SORT, 1 << 25) == -1
        assert cs.tune_get(cs.TUNE_BATCH_SORT, 70_000_000) == 1
        path = str(tmp_path / "tune.json")
        cs.tune_save(path)
        doc = json.load(open(path))
        assert doc["format"] == "cstone-tune-2" and len(doc["entries"]) == 2
        e = {x["kernel"]: x for x in doc["entries"]}
        assert e["sort"]["size_log2"] == 24 and e["sort"]["variant"] == 2
        assert (e["sort"]["digit_bits"], e["sort"]["block"], e["sort"]["items"]) == cs.sort_variants()[2]
        assert e["sort"]["split"] == cs.sort_variant_splits()[2]
        assert e["batch_sort"]["size_log2"] == 26
        cs.tune_clear()
        assert cs.tune_entries() == 0 and cs.tune_get(cs.TUNE_SORT, 1 << 24) == -1
        cs.tune_load(path)
        assert cs.tune_entries() == 2
        assert cs.tune_get(cs.TUNE_SORT, 1 << 24) == 2 and cs.tune_get(cs.TUNE_BATCH_SORT, 1 << 26) == 1
        cs.tune_set(cs.TUNE_SORT, 1 << 24, -1)  # removes the entry
        assert cs.tune_entries() == 1 and cs.tune_get(cs.TUNE_SORT, 1 << 24) == -1
        # an entry naming a shape this library does not have under that index is skipped
        doc["entries"][0]["block"] = 12345
        with open(path, "w") as f:
            f.write('{"format": "cstone-tune-2", "entries": [\n')
            f.write(",\n".join(json.dumps(x) for x in doc["entries"]) + "\n]}\n")
        cs.tune_clear()
        cs.tune_load(path)
        assert cs.tune_entries() == 1
        # a file in another format is refused and leaves the table unchanged
        bad = tmp_path / "bad.json"
        bad.write_text('{"entries": []}\n')
        with pytest.raises(cs.CstoneError):
            cs.tune_load(str(bad))
        assert cs.tune_entries() == 1
        with pytest.raises(cs.CstoneError):
            cs.tune_set(cs.TUNE_SORT, 10, nv)
    finally:
        cs.tune_clear()
