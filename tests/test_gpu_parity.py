"""GPU parity: every stage of the HIP path, called through the C ABI, against
the CPU oracle on the same seeded inputs. Integer outputs must match bit for
bit (keys, permutation, leaves, counts, NK, CO, LO). Sizes span several tiles
with ragged tails; edge cases cover empty input, one particle, duplicates,
non-finite coordinates and the degenerate trees."""
import numpy as np
import pytest
import torch

import oracle
import workloads as wl
from tests import invariants as inv

pytestmark = pytest.mark.gpu

cs = pytest.importorskip("paper_2307_06345_amd")

END = 1 << 63


def say(*a):
    print("[case]", *a, flush=True)


def dev(a):
    return cs.from_numpy(a, "cuda")


def host(t):
    return cs.to_numpy(t)


def eq(a, b, what):
    a = np.asarray(a)
    b = np.asarray(b)
    assert a.shape == b.shape, (what, a.shape, b.shape)
    bad = np.nonzero(a != b)[0]
    assert bad.size == 0, f"{what}: {bad.size} mismatches, first at {bad[:5]}: {a[bad[:5]]} vs {b[bad[:5]]}"


def coords(s):
    return dev(s.x), dev(s.y), dev(s.z)


# ---- keys ------------------------------------------------------------------

@pytest.mark.parametrize("curve", [wl.MORTON, wl.HILBERT])
@pytest.mark.parametrize("kind,n", [("uniform", 1), ("uniform", 1000), ("uniform", 200003), ("plummer", 150001)])
def test_keys_parity(curve, kind, n):
    s = wl.make_set(kind, n, 7, 0, curve, 16)
    say("keys", kind, n, "curve", curve)
    flags = torch.zeros(1, dtype=torch.int32, device="cuda")
    k = cs.compute_keys(*coords(s), s.box, curve, flags=flags)
    torch.cuda.synchronize()
    ref, bad = oracle.compute_keys(s.x, s.y, s.z, s.box, curve)
    eq(host(k), ref, "keys")
    assert not bad and int(flags.item()) == 0


def test_keys_edges_and_nonfinite():
    box = ((-1.0, 0.0, 2.0), (1.0, 4.0, 3.0))
    x = np.array([-1.0, 1.0, -5.0, 7.0, np.nextafter(1.0, -2), 0.0, np.nan, np.inf, -np.inf, 0.3])
    y = np.array([0.0, 4.0, -1.0, 9.0, 2.0, 2.0, 1.0, 1.0, 1.0, 3.9999999999])
    z = np.array([2.0, 3.0, 1.0, 4.0, 2.5, 2.5, 2.5, 2.5, 2.5, 2.0000000001])
    for curve in (wl.MORTON, wl.HILBERT):
        say("keys edges curve", curve)
        flags = torch.zeros(1, dtype=torch.int32, device="cuda")
        k = cs.compute_keys(dev(x), dev(y), dev(z), box, curve, flags=flags)
        torch.cuda.synchronize()
        ref, bad = oracle.compute_keys(x, y, z, box, curve)
        eq(host(k), ref, "keys")
        assert bad and int(flags.item()) == cs.FLAG_NONFINITE


def test_keys_exhaustive_coarse_grid():
    # every cell centre of a 64^3 grid: all 2^18 top-level key prefixes
    g = (np.arange(64) + 0.5) / 64
    x, y, z = (a.ravel() for a in np.meshgrid(g, g, g, indexing="ij"))
    for curve in (wl.MORTON, wl.HILBERT):
        say("keys 64^3 grid curve", curve)
        k = cs.compute_keys(dev(x), dev(y), dev(z), wl.UNIT_BOX, curve)
        ref, _ = oracle.compute_keys(x, y, z, wl.UNIT_BOX, curve)
        eq(host(k), ref, "keys")


# ---- sort ------------------------------------------------------------------

def _keys(kind, n, rng):
    if kind == "uniform":
        return rng.integers(0, END, n, dtype=np.uint64)
    if kind == "dups":
        return rng.integers(0, 50, n).astype(np.uint64) * np.uint64(0x0123456789ABCD)
    if kind == "equal":
        return np.full(n, 0x5555, np.uint64)
    if kind == "sorted":
        return np.sort(rng.integers(0, END, n, dtype=np.uint64))
    if kind == "reversed":
        return np.sort(rng.integers(0, END, n, dtype=np.uint64))[::-1].copy()
    if kind == "clustered":  # a few hundred level-9 prefixes: buckets of hundreds of keys, all low bits varying
        pre = rng.choice(1 << 27, 300, replace=False).astype(np.uint64)
        return (rng.choice(pre, n) << np.uint64(36)) | rng.integers(0, 1 << 36, n, dtype=np.uint64)
    if kind == "mixed":  # bucket sizes from 1 to beyond one block's window, with repeated low bits
        sizes = np.minimum((rng.pareto(0.8, n) * 40).astype(np.int64) + 1, 30000)
        sizes = sizes[: int(np.searchsorted(np.cumsum(sizes), n)) + 1]
        pre = np.sort(rng.choice(1 << 27, sizes.size, replace=False)).astype(np.uint64)
        prefix = np.repeat(pre, sizes)[:n]
        low = rng.integers(0, 1 << 36, n, dtype=np.uint64) >> np.uint64(rng.integers(0, 37))
        keys = (prefix << np.uint64(36)) | (low & np.uint64((1 << 36) - 1))
        return keys[rng.permutation(n)]
    raise ValueError(kind)


@pytest.mark.parametrize("kind,n", [("uniform", 0), ("uniform", 1), ("uniform", 4095), ("uniform", 4097),
                                    ("uniform", 300001), ("dups", 100000), ("equal", 9000), ("sorted", 70000),
                                    ("reversed", 70001), ("uniform", (1 << 22) + 5), ("clustered", 200000),
                                    ("mixed", 300000), ("mixed", (1 << 21) + 3)])
def test_sort_parity(kind, n):
    rng = np.random.default_rng(n + len(kind))
    keys = _keys(kind, n, rng)
    say("sort", kind, n)
    P, perm = cs.sort(dev(keys) if n else torch.empty(0, dtype=torch.int64, device="cuda"))
    torch.cuda.synchronize()
    rP, rperm = oracle.sort(keys)
    eq(host(P), rP, "sorted keys")
    eq(host(perm), rperm, "perm")


def test_sort_buckets_past_the_lookahead_repeatedly():
    """Level-9 buckets of 1500-2000 keys: most blocks of the bucket pass own a
    single bucket that runs past their look-ahead and is read again (the path
    whose end search once shared a word with a value read before it)."""
    rng = np.random.default_rng(91)
    n = (1 << 22) + 17
    sizes = rng.integers(1500, 2001, n // 1500 + 2)
    pre = np.sort(rng.choice(1 << 27, sizes.size, replace=False)).astype(np.uint64)
    keys = (np.repeat(pre, sizes)[:n] << np.uint64(36)) | rng.integers(0, 1 << 36, n, dtype=np.uint64)
    keys = keys[rng.permutation(n)]
    rP, rperm = oracle.sort(keys)
    d = dev(keys)
    for rep in range(8):
        say("sort, buckets past the look-ahead, rep", rep)
        P, perm = cs.sort(d)
        eq(host(P), rP, "sorted keys")
        eq(host(perm), rperm, "perm")


@pytest.mark.parametrize("lo,hi", [(40, 300), (150, 170), (1900, 2100)])
def test_sort_bucket_sizes_around_the_bucket_kernel_limits(lo, hi):
    """Level-9 buckets whose sizes straddle the bucket kernel's limits: the
    64-key look-ahead and the chunk ends (40-300 keys), the size up to which
    a window's buckets are ranked by counting (150-170), and the size one
    block sorts in LDS (1900-2100; larger buckets are listed for the low
    passes). Low bits with many repeats, so ties are checked too; three
    repeated sorts of the same keys."""
    rng = np.random.default_rng(lo * 7 + hi)
    n = (1 << 21) + 33
    sizes = rng.integers(lo, hi + 1, n // lo + 2)
    pre = np.sort(rng.choice(1 << 27, sizes.size, replace=False)).astype(np.uint64)
    low = rng.integers(0, 1 << 12, n, dtype=np.uint64) << np.uint64(rng.integers(0, 24))
    keys = (np.repeat(pre, sizes)[:n] << np.uint64(36)) | (low & np.uint64((1 << 36) - 1))
    keys = keys[rng.permutation(n)]
    rP, rperm = oracle.sort(keys)
    d = dev(keys)
    for rep in range(3):
        say("sort, bucket sizes", lo, hi, "rep", rep)
        P, perm = cs.sort(d)
        eq(host(P), rP, "sorted keys")
        eq(host(perm), rperm, "perm")


def test_sort_twice_identical():
    rng = np.random.default_rng(5)
    keys = dev(_keys("dups", 500000, rng))
    say("sort determinism")
    a = [host(t) for t in cs.sort(keys)]
    b = [host(t) for t in cs.sort(keys)]
    eq(a[0], b[0], "keys")
    eq(a[1], b[1], "perm")


# ---- counts / rebalance ------------------------------------------------------

def _sorted_particle_keys(kind, n, n_crit, seed, curve=wl.HILBERT):
    s = wl.make_set(kind, n, seed, 0, curve, n_crit)
    keys, _ = oracle.compute_keys(s.x, s.y, s.z, s.box, curve)
    return np.sort(keys)


@pytest.mark.parametrize("kind,n,n_crit", [("uniform", 100000, 64), ("plummer", 200000, 16), ("uniform", 5, 1)])
def test_node_counts_parity(kind, n, n_crit):
    P = _sorted_particle_keys(kind, n, n_crit, 11)
    K = oracle.build_leaves(P, n_crit)
    say("counts", kind, n, n_crit, "leaves", K.size - 1)
    c = cs.node_counts(dev(P), dev(K))
    eq(host(c), oracle.node_counts(P, K), "counts")


@pytest.mark.parametrize("kind,n,n_crit", [("uniform", 0, 64), ("uniform", 1, 1), ("uniform", 64, 64),
                                           ("uniform", 65536, 64), ("uniform", 300000, 8),
                                           ("plummer", 400000, 16), ("plummer", 50000, 1)])
def test_rebalance_from_root_parity(kind, n, n_crit):
    P = _sorted_particle_keys(kind, n, n_crit, 12)
    say("rebalance from root", kind, n, n_crit)
    K, counts, rounds = cs.rebalance(dev(P) if n else torch.empty(0, dtype=torch.int64, device="cuda"), n_crit)
    rK, rN, rrounds, conv, _ = oracle.rebalance_iterate(P, np.array([0, END], np.uint64), n_crit)
    assert conv
    eq(host(K), rK, "leaves")
    eq(host(counts), rN, "counts")
    assert rounds == rrounds
    eq(rK, oracle.build_leaves(P, n_crit), "oracle iterate vs top-down")


def test_rebalance_duplicates_at_level_21():
    rng = np.random.default_rng(3)
    P = np.sort(np.concatenate([np.full(500, 0x1234567, np.uint64), rng.integers(0, END, 3000, dtype=np.uint64)]))
    say("rebalance duplicates")
    K, counts, rounds = cs.rebalance(dev(P), 8)
    rK, rN, rrounds, _, _ = oracle.rebalance_iterate(P, np.array([0, END], np.uint64), 8)
    eq(host(K), rK, "leaves")
    eq(host(counts), rN, "counts")
    assert rounds == rrounds


def test_rebalance_every_round_matches_literal_step():
    P = _sorted_particle_keys("plummer", 300000, 16, 13)
    _, _, rrounds, _, hist = oracle.rebalance_iterate(P, np.array([0, END], np.uint64), 16)
    for r in range(1, rrounds):
        say("rebalance max_iters", r)
        with pytest.raises(cs.CstoneError) as e:
            cs.rebalance(dev(P), 16, max_iters=r)
        assert e.value.name == "NOT_CONVERGED" and e.value.rounds == r
        nl = e.value.n_leaves
        eq(host(e.value.buffer[: nl + 1]), hist[r - 1], f"K after round {r}")
        eq(host(e.value.counts[:nl]), oracle.node_counts(P, hist[r - 1]), f"counts after round {r}")


def test_rebalance_incremental_parity():
    s = wl.make_set("plummer", 300000, 14, 0, wl.HILBERT, 16)
    k0, _ = oracle.compute_keys(s.x, s.y, s.z, s.box, wl.HILBERT)
    P0 = np.sort(k0)
    K0 = oracle.build_leaves(P0, 16)
    for step, moved in enumerate(wl.plummer_rebuild_steps(s, steps=3, sigma=5e-2, seed=14), 1):
        k1, _ = oracle.compute_keys(moved.x, moved.y, moved.z, moved.box, wl.HILBERT)
        P1 = np.sort(k1)
        say("rebalance incremental step", step)
        K, counts, rounds = cs.rebalance(dev(P1), 16, leaves=dev(K0))
        rK, rN, rrounds, conv, _ = oracle.rebalance_iterate(P1, K0, 16)
        eq(host(K), rK, "leaves")
        eq(host(counts), rN, "counts")
        assert rounds == rrounds
        # one literal update, as the paper applies between time-steps
        one, changed = oracle.rebalance_step(K0, oracle.node_counts(P1, K0), 16)
        if changed:
            with pytest.raises(cs.CstoneError) as e:
                cs.rebalance(dev(P1), 16, leaves=dev(K0), max_iters=1)
            assert e.value.name == "NOT_CONVERGED"
            eq(host(e.value.buffer[: e.value.n_leaves + 1]), one, "one update")
        else:
            K1, _, r1 = cs.rebalance(dev(P1), 16, leaves=dev(K0), max_iters=1)
            eq(host(K1), one, "one update")
        K0 = rK


def test_rebalance_capacity_error():
    P = _sorted_particle_keys("uniform", 100000, 16, 15)
    say("rebalance capacity")
    with pytest.raises(cs.CstoneError) as e:
        cs.rebalance(dev(P), 16, capacity=100)
    assert e.value.name == "CAPACITY" and e.value.n_leaves > 100
    K = host(e.value.buffer)
    # the array left behind is the last one that fitted: a valid cornerstone array
    _, _, _, _, hist = oracle.rebalance_iterate(P, np.array([0, END], np.uint64), 16)
    fitted = [h for h in hist if h.size - 1 <= 100][-1]
    eq(K[: fitted.size], fitted, "last fitting array")


# ---- link ------------------------------------------------------------------

@pytest.mark.parametrize("by_sort", [False, True])
@pytest.mark.parametrize("kind,n,n_crit", [("uniform", 0, 64), ("uniform", 65536, 64), ("plummer", 300000, 16),
                                           ("plummer", 20000, 1), ("uniform", 200000, 3),
                                           ("uniform", 3000000, 64)])
def test_link_parity(kind, n, n_crit, by_sort):
    P = _sorted_particle_keys(kind, n, n_crit, 16)
    K = oracle.build_leaves(P, n_crit)
    say("link", kind, n, n_crit, "leaves", K.size - 1, "by_sort", by_sort)
    NK, CO, LO = cs.link_octree(dev(K), by_sort=by_sort)
    rNK, rCO, rLO = oracle.link_octree(K)
    eq(host(NK), rNK, "NK")
    eq(host(CO), rCO, "CO")
    eq(host(LO), rLO, "LO")


@pytest.mark.parametrize("by_sort", [False, True])
def test_link_paper_example(golden_fig, by_sort):
    K = np.array([int(p, 8) << (3 * (21 - len(p))) for p in golden_fig["fig1_bottom_octal_prefixes"]] + [END],
                 np.uint64)
    say("link Fig. 2", "by_sort", by_sort)
    NK, CO, LO = cs.link_octree(dev(K), by_sort=by_sort)
    assert list(host(LO)) == golden_fig["fig2_LO_prefix"] + [golden_fig["fig2_LO_tail_value"]] * 20
    assert [int(v) for v in host(NK)] == [int(s, 8) for s in golden_fig["fig2_NK_octal"]]
    assert list(host(CO)) == golden_fig["fig2_CO"]


# ---- whole build -------------------------------------------------------------

def _check_build(s, r, what):
    ref = oracle.build_tree(s.x, s.y, s.z, s.box, s.curve, s.n_crit)
    eq(host(r.sorted_keys), ref["P"], what + " P")
    eq(host(r.perm), ref["perm"], what + " perm")
    eq(host(r.leaves), ref["K"], what + " K")
    eq(host(r.counts), ref["counts"], what + " counts")
    eq(host(r.node_keys), ref["NK"], what + " NK")
    eq(host(r.child), ref["CO"], what + " CO")
    eq(host(r.level_offsets), ref["LO"], what + " LO")
    return ref


def test_build_config_small_full_parity():
    s = wl.config_small()
    say("build 65536 uniform Morton N_crit 64")
    r = cs.build(*coords(s), s.box, s.curve, s.n_crit)
    ref = _check_build(s, r, "small")
    assert ref["K"].size - 1 == 4096 and r.rounds == 5


def test_build_edge_sets():
    for n in (0, 1, 2, 64, 65):
        s = wl.make_set("uniform", n, 21, 0, wl.HILBERT, 64)
        say("build edge n", n)
        r = cs.build(*coords(s) if n else (torch.empty(0, dtype=torch.float64, device="cuda"),) * 3, s.box, s.curve,
                     s.n_crit)
        _check_build(s, r, f"n={n}")


def test_build_nonfinite_reported():
    s = wl.make_set("uniform", 1000, 22, 0, wl.HILBERT, 16)
    x = s.x.copy()
    x[517] = np.nan
    say("build nonfinite")
    with pytest.raises(cs.CstoneError) as e:
        cs.build(dev(x), dev(s.y), dev(s.z), s.box, s.curve, s.n_crit)
    assert e.value.name == "NONFINITE"


def test_build_start_from_sort_table_empty_cells():
    """Builds from the root whose start reads the sort's level-6 table: one
    with empty cells in the last x slab (the start stops between levels), one
    clustered in a corner (runs of more than 64 empty level-6 cells, found by
    searching P instead)."""
    rng = np.random.default_rng(61)
    n = 1 << 20
    x, y, z = rng.random((3, n))
    cases = [("slab", wl.ParticleSet(x * 0.9, y, z, wl.UNIT_BOX, wl.HILBERT, 8, "uniform")),
             ("corner", wl.ParticleSet(np.where(np.arange(n) % 97 == 0, x, x * 0.02), y * 0.03, z, wl.UNIT_BOX,
                                       wl.MORTON, 16, "clustered"))]
    for what, s in cases:
        say("build from the level-6 table,", what)
        r = cs.build(*coords(s), s.box, s.curve, s.n_crit)
        ref = _check_build(s, r, what)
        assert r.rounds == oracle.rebalance_iterate(ref["P"], np.array([0, END], np.uint64), s.n_crit)[2]


def test_build_uniform_2_24_full_parity():
    s = wl.config_uniform_2_24()
    say("build 2^24 uniform Hilbert N_crit 64")
    b = cs.Builder(s.n, s.n_crit)
    r = b.build(*coords(s), s.box, s.curve, s.n_crit)
    ref = _check_build(s, r, "2^24")
    say("leaves", ref["K"].size - 1, "rounds", r.rounds)
    # same build again on the same buffers: bitwise identical
    r2 = b.build(*coords(s), s.box, s.curve, s.n_crit)
    eq(host(r2.perm), ref["perm"], "second build perm")
    eq(host(r2.node_keys), ref["NK"], "second build NK")


def test_sort_autotune_keeps_the_sort_exact():
    """The shape autotuner times every compiled sort shape and records the
    fastest for this size class; every shape, set through the autotune table,
    sorts bit-exactly, and so does a plain build that looks the shape up."""
    s = wl.make_set("plummer", 300001, 41, 0, wl.HILBERT, 16)
    keys, _ = oracle.compute_keys(s.x, s.y, s.z, s.box, s.curve)
    ref_P, ref_perm = oracle.sort(keys)
    nv = len(cs.sort_variants())
    cs.tune_clear()
    try:
        for v in range(nv):
            say("sort with shape", v, cs.sort_variants()[v])
            cs.tune_set(cs.TUNE_SORT, s.n, v)
            assert cs.tune_get(cs.TUNE_SORT, s.n) == v
            P, perm = cs.sort(dev(keys))
            torch.cuda.synchronize()
            eq(host(P), ref_P, f"shape {v} P")
            eq(host(perm), ref_perm, f"shape {v} perm")
        cs.tune_clear()
        say("sort autotune", nv, "shapes")
        chosen, ms = cs.sort_autotune(dev(keys), reps=1)
        assert 0 <= chosen < nv and len(ms) == nv
        assert all(t > 0 for t in ms) and ms[chosen] == min(ms)
        assert cs.tune_entries() == 1 and cs.tune_get(cs.TUNE_SORT, s.n) == chosen
        assert cs.tune_get(cs.TUNE_SORT, 4 * s.n) == -1  # another size class keeps the built-in shape
        P, perm = cs.sort(dev(keys))
        torch.cuda.synchronize()
        eq(host(P), ref_P, "tuned sort P")
        eq(host(perm), ref_perm, "tuned sort perm")
        r = cs.build(*coords(s), s.box, s.curve, s.n_crit)
        _check_build(s, r, "build with the tuned shape")
    finally:
        cs.tune_clear()


@pytest.mark.slow
def test_sort_lookback_fallback_keeps_the_sort_exact():
    """With the look-back patience at 0, every wait on a predecessor tile is
    settled by the waiting block counting that tile's digits itself (and
    publishing them unless the tile's own block got there first): every
    shape still sorts bit-exactly (uniform keys with a ragged tail; buckets
    long enough for the listed low passes, whose tiles come from a table),
    and so does a whole build."""
    rng = np.random.default_rng(77)
    nv = len(cs.sort_variants())
    cs.tune_clear()
    try:
        cs.set_lookback_patience(0)
        for kind, n in (("uniform", (1 << 21) + 7), ("mixed", 300000)):
            keys = _keys(kind, n, rng)
            rP, rperm = oracle.sort(keys)
            for v in range(nv):
                say("fallback sort", kind, n, "shape", v)
                cs.tune_set(cs.TUNE_SORT, n, v)
                P, perm = cs.sort(dev(keys))
                torch.cuda.synchronize()
                eq(host(P), rP, f"{kind} shape {v} P")
                eq(host(perm), rperm, f"{kind} shape {v} perm")
            cs.tune_clear()
        s = wl.make_set("plummer", 400000, 43, 0, wl.HILBERT, 16)
        say("fallback build plummer 400000")
        r = cs.Builder(s.n, s.n_crit).build(*coords(s), s.box, s.curve, s.n_crit)
        _check_build(s, r, "fallback build")
    finally:
        cs.set_lookback_patience(256)
        cs.tune_clear()


def test_sort_beyond_2_30_uses_wide_lookback_words():
    """n >= 2^30 switches the look-back words to 64 bits (epoch-tagged). At this
    size the sort is checked by its characterisation on the device: sorted,
    a permutation, equal keys in ascending original order, and P[i] equal to
    keys[perm[i]] on a sample."""
    from tests import device_checks as dc
    n = (1 << 30) + 12345
    g = torch.Generator(device="cuda")
    g.manual_seed(30)
    say("sort n =", n)
    keys = torch.randint(0, 1 << 62, (n,), device="cuda", dtype=torch.int64, generator=g)
    keys[: n // 8] %= 1 << 16  # runs of equal keys
    P, perm = cs.sort(keys)
    torch.cuda.synchronize()
    dc.check_sorted_perm(P, perm, n)
    i = torch.randint(0, n, (1 << 20,), device="cuda", generator=g)
    assert torch.equal(P[i], keys[perm.long()[i]])
    # the ties: within equal keys the permutation ascends (checked above), and the
    # number of keys below 2^16 is preserved
    assert int((P < (1 << 16)).sum()) == int((keys < (1 << 16)).sum())


def test_rebalance_from_root_start_between_levels():
    """Every level-3 node is over N_crit but some level-4 nodes are empty
    (particles only in x < 0.9): the loop starts at level 4, not at the finer
    level it searched, and still reports the rounds counted from the root."""
    x, y, z = wl.uniform_cube(1 << 20, 17, 0)
    x = x * 0.9
    keys, _ = oracle.compute_keys(x, y, z, wl.UNIT_BOX, wl.HILBERT)
    P, _ = oracle.sort(keys)
    say("rebalance start between levels")
    K, counts, rounds = cs.rebalance(dev(P), 8)
    rK, rN, rrounds, _, _ = oracle.rebalance_iterate(P, np.array([0, END], np.uint64), 8)
    eq(host(K), rK, "leaves")
    eq(host(counts), rN, "counts")
    assert rounds == rrounds
