"""Pins for the oracle's coordinate quantisation and SFC keys (Sec. 3).

Each test checks the oracle against something it does not compute itself: a
closed form, an exact rational bound, an independent ordering rule, or the
invariants the paper states for octree-compatible curves.
"""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle

L = 21


def test_quantize_unit_box_closed_form():
    # x = m * 2^-53 exactly; on the unit box the grid coordinate is floor(x 2^21) = m >> 32.
    rng = np.random.default_rng(11)
    m = rng.integers(0, 1 << 53, size=20000, dtype=np.int64).astype(np.uint64)
    x = m.astype(np.float64) * 2.0 ** -53
    y = np.zeros_like(x)
    ix, iy, iz, bad = oracle.quantize(x, y, y, ((0, 0, 0), (1, 1, 1)))
    assert not bad
    assert np.array_equal(ix.astype(np.uint64), m >> np.uint64(32))
    assert np.all(iy == 0) and np.all(iz == 0)


def test_quantize_general_box_within_rounding():
    # On [-20, 20]^3 the scale 2^21/40 is inexact; the result must equal the exact
    # rational floor((c - lo) 2^21 / (hi - lo)) except within a few ulps of an integer.
    rng = np.random.default_rng(12)
    c = rng.uniform(-20, 20, size=3000)
    lo, hi = -20.0, 20.0
    ix, _, _, bad = oracle.quantize(c, c, c, ((lo,) * 3, (hi,) * 3))
    assert not bad
    for ci, qi in zip(c, ix):
        t = (Fraction(ci) - Fraction(lo)) * (1 << L) / (Fraction(hi) - Fraction(lo))
        fl = math.floor(t)
        frac = t - fl
        if Fraction(1, 10 ** 9) < frac < 1 - Fraction(1, 10 ** 9):
            assert qi == min(fl, (1 << L) - 1)
        else:
            assert abs(int(qi) - fl) <= 1


def test_quantize_edges_and_nonfinite():
    box = ((-1.0, 0.0, 2.0), (1.0, 4.0, 3.0))
    x = np.array([-1.0, 1.0, -5.0, 7.0, np.nextafter(1.0, -2)])
    y = np.array([0.0, 4.0, -1.0, 9.0, 2.0])
    z = np.array([2.0, 3.0, 1.0, 4.0, 2.5])
    ix, iy, iz, bad = oracle.quantize(x, y, z, box)
    top = (1 << L) - 1
    assert not bad
    assert list(ix) == [0, top, 0, top, top]      # lo -> 0, hi -> clamp, below -> 0, above -> clamp
    assert list(iy) == [0, top, 0, top, 1 << 20]  # midpoint of [0, 4) is exactly 2^20
    assert list(iz) == [0, top, 0, top, 1 << 20]
    for v, expect in ((np.nan, 0), (np.inf, top), (-np.inf, 0)):
        a = np.array([v])
        q, _, _, bad = oracle.quantize(a, np.zeros(1), np.zeros(1), ((0, 0, 0), (1, 1, 1)))
        assert bad and q[0] == expect


def test_morton_octant_digits():
    # Sec. 3: matching leading octal digits <=> same octree node at that level.
    rng = np.random.default_rng(13)
    for _ in range(2000):
        a = rng.integers(0, 1 << L, 3)
        lvl = int(rng.integers(1, L + 1))
        sh = L - lvl
        b = (a >> sh << sh) | rng.integers(0, 1 << sh, 3) if sh else a.copy()
        ka = oracle.morton_key(*map(int, a))
        kb = oracle.morton_key(*map(int, b))
        assert ka >> (3 * sh) == kb >> (3 * sh)
        c = b.copy()
        ax = int(rng.integers(0, 3))
        c[ax] ^= 1 << (sh + int(rng.integers(0, lvl)))  # leave the level-lvl cell
        kc = oracle.morton_key(*map(int, c))
        assert ka >> (3 * sh) != kc >> (3 * sh)


def _zorder_less(p, q):
    # Z-order comparison without keys: the axis holding the most significant
    # differing bit decides; on equal bit position x outranks y outranks z.
    best, best_msb = None, -1
    for ax in range(3):
        d = p[ax] ^ q[ax]
        if d and d.bit_length() - 1 > best_msb:
            best, best_msb = ax, d.bit_length() - 1
    if best is None:
        return False
    return p[best] < q[best]


def test_morton_matches_zorder_comparator():
    import functools
    rng = np.random.default_rng(14)
    pts = [tuple(int(v) for v in rng.integers(0, 1 << L, 3)) for _ in range(1500)]
    # add near-duplicates that differ in low bits only
    pts += [(p[0] ^ 1, p[1], p[2]) for p in pts[:200]] + [(p[0], p[1], p[2] ^ 2) for p in pts[:200]]
    by_key = sorted(pts, key=lambda p: oracle.morton_key(*p))
    by_cmp = sorted(pts, key=functools.cmp_to_key(lambda a, b: -1 if _zorder_less(a, b) else (1 if _zorder_less(b, a) else 0)))
    assert by_key == by_cmp


def test_morton_bijection_small_grid():
    b = 4
    keys = {oracle.morton_key(x, y, z) for x, y, z in itertools.product(range(1 << b), repeat=3)}
    assert keys == set(range(8 ** b))


@pytest.mark.parametrize("bits", [1, 2, 3, 4])
def test_hilbert_small_curve_invariants(bits):
    # Exhaustive on a 2^bits grid: bijection onto [0, 8^bits), unit steps,
    # origin at key 0, aligned 8^m key blocks are aligned 2^m cubes (Sec. 3).
    n = 1 << bits
    pts = {}
    for x, y, z in itertools.product(range(n), repeat=3):
        k = oracle.hilbert_key(x, y, z, bits)
        assert k not in pts
        pts[k] = (x, y, z)
    assert set(pts) == set(range(8 ** bits))
    assert pts[0] == (0, 0, 0)
    for k in range(8 ** bits - 1):
        a, b = pts[k], pts[k + 1]
        assert sum(abs(u - v) for u, v in zip(a, b)) == 1, (k, a, b)
    for m in range(1, bits + 1):
        blk = 8 ** m
        side = 1 << m
        for start in range(0, 8 ** bits, blk):
            cube = np.array([pts[k] for k in range(start, start + blk)])
            lo = cube.min(0)
            assert np.all(cube.max(0) - lo == side - 1)
            assert np.all(lo % side == 0)
    for k, p in pts.items():
        assert oracle.hilbert_decode(k, bits) == p


@pytest.mark.parametrize("bits", [5, 6, 7])
def test_hilbert_coarse_curve_of_the_full_keys(bits):
    # Exhaustive over the cells of a 2^bits grid (2^21 cells at 7 bits): the
    # top 3 bits digits of the full 21-bit keys of the cell centres order the
    # cells along a Hilbert curve of order `bits` -- a bijection onto
    # [0, 8^bits), starting at the origin, consecutive cells sharing a face,
    # and every aligned run of 8^m cells an aligned 2^m cube (Sec. 3: the
    # curve refines the octree level by level).
    n = 1 << bits
    ix, iy, iz = (a.ravel() for a in np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij"))
    keys, _ = oracle.compute_keys((ix + 0.5) / n, (iy + 0.5) / n, (iz + 0.5) / n, ((0, 0, 0), (1, 1, 1)),
                                  oracle.HILBERT)
    cell = keys.astype(np.uint64) >> np.uint64(3 * (L - bits))
    order = np.argsort(cell, kind="stable")
    assert np.array_equal(cell[order], np.arange(n ** 3, dtype=np.uint64))
    pts = np.stack([ix[order], iy[order], iz[order]], axis=1).astype(np.int64)
    assert tuple(pts[0]) == (0, 0, 0)
    assert np.all(np.abs(np.diff(pts, axis=0)).sum(axis=1) == 1)
    for m in range(1, bits + 1):
        blocks = pts.reshape(-1, 8 ** m, 3)
        lo, hi = blocks.min(axis=1), blocks.max(axis=1)
        assert np.all(hi - lo == (1 << m) - 1)
        assert np.all(lo % (1 << m) == 0)


def test_hilbert_21bit_roundtrip_and_steps():
    rng = np.random.default_rng(15)
    for _ in range(3000):
        p = tuple(int(v) for v in rng.integers(0, 1 << L, 3))
        k = oracle.hilbert_key(*p)
        assert k < (1 << 63)
        assert oracle.hilbert_decode(k) == p
        k2 = int(rng.integers(0, (1 << 63) - 1, dtype=np.int64))
        a, b = oracle.hilbert_decode(k2), oracle.hilbert_decode(k2 + 1)
        assert sum(abs(u - v) for u, v in zip(a, b)) == 1
    assert oracle.hilbert_key(0, 0, 0) == 0


@pytest.mark.parametrize("m", [1, 2, 3])
def test_hilbert_21bit_coarse_levels(m):
    # The 21-bit curve restricted to level-m cells: every cell's points share the
    # first m octal digits, the cells are visited once each, consecutive cells
    # share a face (Sec. 3: octant-by-octant traversal).
    sh = L - m
    rng = np.random.default_rng(16 + m)
    order = {}
    for cell in itertools.product(range(1 << m), repeat=3):
        base = [c << sh for c in cell]
        ks = set()
        for _ in range(4):
            off = rng.integers(0, 1 << sh, 3)
            ks.add(oracle.hilbert_key(*(int(b + o) for b, o in zip(base, off))) >> (3 * sh))
        assert len(ks) == 1
        order[ks.pop()] = cell
    assert set(order) == set(range(8 ** m))
    for k in range(8 ** m - 1):
        assert sum(abs(u - v) for u, v in zip(order[k], order[k + 1])) == 1


def test_compute_keys_matches_scalar_entry_points():
    rng = np.random.default_rng(17)
    x, y, z = rng.random(500), rng.random(500), rng.random(500)
    box = ((0, 0, 0), (1, 1, 1))
    ix, iy, iz, _ = oracle.quantize(x, y, z, box)
    km, _ = oracle.compute_keys(x, y, z, box, oracle.MORTON)
    kh, _ = oracle.compute_keys(x, y, z, box, oracle.HILBERT)
    for p in range(500):
        assert km[p] == oracle.morton_key(int(ix[p]), int(iy[p]), int(iz[p]))
        assert kh[p] == oracle.hilbert_key(int(ix[p]), int(iy[p]), int(iz[p]))
