"""The tree focused on a range F of the curve (Sec. 7: minimum-distance MAC
as f^LE_2 and the g^LE rebalance) against the oracle, element by element."""
import numpy as np
import pytest
import torch

import oracle
import workloads as wl

pytestmark = pytest.mark.gpu

cs = pytest.importorskip("paper_2307_06345_amd")

END = 1 << 63


def say(*a):
    print("[case]", *a, flush=True)


def sorted_keys(s):
    keys, _ = oracle.compute_keys(s.x, s.y, s.z, s.box, s.curve)
    P, _ = oracle.sort(keys)
    return P


def focus_range(P, lo_frac, hi_frac, align_bits=45):
    a = int(P[int(lo_frac * (P.size - 1))]) >> align_bits << align_bits
    b = (int(P[int(hi_frac * (P.size - 1))]) >> align_bits << align_bits) + (1 << align_bits)
    return a, min(b, END)


CASES = [("plummer", 200001, 16, wl.HILBERT, 0.5, 0.40, 0.45), ("uniform", 150000, 8, wl.MORTON, 0.5, 0.1, 0.3),
         ("plummer", 100000, 1, wl.HILBERT, 1.0, 0.7, 0.71), ("uniform", 120000, 64, wl.HILBERT, 0.25, 0.0, 0.05),
         ("plummer", 80000, 4, wl.MORTON, 0.8, 0.95, 1.0)]


@pytest.mark.parametrize("kind,n,n_crit,curve,theta,lo,hi", CASES)
def test_focus_rebalance_parity(kind, n, n_crit, curve, theta, lo, hi):
    s = wl.make_set(kind, n, 50 + n_crit, 0, curve, n_crit)
    P = sorted_keys(s)
    fa, fb = focus_range(P, lo, hi)
    say("focus", kind, n, n_crit, curve, theta, hex(fa), hex(fb))
    dP = cs.from_numpy(P, "cuda")
    K, N, rounds = cs.focus_rebalance(dP, n_crit, curve, fa, fb, theta)
    ref = oracle.focus_leaves(P, n_crit, curve, fa, fb, theta)
    assert np.array_equal(cs.to_numpy(K), ref)
    assert np.array_equal(cs.to_numpy(N), oracle.node_counts(P, ref))
    Ko, _, ro, conv, _ = oracle.focus_iterate(P, n_crit, curve, fa, fb, theta)
    assert conv and rounds == ro
    # from the plain balanced tree, and after F moves: the same fixed points
    K0 = cs.from_numpy(oracle.build_leaves(P, n_crit), "cuda")
    K2, _, _ = cs.focus_rebalance(dP, n_crit, curve, fa, fb, theta, leaves=K0)
    assert np.array_equal(cs.to_numpy(K2), ref)
    fa2, fb2 = focus_range(P, max(0.0, lo - 0.2), max(0.0, lo - 0.2) + 0.03)
    K3, _, _ = cs.focus_rebalance(dP, n_crit, curve, fa2, fb2, theta, leaves=K)
    assert np.array_equal(cs.to_numpy(K3), oracle.focus_leaves(P, n_crit, curve, fa2, fb2, theta))


def test_focus_special_ranges():
    s = wl.make_set("plummer", 60000, 8, 0, wl.HILBERT, 16)
    P = sorted_keys(s)
    dP = cs.from_numpy(P, "cuda")
    full = oracle.build_leaves(P, 16)
    fa, fb = focus_range(P, 0.3, 0.4)
    K, _, _ = cs.focus_rebalance(dP, 16, wl.HILBERT, fa, fb, 0.0)  # theta 0: every MAC fails
    assert np.array_equal(cs.to_numpy(K), full)
    K, _, _ = cs.focus_rebalance(dP, 16, wl.HILBERT, 0, END, 0.6)  # F = the whole domain
    assert np.array_equal(cs.to_numpy(K), full)
    K, N, r = cs.focus_rebalance(dP, 16, wl.HILBERT, fa, fa, 0.6)  # empty F: nothing to resolve
    assert list(cs.to_numpy(K)) == [0, END] and int(cs.to_numpy(N)[0]) == 60000 and r == 1
    with pytest.raises(cs.CstoneError):
        cs.focus_rebalance(dP, 16, wl.HILBERT, fb, fa, 0.6)  # start after end
    with pytest.raises(cs.CstoneError):
        cs.focus_rebalance(dP, 16, wl.HILBERT, fa, fb, -1.0)


@pytest.mark.parametrize("curve", [wl.MORTON, wl.HILBERT])
@pytest.mark.parametrize("theta", [0.0, 0.4, 1.5])
def test_focus_mac_parity(curve, theta):
    s = wl.make_set("plummer", 100000, 3 + curve, 0, curve, 4)
    P = sorted_keys(s)
    fa, fb = focus_range(P, 0.55, 0.6, align_bits=39)
    K = oracle.focus_leaves(P, 4, curve, fa, fb, 0.5)
    NK, CO, LO = oracle.link_octree(K)
    got = cs.to_numpy(cs.focus_mac(cs.from_numpy(NK, "cuda"), curve, fa, fb, theta))
    ref = np.empty(NK.size, np.uint8)
    for p, key in enumerate(NK):
        level = (int(key).bit_length() - 1) // 3
        start = (int(key) - (1 << (3 * level))) << (3 * (21 - level))
        ref[p] = oracle.mac_fails(start, level, curve, fa, fb, theta)
    assert np.array_equal(got, ref)


def test_focus_rebalance_2_24():
    s = wl.config_uniform_2_24()
    say("focus 2^24")
    x, y, z = (cs.from_numpy(a, "cuda") for a in (s.x, s.y, s.z))
    b = cs.Builder(s.n, s.n_crit)
    r = b.build(x, y, z, s.box, s.curve, s.n_crit)
    P = cs.to_numpy(r.sorted_keys)
    fa, fb = focus_range(P, 0.5, 0.5 + 1 / 64)
    K, N, rounds = cs.focus_rebalance(r.sorted_keys, s.n_crit, s.curve, fa, fb, 0.5)
    ref = oracle.focus_leaves(P, s.n_crit, s.curve, fa, fb, 0.5)
    assert np.array_equal(cs.to_numpy(K), ref)
    assert np.array_equal(cs.to_numpy(N), oracle.node_counts(P, ref))
    say("focused leaves", ref.size - 1, "of", r.n_leaves, "rounds", rounds)
