"""The host-thread oracle helpers used by the full-size GPU tests give
exactly what the single-threaded oracle gives on the whole set (CPU only)."""
import numpy as np
import pytest

import oracle
import workloads as wl
from tests import oracle_pool as pool


def _stacked(n, points, seed):
    x, y, z = wl.uniform_cube(points, seed, 0)
    i = np.arange(n) % points
    return x[i].copy(), y[i].copy(), z[i].copy()


@pytest.mark.parametrize("kind,n,n_crit,job", [("plummer", 400000, 16, 1 << 12), ("uniform", 200000, 64, 5000),
                                               ("plummer", 50000, 1, 3000), ("uniform", 1000, 5000, 10),
                                               ("uniform", 0, 8, 10)])
def test_pool_equals_whole_oracle(kind, n, n_crit, job):
    s = wl.make_set(kind, n, 21, 0, wl.HILBERT, n_crit)
    k = pool.keys(s.x, s.y, s.z, s.box, s.curve, chunk=1 << 14)
    ref, _ = oracle.compute_keys(s.x, s.y, s.z, s.box, s.curve)
    assert np.array_equal(k, ref)
    P, _ = oracle.sort(ref)
    K = oracle.build_leaves(P, n_crit)
    assert np.array_equal(pool.leaves(P, n_crit, job_keys=job), K)
    assert np.array_equal(pool.counts(P, K, chunk=777), oracle.node_counts(P, K))


def test_pool_leaves_with_level_21_stacks():
    """Stacks of equal keys above job_keys reach level 21, where a leaf stays
    whole whatever its count."""
    x, y, z = _stacked(30000, 5, 3)
    keys, _ = oracle.compute_keys(x, y, z, wl.UNIT_BOX, wl.MORTON)
    P, _ = oracle.sort(keys)
    K = oracle.build_leaves(P, 4)
    assert np.array_equal(pool.leaves(P, 4, job_keys=100), K)


def test_pool_reports_mismatches():
    assert pool.mismatch(np.arange(5), np.arange(5), "a") == []
    b = np.arange(5)
    b[3] = 9
    assert "1 mismatches" in pool.mismatch(np.arange(5), b, "a")[0]
    assert "shape" in pool.mismatch(np.arange(4), np.arange(5), "a")[0]
