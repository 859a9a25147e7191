"""Host-side arithmetic of the surrogate pipeline (CPU)."""
from __future__ import annotations

import numpy as np

from paper_1409_4923_amd import surrogate as S


def test_pool_equals_statistics_of_the_joined_sample():
    rng = np.random.default_rng(7)
    for n1, n2 in ((2, 2), (256, 3000), (700, 17)):
        a = rng.normal(0.3, 1.7, (5, n1))
        b = rng.normal(-0.2, 0.4, (5, n2))
        n, m, s = S.pool(np.full(5, n1), a.mean(1), a.std(1, ddof=1), np.full(5, n2), b.mean(1), b.std(1, ddof=1))
        j = np.concatenate([a, b], axis=1)
        assert np.all(n == n1 + n2)
        np.testing.assert_allclose(m, j.mean(1), rtol=0, atol=1e-14)
        np.testing.assert_allclose(s, j.std(1, ddof=1), rtol=1e-12)


def test_calibrate_threshold_picks_the_largest_qualifying_threshold():
    rng = np.random.default_rng(3)
    std = rng.uniform(0.0, 0.04, 20000)
    err = np.abs(rng.normal(0.0, 1.0, 20000)) * std     # error grows with the spread
    tol = 0.01
    grid = [0.0025 * 2.0 ** (k / 4.0) for k in range(13)]
    t, sweep = S.calibrate_threshold(std, err, tol, grid)
    assert t is not None and t in grid
    for row in sweep:
        ok = row["p95"] is not None and row["p95"] <= tol and row["within_tol"] >= 0.95
        assert ok == (row["threshold"] <= t)             # the qualifying thresholds are a prefix here
        k = std <= row["threshold"]
        assert row["answered"] == k.mean()
    assert t < grid[-1]                                  # the largest spreads do not qualify
    assert S.calibrate_threshold(std, err, 1e-6, grid)[0] is None


def test_point_records_equal_the_workload_records():
    """The column-wise records of a scan over many points hold the same bytes as the
    per-point Workload path."""
    import ctypes
    from paper_1409_4923_amd import workloads as W
    x = W.surrogate_queries(37, seed=4)
    counts = np.arange(37) * 3 + 64
    _, _, M, R = S.point_records(x, counts, 7, seed=11, first_point=1000)
    for i, w in enumerate(S.point_workloads(x, counts, 7, seed=11, first_point=1000)):
        m, r = W.to_c(w)
        assert ctypes.string_at(ctypes.addressof(M[i]), ctypes.sizeof(m)) == \
            ctypes.string_at(ctypes.addressof(m), ctypes.sizeof(m))
        assert ctypes.string_at(ctypes.addressof(R[i]), ctypes.sizeof(r)) == \
            ctypes.string_at(ctypes.addressof(r), ctypes.sizeof(r))
