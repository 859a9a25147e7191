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
