"""Host planning of the PCA driver: the Newton schedule of the library's
driver equals the oracle's Lazy Normalization simulation (written apart
from it) and the replication layout round-trips."""
import numpy as np
import pytest

from oracle import power as P
from paper_2305_17341_amd import pca


@pytest.mark.parametrize("l_p", [1, 2, 4, 7, 14, 20])
def test_schedule_matches_oracle_simulation(l_p):
    assert pca.lazy_schedule(l_p) == P.lazy_schedule(l_p)


def test_schedule_other_bounds():
    for S, e in [(0.25, 1e-4), (0.8, 1e-6)]:
        assert pca.lazy_schedule(6, S=S, e=e) == P.lazy_schedule(6, S=S, e=e)


def test_replication_layout():
    v = np.arange(32.0)
    for axis in (0, 1):
        a = pca.replicate(v, 2, 16, axis)
        b = P.replicate(v, 2, 16, axis)
        for x, y in zip(a, b):
            assert np.array_equal(x, y)
        assert np.array_equal(P.unreplicate(a, axis), v)
