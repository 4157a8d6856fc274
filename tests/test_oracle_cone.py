"""The one-by-one first-sweep values agree bit for bit with the oracle's own
full sweep (pins the helper used for full-size sampled GPU checks)."""
import numpy as np
import pytest

from cone import FirstSweepCone, sample_lids
from oracle import su3ref


@pytest.mark.parametrize("L,nlat,hot", [((6, 6, 6, 6), 1, True), ((4, 6, 4, 4), 2, True), ((4, 4, 4, 4), 1, False)])
def test_cone_matches_full_sweep(L, nlat, hot):
    full = su3ref.Oracle(L, nlat=nlat, seed=3)
    full.start(hot)
    full.sweep(1, 5.7)
    ref = su3ref.to_complex(full.links())
    cone = FirstSweepCone(L, nlat=nlat, seed=3, beta=5.7, hot=hot)
    for lid in sample_lids(len(ref), 24, seed=1):
        assert np.array_equal(cone.value(lid), ref[lid])
