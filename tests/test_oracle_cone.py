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


@pytest.mark.parametrize("L,nlat,flip", [((4, 6, 4, 2), 1, None), ((4, 4, 6, 4), 2, 0x7), ((6, 4, 4, 4), 2, 0xF)])
def test_geometry_handle_indexes_like_the_full_oracle(L, nlat, flip):
    full = su3ref.Oracle(L, nlat=nlat, flip_mask=flip)
    geo = su3ref.Geometry(L, nlat=nlat, flip_mask=flip)
    assert geo.V == full.V
    for site in range(nlat * full.V):
        assert geo.parity(site) == full.parity(site)
        for mu in range(4):
            assert np.array_equal(geo.staple_lids(site, mu), full.staple_lids(site, mu))


def test_geometry_handle_at_the_size_limit():
    # 2^30 sites (the largest lattice the library accepts) without any link
    # storage: site indices beyond 2^31 links stay exact
    L = (256, 256, 128, 128)
    geo = su3ref.Geometry(L)
    assert geo.V == 1 << 30
    last = geo.V - 1  # x = (255, 255, 127, 127): odd parity
    assert geo.parity(last) == (255 + 255 + 127 + 127) % 2
    assert geo.neighbor(last, 0, +1) == last - 255
    assert geo.neighbor(last, 3, +1) == last - 127 * 256 * 256 * 128
    lids = geo.staple_lids(last, 2)
    assert lids.min() >= 0 and lids.max() < 4 * geo.V
    # U_nu(x) of the site itself is among the staple links, nu != 2
    assert {4 * last + 0, 4 * last + 1, 4 * last + 3} <= set(int(l) for l in lids)
