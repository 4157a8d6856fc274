"""Pin of the oracle's Cabibbo-Marinari heat bath (projection, embedding and
the alpha = 2 beta k / 3 factor) on one link in a fixed staple A = c G, G Haar:
the chain must sample exp((beta/3) Re Tr(U A)), so <1/3 Re Tr(U A)>/c equals
the one-link Weyl integral u(beta c) for any number of attempts per subgroup
(each attempt is an independent proposal, so rejection keeps detailed balance)."""
import numpy as np
import pytest

from closed_forms import batch_mean_error, weyl_u
from oracle import su3ref


@pytest.mark.parametrize("bc,c,nhit", [(3.0, 2.0, 1), (4.5, 0.7, 1), (11.4, 3.0, 1), (11.4, 3.0, 3),
                                       (1.0, 1.5, 2)])
def test_single_link_chain_matches_weyl_integral(bc, c, nhit):
    G = su3ref.hot_link(4242, 3)
    A = c * G
    U0 = su3ref.hot_link(4242, 4)
    obs, U = su3ref.single_link_chain(U0, A, bc / c, seed=int(bc * 100) + nhit, nsteps=200_000, nhit=nhit)
    mean, err = batch_mean_error(obs[1000:] / c, nbins=40)
    assert abs(mean - weyl_u(bc)) < 4.5 * err, (mean, weyl_u(bc), err)
    assert np.abs(U @ U.conj().T - np.eye(3)).max() < 1e-13


def test_heatbath_changes_only_via_keyed_randoms():
    # same (seed, lid, sweep) -> identical result; any key word changed -> different
    U0 = su3ref.hot_link(1, 0)
    A = 2.0 * su3ref.hot_link(1, 1)
    base, att, acc = su3ref.heatbath_link(U0, A, 5.7, 1, 10, 3)
    again, _, _ = su3ref.heatbath_link(U0, A, 5.7, 1, 10, 3)
    assert np.array_equal(base, again)
    assert att == 3 and 0 <= acc <= 3
    for args in ((5.7, 2, 10, 3), (5.7, 1, 11, 3), (5.7, 1, 10, 4)):
        other, _, _ = su3ref.heatbath_link(U0, A, *args)
        assert not np.allclose(other, base)


def test_heatbath_zero_staple_leaves_link():
    # k = 0 in every subgroup: nothing to sample against, the link only gets reunitarised
    U0 = su3ref.hot_link(3, 3)
    U, att, acc = su3ref.heatbath_link(U0, np.zeros((3, 3), complex), 5.7, 1, 0, 0)
    assert att == 0 and acc == 0
    assert np.abs(U - U0).max() < 1e-15
