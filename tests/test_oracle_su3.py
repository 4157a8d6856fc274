"""Pins of the oracle's SU(3) algebra: Haar start, reunitarisation, staple
covariance and the gauge invariance of the plaquette.

Haar moments of t = Tr U on SU(3) (group theory / Weyl integration):
E t = 0, E|t|^2 = 1, E (Re t)^2 = 1/2, E t^3 = 1 (the singlet in 3x3x3, which
U(3) does not have), E (Re t)^3 = 1/4, E|t|^4 = 2.
"""
import numpy as np
import pytest

from oracle import su3ref


def _haar_sample():
    traces = []
    for seed in (11, 12):
        lat = su3ref.Oracle(12, seed=seed)
        lat.start(True)
        traces.append(np.trace(su3ref.to_complex(lat.links()), axis1=1, axis2=2))
    return np.concatenate(traces)


def test_hot_links_are_special_unitary():
    lat = su3ref.Oracle((4, 4, 6, 8), seed=5)
    lat.start(True)
    U = su3ref.to_complex(lat.links())
    eye = np.eye(3)
    assert np.abs(U @ U.conj().transpose(0, 2, 1) - eye).max() < 1e-13
    assert np.abs(np.linalg.det(U) - 1).max() < 1e-13


def test_hot_start_matches_single_link_primitive():
    lat = su3ref.Oracle(4, seed=77)
    lat.start(True)
    U = su3ref.to_complex(lat.links())
    for lid in (0, 1, 5, 1023):
        assert np.array_equal(U[lid], su3ref.hot_link(77, lid))


def test_haar_moments():
    t = _haar_sample()
    n = len(t)

    def check(x, expect):
        x = np.asarray(x)
        err = x.std() / np.sqrt(n)
        assert abs(x.mean() - expect) < 5 * err + 1e-12, (x.mean(), expect, err)

    check(t.real, 0.0)
    check(t.imag, 0.0)
    check(np.abs(t) ** 2, 1.0)
    check(t.real ** 2, 0.5)
    check((t ** 3).real, 1.0)
    check((t ** 3).imag, 0.0)
    check(t.real ** 3, 0.25)
    check(np.abs(t) ** 4, 2.0)


def test_reunit_projects_onto_su3_and_fixes_su3():
    rng = np.random.default_rng(3)
    for lid in range(20):
        U = su3ref.hot_link(9, lid)
        assert np.abs(su3ref.reunit(U) - U).max() < 1e-15
        noisy = U + 1e-3 * (rng.normal(size=(3, 3)) + 1j * rng.normal(size=(3, 3)))
        R = su3ref.reunit(noisy)
        assert np.abs(R @ R.conj().T - np.eye(3)).max() < 1e-14
        assert abs(np.linalg.det(R) - 1) < 1e-14
        assert np.abs(R - U).max() < 1e-2
        # Gram-Schmidt keeps the direction of row 0
        r0 = noisy[0] / np.linalg.norm(noisy[0])
        assert np.abs(R[0] - r0).max() < 1e-15


@pytest.mark.parametrize("nlat", [1, 2])
def test_staple_is_gauge_covariant(nlat):
    lat = su3ref.Oracle(4, nlat=nlat, seed=21)
    lat.start(True)
    lat.sweep(1, 5.7)
    before = {(x, mu): lat.staple(x, mu) for x in range(0, lat.V * nlat, 7) for mu in range(4)}
    gseed = 99
    lat.gauge_transform(gseed)
    for (x, mu), A in before.items():
        g_x = su3ref.gauge_element(gseed, x)
        g_y = su3ref.gauge_element(gseed, lat.neighbor(x, mu, +1))
        expect = g_y @ A @ g_x.conj().T
        assert np.abs(lat.staple(x, mu) - expect).max() < 1e-13


@pytest.mark.parametrize("nlat", [1, 2])
def test_plaquette_is_gauge_invariant(nlat):
    lat = su3ref.Oracle((4, 6, 4, 4), nlat=nlat, seed=8)
    lat.start(True)
    lat.sweep(2, 5.7)
    p0 = lat.plaquette()
    links0 = lat.links().copy()
    lat.gauge_transform(1234)
    p1 = lat.plaquette()
    assert np.all(np.abs(p1 - p0) <= 1e-13 * np.abs(p0).max())
    # the transformed links are a different configuration
    assert np.abs(lat.links() - links0).max() > 0.1


@pytest.mark.parametrize("nlat", [1, 2])
def test_staple_plaquette_sum_rule(nlat):
    # every plaquette enters the staples of exactly its four links, so
    # sum_{x,mu} Re Tr(U_mu(x) A_mu(x)) = 4 * sum_P Re Tr U_P = 72 V nlat P
    lat = su3ref.Oracle(4, nlat=nlat, seed=31)
    lat.start(True)
    lat.sweep(1, 3.0)
    U = su3ref.to_complex(lat.links())
    s = 0.0
    for x in range(lat.V * nlat):
        for mu in range(4):
            s += np.trace(U[4 * x + mu] @ lat.staple(x, mu)).real
    P = lat.plaquette()[0]
    assert abs(s - 72 * lat.V * nlat * P) < 1e-10 * abs(s)
