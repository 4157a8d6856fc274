"""Pins of the oracle's double-layered-torus measurements: Polyakov loops and
per-layer couplings (a plaquette takes the coupling of its base site's layer).

Polyakov loop: cold start 1; a constant diagonal U_3 = diag(e^{i t_k}) gives
(1/3) sum_k e^{i n t_k} for loops of n = L3 (or 2 L3) links; multiplying the
U_3 links of the x3 = 0 slice by a centre element z of SU(3) multiplies every
loop by z per crossing of that slice; gauge invariance; zero mean on a Haar
start.  Two couplings: beta0 = beta1 is the single-coupling chain (same
decisions, links equal up to rounding); the weighted sum rule
sum_{x,mu} Re Tr(U A_beta) = 72 V (beta0 P0 + beta1 P1); and at strong
coupling each layer's mean plaquette is u(beta_layer) to leading order.
"""
import numpy as np
import pytest

from closed_forms import batch_mean_error, weyl_u
from oracle import su3ref


@pytest.mark.parametrize("nlat,mask", [(1, None), (2, 0x7), (2, 0xF)])
def test_polyakov_cold_and_constant_diagonal(nlat, mask):
    L = (4, 4, 4, 6)
    lat = su3ref.Oracle(L, nlat=nlat, flip_mask=mask)
    lat.start(False)
    assert np.all(lat.polyakov() == 1.0)
    t = np.array([0.3, -1.1, 0.8])
    U3 = np.diag(np.exp(1j * t))
    links = lat.links()
    links[3::4] = su3ref._mat(U3)
    steps = 2 * L[3] if (nlat == 2 and (mask >> 3) & 1) else L[3]
    expect = np.exp(1j * steps * t).sum() / 3
    assert np.abs(lat.polyakov() - expect).max() < 1e-13


@pytest.mark.parametrize("nlat,mask", [(1, None), (2, 0x7), (2, 0xF)])
def test_polyakov_centre_phase_and_gauge_invariance(nlat, mask):
    L = (4, 4, 6, 4)
    lat = su3ref.Oracle(L, nlat=nlat, flip_mask=mask, seed=4)
    lat.start(True)
    lat.sweep(2, 5.7)
    p0 = lat.polyakov()
    lat.gauge_transform(55)
    assert np.abs(lat.polyakov() - p0).max() < 1e-13
    # centre element on the x3 = 0 slice
    z = np.exp(2j * np.pi / 3)
    V = lat.V
    links = lat.links()
    for layer in range(nlat):
        for lex in range(L[0] * L[1] * L[2]):  # x3 = 0
            lid = 4 * (layer * V + lex) + 3
            links[lid] = su3ref._mat(z * su3ref.to_complex(links[lid]))
    crossings = 2 if (nlat == 2 and (mask >> 3) & 1) else 1
    lat2 = su3ref.Oracle(L, nlat=nlat, flip_mask=mask, seed=4)
    lat2.start(True)
    lat2.sweep(2, 5.7)
    lat2.gauge_transform(55)
    assert np.abs(lat.polyakov() - z ** crossings * lat2.polyakov()).max() < 1e-13


def test_polyakov_hot_start_zero_mean():
    lat = su3ref.Oracle((8, 8, 8, 4), nlat=2, seed=8)
    lat.start(True)
    p = lat.polyakov()
    sigma = np.sqrt(1 / 18 / (8 ** 3 * 2))
    assert abs(p[0].real) < 5 * sigma and abs(p[0].imag) < 5 * sigma


def test_two_couplings_equal_reduce_to_one():
    a = su3ref.Oracle(4, nlat=2, seed=6)
    b = su3ref.Oracle(4, nlat=2, seed=6)
    for lat in (a, b):
        lat.start(True)
    a.sweep(2, 5.7)
    b.sweep_betas(2, 5.7, 5.7)
    assert np.abs(a.links() - b.links()).max() < 1e-12
    assert a.counters() == b.counters()


def test_weighted_staple_sum_rule():
    lat = su3ref.Oracle(4, nlat=2, seed=2)
    lat.start(True)
    lat.sweep(1, 3.0)
    b0, b1 = 0.7, 2.3
    U = su3ref.to_complex(lat.links())
    s = 0.0
    for x in range(2 * lat.V):
        for mu in range(4):
            s += np.trace(U[4 * x + mu] @ lat.staple_betas(x, mu, b0, b1)).real
    P = lat.plaquette()
    assert abs(s - 72 * lat.V * (b0 * P[1] + b1 * P[2])) < 1e-10 * abs(s)


def test_strong_coupling_per_layer():
    lat = su3ref.Oracle(6, nlat=2, seed=12)
    lat.start(True)
    b0, b1 = 0.5, 1.0
    lat.sweep_betas(10, b0, b1)
    series = []
    for _ in range(300):
        lat.sweep_betas(1, b0, b1)
        series.append(lat.plaquette())
    series = np.array(series)
    for layer, beta in ((1, b0), (2, b1)):
        mean, err = batch_mean_error(series[:, layer], nbins=20)
        u = weyl_u(beta)
        assert abs(mean - u) < 4 * err + 4 * u ** 5, (layer, mean, u, err)


def test_dlt_layers_equilibrate_like_the_single_torus():
    """beta 5.7, flip mask 0x7: the mean plaquettes of the two layers of a
    2 x 8^4 double-layered torus agree with each other and with an 8^4 single
    torus within 3 combined standard errors (binned), whatever the gluing:
    locally every site sees the same action."""
    dlt = su3ref.Oracle(8, nlat=2, seed=41)
    pbc = su3ref.Oracle(8, nlat=1, seed=42)
    series = {"dlt": [], "pbc": []}
    for name, lat in (("dlt", dlt), ("pbc", pbc)):
        lat.start(False)
        lat.sweep(60, 5.7)
        for _ in range(300):
            lat.sweep(1, 5.7)
            series[name].append(lat.plaquette())
    d = np.array(series["dlt"])
    p = np.array(series["pbc"])
    m0, e0 = batch_mean_error(d[:, 1], nbins=20)
    m1, e1 = batch_mean_error(d[:, 2], nbins=20)
    mp, ep = batch_mean_error(p[:, 0], nbins=20)
    assert abs(m0 - m1) < 3 * np.hypot(e0, e1), (m0, e0, m1, e1)
    assert abs(m0 - mp) < 3 * np.hypot(e0, ep), (m0, e0, mp, ep)
    assert abs(m1 - mp) < 3 * np.hypot(e1, ep), (m1, e1, mp, ep)
