"""Lattice-level pins of the oracle: geometry (PBC and the double-layered
torus, including the identity of a one-flip double-layered torus with the
periodic lattice of doubled extent), cold/hot start, checkerboard independence, resume, strong coupling,
the 1-hit acceptance the paper reports, and the stored per-sweep tables."""
import json
import os

import numpy as np
import pytest

from closed_forms import batch_mean_error, weyl_u
from oracle import su3ref
from unfold import doubled_torus_map, unfold_links

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


# ---------------------------------------------------------------- geometry --

@pytest.mark.parametrize("L,nlat,mask", [((4, 4, 4, 4), 1, 0), ((2, 4, 6, 4), 1, 0), ((4, 4, 4, 4), 2, 0x7),
                                         ((4, 2, 4, 6), 2, 0xF), ((4, 4, 4, 4), 2, 0x0), ((4, 4, 2, 4), 2, 0x5)])
def test_neighbours_commute_invert_and_flip_parity(L, nlat, mask):
    lat = su3ref.Oracle(L, nlat=nlat, flip_mask=mask)
    V = lat.V
    for x in range(V * nlat):
        for mu in range(4):
            xp = lat.neighbor(x, mu, +1)
            assert lat.neighbor(xp, mu, -1) == x
            assert lat.parity(xp) != lat.parity(x)
            for nu in range(4):
                assert lat.neighbor(xp, nu, +1) == lat.neighbor(lat.neighbor(x, nu, +1), mu, +1)
                assert lat.neighbor(lat.neighbor(x, mu, -1), nu, -1) == lat.neighbor(lat.neighbor(x, nu, -1), mu, -1)


@pytest.mark.parametrize("mask", [0x7, 0x1, 0xA])
def test_dlt_layer_switches_only_across_flipped_boundaries(mask):
    L = (4, 4, 4, 4)
    lat = su3ref.Oracle(L, nlat=2, flip_mask=mask)
    V = lat.V
    for x in range(2 * V):
        layer, lex = divmod(x, V)
        coords = [(lex // int(np.prod(L[:m]))) % L[m] for m in range(4)]
        for mu in range(4):
            for d in (+1, -1):
                y = lat.neighbor(x, mu, d)
                wraps = (coords[mu] == L[mu] - 1) if d > 0 else (coords[mu] == 0)
                expect_layer = layer ^ (1 if (wraps and (mask >> mu) & 1) else 0)
                assert y // V == expect_layer


@pytest.mark.parametrize("mu", [0, 1, 2, 3])
def test_dlt_with_one_flip_is_the_doubled_torus(mu):
    """Crossing the direction-mu boundary switches the layer, so the two
    layers form one periodic lattice of extent 2 L_mu in that direction (the
    double-layered torus named in Sec. 1, glued as the oracle reads it, one
    direction at a time).  With the same links in both
    labellings the neighbours correspond, every staple is the same bits (same
    links, same order of terms), and the plaquette and Polyakov loop agree to
    rounding.  A wrong layer flip, a flip on the wrong boundary or a wrong
    site in a staple term fails this."""
    L = (4, 2, 6, 4)  # every extent distinct from its neighbour's
    dlt = su3ref.Oracle(L, nlat=2, flip_mask=1 << mu, seed=13)
    dlt.start(True)
    dlt.sweep(1, 5.7)
    L2, site = doubled_torus_map(L, mu)
    pbc = su3ref.Oracle(L2, nlat=1, seed=13)
    pbc.start(False)
    pbc.set_links(unfold_links(dlt.links(), site))
    for s in range(2 * dlt.V):
        for nu in range(4):
            for d in (+1, -1):
                assert pbc.neighbor(site[s], nu, d) == site[dlt.neighbor(s, nu, d)]
            assert np.array_equal(dlt.staple(s, nu), pbc.staple(site[s], nu)), (s, nu)
    p_dlt, p_pbc = dlt.plaquette(), pbc.plaquette()
    assert abs(p_dlt[0] - p_pbc[0]) < 1e-14
    assert abs(p_dlt[0] - 0.5 * (p_dlt[1] + p_dlt[2])) < 1e-14
    assert abs(dlt.polyakov()[0] - pbc.polyakov()[0]) < 1e-14


def test_invalid_parameters_rejected():
    for kw in (dict(L=(3, 4, 4, 4)), dict(L=(0, 4, 4, 4)), dict(L=4, nlat=3), dict(L=4, nlat=1, flip_mask=1),
               dict(L=4, nhit=0), dict(L=(4, 4, 4, 5))):
        with pytest.raises(ValueError):
            su3ref.Oracle(**kw)


# ------------------------------------------------------------------ starts --

@pytest.mark.parametrize("nlat", [1, 2])
def test_cold_start_plaquette_is_exactly_one(nlat):
    lat = su3ref.Oracle((4, 6, 4, 8), nlat=nlat)
    lat.start(False)
    assert np.all(lat.plaquette() == 1.0)


@pytest.mark.parametrize("nlat", [1, 2])
def test_hot_start_plaquette_is_zero_within_statistics(nlat):
    lat = su3ref.Oracle(8, nlat=nlat, seed=3)
    lat.start(True)
    sigma = np.sqrt(1.0 / (108 * lat.V * nlat))
    assert abs(lat.plaquette()[0]) < 5 * sigma


# ----------------------------------------------------- sweep order / resume --

@pytest.mark.parametrize("L,nlat", [((4, 4, 4, 4), 1), ((6, 4, 2, 4), 1), ((4, 4, 4, 4), 2)])
def test_pass_order_and_threads_do_not_change_result(L, nlat):
    ref = su3ref.Oracle(L, nlat=nlat, seed=17)
    ref.start(True)
    ref.sweep(2, 5.7, nthreads=1)
    for nthreads, order in ((1, 12345), (4, 0), (3, 999)):
        lat = su3ref.Oracle(L, nlat=nlat, seed=17)
        lat.start(True)
        lat.sweep(2, 5.7, nthreads=nthreads, order_seed=order)
        assert np.array_equal(lat.links(), ref.links())
        assert lat.counters() == ref.counters()


def test_split_sweeps_and_restore_equal_one_run():
    full = su3ref.Oracle(4, seed=5)
    full.start(True)
    full.sweep(6, 5.7)
    part = su3ref.Oracle(4, seed=5)
    part.start(True)
    part.sweep(3, 5.7)
    # checkpoint: links + sweep counter, restored into a fresh lattice
    restored = su3ref.Oracle(4, seed=5)
    restored.set_links(part.links())
    restored.sweeps = part.sweeps
    part.sweep(3, 5.7)
    restored.sweep(3, 5.7)
    assert np.array_equal(part.links(), full.links())
    assert np.array_equal(restored.links(), full.links())


def test_dlt_without_flips_is_two_independent_tori():
    pbc = su3ref.Oracle(4, nlat=1, seed=9)
    pbc.start(True)
    pbc.sweep(2, 5.7)
    dlt = su3ref.Oracle(4, nlat=2, flip_mask=0, seed=9)
    dlt.start(True)
    dlt.sweep(2, 5.7)
    n = pbc.links().shape[0]
    # layer 0 carries the same link ids as the periodic lattice
    assert np.array_equal(dlt.links()[:n], pbc.links())
    p = dlt.plaquette()
    assert p[1] == pbc.plaquette()[0]
    assert p[2] != p[1]


def test_dlt_with_flips_couples_layers():
    a = su3ref.Oracle(4, nlat=2, flip_mask=0, seed=9)
    b = su3ref.Oracle(4, nlat=2, flip_mask=0x7, seed=9)
    for lat in (a, b):
        lat.start(True)
        lat.sweep(1, 5.7)
    assert not np.array_equal(a.links(), b.links())


def test_links_stay_special_unitary_after_sweeps():
    lat = su3ref.Oracle(6, nlat=2, seed=2)
    lat.start(True)
    lat.sweep(3, 5.7)
    U = su3ref.to_complex(lat.links())
    assert np.abs(U @ U.conj().transpose(0, 2, 1) - np.eye(3)).max() < 1e-13
    assert np.abs(np.linalg.det(U) - 1).max() < 1e-13


# ------------------------------------------------------------- statistics --

@pytest.mark.parametrize("beta,nlat", [(0.5, 1), (1.0, 1), (1.0, 2)])
def test_strong_coupling_plaquette(beta, nlat):
    # leading strong coupling: <P> = u(beta) + O(u^5); 4 u^5 < 4e-6 here
    lat = su3ref.Oracle(6, nlat=nlat, seed=int(beta * 10) + nlat)
    lat.start(True)
    lat.sweep(10, beta)
    series = []
    for _ in range(400 // nlat):
        lat.sweep(1, beta)
        series.append(lat.plaquette()[0])
    mean, err = batch_mean_error(series, nbins=20)
    u = weyl_u(beta)
    assert abs(mean - u) < 4 * err + 4 * u ** 5, (mean, u, err)
    # and the naive leading term beta/18 alone is excluded at beta = 1
    if beta == 1.0:
        assert abs(mean - beta / 18) > 4 * err


def test_one_hit_acceptance_matches_paper():
    paper = json.load(open(os.path.join(GOLDEN, "paper_values.json")))["one_hit_acceptance_beta_5_7"]["value"]
    lat = su3ref.Oracle(8, seed=1)
    lat.start(False)
    lat.sweep(25, 5.7)
    a0, c0 = lat.counters()
    lat.sweep(10, 5.7)
    a1, c1 = lat.counters()
    rate = (c1 - c0) / (a1 - a0)
    assert abs(rate - paper) < 0.005, rate


# ---------------------------------------------------------- stored tables --

def test_m1_table_reproduces():
    table = json.load(open(os.path.join(GOLDEN, "m1_plaquette.json")))["rows"]
    lat = su3ref.Oracle(8, seed=1)
    lat.start(False)
    for row in table:
        lat.sweep(1, 5.7)
        assert abs(lat.plaquette()[0] - row["plaquette"]) < 1e-12
        assert lat.counters() == (row["attempts"], row["accepts"])


def test_dlt_table_reproduces():
    table = json.load(open(os.path.join(GOLDEN, "dlt_plaquette.json")))["rows"]
    lat = su3ref.Oracle(4, nlat=2, flip_mask=0x7, seed=1)
    lat.start(True)
    for row in table:
        lat.sweep(1, 5.7)
        assert np.abs(lat.plaquette() - np.array(row["plaquette"])).max() < 1e-12
