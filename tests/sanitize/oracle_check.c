/* Runs every entry point of the FP64 oracle on small lattices (periodic and
 * double-layered, all flip masks used in the tests, a ragged shape, several
 * attempts per subgroup, strong and weak coupling) for the sanitizer build:
 * the checks here are coarse (ranges, exact identities); the point is that
 * the address and undefined-behaviour sanitizers see every code path. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../oracle/su3ref.h"

static int fails = 0;
#define CHECK(c, ...)                                      \
    do {                                                   \
        if (!(c)) {                                        \
            fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__); \
            fprintf(stderr, __VA_ARGS__);                  \
            fprintf(stderr, "\n");                         \
            ++fails;                                       \
        }                                                  \
    } while (0)

static void geometry_checks(const su3ref_lattice *lat, int nlat)
{
    const int64_t V = su3ref_volume(lat), nsite = V * nlat;
    for (int64_t s = 0; s < nsite; ++s)
        for (int mu = 0; mu < 4; ++mu) {
            const int64_t f = su3ref_neighbor(lat, s, mu, +1), b = su3ref_neighbor(lat, s, mu, -1);
            CHECK(f >= 0 && f < nsite && b >= 0 && b < nsite, "neighbour out of range");
            CHECK(su3ref_neighbor(lat, f, mu, -1) == s, "neighbour does not invert");
            CHECK(su3ref_parity(lat, f) != su3ref_parity(lat, s), "neighbour of the same parity");
        }
    int64_t lids[18];
    for (int64_t s = 0; s < nsite; s += 7)
        for (int mu = 0; mu < 4; ++mu) {
            su3ref_staple_lids(lat, s, mu, lids);
            for (int k = 0; k < 18; ++k) CHECK(lids[k] >= 0 && lids[k] < 4 * nsite, "staple link id out of range");
        }
}

static void lattice_case(int L0, int L1, int L2, int L3, int nlat, unsigned flip, int nhit, int hot, double beta)
{
    su3ref_params p = {{L0, L1, L2, L3}, nlat, flip, nhit, 7};
    CHECK(su3ref_check_params(&p) == 0, "valid parameters rejected");
    su3ref_lattice *lat = su3ref_create(&p);
    CHECK(lat != NULL, "create failed");
    if (!lat) return;
    double pl[3], poly[6], A[18];
    su3ref_start(lat, hot);
    su3ref_plaquette(lat, pl);
    if (!hot) CHECK(pl[0] == 1.0, "cold start plaquette %.17g", pl[0]);
    su3ref_sweep(lat, 2, beta, 2, 0);
    su3ref_sweep(lat, 1, beta, 1, 12345); /* shuffled order */
    su3ref_plaquette(lat, pl);
    CHECK(isfinite(pl[0]) && pl[0] > -1.0 && pl[0] < 1.0, "plaquette %.17g", pl[0]);
    const int64_t V = su3ref_volume(lat);
    for (int64_t s = 0; s < V * nlat; s += 5)
        for (int mu = 0; mu < 4; ++mu) {
            su3ref_staple(lat, s, mu, A);
            for (int k = 0; k < 18; ++k) CHECK(isfinite(A[k]), "staple not finite");
            if (nlat == 2) su3ref_staple_betas(lat, s, mu, 5.5, 6.0, A);
        }
    su3ref_reunitarise(lat);
    su3ref_gauge_transform(lat, 3);
    su3ref_polyakov(lat, poly);
    CHECK(isfinite(poly[0]) && isfinite(poly[1]), "Polyakov loop not finite");
    if (nlat == 2) su3ref_sweep_betas(lat, 1, 5.5, 6.0, 2);
    uint64_t att = 0, acc = 0;
    su3ref_counters(lat, &att, &acc);
    CHECK(acc <= att && att > 0, "counters %llu %llu", (unsigned long long)att, (unsigned long long)acc);
    CHECK(su3ref_get_sweeps(lat) == (uint64_t)(nlat == 2 ? 4 : 3), "sweep count");
    su3ref_set_sweeps(lat, 10);
    CHECK(su3ref_n_doubles(lat) == 72 * V * nlat, "n_doubles");
    double *links = su3ref_links(lat);
    for (int64_t k = 0; k < su3ref_n_doubles(lat); ++k) CHECK(isfinite(links[k]), "link not finite");
    geometry_checks(lat, nlat);
    su3ref_destroy(lat);
    su3ref_lattice *geo = su3ref_create_geometry(&p);
    CHECK(geo != NULL, "geometry create failed");
    if (geo) {
        geometry_checks(geo, nlat);
        su3ref_destroy(geo);
    }
}

int main(void)
{
    const su3ref_params bad[] = {{{3, 4, 4, 4}, 1, 0, 1, 1}, {{4, 4, 4, 4}, 3, 0, 1, 1}, {{4, 4, 4, 4}, 1, 1, 1, 1},
                                 {{4, 4, 4, 4}, 2, 0x10, 1, 1}, {{4, 4, 4, 4}, 1, 0, 0, 1}, {{0, 4, 4, 4}, 1, 0, 1, 1}};
    for (size_t k = 0; k < sizeof bad / sizeof bad[0]; ++k) {
        CHECK(su3ref_check_params(&bad[k]) != 0, "invalid parameters %zu accepted", k);
        CHECK(su3ref_create(&bad[k]) == NULL, "invalid lattice %zu created", k);
    }
    lattice_case(4, 4, 4, 4, 1, 0, 1, 1, 5.7);
    lattice_case(2, 2, 2, 2, 1, 0, 1, 1, 5.7);
    lattice_case(6, 4, 10, 2, 1, 0, 3, 1, 0.5);
    lattice_case(4, 4, 4, 6, 2, 0x7, 1, 1, 5.7);
    lattice_case(4, 6, 4, 4, 2, 0xF, 1, 0, 5.7);
    lattice_case(4, 4, 6, 2, 2, 0x0, 2, 1, 50.0);
    lattice_case(6, 4, 4, 4, 2, 0x5, 1, 1, 5.7);

    /* single-link primitives */
    uint64_t ctr[4] = {1, 2, 3, 4}, key[2] = {5, 6}, out[4];
    su3ref_philox4x64(ctr, key, out);
    double U[18], G[18], A[18], nb[18 * 18], a[4 * 1000], obs[200];
    su3ref_hot_link(9, 17, U);
    su3ref_gauge_element(9, 17, G);
    su3ref_reunit(U);
    for (int k = 0; k < 18; ++k) nb[k] = 0.0;
    for (int m = 0; m < 18; ++m) su3ref_hot_link(3, (uint64_t)m, nb + 18 * m);
    su3ref_staple_from_links(nb, A);
    uint64_t cnt[2] = {0, 0};
    su3ref_heatbath_link(U, A, 5.7, 1, 17, 0, 3, cnt);
    CHECK(cnt[1] <= cnt[0] && cnt[0] >= 3, "heat-bath counters");
    int64_t tries = 0;
    const int64_t over = su3ref_kp_draws(2.0, 1, 1000, 100, a, &tries);
    CHECK(over >= 0 && tries >= 1000, "KP draws");
    su3ref_single_link_chain(U, A, 5.7, 1, 200, 1, obs);
    for (int k = 0; k < 200; ++k) CHECK(isfinite(obs[k]), "chain observable");
    printf("oracle sanitizer check: %d failures\n", fails);
    return fails != 0;
}
