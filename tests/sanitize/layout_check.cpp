// Host-side layout code of the library (paper_0904_1179_amd/csrc/layout.cpp)
// under the address and undefined-behaviour sanitizers: parameter validation,
// the pass order's domains, invariant division, buffer sizes and scratch
// offsets, the index maps between the tiled store and canonical link ids,
// the column order of the plaquette walk, and the link packing round trip.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <set>
#include <vector>

#include "../../paper_0904_1179_amd/csrc/layout.h"

using namespace su3hb;

static int fails = 0;
#define CHECK(c, ...)                                                 \
    do {                                                              \
        if (!(c)) {                                                   \
            std::fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__); \
            std::fprintf(stderr, __VA_ARGS__);                        \
            std::fprintf(stderr, "\n");                               \
            ++fails;                                                  \
        }                                                             \
    } while (0)

static su3_params params(int L0, int L1, int L2, int L3, int nlat, unsigned flip, int prec, int nhit = 1)
{
    su3_params p;
    p.L[0] = L0;
    p.L[1] = L1;
    p.L[2] = L2;
    p.L[3] = L3;
    p.nlat = nlat;
    p.flip_mask = flip;
    p.precision = prec;
    p.nhit = nhit;
    p.seed = 1;
    return p;
}

static void check_div(const FastDiv &f, std::mt19937_64 &rng)
{
    for (uint32_t x = 0; x < 70000; ++x) CHECK((uint32_t)div_by((int)x, f) == x / f.d, "div %u / %u", x, f.d);
    for (int k = 0; k < 20000; ++k) {
        const uint32_t x = (uint32_t)(rng() & 0x7fffffffu);
        CHECK((uint32_t)div_by((int)x, f) == x / f.d, "div %u / %u", x, f.d);
    }
}

// geometry, sizes and launch shapes at any size (nothing allocated per site)
static void geometry_case(const su3_params &p, std::mt19937_64 &rng)
{
    CHECK(check_params(&p) == SU3_OK, "valid parameters rejected: %s", last_error());
    const Geom g = make_geom(&p);
    CHECK(p.L[1] % g.w1 == 0 && p.L[2] % g.w2 == 0, "domain widths do not divide the extents");
    CHECK(g.nd1 * g.w1 == p.L[1], "nd1");
    const long long nlinks = (long long)g.nlat * g.Vh;
    CHECK(g.stride % 64 == 0 && g.stride >= nlinks + 64, "stride");
    for (const FastDiv *f : {&g.dl0h, &g.dl1, &g.dl2, &g.dl3, &g.dw1, &g.dw2, &g.dnd1}) check_div(*f, rng);
    const size_t esz = p.precision == 64 ? 16 : 8;
    CHECK(link_bytes_of(&p, g) == (size_t)8 * kEntries * (size_t)g.stride * esz, "link bytes");
    CHECK(meas_offset(g) >= kOffPartials + 2 * 8 * (size_t)g.nlat * plaq_blocks(g), "plaquette partials overlap");
    for (int lanes : {1, 2, 4}) {
        CHECK((long long)meas_blocks(g, lanes) * pass_links_per_block(g, lanes) >= nlinks, "measured pass too small");
        CHECK(meas_offset(g) + 3 * 8 * (size_t)g.nlat * meas_blocks(g, lanes) <= polyakov_offset(g),
              "measured partials overlap the Polyakov partials (lanes %d)", lanes);
    }
    CHECK(polyakov_offset(g) + 16 * (size_t)g.nlat * polyakov_blocks(g) <= scratch_bytes_of(g), "scratch size");
    const int lanes = lanes_per_link(g, p.nhit, 0);
    CHECK(lanes == 1 || lanes == 2 || lanes == 4, "lanes %d", lanes);
    if (p.nhit != 1) CHECK(lanes == 1, "several lanes with nhit > 1");
}

// index maps and packing on lattices small enough to enumerate
static void layout_case(const su3_params &p, std::mt19937_64 &rng)
{
    const Geom g = make_geom(&p);
    const long long V = 2LL * g.Vh, nsite = V * g.nlat, nlinks = (long long)g.nlat * g.Vh;
    std::vector<char> seen((size_t)nsite, 0);
    for (int par = 0; par < 2; ++par)
        for (long long n = 0; n < nlinks; ++n) {
            const long long site = site_of_elem(g, par, n);
            CHECK(site >= 0 && site < nsite, "site out of range");
            if (site < 0 || site >= nsite) continue;
            CHECK(!seen[(size_t)site], "site reached twice");
            seen[(size_t)site] = 1;
            long long lex = site % V;
            int x[4], sum = 0;
            for (int mu = 0; mu < 4; ++mu) {
                x[mu] = (int)(lex % p.L[mu]);
                lex /= p.L[mu];
                sum += x[mu];
            }
            CHECK((sum & 1) == par, "parity");
            for (int dir = 0; dir < 4; ++dir) {
                int d2, p2;
                long long n2;
                CHECK(elem_of_lid(g, (uint64_t)(4 * site + dir), &d2, &p2, &n2), "lid rejected");
                CHECK(d2 == dir && p2 == par && n2 == n, "elem_of_lid does not invert site_of_elem");
            }
        }
    int d_, p_;
    long long n_;
    CHECK(!elem_of_lid(g, (uint64_t)(4 * nsite), &d_, &p_, &n_), "lid out of range accepted");
    const size_t esz = p.precision == 64 ? 16 : 8, nelem = link_bytes_of(&p, g) / esz;
    std::set<size_t> idx;
    for (int dir = 0; dir < 4; ++dir)
        for (int par = 0; par < 2; ++par)
            for (int e = 0; e < kEntries; ++e)
                for (long long n = 0; n < nlinks; ++n) {
                    const size_t i = dev_index(g, dir, par, e, n);
                    CHECK(i < nelem, "device index out of range");
                    idx.insert(i);
                }
    CHECK(idx.size() == (size_t)8 * kEntries * nlinks, "device indices collide");
    // pack / unpack: rows 0, 1 random, row 2 = conj(row 0 x row 1) as rebuild_row2_host forms it
    std::vector<double> host((size_t)72 * nsite), back(host.size());
    std::normal_distribution<double> nd;
    for (size_t l = 0; l < host.size() / 18; ++l) {
        for (int k = 0; k < 12; ++k) host[18 * l + k] = nd(rng);
        rebuild_row2_host(&host[18 * l]);
    }
    if (p.precision == 32)  // the stored rows are FP32
        for (size_t l = 0; l < host.size() / 18; ++l) {
            for (int k = 0; k < 12; ++k) host[18 * l + k] = (double)(float)host[18 * l + k];
            rebuild_row2_host(&host[18 * l]);
        }
    std::vector<unsigned char> image(link_bytes_of(&p, g), 0);
    pack_links(p.precision, g, host.data(), image.data());
    unpack_links(p.precision, g, image.data(), back.data());
    bool same = true;
    for (size_t k = 0; k < host.size(); ++k) same = same && host[k] == back[k];
    CHECK(same, "pack/unpack round trip differs");
}

// the plaquette walk: every (column, chunk) exactly once, chunks partitioning
// x3, and a grid that covers the threads within the partials' room
static void walk_case(const su3_params &p, int nch)
{
    const Geom g = make_geom(&p);
    const long long cols = (long long)p.L[0] * p.L[1] * p.L[2], n = cols * nch;
    std::vector<char> seen((size_t)n, 0);
    for (long long w = 0; w < n; ++w) {
        int x[3] = {-1, -1, -1};
        const int c = walk_column(g, nch, (int)w, x);
        const bool ok = c >= 0 && c < nch && x[0] >= 0 && x[0] < p.L[0] && x[1] >= 0 && x[1] < p.L[1] && x[2] >= 0 &&
                        x[2] < p.L[2];
        CHECK(ok, "walk_column out of range at w = %lld", w);
        if (!ok) continue;
        const long long k = (long long)c * cols + x[0] + (long long)p.L[0] * (x[1] + (long long)p.L[1] * x[2]);
        CHECK(!seen[(size_t)k], "walk_column reaches a column and chunk twice");
        seen[(size_t)k] = 1;
    }
    long long covered = 0;
    for (int c = 0; c < nch; ++c) {
        const long long a = (long long)c * p.L[3] / nch, b = (long long)(c + 1) * p.L[3] / nch;
        CHECK(a == covered && b > a, "chunk %d of %d", c, nch);
        covered = b;
    }
    CHECK(covered == p.L[3], "chunks do not cover x3");
    const int nblk = plaq_walk_blocks(g, nch);
    const long long tiles = (n + kPlaqWalkBlock - 1) / kPlaqWalkBlock, tpb = (tiles + nblk - 1) / nblk;
    CHECK(nblk >= 1 && nblk <= plaq_blocks(g), "walk workgroups %d, room for %d", nblk, plaq_blocks(g));
    CHECK(tpb * nblk * kPlaqWalkBlock >= n, "walk grid does not cover its threads");
}

int main()
{
    std::mt19937_64 rng(1);
    const su3_params bad[] = {params(3, 4, 4, 4, 1, 0, 64),      params(4, 4, 4, 4, 3, 0, 64),
                              params(4, 4, 4, 4, 1, 1, 64),      params(4, 4, 4, 4, 2, 0x10, 64),
                              params(4, 4, 4, 4, 1, 0, 16),      params(4, 4, 4, 4, 1, 0, 64, 0),
                              params(4, 4, 4, 4, 1, 0, 64, 65),  params(2048, 2, 2, 2, 1, 0, 64),
                              params(1024, 1024, 1024, 2, 1, 0, 32)};
    for (const su3_params &p : bad) {
        CHECK(check_params(&p) == SU3_EINVAL, "invalid parameters accepted");
        CHECK(last_error()[0] != '\0', "no error text");
    }
    CHECK(check_params(nullptr) == SU3_EINVAL, "NULL parameters accepted");
    const su3_params small[] = {params(2, 2, 2, 2, 1, 0, 64),    params(4, 4, 4, 4, 1, 0, 64),
                                params(6, 4, 10, 2, 1, 0, 64),   params(8, 8, 8, 8, 1, 0, 32),
                                params(4, 4, 4, 6, 2, 0x7, 64),  params(4, 6, 4, 4, 2, 0xF, 32),
                                params(4, 6, 24, 6, 1, 0, 64, 3), params(6, 10, 24, 2, 2, 0x7, 64)};
    for (const su3_params &p : small) {
        geometry_case(p, rng);
        layout_case(p, rng);
    }
    const su3_params large[] = {params(32, 32, 32, 32, 1, 0, 64), params(64, 64, 64, 64, 1, 0, 32),
                                params(16, 16, 16, 16, 2, 0x7, 64), params(256, 256, 128, 128, 1, 0, 32),
                                params(1024, 2, 2, 256, 2, 0x3, 64)};
    for (const su3_params &p : large) geometry_case(p, rng);
    // plaquette walk: the chunk counts the library picks, and forced ones on
    // small and ragged lattices
    for (const su3_params &p : large) {
        const Geom g = make_geom(&p);
        for (int prec : {64, 32}) {
            const int nch = plaq_walk_chunks(g, prec);
            if (p.L[0] == 16) CHECK(nch == 0, "2 x 16^4 walks");
            if (p.L[0] == 32) CHECK(nch == (prec == 64 ? 4 : 0), "32^4 walks in %d chunks", nch);
            if (nch > 0) {
                CHECK(p.L[3] / nch >= 4, "chunks shorter than 4 sites");
                walk_case(p, nch);
            }
        }
    }
    for (const su3_params &p : small)
        for (int nch = 1; nch <= p.L[3]; ++nch) walk_case(p, nch);
    // invariant division: every divisor up to 4096 on dividends around its multiples
    for (uint32_t d = 1; d <= 4096; ++d) {
        const FastDiv f = make_fastdiv(d);
        for (uint32_t q = 0; q < 64; ++q)
            for (int k = -1; k <= 1; ++k) {
                const long long x = (long long)q * d + k;
                if (x >= 0) CHECK((uint32_t)div_by((int)x, f) == (uint32_t)x / d, "div %lld / %u", x, d);
            }
        const uint32_t top = 0x7fffffffu - 0x7fffffffu % d;
        CHECK((uint32_t)div_by((int)top, f) == top / d, "div at the top of the range / %u", d);
    }
    std::printf("layout sanitizer check: %d failures\n", fails);
    return fails != 0;
}
