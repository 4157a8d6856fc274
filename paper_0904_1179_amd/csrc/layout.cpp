// layout.cpp -- host-side geometry, buffer layout and launch shapes (see
// layout.h).  No HIP calls: everything here is plain arithmetic on the
// parameters, so it is validated before any device work and can be checked
// on the CPU under the address and undefined-behaviour sanitizers.
#include "layout.h"

#include <string>

namespace su3hb {

namespace {
thread_local std::string g_last_error;
long long round_up(long long a, long long m) { return (a + m - 1) / m * m; }
long long ceil_div(long long a, long long b) { return (a + b - 1) / b; }
}  // namespace

su3_status fail(su3_status s, const std::string &msg)
{
    g_last_error = msg;
    return s;
}

const char *last_error() { return g_last_error.c_str(); }

su3_status check_params(const su3_params *p)
{
    if (!p) return fail(SU3_EINVAL, "params is NULL");
    for (int mu = 0; mu < 4; ++mu) {
        const int L = p->L[mu];
        if (L < 2 || L > 1024 || (L & 1))
            return fail(SU3_EINVAL, "L[" + std::to_string(mu) + "] = " + std::to_string(L) +
                                        ": extents must be even and in [2, 1024]");
    }
    if (p->nlat != 1 && p->nlat != 2) return fail(SU3_EINVAL, "nlat must be 1 (torus) or 2 (double-layered torus)");
    if (p->nlat == 1 && p->flip_mask != 0) return fail(SU3_EINVAL, "flip_mask must be 0 when nlat = 1");
    if (p->flip_mask > 0xF) return fail(SU3_EINVAL, "flip_mask has bits above direction 3");
    if (p->precision != 64 && p->precision != 32) return fail(SU3_EINVAL, "precision must be 64 or 32");
    if (p->nhit < 1 || p->nhit > 64) return fail(SU3_EINVAL, "nhit must be in [1, 64]");
    const long long V = (long long)p->L[0] * p->L[1] * p->L[2] * p->L[3];
    if ((long long)p->nlat * V > (1LL << 30))
        return fail(SU3_EINVAL, "lattice too large: nlat*V must not exceed 2^30 sites");
    return SU3_OK;
}

// Domains of the pass order (the (x1, x2) cross-section cut into w1 x w2
// pieces, each swept along x3).  A link on a domain's rim is read by two
// XCDs, each from HBM, so the choice takes the fewest rim links, the sum of
// 1/w over the directions that are cut, among the widths that
//  * give every XCD whole domains: nd * nlat a multiple of 8, nd = (L1/w1)(L2/w2);
//  * keep one x3 slab of a domain within kSlabMax = 4096 updates
//    (L0/2 w1 w2 <= 4096), so that the links around it are re-read while
//    still in L2;
//  * keep the lanes of a wave on whole 16-link tiles: L0/2 w1 a multiple of 16,
//    or w1 = L1.
// Ties go to the wider w1 (longer runs of consecutive links).  Without such
// widths the rule keeps w1 = L1 and the largest w2 <= L2/8.
void pick_domains(const int32_t L[4], int nlat, int &w1, int &w2)
{
    constexpr long long kSlabMax = 4096;
    const int l0h = L[0] / 2;
    double best = 1e30;
    w1 = L[1];
    w2 = 0;
    for (int a = L[1]; a >= 1; --a) {
        if (L[1] % a || (a != L[1] && (l0h * a) % 16)) continue;
        for (int b = L[2]; b >= 1; --b) {
            if (L[2] % b) continue;
            const long long nd = (long long)(L[1] / a) * (L[2] / b) * nlat;
            if (nd % 8 || (long long)l0h * a * b > kSlabMax) continue;
            const double rim = (a < L[1] ? 1.0 / a : 0.0) + (b < L[2] ? 1.0 / b : 0.0);
            if (rim < best - 1e-12) {
                best = rim;
                w1 = a;
                w2 = b;
            }
        }
    }
    if (w2 == 0) {
        w1 = L[1];
        w2 = 1;
        for (int b = 1; b <= L[2] / 8; ++b)
            if (L[2] % b == 0) w2 = b;
    }
}

Geom make_geom(const su3_params *p)
{
    Geom g;
    for (int mu = 0; mu < 4; ++mu) g.L[mu] = p->L[mu];
    const long long V = (long long)p->L[0] * p->L[1] * p->L[2] * p->L[3];
    g.Vh = (int)(V / 2);
    g.nlat = p->nlat;
    g.flip = p->nlat == 2 ? p->flip_mask : 0u;
    // +64: the (direction, parity) blocks are offset by 64 links from a large
    // power-of-two spacing, so equal positions in different blocks do not all
    // fall in the same L2 channel and set
    g.stride = round_up((long long)p->nlat * (V / 2), 64) + 64;
    pick_domains(p->L, p->nlat, g.w1, g.w2);
    g.nd1 = p->L[1] / g.w1;
    g.dl0h = make_fastdiv((uint32_t)(p->L[0] / 2));
    g.dl1 = make_fastdiv((uint32_t)p->L[1]);
    g.dl2 = make_fastdiv((uint32_t)p->L[2]);
    g.dl3 = make_fastdiv((uint32_t)p->L[3]);
    g.dw1 = make_fastdiv((uint32_t)g.w1);
    g.dw2 = make_fastdiv((uint32_t)g.w2);
    g.dnd1 = make_fastdiv((uint32_t)g.nd1);
    return g;
}

size_t link_bytes_of(const su3_params *p, const Geom &g)
{
    // 8 (direction, parity) blocks of `stride` links, 6 complex entries each
    return (size_t)8 * kEntries * (size_t)g.stride * (p->precision == 64 ? 16u : 8u);
}

// Passes of at most kLanes4Max links run with 4 lanes per link, of at most
// kLanes2Max with 2, larger ones with 1.  Measured per pass (FP64): 2048 links
// 11.3 us with 1 lane, 9.3 us with 4; 32768 links about even (FP32: 13.5 vs
// 11 us with 2); 65536 links (2 x 16^4) 19 us with 1 lane, 21 us with 2, whose
// two waves per SIMD then issue 1.6 times the instructions of one.  Per sweep,
// 4 against 2 lanes: 2048 to 5000 links (8^4, 2 x 8^4, 10^4) 76-80 against
// 83-85 us in FP64, even in FP32; 10368 links (12^4) 91 against 86 us in FP64,
// 85 against 76 us in FP32.
constexpr long long kLanes4Max = 8192, kLanes2Max = 32768;

int lanes_per_link(const Geom &g, int nhit, int requested)
{
    if (requested > 0) return requested;
    if (nhit != 1) return 1;
    const long long n = (long long)g.nlat * g.Vh;
    return n <= kLanes4Max ? 4 : (n <= kLanes2Max ? 2 : 1);
}

int pass_links_per_block(const Geom &g, int lanes)
{
    if (lanes > 1) return kBlock / lanes;
    return g.nlat == 1 ? kPassBlock : kBlock;
}

int pass_blocks(const Geom &g, int nb) { return (int)ceil_div((long long)g.nlat * g.Vh, nb); }

int plaq_blocks(const Geom &g)
{
    const long long need = ceil_div(g.Vh, kBlock);
    return (int)(need < kPlaqBlocksMax ? need : kPlaqBlocksMax);
}

// The plaquette walk (one thread per column and chunk of x3, which reads
// each link as an own link and as a neighbour in the same step of the walk)
// takes FP64 lattices with enough columns for one wave per SIMD (65536
// threads on the 1024 SIMDs) in chunks of at least kPlaqWalkMinSteps sites,
// aiming at two waves per SIMD (kPlaqWalkThreads).  Smaller lattices, and
// FP32 links (k_plaq_partial, faster there), take the per-site kernels.
constexpr long long kPlaqWalkThreads = 131072, kPlaqWalkMinThreads = 65536, kPlaqWalkMinSteps = 4;

int plaq_walk_chunks(const Geom &g, int precision)
{
    if (precision != 64) return 0;
    const long long cols = (long long)g.nlat * g.L[0] * g.L[1] * g.L[2];
    long long nch = ceil_div(kPlaqWalkThreads, cols);
    if (nch > g.L[3] / kPlaqWalkMinSteps) nch = g.L[3] / kPlaqWalkMinSteps;
    return nch >= 1 && cols * nch >= kPlaqWalkMinThreads ? (int)nch : 0;
}

int plaq_walk_blocks(const Geom &g, int nch)
{
    const long long need = ceil_div((long long)g.L[0] * g.L[1] * g.L[2] * nch, kPlaqWalkBlock);
    const int most = plaq_blocks(g);
    return (int)(need < most ? need : most);
}

int meas_blocks(const Geom &g, int lanes) { return pass_blocks(g, pass_links_per_block(g, lanes)); }

// the most workgroups a measured pass can have: 64 links per workgroup
// (one lane per link on a single torus, or 4 lanes per link)
static int meas_blocks_max(const Geom &g) { return pass_blocks(g, 64); }

int polyakov_blocks(const Geom &g) { return (int)ceil_div((long long)g.L[0] * g.L[1] * g.L[2], kBlock); }

// plaquette partials: per layer and workgroup the plaquette sum, then the
// number of links that fail the unitarity check
size_t meas_offset(const Geom &g) { return (size_t)round_up(kOffPartials + 2 * 8LL * g.nlat * plaq_blocks(g), 256); }

// measured-pass partials: 3 passes x nlat doubles per workgroup
size_t polyakov_offset(const Geom &g)
{
    return (size_t)round_up((long long)meas_offset(g) + 3 * 8LL * g.nlat * meas_blocks_max(g), 256);
}

size_t scratch_bytes_of(const Geom &g)
{
    return (size_t)round_up((long long)polyakov_offset(g) + 16LL * g.nlat * polyakov_blocks(g), 256);
}

size_t dev_index(const Geom &g, int dir, int par, int e, long long n)
{
    return (size_t)(dir * 2 + par) * (size_t)g.stride * kEntries + (size_t)(n >> 4) * (kEntries * kTile) +
           (size_t)e * kTile + (size_t)(n & (kTile - 1));
}

long long site_of_elem(const Geom &g, int par, long long n)
{
    const int layer = n >= g.Vh ? 1 : 0;
    const long long i = n - (long long)layer * g.Vh;
    const int l0h = g.L[0] / 2;
    long long r = i / l0h;
    const int x0h = (int)(i - r * l0h);
    const int x1 = (int)(r % g.L[1]);
    r /= g.L[1];
    const int x2 = (int)(r % g.L[2]);
    const int x3 = (int)(r / g.L[2]);
    const int x0 = 2 * x0h + ((par + x1 + x2 + x3) & 1);
    const long long lex = x0 + (long long)g.L[0] * (x1 + (long long)g.L[1] * (x2 + (long long)g.L[2] * x3));
    return (long long)layer * 2LL * g.Vh + lex;
}

bool elem_of_lid(const Geom &g, uint64_t lid, int *dir, int *par, long long *n)
{
    const uint64_t V = 2ull * (uint64_t)g.Vh;
    if (lid >= 4ull * V * (uint64_t)g.nlat) return false;
    const uint64_t site = lid / 4;
    *dir = (int)(lid % 4);
    const uint64_t layer = site / V;
    const uint64_t lex = site % V;
    uint64_t r = lex;
    int sum = 0;
    for (int mu = 0; mu < 4; ++mu) {
        sum += (int)(r % (uint64_t)g.L[mu]);
        r /= (uint64_t)g.L[mu];
    }
    *par = sum & 1;
    *n = (long long)(layer * (uint64_t)g.Vh + (lex >> 1));
    return true;
}

void rebuild_row2_host(double *m)
{
    for (int k = 0; k < 3; ++k) {
        const int a = (k + 1) % 3, b = (k + 2) % 3;
        const double p_re = m[2 * a] * m[6 + 2 * b] - m[2 * a + 1] * m[6 + 2 * b + 1];
        const double p_im = m[2 * a] * m[6 + 2 * b + 1] + m[2 * a + 1] * m[6 + 2 * b];
        const double q_re = m[2 * b] * m[6 + 2 * a] - m[2 * b + 1] * m[6 + 2 * a + 1];
        const double q_im = m[2 * b] * m[6 + 2 * a + 1] + m[2 * b + 1] * m[6 + 2 * a];
        m[12 + 2 * k] = p_re - q_re;
        m[12 + 2 * k + 1] = -(p_im - q_im);
    }
}

void unpack_links(int precision, const Geom &g, const void *image, double *host)
{
    const long long nelem = (long long)g.nlat * g.Vh;
    for (int par = 0; par < 2; ++par)
        for (long long n = 0; n < nelem; ++n) {
            const long long site = site_of_elem(g, par, n);
            for (int dir = 0; dir < 4; ++dir) {
                double *dst = host + (size_t)(4 * site + dir) * 18;
                for (int el = 0; el < kEntries; ++el) {
                    const size_t idx = dev_index(g, dir, par, el, n);
                    if (precision == 64) {
                        const double *v = (const double *)image + 2 * idx;
                        dst[2 * el] = v[0];
                        dst[2 * el + 1] = v[1];
                    } else {
                        const float *v = (const float *)image + 2 * idx;
                        dst[2 * el] = (double)v[0];
                        dst[2 * el + 1] = (double)v[1];
                    }
                }
                rebuild_row2_host(dst);
            }
        }
}

void pack_links(int precision, const Geom &g, const double *host, void *image)
{
    const long long nelem = (long long)g.nlat * g.Vh;
    for (int par = 0; par < 2; ++par)
        for (long long n = 0; n < nelem; ++n) {
            const long long site = site_of_elem(g, par, n);
            for (int dir = 0; dir < 4; ++dir) {
                const double *src = host + (size_t)(4 * site + dir) * 18;
                for (int el = 0; el < kEntries; ++el) {
                    const size_t idx = dev_index(g, dir, par, el, n);
                    if (precision == 64) {
                        double *v = (double *)image + 2 * idx;
                        v[0] = src[2 * el];
                        v[1] = src[2 * el + 1];
                    } else {
                        float *v = (float *)image + 2 * idx;
                        v[0] = (float)src[2 * el];
                        v[1] = (float)src[2 * el + 1];
                    }
                }
            }
        }
}

}  // namespace su3hb
