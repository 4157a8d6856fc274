/*
 * su3ref.c -- plain FP64 CPU oracle for the checkerboard SU(3) heat-bath sweep.
 *
 * TEST INFRASTRUCTURE ONLY (see su3ref.h).  Written for readability, not
 * speed: explicit 3x3 complex loops, no blocking, no SIMD, built with
 * -O2 -ffp-contract=off so that every product and sum is rounded as written.
 *
 * The paper (Berg & Wu, "... SU(3) Lattice Gauge Theory II") states which
 * computation is timed -- nequi checkerboard updating sweeps of pure SU(3)
 * LGT with the Wilson action, on PBC or DLT lattices, with a 1-hit heat bath
 * (Sec. 1; Sec. 2, eq. (1); Sec. 2.1) -- but none of its formulas; those live
 * in its predecessor.  Each function below therefore states the textbook
 * definition it implements:
 *   Wilson action   S = beta * sum_P (1 - 1/3 Re Tr U_P)
 *   heat bath       Cabibbo & Marinari, Phys. Lett. B119 (1982) 387: SU(2)
 *                   subgroups (0,1), (1,2), (0,2) updated in turn;
 *                   Kennedy & Pendleton, Phys. Lett. B156 (1985) 393: the
 *                   SU(2) sampler, one attempt per subgroup ("1-hit")
 *   random numbers  Philox4x64-10, Salmon, Moraes, Dror & Shaw, SC'11
 *   Haar start      Box-Muller normals + Gram-Schmidt of two complex rows
 * Readings where the paper is silent (subgroup order, counter layout, DLT
 * gluing, uniform mapping) are fixed here and listed in the design notes.
 */
#include "su3ref.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* complex numbers and 3x3 complex matrices                                   */
/* ------------------------------------------------------------------------ */

typedef struct { double re, im; } cplx;
typedef struct { cplx m[3][3]; } mat3;

static cplx c_add(cplx a, cplx b) { cplx r = {a.re + b.re, a.im + b.im}; return r; }
static cplx c_sub(cplx a, cplx b) { cplx r = {a.re - b.re, a.im - b.im}; return r; }
static cplx c_mul(cplx a, cplx b)
{
    cplx r = {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
    return r;
}
static cplx c_conj(cplx a) { cplx r = {a.re, -a.im}; return r; }
static cplx c_scale(cplx a, double s) { cplx r = {a.re * s, a.im * s}; return r; }
static double c_abs2(cplx a) { return a.re * a.re + a.im * a.im; }

static mat3 m_load(const double *p)
{
    mat3 u;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            u.m[a][b].re = p[(3 * a + b) * 2 + 0];
            u.m[a][b].im = p[(3 * a + b) * 2 + 1];
        }
    return u;
}

static void m_store(const mat3 *u, double *p)
{
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            p[(3 * a + b) * 2 + 0] = u->m[a][b].re;
            p[(3 * a + b) * 2 + 1] = u->m[a][b].im;
        }
}

static mat3 m_identity(void)
{
    mat3 u;
    memset(&u, 0, sizeof u);
    for (int a = 0; a < 3; ++a) u.m[a][a].re = 1.0;
    return u;
}

/* (A B)_ab = sum_c A_ac B_cb */
static mat3 m_mul(const mat3 *A, const mat3 *B)
{
    mat3 C;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            cplx s = c_mul(A->m[a][0], B->m[0][b]);
            s = c_add(s, c_mul(A->m[a][1], B->m[1][b]));
            s = c_add(s, c_mul(A->m[a][2], B->m[2][b]));
            C.m[a][b] = s;
        }
    return C;
}

static mat3 m_dag(const mat3 *A)
{
    mat3 C;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) C.m[a][b] = c_conj(A->m[b][a]);
    return C;
}

static mat3 m_add(const mat3 *A, const mat3 *B)
{
    mat3 C;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) C.m[a][b] = c_add(A->m[a][b], B->m[a][b]);
    return C;
}

static double m_retrace(const mat3 *A) { return A->m[0][0].re + A->m[1][1].re + A->m[2][2].re; }

/* ------------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon et al., SC'11): ten rounds of two 64x64->128-bit     */
/* multiplies; round constants and Weyl key increments as published there.    */
/* ------------------------------------------------------------------------ */

#define PHILOX_M0 0xD2E7470EE14C6C93ULL
#define PHILOX_M1 0xCA5A826395121157ULL
#define PHILOX_W0 0x9E3779B97F4A7C15ULL
#define PHILOX_W1 0xBB67AE8584CAA73BULL

void su3ref_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        unsigned __int128 p0 = (unsigned __int128)PHILOX_M0 * x0;
        unsigned __int128 p1 = (unsigned __int128)PHILOX_M1 * x2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t y0 = hi1 ^ x1 ^ k0;
        uint64_t y1 = lo1;
        uint64_t y2 = hi0 ^ x3 ^ k1;
        uint64_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Counter word 3 tags the purpose of a draw, so streams never overlap. */
enum { TAG_HEATBATH = 0, TAG_HOT = 1, TAG_GAUGE = 2 };

/* Uniform in (0,1) from the top 52 bits: (k + 1/2) 2^-52, exact in FP64. */
static double u52(uint64_t w) { return ((double)(w >> 12) + 0.5) * 0x1p-52; }
/* Uniform in (0,1) from a 32-bit half: (h + 1/2) 2^-32, exact in FP64. */
static double u32(uint32_t h) { return ((double)h + 0.5) * 0x1p-32; }

static const double TWO_PI = 6.283185307179586476925286766559;

/* ------------------------------------------------------------------------ */
/* Haar-random SU(3) element from 12 Gaussian reals (Box-Muller):             */
/* rows r0, r1 complex Gaussian, r0 normalised, r1 orthogonalised against r0  */
/* and normalised, r2 = conj(r0 x r1) so that det = 1.                        */
/* ------------------------------------------------------------------------ */

static void reunit_rows(mat3 *u)
{
    cplx *r0 = u->m[0], *r1 = u->m[1], *r2 = u->m[2];
    double n0 = sqrt(c_abs2(r0[0]) + c_abs2(r0[1]) + c_abs2(r0[2]));
    for (int k = 0; k < 3; ++k) { r0[k].re = r0[k].re / n0; r0[k].im = r0[k].im / n0; }
    /* d = <r0, r1> = sum_k conj(r0_k) r1_k */
    cplx d = c_mul(c_conj(r0[0]), r1[0]);
    d = c_add(d, c_mul(c_conj(r0[1]), r1[1]));
    d = c_add(d, c_mul(c_conj(r0[2]), r1[2]));
    for (int k = 0; k < 3; ++k) r1[k] = c_sub(r1[k], c_mul(d, r0[k]));
    double n1 = sqrt(c_abs2(r1[0]) + c_abs2(r1[1]) + c_abs2(r1[2]));
    for (int k = 0; k < 3; ++k) { r1[k].re = r1[k].re / n1; r1[k].im = r1[k].im / n1; }
    r2[0] = c_conj(c_sub(c_mul(r0[1], r1[2]), c_mul(r0[2], r1[1])));
    r2[1] = c_conj(c_sub(c_mul(r0[2], r1[0]), c_mul(r0[0], r1[2])));
    r2[2] = c_conj(c_sub(c_mul(r0[0], r1[1]), c_mul(r0[1], r1[0])));
}

void su3ref_reunit(double *U)
{
    mat3 u = m_load(U);
    reunit_rows(&u);
    m_store(&u, U);
}

/* Haar element keyed by (seed; id, 0, draw, tag). */
static mat3 haar_su3(uint64_t seed, uint64_t id, uint64_t tag)
{
    double g[12];
    uint64_t key[2] = {seed, 0};
    for (int d = 0; d < 3; ++d) {
        uint64_t ctr[4] = {id, 0, (uint64_t)d, tag}, w[4];
        su3ref_philox4x64(ctr, key, w);
        for (int pair = 0; pair < 2; ++pair) {
            double ua = u52(w[2 * pair]), ub = u52(w[2 * pair + 1]);
            double r = sqrt(-2.0 * log(ua));
            g[4 * d + 2 * pair + 0] = r * cos(TWO_PI * ub);
            g[4 * d + 2 * pair + 1] = r * sin(TWO_PI * ub);
        }
    }
    mat3 u;
    memset(&u, 0, sizeof u);
    for (int k = 0; k < 3; ++k) {
        u.m[0][k].re = g[2 * k];
        u.m[0][k].im = g[2 * k + 1];
        u.m[1][k].re = g[6 + 2 * k];
        u.m[1][k].im = g[6 + 2 * k + 1];
    }
    reunit_rows(&u);
    return u;
}

void su3ref_hot_link(uint64_t seed, uint64_t lid, double *U)
{
    mat3 u = haar_su3(seed, lid, TAG_HOT);
    m_store(&u, U);
}

void su3ref_gauge_element(uint64_t gseed, uint64_t site, double *g)
{
    mat3 u = haar_su3(gseed, site, TAG_GAUGE);
    m_store(&u, g);
}

/* ------------------------------------------------------------------------ */
/* Lattice geometry.  site = layer*V + lex, lex = x0 + L0(x1 + L1(x2 + L2 x3)).*/
/* Parity = (x0+x1+x2+x3) mod 2.  x +- mu wraps mod L_mu; on a DLT (nlat=2) a  */
/* wrap across the mu boundary with bit mu of flip_mask set also switches the  */
/* layer.  The paper names the DLT geometry (Sec. 1; Table 1, nlat=2) but its  */
/* gluing is defined elsewhere; this is the reading used throughout.           */
/* ------------------------------------------------------------------------ */

struct su3ref_lattice {
    su3ref_params p;
    int64_t V;
    double *links;
    uint64_t sweeps;
    uint64_t attempts, accepts;
};

int su3ref_check_params(const su3ref_params *p)
{
    if (!p) return -1;
    for (int mu = 0; mu < 4; ++mu)
        if (p->L[mu] < 2 || (p->L[mu] & 1) || p->L[mu] > 4096) return -1;
    if (p->nlat != 1 && p->nlat != 2) return -1;
    if (p->nlat == 1 && p->flip_mask != 0) return -1;
    if (p->flip_mask > 0xF) return -1;
    if (p->nhit < 1) return -1;
    int64_t V = (int64_t)p->L[0] * p->L[1] * p->L[2] * p->L[3];
    if (V * p->nlat * 4 > ((int64_t)1 << 40)) return -1;
    return 0;
}

int64_t su3ref_volume(const su3ref_lattice *lat) { return lat->V; }

static void site_coords(const su3ref_lattice *lat, int64_t site, int x[4], int *layer)
{
    int64_t lex = site % lat->V;
    *layer = (int)(site / lat->V);
    for (int mu = 0; mu < 4; ++mu) {
        x[mu] = (int)(lex % lat->p.L[mu]);
        lex /= lat->p.L[mu];
    }
}

static int64_t coords_site(const su3ref_lattice *lat, const int x[4], int layer)
{
    const int32_t *L = lat->p.L;
    int64_t lex = x[0] + (int64_t)L[0] * (x[1] + (int64_t)L[1] * (x[2] + (int64_t)L[2] * x[3]));
    return layer * lat->V + lex;
}

int64_t su3ref_neighbor(const su3ref_lattice *lat, int64_t site, int mu, int dir)
{
    int x[4], layer;
    site_coords(lat, site, x, &layer);
    int L = lat->p.L[mu];
    int wrapped = 0;
    if (dir > 0) {
        x[mu] += 1;
        if (x[mu] == L) { x[mu] = 0; wrapped = 1; }
    } else {
        x[mu] -= 1;
        if (x[mu] < 0) { x[mu] = L - 1; wrapped = 1; }
    }
    if (wrapped && lat->p.nlat == 2 && ((lat->p.flip_mask >> mu) & 1u)) layer = 1 - layer;
    return coords_site(lat, x, layer);
}

int su3ref_parity(const su3ref_lattice *lat, int64_t site)
{
    int x[4], layer;
    site_coords(lat, site, x, &layer);
    return (x[0] + x[1] + x[2] + x[3]) & 1;
}

static double *link_ptr(const su3ref_lattice *lat, int64_t site, int mu)
{
    return lat->links + (4 * site + mu) * 18;
}

/* ------------------------------------------------------------------------ */
/* Staple: the Wilson action makes the weight of link U = U_mu(x), with all   */
/* other links fixed, proportional to exp((beta/3) Re Tr(U A)) with           */
/*   A = sum_{nu != mu} [ U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+                   */
/*                      + U_nu(x+mu-nu)^+ U_mu(x-nu)^+ U_nu(x-nu) ].          */
/* The 18 neighbour links, for nu ascending over nu != mu, are:               */
/*   U_nu(x+mu), U_mu(x+nu), U_nu(x), U_nu(x+mu-nu), U_mu(x-nu), U_nu(x-nu).  */
/* ------------------------------------------------------------------------ */

void su3ref_staple_lids(const su3ref_lattice *lat, int64_t site, int mu, int64_t *lids)
{
    int k = 0;
    int64_t xpmu = su3ref_neighbor(lat, site, mu, +1);
    for (int nu = 0; nu < 4; ++nu) {
        if (nu == mu) continue;
        int64_t xpnu = su3ref_neighbor(lat, site, nu, +1);
        int64_t xmnu = su3ref_neighbor(lat, site, nu, -1);
        int64_t xpmu_mnu = su3ref_neighbor(lat, xpmu, nu, -1);
        lids[k++] = 4 * xpmu + nu;
        lids[k++] = 4 * xpnu + mu;
        lids[k++] = 4 * site + nu;
        lids[k++] = 4 * xpmu_mnu + nu;
        lids[k++] = 4 * xmnu + mu;
        lids[k++] = 4 * xmnu + nu;
    }
}

void su3ref_staple_from_links(const double *nb, double *Aout)
{
    mat3 A;
    memset(&A, 0, sizeof A);
    for (int j = 0; j < 3; ++j) {
        const double *q = nb + 6 * 18 * j;
        mat3 a = m_load(q + 0 * 18);   /* U_nu(x+mu)     */
        mat3 b = m_load(q + 1 * 18);   /* U_mu(x+nu)     */
        mat3 c = m_load(q + 2 * 18);   /* U_nu(x)        */
        mat3 d = m_load(q + 3 * 18);   /* U_nu(x+mu-nu)  */
        mat3 e = m_load(q + 4 * 18);   /* U_mu(x-nu)     */
        mat3 f = m_load(q + 5 * 18);   /* U_nu(x-nu)     */
        mat3 bd = m_dag(&b), cd = m_dag(&c), dd = m_dag(&d), ed = m_dag(&e);
        mat3 t = m_mul(&a, &bd);
        mat3 upper = m_mul(&t, &cd);
        mat3 s = m_mul(&dd, &ed);
        mat3 lower = m_mul(&s, &f);
        A = m_add(&A, &upper);
        A = m_add(&A, &lower);
    }
    m_store(&A, Aout);
}

/* Staple with per-layer couplings (double-layered torus with two betas): the
 * action is S = sum_P beta_{layer(P)} (1 - 1/3 Re Tr U_P), a plaquette taking
 * the coupling of the layer of its base site.  The upper staple in plane
 * (mu,nu) belongs to the plaquette based at x, the lower one to the plaquette
 * based at x - nu; each enters A with its coupling, and the link weight is
 * exp(1/3 Re Tr(U A)). */
static void staple_betas(const su3ref_lattice *lat, int64_t site, int mu, const double beta[2], double *Aout)
{
    int64_t lids[18];
    su3ref_staple_lids(lat, site, mu, lids);
    mat3 A;
    memset(&A, 0, sizeof A);
    int layer_x = (int)(site / lat->V);
    int j = 0;
    for (int nu = 0; nu < 4; ++nu) {
        if (nu == mu) continue;
        const int64_t *q = lids + 6 * j;
        mat3 a = m_load(lat->links + q[0] * 18), b = m_load(lat->links + q[1] * 18), c = m_load(lat->links + q[2] * 18);
        mat3 d = m_load(lat->links + q[3] * 18), e = m_load(lat->links + q[4] * 18), f = m_load(lat->links + q[5] * 18);
        mat3 bd = m_dag(&b), cd = m_dag(&c), dd = m_dag(&d), ed = m_dag(&e);
        mat3 t = m_mul(&a, &bd);
        mat3 upper = m_mul(&t, &cd);
        mat3 u2 = m_mul(&dd, &ed);
        mat3 lower = m_mul(&u2, &f);
        int layer_lo = (int)(su3ref_neighbor(lat, site, nu, -1) / lat->V);
        for (int r = 0; r < 3; ++r)
            for (int cc = 0; cc < 3; ++cc) {
                A.m[r][cc] = c_add(A.m[r][cc], c_scale(upper.m[r][cc], beta[layer_x]));
                A.m[r][cc] = c_add(A.m[r][cc], c_scale(lower.m[r][cc], beta[layer_lo]));
            }
        ++j;
    }
    m_store(&A, Aout);
}

void su3ref_staple_betas(const su3ref_lattice *lat, int64_t site, int mu, double beta0, double beta1, double *A)
{
    double b[2] = {beta0, beta1};
    staple_betas(lat, site, mu, b, A);
}

void su3ref_staple(const su3ref_lattice *lat, int64_t site, int mu, double *A)
{
    int64_t lids[18];
    double nb[18 * 18];
    su3ref_staple_lids(lat, site, mu, lids);
    for (int k = 0; k < 18; ++k) memcpy(nb + 18 * k, lat->links + lids[k] * 18, 18 * sizeof(double));
    su3ref_staple_from_links(nb, A);
}

/* ------------------------------------------------------------------------ */
/* Kennedy-Pendleton attempt: given alpha and four uniforms, propose           */
/* lambda^2 = -(ln u1 + cos^2(2 pi u2) ln u3) / (2 alpha) and accept iff       */
/* u4^2 <= 1 - lambda^2; then a0 = 1 - 2 lambda^2 has density                  */
/* proportional to sqrt(1 - a0^2) exp(alpha a0) on [-1, 1].                    */
/* Direction: cos(theta) = 2 u5 - 1, phi = 2 pi u6, |a_vec| = sqrt(1 - a0^2).  */
/* Uniforms of heat-bath attempt t of subgroup sub of link lid in sweep s come */
/* from one Philox call with counter (lid, s, sub*2^32 + t, TAG_HEATBATH):     */
/*   u1 = u52(w0), u3 = u52(w1), u2 = u32(lo w2), u4 = u32(hi w2),             */
/*   u5 = u32(lo w3), u6 = u32(hi w3).                                          */
/* ------------------------------------------------------------------------ */

static int kp_attempt(double alpha, const uint64_t w[4], double a[4])
{
    double u1 = u52(w[0]);
    double u3 = u52(w[1]);
    double u2 = u32((uint32_t)(w[2] & 0xffffffffu));
    double u4 = u32((uint32_t)(w[2] >> 32));
    double u5 = u32((uint32_t)(w[3] & 0xffffffffu));
    double u6 = u32((uint32_t)(w[3] >> 32));
    double c = cos(TWO_PI * u2);
    double lam2 = -(log(u1) + c * c * log(u3)) / (2.0 * alpha);
    if (!(u4 * u4 <= 1.0 - lam2)) return 0;
    double a0 = 1.0 - 2.0 * lam2;
    double cth = 2.0 * u5 - 1.0;
    double sth = sqrt(1.0 - cth * cth);
    double phi = TWO_PI * u6;
    double rho2 = 1.0 - a0 * a0;
    double rho = rho2 > 0.0 ? sqrt(rho2) : 0.0;
    a[0] = a0;
    a[1] = rho * sth * cos(phi);
    a[2] = rho * sth * sin(phi);
    a[3] = rho * cth;
    return 1;
}

/* SU(2) element P(p) = p0 + i p.sigma = [[p0 + i p3, p2 + i p1], [-p2 + i p1, p0 - i p3]]. */
static void su2_matrix(const double p[4], cplx r[2][2])
{
    r[0][0].re = p[0];  r[0][0].im = p[3];
    r[0][1].re = p[2];  r[0][1].im = p[1];
    r[1][0].re = -p[2]; r[1][0].im = p[1];
    r[1][1].re = p[0];  r[1][1].im = -p[3];
}

/* Cabibbo-Marinari update of one link: W = U A; for each subgroup (i,j) in   */
/* the order (0,1), (1,2), (0,2) take the 2x2 block w of W on rows/columns    */
/* (i,j), project v = 1/2 (Re(w_ii + w_jj), -Im(w_ij + w_ji), Re(w_ji - w_ij), */
/* Im(w_jj - w_ii)) so that Re Tr(P(r) w) = 2 r.v, set k = |v| and            */
/* alpha = 2 beta k / 3, draw x by Kennedy-Pendleton and multiply rows i, j of */
/* U and W from the left by r = P(x) P(v/k).  Rejected attempts (nhit of them) */
/* leave the subgroup unchanged.  The link is reunitarised afterwards.         */
static void cm_heatbath(mat3 *U, const mat3 *A, double beta, uint64_t seed, uint64_t lid,
                        uint64_t sweep, int nhit, uint64_t *att, uint64_t *acc)
{
    static const int SI[3] = {0, 1, 0};
    static const int SJ[3] = {1, 2, 2};
    mat3 W = m_mul(U, A);
    uint64_t key[2] = {seed, 0};
    for (int sub = 0; sub < 3; ++sub) {
        int i = SI[sub], j = SJ[sub];
        cplx wii = W.m[i][i], wij = W.m[i][j], wji = W.m[j][i], wjj = W.m[j][j];
        double v[4];
        v[0] = 0.5 * (wii.re + wjj.re);
        v[1] = -0.5 * (wij.im + wji.im);
        v[2] = 0.5 * (wji.re - wij.re);
        v[3] = 0.5 * (wjj.im - wii.im);
        double k = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2] + v[3] * v[3]);
        if (k == 0.0) continue;
        double alpha = 2.0 * beta * k / 3.0;
        double x[4];
        int accepted = 0;
        for (int t = 0; t < nhit && !accepted; ++t) {
            uint64_t ctr[4] = {lid, sweep, ((uint64_t)sub << 32) | (uint64_t)t, TAG_HEATBATH}, w[4];
            su3ref_philox4x64(ctr, key, w);
            ++*att;
            accepted = kp_attempt(alpha, w, x);
        }
        if (!accepted) continue;
        ++*acc;
        double vh[4] = {v[0] / k, v[1] / k, v[2] / k, v[3] / k};
        cplx px[2][2], pv[2][2], r[2][2];
        su2_matrix(x, px);
        su2_matrix(vh, pv);
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) r[a][b] = c_add(c_mul(px[a][0], pv[0][b]), c_mul(px[a][1], pv[1][b]));
        for (int col = 0; col < 3; ++col) {
            cplx ui = U->m[i][col], uj = U->m[j][col];
            U->m[i][col] = c_add(c_mul(r[0][0], ui), c_mul(r[0][1], uj));
            U->m[j][col] = c_add(c_mul(r[1][0], ui), c_mul(r[1][1], uj));
            cplx wi = W.m[i][col], wj = W.m[j][col];
            W.m[i][col] = c_add(c_mul(r[0][0], wi), c_mul(r[0][1], wj));
            W.m[j][col] = c_add(c_mul(r[1][0], wi), c_mul(r[1][1], wj));
        }
    }
    reunit_rows(U);
}

void su3ref_heatbath_link(double *U, const double *A, double beta, uint64_t seed, uint64_t lid,
                          uint64_t sweep, int nhit, uint64_t *cnt)
{
    mat3 u = m_load(U), a = m_load(A);
    uint64_t att = 0, acc = 0;
    cm_heatbath(&u, &a, beta, seed, lid, sweep, nhit, &att, &acc);
    m_store(&u, U);
    if (cnt) { cnt[0] += att; cnt[1] += acc; }
}

int64_t su3ref_kp_draws(double alpha, uint64_t seed, int64_t n, int cap, double *a, int64_t *tries)
{
    int64_t over = 0, total = 0;
    uint64_t key[2] = {seed, 0};
    for (int64_t i = 0; i < n; ++i) {
        int accepted = 0;
        double x[4];
        for (int t = 0; t < cap && !accepted; ++t) {
            uint64_t ctr[4] = {(uint64_t)i, 0, (uint64_t)t, TAG_HEATBATH}, w[4];
            su3ref_philox4x64(ctr, key, w);
            ++total;
            accepted = kp_attempt(alpha, w, x);
        }
        if (!accepted) {
            ++over;
            x[0] = x[1] = x[2] = x[3] = NAN;
        }
        for (int c = 0; c < 4; ++c) a[4 * i + c] = x[c];
    }
    if (tries) *tries = total;
    return over;
}

void su3ref_single_link_chain(double *U, const double *A, double beta, uint64_t seed,
                              int64_t nsteps, int nhit, double *obs)
{
    mat3 u = m_load(U), a = m_load(A);
    uint64_t att = 0, acc = 0;
    for (int64_t t = 0; t < nsteps; ++t) {
        cm_heatbath(&u, &a, beta, seed, 0, (uint64_t)t, nhit, &att, &acc);
        mat3 ua = m_mul(&u, &a);
        obs[t] = m_retrace(&ua) / 3.0;
    }
    m_store(&u, U);
}

/* ------------------------------------------------------------------------ */
/* Lattice-level operations                                                   */
/* ------------------------------------------------------------------------ */

su3ref_lattice *su3ref_create(const su3ref_params *p)
{
    if (su3ref_check_params(p) != 0) return NULL;
    su3ref_lattice *lat = (su3ref_lattice *)calloc(1, sizeof *lat);
    if (!lat) return NULL;
    lat->p = *p;
    lat->V = (int64_t)p->L[0] * p->L[1] * p->L[2] * p->L[3];
    lat->links = (double *)malloc((size_t)su3ref_n_doubles(lat) * sizeof(double));
    if (!lat->links) {
        free(lat);
        return NULL;
    }
    return lat;
}

/* Geometry only: no link storage (links is NULL).  Only the index functions
   (volume, parity, neighbor, staple_lids) may be called on it; they serve
   checks of single links of lattices too large to hold on the host. */
su3ref_lattice *su3ref_create_geometry(const su3ref_params *p)
{
    if (su3ref_check_params(p) != 0) return NULL;
    su3ref_lattice *lat = (su3ref_lattice *)calloc(1, sizeof *lat);
    if (!lat) return NULL;
    lat->p = *p;
    lat->V = (int64_t)p->L[0] * p->L[1] * p->L[2] * p->L[3];
    lat->links = NULL;
    return lat;
}

void su3ref_destroy(su3ref_lattice *lat)
{
    if (!lat) return;
    free(lat->links);
    free(lat);
}

int64_t su3ref_n_doubles(const su3ref_lattice *lat) { return 18 * 4 * lat->V * lat->p.nlat; }
double *su3ref_links(su3ref_lattice *lat) { return lat->links; }
uint64_t su3ref_get_sweeps(const su3ref_lattice *lat) { return lat->sweeps; }
void su3ref_set_sweeps(su3ref_lattice *lat, uint64_t s) { lat->sweeps = s; }

void su3ref_counters(const su3ref_lattice *lat, uint64_t *attempts, uint64_t *accepts)
{
    if (attempts) *attempts = lat->attempts;
    if (accepts) *accepts = lat->accepts;
}

void su3ref_start(su3ref_lattice *lat, int hot)
{
    int64_t nlinks = 4 * lat->V * lat->p.nlat;
#pragma omp parallel for schedule(static)
    for (int64_t lid = 0; lid < nlinks; ++lid) {
        mat3 u = hot ? haar_su3(lat->p.seed, (uint64_t)lid, TAG_HOT) : m_identity();
        m_store(&u, lat->links + lid * 18);
    }
    lat->sweeps = 0;
    lat->attempts = lat->accepts = 0;
}

static uint64_t splitmix64(uint64_t *s)
{
    uint64_t z = (*s += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* One sweep = for mu = 0..3, for parity = even, odd: update every link        */
/* U_mu(x) with parity(x) = parity (a checkerboard pass: these links share no  */
/* plaquette, so they may be updated in any order or at once).  The sweep      */
/* index s keys the random numbers and continues across calls.                  */
static void sweep_impl(su3ref_lattice *lat, int n, double beta, const double *betas, int nthreads,
                       uint64_t order_seed);

void su3ref_sweep(su3ref_lattice *lat, int n, double beta, int nthreads, uint64_t order_seed)
{
    sweep_impl(lat, n, beta, NULL, nthreads, order_seed);
}

/* Sweeps with per-layer couplings beta0 (layer 0) and beta1 (layer 1): the
 * heat bath samples exp(1/3 Re Tr(U A)) with the weighted staple above, i.e.
 * the Kennedy-Pendleton strength is alpha = 2k/3 with k from U A. */
void su3ref_sweep_betas(su3ref_lattice *lat, int n, double beta0, double beta1, int nthreads)
{
    double b[2] = {beta0, beta1};
    sweep_impl(lat, n, 1.0, b, nthreads, 0);
}

static void sweep_impl(su3ref_lattice *lat, int n, double beta, const double *betas, int nthreads,
                       uint64_t order_seed)
{
    int64_t nsites = lat->V * lat->p.nlat;
    /* sites of each parity, in lexicographic order */
    int64_t *bypar[2];
    int64_t cnt[2] = {0, 0};
    bypar[0] = (int64_t *)malloc((size_t)nsites * sizeof(int64_t));
    bypar[1] = (int64_t *)malloc((size_t)nsites * sizeof(int64_t));
    for (int64_t s = 0; s < nsites; ++s) {
        int par = su3ref_parity(lat, s);
        bypar[par][cnt[par]++] = s;
    }
    if (order_seed != 0) {
        uint64_t st = order_seed;
        for (int par = 0; par < 2; ++par)
            for (int64_t i = cnt[par] - 1; i > 0; --i) {
                int64_t j = (int64_t)(splitmix64(&st) % (uint64_t)(i + 1));
                int64_t t = bypar[par][i];
                bypar[par][i] = bypar[par][j];
                bypar[par][j] = t;
            }
    }
#ifdef _OPENMP
    int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#else
    int nt = 1;
    (void)nthreads;
#endif
    for (int it = 0; it < n; ++it) {
        uint64_t s = lat->sweeps;
        for (int mu = 0; mu < 4; ++mu)
            for (int par = 0; par < 2; ++par) {
                uint64_t att = 0, acc = 0;
                const int64_t *list = bypar[par];
#pragma omp parallel for num_threads(nt) schedule(static) reduction(+ : att, acc)
                for (int64_t q = 0; q < cnt[par]; ++q) {
                    int64_t site = list[q];
                    double A18[18];
                    if (betas)
                        staple_betas(lat, site, mu, betas, A18);
                    else
                        su3ref_staple(lat, site, mu, A18);
                    mat3 A = m_load(A18);
                    double *up = link_ptr(lat, site, mu);
                    mat3 U = m_load(up);
                    cm_heatbath(&U, &A, beta, lat->p.seed, (uint64_t)(4 * site + mu), s, lat->p.nhit,
                                &att, &acc);
                    m_store(&U, up);
                }
                lat->attempts += att;
                lat->accepts += acc;
            }
        lat->sweeps = s + 1;
    }
    free(bypar[0]);
    free(bypar[1]);
}

/* Mean plaquette: P = sum_{x, mu<nu} Re Tr U_mu(x) U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+
 * divided by 18 V nlat (6 planes per site, Re Tr <= 3).  Sequential sum. */
void su3ref_plaquette(const su3ref_lattice *lat, double *out)
{
    int nlat = lat->p.nlat;
    double tot = 0.0;
    for (int layer = 0; layer < nlat; ++layer) {
        double sum = 0.0;
        for (int64_t lex = 0; lex < lat->V; ++lex) {
            int64_t x = layer * lat->V + lex;
            for (int mu = 0; mu < 4; ++mu)
                for (int nu = mu + 1; nu < 4; ++nu) {
                    int64_t xpmu = su3ref_neighbor(lat, x, mu, +1);
                    int64_t xpnu = su3ref_neighbor(lat, x, nu, +1);
                    mat3 a = m_load(link_ptr(lat, x, mu));
                    mat3 b = m_load(link_ptr(lat, xpmu, nu));
                    mat3 c = m_load(link_ptr(lat, xpnu, mu));
                    mat3 d = m_load(link_ptr(lat, x, nu));
                    mat3 cd = m_dag(&c), dd = m_dag(&d);
                    mat3 ab = m_mul(&a, &b);
                    mat3 abc = m_mul(&ab, &cd);
                    mat3 pl = m_mul(&abc, &dd);
                    sum += m_retrace(&pl);
                }
        }
        out[1 + layer] = sum / (18.0 * (double)lat->V);
        tot += sum;
    }
    out[0] = tot / (18.0 * (double)lat->V * nlat);
}

/* Polyakov loops along direction 3: for every starting site (x0, x1, x2, x3=0,
 * layer) the trace of the ordered product of U_3 links along the closed path
 * that steps +3 until it returns to the start -- L3 steps, or 2 L3 if crossing
 * the direction-3 boundary switches the layer (flip bit 3 on a double-layered
 * torus).  out[0], out[1] = Re, Im of the mean of Tr/3 over all starting
 * sites; out[2 + 2l], out[3 + 2l] = the same over the starts in layer l. */
void su3ref_polyakov(const su3ref_lattice *lat, double *out)
{
    const int32_t *L = lat->p.L;
    int nlat = lat->p.nlat;
    int64_t V3 = (int64_t)L[0] * L[1] * L[2];
    double tre = 0, tim = 0;
    for (int layer = 0; layer < nlat; ++layer) {
        double sre = 0, sim = 0;
        for (int64_t s3 = 0; s3 < V3; ++s3) {
            int64_t start = layer * lat->V + s3; /* x3 = 0 */
            int64_t x = start;
            mat3 P = m_identity();
            do {
                mat3 u = m_load(link_ptr(lat, x, 3));
                P = m_mul(&P, &u);
                x = su3ref_neighbor(lat, x, 3, +1);
            } while (x != start);
            sre += (P.m[0][0].re + P.m[1][1].re + P.m[2][2].re) / 3.0;
            sim += (P.m[0][0].im + P.m[1][1].im + P.m[2][2].im) / 3.0;
        }
        out[2 + 2 * layer] = sre / (double)V3;
        out[3 + 2 * layer] = sim / (double)V3;
        tre += sre;
        tim += sim;
    }
    out[0] = tre / (double)(V3 * nlat);
    out[1] = tim / (double)(V3 * nlat);
}

void su3ref_reunitarise(su3ref_lattice *lat)
{
    int64_t nlinks = 4 * lat->V * lat->p.nlat;
    for (int64_t lid = 0; lid < nlinks; ++lid) su3ref_reunit(lat->links + lid * 18);
}

void su3ref_gauge_transform(su3ref_lattice *lat, uint64_t gseed)
{
    int64_t nsites = lat->V * lat->p.nlat;
    double *out = (double *)malloc((size_t)su3ref_n_doubles(lat) * sizeof(double));
    for (int64_t x = 0; x < nsites; ++x) {
        mat3 g = haar_su3(gseed, (uint64_t)x, TAG_GAUGE);
        for (int mu = 0; mu < 4; ++mu) {
            int64_t y = su3ref_neighbor(lat, x, mu, +1);
            mat3 gy = haar_su3(gseed, (uint64_t)y, TAG_GAUGE);
            mat3 gyd = m_dag(&gy);
            mat3 u = m_load(link_ptr(lat, x, mu));
            mat3 t = m_mul(&g, &u);
            mat3 r = m_mul(&t, &gyd);
            m_store(&r, out + (4 * x + mu) * 18);
        }
    }
    memcpy(lat->links, out, (size_t)su3ref_n_doubles(lat) * sizeof(double));
    free(out);
}
