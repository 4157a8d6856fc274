// device.h -- device-side building blocks of the gfx950 heat-bath kernels:
// complex 3x3 algebra, Philox4x64-10, uniform mapping, lattice indexing.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "geom.h"

namespace su3hb {

// ---------------------------------------------------------------------------
// storage types: one complex entry of a stored link
// ---------------------------------------------------------------------------
template <typename R> struct Store;
template <> struct Store<double> { using type = double2; };
template <> struct Store<float> { using type = float2; };
template <typename R> using store_t = typename Store<R>::type;

template <typename R> struct Cx {
    R re, im;
};

template <typename R> __device__ __forceinline__ Cx<R> cx(R re, R im) { return Cx<R>{re, im}; }

// a * b
template <typename R> __device__ __forceinline__ Cx<R> cmul(Cx<R> a, Cx<R> b)
{
    return Cx<R>{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// c + a * b
template <typename R> __device__ __forceinline__ Cx<R> cmadd(Cx<R> c, Cx<R> a, Cx<R> b)
{
    return Cx<R>{c.re + a.re * b.re - a.im * b.im, c.im + a.re * b.im + a.im * b.re};
}
// c + a * conj(b)
template <typename R> __device__ __forceinline__ Cx<R> cmadd_nc(Cx<R> c, Cx<R> a, Cx<R> b)
{
    return Cx<R>{c.re + a.re * b.re + a.im * b.im, c.im + a.im * b.re - a.re * b.im};
}
// conj(a) * b
template <typename R> __device__ __forceinline__ Cx<R> cmul_cn(Cx<R> a, Cx<R> b)
{
    return Cx<R>{a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
// c + conj(a) * b
template <typename R> __device__ __forceinline__ Cx<R> cmadd_cn(Cx<R> c, Cx<R> a, Cx<R> b)
{
    return Cx<R>{c.re + a.re * b.re + a.im * b.im, c.im + a.re * b.im - a.im * b.re};
}

template <typename R> struct M3 {
    Cx<R> e[3][3];
};

// C += A B
template <typename R> __device__ __forceinline__ void acc_nn(M3<R> &C, const M3<R> &A, const M3<R> &B)
{
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
#pragma unroll
            for (int k = 0; k < 3; ++k) C.e[a][b] = cmadd(C.e[a][b], A.e[a][k], B.e[k][b]);
}
// C += A B^+
template <typename R> __device__ __forceinline__ void acc_nd(M3<R> &C, const M3<R> &A, const M3<R> &B)
{
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
#pragma unroll
            for (int k = 0; k < 3; ++k) C.e[a][b] = cmadd_nc(C.e[a][b], A.e[a][k], B.e[b][k]);
}
// C += A^+ B
template <typename R> __device__ __forceinline__ void acc_dn(M3<R> &C, const M3<R> &A, const M3<R> &B)
{
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
#pragma unroll
            for (int k = 0; k < 3; ++k) C.e[a][b] = cmadd_cn(C.e[a][b], A.e[k][a], B.e[k][b]);
}

template <typename R> __device__ __forceinline__ void set_zero(M3<R> &C)
{
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) C.e[a][b] = Cx<R>{R(0), R(0)};
}

// C += s A
template <typename R> __device__ __forceinline__ void scale_acc(M3<R> &C, const M3<R> &A, R s)
{
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            C.e[a][b].re += s * A.e[a][b].re;
            C.e[a][b].im += s * A.e[a][b].im;
        }
}

template <typename R> __device__ __forceinline__ M3<R> mul_nn(const M3<R> &A, const M3<R> &B)
{
    M3<R> C;
    set_zero(C);
    acc_nn(C, A, B);
    return C;
}

template <typename R> __device__ __forceinline__ R retrace(const M3<R> &A)
{
    return A.e[0][0].re + A.e[1][1].re + A.e[2][2].re;
}

// precision-generic device math (FP32 tier: single-precision functions)
// ---------------------------------------------------------------------------
// FP64 elementary functions on the argument ranges of the heat bath.  The
// general library versions handle every input (signs, infinities, huge
// arguments) and cost 70-100 instructions each; the heat bath only takes
// logarithms of uniforms in (0, 1] and sines/cosines of pi t with t in [0, 2].
// Both below are short series with exact coefficients, accurate to about an
// ulp over those ranges.
// ---------------------------------------------------------------------------

// ln x for 0 < x <= 1 (normal numbers): x = 2^k m with m in [1/sqrt 2, sqrt 2),
// ln m = 2 atanh(s) = 2 (s + s^3/3 + s^5/5 + ...) with s = (m - 1)/(m + 1),
// |s| <= 0.1716; ten terms leave a truncation below 1e-17 relative.  ln 2 is
// split into a 40-bit head (k * head is exact) and the rounded remainder.
__host__ __device__ inline double log_unit(double x)
{
    constexpr double kLn2Hi = 0x1.62e42fefa2000p-1;
    constexpr double kLn2Lo = 0x1.9ef35793c7673p-41;
    constexpr double kSqrtHalf = 0x1.6a09e667f3bcdp-1;
    int k;
    double m = frexp(x, &k);  // m in [1/2, 1)
    if (m < kSqrtHalf) {
        m += m;
        --k;
    }
    const double s = (m - 1.0) / (m + 1.0);
    const double z = s * s;
    double p = 1.0 / 19.0;
    p = fma(p, z, 1.0 / 17.0);
    p = fma(p, z, 1.0 / 15.0);
    p = fma(p, z, 1.0 / 13.0);
    p = fma(p, z, 1.0 / 11.0);
    p = fma(p, z, 1.0 / 9.0);
    p = fma(p, z, 1.0 / 7.0);
    p = fma(p, z, 1.0 / 5.0);
    p = fma(p, z, 1.0 / 3.0);
    const double s2 = s + s;
    const double lnm = fma(s2 * z, p, s2);  // 2 s (1 + z p)
    const double dk = (double)k;
    return fma(dk, kLn2Hi, fma(dk, kLn2Lo, lnm));
}

// sin(pi r), cos(pi r) for |r| <= 1/4 from their Taylor series in y = r^2:
// coefficients (-1)^j pi^(2j+1)/(2j+1)! (sine, j = 0..8) and
// (-1)^j pi^(2j)/(2j)! (cosine, j = 0..9); the first omitted terms are below
// 1e-17 at |pi r| = pi/4.
__host__ __device__ inline void sincospi_quarter(double r, double *sn, double *cs)
{
    const double y = r * r;
    double ps = 7.952054001475513e-07;
    ps = fma(ps, y, -2.1915353447830217e-05);
    ps = fma(ps, y, 0.00046630280576761255);
    ps = fma(ps, y, -0.0073704309457143504);
    ps = fma(ps, y, 0.08214588661112823);
    ps = fma(ps, y, -0.5992645293207921);
    ps = fma(ps, y, 2.5501640398773455);
    ps = fma(ps, y, -5.16771278004997);
    ps = fma(ps, y, 3.141592653589793);
    double pc = -1.3878952462213771e-07;
    pc = fma(pc, y, 4.303069587032947e-06);
    pc = fma(pc, y, -0.0001046381049248457);
    pc = fma(pc, y, 0.0019295743094039231);
    pc = fma(pc, y, -0.02580689139001406);
    pc = fma(pc, y, 0.2353306303588932);
    pc = fma(pc, y, -1.3352627688545895);
    pc = fma(pc, y, 4.0587121264167685);
    pc = fma(pc, y, -4.934802200544679);
    *sn = r * ps;
    *cs = fma(pc, y, 1.0);
}

// t in [0, 2]: q = nearest integer to 2t, r = t - q/2 (exact, |r| <= 1/4),
// pi t = pi r + q pi/2.
__host__ __device__ inline void sincospi_0to2(double t, double *sn, double *cs)
{
    const double q = rint(t + t);
    const double r = fma(q, -0.5, t);
    double s, c;
    sincospi_quarter(r, &s, &c);
    const int iq = (int)q & 3;
    const double ss = (iq & 1) ? c : s, cc = (iq & 1) ? s : c;
    *sn = (iq & 2) ? -ss : ss;
    *cs = (iq == 1 || iq == 2) ? -cc : cc;
}

// cos^2(pi t) for t in [0, 2]: only the parity of the quadrant matters.
__host__ __device__ inline double cospi_sq_0to2(double t)
{
    const double q = rint(t + t);
    const double r = fma(q, -0.5, t);
    double s, c;
    sincospi_quarter(r, &s, &c);
    return ((int)q & 1) ? s * s : c * c;
}

// FP32 versions for the FP32 tier: the same reduction, Taylor series cut where
// the first omitted term is below 3e-9 at |pi r| = pi/4 (sine j = 0..4,
// cosine j = 0..5), coefficients as above rounded to float.
__host__ __device__ inline void sincospi_quarter(float r, float *sn, float *cs)
{
    const float y = r * r;
    float ps = 0.08214588661112823f;
    ps = fmaf(ps, y, -0.5992645293207921f);
    ps = fmaf(ps, y, 2.5501640398773455f);
    ps = fmaf(ps, y, -5.16771278004997f);
    ps = fmaf(ps, y, 3.141592653589793f);
    float pc = -0.02580689139001406f;
    pc = fmaf(pc, y, 0.2353306303588932f);
    pc = fmaf(pc, y, -1.3352627688545895f);
    pc = fmaf(pc, y, 4.0587121264167685f);
    pc = fmaf(pc, y, -4.934802200544679f);
    *sn = r * ps;
    *cs = fmaf(pc, y, 1.0f);
}
__host__ __device__ inline void sincospi_0to2(float t, float *sn, float *cs)
{
    const float q = rintf(t + t);
    const float r = fmaf(q, -0.5f, t);
    float s, c;
    sincospi_quarter(r, &s, &c);
    const int iq = (int)q & 3;
    const float ss = (iq & 1) ? c : s, cc = (iq & 1) ? s : c;
    *sn = (iq & 2) ? -ss : ss;
    *cs = (iq == 1 || iq == 2) ? -cc : cc;
}
__host__ __device__ inline float cospi_sq_0to2(float t)
{
    const float q = rintf(t + t);
    const float r = fmaf(q, -0.5f, t);
    float s, c;
    sincospi_quarter(r, &s, &c);
    return ((int)q & 1) ? s * s : c * c;
}

// Precision-generic helpers of the heat bath (arguments: uniforms in (0, 1]
// and t in [0, 2]): the functions above; FP32 logarithm from the library.
__device__ __forceinline__ double log_r(double x) { return log_unit(x); }
__device__ __forceinline__ float log_r(float x) { return logf(x); }
// 1/sqrt(x) and sqrt(x) for x > 0.  FP64: the library reciprocal square root
// (the hardware estimate plus one correction step, ~11 instructions, about an
// ulp) instead of a correctly rounded square root (~22) and a division (~11);
// FP32: the plain float operations.
__device__ __forceinline__ double rsqrt_r(double x) { return rsqrt(x); }
__device__ __forceinline__ float rsqrt_r(float x) { return 1.0f / sqrtf(x); }
__device__ __forceinline__ double sqrt_pos_r(double x) { return x * rsqrt(x); }
__device__ __forceinline__ float sqrt_pos_r(float x) { return sqrtf(x); }
__device__ __forceinline__ double cospi_sq_r(double t) { return cospi_sq_0to2(t); }
__device__ __forceinline__ float cospi_sq_r(float t) { return cospi_sq_0to2(t); }
__device__ __forceinline__ void sincospi_r(double t, double *s, double *c) { sincospi_0to2(t, s, c); }
__device__ __forceinline__ void sincospi_r(float t, float *s, float *c) { sincospi_0to2(t, s, c); }

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror & Shaw, SC'11)
// ---------------------------------------------------------------------------
struct U64x4 {
    uint64_t w[4];
};

// Full 128-bit product a m, m a compile-time constant, from 32-bit limbs
// a = a1 2^32 + a0, m = m1 2^32 + m0:
//   t = a0 m1 + hi(a0 m0),  u = a1 m0 + lo(t),
//   a m = lo(a0 m0) + 2^32 lo(u) + 2^64 (a1 m1 + hi(t) + hi(u)),
// where no partial sum overflows 64 bits.  Four 32x32+64 multiply-adds; the
// separate low product and high product would form the cross terms twice.
template <uint64_t M> __device__ __forceinline__ void mulhilo64(uint64_t a, uint64_t &lo, uint64_t &hi)
{
    constexpr uint32_t m0 = (uint32_t)M, m1 = (uint32_t)(M >> 32);
    const uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32);
    const uint64_t p = (uint64_t)a0 * m0;
    const uint64_t t = (uint64_t)a0 * m1 + (p >> 32);
    const uint64_t u = (uint64_t)a1 * m0 + (uint32_t)t;
    lo = (u << 32) | (uint32_t)p;
    hi = (uint64_t)a1 * m1 + ((t >> 32) + (u >> 32));
}

__device__ __forceinline__ U64x4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0,
                                               uint64_t k1)
{
    constexpr uint64_t kMul0 = 0xD2E7470EE14C6C93ull, kMul1 = 0xCA5A826395121157ull;
    constexpr uint64_t kBump0 = 0x9E3779B97F4A7C15ull, kBump1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        uint64_t lo_a, hi_a, lo_b, hi_b;
        mulhilo64<kMul0>(c0, lo_a, hi_a);
        mulhilo64<kMul1>(c2, lo_b, hi_b);
        c0 = hi_b ^ c1 ^ k0;
        c1 = lo_b;
        c2 = hi_a ^ c3 ^ k1;
        c3 = lo_a;
        k0 += kBump0;
        k1 += kBump1;
    }
    return U64x4{{c0, c1, c2, c3}};
}

// Purpose tags (counter word 3).
enum : uint64_t { kTagHeatbath = 0, kTagHot = 1, kTagGauge = 2 };

// (k + 1/2) * 2^-52 from the top 52 bits: exact in FP64, never 0 or 1.
__device__ __forceinline__ double unif52(uint64_t w) { return (double(w >> 12) + 0.5) * 0x1p-52; }
// (h + 1/2) * 2^-32 from a 32-bit half: exact in FP64, never 0 or 1.
__device__ __forceinline__ double unif32(uint32_t h) { return (double(h) + 0.5) * 0x1p-32; }

// ---------------------------------------------------------------------------
// XCD-aware workgroup order.  MI355X deals workgroups round-robin to its 8
// XCDs, each with a private L2: workgroup b runs on XCD b % 8.  Remapping b to
// a logical tile index so that XCD k owns the contiguous range of tiles
// [k * n/8, (k+1) * n/8) keeps neighbouring tiles, which share staple links,
// on one L2.  A bijection for any n.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int xcd_tile(int b, int n)
{
    const int xcd = b % kNumXcd, local = b / kNumXcd;
    const int per = n / kNumXcd, rem = n % kNumXcd;
    return xcd < rem ? xcd * (per + 1) + local : rem * (per + 1) + (xcd - rem) * per + local;
}

// ---------------------------------------------------------------------------
// lattice geometry
// ---------------------------------------------------------------------------
// Coordinates of the site with parity `par` and half-index i.
__device__ __forceinline__ void site_coords(const Geom &g, int par, int i, int x[4])
{
    const int l0h = g.L[0] >> 1;
    int r = div_by(i, g.dl0h);
    const int x0h = i - r * l0h;
    int q = div_by(r, g.dl1);
    x[1] = r - q * g.L[1];
    r = q;
    q = div_by(r, g.dl2);
    x[2] = r - q * g.L[2];
    x[3] = q;
    x[0] = 2 * x0h + ((par + x[1] + x[2] + x[3]) & 1);
}

// Step coordinate D by S (+1 / -1, 0 = no step) with periodic wrap; on a
// double-layered torus (DLT = true) crossing the boundary of a direction whose
// flip bit is set switches the layer.
template <int D, int S, bool DLT = true> __device__ __forceinline__ void step(const Geom &g, int y[4], int &layer)
{
    if (S > 0) {
        if (y[D] == g.L[D] - 1) {
            y[D] = 0;
            if (DLT) layer ^= (g.flip >> D) & 1;
        } else {
            y[D] += 1;
        }
    } else if (S < 0) {
        if (y[D] == 0) {
            y[D] = g.L[D] - 1;
            if (DLT) layer ^= (g.flip >> D) & 1;
        } else {
            y[D] -= 1;
        }
    }
}

__device__ __forceinline__ int lex_of(const Geom &g, const int y[4])
{
    return y[0] + g.L[0] * (y[1] + g.L[1] * (y[2] + g.L[2] * y[3]));
}

// Plane element of the site x + SA*A + SB*B.
template <int A, int SA, int B, int SB, bool DLT = true>
__device__ __forceinline__ int nbr_elem(const Geom &g, const int x[4], int layer)
{
    int y[4] = {x[0], x[1], x[2], x[3]};
    int ly = layer;
    step<A, SA, DLT>(g, y, ly);
    step<B, SB, DLT>(g, y, ly);
    const int e = lex_of(g, y) >> 1;
    return DLT ? ly * g.Vh + e : e;
}

// Processing order of one pass.  The (x1, x2) cross-section is cut into
// domains of w1 x w2 sites, numbered d = c1 + nd1 c2 (x1 = c1 w1 + x1',
// x2 = c2 w2 + x2'), and each domain is swept along x3:
//   v = x0h + (L0/2)(x1' + w1 (x2' + w2 (x3 + L3 d))).
// Together with xcd_tile each XCD owns whole domains, so a link is re-read
// while it is still in that XCD's L2, and square-ish domains keep the links
// that two XCDs both read (the domain's rim) few.  Lanes of a wave still
// cover consecutive x0, so loads stay coalesced.  Returns the half-index i of
// thread v's site and fills its coordinates (x0 for parity par).
__device__ __forceinline__ int order_site(const Geom &g, int par, int v, int x[4])
{
    const int l0h = g.L[0] >> 1;
    int r = div_by(v, g.dl0h);
    const int x0h = v - r * l0h;
    int q = div_by(r, g.dw1);
    const int x1p = r - q * g.w1;
    r = q;
    q = div_by(r, g.dw2);
    const int x2p = r - q * g.w2;
    r = q;
    q = div_by(r, g.dl3);
    x[3] = r - q * g.L[3];
    r = q;
    q = div_by(r, g.dnd1);
    x[1] = (r - q * g.nd1) * g.w1 + x1p;
    x[2] = q * g.w2 + x2p;
    x[0] = 2 * x0h + ((par + x[1] + x[2] + x[3]) & 1);
    return x0h + l0h * (x[1] + g.L[1] * (x[2] + g.L[2] * x[3]));
}
__device__ __forceinline__ int order_index(const Geom &g, int v)
{
    int x[4];
    return order_site(g, 0, v, x);
}

// Link storage.  A link is stored as its rows 0 and 1, the six complex
// entries e = 3 row + col < 6; row 2 of an SU(3) matrix is conj(row 0 x row 1)
// and is rebuilt by every reader (rebuild_row2).  The links of one
// (direction, parity) form a block of `stride` links in tiles of kTile = 16
// consecutive links; a tile holds the 6 entries as 6 rows of 16 (entry-major
// inside the tile):
//   element (dir, par, n, e) at block(dir, par) + (n / 16) * 96 + e * 16 + n % 16.
// A wave of 64 consecutive links reads 4 tiles, 256 contiguous bytes (FP64)
// per tile and entry: whole cache lines.  The 6 loads of one link share a
// single per-lane address and differ by the compile-time offset e * 16
// elements, which the load instruction encodes as an immediate.
template <typename R>
__device__ __forceinline__ const store_t<R> *planes(const store_t<R> *links, const Geom &g, int dir, int par)
{
    return links + (size_t)(dir * 2 + par) * (size_t)g.stride * kEntries;
}
template <typename R> __device__ __forceinline__ store_t<R> *planes(store_t<R> *links, const Geom &g, int dir, int par)
{
    return links + (size_t)(dir * 2 + par) * (size_t)g.stride * kEntries;
}

// entry 0 of link n in its block; entry e is at + e * kTile
template <typename R> __device__ __forceinline__ const store_t<R> *link_at(const store_t<R> *block, int n)
{
    return block + (size_t)(n >> 4) * (kEntries * kTile) + (n & (kTile - 1));
}
template <typename R> __device__ __forceinline__ store_t<R> *link_at(store_t<R> *block, int n)
{
    return block + (size_t)(n >> 4) * (kEntries * kTile) + (n & (kTile - 1));
}

// row 2 = conj(row 0 x row 1): the third row of an SU(3) matrix, computed
// exactly as reunit() computes it
template <typename R> __device__ __forceinline__ void rebuild_row2(M3<R> &u)
{
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int a = (k + 1) % 3, b = (k + 2) % 3;
        const Cx<R> p = cmul(u.e[0][a], u.e[1][b]), q = cmul(u.e[0][b], u.e[1][a]);
        u.e[2][k] = Cx<R>{p.re - q.re, -(p.im - q.im)};
    }
}

// Products of SU(3) matrices.  A product is again in SU(3), so only its rows
// 0 and 1 are formed (18 complex multiply-adds instead of 27) and row 2 is
// rebuilt from them; the left factor's row 2 is never read.
// A B
template <typename R> __device__ __forceinline__ M3<R> mul_nn_su3(const M3<R> &A, const M3<R> &B)
{
    M3<R> C;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            Cx<R> t = cmul(A.e[a][0], B.e[0][b]);
            t = cmadd(t, A.e[a][1], B.e[1][b]);
            C.e[a][b] = cmadd(t, A.e[a][2], B.e[2][b]);
        }
    rebuild_row2(C);
    return C;
}
// A B^+
template <typename R> __device__ __forceinline__ M3<R> mul_nd_su3(const M3<R> &A, const M3<R> &B)
{
    M3<R> C;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            Cx<R> t{R(0), R(0)};
#pragma unroll
            for (int k = 0; k < 3; ++k) t = cmadd_nc(t, A.e[a][k], B.e[b][k]);
            C.e[a][b] = t;
        }
    rebuild_row2(C);
    return C;
}
// A^+ B
template <typename R> __device__ __forceinline__ M3<R> mul_dn_su3(const M3<R> &A, const M3<R> &B)
{
    M3<R> C;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            Cx<R> t = cmul_cn(A.e[0][a], B.e[0][b]);
            t = cmadd_cn(t, A.e[1][a], B.e[1][b]);
            C.e[a][b] = cmadd_cn(t, A.e[2][a], B.e[2][b]);
        }
    rebuild_row2(C);
    return C;
}
// C += A
template <typename R> __device__ __forceinline__ void add_to(M3<R> &C, const M3<R> &A)
{
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            C.e[a][b].re += A.e[a][b].re;
            C.e[a][b].im += A.e[a][b].im;
        }
}

// A link as an SU(3) matrix: the stored rows 0 and 1, row 2 rebuilt.
template <typename R> __device__ __forceinline__ M3<R> load_link12(const store_t<R> *block, int n)
{
    M3<R> m;
    const store_t<R> *p = link_at<R>(block, n);
#pragma unroll
    for (int e = 0; e < 6; ++e) {
        const store_t<R> v = p[e * kTile];
        m.e[e / 3][e % 3] = Cx<R>{v.x, v.y};
    }
    rebuild_row2(m);
    return m;
}

template <typename R>
__device__ __forceinline__ void load_link12_pair(M3<R> &p, const store_t<R> *bp, int np, M3<R> &q,
                                                 const store_t<R> *bq, int nq)
{
    const store_t<R> *pp = link_at<R>(bp, np), *pq = link_at<R>(bq, nq);
#pragma unroll
    for (int e = 0; e < 6; ++e) {
        const store_t<R> vp = pp[e * kTile];
        const store_t<R> vq = pq[e * kTile];
        p.e[e / 3][e % 3] = Cx<R>{vp.x, vp.y};
        q.e[e / 3][e % 3] = Cx<R>{vq.x, vq.y};
    }
    rebuild_row2(p);
    rebuild_row2(q);
}

// Nontemporal access to the link a pass updates: no other thread of the pass
// reads it, so it should not displace reusable staple links from L2.
template <typename R> struct NtVec;
template <> struct NtVec<double> { typedef double type __attribute__((ext_vector_type(2))); };
template <> struct NtVec<float> { typedef float type __attribute__((ext_vector_type(2))); };

template <typename R> __device__ __forceinline__ M3<R> load_link12_nt(const store_t<R> *block, int n)
{
    typedef typename NtVec<R>::type V;
    M3<R> m;
    const V *p = reinterpret_cast<const V *>(link_at<R>(block, n));
#pragma unroll
    for (int e = 0; e < 6; ++e) {
        const V v = __builtin_nontemporal_load(p + e * kTile);
        m.e[e / 3][e % 3] = Cx<R>{v.x, v.y};
    }
    rebuild_row2(m);
    return m;
}

template <typename R> __device__ __forceinline__ void store_link_nt(store_t<R> *block, int n, const M3<R> &m)
{
    typedef typename NtVec<R>::type V;
    V *p = reinterpret_cast<V *>(link_at<R>(block, n));
#pragma unroll
    for (int e = 0; e < kEntries; ++e) {
        V v;
        v.x = m.e[e / 3][e % 3].re;
        v.y = m.e[e / 3][e % 3].im;
        __builtin_nontemporal_store(v, p + e * kTile);
    }
}

// Stores rows 0 and 1 of m (row 2 is implied).
template <typename R> __device__ __forceinline__ void store_link(store_t<R> *block, int n, const M3<R> &m)
{
    store_t<R> *p = link_at<R>(block, n);
#pragma unroll
    for (int e = 0; e < kEntries; ++e) {
        store_t<R> v;
        v.x = m.e[e / 3][e % 3].re;
        v.y = m.e[e / 3][e % 3].im;
        p[e * kTile] = v;
    }
}

template <typename To, typename From> __device__ __forceinline__ M3<To> convert(const M3<From> &a)
{
    M3<To> b;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) b.e[r][c] = Cx<To>{To(a.e[r][c].re), To(a.e[r][c].im)};
    return b;
}

// Reunitarisation in FP64: normalise row 0, orthogonalise and normalise row 1,
// row 2 = conj(row0 x row1).
__device__ __forceinline__ void reunit(M3<double> &u)
{
    Cx<double> *r0 = u.e[0], *r1 = u.e[1], *r2 = u.e[2];
    const double i0 = rsqrt(r0[0].re * r0[0].re + r0[0].im * r0[0].im + r0[1].re * r0[1].re + r0[1].im * r0[1].im +
                            r0[2].re * r0[2].re + r0[2].im * r0[2].im);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        r0[k].re *= i0;
        r0[k].im *= i0;
    }
    Cx<double> d{0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 3; ++k) d = cmadd_cn(d, r0[k], r1[k]);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        r1[k].re -= d.re * r0[k].re - d.im * r0[k].im;
        r1[k].im -= d.re * r0[k].im + d.im * r0[k].re;
    }
    const double i1 = rsqrt(r1[0].re * r1[0].re + r1[0].im * r1[0].im + r1[1].re * r1[1].re + r1[1].im * r1[1].im +
                            r1[2].re * r1[2].re + r1[2].im * r1[2].im);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        r1[k].re *= i1;
        r1[k].im *= i1;
    }
    // r2_k = conj(r0_{k+1} r1_{k+2} - r0_{k+2} r1_{k+1})
    (void)r2;
    rebuild_row2(u);
}

// Haar-random SU(3) element keyed by (seed; id, 0, draw, tag): 12 normals by
// Box-Muller from three Philox blocks, two complex Gaussian rows, reunit.
__device__ __forceinline__ M3<double> haar_element(uint64_t seed, uint64_t id, uint64_t tag)
{
    constexpr double kTwoPi = 6.283185307179586476925286766559;
    double gauss[12];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const U64x4 w = philox4x64_10(id, 0, (uint64_t)d, tag, seed, 0);
#pragma unroll
        for (int pr = 0; pr < 2; ++pr) {
            const double ua = unif52(w.w[2 * pr]), ub = unif52(w.w[2 * pr + 1]);
            const double rad = sqrt(-2.0 * log(ua));
            double s, c;
            sincos(kTwoPi * ub, &s, &c);
            gauss[4 * d + 2 * pr] = rad * c;
            gauss[4 * d + 2 * pr + 1] = rad * s;
        }
    }
    M3<double> u;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        u.e[0][k] = Cx<double>{gauss[2 * k], gauss[2 * k + 1]};
        u.e[1][k] = Cx<double>{gauss[6 + 2 * k], gauss[7 + 2 * k]};
        u.e[2][k] = Cx<double>{0.0, 0.0};
    }
    reunit(u);
    return u;
}

}  // namespace su3hb
