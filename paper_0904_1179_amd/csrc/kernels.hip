// kernels.hip -- gfx950 kernels of the checkerboard SU(3) heat bath.
//
// Link storage: the links of one (direction, parity) form a block of tiles of
// 16 consecutive links, each tile holding the 6 complex entries of rows 0 and 1
// entry-major (double2 or float2; row 2 is rebuilt by every reader); see
// link_at.  The link U_dir(x) of site
// x = (layer, parity, i) is element n = layer * Vh + i of block (dir, parity).
// Sixteen lanes with consecutive n read 16 consecutive complex numbers per
// entry: whole 128-byte lines, fully coalesced vector loads.
//
// The hot kernel is k_update<MU, R>: one checkerboard pass, i.e. every link
// U_MU(x) with parity(x) = par, one thread per link (one-wave workgroups on a
// single torus, four-wave ones on a double-layered torus).  It gathers the 18
// neighbour links of the six staples (Wilson action), runs the
// Cabibbo-Marinari heat bath on the SU(2) subgroups (0,1), (1,2), (0,2) with
// Kennedy-Pendleton sampling, reunitarises in FP64 and writes the link back.
// Links of one pass share no plaquette, so threads never read what another
// thread of the same pass writes.
#include <algorithm>

#include "launch.h"

namespace su3hb {

namespace {

// ---------------------------------------------------------------------------
// Staple of U_MU(x): A = sum over nu != MU (ascending) of D_nu,
//   D_nu = up_nu + dn_nu,
//   up_nu = U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+ = a (c b)^+,
//   dn_nu = U_nu(x+mu-nu)^+ U_mu(x-nu)^+ U_nu(x-nu) = (e d)^+ f,
// with a = U_nu(x+mu), b = U_mu(x+nu), c = U_nu(x), d = U_nu(x+mu-nu),
// e = U_mu(x-nu), f = U_nu(x-nu).  up_nu is the plaquette based at x, dn_nu
// the one based at x - nu.
//
// Rounding order, fixed for every kernel: c b, e d and a (c b)^+ are SU(3)
// products (rows 0 and 1 formed, row 2 rebuilt); dn_nu is formed entry by
// entry from zero; D_nu = up_nu + dn_nu entry by entry; A = (D_0 + D_1) + D_2
// over the three directions in increasing order.  The one-lane pass, the
// several-lanes-per-link pass and the batched server pass all add in exactly
// this order, so a lattice gets the same bits from each of them.
// ---------------------------------------------------------------------------

// D = a (c b)^+ + (e d)^+ f from cb = c b and ed = e d.  CROSS: also
// cross += (e d)^+ f when `crosses` (the lower plaquette's base site lies in
// the other layer of a double-layered torus).
template <typename R, bool CROSS>
__device__ __forceinline__ void staple_term(M3<R> &D, const M3<R> &a, const M3<R> &cb, const M3<R> &ed,
                                            const M3<R> &f, M3<R> &cross, bool crosses)
{
    D = mul_nd_su3(a, cb);
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            Cx<R> dn = cmul_cn(ed.e[0][r], f.e[0][c]);
            dn = cmadd_cn(dn, ed.e[1][r], f.e[1][c]);
            dn = cmadd_cn(dn, ed.e[2][r], f.e[2][c]);
            D.e[r][c].re += dn.re;
            D.e[r][c].im += dn.im;
            if constexpr (CROSS) {
                cross.e[r][c].re += crosses ? dn.re : R(0);
                cross.e[r][c].im += crosses ? dn.im : R(0);
            }
        }
}

// D_NU of the one-lane pass; b = U_MU(x+NU) and e = U_MU(x-NU) come from the
// caller.  The pairs (c, d) and (a, f) are loaded together: c of thread x is d
// of thread x + NU - MU, a of thread x is f of thread x + MU + NU.
template <int MU, int NU, typename R, bool DLT, bool CROSS>
__device__ __forceinline__ void staple_dir(M3<R> &D, const M3<R> &b, const M3<R> &e,
                                           const store_t<R> *__restrict__ links, const Geom &g, const int x[4],
                                           int layer, int par, int n, M3<R> &cross, bool take_cross = true)
{
    const int opp = par ^ 1;
    M3<R> c, d, a, f;
    load_link12_pair<R>(c, planes<R>(links, g, NU, par), n, d, planes<R>(links, g, NU, par),
                        nbr_elem<MU, +1, NU, -1, DLT>(g, x, layer));
    const M3<R> cb = mul_nn_su3(c, b);
    const M3<R> ed = mul_nn_su3(e, d);
    load_link12_pair<R>(a, planes<R>(links, g, NU, opp), nbr_elem<MU, +1, NU, 0, DLT>(g, x, layer), f,
                        planes<R>(links, g, NU, opp), nbr_elem<NU, -1, MU, 0, DLT>(g, x, layer));
    staple_term<R, CROSS>(D, a, cb, ed, f, cross, CROSS && take_cross && x[NU] == 0 && ((g.flip >> NU) & 1u));
}

// Per-layer couplings (double-layered torus): A += w(x) up_nu + w(x - nu) dn_nu,
// w = the coupling of the base site's layer.
template <int MU, int NU, typename R>
__device__ __forceinline__ void add_staple_twob(M3<R> &A, const M3<R> &b, const M3<R> &e,
                                                const store_t<R> *__restrict__ links, const Geom &g, const int x[4],
                                                int layer, int par, int n, const R *wb)
{
    const int opp = par ^ 1;
    M3<R> c, d, a, f;
    load_link12_pair<R>(c, planes<R>(links, g, NU, par), n, d, planes<R>(links, g, NU, par),
                        nbr_elem<MU, +1, NU, -1, true>(g, x, layer));
    const M3<R> cb = mul_nn_su3(c, b);
    const M3<R> ed = mul_nn_su3(e, d);
    const int elo = nbr_elem<NU, -1, MU, 0, true>(g, x, layer);
    load_link12_pair<R>(a, planes<R>(links, g, NU, opp), nbr_elem<MU, +1, NU, 0, true>(g, x, layer), f,
                        planes<R>(links, g, NU, opp), elo);
    scale_acc(A, mul_nd_su3(a, cb), wb[layer]);
    M3<R> t;
    set_zero(t);
    acc_dn(t, ed, f);
    scale_acc(A, t, wb[elo >= g.Vh ? 1 : 0]);
}

// ---------------------------------------------------------------------------
// Cabibbo-Marinari heat bath of one link in staple A.  W = U A; for subgroup
// (i,j): v = 1/2 (Re(w_ii + w_jj), -Im(w_ij + w_ji), Re(w_ji - w_ij),
// Im(w_jj - w_ii)), k = |v|, alpha = 2 beta k / 3.  Kennedy-Pendleton attempt t
// uses Philox block (lid, sweep, sub<<32 | t, heat-bath tag):
//   lambda^2 = -(ln u1 + cos^2(2 pi u2) ln u3) / (2 alpha), accept iff u4^2 <= 1 - lambda^2,
//   a0 = 1 - 2 lambda^2, cos(theta) = 2 u5 - 1, phi = 2 pi u6;
// then rows i, j of U and W are multiplied from the left by r = P(a) P(v/k)
// with P(p) = [[p0 + i p3, p2 + i p1], [-p2 + i p1, p0 - i p3]].
// The SU(2) step runs in the link precision R (FP64 links: FP64 throughout,
// accept decisions in FP64); the uniforms are formed exactly in FP64 first.
// The link is reunitarised in FP64 at the end.
// ---------------------------------------------------------------------------

// What an attempt needs from its random numbers, independent of the link:
// q = ln u1 + cos^2(2 pi u2) ln u3 (so lambda^2 = -q / (2 alpha)), u4^2,
// cos(theta), sin(theta) cos(phi), sin(theta) sin(phi).  Several lanes of one
// link compute the three subgroups' draws at once and exchange them; the
// one-lane pass computes each where it is used.  Both produce the same values.
template <typename R> struct KPDraw {
    R q, u4sq, cth, sc, ss;
};

template <typename R>
__device__ __forceinline__ KPDraw<R> kp_draw(uint64_t seed, uint64_t lid, uint64_t sweep, int sub, int t)
{
    const U64x4 w = philox4x64_10(lid, sweep, ((uint64_t)sub << 32) | (uint64_t)t, kTagHeatbath, seed, 0);
    const R u1 = R(unif52(w.w[0]));
    const R u3 = R(unif52(w.w[1]));
    const R u2 = R(unif32((uint32_t)w.w[2]));
    const R u4 = R(unif32((uint32_t)(w.w[2] >> 32)));
    const R u5 = R(unif32((uint32_t)w.w[3]));
    const R u6 = R(unif32((uint32_t)(w.w[3] >> 32)));
    KPDraw<R> d;
    const R c2 = cospi_sq_r(R(2) * u2);
    d.q = log_r(u1) + c2 * log_r(u3);
    d.u4sq = u4 * u4;
    d.cth = R(2) * u5 - R(1);
    // FP64: |cth| < 1 (u5 is never 0 or 1), so the argument is positive
    const R sth = sqrt_pos_r(R(1) - d.cth * d.cth);
    R sph, cph;
    sincospi_r(R(2) * u6, &sph, &cph);
    d.sc = sth * cph;
    d.ss = sth * sph;
    return d;
}

// PRE: the draws of attempt 0 of the three subgroups are given in pre[0..2]
// (1-hit only).  Returns Re Tr W after the last subgroup, i.e. Re Tr(U_new A)
// before the final reunitarisation.
template <typename R, bool HIT1, bool PRE = false>
__device__ __forceinline__ double heatbath(M3<R> &U, const M3<R> &A, double beta_d, uint64_t seed, uint64_t lid,
                                           uint64_t sweep, int nhit, int &att, int &acc,
                                           const KPDraw<R> *pre = nullptr)
{
    static_assert(!PRE || HIT1, "given draws: one attempt per subgroup");
    if (HIT1) nhit = 1;  // 1-hit: a single attempt, no loop
    // 1/(2 alpha) = 3/(4 beta k): one division per link and 1/k per subgroup
    const R q34b = R(0.75) / R(beta_d);
    M3<R> W = mul_nn(U, A);
#pragma unroll
    for (int sub = 0; sub < 3; ++sub) {
        const int i = (sub == 1) ? 1 : 0;
        const int j = (sub == 0) ? 1 : 2;
        const R v0 = R(0.5) * (W.e[i][i].re + W.e[j][j].re);
        const R v1 = R(-0.5) * (W.e[i][j].im + W.e[j][i].im);
        const R v2 = R(0.5) * (W.e[j][i].re - W.e[i][j].re);
        const R v3 = R(0.5) * (W.e[j][j].im - W.e[i][i].im);
        const R k2 = v0 * v0 + v1 * v1 + v2 * v2 + v3 * v3;
        if (k2 == R(0)) continue;
        const R rk = rsqrt_r(k2);  // 1/k
        const R inv2alpha = q34b * rk;
        bool ok = false;
        R a0 = R(1), a1 = R(0), a2 = R(0), a3 = R(0);
        for (int t = 0; t < (HIT1 ? 1 : nhit); ++t) {
            KPDraw<R> d;
            if constexpr (PRE)
                d = pre[sub];
            else
                d = kp_draw<R>(seed, lid, sweep, sub, t);
            ++att;
            const R lam2 = -d.q * inv2alpha;
            if (d.u4sq <= R(1) - lam2) {
                a0 = R(1) - R(2) * lam2;
                const R rho2 = R(1) - a0 * a0;
                const R rho = rho2 > R(0) ? sqrt_pos_r(rho2) : R(0);
                a1 = rho * d.sc;
                a2 = rho * d.ss;
                a3 = rho * d.cth;
                ok = true;
                break;
            }
        }
        if (!ok) continue;
        ++acc;
        const R b0 = v0 * rk, b1 = v1 * rk, b2 = v2 * rk, b3 = v3 * rk;
        // quaternion product c = a * b  <=>  P(c) = P(a) P(b)
        const R c0 = a0 * b0 - a1 * b1 - a2 * b2 - a3 * b3;
        const R c1 = a0 * b1 + b0 * a1 - (a2 * b3 - a3 * b2);
        const R c2 = a0 * b2 + b0 * a2 - (a3 * b1 - a1 * b3);
        const R c3 = a0 * b3 + b0 * a3 - (a1 * b2 - a2 * b1);
        const Cx<R> r00{c0, c3}, r01{c2, c1}, r10{-c2, c1}, r11{c0, -c3};
#pragma unroll
        for (int col = 0; col < 3; ++col) {
            const Cx<R> ui = U.e[i][col], uj = U.e[j][col];
            U.e[i][col] = cmadd(cmul(r00, ui), r01, uj);
            U.e[j][col] = cmadd(cmul(r10, ui), r11, uj);
            const Cx<R> wi = W.e[i][col], wj = W.e[j][col];
            W.e[i][col] = cmadd(cmul(r00, wi), r01, wj);
            W.e[j][col] = cmadd(cmul(r10, wi), r11, wj);
        }
    }
    M3<double> Ud = convert<double>(U);
    reunit(Ud);
    U = convert<R>(Ud);
    return double(W.e[0][0].re) + double(W.e[1][1].re) + double(W.e[2][2].re);
}

// Re Tr(u s), accumulated in FP64.
template <typename R> __device__ __forceinline__ double retr_mul(const M3<R> &u, const M3<R> &s)
{
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k)
            t += (double)u.e[i][k].re * (double)s.e[k][i].re - (double)u.e[i][k].im * (double)s.e[k][i].im;
    return t;
}

// One thread of a pass: the link U_MU at pass-order position v of its layer
// (v < nlat * Vh).  Shared by the single-lattice and the batched kernels: the
// two may load the staple links in different orders (below), but every value
// goes through the same arithmetic in the same order, so a lattice gets
// bit-identical updates from both.
//
// Load order (single torus).  The six links U_MU(x +- nu) (b and e of the
// three staple directions) are links of the other parity that the
// neighbouring sites read in all three direction phases; loaded phase by
// phase, their lines leave L2 between phases.  They are all loaded first,
// entry by entry: b and e of the first direction stay in registers for its
// phase, b and e of the second and b of the third wait in this thread's slots
// of `stash` (3 * 6 * kBlock entries of LDS, slot-major, so the 64 lanes of a
// wave access consecutive entries), e of the third stays in registers.  This
// order is used with STASH (kStashPass, kStashBatch); otherwise b and e are
// loaded in their direction's phase and `stash` is unused.
//
// MEAS: also return tr = Re Tr(U_new S) with S = sum of D_nu over the
// directions nu < MU.  Summed over the sites of one parity these are all
// plaquettes of the planes (nu, MU), nu < MU, each once (the upper term of
// site x is the plaquette based at x, the lower one that based at x - nu).
// After the odd pass of MU no later pass of the sweep changes U_nu or U_MU for
// nu < MU, so the odd passes of MU = 1, 2, 3 together give the final
// plaquettes of all six planes.  On a double-layered torus a lower term whose
// base x - nu lies in the other layer (x_nu = 0 across a flipped boundary) is
// also summed separately, trx = Re Tr(U_new S_cross): its plaquette belongs to
// the other layer.
constexpr int kStashSlots = 3;
// Waves per SIMD the pass kernels are compiled for: register budgets of 256
// (FP64) and 128 (FP32) VGPRs; the stash (3 * 6 * kBlock entries: 72 KiB in
// FP64, 36 KiB in FP32 per workgroup) fits the 160 KiB of LDS at these
// occupancies.
template <typename R> constexpr int kPassWaves = sizeof(R) == 8 ? 2 : 4;
// The stash order pays where a pass is limited by memory traffic: FP64.  The
// FP32 pass is limited by instruction issue (FP32 and FP64 vector operations
// issue at the same rate), so it keeps the direction-by-direction order.  On
// a double-layered torus the six layer-dependent addresses of MU = 0 at once
// spill, and so does the batched pass (which also holds its job record).
// The measured passes of a double-layered torus also hold the cross-layer
// staple sum and would spill with the stash.
template <typename R, bool DLT, int MU, bool MEAS = false>
constexpr bool kStashPass = sizeof(R) == 8 && (!DLT || (MU > 0 && !MEAS));
template <typename R, bool DLT> constexpr bool kStashBatch = sizeof(R) == 8 && !DLT;
// FP32 1-hit passes draw the random numbers of the three subgroups right
// after issuing the first staple loads, so that the Philox and logarithm work
// fills the wait for them (the draws do not depend on the link): +9 % at
// 32^4, +7 % at 64^4.  The FP64 pass, whose two waves per SIMD already keep
// the vector unit busy, lost 1 % with it.
template <typename R> constexpr bool kEarlyDraws = sizeof(R) == 4;
// Measured passes of a double-layered torus keep the measured staple sums S
// and S_cross in LDS across the heat bath (held in registers they spill);
// these passes run with one wave per SIMD, so the LDS is otherwise unused.
template <typename R, int NB> __device__ __forceinline__ void park(store_t<R> *buf, int slot, const M3<R> &m)
{
#pragma unroll
    for (int e = 0; e < 9; ++e) {
        store_t<R> v;
        v.x = m.e[e / 3][e % 3].re;
        v.y = m.e[e / 3][e % 3].im;
        buf[(slot * 9 + e) * NB + threadIdx.x] = v;
    }
}
template <typename R, int NB> __device__ __forceinline__ M3<R> unpark(const store_t<R> *buf, int slot)
{
    M3<R> m;
#pragma unroll
    for (int e = 0; e < 9; ++e) {
        const store_t<R> v = buf[(slot * 9 + e) * NB + threadIdx.x];
        m.e[e / 3][e % 3] = Cx<R>{v.x, v.y};
    }
    return m;
}
template <typename R> struct Raw12 {
    store_t<R> v[6];  // rows 0 and 1 as stored
};
template <typename R> __device__ __forceinline__ M3<R> from_raw(const Raw12<R> &r)
{
    M3<R> m;
#pragma unroll
    for (int e = 0; e < 6; ++e) m.e[e / 3][e % 3] = Cx<R>{r.v[e].x, r.v[e].y};
    rebuild_row2(m);
    return m;
}
// The stash round trip must stay in LDS (kept in registers it would cost
// the occupancy it is meant to preserve): stash_fence() between the writes
// and the reads is a compiler-only memory barrier, so the compiler can
// neither forward the written values nor drop the writes.
template <typename R, int NB> __device__ __forceinline__ void stash_put(store_t<R> *stash, int slot, const Raw12<R> &r)
{
#pragma unroll
    for (int e = 0; e < 6; ++e) stash[(slot * 6 + e) * NB + threadIdx.x] = r.v[e];
}
template <typename R, int NB> __device__ __forceinline__ M3<R> stash_get(const store_t<R> *stash, int slot)
{
    Raw12<R> r;
#pragma unroll
    for (int e = 0; e < 6; ++e) r.v[e] = stash[(slot * 6 + e) * NB + threadIdx.x];
    return from_raw(r);
}
__device__ __forceinline__ void stash_fence() { __asm__ __volatile__("" ::: "memory"); }

template <int MU, typename R, bool HIT1, bool DLT, bool TWOB = false, bool MEAS = false, bool STASH = false,
          int NB = kBlock>
__device__ __forceinline__ void update_link(store_t<R> *__restrict__ links, const Geom &g, int par, int v, double beta,
                                            uint64_t sweep, uint64_t seed, int nhit, int &att, int &acc,
                                            store_t<R> *stash, double &tr, double &trx, const R *wb = nullptr)
{
    static_assert(!MEAS || (MU > 0 && !TWOB), "measured passes: MU = 1, 2, 3 with one coupling");
    constexpr bool CROSS = MEAS && DLT;
    // the staple directions nu != MU in increasing order
    constexpr int N0 = MU == 0 ? 1 : 0;
    constexpr int N1 = MU <= 1 ? 2 : 1;
    constexpr int N2 = MU <= 2 ? 3 : 2;
    const int layer = DLT && v >= g.Vh ? 1 : 0;
    int x[4];
    const int i = order_site(g, par, v - layer * g.Vh, x);
    const int n = layer * g.Vh + i;
    M3<R> A, S, Sx;
    if constexpr (CROSS) set_zero(Sx);
    constexpr bool EARLY = kEarlyDraws<R> && HIT1 && !TWOB;
    const uint64_t site = (uint64_t)layer * (uint64_t)(2 * g.Vh) + (uint64_t)lex_of(g, x);
    KPDraw<R> pre[3];
    __builtin_amdgcn_s_setprio(1);  // gathering the staple: issue loads ahead of waves in the heat bath
    if constexpr (TWOB) {
        const store_t<R> *umu = planes<R>(links, g, MU, par ^ 1);
        M3<R> b, e;
        set_zero(A);
        load_link12_pair<R>(b, umu, nbr_elem<N0, +1, MU, 0, true>(g, x, layer), e, umu,
                            nbr_elem<N0, -1, MU, 0, true>(g, x, layer));
        add_staple_twob<MU, N0, R>(A, b, e, links, g, x, layer, par, n, wb);
        load_link12_pair<R>(b, umu, nbr_elem<N1, +1, MU, 0, true>(g, x, layer), e, umu,
                            nbr_elem<N1, -1, MU, 0, true>(g, x, layer));
        add_staple_twob<MU, N1, R>(A, b, e, links, g, x, layer, par, n, wb);
        load_link12_pair<R>(b, umu, nbr_elem<N2, +1, MU, 0, true>(g, x, layer), e, umu,
                            nbr_elem<N2, -1, MU, 0, true>(g, x, layer));
        add_staple_twob<MU, N2, R>(A, b, e, links, g, x, layer, par, n, wb);
    } else if constexpr (!STASH) {
        // b and e of each direction loaded in its phase
        const store_t<R> *umu = planes<R>(links, g, MU, par ^ 1);
        M3<R> b, e, T;
        load_link12_pair<R>(b, umu, nbr_elem<N0, +1, MU, 0, DLT>(g, x, layer), e, umu,
                            nbr_elem<N0, -1, MU, 0, DLT>(g, x, layer));
        if constexpr (EARLY)
#pragma unroll
            for (int k = 0; k < 3; ++k) pre[k] = kp_draw<R>(seed, 4 * site + MU, sweep, k, 0);
        staple_dir<MU, N0, R, DLT, CROSS>(A, b, e, links, g, x, layer, par, n, Sx);
        if constexpr (MEAS && MU == 1) S = A;
        load_link12_pair<R>(b, umu, nbr_elem<N1, +1, MU, 0, DLT>(g, x, layer), e, umu,
                            nbr_elem<N1, -1, MU, 0, DLT>(g, x, layer));
        staple_dir<MU, N1, R, DLT, CROSS && (N1 < MU)>(T, b, e, links, g, x, layer, par, n, Sx);
        add_to(A, T);
        if constexpr (MEAS && MU == 2) S = A;
        load_link12_pair<R>(b, umu, nbr_elem<N2, +1, MU, 0, DLT>(g, x, layer), e, umu,
                            nbr_elem<N2, -1, MU, 0, DLT>(g, x, layer));
        staple_dir<MU, N2, R, DLT, CROSS && (N2 < MU)>(T, b, e, links, g, x, layer, par, n, Sx);
        add_to(A, T);
    } else {
        Raw12<R> b0, e0, b1, e1, b2, e2;
        {
            const store_t<R> *umu = planes<R>(links, g, MU, par ^ 1);
            const store_t<R> *pb0 = link_at<R>(umu, nbr_elem<N0, +1, MU, 0, DLT>(g, x, layer));
            const store_t<R> *pe0 = link_at<R>(umu, nbr_elem<N0, -1, MU, 0, DLT>(g, x, layer));
            const store_t<R> *pb1 = link_at<R>(umu, nbr_elem<N1, +1, MU, 0, DLT>(g, x, layer));
            const store_t<R> *pe1 = link_at<R>(umu, nbr_elem<N1, -1, MU, 0, DLT>(g, x, layer));
            const store_t<R> *pb2 = link_at<R>(umu, nbr_elem<N2, +1, MU, 0, DLT>(g, x, layer));
            const store_t<R> *pe2 = link_at<R>(umu, nbr_elem<N2, -1, MU, 0, DLT>(g, x, layer));
#pragma unroll
            for (int e = 0; e < 6; ++e) {
                b0.v[e] = pb0[e * kTile];
                e0.v[e] = pe0[e * kTile];
                b1.v[e] = pb1[e * kTile];
                e1.v[e] = pe1[e * kTile];
                b2.v[e] = pb2[e * kTile];
                e2.v[e] = pe2[e * kTile];
            }
        }
        if constexpr (EARLY)
#pragma unroll
            for (int k = 0; k < 3; ++k) pre[k] = kp_draw<R>(seed, 4 * site + MU, sweep, k, 0);
        stash_put<R, NB>(stash, 0, b1);
        stash_put<R, NB>(stash, 1, e1);
        stash_put<R, NB>(stash, 2, b2);
        stash_fence();
        M3<R> T;
        staple_dir<MU, N0, R, DLT, CROSS>(A, from_raw(b0), from_raw(e0), links, g, x, layer, par, n, Sx);
        if constexpr (MEAS && MU == 1) S = A;
        staple_dir<MU, N1, R, DLT, CROSS && (N1 < MU)>(T, stash_get<R, NB>(stash, 0), stash_get<R, NB>(stash, 1),
                                                       links, g, x, layer, par, n, Sx);
        add_to(A, T);
        if constexpr (MEAS && MU == 2) S = A;
        staple_dir<MU, N2, R, DLT, CROSS && (N2 < MU)>(T, stash_get<R, NB>(stash, 2), from_raw(e2), links, g, x,
                                                       layer, par, n, Sx);
        add_to(A, T);
    }
    if constexpr (CROSS) {
        // S and S_cross wait in LDS (`stash`, 2 * 9 * NB entries) across the heat bath
        if constexpr (MU < 3) park<R, NB>(stash, 0, S);
        park<R, NB>(stash, 1, Sx);
        stash_fence();
    }
    store_t<R> *own = planes<R>(links, g, MU, par);
    M3<R> U = load_link12_nt<R>(own, n);
    // with per-layer couplings the staple carries them: alpha = 2k/3
    __builtin_amdgcn_s_setprio(0);
    tr = heatbath<R, HIT1, EARLY>(U, A, TWOB ? 1.0 : beta, seed, 4 * site + MU, sweep, nhit, att, acc, pre);
    // FP64: nontemporal, so the written link does not displace staple links
    // from L2 (a plain store: -3 % at 32^4).  FP32, bound by issue rather
    // than memory: a plain store (+1 %)
    if constexpr (sizeof(R) == 8)
        store_link_nt<R>(own, n, U);
    else
        store_link<R>(own, n, U);
    if constexpr (CROSS) {
        stash_fence();
        if constexpr (MU < 3) tr = retr_mul(U, unpark<R, NB>(stash, 0));
        trx = retr_mul(U, unpark<R, NB>(stash, 1));
    } else if constexpr (MEAS && MU < 3) {
        tr = retr_mul(U, S);
    }
}

// Exact integer heat-bath counts: packed (attempts | accepts << 16) summed
// over the workgroup, then added to counter slot `slot`, so no two
// concurrent workgroups update the same address.
template <int NB = kBlock>
__device__ __forceinline__ void count_block(int att, int acc, unsigned long long *__restrict__ counters, int slot)
{
    unsigned packed = (unsigned)att | ((unsigned)acc << 16);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) packed += __shfl_xor(packed, off);
    __shared__ unsigned wsum[NB / 64];
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = packed;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long a = 0, b = 0;
#pragma unroll
        for (int w = 0; w < NB / 64; ++w) {
            a += wsum[w] & 0xffffu;
            b += wsum[w] >> 16;
        }
        if (a != 0) {
            unsigned long long *c = counters + 2 * slot;
            atomicAdd(&c[0], a);
            atomicAdd(&c[1], b);
        }
    }
}

// Sum of v over the workgroup, in a fixed order (valid in thread 0).
template <int NB = kBlock> __device__ __forceinline__ double block_sum(double v)
{
    __shared__ double wsum[NB / 64];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < NB / 64; ++w) s += wsum[w];
    return s;
}

// Tile of this workgroup in a pass of parity `par`.  Every pass reads the
// whole lattice, and the passes of a sweep alternate in parity, so the odd
// passes walk the tiles backwards: a pass begins on the links its
// predecessor read last, which are still in L2 and in the memory-side cache.
// The order does not change the result, only which links are in cache.
__device__ __forceinline__ int pass_tile(int par)
{
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    return par ? (int)gridDim.x - 1 - t : t;
}

// Sum of a per-layer value pair over the workgroup of a measured pass:
// layer 0 gets s0, layer 1 gets s1 (double-layered torus).
template <int NB>
__device__ __forceinline__ void store_meas(double *__restrict__ meas, bool dlt, double s0, double s1)
{
    __syncthreads();
    if (dlt) {
        const double b0 = block_sum<NB>(s0);
        __syncthreads();
        const double b1 = block_sum<NB>(s1);
        if (threadIdx.x == 0) {
            meas[2 * blockIdx.x] = b0;
            meas[2 * blockIdx.x + 1] = b1;
        }
    } else {
        const double b = block_sum<NB>(s0);
        if (threadIdx.x == 0) meas[blockIdx.x] = b;
    }
}

// One checkerboard pass, one lane per link, in workgroups of NB threads
// (kPassBlock on a single torus, kBlock on a double-layered one).  MEAS (odd
// passes of MU = 1, 2, 3): also store, per workgroup, the sum over its links of
// the final plaquettes of the planes (nu, MU), nu < MU, that update_link
// returns; on a double-layered torus one sum per layer, each plaquette filed
// under its base site's layer.
// The measured passes of a double-layered torus are compiled for one wave per
// SIMD (the whole register file; a 2 x 16^4 pass has one wave per SIMD anyway)
template <typename R, bool DLT, bool MEAS> constexpr int kUpdateWaves = (DLT && MEAS) ? 1 : kPassWaves<R>;

template <int MU, typename R, bool HIT1, bool DLT, bool MEAS = false, int NB = kBlock>
__global__ __launch_bounds__(NB, (kUpdateWaves<R, DLT, MEAS>)) void k_update(store_t<R> *__restrict__ links, const Geom g, const int par,
                                                   const double beta, const uint64_t sweep, const uint64_t seed,
                                                   const int nhit, unsigned long long *__restrict__ counters,
                                                   double *__restrict__ meas = nullptr)
{
    constexpr bool kStash = kStashPass<R, DLT, MU, MEAS>;
    store_t<R> *st = nullptr;
    if constexpr (kStash) {
        __shared__ store_t<R> stash[kStashSlots * 6 * NB];
        st = stash;
    } else if constexpr (MEAS && DLT) {
        __shared__ store_t<R> parked[2 * 9 * NB];
        st = parked;
    }
    const int v = pass_tile(par) * NB + threadIdx.x;
    int att = 0, acc = 0;
    double tr = 0.0, trx = 0.0;
    if (v < g.nlat * g.Vh)
        update_link<MU, R, HIT1, DLT, false, MEAS, kStash, NB>(links, g, par, v, beta, sweep, seed, nhit, att, acc,
                                                               st, tr, trx);
    count_block<NB>(att, acc, counters, blockIdx.x % kCounterSlots);
    if constexpr (MEAS) {
        // the cross-layer lower plaquettes go to the other layer
        const bool l1 = DLT && v >= g.Vh;
        store_meas<NB>(meas, DLT, l1 ? trx : tr - trx, l1 ? tr - trx : trx);
    }
}

// One pass of a double-layered torus with per-layer couplings beta0, beta1.
template <int MU, typename R, bool HIT1>
__global__ __launch_bounds__(kBlock, kPassWaves<R>) void k_update_twob(store_t<R> *__restrict__ links, const Geom g, const int par,
                                                        const double beta0, const double beta1, const uint64_t sweep,
                                                        const uint64_t seed, const int nhit,
                                                        unsigned long long *__restrict__ counters)
{
    const int v = pass_tile(par) * kBlock + threadIdx.x;
    const R b[2] = {R(beta0), R(beta1)};
    int att = 0, acc = 0;
    double tr, trx;
    if (v < g.nlat * g.Vh)
        update_link<MU, R, HIT1, true, true>(links, g, par, v, 1.0, sweep, seed, nhit, att, acc, nullptr, tr, trx, b);
    count_block(att, acc, counters, blockIdx.x % kCounterSlots);
}

// ---------------------------------------------------------------------------
// Several lanes per link (K = 2 or 4, 1-hit): for passes too small to fill
// the GPU with one lane per link, where a pass takes about one update's
// latency.  The K lanes of a link (a quad-aligned group) split the work that
// does not depend on the link's state: lane q computes the staple part
// D_{nu_q} of direction nu_q and the random draw of subgroup q, with the same
// instructions in every lane (the direction is a per-lane value), then the
// parts are added across the group with DPP quad permutes in the canonical
// order (D_0 + D_1) + D_2 and every lane runs the heat bath on the full staple.
//  * K = 4: lanes 0, 1, 2 take directions N0, N1, N2 and subgroups 0, 1, 2;
//    lane 3 repeats lane 2.  Lanes 2 and 3 each halve D_2 (exact), so the
//    butterfly xor 1 gives D_0 + D_1 and D_2/2 + D_2/2 = D_2, and xor 2 gives
//    (D_0 + D_1) + D_2 in every lane.
//  * K = 2: lanes 0, 1 take N0, N1 and subgroups 0, 1; both lanes then form
//    D_2 and draw subgroup 2.  xor 1 gives D_0 + D_1; + D_2.
// Lane 0 stores the link and counts; the values are those of the one-lane
// pass, bit for bit.
// ---------------------------------------------------------------------------
constexpr int kDppXor1 = 0xB1;  // quad_perm [1, 0, 3, 2]
constexpr int kDppXor2 = 0x4E;  // quad_perm [2, 3, 0, 1]
constexpr int dpp_bcast(int k) { return k * 0x55; }  // quad_perm [k, k, k, k]

template <int CTRL> __device__ __forceinline__ float dpp(float x)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}
template <int CTRL> __device__ __forceinline__ double dpp(double x)
{
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
// M += (M of the partner lane)
template <int CTRL, typename R> __device__ __forceinline__ void add_partner(M3<R> &m)
{
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            m.e[r][c].re = m.e[r][c].re + dpp<CTRL>(m.e[r][c].re);
            m.e[r][c].im = m.e[r][c].im + dpp<CTRL>(m.e[r][c].im);
        }
}
template <int CTRL, typename R> __device__ __forceinline__ KPDraw<R> dpp_draw(const KPDraw<R> &d)
{
    return KPDraw<R>{dpp<CTRL>(d.q), dpp<CTRL>(d.u4sq), dpp<CTRL>(d.cth), dpp<CTRL>(d.sc), dpp<CTRL>(d.ss)};
}
template <typename R> __device__ __forceinline__ KPDraw<R> select_draw(bool p, const KPDraw<R> &a, const KPDraw<R> &b)
{
    return p ? a : b;
}

// Plane elements of x + nu, x - nu and x + MU - nu for a direction nu != MU
// held at run time (one per lane), and whether x - nu lies in the other layer.
template <int MU, bool DLT> struct NuElems {
    int xp, xm, xmu_m;
    bool cross;
};
template <int MU, bool DLT>
__device__ __forceinline__ NuElems<MU, DLT> nu_elems(const Geom &g, const int x[4], int layer, int nu)
{
    const int L0 = g.L[0], L1 = g.L[1], L2 = g.L[2], L3 = g.L[3];
    const int xs = nu == 0 ? x[0] : nu == 1 ? x[1] : nu == 2 ? x[2] : x[3];
    const int Ln = nu == 0 ? L0 : nu == 1 ? L1 : nu == 2 ? L2 : L3;
    const int sn = nu == 0 ? 1 : nu == 1 ? L0 : nu == 2 ? L0 * L1 : L0 * L1 * L2;
    const int fb = DLT ? (int)((g.flip >> nu) & 1u) : 0;
    const bool top = xs == Ln - 1, bot = xs == 0;
    const int wrap = (Ln - 1) * sn;
    const int lex = lex_of(g, x);
    int y[4] = {x[0], x[1], x[2], x[3]};
    int lmu = layer;
    step<MU, +1, DLT>(g, y, lmu);  // x + MU; its nu coordinate is x's
    const int lex_mu = lex_of(g, y);
    const int lp = top ? lex - wrap : lex + sn, lyp = layer ^ (top ? fb : 0);
    const int lm = bot ? lex + wrap : lex - sn, lym = layer ^ (bot ? fb : 0);
    const int lmm = bot ? lex_mu + wrap : lex_mu - sn, lymm = lmu ^ (bot ? fb : 0);
    NuElems<MU, DLT> r;
    r.xp = DLT ? lyp * g.Vh + (lp >> 1) : lp >> 1;
    r.xm = DLT ? lym * g.Vh + (lm >> 1) : lm >> 1;
    r.xmu_m = DLT ? lymm * g.Vh + (lmm >> 1) : lmm >> 1;
    r.cross = DLT && bot && fb;
    return r;
}

// D_nu for a direction held at run time (the loads of staple_dir, addresses per lane).
template <int MU, typename R, bool DLT, bool CROSS>
__device__ __forceinline__ void staple_dir_rt(M3<R> &D, const store_t<R> *__restrict__ links, const Geom &g,
                                              const int x[4], int layer, int par, int n, int nu, M3<R> &cross)
{
    const int opp = par ^ 1;
    const NuElems<MU, DLT> ne = nu_elems<MU, DLT>(g, x, layer, nu);
    const store_t<R> *umu = planes<R>(links, g, MU, opp);
    const store_t<R> *unu_par = links + (size_t)(nu * 2 + par) * (size_t)g.stride * kEntries;
    const store_t<R> *unu_opp = links + (size_t)(nu * 2 + opp) * (size_t)g.stride * kEntries;
    M3<R> b, e, c, d, a, f;
    load_link12_pair<R>(b, umu, ne.xp, e, umu, ne.xm);
    load_link12_pair<R>(c, unu_par, n, d, unu_par, ne.xmu_m);
    const M3<R> cb = mul_nn_su3(c, b);
    const M3<R> ed = mul_nn_su3(e, d);
    load_link12_pair<R>(a, unu_opp, nbr_elem<MU, +1, MU, 0, DLT>(g, x, layer), f, unu_opp, ne.xm);
    staple_term<R, CROSS>(D, a, cb, ed, f, cross, CROSS && ne.cross);
}

// M *= s (s = 1 or 1/2: exact)
template <typename R> __device__ __forceinline__ void scale_by(M3<R> &m, R s)
{
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            m.e[r][c].re *= s;
            m.e[r][c].im *= s;
        }
}

// Lane q of the K-lane group of the link U_MU at pass-order position v.
// MEAS: tr, trx as update_link, split over the lanes (each lane's share of S
// and S_cross; the workgroup sum adds them up).
template <int MU, typename R, bool DLT, bool MEAS, int K>
__device__ __forceinline__ void update_link_lanes(store_t<R> *__restrict__ links, const Geom &g, int par, int v,
                                                  int q, double beta, uint64_t sweep, uint64_t seed, bool active,
                                                  int &att, int &acc, double &tr, double &trx)
{
    static_assert(K == 2 || K == 4, "2 or 4 lanes per link");
    static_assert(!MEAS || MU > 0, "measured passes: MU = 1, 2, 3");
    constexpr bool CROSS = MEAS && DLT;
    constexpr int N0 = MU == 0 ? 1 : 0;
    constexpr int N1 = MU <= 1 ? 2 : 1;
    constexpr int N2 = MU <= 2 ? 3 : 2;
    const int layer = DLT && v >= g.Vh ? 1 : 0;
    int x[4];
    const int i = order_site(g, par, v - layer * g.Vh, x);
    const int n = layer * g.Vh + i;
    const uint64_t site = (uint64_t)layer * (uint64_t)(2 * g.Vh) + (uint64_t)lex_of(g, x);
    const uint64_t lid = 4 * site + MU;
    const int sub = q < 2 ? q : 2;  // K = 4: lane 3 repeats lane 2
    const int nu = sub == 0 ? N0 : (sub == 1 ? N1 : N2);
    M3<R> A, S, Sx;
    if constexpr (CROSS) set_zero(Sx);
    __builtin_amdgcn_s_setprio(1);
    staple_dir_rt<MU, R, DLT, CROSS>(A, links, g, x, layer, par, n, nu, Sx);
    const KPDraw<R> mine = kp_draw<R>(seed, lid, sweep, sub, 0);
    KPDraw<R> pre[3];
    if constexpr (K == 4) {
        if (q >= 2) {
            scale_by(A, R(0.5));
            if constexpr (CROSS) scale_by(Sx, R(0.5));
        }
        if constexpr (MEAS) {
            S = A;
            if (nu > MU) set_zero(S);
            if constexpr (CROSS)
                if (nu > MU) set_zero(Sx);
        }
        add_partner<kDppXor1>(A);
        add_partner<kDppXor2>(A);
        pre[0] = dpp_draw<dpp_bcast(0)>(mine);
        pre[1] = dpp_draw<dpp_bcast(1)>(mine);
        pre[2] = dpp_draw<dpp_bcast(2)>(mine);
    } else {
        if constexpr (MEAS) {
            S = A;
            if (nu > MU) set_zero(S);
            if constexpr (CROSS)
                if (nu > MU) set_zero(Sx);
        }
        add_partner<kDppXor1>(A);
        M3<R> T;
        // D_2 in both lanes; its measured share (MU = 3) and cross share in lane 0
        {
            const store_t<R> *umu = planes<R>(links, g, MU, par ^ 1);
            M3<R> b, e;
            load_link12_pair<R>(b, umu, nbr_elem<N2, +1, MU, 0, DLT>(g, x, layer), e, umu,
                                nbr_elem<N2, -1, MU, 0, DLT>(g, x, layer));
            staple_dir<MU, N2, R, DLT, CROSS && (N2 < MU)>(T, b, e, links, g, x, layer, par, n, Sx, q == 0);
        }
        add_to(A, T);
        if constexpr (MEAS && N2 < MU)
            if (q == 0) add_to(S, T);
        const KPDraw<R> other = dpp_draw<kDppXor1>(mine);
        pre[0] = select_draw(q == 0, mine, other);
        pre[1] = select_draw(q == 0, other, mine);
        pre[2] = kp_draw<R>(seed, lid, sweep, 2, 0);
    }
    store_t<R> *own = planes<R>(links, g, MU, par);
    M3<R> U = load_link12_nt<R>(own, n);
    __builtin_amdgcn_s_setprio(0);
    int a_ = 0, c_ = 0;
    heatbath<R, true, true>(U, A, beta, seed, lid, sweep, 1, a_, c_, pre);
    if (active && q == 0) {
        att += a_;
        acc += c_;
        if constexpr (sizeof(R) == 8)
            store_link_nt<R>(own, n, U);
        else
            store_link<R>(own, n, U);
    }
    if constexpr (MEAS) {
        tr = active ? retr_mul(U, S) : 0.0;
        if constexpr (CROSS) trx = active ? retr_mul(U, Sx) : 0.0;
    }
}

// One pass with K lanes per link in workgroups of kBlock threads (kBlock / K links).
template <int MU, typename R, bool DLT, bool MEAS, int K>
__global__ __launch_bounds__(kBlock, 2) void k_update_lanes(store_t<R> *__restrict__ links, const Geom g, const int par,
                                                         const double beta, const uint64_t sweep, const uint64_t seed,
                                                         unsigned long long *__restrict__ counters,
                                                         double *__restrict__ meas)
{
    constexpr int kLinks = kBlock / K;
    const int q = threadIdx.x & (K - 1);
    const int nlinks = g.nlat * g.Vh;
    int v = pass_tile(par) * kLinks + threadIdx.x / K;
    const bool active = v < nlinks;
    if (!active) v = nlinks - 1;  // every lane takes part in the exchanges; nothing is stored
    int att = 0, acc = 0;
    double tr = 0.0, trx = 0.0;
    update_link_lanes<MU, R, DLT, MEAS, K>(links, g, par, v, q, beta, sweep, seed, active, att, acc, tr, trx);
    count_block<kBlock>(att, acc, counters, blockIdx.x % kCounterSlots);
    if constexpr (MEAS) {
        const bool l1 = DLT && v >= g.Vh;
        store_meas<kBlock>(meas, DLT, l1 ? trx : tr - trx, l1 ? tr - trx : trx);
    }
}

// Polyakov loops along direction 3: thread (layer, x0, x1, x2) walks the
// closed path x3 = 0, 1, ... (2 L3 links when crossing the direction-3
// boundary switches the layer) multiplying U_3 in FP64; partial sums of
// Re and Im of Tr/3 per workgroup and layer.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_polyakov(const store_t<R> *__restrict__ links, const Geom g,
                                                     double *__restrict__ partials)
{
    const int layer = blockIdx.y;
    const int V3 = g.L[0] * g.L[1] * g.L[2];
    const int s = blockIdx.x * kBlock + threadIdx.x;
    double re = 0.0, im = 0.0;
    if (s < V3) {
        int y[4] = {s % g.L[0], (s / g.L[0]) % g.L[1], s / (g.L[0] * g.L[1]), 0};
        int ly = layer;
        M3<double> P;
        set_zero(P);
        P.e[0][0].re = P.e[1][1].re = P.e[2][2].re = 1.0;
        do {
            const int lex = lex_of(g, y);
            const int par = (y[0] + y[1] + y[2] + y[3]) & 1;
            const M3<double> u = convert<double>(load_link12<R>(planes<R>(links, g, 3, par), ly * g.Vh + (lex >> 1)));
            P = mul_nn(P, u);
            step<3, +1, true>(g, y, ly);
        } while (y[3] != 0 || ly != layer);
        re = (P.e[0][0].re + P.e[1][1].re + P.e[2][2].re) / 3.0;
        im = (P.e[0][0].im + P.e[1][1].im + P.e[2][2].im) / 3.0;
    }
    const double br = block_sum(re);
    __syncthreads();
    const double bi = block_sum(im);
    if (threadIdx.x == 0) {
        partials[2 * (layer * gridDim.x + blockIdx.x)] = br;
        partials[2 * (layer * gridDim.x + blockIdx.x) + 1] = bi;
    }
}

// out[2 l], out[2 l + 1] = sums of Re, Im over the partials of layer l (fixed order)
__global__ __launch_bounds__(kBlock) void k_polyakov_final(const double *__restrict__ partials, int nblk, int nlat,
                                                           double *__restrict__ out)
{
    for (int l = 0; l < nlat; ++l)
        for (int c = 0; c < 2; ++c) {
            double s = 0.0;
            for (int b = threadIdx.x; b < nblk; b += kBlock) s += partials[2 * (l * nblk + b) + c];
            const double r = block_sum(s);
            __syncthreads();
            if (threadIdx.x == 0) out[2 * l + c] = r;
        }
}

// Batched pass: one launch updates the links U_MU of parity `par` of every
// job in `jobs` (sorted by tile_begin).  The grid has one workgroup per tile
// of the batch; logical tile t (pass_tile) belongs to the job whose tile range
// holds t; job j is at sweep index sweep0 + (step - admit_step).  A 1-hit job
// with two lanes per link (the host's choice for a small batch, whose pass is
// bound by the latency of one update) takes 32 links per workgroup and runs
// update_link_lanes; its links are the same bits either way.
template <int MU, typename R, bool HIT1, bool DLT>
__global__ __launch_bounds__(kPassBlock, kPassWaves<R>) void k_update_batch(const BatchJob *__restrict__ jobs, const int njobs,
                                                             const long long step, const int par)
{
    constexpr bool kStash = kStashBatch<R, DLT>;
    store_t<R> *st = nullptr;
    if constexpr (kStash) {
        __shared__ store_t<R> stash[kStashSlots * 6 * kPassBlock];
        st = stash;
    }
    // the XCD-aware, parity-reversed tile of the whole batch, as for one
    // lattice: each XCD works on contiguous stretches of each job's tiles
    const int t = pass_tile(par);
    __shared__ int sj;
    if (threadIdx.x == 0) {
        int lo = 0, hi = njobs - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (jobs[mid].tile_begin <= t)
                lo = mid;
            else
                hi = mid - 1;
        }
        sj = lo;
    }
    __syncthreads();
    const BatchJob &J = jobs[sj];
    const int local = t - J.tile_begin;
    const uint64_t sweep = J.sweep0 + (uint64_t)(step - J.admit_step);
    const int nlinks = J.g.nlat * J.g.Vh;
    int att = 0, acc = 0;
    double tr, trx;
    if (HIT1 && J.lanes == 2) {
        int v = local * (kPassBlock / 2) + (int)(threadIdx.x >> 1);
        const bool active = v < nlinks;
        if (!active) v = nlinks - 1;  // both lanes take part in the exchanges; nothing is stored
        update_link_lanes<MU, R, DLT, false, 2>((store_t<R> *)J.links, J.g, par, v, (int)(threadIdx.x & 1), J.beta,
                                                sweep, J.seed, active, att, acc, tr, trx);
    } else {
        const int v = local * kPassBlock + threadIdx.x;
        if (v < nlinks)
            update_link<MU, R, HIT1, DLT, false, false, kStash, kPassBlock>((store_t<R> *)J.links, J.g, par, v,
                                                                            J.beta, sweep, J.seed, J.nhit, att, acc,
                                                                            st, tr, trx);
    }
    count_block<kPassBlock>(att, acc, J.counters, local % kCounterSlots);
}

// ---------------------------------------------------------------------------
// start configurations, reunitarisation, gauge transformation: one thread per
// link; blockIdx.y = dir * 2 + parity
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool link_of_thread(const Geom &g, int &n, int &dir, int &par, int &layer, int x[4])
{
    n = blockIdx.x * kBlock + threadIdx.x;
    if (n >= g.nlat * g.Vh) return false;
    dir = blockIdx.y >> 1;
    par = blockIdx.y & 1;
    layer = n >= g.Vh ? 1 : 0;
    site_coords(g, par, n - layer * g.Vh, x);
    return true;
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_start(store_t<R> *__restrict__ links, const Geom g, const int hot,
                                                  const uint64_t seed)
{
    int n, dir, par, layer, x[4];
    if (!link_of_thread(g, n, dir, par, layer, x)) return;
    M3<double> u;
    if (hot) {
        const uint64_t site = (uint64_t)layer * (uint64_t)(2 * g.Vh) + (uint64_t)lex_of(g, x);
        u = haar_element(seed, 4 * site + dir, kTagHot);
    } else {
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c) u.e[r][c] = Cx<double>{r == c ? 1.0 : 0.0, 0.0};
    }
    store_link<R>(planes<R>(links, g, dir, par), n, convert<R>(u));
}

template <typename R> __global__ __launch_bounds__(kBlock) void k_reunit(store_t<R> *__restrict__ links, const Geom g)
{
    int n, dir, par, layer, x[4];
    if (!link_of_thread(g, n, dir, par, layer, x)) return;
    store_t<R> *base = planes<R>(links, g, dir, par);
    M3<double> u = convert<double>(load_link12<R>(base, n));
    reunit(u);
    store_link<R>(base, n, convert<R>(u));
}

template <int D>
__device__ __forceinline__ uint64_t forward_site(const Geom &g, const int x[4], int layer)
{
    int y[4] = {x[0], x[1], x[2], x[3]};
    int ly = layer;
    step<D, +1>(g, y, ly);
    return (uint64_t)ly * (uint64_t)(2 * g.Vh) + (uint64_t)lex_of(g, y);
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_gauge(store_t<R> *__restrict__ links, const Geom g, const uint64_t gseed)
{
    int n, dir, par, layer, x[4];
    if (!link_of_thread(g, n, dir, par, layer, x)) return;
    const uint64_t site = (uint64_t)layer * (uint64_t)(2 * g.Vh) + (uint64_t)lex_of(g, x);
    uint64_t fwd;
    switch (dir) {
    case 0: fwd = forward_site<0>(g, x, layer); break;
    case 1: fwd = forward_site<1>(g, x, layer); break;
    case 2: fwd = forward_site<2>(g, x, layer); break;
    default: fwd = forward_site<3>(g, x, layer); break;
    }
    const M3<double> gx = haar_element(gseed, site, kTagGauge);
    const M3<double> gy = haar_element(gseed, fwd, kTagGauge);
    store_t<R> *base = planes<R>(links, g, dir, par);
    const M3<double> u = convert<double>(load_link12<R>(base, n));
    const M3<double> t = mul_nn(gx, u);
    M3<double> out;
    set_zero(out);
    acc_nd(out, t, gy);
    store_link<R>(base, n, convert<R>(out));
}

// ---------------------------------------------------------------------------
// plaquette: sum over sites of Re Tr U_mu(x) U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+
// = Re Tr P Q^+ with P = U_mu(x) U_nu(x+mu), Q = U_nu(x) U_mu(x+nu), in FP64.
// Grid (nblk, nlat); fixed per-thread order, wave shuffles and a fixed
// per-block order, so the sum is bitwise reproducible.
// ---------------------------------------------------------------------------
// Rows 0 and 1 of a link (row 2 never formed), in FP64.
template <typename R> __device__ __forceinline__ M3<double> load_rows01(const store_t<R> *block, int n)
{
    M3<double> m;
    const store_t<R> *p = link_at<R>(block, n);
#pragma unroll
    for (int e = 0; e < 6; ++e) {
        const store_t<R> v = p[e * kTile];
        m.e[e / 3][e % 3] = Cx<double>{(double)v.x, (double)v.y};
    }
    return m;
}

// Plane (MU, NU) of a site whose own links U (rows 0, 1) are already held:
// Re Tr P Q^+ with P = U_MU(x) U_NU(x+MU), Q = U_NU(x) U_MU(x+NU), both
// SU(3) products formed as rows 0, 1 with row 2 rebuilt.
template <int MU, int NU, typename R, bool DLT>
__device__ __forceinline__ double plaq_plane_own(const store_t<R> *__restrict__ links, const Geom &g, const int x[4],
                                                 int layer, int par, const M3<double> *U)
{
    const int opp = par ^ 1;
    const M3<double> P = mul_nn_su3(
        U[MU], convert<double>(load_link12<R>(planes<R>(links, g, NU, opp), nbr_elem<MU, +1, NU, 0, DLT>(g, x, layer))));
    const M3<double> Q = mul_nn_su3(
        U[NU], convert<double>(load_link12<R>(planes<R>(links, g, MU, opp), nbr_elem<NU, +1, MU, 0, DLT>(g, x, layer))));
    double s = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) s += P.e[a][b].re * Q.e[a][b].re + P.e[a][b].im * Q.e[a][b].im;
    return s;
}

// 1 if the stored rows 0 and 1 of u are not finite or not orthonormal within
// tol (|r0|^2 - 1, |r1|^2 - 1, <r0, r1>), else 0.  Row 2 is conj(r0 x r1), so
// orthonormal rows 0 and 1 make u an SU(3) matrix.  NaN fails every test.
__device__ __forceinline__ int link_bad(const M3<double> &u, double tol)
{
    double n0 = 0.0, n1 = 0.0;
    Cx<double> d{0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        n0 += u.e[0][k].re * u.e[0][k].re + u.e[0][k].im * u.e[0][k].im;
        n1 += u.e[1][k].re * u.e[1][k].re + u.e[1][k].im * u.e[1][k].im;
        d = cmadd_cn(d, u.e[0][k], u.e[1][k]);
    }
    const bool ok = fabs(n0 - 1.0) <= tol && fabs(n1 - 1.0) <= tol && fabs(d.re) <= tol && fabs(d.im) <= tol;
    return ok ? 0 : 1;
}

// FP32 plaquette: the six planes of the site and the check of its four own
// links.  The four own links are loaded once and kept, and compiler-only
// fences between the planes hold the neighbour loads back (two waves per
// SIMD: 87 instead of 122 us at 32^4).
template <typename R, bool DLT>
__device__ __forceinline__ double plaq_site(const store_t<R> *__restrict__ links, const Geom &g, int layer, int par,
                                           int i, double tol, int &bad)
{
    int x[4];
    site_coords(g, par, i, x);
    const int n = layer * g.Vh + i;
    M3<double> U[4];
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        U[mu] = load_rows01<R>(planes<R>(links, g, mu, par), n);
        bad += link_bad(U[mu], tol);
    }
    double s = plaq_plane_own<0, 1, R, DLT>(links, g, x, layer, par, U);
    stash_fence();
    s += plaq_plane_own<0, 2, R, DLT>(links, g, x, layer, par, U);
    stash_fence();
    s += plaq_plane_own<1, 2, R, DLT>(links, g, x, layer, par, U);
    stash_fence();
    s += plaq_plane_own<0, 3, R, DLT>(links, g, x, layer, par, U);
    stash_fence();
    s += plaq_plane_own<1, 3, R, DLT>(links, g, x, layer, par, U);
    stash_fence();
    s += plaq_plane_own<2, 3, R, DLT>(links, g, x, layer, par, U);
    stash_fence();
    return s;
}

// Grid (nblk, nlat).  Workgroup b (XCD-remapped) sums the contiguous run of
// tiles [b T, (b+1) T) of its layer in the pass order; thread v of a tile
// takes both sites with half-index i(v) (x0 neighbours), so the links of both
// parities around a domain are read while they are in that XCD's L2.  Fixed
// per-thread order, wave shuffles and a fixed per-block order: the sum is
// bitwise reproducible.  partials[l nblk + b]: plaquette sum of workgroup b
// of layer l; partials[(nlat + l) nblk + b]: its number of failing links.
template <typename R, bool DLT>
__global__ __launch_bounds__(kBlock) void k_plaq_partial(const store_t<R> *__restrict__ links, const Geom g,
                                                         const int tiles_per_block, const double tol,
                                                         double *__restrict__ partials)
{
    const int layer = DLT ? (int)blockIdx.y : 0;
    const int b = xcd_tile(blockIdx.x, gridDim.x);
    double s = 0.0;
    int bad = 0;
    for (int t = 0; t < tiles_per_block; ++t) {
        const int v = (b * tiles_per_block + t) * kBlock + threadIdx.x;
        if (v < g.Vh) {
            const int i = order_index(g, v);
            s += plaq_site<R, DLT>(links, g, layer, 0, i, tol, bad);
            s += plaq_site<R, DLT>(links, g, layer, 1, i, tol, bad);
        }
    }
    const double bs = block_sum(s);
    __syncthreads();
    const double bb = block_sum((double)bad);
    if (threadIdx.x == 0) {
        partials[blockIdx.y * gridDim.x + blockIdx.x] = bs;
        partials[(gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = bb;
    }
}

// FP64 plaquette, one site per thread: thread w of a tile takes the site with
// half-index i(w / 2) and parity w % 2, so the two threads of a half-index
// read the two parity blocks at the same element.  The six planes (mu, nu)
// each load their four links and form P and Q as SU(3) products (rows 0, 1,
// row 2 rebuilt).  At 32^4: 168 us against 225 us for two sites per thread,
// which needs 256 VGPRs plus 123 AGPRs (one wave per SIMD).  (Fencing the
// planes to cut registers further pins every temporary and spills.)  FP32
// keeps k_plaq_partial, whose fenced planes with held own links take 86 us
// against 120 us.
template <int MU, int NU, typename R, bool DLT>
__device__ __forceinline__ double plaq_plane_su3(const store_t<R> *__restrict__ links, const Geom &g, const int x[4],
                                                 int layer, int par, int n)
{
    const int opp = par ^ 1;
    const M3<double> P = mul_nn_su3(
        convert<double>(load_link12<R>(planes<R>(links, g, MU, par), n)),
        convert<double>(load_link12<R>(planes<R>(links, g, NU, opp), nbr_elem<MU, +1, NU, 0, DLT>(g, x, layer))));
    const M3<double> Q = mul_nn_su3(
        convert<double>(load_link12<R>(planes<R>(links, g, NU, par), n)),
        convert<double>(load_link12<R>(planes<R>(links, g, MU, opp), nbr_elem<NU, +1, MU, 0, DLT>(g, x, layer))));
    double s = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) s += P.e[a][b].re * Q.e[a][b].re + P.e[a][b].im * Q.e[a][b].im;
    return s;
}

template <typename R, bool DLT>
__device__ __forceinline__ double plaq_site1(const store_t<R> *__restrict__ links, const Geom &g, int layer,
                                            int par, int i, double tol, int &bad)
{
    int x[4];
    site_coords(g, par, i, x);
    const int n = layer * g.Vh + i;
    double s = plaq_plane_su3<0, 1, R, DLT>(links, g, x, layer, par, n);
    s += plaq_plane_su3<0, 2, R, DLT>(links, g, x, layer, par, n);
    s += plaq_plane_su3<1, 2, R, DLT>(links, g, x, layer, par, n);
    s += plaq_plane_su3<0, 3, R, DLT>(links, g, x, layer, par, n);
    s += plaq_plane_su3<1, 3, R, DLT>(links, g, x, layer, par, n);
    s += plaq_plane_su3<2, 3, R, DLT>(links, g, x, layer, par, n);
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) bad += link_bad(load_rows01<R>(planes<R>(links, g, mu, par), n), tol);
    return s;
}

template <typename R, bool DLT>
__global__ __launch_bounds__(kBlock, 2) void k_plaq_sites(const store_t<R> *__restrict__ links,
                                                                       const Geom g, const int tiles_per_block,
                                                                       const double tol, double *__restrict__ partials)
{
    const int layer = DLT ? (int)blockIdx.y : 0;
    const int b = xcd_tile(blockIdx.x, gridDim.x);
    double s = 0.0;
    int bad = 0;
    for (int t = 0; t < tiles_per_block; ++t) {
        const int w = (b * tiles_per_block + t) * kBlock + threadIdx.x;
        if (w < 2 * g.Vh) s += plaq_site1<R, DLT>(links, g, layer, w & 1, order_index(g, w >> 1), tol, bad);
    }
    const double bs = block_sum(s);
    __syncthreads();
    const double bb = block_sum((double)bad);
    if (threadIdx.x == 0) {
        partials[blockIdx.y * gridDim.x + blockIdx.x] = bs;
        partials[(gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = bb;
    }
}

// Re Tr P Q^+ of two SU(3) matrices given by rows 0 and 1 (row 2 rebuilt).
__device__ __forceinline__ double retr_pq12(M3<double> P, M3<double> Q)
{
    rebuild_row2(P);
    rebuild_row2(Q);
    double s = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) s += P.e[a][b].re * Q.e[a][b].re + P.e[a][b].im * Q.e[a][b].im;
    return s;
}

// One column of the plaquette walk: the sites (x0, x1, x2, x3) of the
// thread's chunk [x3a, x3b) of x3, in increasing x3.  At each site the four
// own links are loaded once (and checked); the planes (mu, nu), nu < 3, take
// the links of the forward neighbours x + mu in the same x3 slab.  A plane
// (mu, 3) needs U_mu(x + 3), the next site's own link:
//   Re Tr U_mu(x) U_3(x + mu) U_mu(x + 3)^+ U_3(x)^+ = Re Tr M_mu U_mu(x + 3)^+,
//   M_mu = U_3(x)^+ U_mu(x) U_3(x + mu),
// so M_mu (rows 0, 1) is formed at x and carried to the next site.  Every
// link is then read as an own link and by its three backward neighbours in
// the same step of the walk, each own link is loaded and checked once, and
// only the last site of a chunk reads links of the slab above it.
// Summation order: fixed per thread.
template <typename R, bool DLT>
__device__ __forceinline__ double plaq_column(const store_t<R> *__restrict__ links, const Geom &g, int layer,
                                              int nch, int w, double tol, int &bad)
{
    int x[4];
    const int c = walk_column(g, nch, w, x);
    const int x3a = (int)((long long)c * g.L[3] / nch), x3b = (int)((long long)(c + 1) * g.L[3] / nch);
    const int lbase = DLT ? layer * g.Vh : 0;
    M3<double> M0, M1, M2;
    double s = 0.0;
    for (int x3 = x3a; x3 < x3b; ++x3) {
        x[3] = x3;
        const int par = (x[0] + x[1] + x[2] + x3) & 1, opp = par ^ 1;
        const int n = lbase + (lex_of(g, x) >> 1);
        const M3<double> U0 = load_rows01<R>(planes<R>(links, g, 0, par), n);
        const M3<double> U1 = load_rows01<R>(planes<R>(links, g, 1, par), n);
        const M3<double> U2 = load_rows01<R>(planes<R>(links, g, 2, par), n);
        M3<double> U3 = load_rows01<R>(planes<R>(links, g, 3, par), n);
        bad += link_bad(U0, tol) + link_bad(U1, tol) + link_bad(U2, tol) + link_bad(U3, tol);
        if (x3 > x3a) {
            // planes (mu, 3) of the site below
            s += retr_pq12(M0, U0);
            s += retr_pq12(M1, U1);
            s += retr_pq12(M2, U2);
        }
        const int e0 = nbr_elem<0, +1, 0, 0, DLT>(g, x, layer);
        const int e1 = nbr_elem<1, +1, 0, 0, DLT>(g, x, layer);
        const int e2 = nbr_elem<2, +1, 0, 0, DLT>(g, x, layer);
        rebuild_row2(U3);
        s += retr_pq12(mul_nn_su3(U0, convert<double>(load_link12<R>(planes<R>(links, g, 1, opp), e0))),
                       mul_nn_su3(U1, convert<double>(load_link12<R>(planes<R>(links, g, 0, opp), e1))));
        s += retr_pq12(mul_nn_su3(U0, convert<double>(load_link12<R>(planes<R>(links, g, 2, opp), e0))),
                       mul_nn_su3(U2, convert<double>(load_link12<R>(planes<R>(links, g, 0, opp), e2))));
        M0 = mul_dn_su3(U3, mul_nn_su3(U0, convert<double>(load_link12<R>(planes<R>(links, g, 3, opp), e0))));
        s += retr_pq12(mul_nn_su3(U1, convert<double>(load_link12<R>(planes<R>(links, g, 2, opp), e1))),
                       mul_nn_su3(U2, convert<double>(load_link12<R>(planes<R>(links, g, 1, opp), e2))));
        M1 = mul_dn_su3(U3, mul_nn_su3(U1, convert<double>(load_link12<R>(planes<R>(links, g, 3, opp), e1))));
        M2 = mul_dn_su3(U3, mul_nn_su3(U2, convert<double>(load_link12<R>(planes<R>(links, g, 3, opp), e2))));
    }
    if (x3b > x3a) {
        // planes (mu, 3) of the chunk's last site: the links of the slab above
        x[3] = x3b - 1;
        const int opp = ((x[0] + x[1] + x[2] + x[3]) & 1) ^ 1;
        const int e3 = nbr_elem<3, +1, 0, 0, DLT>(g, x, layer);
        s += retr_pq12(M0, load_rows01<R>(planes<R>(links, g, 0, opp), e3));
        s += retr_pq12(M1, load_rows01<R>(planes<R>(links, g, 1, opp), e3));
        s += retr_pq12(M2, load_rows01<R>(planes<R>(links, g, 2, opp), e3));
    }
    return s;
}

// Plaquette of large FP64 lattices by walking x3: grid (nblk, nlat),
// workgroup b (XCD-remapped) takes the threads [b T, (b+1) T) of the column
// order (walk_column), T = tiles_per_block kPlaqWalkBlock.  Output as
// k_plaq_partial.  At 32^4 (4 chunks of 8, two waves per SIMD): 143 us
// against 166 us for one site per thread; at 24^4 53 against 70 us.
template <typename R, bool DLT>
__global__ __launch_bounds__(kPlaqWalkBlock, 2) void k_plaq_walk(const store_t<R> *__restrict__ links, const Geom g,
                                                                 const int nch, const int tiles_per_block,
                                                                 const double tol, double *__restrict__ partials)
{
    const int layer = DLT ? (int)blockIdx.y : 0;
    const int b = xcd_tile(blockIdx.x, gridDim.x);
    const int nthreads = g.L[0] * g.L[1] * g.L[2] * nch;
    double s = 0.0;
    int bad = 0;
    for (int t = 0; t < tiles_per_block; ++t) {
        const int w = (b * tiles_per_block + t) * kPlaqWalkBlock + threadIdx.x;
        if (w < nthreads) s += plaq_column<R, DLT>(links, g, layer, nch, w, tol, bad);
    }
    const double bs = block_sum<kPlaqWalkBlock>(s);
    __syncthreads();
    const double bb = block_sum<kPlaqWalkBlock>((double)bad);
    if (threadIdx.x == 0) {
        partials[blockIdx.y * gridDim.x + blockIdx.x] = bs;
        partials[(gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = bb;
    }
}

// Double-layered torus: per-layer plaquette sums of a measured sweep from the
// nmeas pairs (layer 0, layer 1) of the three measured passes, fixed order:
// sums[1 + l] = the sum of layer l, sums[0] = sums[1] + sums[2].
__global__ __launch_bounds__(kBlock) void k_measure_final_dlt(const double *__restrict__ meas, int nmeas,
                                                              double *__restrict__ sums)
{
    double t0 = 0.0, t1 = 0.0;
    for (int k = threadIdx.x; k < nmeas; k += kBlock) {
        t0 += meas[2 * k];
        t1 += meas[2 * k + 1];
    }
    const double T0 = block_sum(t0);
    __syncthreads();
    const double T1 = block_sum(t1);
    if (threadIdx.x == 0) {
        sums[0] = T0 + T1;
        sums[1] = T0;
        sums[2] = T1;
    }
}

// sums[1 + l] = sum over the partials of layer l; sums[0] = sum over layers;
// sums[3] = number of links that failed the unitarity check.  With `mean`
// non-null also the normalised values: mean[0] = sums[0] / (norm nlat),
// mean[1 + l] = sums[1 + l] / norm, mean[1 + nlat] = sums[3] (norm = 18 V).
__global__ __launch_bounds__(kBlock) void k_plaq_final(const double *__restrict__ partials, int nblk, int nlat,
                                                       double *__restrict__ sums, double *__restrict__ mean,
                                                       double norm)
{
    double tot = 0.0;
    for (int l = 0; l < nlat; ++l) {
        double s = 0.0;
        for (int b = threadIdx.x; b < nblk; b += kBlock) s += partials[l * nblk + b];
        const double r = block_sum(s);
        __syncthreads();
        if (threadIdx.x == 0) {
            sums[1 + l] = r;
            tot += r;
        }
    }
    double nb = 0.0;
    for (int b = threadIdx.x; b < nlat * nblk; b += kBlock) nb += partials[nlat * nblk + b];
    const double r = block_sum(nb);
    if (threadIdx.x == 0) {
        sums[0] = tot;
        if (nlat == 1) sums[2] = 0.0;
        sums[3] = r;
        if (mean) {
            mean[0] = tot / (norm * nlat);
            for (int l = 0; l < nlat; ++l) mean[1 + l] = sums[1 + l] / norm;
            mean[1 + nlat] = r;
        }
    }
}

// single torus: sums[0] = sums[1] = sum of the partials a[0..na), fixed order
constexpr int kSumBlock = 1024;
__global__ __launch_bounds__(kSumBlock) void k_sum_partials(const double *__restrict__ a, int na,
                                                            double *__restrict__ sums)
{
    // thread t adds a[t], a[t + kSumBlock], ... in that order; the loads of
    // eight terms are issued together
    double s = 0.0;
    int k = threadIdx.x;
    for (; k + 7 * kSumBlock < na; k += 8 * kSumBlock) {
        double v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = a[k + j * kSumBlock];
#pragma unroll
        for (int j = 0; j < 8; ++j) s += v[j];
    }
    for (; k < na; k += kSumBlock) s += a[k];
    const double r = block_sum<kSumBlock>(s);
    if (threadIdx.x == 0) {
        sums[0] = r;
        sums[1] = r;
    }
}

__global__ void k_zero_u64(unsigned long long *p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

// bandwidth probe: 16-byte loads and stores, grid-stride over a grid of
// four workgroups per CU (the shape that copied fastest on this chip)
__global__ __launch_bounds__(kBlock) void k_copy(const uint4 *__restrict__ src, uint4 *__restrict__ dst, size_t n)
{
    const size_t step = (size_t)gridDim.x * kBlock;
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += step) dst[i] = src[i];
}

inline unsigned blocks_for(long long n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace


hipError_t launch_start(int precision, void *links, const Geom &g, int hot, uint64_t seed, hipStream_t s)
{
    const dim3 grid(blocks_for((long long)g.nlat * g.Vh), 8);
    if (precision == 64)
        k_start<double><<<grid, kBlock, 0, s>>>((double2 *)links, g, hot, seed);
    else
        k_start<float><<<grid, kBlock, 0, s>>>((float2 *)links, g, hot, seed);
    return hipGetLastError();
}

template <int MU, typename R, bool MEAS>
static void update_launch(store_t<R> *links, const Geom &g, int par, double beta, uint64_t sweep, uint64_t seed,
                          int nhit, int lanes, unsigned long long *counters, double *meas, hipStream_t s)
{
    const bool dlt = g.nlat == 2;
    const unsigned grid = (unsigned)pass_blocks(g, pass_links_per_block(g, lanes));
    // several lanes per link for small passes (1-hit only; the host decides)
    if (lanes == 4) {
        if (dlt)
            k_update_lanes<MU, R, true, MEAS, 4><<<grid, kBlock, 0, s>>>(links, g, par, beta, sweep, seed, counters, meas);
        else
            k_update_lanes<MU, R, false, MEAS, 4><<<grid, kBlock, 0, s>>>(links, g, par, beta, sweep, seed, counters, meas);
        return;
    }
    if (lanes == 2) {
        if (dlt)
            k_update_lanes<MU, R, true, MEAS, 2><<<grid, kBlock, 0, s>>>(links, g, par, beta, sweep, seed, counters, meas);
        else
            k_update_lanes<MU, R, false, MEAS, 2><<<grid, kBlock, 0, s>>>(links, g, par, beta, sweep, seed, counters, meas);
        return;
    }
    // one lane per link: one-wave workgroups on a single torus (a workgroup's
    // LDS stash and slot are released as soon as its one wave ends: 32^4
    // +1.4 %, 64^4 +2 %, 16^4 +7 % over four-wave workgroups); the
    // double-layered torus keeps four-wave workgroups (-1 % with one wave)
    if (nhit == 1 && !dlt)
        k_update<MU, R, true, false, MEAS, kPassBlock>
            <<<grid, kPassBlock, 0, s>>>(links, g, par, beta, sweep, seed, nhit, counters, meas);
    else if (nhit == 1)
        k_update<MU, R, true, true, MEAS><<<grid, kBlock, 0, s>>>(links, g, par, beta, sweep, seed, nhit, counters, meas);
    else if (!dlt)
        k_update<MU, R, false, false, MEAS, kPassBlock>
            <<<grid, kPassBlock, 0, s>>>(links, g, par, beta, sweep, seed, nhit, counters, meas);
    else
        k_update<MU, R, false, true, MEAS><<<grid, kBlock, 0, s>>>(links, g, par, beta, sweep, seed, nhit, counters,
                                                                    meas);
}

template <typename R>
static void update_dispatch(store_t<R> *links, const Geom &g, int mu, int par, double beta, uint64_t sweep,
                            uint64_t seed, int nhit, int lanes, unsigned long long *counters, double *meas,
                            hipStream_t s)
{
    if (meas) {  // measured: odd passes of mu = 1, 2, 3
        switch (mu) {
        case 1: update_launch<1, R, true>(links, g, 1, beta, sweep, seed, nhit, lanes, counters, meas, s); break;
        case 2: update_launch<2, R, true>(links, g, 1, beta, sweep, seed, nhit, lanes, counters, meas, s); break;
        default: update_launch<3, R, true>(links, g, 1, beta, sweep, seed, nhit, lanes, counters, meas, s); break;
        }
        return;
    }
    switch (mu) {
    case 0: update_launch<0, R, false>(links, g, par, beta, sweep, seed, nhit, lanes, counters, nullptr, s); break;
    case 1: update_launch<1, R, false>(links, g, par, beta, sweep, seed, nhit, lanes, counters, nullptr, s); break;
    case 2: update_launch<2, R, false>(links, g, par, beta, sweep, seed, nhit, lanes, counters, nullptr, s); break;
    default: update_launch<3, R, false>(links, g, par, beta, sweep, seed, nhit, lanes, counters, nullptr, s); break;
    }
}

hipError_t launch_update(int precision, void *links, const Geom &g, int mu, int par, double beta, uint64_t sweep,
                         uint64_t seed, int nhit, int lanes, unsigned long long *counters, hipStream_t s)
{
    if (lanes != 1 && (nhit != 1 || (lanes != 2 && lanes != 4))) return hipErrorInvalidValue;
    if (precision == 64)
        update_dispatch<double>((double2 *)links, g, mu, par, beta, sweep, seed, nhit, lanes, counters, nullptr, s);
    else
        update_dispatch<float>((float2 *)links, g, mu, par, beta, sweep, seed, nhit, lanes, counters, nullptr, s);
    return hipGetLastError();
}

template <typename R, bool HIT1, bool DLT>
static void batch_dispatch(const BatchJob *jobs, int njobs, int ntiles, long long step, int mu, int par, hipStream_t s)
{
    switch (mu) {
    case 0: k_update_batch<0, R, HIT1, DLT><<<ntiles, kPassBlock, 0, s>>>(jobs, njobs, step, par); break;
    case 1: k_update_batch<1, R, HIT1, DLT><<<ntiles, kPassBlock, 0, s>>>(jobs, njobs, step, par); break;
    case 2: k_update_batch<2, R, HIT1, DLT><<<ntiles, kPassBlock, 0, s>>>(jobs, njobs, step, par); break;
    default: k_update_batch<3, R, HIT1, DLT><<<ntiles, kPassBlock, 0, s>>>(jobs, njobs, step, par); break;
    }
}

template <typename R>
static void batch_dispatch_r(bool hit1, bool dlt, const BatchJob *jobs, int njobs, int ntiles, long long step, int mu,
                             int par, hipStream_t s)
{
    if (hit1 && !dlt)
        batch_dispatch<R, true, false>(jobs, njobs, ntiles, step, mu, par, s);
    else if (hit1)
        batch_dispatch<R, true, true>(jobs, njobs, ntiles, step, mu, par, s);
    else if (!dlt)
        batch_dispatch<R, false, false>(jobs, njobs, ntiles, step, mu, par, s);
    else
        batch_dispatch<R, false, true>(jobs, njobs, ntiles, step, mu, par, s);
}

hipError_t launch_update_batch(int precision, bool hit1, bool dlt, const BatchJob *d_jobs, int njobs, int ntiles,
                               long long step, int mu, int par, hipStream_t s)
{
    if (njobs <= 0 || ntiles <= 0) return hipSuccess;
    if (precision == 64)
        batch_dispatch_r<double>(hit1, dlt, d_jobs, njobs, ntiles, step, mu, par, s);
    else
        batch_dispatch_r<float>(hit1, dlt, d_jobs, njobs, ntiles, step, mu, par, s);
    return hipGetLastError();
}

hipError_t launch_update_measured(int precision, void *links, const Geom &g, int mu, double beta, uint64_t sweep,
                                  uint64_t seed, int nhit, int lanes, unsigned long long *counters, double *meas,
                                  hipStream_t s)
{
    if (mu < 1 || mu > 3 || !meas) return hipErrorInvalidValue;
    if (lanes != 1 && (nhit != 1 || (lanes != 2 && lanes != 4))) return hipErrorInvalidValue;
    if (precision == 64)
        update_dispatch<double>((double2 *)links, g, mu, 1, beta, sweep, seed, nhit, lanes, counters, meas, s);
    else
        update_dispatch<float>((float2 *)links, g, mu, 1, beta, sweep, seed, nhit, lanes, counters, meas, s);
    return hipGetLastError();
}

hipError_t launch_measure_final(const double *meas, const Geom &g, int lanes, double *sums, hipStream_t s)
{
    const int nmeas = 3 * meas_blocks(g, lanes);
    if (g.nlat == 1)
        k_sum_partials<<<1, kSumBlock, 0, s>>>(meas, nmeas, sums);
    else
        k_measure_final_dlt<<<1, kBlock, 0, s>>>(meas, nmeas, sums);
    return hipGetLastError();
}

hipError_t launch_plaquette(int precision, const void *links, const Geom &g, double *partials, double *sums,
                            hipStream_t s, double *mean)
{
    const bool dlt = g.nlat == 2;
    const double tol = unitarity_tol(precision);
    const int nch = plaq_walk_chunks(g, precision);
    if (nch > 0) {
        // FP64 lattices with enough columns: the x3 walk
        const int nblk = plaq_walk_blocks(g, nch);
        const dim3 grid(nblk, g.nlat);
        const long long tiles = ((long long)g.L[0] * g.L[1] * g.L[2] * nch + kPlaqWalkBlock - 1) / kPlaqWalkBlock;
        const int tpb = (int)((tiles + nblk - 1) / nblk);
        if (dlt)
            k_plaq_walk<double, true><<<grid, kPlaqWalkBlock, 0, s>>>((const double2 *)links, g, nch, tpb, tol,
                                                                      partials);
        else
            k_plaq_walk<double, false><<<grid, kPlaqWalkBlock, 0, s>>>((const double2 *)links, g, nch, tpb, tol,
                                                                       partials);
        k_plaq_final<<<1, kBlock, 0, s>>>(partials, nblk, g.nlat, sums, mean, 36.0 * (double)g.Vh);
        return hipGetLastError();
    }
    const int nblk = plaq_blocks(g);
    const dim3 grid(nblk, g.nlat);
    if (precision == 64) {
        // one site per thread: tiles of kBlock sites
        const long long tiles = (2LL * g.Vh + kBlock - 1) / kBlock;
        const int tpb = (int)((tiles + nblk - 1) / nblk);
        if (dlt)
            k_plaq_sites<double, true><<<grid, kBlock, 0, s>>>((const double2 *)links, g, tpb, tol, partials);
        else
            k_plaq_sites<double, false><<<grid, kBlock, 0, s>>>((const double2 *)links, g, tpb, tol, partials);
    } else {
        // two sites (one half-index) per thread
        const long long tiles = ((long long)g.Vh + kBlock - 1) / kBlock;
        const int tpb = (int)((tiles + nblk - 1) / nblk);
        if (dlt)
            k_plaq_partial<float, true><<<grid, kBlock, 0, s>>>((const float2 *)links, g, tpb, tol, partials);
        else
            k_plaq_partial<float, false><<<grid, kBlock, 0, s>>>((const float2 *)links, g, tpb, tol, partials);
    }
    k_plaq_final<<<1, kBlock, 0, s>>>(partials, nblk, g.nlat, sums, mean, 36.0 * (double)g.Vh);
    return hipGetLastError();
}

template <int MU, typename R>
static void twob_launch(store_t<R> *links, const Geom &g, int par, double b0, double b1, uint64_t sweep, uint64_t seed,
                        int nhit, unsigned long long *counters, hipStream_t s)
{
    const dim3 grid(blocks_for((long long)g.nlat * g.Vh));
    if (nhit == 1)
        k_update_twob<MU, R, true><<<grid, kBlock, 0, s>>>(links, g, par, b0, b1, sweep, seed, nhit, counters);
    else
        k_update_twob<MU, R, false><<<grid, kBlock, 0, s>>>(links, g, par, b0, b1, sweep, seed, nhit, counters);
}

template <typename R>
static void twob_dispatch(store_t<R> *links, const Geom &g, int mu, int par, double b0, double b1, uint64_t sweep,
                          uint64_t seed, int nhit, unsigned long long *counters, hipStream_t s)
{
    switch (mu) {
    case 0: twob_launch<0, R>(links, g, par, b0, b1, sweep, seed, nhit, counters, s); break;
    case 1: twob_launch<1, R>(links, g, par, b0, b1, sweep, seed, nhit, counters, s); break;
    case 2: twob_launch<2, R>(links, g, par, b0, b1, sweep, seed, nhit, counters, s); break;
    default: twob_launch<3, R>(links, g, par, b0, b1, sweep, seed, nhit, counters, s); break;
    }
}

hipError_t launch_update_twob(int precision, void *links, const Geom &g, int mu, int par, double beta0,
                              double beta1, uint64_t sweep, uint64_t seed, int nhit, unsigned long long *counters,
                              hipStream_t s)
{
    if (precision == 64)
        twob_dispatch<double>((double2 *)links, g, mu, par, beta0, beta1, sweep, seed, nhit, counters, s);
    else
        twob_dispatch<float>((float2 *)links, g, mu, par, beta0, beta1, sweep, seed, nhit, counters, s);
    return hipGetLastError();
}

hipError_t launch_polyakov(int precision, const void *links, const Geom &g, double *partials, double *out,
                           hipStream_t s)
{
    const int nblk = polyakov_blocks(g);
    const dim3 grid(nblk, g.nlat);
    if (precision == 64)
        k_polyakov<double><<<grid, kBlock, 0, s>>>((const double2 *)links, g, partials);
    else
        k_polyakov<float><<<grid, kBlock, 0, s>>>((const float2 *)links, g, partials);
    k_polyakov_final<<<1, kBlock, 0, s>>>(partials, nblk, g.nlat, out);
    return hipGetLastError();
}

hipError_t launch_reunit(int precision, void *links, const Geom &g, hipStream_t s)
{
    const dim3 grid(blocks_for((long long)g.nlat * g.Vh), 8);
    if (precision == 64)
        k_reunit<double><<<grid, kBlock, 0, s>>>((double2 *)links, g);
    else
        k_reunit<float><<<grid, kBlock, 0, s>>>((float2 *)links, g);
    return hipGetLastError();
}

hipError_t launch_gauge(int precision, void *links, const Geom &g, uint64_t gseed, hipStream_t s)
{
    const dim3 grid(blocks_for((long long)g.nlat * g.Vh), 8);
    if (precision == 64)
        k_gauge<double><<<grid, kBlock, 0, s>>>((double2 *)links, g, gseed);
    else
        k_gauge<float><<<grid, kBlock, 0, s>>>((float2 *)links, g, gseed);
    return hipGetLastError();
}

hipError_t launch_zero_u64(unsigned long long *p, int n, hipStream_t s)
{
    k_zero_u64<<<(n + kBlock - 1) / kBlock, kBlock, 0, s>>>(p, n);
    return hipGetLastError();
}

hipError_t launch_copy(void *dst, const void *src, size_t bytes, hipStream_t s)
{
    const size_t n = bytes / 16;
    long long want = (long long)((n + kBlock - 1) / kBlock);
    const unsigned grid = (unsigned)(want < 1024 ? (want > 0 ? want : 1) : 1024);
    k_copy<<<grid, kBlock, 0, s>>>((const uint4 *)src, (uint4 *)dst, n);
    return hipGetLastError();
}

}  // namespace su3hb
