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
// staple: A += U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+ + U_nu(x+mu-nu)^+ U_mu(x-nu)^+ U_nu(x-nu)
// written as a (c b)^+ + (e d)^+ f with
//   a = U_nu(x+mu), b = U_mu(x+nu), c = U_nu(x), d = U_nu(x+mu-nu), e = U_mu(x-nu), f = U_nu(x-nu)
// b and e come from the caller (see update_link); the pairs (c, d) and (a, f)
// are loaded together: c of thread x is d of thread x + nu - mu, a of thread
// x is f of thread x + mu + nu.
// ---------------------------------------------------------------------------
// TWOB (double-layered torus with per-layer couplings wb[0], wb[1]): the upper
// term belongs to the plaquette based at x, the lower one to the plaquette
// based at x - nu; each is weighted by the coupling of that base site's layer.
template <int MU, int NU, typename R, bool DLT, bool TWOB = false>
__device__ __forceinline__ void add_staple(M3<R> &A, const M3<R> &b, const M3<R> &e,
                                           const store_t<R> *__restrict__ links, const Geom &g, const int x[4],
                                           int layer, int par, int n, const R *wb = nullptr)
{
    const int opp = par ^ 1;
    M3<R> c, d, a, f;
    load_link12_pair<R>(c, planes<R>(links, g, NU, par), n, d, planes<R>(links, g, NU, par),
                        nbr_elem<MU, +1, NU, -1, DLT>(g, x, layer));
    // c b, e d and a (c b)^+ are SU(3) products: rows 0 and 1 formed, row 2
    // rebuilt (so the third rows of c, e and a are never needed)
    const M3<R> cb = mul_nn_su3(c, b);
    const M3<R> ed = mul_nn_su3(e, d);
    const int elo = nbr_elem<NU, -1, MU, 0, DLT>(g, x, layer);
    load_link12_pair<R>(a, planes<R>(links, g, NU, opp), nbr_elem<MU, +1, NU, 0, DLT>(g, x, layer), f,
                        planes<R>(links, g, NU, opp), elo);
    const M3<R> up = mul_nd_su3(a, cb);
    if constexpr (TWOB) {
        scale_acc(A, up, wb[layer]);
        M3<R> t;
        set_zero(t);
        acc_dn(t, ed, f);
        scale_acc(A, t, wb[elo >= g.Vh ? 1 : 0]);
    } else {
        add_to(A, up);
        acc_dn(A, ed, f);
    }
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
// Returns Re Tr W after the last subgroup, i.e. Re Tr(U_new A) before the
// final reunitarisation: the sum of the six plaquettes through the new link.
template <typename R, bool HIT1>
__device__ __forceinline__ double heatbath(M3<R> &U, const M3<R> &A, double beta_d, uint64_t seed, uint64_t lid,
                                           uint64_t sweep, int nhit, int &att, int &acc)
{
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
            const U64x4 w = philox4x64_10(lid, sweep, ((uint64_t)sub << 32) | (uint64_t)t, kTagHeatbath, seed, 0);
            ++att;
            const R u1 = R(unif52(w.w[0]));
            const R u3 = R(unif52(w.w[1]));
            const R u2 = R(unif32((uint32_t)w.w[2]));
            const R u4 = R(unif32((uint32_t)(w.w[2] >> 32)));
            const R c2 = cospi_sq_r(R(2) * u2);
            const R lam2 = -(log_r(u1) + c2 * log_r(u3)) * inv2alpha;
            if (u4 * u4 <= R(1) - lam2) {
                const R u5 = R(unif32((uint32_t)w.w[3]));
                const R u6 = R(unif32((uint32_t)(w.w[3] >> 32)));
                a0 = R(1) - R(2) * lam2;
                const R cth = R(2) * u5 - R(1);
                // FP64: |cth| < 1 (u5 is never 0 or 1), so the argument is positive
                const R sth = sqrt_pos_r(R(1) - cth * cth);
                R sph, cph;
                sincospi_r(R(2) * u6, &sph, &cph);
                const R rho2 = R(1) - a0 * a0;
                const R rho = rho2 > R(0) ? sqrt_pos_r(rho2) : R(0);
                a1 = rho * sth * cph;
                a2 = rho * sth * sph;
                a3 = rho * cth;
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
// MEAS: also return Re Tr(U_new S) with S the staple terms of the directions
// nu < MU.  Summed over the sites of one parity these are all plaquettes of
// the planes (nu, MU), nu < MU, each once (the upper term of site x is the
// plaquette based at x, the lower one that based at x - nu).  After the odd
// pass of MU no later pass of the sweep changes U_nu or U_MU for nu < MU, so
// the odd passes of MU = 1, 2, 3 together give the final plaquettes of all
// six planes.  Without MEAS the return value is Re Tr(U_new A) (unused).
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
template <typename R, bool DLT, int MU> constexpr bool kStashPass = sizeof(R) == 8 && (!DLT || MU > 0);
template <typename R, bool DLT> constexpr bool kStashBatch = sizeof(R) == 8 && !DLT;
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
__device__ __forceinline__ double update_link(store_t<R> *__restrict__ links, const Geom &g, int par, int v,
                                              double beta, uint64_t sweep, uint64_t seed, int nhit, int &att, int &acc,
                                              store_t<R> *stash, const R *wb = nullptr)
{
    static_assert(!MEAS || (MU > 0 && !TWOB), "measured passes: MU = 1, 2, 3 with one coupling");
    // the staple directions nu != MU in increasing order
    constexpr int N0 = MU == 0 ? 1 : 0;
    constexpr int N1 = MU <= 1 ? 2 : 1;
    constexpr int N2 = MU <= 2 ? 3 : 2;
    const int layer = DLT && v >= g.Vh ? 1 : 0;
    int x[4];
    const int i = order_site(g, par, v - layer * g.Vh, x);
    const int n = layer * g.Vh + i;
    M3<R> A, S;
    set_zero(A);
    __builtin_amdgcn_s_setprio(1);  // gathering the staple: issue loads ahead of waves in the heat bath
    if constexpr (!STASH) {
        // b and e of each direction loaded in its phase
        const store_t<R> *umu = planes<R>(links, g, MU, par ^ 1);
        M3<R> b, e;
        load_link12_pair<R>(b, umu, nbr_elem<N0, +1, MU, 0, DLT>(g, x, layer), e, umu,
                            nbr_elem<N0, -1, MU, 0, DLT>(g, x, layer));
        add_staple<MU, N0, R, DLT, TWOB>(A, b, e, links, g, x, layer, par, n, wb);
        if constexpr (MEAS && MU == 1) S = A;
        load_link12_pair<R>(b, umu, nbr_elem<N1, +1, MU, 0, DLT>(g, x, layer), e, umu,
                            nbr_elem<N1, -1, MU, 0, DLT>(g, x, layer));
        add_staple<MU, N1, R, DLT, TWOB>(A, b, e, links, g, x, layer, par, n, wb);
        if constexpr (MEAS && MU == 2) S = A;
        load_link12_pair<R>(b, umu, nbr_elem<N2, +1, MU, 0, DLT>(g, x, layer), e, umu,
                            nbr_elem<N2, -1, MU, 0, DLT>(g, x, layer));
        add_staple<MU, N2, R, DLT, TWOB>(A, b, e, links, g, x, layer, par, n, wb);
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
        stash_put<R, NB>(stash, 0, b1);
        stash_put<R, NB>(stash, 1, e1);
        stash_put<R, NB>(stash, 2, b2);
        stash_fence();
        add_staple<MU, N0, R, DLT, TWOB>(A, from_raw(b0), from_raw(e0), links, g, x, layer, par, n, wb);
        if constexpr (MEAS && MU == 1) S = A;
        add_staple<MU, N1, R, DLT, TWOB>(A, stash_get<R, NB>(stash, 0), stash_get<R, NB>(stash, 1), links, g, x, layer, par,
                                         n, wb);
        if constexpr (MEAS && MU == 2) S = A;
        add_staple<MU, N2, R, DLT, TWOB>(A, stash_get<R, NB>(stash, 2), from_raw(e2), links, g, x, layer, par, n, wb);
    }
    store_t<R> *own = planes<R>(links, g, MU, par);
    M3<R> U = load_link12_nt<R>(own, n);
    const uint64_t site = (uint64_t)layer * (uint64_t)(2 * g.Vh) + (uint64_t)lex_of(g, x);
    // with per-layer couplings the staple carries them: alpha = 2k/3
    __builtin_amdgcn_s_setprio(0);
    double trw = heatbath<R, HIT1>(U, A, TWOB ? 1.0 : beta, seed, 4 * site + MU, sweep, nhit, att, acc);
    // FP64: nontemporal, so the written link does not displace staple links
    // from L2 (a plain store: -3 % at 32^4).  FP32, bound by issue rather
    // than memory: a plain store (+1 %)
    if constexpr (sizeof(R) == 8)
        store_link_nt<R>(own, n, U);
    else
        store_link<R>(own, n, U);
    if constexpr (MEAS && MU < 3) trw = retr_mul(U, S);
    return trw;
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

// One checkerboard pass in workgroups of NB threads (kBlock, or kPassBlock
// for the unmeasured passes of a single torus).  MEAS (odd passes of MU = 1,
// 2, 3; NB = kBlock): also store, per workgroup, the sum over its links of
// the final plaquettes of the planes (nu, MU), nu < MU, that update_link
// returns; on a double-layered torus one sum per layer of the updated site.
template <int MU, typename R, bool HIT1, bool DLT, bool MEAS = false, int NB = kBlock>
__global__ __launch_bounds__(NB, kPassWaves<R>) void k_update(store_t<R> *__restrict__ links, const Geom g, const int par,
                                                   const double beta, const uint64_t sweep, const uint64_t seed,
                                                   const int nhit, unsigned long long *__restrict__ counters,
                                                   double *__restrict__ meas = nullptr)
{
    constexpr bool kStash = kStashPass<R, DLT, MU>;
    store_t<R> *st = nullptr;
    if constexpr (kStash) {
        __shared__ store_t<R> stash[kStashSlots * 6 * NB];
        st = stash;
    }
    const int v = pass_tile(par) * NB + threadIdx.x;
    int att = 0, acc = 0;
    double trw = 0.0;
    if (v < g.nlat * g.Vh)
        trw = update_link<MU, R, HIT1, DLT, false, MEAS, kStash, NB>(links, g, par, v, beta, sweep, seed, nhit, att, acc,
                                                                 st);
    count_block<NB>(att, acc, counters, blockIdx.x % kCounterSlots);
    if (MEAS) {
        __syncthreads();
        if constexpr (DLT) {
            // per layer of the updated site: meas[2 b + layer]
            const bool l1 = v >= g.Vh;
            const double b0 = block_sum<NB>(l1 ? 0.0 : trw);
            __syncthreads();
            const double b1 = block_sum<NB>(l1 ? trw : 0.0);
            if (threadIdx.x == 0) {
                meas[2 * blockIdx.x] = b0;
                meas[2 * blockIdx.x + 1] = b1;
            }
        } else {
            const double b = block_sum<NB>(trw);
            if (threadIdx.x == 0) meas[blockIdx.x] = b;
        }
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
    if (v < g.nlat * g.Vh)
        update_link<MU, R, HIT1, true, true>(links, g, par, v, 1.0, sweep, seed, nhit, att, acc, nullptr, b);
    count_block(att, acc, counters, blockIdx.x % kCounterSlots);
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
// holds t; job j is at sweep index sweep0 + (step - admit_step).
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
    const int v = local * kPassBlock + threadIdx.x;
    const uint64_t sweep = J.sweep0 + (uint64_t)(step - J.admit_step);
    int att = 0, acc = 0;
    if (v < J.g.nlat * J.g.Vh)
        update_link<MU, R, HIT1, DLT, false, false, kStash, kPassBlock>((store_t<R> *)J.links, J.g, par, v, J.beta,
                                                                        sweep, J.seed, J.nhit, att, acc, st);
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
// Re Tr U_mu(x) U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+ = Re Tr P Q^+ with
// P = U_mu(x) U_nu(x+mu), Q = U_nu(x) U_mu(x+nu), in FP64.
template <int MU, int NU, typename R, bool DLT>
__device__ __forceinline__ double plaq_plane(const store_t<R> *__restrict__ links, const Geom &g, const int x[4],
                                             int layer, int par, int n)
{
    const int opp = par ^ 1;
    const M3<double> umu = convert<double>(load_link12<R>(planes<R>(links, g, MU, par), n));
    const M3<double> unu_xmu =
        convert<double>(load_link12<R>(planes<R>(links, g, NU, opp), nbr_elem<MU, +1, NU, 0, DLT>(g, x, layer)));
    const M3<double> unu = convert<double>(load_link12<R>(planes<R>(links, g, NU, par), n));
    const M3<double> umu_xnu =
        convert<double>(load_link12<R>(planes<R>(links, g, MU, opp), nbr_elem<NU, +1, MU, 0, DLT>(g, x, layer)));
    const M3<double> P = mul_nn(umu, unu_xmu);
    const M3<double> Q = mul_nn(unu, umu_xnu);
    double s = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) s += P.e[a][b].re * Q.e[a][b].re + P.e[a][b].im * Q.e[a][b].im;
    return s;
}

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

// The six planes of the site, and the check of its four own links.
//  * FP64: every plane loads its four links; the compiler issues the loads of
//    both sites of a thread at once (one wave per SIMD).
//  * FP32: the four own links are loaded once and kept, and compiler-only
//    fences between the planes hold the neighbour loads back (two waves per
//    SIMD: 87 instead of 122 us at 32^4).  In FP64 the same scheme took the
//    same time with 31 % more bytes fetched.
template <typename R, bool DLT>
__device__ __forceinline__ double plaq_site(const store_t<R> *__restrict__ links, const Geom &g, int layer, int par,
                                           int i, double tol, int &bad)
{
    int x[4];
    site_coords(g, par, i, x);
    const int n = layer * g.Vh + i;
    if constexpr (sizeof(R) == 8) {
        double s = plaq_plane<0, 1, R, DLT>(links, g, x, layer, par, n);
        s += plaq_plane<0, 2, R, DLT>(links, g, x, layer, par, n);
        s += plaq_plane<1, 2, R, DLT>(links, g, x, layer, par, n);
        s += plaq_plane<0, 3, R, DLT>(links, g, x, layer, par, n);
        s += plaq_plane<1, 3, R, DLT>(links, g, x, layer, par, n);
        s += plaq_plane<2, 3, R, DLT>(links, g, x, layer, par, n);
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) bad += link_bad(load_rows01<R>(planes<R>(links, g, mu, par), n), tol);
        return s;
    } else {
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

// Double-layered torus, fused measurement: the measured odd pass of MU files
// the plaquette of the lower staple term of site x (based at y = x - nu) under
// the layer of x.  y lies in the other layer exactly when the step crosses a
// flipped boundary of direction nu, i.e. y_nu = L_nu - 1, y even.  This kernel
// sums those plaquettes, planes (nu, mu) with mu > nu, per layer of y, so that
// the per-layer sums can be moved to the right layer.  Grid (nblk,
// kFaceGroups): blockIdx.y is one plane (nu, mu), so that each thread forms
// one plaquette; thread q enumerates the face y_nu = L_nu - 1 (both parities;
// odd sites contribute nothing: a grid of half the size over the even sites
// alone took 13 instead of 9 us at 2 x 16^4); partials[2 (c nblk + b) + layer].
template <int NU, int MU, typename R>
__device__ __forceinline__ void face_plane(const store_t<R> *__restrict__ links, const Geom &g, long long q, double &s0,
                                           double &s1)
{
    int y[4];
    long long r = q;
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        if (d == NU) continue;
        y[d] = (int)(r % g.L[d]);
        r /= g.L[d];
    }
    const int layer = (int)r;
    y[NU] = g.L[NU] - 1;
    if ((y[0] + y[1] + y[2] + y[3]) & 1) return;
    const int n = layer * g.Vh + (lex_of(g, y) >> 1);
    const double t = plaq_plane<NU, MU, R, true>(links, g, y, layer, 0, n);
    if (layer)
        s1 += t;
    else
        s0 += t;
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_plaq_faces(const store_t<R> *__restrict__ links, const Geom g,
                                                       double *__restrict__ partials)
{
    // plane c = blockIdx.y: (0,1) (0,2) (0,3) (1,2) (1,3) (2,3)
    const int c = blockIdx.y;
    const int nu = c < 3 ? 0 : (c < 5 ? 1 : 2);
    double s0 = 0.0, s1 = 0.0;
    const long long nface = (long long)g.nlat * (2LL * g.Vh / g.L[nu]);
    const long long q = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (((g.flip >> nu) & 1) && q < nface) {
        switch (c) {
        case 0: face_plane<0, 1, R>(links, g, q, s0, s1); break;
        case 1: face_plane<0, 2, R>(links, g, q, s0, s1); break;
        case 2: face_plane<0, 3, R>(links, g, q, s0, s1); break;
        case 3: face_plane<1, 2, R>(links, g, q, s0, s1); break;
        case 4: face_plane<1, 3, R>(links, g, q, s0, s1); break;
        default: face_plane<2, 3, R>(links, g, q, s0, s1); break;
        }
    }
    const double b0 = block_sum(s0);
    __syncthreads();
    const double b1 = block_sum(s1);
    if (threadIdx.x == 0) {
        const size_t k = (size_t)c * gridDim.x + blockIdx.x;
        partials[2 * k] = b0;
        partials[2 * k + 1] = b1;
    }
}

// Double-layered torus: per-layer plaquette sums of a measured sweep.  meas:
// nmeas pairs (T_0, T_1) of the three measured passes; faces: nfaces pairs
// (C_0, C_1).  sums[1 + l] = T_l + C_l - C_{1-l}, sums[0] = sums[1] + sums[2].
__global__ __launch_bounds__(kBlock) void k_measure_final_dlt(const double *__restrict__ meas, int nmeas,
                                                              const double *__restrict__ faces, int nfaces,
                                                              double *__restrict__ sums)
{
    double t0 = 0.0, t1 = 0.0, c0 = 0.0, c1 = 0.0;
    for (int k = threadIdx.x; k < nmeas; k += kBlock) {
        t0 += meas[2 * k];
        t1 += meas[2 * k + 1];
    }
    for (int k = threadIdx.x; k < nfaces; k += kBlock) {
        c0 += faces[2 * k];
        c1 += faces[2 * k + 1];
    }
    const double T0 = block_sum(t0);
    __syncthreads();
    const double T1 = block_sum(t1);
    __syncthreads();
    const double C0 = block_sum(c0);
    __syncthreads();
    const double C1 = block_sum(c1);
    if (threadIdx.x == 0) {
        const double p0 = T0 + C0 - C1, p1 = T1 + C1 - C0;
        sums[0] = p0 + p1;
        sums[1] = p0;
        sums[2] = p1;
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

template <int MU, typename R>
static void update_launch(store_t<R> *links, const Geom &g, int par, double beta, uint64_t sweep, uint64_t seed,
                          int nhit, unsigned long long *counters, hipStream_t s)
{
    const bool dlt = g.nlat == 2;
    // one-wave workgroups on a single torus: a workgroup's LDS stash and slot
    // are released as soon as its one wave ends (32^4: +1.4 %, 64^4: +2 %,
    // 16^4: +7 % over four-wave workgroups); the double-layered torus keeps
    // four-wave workgroups (-1 % with one wave)
    if (nhit == 1 && !dlt)
        k_update<MU, R, true, false, false, kPassBlock>
            <<<pass_blocks(g, kPassBlock), kPassBlock, 0, s>>>(links, g, par, beta, sweep, seed, nhit, counters);
    else if (nhit == 1)
        k_update<MU, R, true, true><<<pass_blocks(g, kBlock), kBlock, 0, s>>>(links, g, par, beta, sweep, seed, nhit,
                                                                              counters);
    else if (!dlt)
        k_update<MU, R, false, false, false, kPassBlock>
            <<<pass_blocks(g, kPassBlock), kPassBlock, 0, s>>>(links, g, par, beta, sweep, seed, nhit, counters);
    else
        k_update<MU, R, false, true><<<pass_blocks(g, kBlock), kBlock, 0, s>>>(links, g, par, beta, sweep, seed, nhit,
                                                                               counters);
}

template <typename R>
static void update_dispatch(store_t<R> *links, const Geom &g, int mu, int par, double beta, uint64_t sweep,
                            uint64_t seed, int nhit, unsigned long long *counters, hipStream_t s)
{
    switch (mu) {
    case 0: update_launch<0, R>(links, g, par, beta, sweep, seed, nhit, counters, s); break;
    case 1: update_launch<1, R>(links, g, par, beta, sweep, seed, nhit, counters, s); break;
    case 2: update_launch<2, R>(links, g, par, beta, sweep, seed, nhit, counters, s); break;
    default: update_launch<3, R>(links, g, par, beta, sweep, seed, nhit, counters, s); break;
    }
}

hipError_t launch_update(int precision, void *links, const Geom &g, int mu, int par, double beta, uint64_t sweep,
                         uint64_t seed, int nhit, unsigned long long *counters, hipStream_t s)
{
    if (precision == 64)
        update_dispatch<double>((double2 *)links, g, mu, par, beta, sweep, seed, nhit, counters, s);
    else
        update_dispatch<float>((float2 *)links, g, mu, par, beta, sweep, seed, nhit, counters, s);
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

template <int MU, typename R>
static void update_meas_launch(store_t<R> *links, const Geom &g, double beta, uint64_t sweep, uint64_t seed, int nhit,
                               unsigned long long *counters, double *meas, hipStream_t s)
{
    // workgroups of meas_block_size(g) threads, as the unmeasured passes
    const dim3 grid(meas_blocks(g));
    const bool dlt = g.nlat == 2;
    if (nhit == 1 && !dlt)
        k_update<MU, R, true, false, true, kPassBlock><<<grid, kPassBlock, 0, s>>>(links, g, 1, beta, sweep, seed, nhit,
                                                                                  counters, meas);
    else if (nhit == 1)
        k_update<MU, R, true, true, true><<<grid, kBlock, 0, s>>>(links, g, 1, beta, sweep, seed, nhit, counters,
                                                                   meas);
    else if (!dlt)
        k_update<MU, R, false, false, true, kPassBlock><<<grid, kPassBlock, 0, s>>>(links, g, 1, beta, sweep, seed,
                                                                                   nhit, counters, meas);
    else
        k_update<MU, R, false, true, true><<<grid, kBlock, 0, s>>>(links, g, 1, beta, sweep, seed, nhit, counters,
                                                                    meas);
}

template <typename R>
static void update_meas_dispatch(store_t<R> *links, const Geom &g, int mu, double beta, uint64_t sweep,
                                 uint64_t seed, int nhit, unsigned long long *counters, double *meas, hipStream_t s)
{
    switch (mu) {
    case 1: update_meas_launch<1, R>(links, g, beta, sweep, seed, nhit, counters, meas, s); break;
    case 2: update_meas_launch<2, R>(links, g, beta, sweep, seed, nhit, counters, meas, s); break;
    default: update_meas_launch<3, R>(links, g, beta, sweep, seed, nhit, counters, meas, s); break;
    }
}

hipError_t launch_plaq_faces(int precision, const void *links, const Geom &g, double *partials, hipStream_t s)
{
    const dim3 grid(face_blocks(g), kFaceGroups);
    if (precision == 64)
        k_plaq_faces<double><<<grid, kBlock, 0, s>>>((const double2 *)links, g, partials);
    else
        k_plaq_faces<float><<<grid, kBlock, 0, s>>>((const float2 *)links, g, partials);
    return hipGetLastError();
}

hipError_t launch_update_measured(int precision, void *links, const Geom &g, int mu, double beta, uint64_t sweep,
                                  uint64_t seed, int nhit, unsigned long long *counters, double *meas, hipStream_t s)
{
    if (mu < 1 || mu > 3) return hipErrorInvalidValue;
    if (precision == 64)
        update_meas_dispatch<double>((double2 *)links, g, mu, beta, sweep, seed, nhit, counters, meas, s);
    else
        update_meas_dispatch<float>((float2 *)links, g, mu, beta, sweep, seed, nhit, counters, meas, s);
    return hipGetLastError();
}

hipError_t launch_measure_final(const double *meas, const double *faces, const Geom &g, double *sums, hipStream_t s)
{
    if (g.nlat == 1)
        k_sum_partials<<<1, kSumBlock, 0, s>>>(meas, 3 * meas_blocks(g), sums);
    else
        k_measure_final_dlt<<<1, kBlock, 0, s>>>(meas, 3 * meas_blocks(g), faces, kFaceGroups * face_blocks(g),
                                                  sums);
    return hipGetLastError();
}

hipError_t launch_plaquette(int precision, const void *links, const Geom &g, double *partials, double *sums,
                            hipStream_t s, double *mean)
{
    const int nblk = plaq_blocks(g);
    const long long tiles = ((long long)g.Vh + kBlock - 1) / kBlock;
    const int tpb = (int)((tiles + nblk - 1) / nblk);
    const dim3 grid(nblk, g.nlat);
    const bool dlt = g.nlat == 2;
    const double tol = unitarity_tol(precision);
    if (precision == 64) {
        if (dlt)
            k_plaq_partial<double, true><<<grid, kBlock, 0, s>>>((const double2 *)links, g, tpb, tol, partials);
        else
            k_plaq_partial<double, false><<<grid, kBlock, 0, s>>>((const double2 *)links, g, tpb, tol, partials);
    } else {
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
