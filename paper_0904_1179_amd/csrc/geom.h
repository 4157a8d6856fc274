// geom.h -- lattice geometry, link-storage layout and launch-shape constants
// shared by the host runtime and the gfx950 kernels.  Plain C++ with no HIP
// header, so that the host-side layout code (layout.cpp) also builds with an
// ordinary C++ compiler (the sanitizer build of the test suite).
#pragma once

#include <stddef.h>
#include <stdint.h>

namespace su3hb {

// Link storage: the links of one (direction, parity) form a block of tiles of
// kTile consecutive links; a tile holds the kEntries complex entries of rows 0
// and 1 entry-major (row 2 of an SU(3) matrix is conj(row 0 x row 1)).
constexpr int kTile = 16;
constexpr int kEntries = 6;

constexpr int kBlock = 256;          // threads per workgroup (4 waves of 64)
constexpr int kPassBlock = 64;       // threads per workgroup of the one-wave pass kernels
constexpr int kPlaqBlocksMax = 4096; // workgroups per layer of the plaquette reduction
constexpr int kPlaqWalkBlock = 256;  // threads per workgroup of the plaquette walk
constexpr int kCounterSlots = 4096;  // heat-bath counter slots (pairs of u64: attempts, accepts)
constexpr int kNumXcd = 8;           // MI355X: 8 XCDs, workgroup b runs on XCD b % 8
constexpr int kMeasureChunk = 256;   // sweeps per read-back of su3_sweep_measure

// Scratch layout (bytes): [0, 16 kCounterSlots) heat-bath counter slots; 256
// bytes of sums (plaquette: [0] total, [1], [2] per layer, [3] links failing
// the unitarity check; Polyakov loops at [8..12)); the per-sweep plaquette
// sums of su3_sweep_measure (kMeasureChunk sweeps x 4 doubles); then the
// plaquette partials and the regions whose sizes depend on the lattice
// (layout.cpp: meas_offset, polyakov_offset, scratch_bytes_of).
constexpr size_t kOffCounters = 0;
constexpr size_t kOffSums = 16 * (size_t)kCounterSlots;
constexpr size_t kOffMeasure = kOffSums + 256;
constexpr size_t kOffPartials = kOffMeasure + 32 * (size_t)kMeasureChunk;

// Unsigned division by a divisor fixed for a launch (Granlund and Montgomery,
// "Division by invariant integers using multiplication", 1994): with
// l = ceil(log2 d), m = floor(2^32 (2^l - d) / d) + 1, s1 = min(l, 1),
// s2 = max(l - 1, 0) and t = floor(m x / 2^32),
//   floor(x / d) = (t + ((x - t) >> s1)) >> s2   for every 0 <= x < 2^32,
// a multiply-high and three shifts/adds instead of a division sequence.
struct FastDiv {
    uint32_t d, m, s1, s2;
};

inline FastDiv make_fastdiv(uint32_t d)
{
    uint32_t l = 0;
    while ((1ull << l) < d) ++l;
    FastDiv f;
    f.d = d;
    f.m = (uint32_t)((((uint64_t)1 << 32) * ((1ull << l) - d)) / d + 1);
    f.s1 = l < 1 ? l : 1;
    f.s2 = l > 1 ? l - 1 : 0;
    return f;
}

// constexpr: usable in host and device code alike
constexpr int div_by(int x, const FastDiv &f)
{
    const uint32_t ux = (uint32_t)x;
    const uint32_t t = (uint32_t)(((uint64_t)f.m * ux) >> 32);
    return (int)((t + ((ux - t) >> f.s1)) >> f.s2);
}

// Sites are addressed by (layer, parity, i): i = lex >> 1 with
// lex = x0 + L0 (x1 + L1 (x2 + L2 x3)); with L0 even, the two sites sharing
// lex >> 1 have opposite parity.  Within a (direction, parity) block the link
// of site (layer, parity, i) is element n = layer * Vh + i.
struct Geom {
    int L[4];
    int Vh;             // V / 2
    int nlat;
    unsigned flip;      // layer-switch mask, 0 on a single torus
    long long stride;   // links per (direction, parity) block (>= nlat * Vh, multiple of 64)
    int w1, w2;         // domain widths of the pass order (divide L1, L2)
    int nd1;            // L1 / w1
    FastDiv dl0h, dl1, dl2, dl3, dw1, dw2, dnd1;  // division by L0/2, L1, L2, L3, w1, w2, nd1
};

// Column order of the plaquette walk.  Thread w (0 <= w < nch L0 L1 L2) of a
// layer takes the column (x0, x1, x2) and the chunk c of x3 with
//   w = (d nch + c) S + x0 + L0 (x1' + w1 x2'),  S = L0 w1 w2,
// d the domain of (x1, x2) numbered as in the pass order (x1 = (d mod nd1) w1
// + x1', x2 = (d / nd1) w2 + x2').  So an XCD's contiguous range of threads
// covers whole domains with all their chunks, and the lanes of a wave cover
// consecutive x0.  Chunk c covers x3 in [c L3 / nch, (c + 1) L3 / nch).
// Returns c and fills x[0..2].
constexpr int walk_column(const Geom &g, int nch, int w, int x[3])
{
    const int a = div_by(w >> 1, g.dl0h);  // floor(w / L0) = floor(floor(w / 2) / (L0 / 2))
    x[0] = w - a * g.L[0];
    const int b = div_by(a, g.dw1);
    const int x1p = a - b * g.w1;
    const int q = div_by(b, g.dw2);
    const int x2p = b - q * g.w2;
    const int d = q / nch;
    const int c = q - d * nch;
    const int d2 = div_by(d, g.dnd1);
    x[1] = (d - d2 * g.nd1) * g.w1 + x1p;
    x[2] = d2 * g.w2 + x2p;
    return c;
}

}  // namespace su3hb
