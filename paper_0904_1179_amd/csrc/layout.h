// layout.h -- host-side geometry, buffer layout and launch shapes of the
// library: parameter validation, the pass order's domains, buffer sizes and
// scratch offsets, workgroup counts, and the conversion between the device's
// tiled link store and the canonical host layout.  Plain C++ (no HIP): the
// same code is built into the library and, for the sanitizer tests, with an
// ordinary C++ compiler.
#pragma once

#include <string>

#include "../../include/su3hb.h"
#include "geom.h"

namespace su3hb {

// record `msg` as the calling thread's last error and return `s`
su3_status fail(su3_status s, const std::string &msg);
const char *last_error();

su3_status check_params(const su3_params *p);
void pick_domains(const int32_t L[4], int nlat, int &w1, int &w2);
Geom make_geom(const su3_params *p);
size_t link_bytes_of(const su3_params *p, const Geom &g);

// Largest deviation from orthonormality of the stored rows 0 and 1 of a link
// that su3_plaquette accepts: FP64 links carry rounding of ~1e-15, FP32 links
// ~1e-7 from the rounding of FP64-reunitarised rows.
inline double unitarity_tol(int precision) { return precision == 64 ? 1e-10 : 1e-5; }

// Lanes per link of a pass: 1, or 2 or 4 for passes too small to fill the
// GPU with one lane per link (1-hit only).  `requested` = 0 picks by the
// number of links per pass; 1, 2, 4 force that count (2, 4 need nhit = 1).
int lanes_per_link(const Geom &g, int nhit, int requested);
// Links per workgroup of a pass with `lanes` lanes per link.
int pass_links_per_block(const Geom &g, int lanes);
// workgroups covering the nlat * Vh links of one pass, nb links each
int pass_blocks(const Geom &g, int nb);
// plaquette reduction: workgroups per layer (the most any plaquette kernel uses)
int plaq_blocks(const Geom &g);
// Chunks of x3 per column of the plaquette walk (k_plaq_walk) for links of
// the given precision, or 0 where the per-site kernels run instead (FP32, and
// lattices too small to walk).
int plaq_walk_chunks(const Geom &g, int precision);
// workgroups per layer of the plaquette walk with nch chunks (<= plaq_blocks)
int plaq_walk_blocks(const Geom &g, int nch);
// workgroups of a measured pass of su3_sweep_measure with `lanes` lanes per link
int meas_blocks(const Geom &g, int lanes);
// Polyakov loops: workgroups per layer
int polyakov_blocks(const Geom &g);

// scratch regions whose size depends on the lattice (bytes from the start)
size_t meas_offset(const Geom &g);
size_t polyakov_offset(const Geom &g);
size_t scratch_bytes_of(const Geom &g);

// Element index (in complex numbers) of entry e of link n of block (dir, par)
// in the tiled link store.
size_t dev_index(const Geom &g, int dir, int par, int e, long long n);
// Canonical site (layer * V + lex) of element n of a block of parity par.
long long site_of_elem(const Geom &g, int par, long long n);
// Block (dir, par) and element n of canonical link id lid = 4 site + dir;
// false if lid is out of range.
bool elem_of_lid(const Geom &g, uint64_t lid, int *dir, int *par, long long *n);
// Row 2 of an SU(3) matrix in the canonical 18-double layout from rows 0 and 1:
// conj(row 0 x row 1), the formula the kernels use.
void rebuild_row2_host(double *m);
// The tiled device image (link_bytes_of bytes, FP64 or FP32 entries) to and
// from the canonical FP64 layout host[(4 site + dir) 18 + (3 row + col) 2 + reim]
// of 72 V nlat doubles.  unpack rebuilds row 2 in FP64; pack stores rows 0, 1
// (rounded to FP32 for precision 32) and leaves padding untouched.
void unpack_links(int precision, const Geom &g, const void *image, double *host);
void pack_links(int precision, const Geom &g, const double *host, void *image);

}  // namespace su3hb
