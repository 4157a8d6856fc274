// launch.h -- host-side launchers of the gfx950 kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device.h"
#include "layout.h"

namespace su3hb {

// One job of a batched pass (continuous batching of several lattices).
struct BatchJob {
    void *links;                   // this job's link buffer (tiled layout, its own precision)
    unsigned long long *counters;  // this job's heat-bath counter slots
    Geom g;
    double beta;
    uint64_t seed;
    uint64_t sweep0;               // sweep index at global step admit_step
    long long admit_step;
    int nhit;
    int lanes;                     // lanes per link: 1, or 2 (nhit = 1 only)
    int tile_begin;                // first workgroup of this job in the launch
};

hipError_t launch_start(int precision, void *links, const Geom &g, int hot, uint64_t seed, hipStream_t s);
// One checkerboard pass (mu, par) with `lanes` lanes per link (1; 2 or 4 with nhit = 1).
hipError_t launch_update(int precision, void *links, const Geom &g, int mu, int par, double beta, uint64_t sweep,
                         uint64_t seed, int nhit, int lanes, unsigned long long *counters, hipStream_t s);
// one pass (mu, par) of every job in d_jobs (device copy, sorted by tile_begin);
// all jobs share `precision`; hit1: every job has nhit = 1; dlt: every job is
// a double-layered torus (else every job is a single torus).  A job with
// `lanes` lanes per link takes ceil(lanes * nlat * Vh / 64) workgroups.
hipError_t launch_update_batch(int precision, bool hit1, bool dlt, const BatchJob *d_jobs, int njobs, int ntiles,
                               long long step, int mu, int par, hipStream_t s);
// Plaquette sums of the whole lattice into sums[0..3] (total, per layer,
// number of links failing the unitarity check); partials: 2 * nlat *
// plaq_blocks(g) doubles.  With `mean` non-null also the normalised values
// mean[0..nlat] and the failing-link count mean[1 + nlat], on the device.
hipError_t launch_plaquette(int precision, const void *links, const Geom &g, double *partials, double *sums,
                            hipStream_t s, double *mean = nullptr);
// The odd pass of mu (1, 2 or 3) that also stores, per workgroup, the sum of
// its final plaquettes in the planes (nu, mu), nu < mu: meas[b] on a single
// torus, meas[2 b + l] for layer l on a double-layered torus (each plaquette
// under its base site's layer), b < meas_blocks(g, lanes).  The three passes
// write consecutive slices of nlat * meas_blocks(g, lanes) doubles, which
// launch_measure_final adds up into sums[0] (total) and sums[1 + l] (layer l).
hipError_t launch_update_measured(int precision, void *links, const Geom &g, int mu, double beta, uint64_t sweep,
                                  uint64_t seed, int nhit, int lanes, unsigned long long *counters, double *meas,
                                  hipStream_t s);
hipError_t launch_measure_final(const double *meas, const Geom &g, int lanes, double *sums, hipStream_t s);
// double-layered torus with per-layer couplings (a plaquette takes its base site's layer coupling)
hipError_t launch_update_twob(int precision, void *links, const Geom &g, int mu, int par, double beta0,
                              double beta1, uint64_t sweep, uint64_t seed, int nhit, unsigned long long *counters,
                              hipStream_t s);
// Polyakov loops along direction 3: out[2 l], out[2 l + 1] = sums of Re, Im of Tr/3 over the starts in layer l;
// partials: 2 * nlat * polyakov_blocks(g) doubles
hipError_t launch_polyakov(int precision, const void *links, const Geom &g, double *partials, double *out,
                           hipStream_t s);
hipError_t launch_reunit(int precision, void *links, const Geom &g, hipStream_t s);
hipError_t launch_gauge(int precision, void *links, const Geom &g, uint64_t gseed, hipStream_t s);
hipError_t launch_zero_u64(unsigned long long *p, int n, hipStream_t s);
hipError_t launch_copy(void *dst, const void *src, size_t bytes, hipStream_t s);

}  // namespace su3hb
