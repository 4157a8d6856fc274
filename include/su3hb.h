/*
 * su3hb.h -- C ABI of the MI355X (gfx950) checkerboard SU(3) heat-bath library.
 *
 * What it computes (Berg & Wu, "Fortran MPI Checkerboard Code for SU(3)
 * Lattice Gauge Theory II"): nequi checkerboard updating sweeps of pure SU(3)
 * lattice gauge theory with the Wilson action, S = beta sum_P (1 - 1/3 Re Tr U_P),
 * on a periodic 4D torus (nlat = 1) or a double-layered torus (nlat = 2)
 * (Sec. 1; Sec. 2, eq. (1) and the nequi/lswp description; Table 1).  Every
 * link is an SU(3) matrix of 18 reals (App. A, eq. (4)); the paper reports the
 * cost per SU(3) matrix update (Sec. 2.1, Fig. 1), which is the unit of this
 * library's throughput.  A sweep is 8 checkerboard passes (direction mu = 0..3,
 * parity even then odd); each updated link gets the Cabibbo-Marinari heat bath
 * in its SU(2) subgroups (0,1), (1,2), (0,2) with nhit Kennedy-Pendleton
 * attempts per subgroup ("1-hit" for nhit = 1, Sec. 2.1) and is then
 * reunitarised.  Random numbers are Philox4x64-10 keyed by (seed; link id,
 * sweep index, subgroup/attempt, purpose), so a result does not depend on the
 * launch configuration, and resuming from a checkpoint is exact.
 *
 * Storage: the device keeps rows 0 and 1 of every link (12 reals); row 2 of an
 * SU(3) matrix is conj(row 0 x row 1) and is rebuilt wherever a link is read,
 * on the device and in the host copies below.
 *
 * Memory ownership: the caller allocates the device buffers (sizes from
 * su3_footprint) and the HIP stream; the library never allocates or frees
 * device memory.  All calls enqueue on the stream given to su3_create and
 * return without waiting, except su3_plaquette, su3_sweep_measure, su3_get_links,
 * su3_set_links, su3_get_link_sample, su3_counters and su3_profile_read, which
 * synchronise that stream.
 *
 * Errors: every call returns an su3_status; nothing aborts or throws across
 * the ABI.  su3_last_error() gives a thread-local description of the last
 * failure.  A launch or asynchronous device fault is reported as SU3_EDEVICE
 * by the call that detects it.
 *
 * Threading: one context per stream.  Distinct contexts are independent and
 * may be used from different threads; one context must not be used from two
 * threads at once.  The same holds for a job server.
 */
#ifndef SU3HB_H
#define SU3HB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SU3_OK = 0,
    SU3_EINVAL = -1,  /* invalid argument (parameters, sizes, null pointers, beta) */
    SU3_ENOSPC = -2,  /* a caller buffer is smaller than su3_footprint requires */
    SU3_EDEVICE = -3, /* HIP launch or runtime error */
    SU3_ESTATE = -4,  /* call out of order, e.g. sweep or plaquette before start */
    SU3_ENUMERIC = -5 /* the link data are not finite or not in SU(3): a property of the data, not
                         a device fault; the call still completes and writes its outputs */
} su3_status;

typedef struct su3_ctx su3_ctx;

typedef struct {
    int32_t L[4];       /* lattice extents L0..L3 (the paper's nl1..nl4); each even, 2 <= L <= 1024,
                           nlat*L0*L1*L2*L3 <= 2^30 */
    int32_t nlat;       /* 1 = periodic torus, 2 = double-layered torus (Table 1, nlat) */
    uint32_t flip_mask; /* nlat = 2: bit mu set => stepping across the mu boundary moves to the other
                           layer (default reading 0x7: the three partitioned directions of Table 3);
                           must be 0 for nlat = 1 */
    int32_t precision;  /* 64: links stored and multiplied in FP64.
                           32: links stored and multiplied in FP32; reunitarisation, plaquette
                           products and all global sums in FP64 */
    int32_t nhit;       /* Kennedy-Pendleton attempts per SU(2) subgroup, >= 1 (1 = 1-hit) */
    uint64_t seed;      /* Philox key */
} su3_params;

/* Device bytes the caller must provide for the links and the scratch area.
 * Links: 8 blocks (4 directions x 2 parities) of round_up(nlat*V/2, 64) + 64
 * links, each link stored as its rows 0 and 1 (6 complex numbers of the link
 * precision).
 * Scratch: heat-bath counter slots (64 KiB), plaquette partial sums and
 * failing-link counts (at most 64 KiB per layer), Polyakov partial sums (16
 * bytes per 256 sites of a time slice, per layer) and the partial sums of the
 * measured passes of su3_sweep_measure (3 passes x nlat doubles per 64 links
 * of one pass: 24 bytes on a single torus, 48 on a double-layered torus).
 * SU3_EINVAL on invalid parameters. */
su3_status su3_footprint(const su3_params *p, size_t *link_bytes, size_t *scratch_bytes);

/* Bind a context to caller-owned device memory and a hipStream_t (NULL = the
 * null stream).  d_links and d_scratch must be device pointers, 256-byte
 * aligned, of at least the footprint sizes (else SU3_ENOSPC).  Parameters are
 * validated before any HIP call.  The links are undefined until su3_start or
 * su3_set_links. */
su3_status su3_create(const su3_params *p, void *d_links, size_t link_bytes, void *d_scratch,
                      size_t scratch_bytes, void *hip_stream, su3_ctx **out);

/* Start configuration (Sec. 2: created before the timed sweeps and excluded
 * from the timing).  hot = 0: every link the identity; hot = 1: Haar-random
 * links.  Resets the sweep counter and the heat-bath counters. */
su3_status su3_start(su3_ctx *c, int32_t hot);

/* Enqueue n >= 0 sweeps at coupling beta (finite, > 0): the nequi updating
 * sweeps without measurements that the paper times (Sec. 2, eq. (1) and the
 * paragraph after it; Tables 1-3 give the sweep counts per lattice).  One
 * sweep is the eight checkerboard passes mu = 0..3 x parity (even, odd), each
 * updating every link U_mu(x) of that parity once (4 V nlat updates per
 * sweep, the paper's unit of "SU(3) matrix updates", Sec. 2.1).  The sweep
 * counter advances by n; it keys the random numbers, so sweep(a) then
 * sweep(b) equals sweep(a + b) bit for bit.  Asynchronous: the call only
 * enqueues the 8 n pass kernels on the context's stream.  SU3_ESTATE before
 * su3_start/su3_set_links; SU3_EINVAL for n < 0 or beta not finite and > 0. */
su3_status su3_sweep(su3_ctx *c, int32_t n, double beta);

/* n sweeps, each followed by a plaquette measurement (the measurement
 * routines the paper advises timing together with the sweeps, Sec. 2.2, last
 * paragraph), with one stream synchronisation at the end (per 256 sweeps)
 * instead of one per sweep: out[k*(1+nlat) + 0] is the mean plaquette after
 * sweep k, out[k*(1+nlat) + 1 + l] that of layer l (as su3_plaquette).
 * n_out >= n * (1 + nlat).
 * No separate plaquette pass runs: after the odd pass of direction mu no
 * later pass of the sweep changes U_nu or U_mu for nu < mu, so the odd passes
 * of mu = 1, 2, 3 each also sum Re Tr(U_new S) over their links, S being the
 * staple terms of the directions nu < mu, which is the final plaquette sum of
 * the planes (nu, mu), nu < mu; the three passes give all six planes.  On a
 * double-layered torus a plaquette based at x - nu lies in the other layer
 * than x when that step crosses a flipped boundary; the measured passes sum
 * those lower terms separately and file them under that layer, so that each
 * plaquette counts for its base site's layer.  One small kernel per sweep adds
 * the per-workgroup sums in a fixed order.  The
 * value equals su3_plaquette's up to rounding (products in the link
 * precision, before the final reunitarisation of the new link; sums in
 * FP64).  SU3_ENUMERIC (outputs written) if a measured plaquette is not
 * finite. */
su3_status su3_sweep_measure(su3_ctx *c, int32_t n, double beta, double *out, size_t n_out);

/* Double-layered torus only (nlat = 2, else SU3_EINVAL): n sweeps with
 * per-layer couplings, action S = sum_P beta_{layer(P)} (1 - 1/3 Re Tr U_P)
 * where a plaquette takes the coupling of the layer of its base site.  The
 * heat bath samples exp(1/3 Re Tr(U A)) with each staple term weighted by its
 * plaquette's coupling ("hot" and "cold" layers; the paper leaves the DLT to
 * be explored, Sec. 1).  Asynchronous, like su3_sweep. */
su3_status su3_sweep_betas(su3_ctx *c, int32_t n, double beta0, double beta1);

/* Polyakov loops along direction 3: for every start (x0, x1, x2, x3 = 0,
 * layer) the trace over 3 of the ordered product of U_3 along the closed path
 * in +3 (2 L3 links when crossing the direction-3 boundary switches the layer,
 * i.e. flip bit 3 on a double-layered torus).  out[0], out[1] = Re, Im of the
 * mean over all starts; out[2 + 2l], out[3 + 2l] over the starts in layer l.
 * n >= 2 (1 + nlat).  Products and sums in FP64.  Synchronises the stream. */
su3_status su3_polyakov(su3_ctx *c, double *out, int32_t n);

/* Mean plaquette 1/3 Re Tr U_P: out[0] over the whole lattice, out[1..nlat] per
 * layer (a plaquette belongs to the layer of its base site).  The paper's
 * runs time sweeps without measurements (Sec. 2) and advise timing the
 * measurement routines as well before production runs (Sec. 2.2, last
 * paragraph); the plaquette is the basic one.  n >= 1 + nlat.  Accumulated in
 * FP64 with a fixed reduction order (bitwise reproducible).  The same pass
 * checks every link: SU3_ENUMERIC (out still written) if any link is not
 * finite or its stored rows 0 and 1 are not orthonormal within 1e-10 (FP64
 * links) or 1e-5 (FP32 links); the last-error text gives the count.
 * Synchronises the stream. */
su3_status su3_plaquette(su3_ctx *c, double *out, int32_t n);

/* For callers that cannot allocate device memory or synchronise -- code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc --
 * the plaquette of su3_plaquette without a context or a workspace: the links
 * in d_links (the tiled layout a context with parameters p keeps, link_bytes
 * >= su3_footprint's link bytes, 256-byte aligned) are summed with the same
 * kernels and reduction order, and the results are written to the device
 * buffer d_out (n_out >= 2 + nlat doubles): d_out[0] the mean plaquette,
 * d_out[1..nlat] per layer, d_out[1 + nlat] the number of links failing the
 * check of su3_plaquette (as a double).  Enqueued on hip_stream; nothing is
 * allocated (no hipMalloc, hipFree or allocating library call) and nothing
 * waits.  The partial sums live in a library-owned device array of 256 KiB
 * per GPU (held until the process ends; the largest lattice needs 128 KiB):
 * every call on a GPU shares it, so calls that overlap on one GPU race, and
 * the caller must order them (one stream, or events).  Every call overwrites
 * all of the array it reads, so nothing needs clearing between calls.
 * SU3_EINVAL / SU3_ENOSPC for invalid parameters, pointers or sizes (checked
 * before any HIP call), SU3_EDEVICE for a launch failure. */
su3_status su3_plaquette_noalloc(const su3_params *p, const void *d_links, size_t link_bytes, double *d_out,
                                 int32_t n_out, void *hip_stream);

/* Project every link back onto SU(3) (Gram-Schmidt of rows 0 and 1, row 2 =
 * conj(row0 x row1)), in FP64 for both precisions.  Not described in the
 * paper, which stores 18 reals per link (App. A, eq. (4)) without saying how
 * rounding drift off SU(3) is held back; here it is part of the method's
 * specification, and the heat bath already applies it to every link it
 * updates.  This call applies it to the whole lattice, e.g. after
 * su3_set_links of data from elsewhere.  Asynchronous. */
su3_status su3_reunitarise(su3_ctx *c);

/* Copy the links to / from host memory in the canonical FP64 layout
 * host[(4*site + mu)*18 + (3*row + col)*2 + reim], site = layer*V + lex,
 * lex = x0 + L0*(x1 + L1*(x2 + L2*x3)).  n_doubles must be 72*V*nlat.
 * For precision 32 the values are widened / rounded to FP32.  su3_get_links
 * returns row 2 rebuilt in FP64 from the stored rows 0 and 1; su3_set_links
 * stores rows 0 and 1 and ignores row 2 (exact for SU(3) input; other input
 * is thereby read as rows 0, 1 and conj(row 0 x row 1)).  Synchronise the
 * stream.  su3_set_links also marks the context started. */
su3_status su3_get_links(su3_ctx *c, double *host, size_t n_doubles);
su3_status su3_set_links(su3_ctx *c, const double *host, size_t n_doubles);

/* Copy the n links with canonical ids lids[k] = 4*site + mu (site as above) to
 * host[18*k .. 18*k+17], same element order and row-2 rebuild as
 * su3_get_links: a sampled check
 * of a lattice too large to copy whole.  SU3_EINVAL for an id out of range.
 * Synchronises the stream. */
su3_status su3_get_link_sample(su3_ctx *c, const uint64_t *lids, size_t n, double *host);

/* Sweep counter (the sweep index of the next sweep) for checkpoint / resume. */
su3_status su3_get_sweep_index(su3_ctx *c, uint64_t *sweep_index);
su3_status su3_set_sweep_index(su3_ctx *c, uint64_t sweep_index);

/* Sweeps done since start and Kennedy-Pendleton attempts / acceptances (exact
 * integer counts).  The paper quotes the acceptance rate of its 1-hit heat
 * bath, 97.2 % at beta = 5.7 (Sec. 2.1); kp_accepts / kp_attempts is that
 * rate.  Every SU(2) subgroup of every updated link makes nhit attempts at
 * most and stops at its first acceptance, so with nhit = 1 kp_attempts is
 * 3 x 4 V nlat per sweep, less one for every subgroup whose staple projection
 * vanishes exactly (k = 0: nothing to sample, no attempt).  Any pointer may be
 * NULL.  Synchronises the stream. */
su3_status su3_counters(su3_ctx *c, uint64_t *sweeps, uint64_t *kp_attempts, uint64_t *kp_accepts);

/* Random gauge transformation U_mu(x) -> g(x) U_mu(x) g(x+mu)^+ with Haar g
 * drawn from key gseed (a test of gauge invariance; not part of a sweep). */
su3_status su3_gauge_transform(su3_ctx *c, uint64_t gseed);

/* Per-pass timing: while enabled, one heat-bath pass launch per sweep is
 * bracketed by HIP events on the context's stream, pass 2 mu + parity of the
 * sweep with index s when 2 mu + parity = s mod 8, so eight consecutive sweeps
 * time each of the eight passes once at two event records per sweep.
 * su3_profile_read synchronises and returns the summed time of the timed
 * passes in ms and their number since the last read (then resets both).
 * The context holds two HIP events per timed sweep until the next read and
 * reuses them afterwards: read at least every few ten thousand sweeps. */
su3_status su3_profile(su3_ctx *c, int32_t enable);
su3_status su3_profile_read(su3_ctx *c, double *total_ms, uint64_t *passes);

/* Lanes per link of the heat-bath passes.  By default (lanes = 0) a pass of
 * more than 32768 links runs one lane per link; smaller passes, which would
 * leave most of the GPU idle and take about one link update's latency, run 2
 * (up to 32768 links) or 4 (up to 8192) lanes per link that share the
 * staple directions and the random draws of the update (1-hit only).  The
 * result does not depend on the choice: every variant adds in the same order
 * and gives the same bits.  lanes = 1, 2 or 4 forces that count (2 and 4 need
 * nhit = 1, else SU3_EINVAL).  su3_get_lanes_per_link returns the count the
 * passes use. */
su3_status su3_set_lanes_per_link(su3_ctx *c, int32_t lanes);
su3_status su3_get_lanes_per_link(su3_ctx *c, int32_t *lanes);

/* Releases the context (host memory and events); never frees caller memory. */
su3_status su3_destroy(su3_ctx *c);

/* Bandwidth probe: copy `bytes` (multiple of 16) from src to dst on the given
 * stream with 16-byte vector loads and stores.  Asynchronous. */
su3_status su3_stream_copy(void *dst, const void *src, size_t bytes, void *hip_stream);

/* ------------------------------------------------------------------------
 * Job server: continuous batching of many independent lattices on one GPU.
 *
 * The caller gives the server one device buffer, its HBM budget.  Submitted
 * jobs wait in submission order and are admitted when fewer than max_active
 * jobs run and a first-fit allocation of the job's footprint (su3_footprint:
 * links + scratch) succeeds inside the buffer.  Each su3_server_step admits
 * what fits, runs one sweep of every admitted job -- 8 batched launches per
 * group of jobs with the same precision, hit count and geometry, one per
 * checkerboard pass -- and retires
 * the jobs that reached their sweep count (final plaquette and heat-bath
 * counters kept, memory freed); su3_server_run does the same for several
 * sweeps per call.  A group of 1-hit jobs with at most 32768 links per pass
 * in total runs two lanes per link (such a pass is bound by the latency of
 * one update).  A job's links get the same per-link
 * arithmetic and the same keyed random numbers as a single lattice run with
 * su3_start/su3_sweep, so its result is the same alone and in the mix.
 * su3_server_step synchronises the server's stream.
 * ------------------------------------------------------------------------ */
typedef struct su3_server su3_server;

typedef struct {
    su3_params params; /* lattice, precision, nhit and Philox key of the job */
    double beta;       /* coupling, finite and > 0 */
    int32_t nsweeps;   /* sweeps to run, >= 1 */
    int32_t hot;       /* start: 0 cold, 1 Haar hot */
} su3_job;

typedef enum { SU3_JOB_QUEUED = 0, SU3_JOB_ACTIVE = 1, SU3_JOB_DONE = 2 } su3_job_state;

typedef struct {
    int32_t state;        /* su3_job_state */
    int32_t sweeps_done;
    double plaquette[3];  /* once done: total, then per layer (as su3_plaquette) */
    uint64_t kp_attempts; /* once done */
    uint64_t kp_accepts;
    int64_t bad_links;    /* once done: links failing the check of su3_plaquette (0 for a healthy chain) */
} su3_job_result;

/* d_arena: device buffer of arena_bytes, 256-byte aligned; the server keeps
 * its job tables at the start and allocates job footprints from the rest.
 * max_active in [1, 4096].  SU3_ENOSPC if the arena cannot hold the tables. */
su3_status su3_server_create(void *d_arena, size_t arena_bytes, int32_t max_active, void *hip_stream,
                             su3_server **out);
/* Queue a job; SU3_EINVAL for invalid parameters, SU3_ENOSPC if its footprint
 * exceeds the whole arena (it could never be admitted). */
su3_status su3_server_submit(su3_server *s, const su3_job *job, int64_t *job_id);
/* Admit, run one batched sweep, retire; counts after the step (any pointer may be NULL). */
su3_status su3_server_step(su3_server *s, int32_t *n_active, int32_t *n_queued, int32_t *n_finished);
/* As su3_server_step, but runs k = min(max_sweeps, fewest remaining sweeps of
 * an admitted job) sweeps before retiring, with a single synchronisation: no
 * job finishes inside the call, and every job's results are those of k single
 * steps.  Newly submitted jobs wait for the call to end before admission.
 * SU3_EINVAL if max_sweeps < 1. */
su3_status su3_server_run(su3_server *s, int32_t max_sweeps, int32_t *n_active, int32_t *n_queued,
                          int32_t *n_finished);
/* State, sweeps done and, once done, the final plaquette and counters of a job.
 * SU3_EINVAL for an unknown (or released) id. */
su3_status su3_server_poll(su3_server *s, int64_t job_id, su3_job_result *out);
/* Drop the record of a finished job (after its result was polled): the server
 * keeps every job's record until then, so a long-running caller releases the
 * jobs it has read.  SU3_ESTATE if the job is not done, SU3_EINVAL for an
 * unknown id. */
su3_status su3_server_release(su3_server *s, int64_t job_id);
/* Copy an active job's links to host memory in the canonical FP64 layout of
 * su3_get_links (n_doubles = 72 V nlat of the job), between server calls:
 * the read-back for checking a served job link by link.  SU3_ESTATE if the
 * job is queued or done (its links are then not on the device).
 * Synchronises the server's stream. */
su3_status su3_server_get_links(su3_server *s, int64_t job_id, double *host, size_t n_doubles);
su3_status su3_server_stats(su3_server *s, size_t *arena_used, size_t *arena_peak, uint64_t *steps);
/* Waits for the stream, frees host resources; never frees the arena. */
su3_status su3_server_destroy(su3_server *s);

const char *su3_strerror(su3_status s);
const char *su3_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
