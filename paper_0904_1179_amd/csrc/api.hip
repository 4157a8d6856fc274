// api.hip -- host runtime behind the C ABI declared in include/su3hb.h.
//
// The context binds caller-owned device buffers and a stream; every entry
// point validates its arguments before touching HIP, enqueues work on the
// context's stream and reports failures as su3_status plus a thread-local
// message.  A sweep is the 8-pass schedule mu = 0..3 x parity (even, odd),
// each pass one k_update launch; the sweep index keys the random numbers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/su3hb.h"
#include "runtime.h"

struct su3_ctx {
    su3_params p;
    su3hb::Geom g;
    size_t V;
    void *links;
    size_t link_bytes;
    unsigned char *scratch;
    size_t scratch_bytes;
    hipStream_t stream;
    bool started;
    uint64_t sweep_index;  // index of the next sweep (keys the random numbers)
    uint64_t sweeps_done;  // since the last start
    int lanes_requested;   // lanes per link of the passes: 0 = by pass size (lanes_per_link)
    // profiling
    bool profile;
    std::vector<hipEvent_t> ev;  // pairs (start, stop)
    size_t ev_used;
};

namespace su3hb {

su3_status hip_fail(hipError_t e, const char *where)
{
    return fail(SU3_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

}  // namespace su3hb

using namespace su3hb;

namespace {

su3_status check_ctx(su3_ctx *c)
{
    if (!c) return fail(SU3_EINVAL, "context is NULL");
    return SU3_OK;
}

su3_status check_started(su3_ctx *c)
{
    if (!c->started) return fail(SU3_ESTATE, "links are undefined: call su3_start or su3_set_links first");
    return SU3_OK;
}

unsigned long long *counters_of(su3_ctx *c) { return (unsigned long long *)(c->scratch + kOffCounters); }

}  // namespace

extern "C" {

const char *su3_strerror(su3_status s)
{
    switch (s) {
    case SU3_OK: return "success";
    case SU3_EINVAL: return "invalid argument";
    case SU3_ENOSPC: return "buffer smaller than the footprint";
    case SU3_EDEVICE: return "HIP device error";
    case SU3_ESTATE: return "call out of order";
    case SU3_ENUMERIC: return "non-finite or non-unitary link data";
    }
    return "unknown status";
}

const char *su3_last_error(void) { return su3hb::last_error(); }

su3_status su3_footprint(const su3_params *p, size_t *link_bytes, size_t *scratch_bytes)
{
    su3_status st = check_params(p);
    if (st != SU3_OK) return st;
    const Geom g = make_geom(p);
    if (link_bytes) *link_bytes = link_bytes_of(p, g);
    if (scratch_bytes) *scratch_bytes = scratch_bytes_of(g);
    return SU3_OK;
}

su3_status su3_create(const su3_params *p, void *d_links, size_t link_bytes, void *d_scratch, size_t scratch_bytes,
                      void *hip_stream, su3_ctx **out)
{
    if (!out) return fail(SU3_EINVAL, "out is NULL");
    *out = nullptr;
    su3_status st = check_params(p);
    if (st != SU3_OK) return st;
    if (!d_links || !d_scratch) return fail(SU3_EINVAL, "device buffers must not be NULL");
    if (((uintptr_t)d_links & 255u) || ((uintptr_t)d_scratch & 255u))
        return fail(SU3_EINVAL, "device buffers must be 256-byte aligned");
    const Geom g = make_geom(p);
    if (link_bytes < link_bytes_of(p, g))
        return fail(SU3_ENOSPC, "link buffer has " + std::to_string(link_bytes) + " bytes, needs " +
                                    std::to_string(link_bytes_of(p, g)));
    if (scratch_bytes < scratch_bytes_of(g))
        return fail(SU3_ENOSPC, "scratch buffer has " + std::to_string(scratch_bytes) + " bytes, needs " +
                                    std::to_string(scratch_bytes_of(g)));
    su3_ctx *c = new (std::nothrow) su3_ctx();
    if (!c) return fail(SU3_EINVAL, "out of host memory");
    c->p = *p;
    c->g = g;
    c->V = (size_t)p->L[0] * p->L[1] * p->L[2] * p->L[3];
    c->links = d_links;
    c->link_bytes = link_bytes;
    c->scratch = (unsigned char *)d_scratch;
    c->scratch_bytes = scratch_bytes;
    c->stream = (hipStream_t)hip_stream;
    c->started = false;
    c->sweep_index = 0;
    c->sweeps_done = 0;
    c->profile = false;
    c->ev_used = 0;
    c->lanes_requested = 0;
    *out = c;
    return SU3_OK;
}

su3_status su3_destroy(su3_ctx *c)
{
    if (!c) return SU3_OK;
    for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
    delete c;
    return SU3_OK;
}

su3_status su3_start(su3_ctx *c, int32_t hot)
{
    su3_status st = check_ctx(c);
    if (st != SU3_OK) return st;
    if (hot != 0 && hot != 1) return fail(SU3_EINVAL, "hot must be 0 (cold) or 1 (hot)");
    hipError_t e = su3hb::launch_start(c->p.precision, c->links, c->g, hot, c->p.seed, c->stream);
    if (e != hipSuccess) return hip_fail(e, "start kernel");
    e = su3hb::launch_zero_u64(counters_of(c), 2 * kCounterSlots, c->stream);
    if (e != hipSuccess) return hip_fail(e, "counter reset");
    c->started = true;
    c->sweep_index = 0;
    c->sweeps_done = 0;
    return SU3_OK;
}

namespace {

// enqueue n sweeps (8 pass launches each); arguments already validated.
// meas != NULL: in the last sweep the odd passes of mu = 1, 2, 3 also store
// their per-workgroup (and per-layer) plaquette sums of the planes (nu, mu),
// nu < mu, in meas[(mu - 1) * nlat * meas_blocks .. mu * nlat * meas_blocks).
su3_status enqueue_sweeps(su3_ctx *c, int32_t n, double beta, double *meas = nullptr, const double *betas = nullptr)
{
    const int lanes = lanes_per_link(c->g, c->p.nhit, c->lanes_requested);
    for (int32_t s = 0; s < n; ++s) {
        for (int mu = 0; mu < 4; ++mu)
            for (int par = 0; par < 2; ++par) {
                // one timed pass per sweep, rotating through the eight passes
                const bool timed = c->profile && (uint64_t)(2 * mu + par) == c->sweep_index % 8;
                if (timed) {
                    while (c->ev_used + 2 > c->ev.size()) {
                        hipEvent_t ev;
                        hipError_t e = hipEventCreate(&ev);
                        if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
                        c->ev.push_back(ev);
                    }
                    hipError_t e = hipEventRecord(c->ev[c->ev_used], c->stream);
                    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
                }
                const bool measured = meas && s == n - 1 && mu >= 1 && par == 1;
                hipError_t e;
                if (betas)
                    e = su3hb::launch_update_twob(c->p.precision, c->links, c->g, mu, par, betas[0], betas[1],
                                                  c->sweep_index, c->p.seed, c->p.nhit, counters_of(c), c->stream);
                else if (measured)
                    e = su3hb::launch_update_measured(
                        c->p.precision, c->links, c->g, mu, beta, c->sweep_index, c->p.seed, c->p.nhit, lanes,
                        counters_of(c), meas + (size_t)(mu - 1) * c->g.nlat * su3hb::meas_blocks(c->g, lanes),
                        c->stream);
                else
                    e = su3hb::launch_update(c->p.precision, c->links, c->g, mu, par, beta, c->sweep_index, c->p.seed,
                                             c->p.nhit, lanes, counters_of(c), c->stream);
                if (e != hipSuccess) return hip_fail(e, "update kernel");
                if (timed) {
                    e = hipEventRecord(c->ev[c->ev_used + 1], c->stream);
                    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
                    c->ev_used += 2;
                }
            }
        c->sweep_index += 1;
        c->sweeps_done += 1;
    }
    return SU3_OK;
}

su3_status check_sweep_args(su3_ctx *c, int32_t n, double beta)
{
    su3_status st = check_ctx(c);
    if (st != SU3_OK) return st;
    if (n < 0) return fail(SU3_EINVAL, "n must be >= 0");
    if (!std::isfinite(beta) || !(beta > 0.0)) return fail(SU3_EINVAL, "beta must be finite and > 0");
    return check_started(c);
}

}  // namespace

extern "C" {

su3_status su3_sweep(su3_ctx *c, int32_t n, double beta)
{
    su3_status st = check_sweep_args(c, n, beta);
    if (st != SU3_OK) return st;
    return enqueue_sweeps(c, n, beta);
}

su3_status su3_sweep_betas(su3_ctx *c, int32_t n, double beta0, double beta1)
{
    su3_status st = check_sweep_args(c, n, beta0);
    if (st != SU3_OK) return st;
    if (!std::isfinite(beta1) || !(beta1 > 0.0)) return fail(SU3_EINVAL, "beta1 must be finite and > 0");
    if (c->p.nlat != 2) return fail(SU3_EINVAL, "per-layer couplings need a double-layered torus (nlat = 2)");
    const double b[2] = {beta0, beta1};
    return enqueue_sweeps(c, n, 1.0, nullptr, b);
}

su3_status su3_polyakov(su3_ctx *c, double *out, int32_t n)
{
    su3_status st = check_ctx(c);
    if (st != SU3_OK) return st;
    if (!out || n < 2 * (1 + c->p.nlat)) return fail(SU3_EINVAL, "out must hold 2 * (1 + nlat) doubles");
    st = check_started(c);
    if (st != SU3_OK) return st;
    double *partials = (double *)(c->scratch + polyakov_offset(c->g));
    double *sums = (double *)(c->scratch + kOffSums) + 8;
    hipError_t e = launch_polyakov(c->p.precision, c->links, c->g, partials, sums, c->stream);
    if (e != hipSuccess) return hip_fail(e, "Polyakov kernels");
    double h[4] = {0, 0, 0, 0};
    e = hipMemcpyAsync(h, sums, sizeof(double) * 2 * c->p.nlat, hipMemcpyDeviceToHost, c->stream);
    if (e != hipSuccess) return hip_fail(e, "Polyakov copy");
    e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "Polyakov sync");
    const double V3 = (double)c->g.L[0] * c->g.L[1] * c->g.L[2];
    out[0] = out[1] = 0.0;
    for (int l = 0; l < c->p.nlat; ++l) {
        out[2 + 2 * l] = h[2 * l] / V3;
        out[3 + 2 * l] = h[2 * l + 1] / V3;
        out[0] += h[2 * l];
        out[1] += h[2 * l + 1];
    }
    out[0] /= V3 * c->p.nlat;
    out[1] /= V3 * c->p.nlat;
    return SU3_OK;
}

su3_status su3_sweep_measure(su3_ctx *c, int32_t n, double beta, double *out, size_t n_out)
{
    su3_status st = check_sweep_args(c, n, beta);
    if (st != SU3_OK) return st;
    const int w = 1 + c->p.nlat;
    if (!out && n > 0) return fail(SU3_EINVAL, "out is NULL");
    if (n_out < (size_t)n * (size_t)w) return fail(SU3_EINVAL, "out must hold n * (1 + nlat) doubles");
    double *slots = (double *)(c->scratch + kOffMeasure);
    std::vector<double> h((size_t)kMeasureChunk * 4);
    const double norm = 18.0 * (double)c->V;
    su3_status bad = SU3_OK;
    for (int32_t done = 0; done < n;) {
        const int32_t m = std::min<int32_t>(kMeasureChunk, n - done);
        for (int32_t k = 0; k < m; ++k) {
            hipError_t e;
            // the odd passes of mu = 1, 2, 3 measure all six planes (per layer of each plaquette's base
            // site); one workgroup adds the partials
            double *meas = (double *)(c->scratch + meas_offset(c->g));
            st = enqueue_sweeps(c, 1, beta, meas);
            if (st != SU3_OK) return st;
            e = launch_measure_final(meas, c->g, lanes_per_link(c->g, c->p.nhit, c->lanes_requested),
                                     slots + 4 * k, c->stream);
            if (e != hipSuccess) return hip_fail(e, "plaquette kernels");
        }
        hipError_t e = hipMemcpyAsync(h.data(), slots, sizeof(double) * 4 * m, hipMemcpyDeviceToHost, c->stream);
        if (e != hipSuccess) return hip_fail(e, "measurement copy");
        e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return hip_fail(e, "measurement sync");
        for (int32_t k = 0; k < m; ++k) {
            double *o = out + (size_t)(done + k) * w;
            o[0] = h[4 * k] / (norm * c->p.nlat);
            for (int l = 0; l < c->p.nlat; ++l) o[1 + l] = h[4 * k + 1 + l] / norm;
            if (!std::isfinite(o[0]) && !bad)
                bad = fail(SU3_ENUMERIC, "plaquette after sweep " + std::to_string(done + k) +
                                             " of this call is not finite: the lattice holds non-finite links");
        }
        done += m;
    }
    return bad ? SU3_ENUMERIC : SU3_OK;
}

}  // extern "C"

su3_status su3_plaquette(su3_ctx *c, double *out, int32_t n)
{
    su3_status st = check_ctx(c);
    if (st != SU3_OK) return st;
    if (!out || n < 1 + c->p.nlat) return fail(SU3_EINVAL, "out must hold 1 + nlat doubles");
    st = check_started(c);
    if (st != SU3_OK) return st;
    double *sums = (double *)(c->scratch + kOffSums);
    double *partials = (double *)(c->scratch + kOffPartials);
    hipError_t e = su3hb::launch_plaquette(c->p.precision, c->links, c->g, partials, sums, c->stream);
    if (e != hipSuccess) return hip_fail(e, "plaquette kernels");
    double h[4] = {0, 0, 0, 0};
    e = hipMemcpyAsync(h, sums, sizeof(h), hipMemcpyDeviceToHost, c->stream);
    if (e != hipSuccess) return hip_fail(e, "plaquette copy");
    e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "plaquette sync");
    const double norm = 18.0 * (double)c->V;
    out[0] = h[0] / (norm * c->p.nlat);
    for (int l = 0; l < c->p.nlat; ++l) out[1 + l] = h[1 + l] / norm;
    if (h[3] != 0.0 || !std::isfinite(out[0]))
        return fail(SU3_ENUMERIC, std::to_string((long long)h[3]) +
                                      " links are not finite or have rows 0, 1 that are not orthonormal within " +
                                      std::to_string(unitarity_tol(c->p.precision)) + "; plaquette " +
                                      std::to_string(out[0]));
    return SU3_OK;
}

}  // extern "C"

namespace {

// Workspace of su3_plaquette_noalloc: a file-scope device array, one copy per
// GPU, held until the process ends.  Host code never uses the array's name
// as an address (on the host it is only a handle for the symbol lookup); the
// device address comes from hipGetSymbolAddress, once per device, and is
// kept per device.
constexpr size_t kNoallocScratchBytes = 256 << 10;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

std::mutex g_scratch_mutex;
void *g_scratch_ptr[kMaxDevices] = {};

// The current device's copy of `scratch` (looked up on its first use there).
su3_status noalloc_scratch(unsigned char **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(SU3_EDEVICE, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!ptr) return fail(SU3_EDEVICE, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[dev] = ptr;
    }
    *out = (unsigned char *)g_scratch_ptr[dev];
    return SU3_OK;
}

}  // namespace

extern "C" {

su3_status su3_plaquette_noalloc(const su3_params *p, const void *d_links, size_t link_bytes, double *d_out,
                                 int32_t n_out, void *hip_stream)
{
    su3_status st = check_params(p);
    if (st != SU3_OK) return st;
    if (!d_links || !d_out) return fail(SU3_EINVAL, "d_links and d_out must not be NULL");
    if ((uintptr_t)d_links & 255u) return fail(SU3_EINVAL, "d_links must be 256-byte aligned");
    if (n_out < 2 + p->nlat) return fail(SU3_EINVAL, "d_out must hold 2 + nlat doubles");
    const Geom g = make_geom(p);
    if (link_bytes < link_bytes_of(p, g))
        return fail(SU3_ENOSPC, "link buffer has " + std::to_string(link_bytes) + " bytes, needs " +
                                    std::to_string(link_bytes_of(p, g)));
    // partial sums, then the 4 sums (the same layout as a context's scratch from kOffSums on)
    const size_t partial_bytes = 2 * sizeof(double) * (size_t)p->nlat * (size_t)plaq_blocks(g);
    const size_t need = 256 + partial_bytes;
    if (need > kNoallocScratchBytes)
        return fail(SU3_EINVAL, "lattice needs " + std::to_string(need) + " bytes of workspace, more than the " +
                                    std::to_string(kNoallocScratchBytes) + " of su3_plaquette_noalloc");
    unsigned char *ws = nullptr;
    st = noalloc_scratch(&ws);
    if (st != SU3_OK) return st;
    hipError_t e = su3hb::launch_plaquette(p->precision, d_links, g, (double *)(ws + 256), (double *)ws,
                                           (hipStream_t)hip_stream, d_out);
    if (e != hipSuccess) return hip_fail(e, "plaquette kernels");
    return SU3_OK;
}

su3_status su3_reunitarise(su3_ctx *c)
{
    su3_status st = check_ctx(c);
    if (st != SU3_OK) return st;
    st = check_started(c);
    if (st != SU3_OK) return st;
    hipError_t e = su3hb::launch_reunit(c->p.precision, c->links, c->g, c->stream);
    if (e != hipSuccess) return hip_fail(e, "reunitarise kernel");
    return SU3_OK;
}

su3_status su3_gauge_transform(su3_ctx *c, uint64_t gseed)
{
    su3_status st = check_ctx(c);
    if (st != SU3_OK) return st;
    st = check_started(c);
    if (st != SU3_OK) return st;
    hipError_t e = su3hb::launch_gauge(c->p.precision, c->links, c->g, gseed, c->stream);
    if (e != hipSuccess) return hip_fail(e, "gauge kernel");
    return SU3_OK;
}

su3_status su3_get_links(su3_ctx *c, double *host, size_t n_doubles)
{
    su3_status st = check_ctx(c);
    if (st != SU3_OK) return st;
    if (!host) return fail(SU3_EINVAL, "host buffer is NULL");
    const size_t need = (size_t)72 * c->V * c->p.nlat;
    if (n_doubles != need) return fail(SU3_EINVAL, "n_doubles must be 72*V*nlat = " + std::to_string(need));
    st = check_started(c);
    if (st != SU3_OK) return st;
    std::vector<unsigned char> buf;
    try {
        buf.resize(link_bytes_of(&c->p, c->g));
    } catch (...) {
        return fail(SU3_EINVAL, "out of host memory for the staging copy");
    }
    hipError_t e = hipMemcpyAsync(buf.data(), c->links, buf.size(), hipMemcpyDeviceToHost, c->stream);
    if (e != hipSuccess) return hip_fail(e, "link copy");
    e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "link copy sync");
    unpack_links(c->p.precision, c->g, buf.data(), host);
    return SU3_OK;
}

su3_status su3_set_links(su3_ctx *c, const double *host, size_t n_doubles)
{
    su3_status st = check_ctx(c);
    if (st != SU3_OK) return st;
    if (!host) return fail(SU3_EINVAL, "host buffer is NULL");
    const size_t need = (size_t)72 * c->V * c->p.nlat;
    if (n_doubles != need) return fail(SU3_EINVAL, "n_doubles must be 72*V*nlat = " + std::to_string(need));
    const size_t bytes = link_bytes_of(&c->p, c->g);
    std::vector<unsigned char> buf;
    try {
        buf.assign(bytes, 0);
    } catch (...) {
        return fail(SU3_EINVAL, "out of host memory for the staging copy");
    }
    pack_links(c->p.precision, c->g, host, buf.data());
    hipError_t e = hipMemcpyAsync(c->links, buf.data(), bytes, hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) return hip_fail(e, "link copy");
    e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "link copy sync");
    if (!c->started) {
        e = su3hb::launch_zero_u64(counters_of(c), 2 * kCounterSlots, c->stream);
        if (e != hipSuccess) return hip_fail(e, "counter reset");
    }
    c->started = true;
    return SU3_OK;
}

su3_status su3_get_link_sample(su3_ctx *c, const uint64_t *lids, size_t n, double *host)
{
    su3_status st = check_ctx(c);
    if (st != SU3_OK) return st;
    if (n == 0) return SU3_OK;
    if (!lids || !host) return fail(SU3_EINVAL, "lids and host must not be NULL");
    st = check_started(c);
    if (st != SU3_OK) return st;
    const Geom &g = c->g;
    const size_t esz = c->p.precision == 64 ? 16 : 8;
    std::vector<unsigned char> buf;
    try {
        buf.resize(n * kEntries * esz);
    } catch (...) {
        return fail(SU3_EINVAL, "out of host memory for the sample");
    }
    for (size_t k = 0; k < n; ++k) {
        int dir, par;
        long long elem;
        if (!elem_of_lid(g, lids[k], &dir, &par, &elem))
            return fail(SU3_EINVAL, "link id " + std::to_string(lids[k]) + " out of range");
        for (int el = 0; el < kEntries; ++el) {
            const size_t idx = dev_index(g, dir, par, el, elem);
            hipError_t e = hipMemcpyAsync(buf.data() + (k * kEntries + el) * esz,
                                          (const unsigned char *)c->links + idx * esz, esz, hipMemcpyDeviceToHost,
                                          c->stream);
            if (e != hipSuccess) return hip_fail(e, "sample copy");
        }
    }
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "sample sync");
    for (size_t k = 0; k < n; ++k) {
        double *dst = host + 18 * k;
        for (int el = 0; el < kEntries; ++el) {
            const size_t i = k * kEntries + el;
            if (c->p.precision == 64) {
                dst[2 * el] = ((const double *)buf.data())[2 * i];
                dst[2 * el + 1] = ((const double *)buf.data())[2 * i + 1];
            } else {
                dst[2 * el] = (double)((const float *)buf.data())[2 * i];
                dst[2 * el + 1] = (double)((const float *)buf.data())[2 * i + 1];
            }
        }
        rebuild_row2_host(dst);
    }
    return SU3_OK;
}

su3_status su3_get_sweep_index(su3_ctx *c, uint64_t *sweep_index)
{
    su3_status st = check_ctx(c);
    if (st != SU3_OK) return st;
    if (!sweep_index) return fail(SU3_EINVAL, "sweep_index is NULL");
    *sweep_index = c->sweep_index;
    return SU3_OK;
}

su3_status su3_set_sweep_index(su3_ctx *c, uint64_t sweep_index)
{
    su3_status st = check_ctx(c);
    if (st != SU3_OK) return st;
    c->sweep_index = sweep_index;
    return SU3_OK;
}

su3_status su3_counters(su3_ctx *c, uint64_t *sweeps, uint64_t *kp_attempts, uint64_t *kp_accepts)
{
    su3_status st = check_ctx(c);
    if (st != SU3_OK) return st;
    st = check_started(c);
    if (st != SU3_OK) return st;
    std::vector<unsigned long long> h(2 * kCounterSlots);
    hipError_t e = hipMemcpyAsync(h.data(), counters_of(c), h.size() * sizeof(unsigned long long),
                                  hipMemcpyDeviceToHost, c->stream);
    if (e != hipSuccess) return hip_fail(e, "counter copy");
    e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "counter sync");
    unsigned long long att = 0, acc = 0;
    for (int k = 0; k < kCounterSlots; ++k) {
        att += h[2 * k];
        acc += h[2 * k + 1];
    }
    if (sweeps) *sweeps = c->sweeps_done;
    if (kp_attempts) *kp_attempts = att;
    if (kp_accepts) *kp_accepts = acc;
    return SU3_OK;
}

su3_status su3_set_lanes_per_link(su3_ctx *c, int32_t lanes)
{
    su3_status st = check_ctx(c);
    if (st != SU3_OK) return st;
    if (lanes != 0 && lanes != 1 && lanes != 2 && lanes != 4) return fail(SU3_EINVAL, "lanes must be 0, 1, 2 or 4");
    if (lanes > 1 && c->p.nhit != 1) return fail(SU3_EINVAL, "2 or 4 lanes per link need nhit = 1");
    c->lanes_requested = lanes;
    return SU3_OK;
}

su3_status su3_get_lanes_per_link(su3_ctx *c, int32_t *lanes)
{
    su3_status st = check_ctx(c);
    if (st != SU3_OK) return st;
    if (!lanes) return fail(SU3_EINVAL, "lanes is NULL");
    *lanes = lanes_per_link(c->g, c->p.nhit, c->lanes_requested);
    return SU3_OK;
}

su3_status su3_profile(su3_ctx *c, int32_t enable)
{
    su3_status st = check_ctx(c);
    if (st != SU3_OK) return st;
    c->profile = enable != 0;
    return SU3_OK;
}

su3_status su3_profile_read(su3_ctx *c, double *total_ms, uint64_t *passes)
{
    su3_status st = check_ctx(c);
    if (st != SU3_OK) return st;
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "profile sync");
    double tot = 0.0;
    for (size_t k = 0; k + 1 < c->ev_used; k += 2) {
        float ms = 0.0f;
        e = hipEventElapsedTime(&ms, c->ev[k], c->ev[k + 1]);
        if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
        tot += ms;
    }
    if (total_ms) *total_ms = tot;
    if (passes) *passes = c->ev_used / 2;
    c->ev_used = 0;
    return SU3_OK;
}

su3_status su3_stream_copy(void *dst, const void *src, size_t bytes, void *hip_stream)
{
    if (!dst || !src) return fail(SU3_EINVAL, "dst and src must not be NULL");
    if (bytes % 16) return fail(SU3_EINVAL, "bytes must be a multiple of 16");
    if (((uintptr_t)dst & 15u) || ((uintptr_t)src & 15u)) return fail(SU3_EINVAL, "buffers must be 16-byte aligned");
    if (bytes == 0) return SU3_OK;
    hipError_t e = su3hb::launch_copy(dst, src, bytes, (hipStream_t)hip_stream);
    if (e != hipSuccess) return hip_fail(e, "copy kernel");
    return SU3_OK;
}

}  // extern "C"
