// server.hip -- continuous batching of many independent lattices on one GPU.
//
// The caller hands over one device buffer (the HBM budget).  Jobs are queued
// in submission order and admitted when a slot is free and a first-fit
// allocation of their footprint (links + scratch) succeeds in the arena.
// Every su3_server_step runs one sweep of every admitted job as 8 batched
// launches (one per pass, all jobs of a precision in the same launch),
// then retires the jobs that reached their sweep count: plaquette and
// counters are copied back and their arena block is freed.  A small 1-hit
// batch runs two lanes per link.  A job's links
// get exactly the per-link arithmetic of the single-lattice path and the
// same keyed random numbers, so its result does not depend on what else runs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <deque>
#include <map>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "runtime.h"

using namespace su3hb;

namespace {

constexpr size_t kAlign = 256;
constexpr int kGroups = 8;  // (precision 64/32) x (1-hit / general) x (single / double-layered torus)
constexpr long long kBatchLanes2Max = 32768;

size_t align_up(size_t a) { return (a + kAlign - 1) / kAlign * kAlign; }

struct Job {
    su3_job spec;
    Geom g;
    size_t link_bytes = 0, scratch_bytes = 0, off = 0;
    long long admit_step = 0;
    int state = SU3_JOB_QUEUED;
    int sweeps_done = 0;
    double plaq[3] = {0, 0, 0};
    uint64_t att = 0, acc = 0;
    int64_t bad_links = 0;
    int slot = -1;  // index into the pinned read-back buffers while retiring
};

struct Group {
    BatchJob *d_table = nullptr;  // device copy
    int njobs = 0, ntiles = 0;
};

}  // namespace

struct su3_server {
    unsigned char *arena = nullptr;
    size_t arena_bytes = 0, heap_begin = 0;
    int max_active = 0;
    hipStream_t stream = nullptr;
    std::map<size_t, size_t> free_blocks;  // offset -> size, coalesced
    size_t used = 0, peak = 0;
    std::unordered_map<int64_t, Job> jobs;
    std::deque<int64_t> queue;
    std::vector<int64_t> active;
    long long step = 0;
    int64_t next_id = 0;
    bool dirty = true;
    Group groups[kGroups];
    BatchJob *h_table = nullptr;       // pinned, kGroups * max_active entries
    double *h_sums = nullptr;          // pinned, 4 per retiring job
    unsigned long long *h_cnt = nullptr;  // pinned, 2 * kCounterSlots per retiring job

    bool alloc(size_t need, size_t *off)
    {
        for (auto it = free_blocks.begin(); it != free_blocks.end(); ++it) {
            if (it->second >= need) {
                *off = it->first;
                const size_t rest = it->second - need;
                const size_t at = it->first + need;
                free_blocks.erase(it);
                if (rest) free_blocks[at] = rest;
                used += need;
                peak = std::max(peak, used);
                return true;
            }
        }
        return false;
    }

    void release(size_t off, size_t size)
    {
        used -= size;
        auto it = free_blocks.emplace(off, size).first;
        auto next = std::next(it);
        if (next != free_blocks.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_blocks.erase(next);
        }
        if (it != free_blocks.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_blocks.erase(it);
            }
        }
    }
};

namespace {

int group_of(const su3_job &j)
{
    return (j.params.precision == 64 ? 0 : 4) + (j.params.nhit == 1 ? 0 : 2) + (j.params.nlat == 2 ? 1 : 0);
}

su3_status check_job(const su3_job *j)
{
    if (!j) return fail(SU3_EINVAL, "job is NULL");
    su3_status st = check_params(&j->params);
    if (st != SU3_OK) return st;
    if (!std::isfinite(j->beta) || !(j->beta > 0.0)) return fail(SU3_EINVAL, "job beta must be finite and > 0");
    if (j->nsweeps < 1) return fail(SU3_EINVAL, "job nsweeps must be >= 1");
    if (j->hot != 0 && j->hot != 1) return fail(SU3_EINVAL, "job hot must be 0 or 1");
    return SU3_OK;
}

su3_status build_tables(su3_server *s)
{
    std::vector<BatchJob> per[kGroups];
    for (int64_t id : s->active) {
        const Job &j = s->jobs[id];
        BatchJob b;
        b.links = s->arena + j.off;
        b.counters = (unsigned long long *)(s->arena + j.off + j.link_bytes + kOffCounters);
        b.g = j.g;
        b.beta = j.spec.beta;
        b.seed = j.spec.params.seed;
        b.sweep0 = 0;
        b.admit_step = j.admit_step;
        b.nhit = j.spec.params.nhit;
        b.lanes = 1;
        b.tile_begin = 0;
        per[group_of(j.spec)].push_back(b);
    }
    for (int gi = 0; gi < kGroups; ++gi) {
        Group &G = s->groups[gi];
        BatchJob *h = s->h_table + (size_t)gi * s->max_active;
        // a 1-hit batch of at most kBatchLanes2Max links per pass (fewer than
        // one wave per SIMD) is bound by the latency of one update: two lanes
        // per link shorten it (10^4 - 16^4 FP32: 12 % per sweep)
        long long links = 0;
        for (const BatchJob &b : per[gi]) links += (long long)b.g.nlat * b.g.Vh;
        const int lanes = (gi & 2) == 0 && links <= kBatchLanes2Max ? 2 : 1;
        int tiles = 0;
        for (size_t k = 0; k < per[gi].size(); ++k) {
            h[k] = per[gi][k];
            h[k].lanes = lanes;
            h[k].tile_begin = tiles;
            tiles += (int)(((long long)lanes * h[k].g.nlat * h[k].g.Vh + kPassBlock - 1) / kPassBlock);
        }
        G.d_table = (BatchJob *)s->arena + (size_t)gi * s->max_active;
        G.njobs = (int)per[gi].size();
        G.ntiles = tiles;
        if (G.njobs) {
            hipError_t e = hipMemcpyAsync(G.d_table, h, sizeof(BatchJob) * G.njobs, hipMemcpyHostToDevice, s->stream);
            if (e != hipSuccess) return hip_fail(e, "job table copy");
        }
    }
    s->dirty = false;
    return SU3_OK;
}

}  // namespace

extern "C" {

su3_status su3_server_create(void *d_arena, size_t arena_bytes, int32_t max_active, void *hip_stream,
                             su3_server **out)
{
    if (!out) return fail(SU3_EINVAL, "out is NULL");
    *out = nullptr;
    if (!d_arena || ((uintptr_t)d_arena & (kAlign - 1))) return fail(SU3_EINVAL, "arena must be 256-byte aligned");
    if (max_active < 1 || max_active > 4096) return fail(SU3_EINVAL, "max_active must be in [1, 4096]");
    const size_t table = align_up(sizeof(BatchJob) * (size_t)kGroups * (size_t)max_active);
    if (arena_bytes < table + kAlign) return fail(SU3_ENOSPC, "arena smaller than the job tables");
    su3_server *s = new (std::nothrow) su3_server();
    if (!s) return fail(SU3_EINVAL, "out of host memory");
    s->arena = (unsigned char *)d_arena;
    s->arena_bytes = arena_bytes;
    s->heap_begin = table;
    s->max_active = max_active;
    s->stream = (hipStream_t)hip_stream;
    s->free_blocks[table] = (arena_bytes - table) / kAlign * kAlign;
    hipError_t e = hipHostMalloc((void **)&s->h_table, sizeof(BatchJob) * (size_t)kGroups * max_active);
    if (e == hipSuccess) e = hipHostMalloc((void **)&s->h_sums, sizeof(double) * 4 * (size_t)max_active);
    if (e == hipSuccess)
        e = hipHostMalloc((void **)&s->h_cnt, sizeof(unsigned long long) * 2 * kCounterSlots * (size_t)max_active);
    if (e != hipSuccess) {
        if (s->h_table) (void)hipHostFree(s->h_table);
        if (s->h_sums) (void)hipHostFree(s->h_sums);
        delete s;
        return hip_fail(e, "pinned host buffers");
    }
    *out = s;
    return SU3_OK;
}

su3_status su3_server_destroy(su3_server *s)
{
    if (!s) return SU3_OK;
    (void)hipStreamSynchronize(s->stream);
    (void)hipHostFree(s->h_table);
    (void)hipHostFree(s->h_sums);
    (void)hipHostFree(s->h_cnt);
    delete s;
    return SU3_OK;
}

su3_status su3_server_submit(su3_server *s, const su3_job *job, int64_t *job_id)
{
    if (!s || !job_id) return fail(SU3_EINVAL, "server and job_id must not be NULL");
    su3_status st = check_job(job);
    if (st != SU3_OK) return st;
    Job j;
    j.spec = *job;
    j.g = make_geom(&job->params);
    j.link_bytes = align_up(link_bytes_of(&job->params, j.g));
    j.scratch_bytes = align_up(scratch_bytes_of(j.g));
    if (j.link_bytes + j.scratch_bytes > s->arena_bytes - s->heap_begin)
        return fail(SU3_ENOSPC, "job footprint exceeds the whole arena");
    *job_id = s->next_id++;
    s->jobs.emplace(*job_id, j);
    s->queue.push_back(*job_id);
    return SU3_OK;
}

}  // extern "C"

namespace {

// Admit, run k sweeps of every admitted job (k = min(max_sweeps, fewest
// remaining sweeps of an active job), so no job finishes inside the call),
// then retire with one synchronisation.
su3_status run_sweeps(su3_server *s, int32_t max_sweeps, int32_t *n_active, int32_t *n_queued, int32_t *n_finished)
{
    if (!s) return fail(SU3_EINVAL, "server is NULL");
    if (max_sweeps < 1) return fail(SU3_EINVAL, "max_sweeps must be >= 1");
    hipError_t e;
    // admission: first come, first served, while a slot and the footprint are free
    while (!s->queue.empty() && (int)s->active.size() < s->max_active) {
        Job &j = s->jobs[s->queue.front()];
        size_t off;
        if (!s->alloc(j.link_bytes + j.scratch_bytes, &off)) break;
        j.off = off;
        e = launch_start(j.spec.params.precision, s->arena + off, j.g, j.spec.hot, j.spec.params.seed, s->stream);
        if (e != hipSuccess) return hip_fail(e, "job start");
        e = launch_zero_u64((unsigned long long *)(s->arena + off + j.link_bytes + kOffCounters), 2 * kCounterSlots,
                            s->stream);
        if (e != hipSuccess) return hip_fail(e, "job counters");
        j.admit_step = s->step;
        j.state = SU3_JOB_ACTIVE;
        s->active.push_back(s->queue.front());
        s->queue.pop_front();
        s->dirty = true;
    }
    int finished = 0;
    if (!s->active.empty()) {
        if (s->dirty) {
            su3_status st = build_tables(s);
            if (st != SU3_OK) return st;
        }
        int k = max_sweeps;
        for (int64_t id : s->active) {
            const Job &j = s->jobs[id];
            k = std::min(k, j.spec.nsweeps - j.sweeps_done);
        }
        for (int sw = 0; sw < k; ++sw) {
            for (int mu = 0; mu < 4; ++mu)
                for (int par = 0; par < 2; ++par)
                    for (int gi = 0; gi < kGroups; ++gi) {
                        const Group &G = s->groups[gi];
                        if (!G.njobs) continue;
                        e = launch_update_batch(gi < 4 ? 64 : 32, (gi & 2) == 0, (gi & 1) != 0, G.d_table, G.njobs,
                                                G.ntiles, s->step, mu, par, s->stream);
                        if (e != hipSuccess) return hip_fail(e, "batched pass");
                    }
            s->step += 1;
        }
        std::vector<int64_t> done;
        for (int64_t id : s->active) {
            Job &j = s->jobs[id];
            j.sweeps_done += k;
            if (j.sweeps_done == j.spec.nsweeps) {
                j.slot = (int)done.size();
                done.push_back(id);
            }
        }
        for (int64_t id : done) {
            Job &j = s->jobs[id];
            unsigned char *scr = s->arena + j.off + j.link_bytes;
            e = launch_plaquette(j.spec.params.precision, s->arena + j.off, j.g, (double *)(scr + kOffPartials),
                                 (double *)(scr + kOffSums), s->stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(s->h_sums + 4 * j.slot, scr + kOffSums, sizeof(double) * 4, hipMemcpyDeviceToHost,
                                   s->stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(s->h_cnt + (size_t)2 * kCounterSlots * j.slot, scr + kOffCounters,
                                   sizeof(unsigned long long) * 2 * kCounterSlots, hipMemcpyDeviceToHost, s->stream);
            if (e != hipSuccess) return hip_fail(e, "job read-back");
        }
        e = hipStreamSynchronize(s->stream);
        if (e != hipSuccess) return hip_fail(e, "step sync");
        for (int64_t id : done) {
            Job &j = s->jobs[id];
            const double V = (double)j.g.Vh * 2.0;
            const double *sums = s->h_sums + 4 * j.slot;
            j.plaq[0] = sums[0] / (18.0 * V * j.g.nlat);
            for (int l = 0; l < j.g.nlat; ++l) j.plaq[1 + l] = sums[1 + l] / (18.0 * V);
            j.bad_links = (int64_t)sums[3];
            const unsigned long long *c = s->h_cnt + (size_t)2 * kCounterSlots * j.slot;
            for (int k = 0; k < kCounterSlots; ++k) {
                j.att += c[2 * k];
                j.acc += c[2 * k + 1];
            }
            j.state = SU3_JOB_DONE;
            s->release(j.off, j.link_bytes + j.scratch_bytes);
            s->active.erase(std::find(s->active.begin(), s->active.end(), id));
            s->dirty = true;
            ++finished;
        }
    }
    if (n_active) *n_active = (int32_t)s->active.size();
    if (n_queued) *n_queued = (int32_t)s->queue.size();
    if (n_finished) *n_finished = finished;
    return SU3_OK;
}

}  // namespace

extern "C" {

su3_status su3_server_step(su3_server *s, int32_t *n_active, int32_t *n_queued, int32_t *n_finished)
{
    return run_sweeps(s, 1, n_active, n_queued, n_finished);
}

su3_status su3_server_run(su3_server *s, int32_t max_sweeps, int32_t *n_active, int32_t *n_queued,
                          int32_t *n_finished)
{
    return run_sweeps(s, max_sweeps, n_active, n_queued, n_finished);
}

su3_status su3_server_poll(su3_server *s, int64_t job_id, su3_job_result *out)
{
    if (!s || !out) return fail(SU3_EINVAL, "server and out must not be NULL");
    auto it = s->jobs.find(job_id);
    if (it == s->jobs.end()) return fail(SU3_EINVAL, "unknown job id");
    const Job &j = it->second;
    out->state = j.state;
    out->sweeps_done = j.sweeps_done;
    for (int k = 0; k < 3; ++k) out->plaquette[k] = j.plaq[k];
    out->kp_attempts = j.att;
    out->kp_accepts = j.acc;
    out->bad_links = j.bad_links;
    return SU3_OK;
}

su3_status su3_server_release(su3_server *s, int64_t job_id)
{
    if (!s) return fail(SU3_EINVAL, "server is NULL");
    auto it = s->jobs.find(job_id);
    if (it == s->jobs.end()) return fail(SU3_EINVAL, "unknown job id");
    if (it->second.state != SU3_JOB_DONE) return fail(SU3_ESTATE, "only a finished job can be released");
    s->jobs.erase(it);
    return SU3_OK;
}

su3_status su3_server_get_links(su3_server *s, int64_t job_id, double *host, size_t n_doubles)
{
    if (!s || !host) return fail(SU3_EINVAL, "server and host must not be NULL");
    auto it = s->jobs.find(job_id);
    if (it == s->jobs.end()) return fail(SU3_EINVAL, "unknown job id");
    const Job &j = it->second;
    if (j.state != SU3_JOB_ACTIVE) return fail(SU3_ESTATE, "the job's links are on the device only while it is active");
    const size_t need = (size_t)144 * j.g.Vh * j.g.nlat;
    if (n_doubles != need) return fail(SU3_EINVAL, "n_doubles must be 72*V*nlat = " + std::to_string(need));
    std::vector<unsigned char> buf;
    try {
        buf.resize(link_bytes_of(&j.spec.params, j.g));
    } catch (...) {
        return fail(SU3_EINVAL, "out of host memory for the staging copy");
    }
    hipError_t e = hipMemcpyAsync(buf.data(), s->arena + j.off, buf.size(), hipMemcpyDeviceToHost, s->stream);
    if (e != hipSuccess) return hip_fail(e, "job link copy");
    e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hip_fail(e, "job link copy sync");
    unpack_links(j.spec.params.precision, j.g, buf.data(), host);
    return SU3_OK;
}

su3_status su3_server_stats(su3_server *s, size_t *arena_used, size_t *arena_peak, uint64_t *steps)
{
    if (!s) return fail(SU3_EINVAL, "server is NULL");
    if (arena_used) *arena_used = s->used;
    if (arena_peak) *arena_peak = s->peak;
    if (steps) *steps = (uint64_t)s->step;
    return SU3_OK;
}

}  // extern "C"
