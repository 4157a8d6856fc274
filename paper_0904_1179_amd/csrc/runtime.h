// runtime.h -- host-side helpers shared by the C-ABI entry points (api.hip)
// and the job server (server.hip): parameter validation, geometry, buffer
// sizes, error reporting.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "../../include/su3hb.h"
#include "launch.h"

namespace su3hb {

// record `msg` as the thread's last error and return `s`
su3_status fail(su3_status s, const std::string &msg);
su3_status hip_fail(hipError_t e, const char *where);
const char *last_error();

// scratch layout (bytes): [0, 16*kCounterSlots) heat-bath counter slots (pairs
// of u64 attempts, accepts); then 256 bytes of plaquette sums; then the
// per-sweep plaquette sums of su3_sweep_measure (kMeasureChunk sweeps x 4
// doubles); then the plaquette partials
constexpr size_t kOffCounters = 0;
constexpr size_t kOffSums = 16 * (size_t)kCounterSlots;
constexpr int kMeasureChunk = 256;
constexpr size_t kOffMeasure = kOffSums + 256;
constexpr size_t kOffPartials = kOffMeasure + 32 * (size_t)kMeasureChunk;

su3_status check_params(const su3_params *p);
void pick_domains(const int32_t L[4], int nlat, int &w1, int &w2);
Geom make_geom(const su3_params *p);
size_t link_bytes_of(const su3_params *p, const Geom &g);
size_t scratch_bytes_of(const Geom &g);

}  // namespace su3hb
