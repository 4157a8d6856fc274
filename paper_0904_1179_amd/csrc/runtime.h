// runtime.h -- host-side helpers shared by the C-ABI entry points (api.hip)
// and the job server (server.hip): the layout code of layout.h, the kernel
// launchers of launch.h and HIP error reporting.
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/su3hb.h"
#include "launch.h"
#include "layout.h"

namespace su3hb {

// record a HIP error as the calling thread's last error; returns SU3_EDEVICE
su3_status hip_fail(hipError_t e, const char *where);

}  // namespace su3hb
