// kdt_host.h -- host-side entry points shared by the C ABI translation units
// (single and batched builds in kdt_api.hip, the server in kdt_server.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <functional>

#include "../../include/kdt.h"
#include "kdt_plan.h"

namespace kdt {

// Enqueue every kernel of a planned call on `st`.  pts/tree/perm/dim/status
// as in kdt_build_ws for the concatenated trees; ws holds p.total bytes;
// h_tables is the plan's share tables in pinned host memory (needed when
// p.tables), read by an asynchronous copy on `st`.
kdt_status enqueue_plan(const Plan& p, const float* pts, float* tree, uint32_t* perm, uint8_t* dim,
                        uint32_t* status, char* ws, const void* h_tables, hipStream_t st);

// Kernels as the profiler (kdt_profile_collect) names them.
enum Kind { KIND_INIT, KIND_PREP, KIND_ROOT, KIND_PRESORT, KIND_LEVEL0, KIND_SELECT, KIND_PIVOT, KIND_PART,
            KIND_TAIL, KIND_WHOLE, KIND_TABLES, KIND_STATUS, KIND_BUCKET, KIND_WINDOW,
            KIND_IP_INIT, KIND_IP_SETUP, KIND_IP_BLOCK, KIND_IP_MIRROR, KIND_IP_GROUP, KIND_IP_DEEP, KIND_IP_PERM,
            KIND_COUNT };

// Enqueue one launch through fn on st; while profiling is enabled it is
// bracketed by two events and recorded under `kind` with `bytes` (moved by
// this implementation) and `mbytes` (moved by the paper's method for the
// work the launch completes).  Returns KDT_EDEVICE if the launch failed.
kdt_status launch_profiled(hipStream_t st, int kind, double bytes, double mbytes, const std::function<void()>& fn);

// Message of kdt_last_error() for the calling thread.
void set_last_error(const char* fmt, ...);

}  // namespace kdt
