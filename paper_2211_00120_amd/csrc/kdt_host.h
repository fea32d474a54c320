// kdt_host.h -- host-side entry points shared by the C ABI translation units
// (single and batched builds in kdt_api.hip, the server in kdt_server.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/kdt.h"
#include "kdt_plan.h"

namespace kdt {

// Enqueue every kernel of a planned call on `st`.  pts/tree/perm/dim/status
// as in kdt_build_ws for the concatenated trees; ws holds p.total bytes;
// h_tables is the plan's share tables in pinned host memory (needed when
// p.tables), read by an asynchronous copy on `st`.
kdt_status enqueue_plan(const Plan& p, const float* pts, float* tree, uint32_t* perm, uint8_t* dim,
                        uint32_t* status, char* ws, const void* h_tables, hipStream_t st);

// Message of kdt_last_error() for the calling thread.
void set_last_error(const char* fmt, ...);

}  // namespace kdt
