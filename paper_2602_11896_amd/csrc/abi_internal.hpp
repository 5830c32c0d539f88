// Library-internal entry points of abi.cpp used by other C ABI sources.
#pragma once
#include <hip/hip_runtime.h>

#include <string>

#include "../../include/jtfs.h"

namespace jtfs {
// Records `msg` for jtfs_last_error and returns s.
jtfs_status report(jtfs_status s, const std::string& msg);
// Uploads the plan's tables to the current device if they are not there yet.
jtfs_status prepare_tables(jtfs_plan_t plan);
// Workspace bytes of one signal's forward segment (the largest over the batch).
size_t shared_forward_bytes(jtfs_plan_t plan);
// Forward of every signal in turn on `stream` in the one segment at ws; the tables must
// already be on the device (JTFS_ERR_ARG otherwise). Enqueues kernels only.
jtfs_status forward_prepared(jtfs_plan_t plan, const float* x, float* S, void* ws, hipStream_t stream);
}  // namespace jtfs
