// Batched rendering: cache of captured HIP graphs per batch signature.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "osog.h"

namespace osog {
struct BatchCache;
BatchCache* batch_cache_create();
void batch_cache_destroy(BatchCache* c);
size_t batch_workspace_bytes(const osog_context* ctx, const osog_frame* frames, int nf, int ppp);
hipError_t batch_render(osog_context* ctx, hipStream_t stream, const osog_frame* frames, int nf, int ppp,
                        int group, void* workspace, size_t ws_bytes, uint64_t* frame_done_ns,
                        std::string* err);
hipError_t batch_error_flag(void* workspace, int* flag);
}  // namespace osog
