// Entry points not built yet.
#include <hip/hip_runtime.h>

#include "batch.h"
#include "osog.h"
#include "osog_internal.h"

namespace osog {
struct BatchCache {};
BatchCache* batch_cache_create() { return new BatchCache(); }
void batch_cache_destroy(BatchCache* c) { delete c; }
}  // namespace osog

extern "C" {
osog_status osog_batch_workspace_size(osog_context*, const osog_frame*, int32_t, int32_t, size_t*) {
  osog::set_error("osog_batch_workspace_size: not built");
  return OSOG_ERR_UNSUPPORTED;
}
osog_status osog_batch_render(osog_context*, void*, const osog_frame*, int32_t, void*, size_t,
                              uint64_t*) {
  osog::set_error("osog_batch_render: not built");
  return OSOG_ERR_UNSUPPORTED;
}
}
