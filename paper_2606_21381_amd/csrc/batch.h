// Batched persistent rendering: cache of captured HIP graphs per batch signature.
#pragma once

namespace osog {
struct BatchCache;
BatchCache* batch_cache_create();
void batch_cache_destroy(BatchCache* c);
}  // namespace osog
