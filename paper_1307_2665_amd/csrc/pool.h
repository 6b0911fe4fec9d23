// Device memory cache.  Builds allocate hundreds of megabytes per operator
// (DtN arenas, solution operators, pivots, descriptors); going to hipMalloc and
// hipFree for each of them costs milliseconds per build.  Blocks released here
// are kept per device and handed out again for requests of similar size.
#pragma once

#include <cstddef>

namespace hps {

// A block of at least `bytes` on the current device.  Falls back to
// hipMalloc, and on out-of-memory releases the cached blocks and retries.
void* pool_alloc(size_t bytes);
// Returns a block to the cache.  Callers release a block only after the work
// that used it has completed (every library call synchronizes its stream
// before returning).
void pool_release(void* p);
// Frees every cached block on every device; returns the bytes freed.
size_t pool_trim();
// Bytes currently cached (not in use) and in use.
void pool_stats(size_t* cached, size_t* in_use);

}  // namespace hps
