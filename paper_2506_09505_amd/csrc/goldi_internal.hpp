// Library-internal entry points shared between translation units of
// libgoldi.so (not part of the C ABI; hidden from the exported symbols).
#pragma once
#include <hip/hip_runtime.h>

#include "goldi.h"

#define GOLDI_HIDDEN __attribute__((visibility("hidden")))

// Enqueues the batched build of `trees` on `stream` (no graph capture); the
// trees were validated by the caller.
GOLDI_HIDDEN int goldi_internal_enqueue_many(const goldi_tree_t *trees, size_t n_trees, uint32_t *dev_status,
                                             hipStream_t stream);

// GOLDI_OK if [p, p + bytes) lies inside one device allocation of the
// current device, else GOLDI_EINVAL with a message for goldi_last_error().
GOLDI_HIDDEN int goldi_internal_check_device_range(const void *p, size_t bytes, const char *what);
