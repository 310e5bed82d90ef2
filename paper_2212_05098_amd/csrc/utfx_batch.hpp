// utfx_batch.hpp -- batched path (placeholder until the persistent kernel lands).
#pragma once
#include <hip/hip_runtime.h>
#include <stdio.h>
#include "utfx.h"

struct BatchWs {
  void* mem = nullptr;
};
inline hipError_t batch_ws_init(BatchWs&) { return hipSuccess; }
inline void batch_ws_free(BatchWs&) {}
inline utfx_status batch_run(BatchWs&, hipStream_t, int, uint32_t, uint32_t, const uint8_t*, uint8_t*,
                             const utfx_item*, uint32_t, uint64_t, utfx_result*, char* err, size_t errlen) {
  snprintf(err, errlen, "batched path not available in this build");
  return UTFX_E_INVALID_ARG;
}
