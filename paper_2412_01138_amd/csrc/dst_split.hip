// Per-axis DST-I products in split-bf16 with fp32 accumulation (placeholder
// until the split kernels land).
#include "pe_internal.h"

namespace pe {

pe_status dst_fields_split(pe_grid g, int64_t count, float *buf0, float *buf1, float **result,
                           hipStream_t st) {
  (void)g; (void)count; (void)buf0; (void)buf1; (void)result; (void)st;
  return set_error(PE_E_UNSUPPORTED, "split-bf16 transforms are not built yet");
}

}  // namespace pe
