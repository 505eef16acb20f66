// encode.hip -- placeholder until the GPU encoder lands.
#include <hip/hip_runtime.h>

#include "pivco_int.h"

namespace pivco {
pivco_status encode_stream(const void *, uint64_t, void *, uint64_t, uint64_t *,
                           const pivco_encode_opts *, void *, uint64_t, hipStream_t) {
  return PIVCO_E_UNSUPPORTED;
}
uint64_t encode_bound(uint64_t, const pivco_encode_opts *) { return 0; }
uint64_t encode_workspace(uint64_t, const pivco_encode_opts *) { return 0; }
}  // namespace pivco
