// LDS-tiled MFMA complex GEMM for wide tree nodes (not yet enabled by the
// planner).
#include "gemm.h"
#include "internal.h"

namespace tcx {
void launch_gemm(const DevOp*, uint32_t, const uint32_t*, float2*, uint64_t, int,
                 hipStream_t) {
  fail(TC_ERR_UNSUPPORTED, "GEMM path not built");
}
}  // namespace tcx
