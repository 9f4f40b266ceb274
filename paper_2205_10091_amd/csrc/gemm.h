// LDS-tiled MFMA complex GEMM over gathered operands (wide tree nodes).
#pragma once
#include <hip/hip_runtime.h>

#include "ops.h"

namespace tcx {
// Launches the GEMM kernel for ops[0..n_ops) (tile work items); precision 0
// = FP32 MFMA, 1 = split-BF16 (hi+lo) MFMA with FP32 accumulation.
void launch_gemm(const DevOp* ops, uint32_t n_ops, const uint32_t* tabs, float2* arena,
                 uint64_t tiles, int precision, hipStream_t stream, int n_cu);
}  // namespace tcx
