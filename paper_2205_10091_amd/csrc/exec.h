// Internal interface of the device executor (shared by the single-plan path
// and the serving engine).
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "plan.h"

namespace tcx {

#define HIP_CHECK(x)                                                                     \
  do {                                                                                   \
    hipError_t e_ = (x);                                                                 \
    if (e_ != hipSuccess)                                                                \
      ::tcx::fail(TC_ERR_DEVICE, std::string(#x) + ": " + hipGetErrorString(e_));         \
  } while (0)

struct DeviceState {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  char* ws = nullptr;
  bool ws_owned = false;
  uint64_t ws_bytes = 0;
  WorkspaceLayout lay{};
  hipGraph_t graph[2] = {nullptr, nullptr};
  hipGraphExec_t exec[2] = {nullptr, nullptr};
  // the gradient graph captured for one set of caller buffers (parameters
  // read and E, dE/dtheta written in place), kept while the caller passes
  // the same three pointers
  hipGraph_t dgraph = nullptr;
  hipGraphExec_t dexec = nullptr;
  const void* dkey[3] = {nullptr, nullptr, nullptr};
  int n_cu = 256;
};

// One plan's launch, located in that plan's workspace.
struct SegRef {
  const Plan* plan;
  const char* ws;               // workspace base of this plan
  const WorkspaceLayout* lay;
  const Launch* launch;
  // caller buffers used in place of the workspace's own (null: the
  // workspace): the parameter vectors (batch x n_params floats), E's real
  // parts (batch doubles), the gradient (batch x n_params doubles)
  const float* params = nullptr;
  double* value_re = nullptr;
  double* grad = nullptr;
};

// Largest number of plans one merged launch carries (kernel-argument space).
constexpr int MAX_SEG = 24;

// Launch parts of a level: GEMM tiles (64 x 64 and wave tiles), gather
// items, 128 x 128 tiles with their split pass, row tiles, split sums with
// their reduction.
constexpr int PART_GEMM = 1, PART_GATHER = 2, PART_WIDE = 4, PART_ROWTILE = 8, PART_GSPLIT = 16;
constexpr int PART_ALL = PART_GEMM | PART_GATHER | PART_WIDE | PART_ROWTILE | PART_GSPLIT;

// Enqueue one launch of `kind` covering all `segs` (at most MAX_SEG, all of
// that kind) on `stream`; for levels, only the kernels named in `parts`
// (GEMM kernels first, then the gather kernels, in stream order: a second
// stream for the GEMM half measured slower once captured in a graph).
void launch_segments(int kind, const SegRef* segs, int nseg, hipStream_t stream, int n_cu,
                     int precision, int parts = PART_ALL);

// Asynchronous upload of a plan's tables and seeds into a workspace.
void upload_tables(const Plan& P, char* ws, const WorkspaceLayout& lay, hipStream_t stream);

int device_cu_count(int device);

}  // namespace tcx
