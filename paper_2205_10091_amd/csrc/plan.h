// Host-side plan: everything the device executor needs, as flat tables.
#pragma once

#include <atomic>
#include <cstdint>
#include <vector>

#include "internal.h"
#include "ops.h"

namespace tcx {

enum LaunchKind : int32_t {
  L_LEAF = 0,   // materialise leaf tensors from parameters
  L_LEVEL = 1,  // one contraction level: MFMA GEMM tiles + gather contractions
  L_ROOT = 4,   // FP64 weighted sum of the term roots
  L_GRAD = 5,   // FP64 leaf-gradient reduction
  L_TERM = 6,   // one workgroup per term runs the term's nodes of a run of steps
  L_QGT = 7     // geometric tensor from the per-use values and adjoint sums
};
// kernel kinds reported by profiling: a level's GEMM tiles (64 x 64 and
// wave tiles), gathers, and 128 x 128 GEMM tiles
constexpr int32_t PROF_GEMM = 2, PROF_GATHER = 3, PROF_WIDE = 7, PROF_ROWTILE = 8,
                  PROF_GSPLIT = 9;

constexpr uint64_t NO_ITEMS = ~uint64_t(0);
// levels with at most this many gather items get a per-item op index table
constexpr uint64_t ITEM_TABLE_MAX = uint64_t(1) << 18;
// all per-item tables of a plan together (levels past it search instead)
constexpr uint64_t ITEM_TABLES_TOTAL_MAX = uint64_t(1) << 24;
// automatic term launches: at most this many gather items per term and step
// (two per thread of the 1024-thread workgroup)
constexpr uint64_t TERM_MODE_MAX_ITEMS = 2048;
// ... and at most this many k-steps per lane in any of its sums
constexpr uint32_t TERM_MODE_MAX_KSTEPS = 8;
// lanes a gather node may spread its k-split over: a level launch, a term's
// workgroup
constexpr uint64_t LEVEL_LANES = 65536, TERM_LANES = 1024;
// level launches whose gather ops would take more items than this (about
// two passes of the chip at 7 wavefronts per SIMD) keep at least 8 k-steps
// per lane instead of 4 (measured on the 20-qubit chain's reverse sweep:
// 257 against 264 us per evaluation)
constexpr uint64_t LEVEL_SHORT_SPLIT_ITEMS = 600000;
// levels with at most this many wave tiles get a per-tile op index table
constexpr uint64_t WAVE_TABLE_MAX = uint64_t(1) << 20;
// batched nodes below the GEMM rule take masked wave tiles from this many rows
constexpr uint32_t SMALL_WAVE_MIN_ROWS = 64;
// row tiles: a workgroup stages whole batch rows of both operands in LDS,
// at most this many complex elements (16 KB)
constexpr uint32_t ROW_TILE_ELEMS = 2048;
// ... and a workgroup stages up to this many rows' operands at once, at
// most ROW_TILE_LDS complex elements (16 KB; measured on the 1024-row VQE
// sweep, 128 rows in 32 KB ran the row tiles 7 % slower)
constexpr uint32_t ROW_TILE_ROWS = 64, ROW_TILE_LDS = 2048;
// index tables of one plan (uint32 entries)
constexpr uint64_t TABLE_MAX_ENTRIES = uint64_t(1) << 27;

struct Launch {
  int32_t kind;
  int32_t step = 0;               // timeline step (the first one of a term launch)
  uint32_t begin = 0, end = 0;    // gather ops in Plan::ops
  uint64_t work = 0;              // gather work items / leaf, root, grad items
  uint32_t xbegin = 0;            // L_LEVEL: split gather ops are [xbegin, end)
  uint64_t xwork = 0;             // their work items (a space of their own)
  uint32_t rbegin = 0, rend = 0;  // L_LEVEL: row-tile ops (batched small nodes)
  uint64_t rblocks = 0;           // their workgroups
  uint32_t gbegin = 0, gend = 0;  // GEMM ops in 64 x 64 tiles, in Plan::ops
  uint64_t tiles = 0;             // 64 x 64 GEMM tiles
  uint32_t wbegin = 0, wend = 0;  // GEMM ops in wave tiles, in Plan::ops
  uint64_t wtiles = 0;            // wave tiles
  uint32_t hbegin = 0, hend = 0;  // GEMM ops in 128 x 128 tiles (dense operands)
  uint64_t htiles = 0;            // 128 x 128 tiles
  uint64_t wchunks = 0;           // split BF16: operand chunks of the split pass
  uint32_t sbegin = 0, send = 0;  // split-K output tiles, in Plan::split_units
  uint32_t gsbegin = 0, gsend = 0;  // split gather outputs (256 a unit), in Plan::gsplit_units
  uint64_t item_begin = NO_ITEMS; // per-item op index table in Plan::item_op
  uint64_t wunit_begin = NO_ITEMS;  // per-wave-tile op index table in Plan::item_op
  uint64_t rtunit_begin = NO_ITEMS; // per-row-tile-workgroup op index table in Plan::item_op
  bool with_leaves = false;       // L_TERM: materialise the leaves first
  bool deep_gather = false;       // L_LEVEL: gather items with long sums (deep unroll)
  // resident term launches: 1 the forward pass alone (calls without the
  // gradient), 2 the forward pass and reverse sweep (calls with it), 3 a
  // run of light steps of the automatic mode (calls with or without it)
  int32_t resident = 0;
  double flops = 0;               // algorithmic flops (8 per complex MAC)
  double bytes = 0;               // algorithmic bytes: operands read + results written
  double gemm_flops = 0;          // the part of flops / bytes in GEMM tiles
  double gemm_bytes = 0;
  double wide_flops = 0;          // ... of which in 128 x 128 tiles
  double wide_bytes = 0;
  double rt_flops = 0;            // the part in row tiles
  double rt_bytes = 0;
  double gs_flops = 0;            // the part in split sums
  double gs_bytes = 0;
};

struct DeviceState;  // defined by the executor

struct Plan {
  // options
  int32_t precision = 0, batch = 1, want_grad = 0, device = 0;
  uint64_t budget = 0;
  void* user_stream = nullptr;
  int32_t n_params = 0, n_terms = 0;
  // nodes with K >= gemm_min_k, M, N >= gemm_min_mn and at least
  // gemm_min_macs complex multiply-adds (over their batch rows) go to the
  // MFMA GEMM; smaller ones finish sooner on the gather path
  int32_t gemm_min_k = 8, gemm_min_mn = 16;
  uint64_t gemm_min_macs = uint64_t(1) << 20;
  // GEMM nodes with M, N >= 64 and K >= 16 use 64 x 64 LDS tiles; the
  // narrower ones run as one-wavefront MFMA tiles
  int32_t block_tile_min_mn = 64, block_tile_min_k = 16;
  // 128 x 128 tiles for GEMM nodes with dense operands: 0 never, 1 when
  // they give at least one tile per CU, 2 always
  int32_t wide_tiles = 1;
  // execution: 0 = automatic, 1 = level-synchronous launches, 2 = term
  // mode (all nodes as gathers), 3 = resident term launches
  int32_t exec_mode = 0;
  // complex elements of one workgroup's LDS arena for resident term
  // launches (set by the executor from the device; 0 = none)
  uint32_t lds_elems = 0;
  bool resident = false;    // resident term launches (batch 1, gathers only)
  bool resident_runs = false;  // automatic mode: forward light runs as resident term launches
  bool term_mode = false;   // some steps run in term launches
  int32_t exec_used = 1;    // 1 level launches only, 2 term launches only, 3 both,
                            // 4 resident term launches
  // checkpoint segment length: 0 = only when the budget requires it,
  // >= 2 = always with that length, -1 = never
  int32_t checkpoint = 0;
  int32_t checkpoint_used = 0;
  // terms run in this many groups, one after another (1 = all together)
  int32_t term_groups = 1;
  // geometric tensor: batch rows are the ket's gate uses, all reading one
  // parameter vector
  int32_t qgt = 0;
  int32_t qgt_rows = 0;
  uint32_t param_stride() const { return qgt ? 0u : (uint32_t)n_params; }

  // tables uploaded once
  std::vector<DevOp> ops;
  std::vector<uint32_t> tabs;
  std::vector<uint32_t> item_op;      // gather item -> op index, per small level
  std::vector<DevLeaf> leaves;
  std::vector<float> ftab;
  std::vector<DevGradUse> uses;       // sorted by slot
  std::vector<uint32_t> slot_begin;   // n_params + 1
  std::vector<DevRoot> roots;
  std::vector<DevTerm> terms;         // term launches: each term's leaves
  std::vector<DevGroup> groups;       // term launches: a term's nodes at one step
  std::vector<DevRange> ranges;       // term launches: each term's groups, per launch
  std::vector<DevROp> rops;           // resident term launches: the nodes (groups index them)
  std::vector<DevSplitUnit> split_units;  // split-K output tiles, per level
  std::vector<DevSplitUnit> gsplit_units; // split gather outputs, per level
  std::vector<float> seeds;           // (re, im) per term, arena offset 0
  std::vector<uint32_t> qslot_begin;  // qgt: n_params + 1, rows of each slot in qrows
  std::vector<uint32_t> qrows;        // qgt: batch rows (ket gate uses) by slot
  uint64_t leaf_work = 0;

  std::vector<Launch> fwd;            // leaf, levels, root
  std::vector<Launch> bwd;            // adjoint levels, grad
  uint64_t arena_elems = 0;           // complex64 elements
  uint64_t split_floats = 0;          // split-K partial tiles of the largest level
  uint64_t peak_tensor_elems = 0;

  tc_plan_info info{};

  // device side
  DeviceState* dev = nullptr;
  std::atomic<int> busy{0};
};

void build_plan(Plan& plan, const Network& net, const Path& path);

// The launches of one call in timeline order: the forward list alone, or
// the forward and reverse lists merged by step (with term groups each
// group's reverse sweep runs before the next group's forward pass).
std::vector<const Launch*> launch_order(const Plan& p, bool with_grad);

// Byte layout of the workspace: [tables][params][values][grad][arena]
struct WorkspaceLayout {
  uint64_t ops, tabs, item_op, leaves, ftab, uses, slot_begin, roots, terms, groups, ranges, rops;
  uint64_t split, sunits, gsunits;  // split-K partials (float), units to reduce
  uint64_t qslot, qrows;             // qgt: slot -> rows tables
  uint64_t params, value, grad, qgt, arena, total;
};
WorkspaceLayout workspace_layout(const Plan& p);

}  // namespace tcx
