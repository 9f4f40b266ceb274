// Device executor: kernels, workspace binding, HIP-graph capture, and the
// plan / contraction entry points of the C ABI.
//
// Paper, section "Tensor network engine" and the workflow figure: after the
// path is fixed, the contraction is a sequence of pairwise tensor
// contractions run by the backend; JIT (section "Gradients, optimization and
// variational algorithms") compiles that sequence once and replays it.
// Here the sequence is level-ordered launches of hand-written kernels,
// captured once into a HIP graph and replayed per call with new
// parameters.
//
// Every kernel takes a small table of segments by value: one segment per
// plan, each pointing at that plan's own tables and workspace.  A single
// plan is one segment; the serving engine merges the current launch of
// every live request into one launch per kernel class.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "exec.h"
#include "gates.h"
#include "gemm_tile.h"

struct tc_network;
struct tc_path;

namespace tcx {
const Network& network_of(const tc_network* n);
const Path& path_of(const tc_path* p);
}  // namespace tcx

struct tc_plan {
  tcx::Plan p;
};

namespace tcx {

// ------------------------------------------------------------------ segments

struct LeafSeg {
  const DevLeaf* leaves;
  const uint32_t* item_leaf;  // leaf entry -> leaf index, or null (search)
  const float* ftab;
  const float* params;
  float2* arena;
  uint64_t start;  // first work item of this segment in the launch
  uint32_t n;
  uint32_t param_stride;  // floats between rows' parameter vectors (0: shared)
};
struct LeafArgs {
  LeafSeg seg[MAX_SEG];
  uint32_t nseg;
  uint64_t total;
};

struct LevelSeg {
  const DevOp* gemm_ops;
  const DevOp* wave_ops;
  const uint32_t* wave_unit_op;  // wave tile -> op index, or null (search)
  const DevOp* gc_ops;
  const uint32_t* tab;
  const uint32_t* item_op;  // gather wavefront (64 items) -> op index, or null (search)
  float2* arena;
  SplitK split;             // split-K partial tiles
  const DevSplitUnit* sunits;  // split-K output tiles of this level
  uint64_t split_start;     // first split-K output tile of this segment
  uint32_t n_split;
  const DevOp* wide_ops;    // GEMM ops in 128 x 128 tiles
  uint64_t wide_start;      // first wide tile of this segment
  uint32_t n_wide;
  const DevOp* rt_ops;      // row-tile ops (batched small nodes)
  const uint32_t* rt_unit_op;  // row-tile workgroup -> op index, or null (search)
  uint64_t rt_start;        // first row-tile workgroup of this segment
  uint32_t n_rt;
  const DevOp* gs_ops;      // split gather ops (V == 1), in their own work space
  uint64_t gs_start;        // first split gather item of this segment
  uint32_t n_gs;
  const DevSplitUnit* gsunits;  // their outputs, 256 a unit (op relative to gs_ops)
  uint64_t gsplit_start;
  uint32_t n_gsplit;
  uint64_t gemm_start;  // first GEMM tile of this segment
  uint64_t wave_start;  // first wave tile of this segment
  uint64_t gc_start;    // first gather item (a multiple of 64)
  uint32_t n_gemm;
  uint32_t n_wave;
  uint32_t n_gc;
};
struct LevelArgs {
  LevelSeg seg[MAX_SEG];
  uint32_t nseg;
  uint32_t tile_blocks;  // k_gemm blocks [0, tile_blocks) run 64 x 64 tiles
  uint64_t gemm_tiles;
  uint64_t wave_tiles;
  uint64_t split_units;  // split-K output tiles over all segments
  uint64_t gsplit_units;  // split gather units over all segments
  uint64_t wide_tiles;    // 128 x 128 tiles over all segments
  uint64_t wide_chunks;   // split BF16: operand chunks of the split pass
  uint64_t rt_blocks;     // row-tile workgroups over all segments
  uint64_t gc_work;
  uint64_t gs_work;       // split gather items over all segments
  int32_t xcd_order;      // gather chunks in XCD order (plans at batch 1)
};

struct RootSeg {
  const DevRoot* roots;
  const float2* arena;
  double* value;
  double* value_re;  // also E's real part here, one double per row (or null)
  uint64_t start;  // first wavefront (batch row) of this segment
  uint32_t n_terms;
  uint32_t batch;
};
struct RootArgs {
  RootSeg seg[MAX_SEG];
  uint32_t nseg;
  uint64_t total;  // wavefronts
};

struct TermArgs {
  const DevTerm* terms;
  const DevRange* ranges;     // this launch's range of each term
  const DevGroup* groups;
  const DevOp* ops;
  const uint32_t* tab;
  const uint32_t* item_op;    // per-item op tables (groups hold their base)
  const uint32_t* item_leaf;  // leaf entry -> leaf index, or null (search)
  const DevLeaf* leaves;
  const float* ftab;
  const float* params;
  float2* arena;
  uint32_t param_stride;      // floats between rows' parameter vectors
  int32_t with_leaves;        // materialise the term's leaves first
  const DevROp* rops;         // resident launches: the node records
};

struct GradSeg {
  const DevGradUse* uses;
  const uint32_t* slot_begin;
  const DevLeaf* leaves;
  const float* params;
  const float2* arena;
  double* grad;
  uint64_t start;  // first wavefront (row, slot) of this segment
  int32_t n_params;
  uint32_t param_stride;  // floats between rows' parameter vectors
  int32_t cplx;           // 1: complex sums, (re, im) per (row, slot)
};

// Geometric tensor: G[i][j] = sum over the rows u of slot j of
// S[u][i] - conj(v_i) v_j with v_j = sum over the rows u of slot j of
// value[u] (value[u] = <psi|d_u psi>, S[u][i] = <d_i psi|d_u psi>).
struct QgtArgs {
  const double* value;       // (re, im) per row
  const double* sums;        // (re, im) per (row, slot)
  const uint32_t* slot_begin;  // n_params + 1
  const uint32_t* rows;        // rows by slot
  double* out;                 // (re, im) per (i, j)
  int32_t n_params;
};
struct GradArgs {
  GradSeg seg[MAX_SEG];
  uint32_t nseg;
  uint64_t total;  // wavefronts
};

// last segment whose start is <= w (an empty segment shares the next start)
template <typename A, typename F>
__device__ __forceinline__ uint32_t find_seg(const A& args, uint64_t w, F start) {
  uint32_t s = 0;
  for (uint32_t i = 1; i < args.nseg; ++i)
    if (start(args.seg[i]) <= w) s = i;
  return s;
}

// ------------------------------------------------------------------ kernels

template <typename T>
__device__ __forceinline__ uint32_t find_item(const T* __restrict__ items, uint32_t n,
                                              uint64_t w) {
  // largest i with items[i].work0 <= w (items sorted by work0, items[0].work0 == 0)
  uint32_t lo = 0, hi = n;
  while (hi - lo > 1) {
    uint32_t mid = (lo + hi) >> 1;
    if (items[mid].work0 <= w)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

__device__ __forceinline__ void cfma(c32& acc, float2 a, float2 b) {
  acc.re = fmaf(a.x, b.x, acc.re);
  acc.re = fmaf(-a.y, b.y, acc.re);
  acc.im = fmaf(a.x, b.y, acc.im);
  acc.im = fmaf(a.y, b.x, acc.im);
}

// acc[j] += sum over k = kb + sub, kb + sub + S, ... < K of
// A[ak(k)] * B[bk(k) + bn[j]], j < V, accumulated in increasing k.  U steps
// are issued together so that their table and operand loads overlap instead
// of forming one dependent chain per step.  Level launches (DEEP = false)
// take U small (2 steps at V = 1): the gather kernel then fits 72 VGPRs and
// 7 wavefronts per SIMD, and more items in flight beat deeper unrolling
// (20-qubit VQE chain, energy + gradient: 365 us at U = 8 / 4 / 2 and 5
// waves, 338 us at 4 / 2 / 1 and 6, 325 us at 2 / 1 / 1 and 7; 8 waves
// spill).  Term launches have one workgroup per term, so their items gain
// from the deeper unroll (DEEP = true: 8 / 4 / 2).
template <int V, bool TABLES, bool DEEP = false>
__device__ __forceinline__ void gather_dot(c32 (&acc)[4], const float2* __restrict__ A,
                                           const float2* __restrict__ Bp,
                                           const uint32_t* __restrict__ tab, uint32_t ak,
                                           uint32_t bk,
                                           const uint32_t (&bn)[4], uint32_t sub, uint32_t S,
                                           uint32_t kb, uint32_t K) {
  constexpr int U = DEEP ? (V == 4 ? 2 : (V == 2 ? 4 : 8)) : (V == 4 ? 1 : (V == 2 ? 1 : 2));
  uint32_t k = kb + sub;
  for (; k + (U - 1) * S < K; k += U * S) {
    uint32_t ia[U], ib[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      ia[u] = ixt<TABLES>(tab, ak, k + u * S);
      ib[u] = ixt<TABLES>(tab, bk, k + u * S);
    }
    float2 av[U], bv[U][V];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      av[u] = A[ia[u]];
#pragma unroll
      for (int j = 0; j < V; ++j) bv[u][j] = Bp[ib[u] + bn[j]];
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int j = 0; j < V; ++j) cfma(acc[j], av[u], bv[u][j]);
  }
  for (; k < K; k += S) {
    const float2 av = A[ixt<TABLES>(tab, ak, k)];
    const float2* __restrict__ bb = Bp + ixt<TABLES>(tab, bk, k);
#pragma unroll
    for (int j = 0; j < V; ++j) cfma(acc[j], av, bb[bn[j]]);
  }
}

// Leaf work item w (row-major over the leaf's rows and entries): one entry
// of one leaf tensor for one batch row.
__device__ __forceinline__ void leaf_item(const DevLeaf& L, uint64_t w,
                                          const float* __restrict__ params, uint32_t param_stride,
                                          const float* __restrict__ ftab,
                                          float2* __restrict__ arena) {
  const uint64_t l = w - L.work0;
  const int e = (int)(l & ((1u << L.rank) - 1));
  const uint64_t r = l >> L.rank;
  const float* pr = params + r * (uint64_t)param_stride;
  const float t0 = L.param[0] >= 0 ? pr[L.param[0]] : L.fixed[0];
  const float t1 = L.param[1] >= 0 ? pr[L.param[1]] : L.fixed[1];
  // (geometric tensor plans: the row of a gate use holds its derivative)
  const c32 v = (int64_t)r == L.dsel[0]   ? dleaf_entry(L, e, t0, t1, 0)
                : (int64_t)r == L.dsel[1] ? dleaf_entry(L, e, t0, t1, 1)
                                          : leaf_entry(L, e, t0, t1, ftab);
  arena[L.out + (r << L.rank) + e] = make_float2(v.re, v.im);
}

// Materialise every leaf tensor (gates, boundary vectors, Pauli matrices)
// for every batch row from the parameter vectors.
__global__ void __launch_bounds__(256) k_leaf(LeafArgs a) {
  // contiguous chunk per block; the leaf index only walks forward
  const uint64_t chunk = (((a.total + gridDim.x - 1) / gridDim.x) + 255) & ~uint64_t(255);
  const uint64_t begin = (uint64_t)blockIdx.x * chunk;
  const uint64_t end = begin + chunk < a.total ? begin + chunk : a.total;
  uint32_t si = 0xffffffffu, li = 0xffffffffu;
  for (uint64_t w = begin + threadIdx.x; w < end; w += blockDim.x) {
    if (si == 0xffffffffu) {
      si = find_seg(a, w, [](const LeafSeg& s) { return s.start; });
    } else {
      while (si + 1 < a.nseg && a.seg[si + 1].start <= w) {
        ++si;
        li = 0xffffffffu;
      }
    }
    const LeafSeg& S = a.seg[si];
    const uint64_t ws = w - S.start;
    if (S.item_leaf)
      li = S.item_leaf[ws];
    else if (li == 0xffffffffu)
      li = find_item(S.leaves, S.n, ws);
    else
      while (li + 1 < S.n && S.leaves[li + 1].work0 <= ws) ++li;
    leaf_item(S.leaves[li], ws, S.params, S.param_stride, S.ftab, S.arena);
  }
}

// One contraction level is two kernels over the same arguments: k_gemm runs
// the level's GEMM nodes as 64 x 64 MFMA tiles and wave tiles, k_gather its
// other nodes.  They touch disjoint outputs, so they may run concurrently,
// and each keeps its own register budget (the GEMM tiles' accumulators
// would otherwise cap the gather waves' occupancy).  FP32 is held to 128
// registers for 4 waves per SIMD: the batched per-row wave tiles are
// latency bound, and 4 waves beat 3 without the cap (22.5 against 23.2 ms
// for the 1024-row VQE sweep) despite a 12-byte spill.
// Block b of a grid of n runs on XCD b mod 8 (round-robin dispatch); the
// logical block that gives XCD x a contiguous range of [0, n), so that
// neighbouring work (items of one op, which read the same operands) shares
// one XCD's L2.  A bijection on [0, n) for any n; blocks at or past n keep
// their number.  (The 64 x 64 GEMM tiles measured no better in this order
// on the 6x6 depth-8 grid.)
__device__ __forceinline__ uint64_t xcd_block(uint64_t n) {
  const uint64_t b = blockIdx.x;
  if (b >= n) return b;
  const uint64_t x = b & 7u, slot = b >> 3, q = n >> 3, r = n & 7u;
  return x * q + (x < r ? x : r) + slot;
}

template <int PREC>
__global__ void __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(PREC == TC_PREC_C64 ? 4 : 2))) k_gemm(LevelArgs a) {
  if (blockIdx.x >= a.tile_blocks) {
    // wave tiles: one unit per wavefront, grid-stride over the units
    const int lane = threadIdx.x & 63;
    const uint64_t waves = (uint64_t)(gridDim.x - a.tile_blocks) * (blockDim.x >> 6);
    for (uint64_t u = (uint64_t)(blockIdx.x - a.tile_blocks) * (blockDim.x >> 6) +
                      (threadIdx.x >> 6);
         u < a.wave_tiles; u += waves) {
      const LevelSeg& S = a.seg[find_seg(a, u, [](const LevelSeg& s) { return s.wave_start; })];
      const uint64_t lu = u - S.wave_start;
      // the unit is the same for the whole wavefront: its op index is uniform
      const uint32_t oi = __builtin_amdgcn_readfirstlane(
          S.wave_unit_op ? S.wave_unit_op[lu] : find_item(S.wave_ops, S.n_wave, lu));
      const DevOp op = S.wave_ops[oi];
      const uint32_t shape = op_has_tables(op) ? (((op.flags >> 12) & 3u) | 4u)
                             : (op.flags & OPF_AVEC) ? (((op.flags >> 12) & 3u) | 8u)
                                                     : ((op.flags >> 12) & 3u);
      switch (shape) {
        case 8: wave_tile_f32<1, 1, false, true>(op, lu, S.tab, S.arena, lane, S.split); break;
        case 9: wave_tile_f32<2, 1, false, true>(op, lu, S.tab, S.arena, lane, S.split); break;
        case 10: wave_tile_f32<1, 2, false, true>(op, lu, S.tab, S.arena, lane, S.split); break;
        case 11: wave_tile_f32<2, 2, false, true>(op, lu, S.tab, S.arena, lane, S.split); break;
        case 0: wave_tile_f32<1, 1, false>(op, lu, S.tab, S.arena, lane, S.split); break;
        case 1: wave_tile_f32<2, 1, false>(op, lu, S.tab, S.arena, lane, S.split); break;
        case 2: wave_tile_f32<1, 2, false>(op, lu, S.tab, S.arena, lane, S.split); break;
        case 3: wave_tile_f32<2, 2, false>(op, lu, S.tab, S.arena, lane, S.split); break;
        case 4: wave_tile_f32<1, 1, true>(op, lu, S.tab, S.arena, lane, S.split); break;
        case 5: wave_tile_f32<2, 1, true>(op, lu, S.tab, S.arena, lane, S.split); break;
        case 6: wave_tile_f32<1, 2, true>(op, lu, S.tab, S.arena, lane, S.split); break;
        default: wave_tile_f32<2, 2, true>(op, lu, S.tab, S.arena, lane, S.split); break;
      }
    }
    return;
  }
  if constexpr (PREC == TC_PREC_BF16X3) {
    __shared__ SmemBF16 smem;
    for (uint64_t tile = blockIdx.x; tile < a.gemm_tiles; tile += a.tile_blocks) {
      const LevelSeg& S =
          a.seg[find_seg(a, tile, [](const LevelSeg& s) { return s.gemm_start; })];
      const uint64_t lt = tile - S.gemm_start;
      const uint32_t oi = __builtin_amdgcn_readfirstlane(find_item(S.gemm_ops, S.n_gemm, lt));
      const DevOp op = S.gemm_ops[oi];
      if (op_has_tables(op))
        gemm_tile_bf16x3<true>(op, lt, S.tab, S.arena, smem, S.split);
      else
        gemm_tile_bf16x3<false>(op, lt, S.tab, S.arena, smem, S.split);
    }
  } else {
    __shared__ SmemF32 smem;
    for (uint64_t tile = blockIdx.x; tile < a.gemm_tiles; tile += a.tile_blocks) {
      const LevelSeg& S =
          a.seg[find_seg(a, tile, [](const LevelSeg& s) { return s.gemm_start; })];
      const uint64_t lt = tile - S.gemm_start;
      const uint32_t oi = __builtin_amdgcn_readfirstlane(find_item(S.gemm_ops, S.n_gemm, lt));
      const DevOp op = S.gemm_ops[oi];
      if (op_has_tables(op))
        gemm_tile_f32<true>(op, lt, S.tab, S.arena, smem, S.split);
      else
        gemm_tile_f32<false>(op, lt, S.tab, S.arena, smem, S.split);
    }
  }
}

// 128 x 128 tiles of a level's wide GEMM ops: one workgroup per CU walks
// the tiles (the grid is a multiple of 8, which the tile order relies on
// for its XCD placement; any grid is correct).
template <int PREC>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1)))
k_gemm_wide(LevelArgs a) {
  using Smem = typename std::conditional<PREC == TC_PREC_BF16X3, SmemWideBF16, SmemWideF32>::type;
  __shared__ Smem smem[2];
  for (uint64_t tile = blockIdx.x; tile < a.wide_tiles; tile += gridDim.x) {
    const LevelSeg& S = a.seg[find_seg(a, tile, [](const LevelSeg& s) { return s.wide_start; })];
    const uint64_t lt = tile - S.wide_start;
    const uint32_t oi = __builtin_amdgcn_readfirstlane(find_item(S.wide_ops, S.n_wide, lt));
    const DevOp op = S.wide_ops[oi];
    gemm_wide<PREC == TC_PREC_BF16X3 ? 1 : 0>(
        op, lt - op.work0, S.tab, S.arena,
        reinterpret_cast<const uint4*>(S.split.part + op.part), smem);
  }
}

// Split pass of a level's wide ops: every operand element once into the
// planes the tiles load from (layout at split_chunk).  Thread w converts 8
// k of one row of the level's operands, per op A's rows then B's.  FP32
// (k-major planes): rows fastest, so that neighbouring threads write
// neighbouring floats; split BF16 (per row, each 32-k stage is one 256-byte
// block holding the four planes' 64 bytes, wide_plane_chunk): A's k fastest
// (contiguous reads), B's columns fastest (coalesced reads of B's k rows).
template <int PREC>
__global__ void __launch_bounds__(256) k_split_wide(LevelArgs a) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; w < a.wide_chunks; w += stride) {
    uint64_t e = w;
    for (uint32_t s = 0; s < a.nseg; ++s) {
      const LevelSeg& S = a.seg[s];
      for (uint32_t o = 0; o < S.n_wide; ++o) {
        const DevOp& op = S.wide_ops[o];
        const uint64_t kc = op.K / 8;
        const uint64_t RA = (op.a_bs ? op.rows : 1) * (uint64_t)op.M;
        const uint64_t RB = (op.b_bs ? op.rows : 1) * (uint64_t)op.N;
        const uint64_t na = RA * kc, nb = RB * kc;
        if (e >= na + nb) {
          e -= na + nb;
          continue;
        }
        float2 x[8];
        if (PREC == TC_PREC_C64) {
          float* pl = S.split.part + op.part;
          const uint64_t K = op.K;
          if (e < na) {  // A row `row` (= r M + m), k .. k + 7
            const uint64_t row = e % RA, k = (e / RA) * 8;
            const float2* src = S.arena + op.a + (row / op.M) * op.a_bs + (row % op.M) * K + k;
#pragma unroll
            for (int q = 0; q < 8; ++q) x[q] = src[q];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
              pl[(k + q) * RA + row] = x[q].x;
              pl[K * RA + (k + q) * RA + row] = x[q].y;
            }
          } else {  // B column `col` (= r N + n), k .. k + 7
            const uint64_t f = e - na, col = f % RB, k = (f / RB) * 8;
            const float2* src = S.arena + op.b + (col / op.N) * op.b_bs + k * op.N + col % op.N;
#pragma unroll
            for (int q = 0; q < 8; ++q) x[q] = src[(uint64_t)q * op.N];
            float* pb = pl + 2 * K * RA;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
              pb[(k + q) * RB + col] = x[q].x;
              pb[K * RB + (k + q) * RB + col] = x[q].y;
            }
          }
        } else {
          uint4* planes = reinterpret_cast<uint4*>(S.split.part + op.part);
          if (e < na) {
            const uint64_t row = e / kc, k = (e % kc) * 8;  // row = r M + m
            const float2* src = S.arena + op.a + (row / op.M) * op.a_bs + (row % op.M) * op.K + k;
#pragma unroll
            for (int q = 0; q < 8; ++q) x[q] = src[q];
            split_chunk(x, planes + wide_plane_chunk(row, k / 8, kc), 4);
          } else {
            const uint64_t f = e - na;
            const uint64_t n = f % op.N, k = ((f / op.N) % kc) * 8, r = f / (op.N * kc);
            const float2* src = S.arena + op.b + r * op.b_bs + k * op.N + n;
#pragma unroll
            for (int q = 0; q < 8; ++q) x[q] = src[(uint64_t)q * op.N];
            // B's planes follow A's; B's rows are (r, n)
            split_chunk(x, planes + 4 * na + wide_plane_chunk(r * op.N + n, k / 8, kc), 4);
          }
        }
        e = ~uint64_t(0);  // done
        break;
      }
      if (e == ~uint64_t(0)) break;
    }
  }
}

// Split-K reduction of a level: workgroup u adds the slices of split-K
// output tile u in slice order and stores C (a block tile with all 256
// threads, a wave tile with the first wavefront).
__global__ void __launch_bounds__(256) k_reduce(LevelArgs a) {
  const uint64_t u = blockIdx.x;
  const LevelSeg& S = a.seg[find_seg(a, u, [](const LevelSeg& s) { return s.split_start; })];
  const DevSplitUnit su = S.sunits[u - S.split_start];
  const DevOp op = S.gemm_ops[su.op];
  if (su.op < S.n_gemm) {
    f4 cr[2][2], ci[2][2];
    sum_part_block(op, su.tile, S.split, cr, ci);
    const TileCtx c = unit_ctx(op, (uint64_t)su.tile * op.ksplit, S.arena, BM, BN);
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    store_tile(op, c, S.tab, S.arena, cr, ci, wave >> 1, wave & 1, lane);
  } else if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    switch ((op.flags >> 12) & 3u) {
      case 0: reduce_wave<1, 1>(op, su.tile, S.tab, S.arena, lane, S.split); break;
      case 1: reduce_wave<2, 1>(op, su.tile, S.tab, S.arena, lane, S.split); break;
      case 2: reduce_wave<1, 2>(op, su.tile, S.tab, S.arena, lane, S.split); break;
      default: reduce_wave<2, 2>(op, su.tile, S.tab, S.arena, lane, S.split); break;
    }
  }
}

// Gather item: an op with k-split S = 2^ls and n-vector V = 2^lv assigns S
// consecutive lanes to a group of V outputs (row, m, n0 .. n0+V-1); lane
// `sub` sums k = sub, sub + S, ... and the S lanes combine by butterfly
// shuffles.  Ops with S > 1 start and end on wavefront boundaries (the
// planner pads them, and segments start on multiples of 64), so every lane
// of such a wave runs the same shuffles.
// Gather item l of op (item layout above).  All lanes of a wavefront call
// this together (the k-split combines across lanes); `has` = false makes
// the call a no-op that still joins the shuffles.  TABLES: the op has an
// index table (else every index is computed, branch-free).
template <bool TABLES, bool SPLIT, bool DEEP = false>
__device__ __forceinline__ void gather_item_t(const DevOp& op, uint64_t l, bool has,
                                              const uint32_t* __restrict__ tab,
                                              float2* __restrict__ arena,
                                              float* __restrict__ part) {
  const uint32_t ls = has ? (op.flags >> 4) & 7u : 0u;
  const uint32_t lv = has ? (op.flags >> 8) & 3u : 0u;
  const uint32_t S = 1u << ls, V = 1u << lv;
  bool valid = false;
  uint64_t e = 0;
  uint32_t sub = 0, ln = 0, lm = 0;
  // split sums (ksplit > 1): item group e covers slice e / G of output
  // group e % G, over k in [slice K / P, (slice + 1) K / P); its partial
  // sum is entry e of the op's partials ([slice][output group])
  uint32_t kb = 0, ke = 0;
  uint64_t eo = 0;  // output group
  if (has) {
    ln = __builtin_ctz(op.N) - lv;
    lm = __builtin_ctz(op.M);
    e = l >> ls;
    sub = (uint32_t)(l & (S - 1));
    const uint64_t G = (uint64_t)op.rows << (ln + lm);
    valid = e < (SPLIT ? G * op.ksplit : G);
    ke = op.K;
    eo = e;
    if (SPLIT && valid) {
      const uint32_t slice = (uint32_t)(e / G);
      eo = e - (uint64_t)slice * G;
      const uint32_t ks = op.K / op.ksplit;
      kb = slice * ks;
      ke = kb + ks;
    }
  }
  c32 acc[4] = {cx(0.f, 0.f), cx(0.f, 0.f), cx(0.f, 0.f), cx(0.f, 0.f)};
  uint32_t m = 0, n0 = 0;
  uint64_t r = 0;
  if (valid) {
    n0 = (uint32_t)(eo & ((1u << ln) - 1)) << lv;
    m = (uint32_t)((eo >> ln) & (op.M - 1));
    r = eo >> (ln + lm);
    const float2* __restrict__ A = arena + op.a + r * op.a_bs + ixt<TABLES>(tab, op.a_m, m);
    const float2* __restrict__ Bp = arena + op.b + r * op.b_bs;
    uint32_t bn[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) bn[j] = (uint32_t)j < V ? ixt<TABLES>(tab, op.b_n, n0 + j) : 0u;
    if (SPLIT)  // split ops have V == 1
      gather_dot<1, TABLES, DEEP>(acc, A, Bp, tab, op.a_k, op.b_k, bn, sub, S, kb, ke);
    else if (V == 4)
      gather_dot<4, TABLES, DEEP>(acc, A, Bp, tab, op.a_k, op.b_k, bn, sub, S, kb, ke);
    else if (V == 2)
      gather_dot<2, TABLES, DEEP>(acc, A, Bp, tab, op.a_k, op.b_k, bn, sub, S, kb, ke);
    else
      gather_dot<1, TABLES, DEEP>(acc, A, Bp, tab, op.a_k, op.b_k, bn, sub, S, kb, ke);
  }
  if (S > 1) {
    // V == 1 whenever S > 1
    for (uint32_t off = S >> 1; off > 0; off >>= 1) {
      acc[0].re += __shfl_xor(acc[0].re, (int)off, 64);
      acc[0].im += __shfl_xor(acc[0].im, (int)off, 64);
    }
  }
  if (SPLIT && valid && sub == 0) {
    reinterpret_cast<float2*>(part + op.part)[e] = make_float2(acc[0].re, acc[0].im);
  } else if (valid && sub == 0) {
    const uint64_t cb = op.c + r * op.c_bs + ixt<TABLES>(tab, op.c_m, m);
#pragma unroll
    for (uint32_t j = 0; j < 4; ++j)
      if (j < V) arena[cb + ixt<TABLES>(tab, op.c_n, n0 + j)] = make_float2(acc[j].re, acc[j].im);
  }
}

// An unsplit gather op's item.
template <bool DEEP = false>
__device__ __forceinline__ void gather_item(const DevOp& op, uint64_t l, bool has,
                                            const uint32_t* __restrict__ tab,
                                            float2* __restrict__ arena) {
  if (has && op_has_tables(op))
    gather_item_t<true, false, DEEP>(op, l, has, tab, arena, nullptr);
  else
    gather_item_t<false, false, DEEP>(op, l, has, tab, arena, nullptr);
}

// Split gather sums of a level: workgroup u adds, for up to 256 output
// groups of one split op, its slices in slice order and stores C.
__global__ void __launch_bounds__(256) k_reduce_g(LevelArgs a) {
  const uint64_t u = blockIdx.x;
  const LevelSeg& S = a.seg[find_seg(a, u, [](const LevelSeg& s) { return s.gsplit_start; })];
  const DevSplitUnit su = S.gsunits[u - S.gsplit_start];
  const DevOp& op = S.gs_ops[su.op];
  const uint32_t ln = __builtin_ctz(op.N), lm = __builtin_ctz(op.M);  // V == 1
  const uint64_t G = (uint64_t)op.rows << (ln + lm);
  const uint64_t e = (uint64_t)su.tile * 256 + threadIdx.x;
  if (e >= G) return;
  const float2* src = reinterpret_cast<const float2*>(S.split.part + op.part) + e;
  c32 acc = cx(0.f, 0.f);
  for (uint32_t q = 0; q < op.ksplit; ++q) {
    const float2 v = src[q * G];
    acc.re += v.x;
    acc.im += v.y;
  }
  const uint32_t n = (uint32_t)(e & (op.N - 1));
  const uint32_t m = (uint32_t)((e >> ln) & (op.M - 1));
  const uint64_t r = e >> (ln + lm);
  S.arena[op.c + r * op.c_bs + ix(S.tab, op.c_m, m) + ix(S.tab, op.c_n, n)] =
      make_float2(acc.re, acc.im);
}

// Row tiles: workgroup b copies RPB (= op.tiles_m) whole batch rows of both
// operands of one small batched node into LDS (a batched tensor's row is
// one block of M K or K N elements, so the copy is coalesced; a shared
// operand is copied once), then computes the rows' M N outputs each from
// LDS, k in increasing order, and stores them.
__global__ void __launch_bounds__(256) k_rowtile(LevelArgs a) {
  __shared__ float2 buf[ROW_TILE_LDS];
  // A's and B's offsets of each k (K <= ROW_TILE_LDS / 2, as a row of both
  // operands fits the staging buffer), decoded once per workgroup: the sum
  // over k runs the same k on every lane, so decoding it there kept the
  // scalar unit busy for every output
  __shared__ uint32_t koff[2][ROW_TILE_LDS / 2];
  const uint64_t b = blockIdx.x;
  const LevelSeg& S = a.seg[find_seg(a, b, [](const LevelSeg& s) { return s.rt_start; })];
  const uint64_t lb = b - S.rt_start;
  const uint32_t oi = __builtin_amdgcn_readfirstlane(
      S.rt_unit_op ? S.rt_unit_op[lb] : find_item(S.rt_ops, S.n_rt, lb));
  const DevOp op = S.rt_ops[oi];
  const uint32_t rpb = op.tiles_m;
  const uint64_t r0 = (lb - op.work0) * rpb;
  const uint32_t nr = (uint32_t)min((uint64_t)rpb, op.rows - r0);
  const uint32_t MK = op.M * op.K, KN = op.K * op.N, MN = op.M * op.N;
  const uint32_t ra = op.a_bs ? nr : 1, rb = op.b_bs ? nr : 1;
  const int t = threadIdx.x;
  const float2* __restrict__ A = S.arena + op.a + r0 * op.a_bs;
  const float2* __restrict__ B = S.arena + op.b + r0 * op.b_bs;
  // rows r0 .. r0 + nr - 1 of A, then of B (row stride a_bs, b_bs): all of
  // a thread's loads (at most ROW_TILE_LDS / 256) are issued before the
  // first LDS store, so the copy costs one memory round trip
  const uint32_t lmk = __builtin_ctz(MK), lkn = __builtin_ctz(KN);
  const uint32_t na = ra * MK, ntot = na + rb * KN;
  constexpr uint32_t PER = ROW_TILE_LDS / 256;
  float2 v[PER];
#pragma unroll
  for (uint32_t q = 0; q < PER; ++q) {
    const uint32_t e = t + q * 256;
    if (e < na)
      v[q] = A[(uint64_t)(e >> lmk) * op.a_bs + (e & (MK - 1))];
    else if (e < ntot)
      v[q] = B[(uint64_t)((e - na) >> lkn) * op.b_bs + ((e - na) & (KN - 1))];
  }
#pragma unroll
  for (uint32_t q = 0; q < PER; ++q) {
    const uint32_t e = t + q * 256;
    if (e < ntot) buf[e] = v[q];
  }
  for (uint32_t k = t; k < op.K; k += 256) {
    koff[0][k] = ix(S.tab, op.a_k, k);
    koff[1][k] = ix(S.tab, op.b_k, k);
  }
  __syncthreads();
  const uint32_t lmn = __builtin_ctz(MN), ln = __builtin_ctz(op.N);
  for (uint32_t o = t; o < nr * MN; o += 256) {
    const uint32_t rr = o >> lmn, y = o & (MN - 1);
    const uint32_t m = y >> ln, n = y & (op.N - 1);
    const float2* Ar = buf + (op.a_bs ? rr * MK : 0) + ix(S.tab, op.a_m, m);
    const float2* Br = buf + ra * MK + (op.b_bs ? rr * KN : 0) + ix(S.tab, op.b_n, n);
    float re = 0.f, im = 0.f;
    for (uint32_t k = 0; k < op.K; ++k) {
      const float2 x = Ar[koff[0][k]], w = Br[koff[1][k]];
      re += x.x * w.x - x.y * w.y;
      im += x.x * w.y + x.y * w.x;
    }
    S.arena[op.c + (r0 + rr) * op.c_bs + ix(S.tab, op.c_m, m) + ix(S.tab, op.c_n, n)] =
        make_float2(re, im);
  }
}

// Gather ops of a level; SPLIT: the split ones (their own kernel, so that
// the split bookkeeping takes no registers from the others).
// Op records read at wave-uniform addresses through the constant address
// space, so that the loads are scalar (the compiler's host pass, which
// only parses device code, sees a plain pointer).
#if defined(__HIP_DEVICE_COMPILE__)
typedef const __attribute__((address_space(4))) DevOp* ScalarOpPtr;
typedef const __attribute__((address_space(4))) uint32_t* ScalarU32Ptr;
#else
typedef const DevOp* ScalarOpPtr;
typedef const uint32_t* ScalarU32Ptr;
#endif

// DEEP: the deep k unroll at 5 wavefronts per SIMD, for levels whose items
// hold long sums (bandwidth bound: bytes in flight per wavefront matter);
// else the short unroll at 7 (latency bound: items in flight matter).
template <bool SPLIT, bool DEEP>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(DEEP ? 5 : 7)))
k_gather(LevelArgs a) {
  // each block takes one contiguous chunk (a multiple of 256 items, so
  // wavefronts never straddle its end); a thread finds its segment and op
  // once (or reads it from the per-item table) and then only walks forward
  const uint64_t total = SPLIT ? a.gs_work : a.gc_work;
  const uint64_t nblk = gridDim.x;
  const uint64_t chunk = (((total + nblk - 1) / nblk) + 255) & ~uint64_t(255);
  // Workgroups are dispatched to the 8 XCDs round robin (block b to XCD
  // b mod 8), and each XCD has its own L2: each XCD takes a contiguous
  // range of chunks, so that an op's items, which read the same operands,
  // mostly share one L2 instead of fetching those operands once per XCD.
  const uint64_t begin = (a.xcd_order ? xcd_block(nblk) : (uint64_t)blockIdx.x) * chunk;
  const uint64_t end = begin + chunk < total ? begin + chunk : total;
  uint32_t si = 0xffffffffu, oi = 0xffffffffu;
  for (uint64_t w = begin + threadIdx.x; w < end; w += blockDim.x) {
    if (si == 0xffffffffu) {
      si = SPLIT ? find_seg(a, w, [](const LevelSeg& s) { return s.gs_start; })
                 : find_seg(a, w, [](const LevelSeg& s) { return s.gc_start; });
    } else {
      while (si + 1 < a.nseg && (SPLIT ? a.seg[si + 1].gs_start : a.seg[si + 1].gc_start) <= w) {
        ++si;
        oi = 0xffffffffu;
      }
    }
    const LevelSeg& Sg = a.seg[si];
    const DevOp* ops = SPLIT ? Sg.gs_ops : Sg.gc_ops;
    const uint32_t n = SPLIT ? Sg.n_gs : Sg.n_gc;
    const uint64_t ws = w - (SPLIT ? Sg.gs_start : Sg.gc_start);
    const bool has = n > 0;
    if (has) {
      if (!SPLIT && Sg.item_op) {
        // a level's ops start on wavefronts: one table entry per wavefront,
        // read with a scalar load
        const uint32_t wv = __builtin_amdgcn_readfirstlane((uint32_t)(ws >> 6));
        oi = ((ScalarU32Ptr)Sg.item_op)[wv];
      } else if (oi == 0xffffffffu) {
        oi = find_item(ops, n, ws);
      } else {
        while (oi + 1 < n && ops[oi + 1].work0 <= ws) ++oi;
      }
    } else {
      oi = 0;
    }
    const DevOp& op = ops[oi];
    if (SPLIT) {
      if (has && op_has_tables(op))
        gather_item_t<true, true, DEEP>(op, has ? ws - op.work0 : 0, has, Sg.tab, Sg.arena, Sg.split.part);
      else
        gather_item_t<false, true, DEEP>(op, has ? ws - op.work0 : 0, has, Sg.tab, Sg.arena, Sg.split.part);
    } else {
      // Segments start at multiples of 64 items, so a wavefront's lanes
      // share the segment; when they share the op too (all but the
      // wavefronts that straddle two ops), the op record is read once
      // through the constant address space (scalar loads) and its
      // descriptor arithmetic stays scalar.
      const uint32_t siu = __builtin_amdgcn_readfirstlane(si);
      const uint32_t oiu = __builtin_amdgcn_readfirstlane(oi);
      if (has && __builtin_amdgcn_ballot_w64(oi != oiu) == 0) {
        const LevelSeg& Su = a.seg[siu];
        const DevOp opu = ((ScalarOpPtr)Su.gc_ops)[oiu];
        gather_item<DEEP>(opu, ws - opu.work0, true, Su.tab, Su.arena);
      } else {
        gather_item<DEEP>(op, has ? ws - op.work0 : 0, has, Sg.tab, Sg.arena);
      }
    }
  }
}

// largest i in [lo, hi) with items[i].work0 <= w (items[lo].work0 <= w)
template <typename T>
__device__ __forceinline__ uint32_t find_in(const T* __restrict__ items, uint32_t lo, uint32_t hi,
                                            uint64_t w) {
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (items[mid].work0 <= w)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// Term launch: workgroup t runs term t alone over a run of steps (first
// its leaves, if asked), each group (its nodes at one step) followed by a
// workgroup barrier; the terms advance independently, each in its own arena
// region, so a run of light steps costs barriers instead of kernel
// launches.  Group items are whole wavefronts (a multiple of 64) and the
// block strides over them in steps of 1024, so the lanes of a wavefront
// always share one op.
// Groups and op records of a term launch are staged in LDS: the groups of
// the term's range once, and each group's op records (up to TERM_LDS_OPS of
// them) double-buffered, the next group's loaded into registers while the
// current group computes and written to the other buffer before the
// barrier.  Reading op records and finding an item's op then costs LDS
// accesses instead of dependent global loads on every step.
constexpr uint32_t TERM_LDS_OPS = 128, TERM_LDS_GROUPS = 64;
constexpr uint32_t OP_WORDS = sizeof(DevOp) / 4;
static_assert(sizeof(DevOp) % 4 == 0, "op records are copied as 32-bit words");
constexpr uint32_t TERM_PRE = (TERM_LDS_OPS * OP_WORDS + 1023) / 1024;  // words per thread

__global__ void __launch_bounds__(1024) k_term(TermArgs a) {
  __shared__ DevOp sops[2][TERM_LDS_OPS];
  __shared__ DevGroup sgroups[TERM_LDS_GROUPS];
  const DevTerm T = a.terms[blockIdx.x];
  const DevRange R = a.ranges[blockIdx.x];
  const uint32_t ng = R.g_end - R.g_begin;
  const bool groups_staged = ng <= TERM_LDS_GROUPS;
  if (groups_staged && threadIdx.x < ng) sgroups[threadIdx.x] = a.groups[R.g_begin + threadIdx.x];
  auto group = [&](uint32_t g) -> DevGroup {
    return groups_staged ? sgroups[g - R.g_begin] : a.groups[g];
  };
  uint32_t pre[TERM_PRE];
  auto fetch = [&](uint32_t g) {  // the op records of group g, into registers
    if (g >= R.g_end) return;
    const DevGroup G = a.groups[g];
    const uint32_t n = G.op_end - G.op_begin;
    if (n > TERM_LDS_OPS) return;
    const uint32_t* src = (const uint32_t*)(a.ops + G.op_begin);
#pragma unroll
    for (uint32_t q = 0; q < TERM_PRE; ++q) {
      const uint32_t x = threadIdx.x + q * 1024;
      pre[q] = x < n * OP_WORDS ? src[x] : 0u;
    }
  };
  auto commit = [&](uint32_t g, int buf) {  // registers -> LDS buffer
    if (g >= R.g_end) return;
    const DevGroup G = a.groups[g];
    const uint32_t n = G.op_end - G.op_begin;
    if (n > TERM_LDS_OPS) return;
    uint32_t* dst = (uint32_t*)&sops[buf][0];
#pragma unroll
    for (uint32_t q = 0; q < TERM_PRE; ++q) {
      const uint32_t x = threadIdx.x + q * 1024;
      if (x < n * OP_WORDS) dst[x] = pre[q];
    }
  };
  fetch(R.g_begin);
  if (a.with_leaves) {
    for (uint64_t w = T.leaf_work0 + threadIdx.x; w < T.leaf_work_end; w += blockDim.x) {
      const uint32_t li =
          a.item_leaf ? a.item_leaf[w] : find_in(a.leaves, T.leaf_begin, T.leaf_end, w);
      leaf_item(a.leaves[li], w, a.params, a.param_stride, a.ftab, a.arena);
    }
  }
  commit(R.g_begin, 0);
  __syncthreads();
  for (uint32_t g = R.g_begin; g < R.g_end; ++g) {
    const int buf = (int)((g - R.g_begin) & 1u);
    const DevGroup G = group(g);
    const uint32_t n = G.op_end - G.op_begin;
    fetch(g + 1);  // in flight while this group computes
    if (n <= TERM_LDS_OPS) {
      const DevOp* ops = sops[buf];
      for (uint64_t w = threadIdx.x; w < G.items; w += blockDim.x) {
        // largest op with work0 <= w, by binary search over the LDS records
        uint32_t lo = 0, hi = n;
        while (hi - lo > 1) {
          const uint32_t mid = (lo + hi) >> 1;
          if (ops[mid].work0 <= w)
            lo = mid;
          else
            hi = mid;
        }
        const DevOp& op = ops[lo];
        gather_item<true>(op, w - op.work0, true, a.tab, a.arena);
      }
    } else {
      const DevOp* __restrict__ ops = a.ops + G.op_begin;
      uint32_t oi = 0xffffffffu;
      for (uint64_t w = threadIdx.x; w < G.items; w += blockDim.x) {
        if (G.item_base != NO_ITEMS)
          oi = a.item_op[G.item_base + w];
        else if (oi == 0xffffffffu)
          oi = find_item(ops, n, w);
        else
          while (oi + 1 < n && ops[oi + 1].work0 <= w) ++oi;
        const DevOp& op = ops[oi];
        gather_item<true>(op, w - op.work0, true, a.tab, a.arena);
      }
    }
    commit(g + 1, buf ^ 1);
    __syncthreads();
  }
}

// Resident term launch: workgroup t runs term t's whole evaluation, its
// leaves, every forward step and (with the gradient) every reverse-sweep
// step, with a workgroup barrier after each step.  Each node reads its
// operands from the LDS arena (extern shared memory, sized by the plan) or
// the global arena, as its record says, and writes its result to one or
// both; the planner placed the tensors so that a step's reads never meet a
// region written in the same step.  Operand pointers are generic (flat)
// so that one code path serves either memory.  Op records of a step are
// double-buffered in LDS as in k_term.
constexpr uint32_t RES_LDS_OPS = 160;
constexpr uint32_t ROP_WORDS = sizeof(DevROp) / 4;
static_assert(sizeof(DevROp) % 4 == 0, "resident op records are copied as 32-bit words");
constexpr uint32_t RES_PRE = (RES_LDS_OPS * ROP_WORDS + 1023) / 1024;  // words per thread

// Item l of a resident node (the item layout of gather_item_t, batch 1).
// All lanes of a wavefront whose node splits its sums (S > 1) call this
// together: such nodes start and end on wavefront boundaries.
template <bool TABLES>
__device__ __forceinline__ void res_item_t(const DevROp& op, uint32_t l,
                                           const uint32_t* __restrict__ tab,
                                           float2* __restrict__ arena, float2* lds) {
  const uint32_t sh = op.shape;
  const uint32_t lm = sh & 31u, lk = (sh >> 10) & 31u, ls = (sh >> 15) & 7u, lv = (sh >> 18) & 3u;
  const uint32_t ln = ((sh >> 5) & 31u) - lv;
  const uint32_t S = 1u << ls, V = 1u << lv;
  const uint32_t e = l >> ls, sub = l & (S - 1);
  const bool valid = e < (1u << (ln + lm));
  c32 acc[4] = {cx(0.f, 0.f), cx(0.f, 0.f), cx(0.f, 0.f), cx(0.f, 0.f)};
  uint32_t m = 0, n0 = 0;
  if (valid) {
    n0 = (e & ((1u << ln) - 1)) << lv;
    m = e >> ln;
    const float2* A = ((sh & RES_A_LDS) ? lds : arena) + op.a + ixt<TABLES>(tab, op.a_m, m);
    const float2* Bp = ((sh & RES_B_LDS) ? lds : arena) + op.b;
    uint32_t bn[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) bn[j] = (uint32_t)j < V ? ixt<TABLES>(tab, op.b_n, n0 + j) : 0u;
    const uint32_t K = 1u << lk;
    if (V == 4)
      gather_dot<4, TABLES, true>(acc, A, Bp, tab, op.a_k, op.b_k, bn, sub, S, 0, K);
    else if (V == 2)
      gather_dot<2, TABLES, true>(acc, A, Bp, tab, op.a_k, op.b_k, bn, sub, S, 0, K);
    else
      gather_dot<1, TABLES, true>(acc, A, Bp, tab, op.a_k, op.b_k, bn, sub, S, 0, K);
  }
  if (S > 1) {
    // V == 1 whenever S > 1
    for (uint32_t off = S >> 1; off > 0; off >>= 1) {
      acc[0].re += __shfl_xor(acc[0].re, (int)off, 64);
      acc[0].im += __shfl_xor(acc[0].im, (int)off, 64);
    }
  }
  if (valid && sub == 0) {
    float2* C = ((sh & RES_C_LDS) ? lds : arena) + op.c + ixt<TABLES>(tab, op.c_m, m);
    float2* C2 = arena + op.c2 + ixt<TABLES>(tab, op.c_m, m);
#pragma unroll
    for (uint32_t j = 0; j < 4; ++j)
      if (j < V) {
        const uint32_t o = ixt<TABLES>(tab, op.c_n, n0 + j);
        const float2 v = make_float2(acc[j].re, acc[j].im);
        C[o] = v;
        if (sh & RES_C2) C2[o] = v;
      }
  }
}

__device__ __forceinline__ void res_item(const DevROp& op, uint32_t l,
                                         const uint32_t* __restrict__ tab,
                                         float2* __restrict__ arena, float2* lds) {
  if (op.shape & RES_TABLES)
    res_item_t<true>(op, l, tab, arena, lds);
  else
    res_item_t<false>(op, l, tab, arena, lds);
}

__global__ void __launch_bounds__(1024) k_term_res(TermArgs a) {
  extern __shared__ float2 lds[];
  __shared__ DevROp sops[2][RES_LDS_OPS];
  __shared__ DevGroup sgroups[TERM_LDS_GROUPS];
  const DevTerm T = a.terms[blockIdx.x];
  const DevRange R = a.ranges[blockIdx.x];
  const uint32_t ng = R.g_end - R.g_begin;
  const bool groups_staged = ng <= TERM_LDS_GROUPS;
  if (groups_staged && threadIdx.x < ng) sgroups[threadIdx.x] = a.groups[R.g_begin + threadIdx.x];
  uint32_t pre[RES_PRE];
  auto fetch = [&](uint32_t g) {  // the op records of group g, into registers
    if (g >= R.g_end) return;
    const DevGroup G = a.groups[g];
    const uint32_t n = G.op_end - G.op_begin;
    if (n > RES_LDS_OPS) return;
    const uint32_t* src = (const uint32_t*)(a.rops + G.op_begin);
#pragma unroll
    for (uint32_t q = 0; q < RES_PRE; ++q) {
      const uint32_t x = threadIdx.x + q * 1024;
      pre[q] = x < n * ROP_WORDS ? src[x] : 0u;
    }
  };
  auto commit = [&](uint32_t g, int buf) {  // registers -> LDS buffer
    if (g >= R.g_end) return;
    const DevGroup G = a.groups[g];
    const uint32_t n = G.op_end - G.op_begin;
    if (n > RES_LDS_OPS) return;
    uint32_t* dst = (uint32_t*)&sops[buf][0];
#pragma unroll
    for (uint32_t q = 0; q < RES_PRE; ++q) {
      const uint32_t x = threadIdx.x + q * 1024;
      if (x < n * ROP_WORDS) dst[x] = pre[q];
    }
  };
  fetch(R.g_begin);
  // the term's leaves, at batch row 0, into LDS and / or the global arena
  // (only in the launch that materialises them: a later run's LDS arena
  // and the leaves' freed global regions hold other tensors by then)
  for (uint64_t w = T.leaf_work0 + threadIdx.x; a.with_leaves && w < T.leaf_work_end;
       w += blockDim.x) {
    const uint32_t li =
        a.item_leaf ? a.item_leaf[w] : find_in(a.leaves, T.leaf_begin, T.leaf_end, w);
    const DevLeaf& L = a.leaves[li];
    const int e = (int)(w - L.work0);
    const float t0 = L.param[0] >= 0 ? a.params[L.param[0]] : L.fixed[0];
    const float t1 = L.param[1] >= 0 ? a.params[L.param[1]] : L.fixed[1];
    const c32 v = leaf_entry(L, e, t0, t1, a.ftab);
    if (L.where & 1u) a.arena[L.out + e] = make_float2(v.re, v.im);
    if (L.where & 2u) lds[L.lds_out + e] = make_float2(v.re, v.im);
  }
  commit(R.g_begin, 0);
  __syncthreads();
  for (uint32_t g = R.g_begin; g < R.g_end; ++g) {
    const int buf = (int)((g - R.g_begin) & 1u);
    const DevGroup G = groups_staged ? sgroups[g - R.g_begin] : a.groups[g];
    const uint32_t n = G.op_end - G.op_begin;
    fetch(g + 1);  // in flight while this group computes
    const DevROp* ops = n <= RES_LDS_OPS ? sops[buf] : a.rops + G.op_begin;
    uint32_t oi = 0xffffffffu;
    for (uint32_t w = threadIdx.x; w < (uint32_t)G.items; w += blockDim.x) {
      if (oi == 0xffffffffu) {
        // largest op with work0 <= w
        uint32_t lo = 0, hi = n;
        while (hi - lo > 1) {
          const uint32_t mid = (lo + hi) >> 1;
          if (ops[mid].work0 <= w)
            lo = mid;
          else
            hi = mid;
        }
        oi = lo;
      } else {
        while (oi + 1 < n && ops[oi + 1].work0 <= w) ++oi;
      }
      const DevROp op = ops[oi];
      res_item(op, w - op.work0, a.tab, a.arena, lds);
    }
    commit(g + 1, buf ^ 1);
    __syncthreads();
  }
}

// E[b] = sum_j alpha_j T_j[b] in FP64: one wavefront per batch row, lane l
// takes terms l, l + 64, ...; the 64 partial sums combine in a fixed
// butterfly order (deterministic).
// Root rows for block `blk` of the root part of a launch.
__device__ __forceinline__ void root_rows(const RootArgs& a, uint64_t blk) {
  const uint32_t lane = threadIdx.x & 63;
  const uint64_t wv = (blk * blockDim.x + threadIdx.x) >> 6;
  if (wv >= a.total) return;  // whole wavefronts leave together
  const RootSeg& S = a.seg[find_seg(a, wv, [](const RootSeg& s) { return s.start; })];
  const uint64_t b = wv - S.start;
  double re = 0.0, im = 0.0;
  for (uint32_t j = lane; j < S.n_terms; j += 64) {
    const DevRoot& R = S.roots[j];
    double vr = 1.0, vi = 0.0;
    if (R.present) {
      const float2 v = S.arena[R.val + b * R.bs];
      vr = v.x;
      vi = v.y;
    }
    re += R.weight * vr;
    im += R.weight * vi;
  }
  for (int off = 32; off > 0; off >>= 1) {
    re += __shfl_xor(re, off, 64);
    im += __shfl_xor(im, off, 64);
  }
  if (lane == 0) {
    S.value[2 * b] = re;
    S.value[2 * b + 1] = im;
    if (S.value_re) S.value_re[b] = re;
  }
}

__global__ void __launch_bounds__(256) k_root(RootArgs a) { root_rows(a, blockIdx.x); }

// grad[b][slot] = Re sum_{uses of slot} sum_e adj[e] dleaf[e]/dangle in FP64:
// one wavefront per (row, slot), lanes over the slot's uses, fixed-order
// butterfly combination.
// Gradient waves for block `blk` of `nblk` blocks of the gradient part of
// a launch (grid-stride over the (row, slot) waves).
__device__ __forceinline__ void grad_waves(const GradArgs& a, uint64_t blk, uint64_t nblk) {
  const uint32_t lane = threadIdx.x & 63;
  const uint64_t waves = (nblk * blockDim.x) >> 6;
  for (uint64_t wv = (blk * blockDim.x + threadIdx.x) >> 6; wv < a.total; wv += waves) {
    const GradSeg& S = a.seg[find_seg(a, wv, [](const GradSeg& s) { return s.start; })];
    const uint64_t w = wv - S.start;
    const uint64_t b = w / (uint32_t)S.n_params;
    const uint32_t slot = (uint32_t)(w - b * (uint32_t)S.n_params);
    const float* pr = S.params + b * (uint64_t)S.param_stride;
    double acc = 0.0, acc_im = 0.0;
    for (uint32_t u = S.slot_begin[slot] + lane; u < S.slot_begin[slot + 1]; u += 64) {
      const DevGradUse& U = S.uses[u];
      const DevLeaf& L = S.leaves[U.leaf];
      const float t0 = L.param[0] >= 0 ? pr[L.param[0]] : L.fixed[0];
      const float t1 = L.param[1] >= 0 ? pr[L.param[1]] : L.fixed[1];
      const float2* ad = S.arena + U.adj + b * U.adj_bs;
      const int ne = 1 << L.rank;
      for (int e = 0; e < ne; ++e) {
        const c32 d = dleaf_entry(L, e, t0, t1, U.which);
        const float2 x = ad[e];
        acc += (double)x.x * d.re - (double)x.y * d.im;
        acc_im += (double)x.x * d.im + (double)x.y * d.re;
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
      acc += __shfl_xor(acc, off, 64);
      acc_im += __shfl_xor(acc_im, off, 64);
    }
    if (lane == 0) {
      if (S.cplx) {
        S.grad[2 * w] = acc;
        S.grad[2 * w + 1] = acc_im;
      } else {
        S.grad[w] = acc;
      }
    }
  }
}

__global__ void __launch_bounds__(256) k_grad(GradArgs a) { grad_waves(a, blockIdx.x, gridDim.x); }

// The last two launches of a gradient call in one: blocks [0, root_blocks)
// sum the roots, the others the gradient (independent: the root sum reads
// the terms' root values and writes E, the gradient sum reads adjoints and
// parameters and writes dE/dtheta).
__global__ void __launch_bounds__(256) k_root_grad(RootArgs r, GradArgs g, uint32_t root_blocks) {
  if (blockIdx.x < root_blocks)
    root_rows(r, blockIdx.x);
  else
    grad_waves(g, blockIdx.x - root_blocks, gridDim.x - root_blocks);
}

// One wavefront per (i, j): lanes over the rows of slot j (sums and v_j)
// and of slot i (v_i), fixed-order butterflies, FP64.
__global__ void __launch_bounds__(256) k_qgt(QgtArgs a) {
  const uint32_t lane = threadIdx.x & 63;
  const uint64_t wv = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const uint64_t np = (uint64_t)a.n_params;
  if (wv >= np * np) return;  // whole wavefronts leave together
  const uint32_t i = (uint32_t)(wv / np), j = (uint32_t)(wv - (uint64_t)i * np);
  double sr = 0.0, si = 0.0, vjr = 0.0, vji = 0.0, vir = 0.0, vii = 0.0;
  for (uint32_t k = a.slot_begin[j] + lane; k < a.slot_begin[j + 1]; k += 64) {
    const uint64_t u = a.rows[k];
    sr += a.sums[2 * (u * np + i)];
    si += a.sums[2 * (u * np + i) + 1];
    vjr += a.value[2 * u];
    vji += a.value[2 * u + 1];
  }
  for (uint32_t k = a.slot_begin[i] + lane; k < a.slot_begin[i + 1]; k += 64) {
    const uint64_t u = a.rows[k];
    vir += a.value[2 * u];
    vii += a.value[2 * u + 1];
  }
  for (int off = 32; off > 0; off >>= 1) {
    sr += __shfl_xor(sr, off, 64);
    si += __shfl_xor(si, off, 64);
    vjr += __shfl_xor(vjr, off, 64);
    vji += __shfl_xor(vji, off, 64);
    vir += __shfl_xor(vir, off, 64);
    vii += __shfl_xor(vii, off, 64);
  }
  if (lane == 0) {
    // conj(v_i) v_j
    const double pr = vir * vjr + vii * vji, pi = vir * vji - vii * vjr;
    a.out[2 * wv] = sr - pr;
    a.out[2 * wv + 1] = si - pi;
  }
}

// ------------------------------------------------------------------ launching

static unsigned grid_for(uint64_t work, int threads, int n_cu) {
  uint64_t g = (work + threads - 1) / threads;
  uint64_t cap = (uint64_t)n_cu * 64;  // grid-stride beyond this
  return (unsigned)std::max<uint64_t>(1, std::min(g, cap));
}

int device_cu_count(int device) {
  hipDeviceProp_t prop;
  HIP_CHECK(hipGetDeviceProperties(&prop, device));
  return prop.multiProcessorCount;
}

// Profiling: while set, every kernel launch records its start (the first
// launch) and end (each launch, so the last one's remains) on these events,
// stamped by the kernel dispatch itself rather than queued beside it.
struct ProfEvents {
  hipEvent_t start, stop;
  bool started;
};
static thread_local ProfEvents* t_prof = nullptr;

template <typename... Args>
static void launch_shm(void (*kernel)(Args...), dim3 grid, dim3 block, size_t shm, hipStream_t st,
                       Args... args) {
  if (t_prof) {
    hipEvent_t s = t_prof->started ? nullptr : t_prof->start;
    t_prof->started = true;
    hipExtLaunchKernelGGL(kernel, grid, block, shm, st, s, t_prof->stop, 0, args...);
  } else {
    hipLaunchKernelGGL(kernel, grid, block, shm, st, args...);
  }
}

template <typename... Args>
static void launch(void (*kernel)(Args...), dim3 grid, dim3 block, hipStream_t st,
                   Args... args) {
  launch_shm(kernel, grid, block, 0, st, args...);
}

// Elements of the LDS arena a resident term launch can have on `device`:
// the device's shared memory per workgroup less k_term_res's own, in whole
// 256-element blocks; 0 when the device cannot be queried.
uint32_t resident_lds_elems(int device) {
  int max_shared = 0;
  if (hipDeviceGetAttribute(&max_shared, hipDeviceAttributeMaxSharedMemoryPerBlock, device) !=
      hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  hipFuncAttributes fa{};
  if (hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(k_term_res)) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  const int64_t avail = (int64_t)max_shared - (int64_t)fa.sharedSizeBytes - 1024;
  if (avail < 8 * 4096) return 0;
  const uint32_t elems = (uint32_t)((avail / 8) & ~int64_t(255));
  // (the launch asks for this much dynamic shared memory)
  if (hipFuncSetAttribute(reinterpret_cast<const void*>(k_term_res),
                          hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)(elems * sizeof(float2))) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return elems;
}

// Arguments of the root sum over `segs` (one segment per plan).
static RootArgs root_args(const SegRef* segs, int nseg) {
  RootArgs a{};
  uint64_t w = 0;
  for (int i = 0; i < nseg; ++i) {
    const SegRef& s = segs[i];
    const WorkspaceLayout& L = *s.lay;
    RootSeg& g = a.seg[i];
    g.roots = (const DevRoot*)(s.ws + L.roots);
    g.arena = (const float2*)(s.ws + L.arena);
    g.value = (double*)(s.ws + L.value);
    g.value_re = s.value_re;
    g.n_terms = (uint32_t)s.plan->roots.size();
    g.batch = (uint32_t)s.plan->batch;
    g.start = w;
    w += (uint64_t)s.plan->batch;
  }
  a.nseg = (uint32_t)nseg;
  a.total = w;
  return a;
}

// Arguments of the gradient sum over `segs`.
static GradArgs grad_args(const SegRef* segs, int nseg) {
  GradArgs a{};
  uint64_t w = 0;
  for (int i = 0; i < nseg; ++i) {
    const SegRef& s = segs[i];
    const WorkspaceLayout& L = *s.lay;
    GradSeg& g = a.seg[i];
    g.uses = (const DevGradUse*)(s.ws + L.uses);
    g.slot_begin = (const uint32_t*)(s.ws + L.slot_begin);
    g.leaves = (const DevLeaf*)(s.ws + L.leaves);
    g.params = s.params ? s.params : (const float*)(s.ws + L.params);
    g.arena = (const float2*)(s.ws + L.arena);
    g.grad = s.grad ? s.grad : (double*)(s.ws + L.grad);
    g.n_params = s.plan->n_params;
    g.param_stride = s.plan->param_stride();
    g.cplx = s.plan->qgt ? 1 : 0;
    g.start = w;
    w += s.launch->work;
  }
  a.nseg = (uint32_t)nseg;
  a.total = w;
  return a;
}

// The root sum of plan segment `r` and the gradient sum of `g` as one
// kernel (k_root_grad), or the root sum alone when there is no gradient
// work.
static_assert(sizeof(RootArgs) + sizeof(GradArgs) + 8 <= 4096,
              "k_root_grad's arguments fit the kernel argument segment");
static void launch_root_grad(const SegRef& r, const SegRef& g, hipStream_t stream, int n_cu) {
  const RootArgs ra = root_args(&r, 1);
  const GradArgs ga = grad_args(&g, 1);
  const unsigned rb = (unsigned)((ra.total * 64 + 255) / 256);
  if (ga.total == 0) {
    launch(k_root, dim3(rb), dim3(256), stream, ra);
  } else {
    const unsigned gb = grid_for(ga.total * 64, 256, n_cu);
    launch(k_root_grad, dim3(rb + gb), dim3(256), stream, ra, ga, (uint32_t)rb);
  }
  HIP_CHECK(hipGetLastError());
}

void launch_segments(int kind, const SegRef* segs, int nseg, hipStream_t stream, int n_cu,
                     int precision, int parts) {
  if (nseg <= 0) return;
  if (nseg > MAX_SEG) fail(TC_ERR_INVALID_ARG, "internal: too many segments");
  switch (kind) {
    case L_LEAF: {
      LeafArgs a{};
      uint64_t w = 0;
      for (int i = 0; i < nseg; ++i) {
        const SegRef& s = segs[i];
        const WorkspaceLayout& L = *s.lay;
        LeafSeg& g = a.seg[i];
        g.leaves = (const DevLeaf*)(s.ws + L.leaves);
        g.item_leaf = s.launch->item_begin != NO_ITEMS
                          ? (const uint32_t*)(s.ws + L.item_op) + s.launch->item_begin
                          : nullptr;
        g.ftab = (const float*)(s.ws + L.ftab);
        g.params = s.params ? s.params : (const float*)(s.ws + L.params);
        g.arena = (float2*)(s.ws + L.arena);
        g.n = (uint32_t)s.plan->leaves.size();
        g.param_stride = s.plan->param_stride();
        g.start = w;
        w += s.launch->work;
      }
      a.nseg = (uint32_t)nseg;
      a.total = w;
      if (w == 0) return;
      launch(k_leaf, dim3(grid_for(w, 256, n_cu)), dim3(256), stream, a);
      break;
    }
    case L_LEVEL: {
      LevelArgs a{};
      uint64_t tiles = 0, wtiles = 0, work = 0, sunits = 0, gsunits = 0, gswork = 0, htiles = 0,
               wchunks = 0, rtblocks = 0;
      for (int i = 0; i < nseg; ++i) {
        const SegRef& s = segs[i];
        const WorkspaceLayout& L = *s.lay;
        const DevOp* ops = (const DevOp*)(s.ws + L.ops);
        LevelSeg& g = a.seg[i];
        g.gemm_ops = ops + s.launch->gbegin;
        g.n_gemm = s.launch->gend - s.launch->gbegin;
        g.wave_ops = ops + s.launch->wbegin;
        g.wave_unit_op = s.launch->wunit_begin != NO_ITEMS
                             ? (const uint32_t*)(s.ws + L.item_op) + s.launch->wunit_begin
                             : nullptr;
        g.n_wave = s.launch->wend - s.launch->wbegin;
        g.wide_ops = ops + s.launch->hbegin;
        g.n_wide = s.launch->hend - s.launch->hbegin;
        g.wide_start = htiles;
        htiles += s.launch->htiles;
        wchunks += s.launch->wchunks;
        g.gc_ops = ops + s.launch->begin;
        g.n_gc = s.launch->xbegin - s.launch->begin;
        g.rt_ops = ops + s.launch->rbegin;
        g.rt_unit_op = s.launch->rtunit_begin != NO_ITEMS
                           ? (const uint32_t*)(s.ws + L.item_op) + s.launch->rtunit_begin
                           : nullptr;
        g.n_rt = s.launch->rend - s.launch->rbegin;
        g.rt_start = rtblocks;
        rtblocks += s.launch->rblocks;
        g.gs_ops = ops + s.launch->xbegin;
        g.n_gs = s.launch->end - s.launch->xbegin;
        g.gs_start = gswork;
        gswork += s.launch->xwork;
        g.tab = (const uint32_t*)(s.ws + L.tabs);
        g.item_op = s.launch->item_begin != NO_ITEMS
                        ? (const uint32_t*)(s.ws + L.item_op) + s.launch->item_begin
                        : nullptr;
        g.arena = (float2*)(s.ws + L.arena);
        g.split = SplitK{(float*)(s.ws + L.split)};
        g.sunits = (const DevSplitUnit*)(s.ws + L.sunits) + s.launch->sbegin;
        g.n_split = s.launch->send - s.launch->sbegin;
        g.split_start = sunits;
        sunits += g.n_split;
        g.gsunits = (const DevSplitUnit*)(s.ws + L.gsunits) + s.launch->gsbegin;
        g.n_gsplit = s.launch->gsend - s.launch->gsbegin;
        g.gsplit_start = gsunits;
        gsunits += g.n_gsplit;
        g.gemm_start = tiles;
        g.wave_start = wtiles;
        g.gc_start = work;
        tiles += s.launch->tiles;
        wtiles += s.launch->wtiles;
        work += (s.launch->work + 63) & ~uint64_t(63);
      }
      a.nseg = (uint32_t)nseg;
      a.gemm_tiles = tiles;
      a.wave_tiles = wtiles;
      a.split_units = sunits;
      a.gsplit_units = gsunits;
      a.gc_work = work;
      a.gs_work = gswork;
      a.wide_tiles = htiles;
      a.wide_chunks = wchunks;
      a.rt_blocks = rtblocks;
      a.tile_blocks = (unsigned)std::min<uint64_t>(tiles, (uint64_t)n_cu * 8);
      const unsigned wvb = (unsigned)std::min<uint64_t>((wtiles + 3) / 4, (uint64_t)n_cu * 16);
      const unsigned gmb = (parts & PART_GEMM) ? a.tile_blocks + wvb : 0u;
      const unsigned whb = (parts & PART_WIDE) ? (unsigned)std::min<uint64_t>(htiles, (uint64_t)n_cu) : 0u;
      const unsigned gcb = (parts & PART_GATHER) && work ? grid_for(work, 256, n_cu) : 0u;
      bool deep = false;  // any merged level asking for the deep unroll
      for (int i = 0; i < nseg; ++i) deep = deep || segs[i].launch->deep_gather;
      // XCD order pays at batch 1, where an op's items read the same small
      // operands (batched levels measured slower with it: each row's
      // operands are its own)
      a.xcd_order = 1;
      for (int i = 0; i < nseg; ++i) a.xcd_order = a.xcd_order && segs[i].plan->batch == 1;
      const unsigned gsb = (parts & PART_GSPLIT) && gswork ? grid_for(gswork, 256, n_cu) : 0u;
      const unsigned rtb = (parts & PART_ROWTILE) ? (unsigned)rtblocks : 0u;
      auto gemm = [&](hipStream_t st) {
        if (whb) {
          // the operands' planes first
          if (precision == TC_PREC_BF16X3) {
            launch(k_split_wide<TC_PREC_BF16X3>, dim3(grid_for(wchunks, 256, n_cu)), dim3(256), st, a);
            launch(k_gemm_wide<TC_PREC_BF16X3>, dim3(whb), dim3(256), st, a);
          } else {
            launch(k_split_wide<TC_PREC_C64>, dim3(grid_for(wchunks, 256, n_cu)), dim3(256), st, a);
            launch(k_gemm_wide<TC_PREC_C64>, dim3(whb), dim3(256), st, a);
          }
        }
        if (!gmb) return;
        if (precision == TC_PREC_BF16X3)
          launch(k_gemm<TC_PREC_BF16X3>, dim3(gmb), dim3(256), st, a);
        else
          launch(k_gemm<TC_PREC_C64>, dim3(gmb), dim3(256), st, a);
        // split-K tiles: their slices are all written once k_gemm is done
        if (a.split_units)
          launch(k_reduce, dim3((unsigned)a.split_units), dim3(256), st, a);
      };
      auto gather = [&](hipStream_t st) {
        if (gcb && deep)
          launch(k_gather<false, true>, dim3(gcb), dim3(256), st, a);
        else if (gcb)
          launch(k_gather<false, false>, dim3(gcb), dim3(256), st, a);
        if (rtb) launch(k_rowtile, dim3(rtb), dim3(256), st, a);
        if (gsb) {
          launch(k_gather<true, true>, dim3(gsb), dim3(256), st, a);
          // split sums: their slices are all written once k_gather is done
          launch(k_reduce_g, dim3((unsigned)a.gsplit_units), dim3(256), st, a);
        }
      };
      if (gmb || whb) gemm(stream);
      if (gcb || gsb || rtb) gather(stream);
      break;
    }
    case L_TERM: {
      if (nseg != 1) fail(TC_ERR_INVALID_ARG, "internal: term mode runs one plan per launch");
      const SegRef& s = segs[0];
      const WorkspaceLayout& L = *s.lay;
      const Plan& P = *s.plan;
      if (P.terms.empty()) return;
      TermArgs a{};
      a.terms = (const DevTerm*)(s.ws + L.terms);
      a.ranges = (const DevRange*)(s.ws + L.ranges) + s.launch->begin;
      a.groups = (const DevGroup*)(s.ws + L.groups);
      a.ops = (const DevOp*)(s.ws + L.ops);
      a.tab = (const uint32_t*)(s.ws + L.tabs);
      a.item_op = (const uint32_t*)(s.ws + L.item_op);
      a.item_leaf = s.launch->item_begin != NO_ITEMS
                        ? (const uint32_t*)(s.ws + L.item_op) + s.launch->item_begin
                        : nullptr;
      a.leaves = (const DevLeaf*)(s.ws + L.leaves);
      a.ftab = (const float*)(s.ws + L.ftab);
      a.params = s.params ? s.params : (const float*)(s.ws + L.params);
      a.arena = (float2*)(s.ws + L.arena);
      a.param_stride = P.param_stride();
      a.with_leaves = s.launch->with_leaves ? 1 : 0;
      if (s.launch->resident) {
        a.rops = (const DevROp*)(s.ws + L.rops);
        launch_shm(k_term_res, dim3((unsigned)P.terms.size()), dim3(1024),
                   (size_t)P.lds_elems * sizeof(float2), stream, a);
      } else {
        launch(k_term, dim3((unsigned)P.terms.size()), dim3(1024), stream, a);
      }
      break;
    }
    case L_ROOT: {
      const RootArgs a = root_args(segs, nseg);
      launch(k_root, dim3((unsigned)((a.total * 64 + 255) / 256)), dim3(256), stream, a);
      break;
    }
    case L_GRAD: {
      const GradArgs a = grad_args(segs, nseg);
      if (a.total == 0) return;
      launch(k_grad, dim3(grid_for(a.total * 64, 256, n_cu)), dim3(256), stream, a);
      break;
    }
    case L_QGT: {
      if (nseg != 1) fail(TC_ERR_INVALID_ARG, "internal: one plan per geometric tensor launch");
      const SegRef& s = segs[0];
      const WorkspaceLayout& L = *s.lay;
      QgtArgs a{};
      a.value = (const double*)(s.ws + L.value);
      a.sums = (const double*)(s.ws + L.grad);
      a.slot_begin = (const uint32_t*)(s.ws + L.qslot);
      a.rows = (const uint32_t*)(s.ws + L.qrows);
      a.out = (double*)(s.ws + L.qgt);
      a.n_params = s.plan->n_params;
      const uint64_t waves = (uint64_t)a.n_params * a.n_params;
      if (!waves) return;
      launch(k_qgt, dim3((unsigned)((waves * 64 + 255) / 256)), dim3(256), stream, a);
      break;
    }
    default:
      fail(TC_ERR_INVALID_ARG, "internal: unknown launch kind");
  }
  HIP_CHECK(hipGetLastError());
}

static void enqueue(const Plan& P, DeviceState& D, const std::vector<const Launch*>& seq,
                    int parts = PART_ALL, const float* params = nullptr,
                    double* value_re = nullptr, double* grad = nullptr) {
  for (size_t i = 0; i < seq.size(); ++i) {
    const Launch* x = seq[i];
    SegRef s{&P, D.ws, &D.lay, x, params, value_re, grad};
    if (x->kind == L_ROOT && i + 2 == seq.size() && seq[i + 1]->kind == L_GRAD) {
      // a gradient call ends with the root sum and the gradient sum, which
      // do not depend on each other: one launch
      const SegRef sg{&P, D.ws, &D.lay, seq[i + 1], params, value_re, grad};
      launch_root_grad(s, sg, D.stream, D.n_cu);
      break;
    }
    launch_segments(x->kind, &s, 1, D.stream, D.n_cu, P.precision, parts);
  }
}

template <typename T>
static void upload(char* ws, uint64_t off, const std::vector<T>& v, hipStream_t stream) {
  if (v.empty()) return;
  HIP_CHECK(hipMemcpyAsync(ws + off, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice,
                           stream));
}

void upload_tables(const Plan& P, char* ws, const WorkspaceLayout& lay, hipStream_t stream) {
  upload(ws, lay.ops, P.ops, stream);
  upload(ws, lay.tabs, P.tabs, stream);
  upload(ws, lay.item_op, P.item_op, stream);
  upload(ws, lay.leaves, P.leaves, stream);
  upload(ws, lay.ftab, P.ftab, stream);
  upload(ws, lay.uses, P.uses, stream);
  upload(ws, lay.slot_begin, P.slot_begin, stream);
  upload(ws, lay.roots, P.roots, stream);
  upload(ws, lay.terms, P.terms, stream);
  upload(ws, lay.groups, P.groups, stream);
  upload(ws, lay.ranges, P.ranges, stream);
  upload(ws, lay.rops, P.rops, stream);
  upload(ws, lay.sunits, P.split_units, stream);
  upload(ws, lay.gsunits, P.gsplit_units, stream);
  upload(ws, lay.qslot, P.qslot_begin, stream);
  upload(ws, lay.qrows, P.qrows, stream);
  upload(ws, lay.arena, P.seeds, stream);  // seeds sit at arena offset 0
}

// ------------------------------------------------------------------ device state

static void release(DeviceState* D) {
  if (!D) return;
  // teardown: errors here cannot be reported to anyone, so they are dropped
  (void)hipSetDevice(D->device);
  if (D->stream) (void)hipStreamSynchronize(D->stream);
  for (int i = 0; i < 2; ++i) {
    if (D->exec[i]) (void)hipGraphExecDestroy(D->exec[i]);
    if (D->graph[i]) (void)hipGraphDestroy(D->graph[i]);
  }
  if (D->dexec) (void)hipGraphExecDestroy(D->dexec);
  if (D->dgraph) (void)hipGraphDestroy(D->dgraph);
  if (D->ws_owned && D->ws) (void)hipFree(D->ws);
  if (D->own_stream && D->stream) (void)hipStreamDestroy(D->stream);
  delete D;
}

static void capture(const Plan& P, DeviceState& D, int which) {
  const std::vector<const Launch*> seq = launch_order(P, which == 1);
  HIP_CHECK(hipStreamBeginCapture(D.stream, hipStreamCaptureModeThreadLocal));
  try {
    enqueue(P, D, seq);
  } catch (...) {
    hipGraph_t g = nullptr;
    (void)hipStreamEndCapture(D.stream, &g);
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  HIP_CHECK(hipStreamEndCapture(D.stream, &D.graph[which]));
  HIP_CHECK(hipGraphInstantiate(&D.exec[which], D.graph[which], nullptr, nullptr, 0));
}

// The gradient graph for caller buffers: captured again whenever the three
// pointers differ from the last call's.
static void run_direct(const Plan& P, DeviceState& D, const float* params, double* value,
                       double* grad) {
  if (!D.dexec || D.dkey[0] != params || D.dkey[1] != value || D.dkey[2] != grad) {
    // the previous graph may still run on the stream: let it finish first
    if (D.dexec) HIP_CHECK(hipStreamSynchronize(D.stream));
    if (D.dexec) HIP_CHECK(hipGraphExecDestroy(D.dexec));
    if (D.dgraph) HIP_CHECK(hipGraphDestroy(D.dgraph));
    D.dexec = nullptr;
    D.dgraph = nullptr;
    D.dkey[0] = D.dkey[1] = D.dkey[2] = nullptr;
    const std::vector<const Launch*> seq = launch_order(P, true);
    HIP_CHECK(hipStreamBeginCapture(D.stream, hipStreamCaptureModeThreadLocal));
    try {
      enqueue(P, D, seq, PART_ALL, params, value, grad);
    } catch (...) {
      hipGraph_t g = nullptr;
      (void)hipStreamEndCapture(D.stream, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    HIP_CHECK(hipStreamEndCapture(D.stream, &D.dgraph));
    HIP_CHECK(hipGraphInstantiate(&D.dexec, D.dgraph, nullptr, nullptr, 0));
    D.dkey[0] = params;
    D.dkey[1] = value;
    D.dkey[2] = grad;
  }
  HIP_CHECK(hipGraphLaunch(D.dexec, D.stream));
}

void bind_plan(Plan& P, void* workspace, uint64_t bytes) {
  if (P.dev) fail(TC_ERR_STATE, "plan is already bound");
  auto* D = new DeviceState;
  try {
    D->device = P.device;
    HIP_CHECK(hipSetDevice(P.device));
    D->n_cu = device_cu_count(P.device);
    if (P.user_stream) {
      D->stream = (hipStream_t)P.user_stream;
    } else {
      HIP_CHECK(hipStreamCreateWithFlags(&D->stream, hipStreamNonBlocking));
      D->own_stream = true;
    }
    D->lay = workspace_layout(P);
    if (workspace) {
      if (bytes < D->lay.total)
        fail(TC_ERR_INVALID_ARG, "workspace smaller than workspace_bytes");
      if (((uintptr_t)workspace & 255) != 0) fail(TC_ERR_INVALID_ARG, "workspace not 256-byte aligned");
      D->ws = (char*)workspace;
      D->ws_bytes = bytes;
    } else {
      hipError_t e = hipMalloc(&D->ws, D->lay.total);
      if (e != hipSuccess) {
        (void)hipGetLastError();
        fail(TC_ERR_OUT_OF_MEMORY, "hipMalloc of the workspace failed");
      }
      D->ws_owned = true;
      D->ws_bytes = D->lay.total;
    }
    upload_tables(P, D->ws, D->lay, D->stream);
    HIP_CHECK(hipStreamSynchronize(D->stream));
    capture(P, *D, 0);
    if (P.want_grad) capture(P, *D, 1);
  } catch (...) {
    release(D);
    throw;
  }
  P.dev = D;
}

struct BusyGuard {
  std::atomic<int>& f;
  explicit BusyGuard(std::atomic<int>& x) : f(x) {
    int expect = 0;
    if (!f.compare_exchange_strong(expect, 1)) fail(TC_ERR_BUSY, "plan has a call in flight");
  }
  ~BusyGuard() { f.store(0); }
};

static void stage_params(Plan& P, const float* params) {
  if (!params) fail(TC_ERR_INVALID_ARG, "params is NULL");
  if (!P.dev) bind_plan(P, nullptr, 0);
  DeviceState& D = *P.dev;
  HIP_CHECK(hipSetDevice(D.device));
  uint64_t pbytes = (P.qgt ? 1 : (uint64_t)P.batch) * P.n_params * sizeof(float);
  if (pbytes)
    HIP_CHECK(hipMemcpyAsync(D.ws + D.lay.params, params, pbytes, hipMemcpyDeviceToDevice,
                             D.stream));
}

void contract(Plan& P, const float* params, double* out, bool device_out) {
  if (P.qgt) fail(TC_ERR_STATE, "a geometric tensor plan runs through tc_contract_qgt");
  BusyGuard g(P.busy);
  stage_params(P, params);
  DeviceState& D = *P.dev;
  HIP_CHECK(hipGraphLaunch(D.exec[0], D.stream));
  HIP_CHECK(hipMemcpyAsync(out, D.ws + D.lay.value, (uint64_t)P.batch * 16,
                           device_out ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                           D.stream));
  if (!device_out) HIP_CHECK(hipStreamSynchronize(D.stream));
}

void contract_grad(Plan& P, const float* params, double* value, double* grad,
                   bool device_out) {
  if (!P.want_grad) fail(TC_ERR_STATE, "plan was compiled without want_grad");
  if (P.qgt) fail(TC_ERR_STATE, "a geometric tensor plan runs through tc_contract_qgt");
  BusyGuard g(P.busy);
  if (device_out && value && grad && params && P.n_params > 0) {
    // caller buffers on the device: the graph reads and writes them in
    // place (no staging copies around it), unless the caller is capturing
    // the plan's stream (a capture cannot be started inside another)
    if (!P.dev) bind_plan(P, nullptr, 0);
    DeviceState& D = *P.dev;
    HIP_CHECK(hipSetDevice(D.device));
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIP_CHECK(hipStreamIsCapturing(D.stream, &cs));
    if (cs == hipStreamCaptureStatusNone) {
      run_direct(P, D, params, value, grad);
      return;
    }
  }
  stage_params(P, params);
  DeviceState& D = *P.dev;
  HIP_CHECK(hipGraphLaunch(D.exec[1], D.stream));
  hipMemcpyKind kind = device_out ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  if (value)
    HIP_CHECK(hipMemcpy2DAsync(value, sizeof(double), D.ws + D.lay.value, 2 * sizeof(double),
                               sizeof(double), (size_t)P.batch, kind, D.stream));
  if (grad && P.n_params)
    HIP_CHECK(hipMemcpyAsync(grad, D.ws + D.lay.grad,
                             (uint64_t)P.batch * P.n_params * sizeof(double), kind, D.stream));
  if (!device_out) HIP_CHECK(hipStreamSynchronize(D.stream));
}

void contract_qgt(Plan& P, const float* params, double* out) {
  if (!P.qgt) fail(TC_ERR_STATE, "plan was compiled without qgt");
  BusyGuard g(P.busy);
  stage_params(P, params);
  DeviceState& D = *P.dev;
  HIP_CHECK(hipGraphLaunch(D.exec[1], D.stream));
  const uint64_t n = 2 * (uint64_t)P.n_params * P.n_params;
  if (n)
    HIP_CHECK(hipMemcpyAsync(out, D.ws + D.lay.qgt, n * sizeof(double), hipMemcpyDeviceToHost,
                             D.stream));
  HIP_CHECK(hipStreamSynchronize(D.stream));
}

void profile(Plan& P, const float* params, int which, int reps, int cap, int* n_out,
             int* kinds, double* ms, double* flops, double* bytes) {
  if (which == 1 && !P.want_grad) fail(TC_ERR_STATE, "plan was compiled without want_grad");
  if (reps < 1) fail(TC_ERR_INVALID_ARG, "reps must be >= 1");
  BusyGuard g(P.busy);
  stage_params(P, params);
  DeviceState& D = *P.dev;
  const std::vector<const Launch*> all = launch_order(P, which == 1);
  // one entry per kernel: a level contributes its GEMM and gather kernels
  struct Entry {
    const Launch* Lp;
    int kind, parts;
    double flops, bytes;
  };
  std::vector<Entry> seq;
  for (const Launch* Lp : all) {
    const Launch& L = *Lp;
    if (L.kind != L_LEVEL) {
      seq.push_back({Lp, L.kind, PART_ALL, L.flops, L.bytes});
      continue;
    }
    if (L.htiles) seq.push_back({Lp, PROF_WIDE, PART_WIDE, L.wide_flops, L.wide_bytes});
    if (L.tiles || L.wtiles)
      seq.push_back({Lp, PROF_GEMM, PART_GEMM, L.gemm_flops - L.wide_flops,
                     L.gemm_bytes - L.wide_bytes});
    if (L.work)
      seq.push_back({Lp, PROF_GATHER, PART_GATHER, L.flops - L.gemm_flops - L.rt_flops - L.gs_flops,
                     L.bytes - L.gemm_bytes - L.rt_bytes - L.gs_bytes});
    if (L.rblocks) seq.push_back({Lp, PROF_ROWTILE, PART_ROWTILE, L.rt_flops, L.rt_bytes});
    if (L.xwork) seq.push_back({Lp, PROF_GSPLIT, PART_GSPLIT, L.gs_flops, L.gs_bytes});
  }
  // per entry: the start of its first kernel to the end of its last, as
  // stamped by the kernel dispatches (no queueing gap between launches)
  std::vector<hipEvent_t> ev(2 * seq.size(), nullptr);
  std::vector<double> acc(seq.size(), 0.0);
  std::vector<char> ran(seq.size(), 0);
  try {
    for (auto& e : ev) HIP_CHECK(hipEventCreate(&e));
    for (int r = 0; r < reps; ++r) {
      for (size_t i = 0; i < seq.size(); ++i) {
        ProfEvents pe{ev[2 * i], ev[2 * i + 1], false};
        t_prof = &pe;
        try {
          enqueue(P, D, std::vector<const Launch*>{seq[i].Lp}, seq[i].parts);
        } catch (...) {
          t_prof = nullptr;
          throw;
        }
        t_prof = nullptr;
        ran[i] = pe.started;
      }
      HIP_CHECK(hipStreamSynchronize(D.stream));
      for (size_t i = 0; i < seq.size(); ++i) {
        if (!ran[i]) continue;
        float t = 0;
        HIP_CHECK(hipEventElapsedTime(&t, ev[2 * i], ev[2 * i + 1]));
        acc[i] += t;
      }
    }
  } catch (...) {
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
    throw;
  }
  for (auto& e : ev) (void)hipEventDestroy(e);
  *n_out = (int)seq.size();
  for (size_t i = 0; i < seq.size() && (int)i < cap; ++i) {
    if (kinds) kinds[i] = seq[i].kind;
    if (ms) ms[i] = acc[i] / reps;
    if (flops) flops[i] = seq[i].flops;
    if (bytes) bytes[i] = seq[i].bytes;
  }
}

void free_device(Plan& P) {
  release(P.dev);
  P.dev = nullptr;
}

// ------------------------------------------------------------------ static scratch
//
// Workspace for callers that cannot allocate device memory: one array per
// GPU, reserved when the code object is loaded and held until the process
// ends.  Host code never passes `scratch` itself to a kernel or a copy (on
// the host it names a stand-in, not the device copy); it uses the device
// address that hipGetSymbolAddress returns for the current device.

static __device__ __align__(256) char scratch[TC_NOALLOC_MAX_BYTES];

struct ScratchSlot {
  char* ptr = nullptr;
  int n_cu = 0;
};
constexpr int MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static ScratchSlot g_scratch[MAX_DEVICES];

// The calling thread's current device must be `device`.
static ScratchSlot scratch_slot(int device) {
  if (device < 0 || device >= MAX_DEVICES) fail(TC_ERR_INVALID_ARG, "device ordinal out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  ScratchSlot& s = g_scratch[device];
  if (!s.ptr) {
    void* p = nullptr;
    HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p || ((uintptr_t)p & 255) != 0) fail(TC_ERR_DEVICE, "scratch array has no usable address");
    int cu = 0;
    HIP_CHECK(hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, device));
    s.n_cu = cu > 0 ? cu : 256;
    s.ptr = (char*)p;
  }
  return s;
}

void contract_grad_noalloc(Plan& P, const float* params, double* value_dev, double* grad_dev) {
  if (!P.want_grad) fail(TC_ERR_STATE, "plan was compiled without want_grad");
  if (P.qgt) fail(TC_ERR_STATE, "a geometric tensor plan runs through tc_contract_qgt");
  if (!params) fail(TC_ERR_INVALID_ARG, "params is NULL");
  const WorkspaceLayout lay = workspace_layout(P);
  if (lay.total > TC_NOALLOC_MAX_BYTES)
    fail(TC_ERR_TOO_LARGE, "plan needs " + std::to_string(lay.total) +
                               " bytes of workspace, more than the static scratch holds (" +
                               std::to_string((uint64_t)TC_NOALLOC_MAX_BYTES) + ")");
  BusyGuard g(P.busy);
  HIP_CHECK(hipSetDevice(P.device));
  const ScratchSlot s = scratch_slot(P.device);
  hipStream_t st = (hipStream_t)P.user_stream;
  // the tables of whichever plan ran here last are replaced; every value
  // the kernels read is either uploaded here or written by an earlier
  // kernel of this call, so nothing needs clearing
  upload_tables(P, s.ptr, lay, st);
  const uint64_t pbytes = (uint64_t)P.batch * P.n_params * sizeof(float);
  if (pbytes)
    HIP_CHECK(hipMemcpyAsync(s.ptr + lay.params, params, pbytes, hipMemcpyDeviceToDevice, st));
  for (const Launch* x : launch_order(P, true)) {
    SegRef r{&P, s.ptr, &lay, x};
    launch_segments(x->kind, &r, 1, st, s.n_cu, P.precision);
  }
  if (value_dev)
    HIP_CHECK(hipMemcpy2DAsync(value_dev, sizeof(double), s.ptr + lay.value, 2 * sizeof(double),
                               sizeof(double), (size_t)P.batch, hipMemcpyDeviceToDevice, st));
  if (grad_dev && P.n_params)
    HIP_CHECK(hipMemcpyAsync(grad_dev, s.ptr + lay.grad,
                             (uint64_t)P.batch * P.n_params * sizeof(double),
                             hipMemcpyDeviceToDevice, st));
}

}  // namespace tcx

// ------------------------------------------------------------------ C ABI

#define TC_GUARD_BEGIN try {
#define TC_GUARD_END                                               \
  }                                                                \
  catch (const tcx::Error& e) {                                    \
    tcx::set_error(e.msg);                                         \
    return e.status;                                               \
  }                                                                \
  catch (const std::bad_alloc&) {                                  \
    tcx::set_error("host allocation failed");                      \
    return TC_ERR_OUT_OF_MEMORY;                                   \
  }                                                                \
  catch (const std::exception& e) {                                \
    tcx::set_error(std::string("internal error: ") + e.what());    \
    return TC_ERR_INVALID_ARG;                                     \
  }

extern "C" {

tc_status tc_plan_create(const tc_network* net, const tc_path* path,
                         const tc_plan_opts* opts, tc_plan** out) {
  TC_GUARD_BEGIN
  if (!net || !path || !out) tcx::fail(TC_ERR_INVALID_ARG, "NULL argument");
  tc_plan_opts o{0, 1, 0, 0, 0, nullptr, 0, 0, 0, 0, 0, 0};
  if (opts) o = *opts;
  if (o.gemm_min_k < 0) tcx::fail(TC_ERR_INVALID_ARG, "gemm_min_k must be >= 0");
  if (o.exec_mode < 0 || o.exec_mode > 3) tcx::fail(TC_ERR_INVALID_ARG, "exec_mode must be 0, 1, 2 or 3");
  // resident term launches size their LDS arena from the device
  const uint32_t lds_elems =
      (o.exec_mode == 0 || o.exec_mode == 3) && o.batch == 1 && !o.qgt ? tcx::resident_lds_elems(o.device) : 0;
  if (o.tile_mode < 0 || o.tile_mode > 2) tcx::fail(TC_ERR_INVALID_ARG, "tile_mode must be 0, 1 or 2");
  if (o.checkpoint_every < -1 || o.checkpoint_every == 1)
    tcx::fail(TC_ERR_INVALID_ARG, "checkpoint_every must be -1, 0 or >= 2");
  if (o.batch < 1 || o.batch > (1 << 20)) tcx::fail(TC_ERR_INVALID_ARG, "batch must be in 1..2^20");
  if (o.precision != TC_PREC_C64 && o.precision != TC_PREC_BF16X3)
    tcx::fail(TC_ERR_UNSUPPORTED, "unknown precision");
  auto make = [&](int32_t wide_tiles) {
    auto* p = new tc_plan;
    p->p.precision = o.precision;
    p->p.batch = o.batch;
    p->p.want_grad = o.want_grad ? 1 : 0;
    p->p.device = o.device;
    p->p.budget = o.mem_budget_bytes;
    p->p.user_stream = o.stream;
    if (o.gemm_min_k > 0) p->p.gemm_min_k = o.gemm_min_k;
    if (o.gemm_min_macs > 0) p->p.gemm_min_macs = o.gemm_min_macs;
    p->p.exec_mode = o.exec_mode;
    p->p.lds_elems = lds_elems;
    p->p.wide_tiles = wide_tiles;
    p->p.checkpoint = o.checkpoint_every;
    p->p.qgt = o.qgt ? 1 : 0;
    try {
      tcx::build_plan(p->p, tcx::network_of(net), tcx::path_of(path));
    } catch (...) {
      delete p;
      throw;
    }
    return p;
  };
  const int32_t wide = o.tile_mode == 0 ? 1 : (o.tile_mode == 1 ? 0 : 2);
  try {
    *out = make(wide);
  } catch (const tcx::Error& e) {
    // under a memory budget the wide tiles' operand planes may be what does
    // not fit; the 64 x 64 tiles need none
    if (e.status != TC_ERR_TOO_LARGE || wide != 1 || !o.mem_budget_bytes) throw;
    *out = make(0);
  }
  return TC_OK;
  TC_GUARD_END
}

void tc_plan_free(tc_plan* plan) {
  if (!plan) return;
  tcx::free_device(plan->p);
  delete plan;
}

tc_status tc_plan_info_get(const tc_plan* plan, tc_plan_info* out) {
  TC_GUARD_BEGIN
  if (!plan || !out) tcx::fail(TC_ERR_INVALID_ARG, "NULL argument");
  *out = plan->p.info;
  return TC_OK;
  TC_GUARD_END
}

tc_status tc_plan_bind(tc_plan* plan, void* workspace, uint64_t bytes) {
  TC_GUARD_BEGIN
  if (!plan) tcx::fail(TC_ERR_INVALID_ARG, "NULL argument");
  tcx::bind_plan(plan->p, workspace, bytes);
  return TC_OK;
  TC_GUARD_END
}

tc_status tc_contract(tc_plan* plan, const float* params, double* out) {
  TC_GUARD_BEGIN
  if (!plan || !out) tcx::fail(TC_ERR_INVALID_ARG, "NULL argument");
  tcx::contract(plan->p, params, out, false);
  return TC_OK;
  TC_GUARD_END
}

tc_status tc_contract_grad(tc_plan* plan, const float* params, double* value, double* grad) {
  TC_GUARD_BEGIN
  if (!plan) tcx::fail(TC_ERR_INVALID_ARG, "NULL argument");
  tcx::contract_grad(plan->p, params, value, grad, false);
  return TC_OK;
  TC_GUARD_END
}

tc_status tc_contract_device(tc_plan* plan, const float* params, double* out_dev) {
  TC_GUARD_BEGIN
  if (!plan || !out_dev) tcx::fail(TC_ERR_INVALID_ARG, "NULL argument");
  tcx::contract(plan->p, params, out_dev, true);
  return TC_OK;
  TC_GUARD_END
}

tc_status tc_contract_grad_device(tc_plan* plan, const float* params, double* value_dev,
                                  double* grad_dev) {
  TC_GUARD_BEGIN
  if (!plan) tcx::fail(TC_ERR_INVALID_ARG, "NULL argument");
  tcx::contract_grad(plan->p, params, value_dev, grad_dev, true);
  return TC_OK;
  TC_GUARD_END
}

tc_status tc_contract_qgt(tc_plan* plan, const float* params, double* qgt) {
  TC_GUARD_BEGIN
  if (!plan || !params || !qgt) tcx::fail(TC_ERR_INVALID_ARG, "NULL argument");
  tcx::contract_qgt(plan->p, params, qgt);
  return TC_OK;
  TC_GUARD_END
}

tc_status tc_contract_grad_device_noalloc(tc_plan* plan, const float* params,
                                          double* value_dev, double* grad_dev) {
  TC_GUARD_BEGIN
  if (!plan) tcx::fail(TC_ERR_INVALID_ARG, "NULL argument");
  tcx::contract_grad_noalloc(plan->p, params, value_dev, grad_dev);
  return TC_OK;
  TC_GUARD_END
}

tc_status tc_plan_profile(tc_plan* plan, const float* params, int32_t which, int32_t reps,
                          int32_t cap, int32_t* n_launches, int32_t* kinds, double* ms,
                          double* flops, double* bytes) {
  TC_GUARD_BEGIN
  if (!plan || !params || !n_launches) tcx::fail(TC_ERR_INVALID_ARG, "NULL argument");
  tcx::profile(plan->p, params, which, reps, cap, n_launches, kinds, ms, flops, bytes);
  return TC_OK;
  TC_GUARD_END
}

}  // extern "C"
