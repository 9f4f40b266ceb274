// Plain-data descriptors shared by the host planner and the HIP kernels.
//
// Tensor storage: complex64 (float2) elements; a tensor of rank r holds 2^r
// entries whose index bits follow its leg list (first leg = most
// significant bit).  A batched tensor is stored as [batch][2^r]; an
// unbatched one holds one copy that every batch row reads (batch stride 0).
// Offsets are in complex64 elements from the arena base.
#pragma once
#include <stdint.h>

namespace tcx {

// One pairwise contraction C[m, n] = sum_k A[m, k] B[k, n] over index-
// permuted operands: element (m, k) of A lives at A + tab[a_m + m] +
// tab[a_k + k]; element (k, n) of B at B + tab[b_k + k] + tab[b_n + n];
// element (m, n) of C at C + tab[c_m + m] + tab[c_n + n].  Batch row r adds
// r * a_bs, r * b_bs, r * c_bs.
// Index descriptor of one index group (the m, k or n legs of an operand):
// maps an index i over the group (first leg most significant) to the
// element offset of that index inside the tensor.
//   bit 31 set:   table; offset(i) = tab[(d & 0x7fffffff) + i]
//   bit 31 clear: up to IX_RUNS bit-field runs, run r in bits [10 r, 10 r + 10)
//                 as len (5 bits) | dst (5 bits) << 5, run 0 on the lowest
//                 index bits: with s_r = len_0 + ... + len_(r-1),
//                 offset(i) = OR_r ((i >> s_r) & (2^len_r - 1)) << dst_r
//                 (a run of len 0 contributes nothing).
// A run is a stretch of the group's legs that sits, in the same order, on
// consecutive bits of the tensor.  Nearly every group needs one to three
// runs (three when two legs are taken out of the middle of a tensor, as
// when a gate meets a state) and no memory at all; tables remain for the
// more permuted ones.
constexpr int IX_RUNS = 3;
constexpr uint32_t OPF_WIDE = 1u << 14;  // op flag: 128 x 128 GEMM tiles
// op flag, wave tiles without index tables: A's k index is the lowest bits
// of A (k contiguous) and A's offsets are even, so a lane reads four
// consecutive k of a row with two 16-byte loads
constexpr uint32_t OPF_AVEC = 1u << 15;
constexpr uint32_t IX_TABLE = 0x80000000u;

struct DevOp {
  uint64_t a, b, c;        // arena element offsets
  uint64_t work0;          // first work item of this op inside its launch
  uint32_t a_bs, b_bs, c_bs;  // batch strides in elements (0 = shared)
  uint32_t M, N, K;
  uint32_t a_m, a_k, b_k, b_n, c_m, c_n;  // index descriptors
  uint32_t rows;           // batch rows covered (1 if nothing is batched)
  uint32_t tiles_m, tiles_n;  // GEMM path: tile grid per batch row
  uint32_t flags;          // bit 0: A is k-contiguous; bit 1: B is k-contiguous;
                           // gather k-split (bits 4-6) and n-vector (8-9);
                           // wave-tile blocks (12, 13); 128 x 128 tiles (14)
  // GEMM split-K: K is cut into ksplit slices (1 = none); slice results go
  // to partial tiles from float `part` of the split region
  uint64_t part;
  uint32_t ksplit;
};

// One output tile of a split-K GEMM op for the reduction kernel: the op
// (index among the level's GEMM ops, block tiles first, then wave tiles)
// and the tile within it.
struct DevSplitUnit {
  uint32_t op;
  uint32_t tile;
};

// Term launches: one workgroup runs one term's nodes over a run of steps.
// A group is the term's gather ops at one step (between two workgroup
// barriers); a range names one term's groups in one term launch.
struct DevGroup {
  uint32_t op_begin, op_end;  // ops in the op table, work0 relative to the group
  uint64_t items;             // gather items (a multiple of 64)
  uint64_t item_base;         // first entry in the per-item op table
};

struct DevRange {
  uint32_t g_begin, g_end;
};

// Resident term launch: one workgroup runs a term's whole forward pass and
// reverse sweep, with the tensors the planner places there in the
// workgroup's LDS arena and the rest in the global arena.  A node of such
// a launch (no batch axis; M = 2^lm, N = 2^ln, K = 2^lk):
//   a, b, c   element offsets, each in the LDS arena when its RES_*_LDS
//             flag is set, else in the global arena;
//   c2        global arena offset of a second copy of C (RES_C2): a value
//             that later steps read from global memory once its LDS copy
//             is released;
//   work0     first gather item within its group;
//   shape     lm | ln << 5 | lk << 10 | ls << 15 | lv << 18 | flags.
constexpr uint32_t RES_A_LDS = 1u << 21, RES_B_LDS = 1u << 22, RES_C_LDS = 1u << 23,
                   RES_C2 = 1u << 24, RES_TABLES = 1u << 25;
struct DevROp {
  uint32_t a, b, c, c2;
  uint32_t work0;
  uint32_t a_m, a_k, b_k, b_n, c_m, c_n;
  uint32_t shape;
};

struct DevTerm {
  uint64_t leaf_work0, leaf_work_end;  // the term's leaf entries (leaf work items)
  uint32_t leaf_begin, leaf_end;       // the term's leaves
};

enum : int32_t {
  DLEAF_GATE = 0, DLEAF_KET0 = 1, DLEAF_BRA = 2, DLEAF_PAULI = 3, DLEAF_MPO = 4
};

struct DevLeaf {
  uint64_t out;            // arena element offset
  uint64_t work0;          // first work item (batch row * elems + e)
  int32_t kind;            // DLEAF_*
  int32_t gkind;           // tc_gate_kind for gate leaves
  int32_t part;            // 0 whole, 1/2 split factors
  int32_t conj;
  int32_t value;           // bit for BRA, Pauli for PAULI
  int32_t rank;
  int32_t param[2];        // parameter slots, -1 = fixed
  float fixed[2];
  uint32_t rows;           // batch rows written (1 = shared)
  uint32_t mat;            // offset in the float table: 32 floats (U1/U2), or
                           // 2^(rank+1) (the entries of an MPO site)
  int32_t dsel[2];         // batch row that takes d/d(angle a) instead of the
                           // gate (geometric tensor plans), -1 none
  uint32_t lds_out;        // resident term launches: LDS arena offset
  uint32_t where;          // resident term launches: bit 0 written at `out`
                           // (global arena), bit 1 at `lds_out` (LDS)
};

// d(term root)/d(angle) for one leaf use: sum_e adj[e] * dleaf[e]/dangle
struct DevGradUse {
  uint64_t adj;            // arena element offset of the leaf's adjoint
  uint32_t adj_bs;         // batch stride of the adjoint
  uint32_t leaf;           // index into the leaf table
  int32_t which;           // angle number (0 or 1)
  int32_t slot;            // parameter slot
};

struct DevRoot {
  uint64_t val;            // arena element offset of the term's scalar
  uint32_t bs;             // batch stride (0 = shared)
  int32_t present;         // 0: empty network, value 1
  double weight;
};

}  // namespace tcx
