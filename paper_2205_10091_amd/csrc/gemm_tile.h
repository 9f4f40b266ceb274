// LDS-tiled MFMA complex GEMM tiles for the wider tree nodes (device code,
// included by the executor).
//
// Paper, section "Tensor network engine": each pairwise contraction is
// executed as an einsum / matmul.  A node C[m, n] = sum_k A[m, k] B[k, n]
// is computed here directly from the operands' own layouts: tiles of A and
// B are gathered through the per-op index tables into LDS (no separate
// permute pass), split into real and imaginary planes, and multiplied on
// the matrix cores:
//   FP32:   Cr += Ar Br - Ai Bi, Ci += Ar Bi + Ai Br with
//           v_mfma_f32_16x16x4_f32 (four real products, FP32 accumulate);
//   BF16X3: every real product X Y is taken as Xh Yh + Xh Yl + Xl Yh with
//           X = Xh + Xl split into two bfloat16 numbers (Henry, Tang &
//           Heinecke, "Leveraging the bfloat16 artificial intelligence
//           datatype for higher-precision computations", ARITH 2019),
//           on v_mfma_f32_16x16x32_bf16 with FP32 accumulation.
// A workgroup of four wavefronts computes a 64 x 64 tile of C; each wave a
// 32 x 32 quarter as 2 x 2 blocks of 16 x 16.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "ops.h"

namespace tcx {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f16 __attribute__((ext_vector_type(16)));

// Offset of index i of an index group under its descriptor d (layout in
// ops.h): a table lookup, or the OR of up to IX_RUNS shifted bit fields.
__device__ __forceinline__ uint32_t ix(const uint32_t* __restrict__ tab, uint32_t d, uint32_t i) {
  if (d & IX_TABLE) return tab[(d & ~IX_TABLE) + i];
  uint32_t off = 0, src = 0;
#pragma unroll
  for (int r = 0; r < IX_RUNS; ++r) {
    const uint32_t len = (d >> (10 * r)) & 31u, dst = (d >> (10 * r + 5)) & 31u;
    off |= ((i >> src) & ((1u << len) - 1u)) << dst;
    src += len;
  }
  return off;
}

// The same without the table case: branch-free, for ops whose descriptors
// are all runs (a branch around a table load in an unrolled loop splits it
// into blocks, and the compiler then waits for every load at each join).
__device__ __forceinline__ uint32_t ix_runs(uint32_t d, uint32_t i) {
  uint32_t off = 0, src = 0;
#pragma unroll
  for (int r = 0; r < IX_RUNS; ++r) {
    const uint32_t len = (d >> (10 * r)) & 31u, dst = (d >> (10 * r + 5)) & 31u;
    off |= ((i >> src) & ((1u << len) - 1u)) << dst;
    src += len;
  }
  return off;
}

// ix<TABLES>: TABLES = false for ops without table descriptors
template <bool TABLES>
__device__ __forceinline__ uint32_t ixt(const uint32_t* __restrict__ tab, uint32_t d, uint32_t i) {
  if constexpr (TABLES)
    return ix(tab, d, i);
  else
    return ix_runs(d, i);
}

__device__ __forceinline__ bool op_has_tables(const DevOp& op) {
  return ((op.a_m | op.a_k | op.b_k | op.b_n | op.c_m | op.c_n) & IX_TABLE) != 0;
}

constexpr int BM = 64, BN = 64;
constexpr int BK32 = 16;   // k per LDS stage, FP32 path
constexpr int BK16 = 32;   // k per LDS stage, split-BF16 path
constexpr int PAD = 16;    // row padding (floats) against LDS bank conflicts

struct TileCtx {
  const float2* A;
  const float2* B;
  uint64_t cbase;
  uint32_t m0, n0;
  uint32_t kb, ke;   // this unit's K slice
  uint32_t slice;    // p of ksplit
  uint64_t tile;     // output tile index within the op (row-major over rows, m, n)
};

// Unit u of op (relative to op.work0): slice p fastest, then the tile grid
// (n fastest, then m, then batch row); tile edges tm x tn in elements.
__device__ __forceinline__ TileCtx unit_ctx(const DevOp& op, uint64_t u, const float2* arena,
                                            uint32_t tm_size, uint32_t tn_size) {
  // P, tiles_n and tiles_m are powers of two (checked by the planner)
  const uint32_t P = op.ksplit;
  const uint32_t lp = __builtin_ctz(P), ln = __builtin_ctz(op.tiles_n), lm = __builtin_ctz(op.tiles_m);
  TileCtx t;
  t.slice = (uint32_t)(u & (P - 1));
  uint64_t l = u >> lp;
  t.tile = l;
  const uint32_t tn = (uint32_t)(l & (op.tiles_n - 1));
  l >>= ln;
  const uint32_t tm = (uint32_t)(l & (op.tiles_m - 1));
  const uint64_t r = l >> lm;
  t.A = arena + op.a + r * op.a_bs;
  t.B = arena + op.b + r * op.b_bs;
  t.cbase = op.c + r * op.c_bs;
  t.m0 = tm * tm_size;
  t.n0 = tn * tn_size;
  const uint32_t ks = op.K >> lp;
  t.kb = t.slice * ks;
  t.ke = t.kb + ks;
  return t;
}

__device__ __forceinline__ TileCtx tile_ctx(const DevOp& op, uint64_t tile,
                                            const float2* arena) {
  return unit_ctx(op, tile - op.work0, arena, BM, BN);
}

__device__ __forceinline__ void store_tile(const DevOp& op, const TileCtx& t,
                                           const uint32_t* __restrict__ tab,
                                           float2* __restrict__ arena, const f4 (&cr)[2][2],
                                           const f4 (&ci)[2][2], int wm, int wn, int lane) {
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        uint32_t m = t.m0 + wm * 32 + bi * 16 + 4 * (lane >> 4) + v;
        uint32_t n = t.n0 + wn * 32 + bj * 16 + (lane & 15);
        if (m < op.M && n < op.N)
          arena[t.cbase + ix(tab, op.c_m, m) + ix(tab, op.c_n, n)] =
              make_float2(cr[bi][bj][v], ci[bi][bj][v]);
      }
}

// Split-K partial tiles of one launch (floats).  A slice of a tile writes
// its accumulators there with plain stores; the level's k_reduce kernel,
// launched after the GEMM kernel, adds the slices of every tile in slice
// order and stores C.  The kernel boundary between them makes the partial
// tiles visible, so no slice waits, fences or counts arrivals.
struct SplitK {
  float* part;
};

// Block tile: element j of thread t at j * 256 + t of the slice's partial
// tile (coalesced), j = (block * 2 + re/im) * 4 + v over the 2 x 2 blocks.
__device__ __forceinline__ void write_part_block(const DevOp& op, const TileCtx& c,
                                                 const SplitK& sk, const f4 (&cr)[2][2],
                                                 const f4 (&ci)[2][2]) {
  const int t = threadIdx.x;
  float* mine = sk.part + op.part + (c.tile * op.ksplit + c.slice) * (32 * 256);
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        mine[((i * 2 + j) * 8 + v) * 256 + t] = cr[i][j][v];
        mine[((i * 2 + j) * 8 + 4 + v) * 256 + t] = ci[i][j][v];
      }
}

// the sum over slices 0, 1, ... of a block tile's partials (same layout)
__device__ __forceinline__ void sum_part_block(const DevOp& op, uint64_t tile, const SplitK& sk,
                                               f4 (&cr)[2][2], f4 (&ci)[2][2]) {
  const int t = threadIdx.x;
  const float* base = sk.part + op.part + tile * op.ksplit * (32 * 256);
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      cr[i][j] = f4{0.f, 0.f, 0.f, 0.f};
      ci[i][j] = f4{0.f, 0.f, 0.f, 0.f};
    }
  for (uint32_t q = 0; q < op.ksplit; ++q) {
    const float* src = base + (uint64_t)q * (32 * 256);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          cr[i][j][v] += src[((i * 2 + j) * 8 + v) * 256 + t];
          ci[i][j][v] += src[((i * 2 + j) * 8 + 4 + v) * 256 + t];
        }
  }
}

// ------------------------------------------------------------------ FP32

struct SmemF32 {
  float A[2][BK32][BM + PAD];  // [re/im][k][m]
  float B[2][BK32][BN + PAD];  // [re/im][k][n]
};

// One 64 x 64 tile of C (or one K slice of it) for the FP32 path; called by
// all 256 threads.  The op record is taken by value: held in registers, it
// is not reloaded from memory after every barrier of the k loop (a reload
// would wait for the prefetched operands too).
template <bool TABLES>
__device__ __forceinline__ void gemm_tile_f32(const DevOp op, uint64_t tile,
                                              const uint32_t* __restrict__ tab,
                                              float2* __restrict__ arena, SmemF32& S,
                                              const SplitK& sk) {
  auto& As = S.A;
  auto& Bs = S.B;
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  {
    const TileCtx c = tile_ctx(op, tile, arena);
    const bool akf = op.flags & 1u, bkf = op.flags & 2u;
    // fixed row / column offsets of this thread's loads
    uint32_t aoff[4], boff[4];
    bool aok[4], bok[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      uint32_t m = c.m0 + (akf ? (t >> 4) + 16 * p : (t & 63));
      aok[p] = m < op.M;
      aoff[p] = aok[p] ? ix(tab, op.a_m, m) : 0;
      uint32_t n = c.n0 + (bkf ? (t >> 4) + 16 * p : (t & 63));
      bok[p] = n < op.N;
      boff[p] = bok[p] ? ix(tab, op.b_n, n) : 0;
    }
    f4 cr[2][2], ci[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        cr[i][j] = f4{0.f, 0.f, 0.f, 0.f};
        ci[i][j] = f4{0.f, 0.f, 0.f, 0.f};
      }
    // register prefetch: the next k-tile's global loads are in flight while
    // the current tile's MFMAs run
    float2 pa[4], pb[4];
    auto fetch = [&](uint32_t k0) {
      // every index first, then every load: a wait for an index-table entry
      // must not also wait for operand loads already in flight
      uint32_t ka[4], kb[4];
      bool va[4], vb[4];
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        // A element (m, k): k fastest across threads when A is k-contiguous
        const uint32_t k = k0 + (akf ? (t & 15) : (t >> 6) + 4 * p);
        va[p] = aok[p] && k < c.ke;
        ka[p] = va[p] ? aoff[p] + ixt<TABLES>(tab, op.a_k, k) : 0u;
        const uint32_t kk = k0 + (bkf ? (t & 15) : (t >> 6) + 4 * p);
        vb[p] = bok[p] && kk < c.ke;
        kb[p] = vb[p] ? boff[p] + ixt<TABLES>(tab, op.b_k, kk) : 0u;
      }
      // unconditional loads (an invalid element reads the operand's first
      // entry and is zeroed), so that the loads issue back to back
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        const float2 x = c.A[ka[p]], y = c.B[kb[p]];
        pa[p] = va[p] ? x : make_float2(0.f, 0.f);
        pb[p] = vb[p] ? y : make_float2(0.f, 0.f);
      }
    };
    fetch(c.kb);
    for (uint32_t k0 = c.kb; k0 < c.ke; k0 += BK32) {
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        int kk = akf ? (t & 15) : (t >> 6) + 4 * p;
        int mm = akf ? (t >> 4) + 16 * p : (t & 63);
        As[0][kk][mm] = pa[p].x;
        As[1][kk][mm] = pa[p].y;
        kk = bkf ? (t & 15) : (t >> 6) + 4 * p;
        int nn = bkf ? (t >> 4) + 16 * p : (t & 63);
        Bs[0][kk][nn] = pb[p].x;
        Bs[1][kk][nn] = pb[p].y;
      }
      __syncthreads();
      if (k0 + BK32 < c.ke) fetch(k0 + BK32);
#pragma unroll
      for (int kk = 0; kk < BK32; kk += 4) {
        const int kr = kk + (lane >> 4);
        float ar[2], ai[2], br[2], bi_[2], nbi[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          ar[i] = As[0][kr][wm * 32 + i * 16 + (lane & 15)];
          ai[i] = As[1][kr][wm * 32 + i * 16 + (lane & 15)];
          br[i] = Bs[0][kr][wn * 32 + i * 16 + (lane & 15)];
          bi_[i] = Bs[1][kr][wn * 32 + i * 16 + (lane & 15)];
          nbi[i] = -bi_[i];
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) {
            cr[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[i], br[j], cr[i][j], 0, 0, 0);
            cr[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai[i], nbi[j], cr[i][j], 0, 0, 0);
            ci[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[i], bi_[j], ci[i][j], 0, 0, 0);
            ci[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai[i], br[j], ci[i][j], 0, 0, 0);
          }
      }
      __syncthreads();
    }
    if (op.ksplit > 1) {
      write_part_block(op, c, sk, cr, ci);
      return;
    }
    store_tile(op, c, tab, arena, cr, ci, wm, wn, lane);
  }
}

// ------------------------------------------------------------------ wave tiles

// One (16 BI) x (16 BJ) block of C for one batch row, computed by a single
// wavefront with FP32 MFMA straight from the arena: the operands are read
// in the matrix cores' register layout (lane l holds A[m0 + l % 16][k + l / 16]
// and B[k + l / 16][n0 + l % 16]), so there is no LDS staging and no
// barrier.  This is the form for nodes too narrow for 64 x 64 tiles (M or
// N below 64, as in per-row batched contractions), where a block tile
// would mostly multiply padding, and for batched nodes with M or N below
// 16 (one block, the rows and columns past the edge masked).  K is a power
// of two >= 4.
// C of a wave tile: lane l holds C[m0 + 16 bi + 4 (l / 16) + v][n0 + 16 bj + l % 16]
template <int BI, int BJ>
__device__ __forceinline__ void store_wave(const DevOp& op, const TileCtx& c,
                                           const uint32_t* __restrict__ tab,
                                           float2* __restrict__ arena, const f4 (&cr)[BI][BJ],
                                           const f4 (&ci)[BI][BJ], int lane) {
  const int i = lane & 15, kq = lane >> 4;
#pragma unroll
  for (int bi = 0; bi < BI; ++bi)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const uint32_t m = c.m0 + bi * 16 + 4 * kq + v;
      if (m >= op.M) continue;  // M < 16: rows past the edge
      const uint32_t cm = ix(tab, op.c_m, m);
#pragma unroll
      for (int bj = 0; bj < BJ; ++bj) {
        const uint32_t n = c.n0 + bj * 16 + i;
        if (n < op.N)
          arena[c.cbase + cm + ix(tab, op.c_n, n)] = make_float2(cr[bi][bj][v], ci[bi][bj][v]);
      }
    }
}

// AVEC (op flag OPF_AVEC, no tables): in each group of U = 4 k-steps over
// k = base .. base + 15, lane kq takes k = base + 4 kq + u at step u
// instead of base + 4 u + kq (a sum over k may visit k in any order, the
// same for A and B), so its four A values of a row are consecutive and
// come in two 16-byte loads instead of four 8-byte loads.
template <int BI, int BJ, bool TABLES, bool AVEC = false>
__device__ __forceinline__ void wave_tile_f32(const DevOp op, uint64_t unit,
                                              const uint32_t* __restrict__ tab,
                                              float2* __restrict__ arena, int lane,
                                              const SplitK& sk) {
  const TileCtx c = unit_ctx(op, unit - op.work0, arena, 16 * BI, 16 * BJ);
  const float2* __restrict__ A = c.A;
  const float2* __restrict__ B = c.B;
  const uint32_t m0 = c.m0, n0 = c.n0;
  const int i = lane & 15, kq = lane >> 4;
  // M or N below 16: lanes past the edge read the last row / column (their
  // products only reach outputs that are not stored)
  uint32_t am[BI], bn[BJ];
#pragma unroll
  for (int bi = 0; bi < BI; ++bi) am[bi] = ix(tab, op.a_m, min(m0 + bi * 16 + i, op.M - 1));
#pragma unroll
  for (int bj = 0; bj < BJ; ++bj) bn[bj] = ix(tab, op.b_n, min(n0 + bj * 16 + i, op.N - 1));
  f4 cr[BI][BJ], ci[BI][BJ];
#pragma unroll
  for (int bi = 0; bi < BI; ++bi)
#pragma unroll
    for (int bj = 0; bj < BJ; ++bj) {
      cr[bi][bj] = f4{0.f, 0.f, 0.f, 0.f};
      ci[bi][bj] = f4{0.f, 0.f, 0.f, 0.f};
    }
  auto step = [&](const float2 (&av)[BI], const float2 (&bv)[BJ]) {
#pragma unroll
    for (int bi = 0; bi < BI; ++bi)
#pragma unroll
      for (int bj = 0; bj < BJ; ++bj) {
        cr[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[bi].x, bv[bj].x, cr[bi][bj], 0, 0, 0);
        cr[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[bi].y, -bv[bj].y, cr[bi][bj], 0, 0, 0);
        ci[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[bi].x, bv[bj].y, ci[bi][bj], 0, 0, 0);
        ci[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[bi].y, bv[bj].x, ci[bi][bj], 0, 0, 0);
      }
  };
  const uint32_t steps = c.ke >> 2;
  uint32_t s = c.kb >> 2;
  // U k-steps issued together: their table and operand loads overlap
  constexpr int U = 4;
  for (; s + U <= steps; s += U) {
    uint32_t ka[U], kb[U];
    float2 av[U][BI], bv[U][BJ];
    if constexpr (AVEC) {
      const uint32_t k0 = 4 * s + 4 * kq;  // this lane's four consecutive k
#pragma unroll
      for (int u = 0; u < U; ++u) kb[u] = ixt<TABLES>(tab, op.b_k, k0 + u);
#pragma unroll
      for (int bi = 0; bi < BI; ++bi) {
        const float4* p = reinterpret_cast<const float4*>(A + am[bi] + k0);
        const float4 lo = p[0], hi = p[1];
        av[0][bi] = make_float2(lo.x, lo.y);
        av[1][bi] = make_float2(lo.z, lo.w);
        av[2][bi] = make_float2(hi.x, hi.y);
        av[3][bi] = make_float2(hi.z, hi.w);
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int bj = 0; bj < BJ; ++bj) bv[u][bj] = B[kb[u] + bn[bj]];
    } else {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        ka[u] = ixt<TABLES>(tab, op.a_k, 4 * (s + u) + kq);
        kb[u] = ixt<TABLES>(tab, op.b_k, 4 * (s + u) + kq);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
#pragma unroll
        for (int bi = 0; bi < BI; ++bi) av[u][bi] = A[am[bi] + ka[u]];
#pragma unroll
        for (int bj = 0; bj < BJ; ++bj) bv[u][bj] = B[kb[u] + bn[bj]];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) step(av[u], bv[u]);
  }
  for (; s < steps; ++s) {
    const uint32_t ka = ixt<TABLES>(tab, op.a_k, 4 * s + kq), kb = ixt<TABLES>(tab, op.b_k, 4 * s + kq);
    float2 av[BI], bv[BJ];
#pragma unroll
    for (int bi = 0; bi < BI; ++bi) av[bi] = A[am[bi] + ka];
#pragma unroll
    for (int bj = 0; bj < BJ; ++bj) bv[bj] = B[kb + bn[bj]];
    step(av, bv);
  }
  if (op.ksplit > 1) {
    // element j of lane l at j * 64 + l of the slice's partial tile
    constexpr int NF = 8 * BI * BJ;
    float* mine = sk.part + op.part + (c.tile * op.ksplit + c.slice) * (NF * 64);
#pragma unroll
    for (int bi = 0; bi < BI; ++bi)
#pragma unroll
      for (int bj = 0; bj < BJ; ++bj)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          mine[((bi * BJ + bj) * 8 + v) * 64 + lane] = cr[bi][bj][v];
          mine[((bi * BJ + bj) * 8 + 4 + v) * 64 + lane] = ci[bi][bj][v];
        }
    return;
  }
  store_wave<BI, BJ>(op, c, tab, arena, cr, ci, lane);
}

// the sum over slices 0, 1, ... of a wave tile's partials (layout as written
// by wave_tile_f32), then the store
template <int BI, int BJ>
__device__ __forceinline__ void reduce_wave(const DevOp op, uint64_t tile,
                                            const uint32_t* __restrict__ tab,
                                            float2* __restrict__ arena, int lane,
                                            const SplitK& sk) {
  constexpr int NF = 8 * BI * BJ;
  const TileCtx c = unit_ctx(op, tile * op.ksplit, arena, 16 * BI, 16 * BJ);
  f4 cr[BI][BJ], ci[BI][BJ];
#pragma unroll
  for (int bi = 0; bi < BI; ++bi)
#pragma unroll
    for (int bj = 0; bj < BJ; ++bj) {
      cr[bi][bj] = f4{0.f, 0.f, 0.f, 0.f};
      ci[bi][bj] = f4{0.f, 0.f, 0.f, 0.f};
    }
  const float* base = sk.part + op.part + tile * op.ksplit * (NF * 64);
  for (uint32_t q = 0; q < op.ksplit; ++q) {
    const float* src = base + (uint64_t)q * (NF * 64);
#pragma unroll
    for (int bi = 0; bi < BI; ++bi)
#pragma unroll
      for (int bj = 0; bj < BJ; ++bj)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          cr[bi][bj][v] += src[((bi * BJ + bj) * 8 + v) * 64 + lane];
          ci[bi][bj][v] += src[((bi * BJ + bj) * 8 + 4 + v) * 64 + lane];
        }
  }
  store_wave<BI, BJ>(op, c, tab, arena, cr, ci, lane);
}

// ------------------------------------------------------------------ BF16X3

__device__ __forceinline__ void split_bf16(float x, __bf16& hi, __bf16& lo) {
  hi = (__bf16)x;
  lo = (__bf16)(x - (float)hi);
}

struct SmemBF16 {
  // [re/im][hi/lo][row][k], k contiguous so that a lane reads 8 k at once
  __attribute__((aligned(16))) __bf16 A[2][2][BM][BK16 + 8];
  __attribute__((aligned(16))) __bf16 B[2][2][BN][BK16 + 8];
};

// One 64 x 64 tile of C (or one K slice of it) for the split-BF16 path;
// called by all 256 threads.
template <bool TABLES>
__device__ __forceinline__ void gemm_tile_bf16x3(const DevOp op, uint64_t tile,
                                                 const uint32_t* __restrict__ tab,
                                                 float2* __restrict__ arena, SmemBF16& S,
                                                 const SplitK& sk) {
  auto& As = S.A;
  auto& Bs = S.B;
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  {
    const TileCtx c = tile_ctx(op, tile, arena);
    const bool akf = op.flags & 1u, bkf = op.flags & 2u;
    uint32_t aoff[8], boff[8];
    bool aok[8], bok[8];
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      uint32_t m = c.m0 + (akf ? (t >> 5) + 8 * p : (t & 63));
      aok[p] = m < op.M;
      aoff[p] = aok[p] ? ix(tab, op.a_m, m) : 0;
      uint32_t n = c.n0 + (bkf ? (t >> 5) + 8 * p : (t & 63));
      bok[p] = n < op.N;
      boff[p] = bok[p] ? ix(tab, op.b_n, n) : 0;
    }
    f4 pr[2][2], pq[2][2], ci[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        pr[i][j] = f4{0.f, 0.f, 0.f, 0.f};
        pq[i][j] = f4{0.f, 0.f, 0.f, 0.f};
        ci[i][j] = f4{0.f, 0.f, 0.f, 0.f};
      }
    for (uint32_t k0 = c.kb; k0 < c.ke; k0 += BK16) {
      // every index, then every load, then the LDS stores (as in the FP32 tile)
      uint32_t ka[8], kb[8];
      bool va[8], vb[8];
#pragma unroll
      for (int p = 0; p < 8; ++p) {
        const uint32_t k = k0 + (akf ? (t & 31) : (t >> 6) + 4 * p);
        va[p] = aok[p] && k < c.ke;
        ka[p] = va[p] ? aoff[p] + ixt<TABLES>(tab, op.a_k, k) : 0u;
        const uint32_t kk = k0 + (bkf ? (t & 31) : (t >> 6) + 4 * p);
        vb[p] = bok[p] && kk < c.ke;
        kb[p] = vb[p] ? boff[p] + ixt<TABLES>(tab, op.b_k, kk) : 0u;
      }
      float2 av[8], bv[8];
#pragma unroll
      for (int p = 0; p < 8; ++p) {
        const float2 x = c.A[ka[p]], y = c.B[kb[p]];
        av[p] = va[p] ? x : make_float2(0.f, 0.f);
        bv[p] = vb[p] ? y : make_float2(0.f, 0.f);
      }
#pragma unroll
      for (int p = 0; p < 8; ++p) {
        int kk = akf ? (t & 31) : (t >> 6) + 4 * p;
        int mm = akf ? (t >> 5) + 8 * p : (t & 63);
        split_bf16(av[p].x, As[0][0][mm][kk], As[0][1][mm][kk]);
        split_bf16(av[p].y, As[1][0][mm][kk], As[1][1][mm][kk]);
        kk = bkf ? (t & 31) : (t >> 6) + 4 * p;
        int nn = bkf ? (t >> 5) + 8 * p : (t & 63);
        split_bf16(bv[p].x, Bs[0][0][nn][kk], Bs[0][1][nn][kk]);
        split_bf16(bv[p].y, Bs[1][0][nn][kk], Bs[1][1][nn][kk]);
      }
      __syncthreads();
      const int kr = 8 * (lane >> 4);
      bf8 a[2][2][2], b[2][2][2];  // [block][re/im][hi/lo]
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int c2 = 0; c2 < 2; ++c2)
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            a[i][c2][h] = *(const bf8*)&As[c2][h][wm * 32 + i * 16 + (lane & 15)][kr];
            b[i][c2][h] = *(const bf8*)&Bs[c2][h][wn * 32 + i * 16 + (lane & 15)][kr];
          }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          // Ar Br
          pr[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][0][0], b[j][0][0], pr[i][j], 0, 0, 0);
          pr[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][0][0], b[j][0][1], pr[i][j], 0, 0, 0);
          pr[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][0][1], b[j][0][0], pr[i][j], 0, 0, 0);
          // Ai Bi
          pq[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][1][0], b[j][1][0], pq[i][j], 0, 0, 0);
          pq[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][1][0], b[j][1][1], pq[i][j], 0, 0, 0);
          pq[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][1][1], b[j][1][0], pq[i][j], 0, 0, 0);
          // Ar Bi + Ai Br
          ci[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][0][0], b[j][1][0], ci[i][j], 0, 0, 0);
          ci[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][0][0], b[j][1][1], ci[i][j], 0, 0, 0);
          ci[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][0][1], b[j][1][0], ci[i][j], 0, 0, 0);
          ci[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][1][0], b[j][0][0], ci[i][j], 0, 0, 0);
          ci[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][1][0], b[j][0][1], ci[i][j], 0, 0, 0);
          ci[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][1][1], b[j][0][0], ci[i][j], 0, 0, 0);
        }
      __syncthreads();
    }
    f4 cr[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) cr[i][j] = pr[i][j] - pq[i][j];
    if (op.ksplit > 1) {
      write_part_block(op, c, sk, cr, ci);
      return;
    }
    store_tile(op, c, tab, arena, cr, ci, wm, wn, lane);
  }
}

}  // namespace tcx

namespace tcx {

// ------------------------------------------------------------------ wide tiles
//
// Nodes with dense operands, A stored as [m][k] and B as [k][n] (the
// planner stores intermediates that feed GEMM-tile nodes this way) and a
// grid of at least one 128 x 128 tile per CU run 128 x 128 tiles: four
// wavefronts of 64 x 64 each, one workgroup per CU, K in stages of 32
// through LDS.  A split pass first writes each operand once as planes laid
// out like the LDS stages, so that a stage is a set of 16-byte direct
// global-to-LDS loads (no registers, no LDS writes by the waves).  Per unit
// of work a tile reads half the operand bytes of 64 x 64 tiles.
constexpr int HM = 128, HN = 128, HK = 32;  // tile edges, k per stage

struct SmemWideF32 {
  // [re/im][k][m] (and [k][n]), m contiguous in 16-byte chunks of 4; chunk
  // q of k row k sits at q ^ (4 (k % 2)), so that the 32 lanes of half a
  // fragment read (16 m of two k rows) touch all 32 banks once
  __attribute__((aligned(16))) float A[2][HK][HM];
  __attribute__((aligned(16))) float B[2][HK][HN];
};
__device__ __forceinline__ int wide_m(int k, int m) {
  return ((((m >> 2) ^ ((k & 1) << 2))) << 2) | (m & 3);
}
struct SmemWideBF16 {
  // [re/im][hi/lo][row][k], k contiguous in 16-byte chunks of 8 (a lane
  // reads one chunk at once); chunk c of a row sits at c ^ ((row / 2) % 4),
  // so that 8 lanes reading one chunk of 8 consecutive rows, or writing
  // two chunks of 4 rows, touch all 32 banks once
  __attribute__((aligned(16))) __bf16 A[2][2][HM][HK];
  __attribute__((aligned(16))) __bf16 B[2][2][HN][HK];
};
__device__ __forceinline__ int wide_chunk(int row, int k) {
  return (((k >> 3) ^ ((row >> 1) & 3)) << 3);
}

// x = hi + lo into element e of two bfloat16 vectors
__device__ __forceinline__ void split_into(float x, bf8& hi, bf8& lo, int e) {
  __bf16 h, l;
  split_bf16(x, h, l);
  hi[e] = h;
  lo[e] = l;
}

// -x for eight bfloat16 numbers: flip the sign bits
__device__ __forceinline__ bf8 neg_bf8(const bf8& x) {
  uint4 u = __builtin_bit_cast(uint4, x);
  u.x ^= 0x80008000u;
  u.y ^= 0x80008000u;
  u.z ^= 0x80008000u;
  u.w ^= 0x80008000u;
  return __builtin_bit_cast(bf8, u);
}

// Tile u of a wide op (0 .. rows tiles_m tiles_n - 1).  Inside a batch row
// the order is XCD-aware: the persistent grid is a multiple of the 8 XCDs,
// so tile u runs on XCD u % 8; XCD x takes column stripe x of the tile grid
// in groups of 4 tile rows, so that its 32 CUs share 4 row slabs of A and 8
// column slabs of B in its L2 at any time.
__device__ __forceinline__ void wide_tile(const DevOp& op, uint64_t u, uint64_t& r, uint32_t& tm,
                                          uint32_t& tn) {
  const uint32_t TM = op.tiles_m, TN = op.tiles_n;
  const uint64_t per_row = (uint64_t)TM * TN;
  r = u / per_row;
  const uint32_t l = (uint32_t)(u - r * per_row);
  if (TN % 8 == 0 && TM % 4 == 0) {
    const uint32_t x = l % 8, q = l / 8, TNx = TN / 8;
    const uint32_t g = q / (4 * TNx), w = q % (4 * TNx);
    tm = g * 4 + w % 4;
    tn = x * TNx + w / 4;
  } else {
    tm = l / TN;
    tn = l % TN;
  }
}

// Operand planes (written by the level's split pass; A's, then B's).
// FP32: re and im planes, k-major: element (k, row) of an operand of R
// rows in all (over its batch rows) at float k R + row; A's re, A's im,
// B's re, B's im.  Split BF16: four planes p = 2 re/im + hi/lo in 16-byte
// chunks of 8 k, interleaved by LDS stage: row by row, each stage (32 k)
// of a row is one 256-byte block of the 4 planes' 64 bytes, so a stage
// reads whole cache lines; chunk kc of plane p of row `row` is uint4
// wide_plane_chunk(row, kc, K / 8) + 4 p.  A's R_A K / 2 uint4, then B's.
__host__ __device__ __forceinline__ uint64_t wide_plane_chunk(uint64_t row, uint64_t kc,
                                                            uint64_t kc_total) {
  return row * kc_total * 4 + (kc >> 2) * 16 + (kc & 3);
}
__device__ __forceinline__ void split_chunk(const float2 (&x)[8], uint4* __restrict__ dst,
                                            uint64_t stride) {
  bf8 rh, rl, ih, il;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    split_into(x[q].x, rh, rl, q);
    split_into(x[q].y, ih, il, q);
  }
  dst[0] = *reinterpret_cast<const uint4*>(&rh);
  dst[stride] = *reinterpret_cast<const uint4*>(&rl);
  dst[2 * stride] = *reinterpret_cast<const uint4*>(&ih);
  dst[3 * stride] = *reinterpret_cast<const uint4*>(&il);
}

// One 128 x 128 tile of C; called by all 256 threads.  PREC 0: FP32 MFMA
// (16 x 16 x 4 f32), 1: split BF16 (32 x 32 x 16 bf16); the operands come
// from their planes (`planes`: the op's).  Two LDS buffers of one stage
// (32 k) each, filled by direct loads two stages ahead, with one barrier
// per stage in its middle (the schedule is described at the split-BF16
// path).
template <int PREC, typename Smem>
__device__ __forceinline__ void gemm_wide(const DevOp& op, uint64_t u,
                                          const uint32_t* __restrict__ tab,
                                          float2* __restrict__ arena,
                                          const uint4* __restrict__ planes, Smem (&S)[2]) {
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  uint64_t r;
  uint32_t tm, tn;
  wide_tile(op, u, r, tm, tn);
  const uint32_t m0 = tm * HM, n0 = tn * HN, K = op.K, N = op.N;
  // the planes' rows of this tile (A rows m0.., B columns n0..)
  const uint64_t RA = (op.a_bs ? op.rows : 1) * (uint64_t)op.M;
  const uint64_t RB = (op.b_bs ? op.rows : 1) * (uint64_t)op.N;
  const uint64_t arow = (op.a_bs ? r * op.M : 0) + m0, brow = (op.b_bs ? r * op.N : 0) + n0;
  // one stage straight from the planes into LDS buffer Dst with 16-byte
  // direct loads: lane l of a load lands at the load's base + 16 l, so each
  // lane fetches the 16 bytes that belong at that slot of the swizzle
  auto issue = [&](uint32_t k0, Smem& Dst) {
    if constexpr (PREC == 0) {
      // 1 KB = two k rows of one plane; load g of 32 per operand
      const float* pl = reinterpret_cast<const float*>(planes);
      const float* Ap[2] = {pl, pl + (uint64_t)K * RA};
      const float* Bp[2] = {pl + 2 * (uint64_t)K * RA, pl + 2 * (uint64_t)K * RA + (uint64_t)K * RB};
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int g = wave * 8 + j, c = g >> 4, kp = g & 15;
        const int kr = 2 * kp + (lane >> 5);
        const int q = (lane & 31) ^ ((kr & 1) << 2);
        __builtin_amdgcn_global_load_lds(Ap[c] + (uint64_t)(k0 + kr) * RA + arow + 4 * q,
                                         &Dst.A[c][2 * kp][0], 16, 0, 0);
        __builtin_amdgcn_global_load_lds(Bp[c] + (uint64_t)(k0 + kr) * RB + brow + 4 * q,
                                         &Dst.B[c][2 * kp][0], 16, 0, 0);
      }
    } else {
      // 1 KB = 16 rows of one plane: row 16 rb + l / 4, stored chunk l % 4,
      // which holds logical chunk (l % 4) ^ ((row / 2) % 4)
      const uint64_t kcT = K / 8;
      const uint4* qA = planes + wide_plane_chunk(arow, k0 / 8, kcT);
      const uint4* qB = planes + 4 * RA * kcT + wide_plane_chunk(brow, k0 / 8, kcT);
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int g = wave * 8 + j, p = g >> 3, rb16 = g & 7;
        const int row = rb16 * 16 + (lane >> 2);
        const int c = (lane & 3) ^ ((row >> 1) & 3);
        const uint64_t off = (uint64_t)row * kcT * 4 + 4 * p + c;
        __builtin_amdgcn_global_load_lds(qA + off, &Dst.A[p >> 1][p & 1][rb16 * 16][0], 16, 0, 0);
        __builtin_amdgcn_global_load_lds(qB + off, &Dst.B[p >> 1][p & 1][rb16 * 16][0], 16, 0, 0);
      }
    }
  };
  const uint64_t cb = op.c + r * op.c_bs;
  const uint32_t ns = K / HK;  // stages (K is a multiple of HK)
  if constexpr (PREC == 0) {
    f4 cr[4][4], ci[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        cr[i][j] = f4{0.f, 0.f, 0.f, 0.f};
        ci[i][j] = f4{0.f, 0.f, 0.f, 0.f};
      }
    // 16 x 16 x 4 blocks, 4 x 4 per wave; a stage is two halves of four k
    // steps.  Fragments of half h: [k step][A re, A im, B re, B im][block],
    // lane l holding row (A) or column (B) l % 16 at k 4 t + l / 16.
    typedef float FragF[4][4][4];
    auto load = [&](const Smem& D, int h, FragF& F) {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int kr = 16 * h + 4 * t + (lane >> 4);
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          F[t][0][b] = D.A[0][kr][wide_m(kr, wm * 64 + b * 16 + (lane & 15))];
          F[t][1][b] = D.A[1][kr][wide_m(kr, wm * 64 + b * 16 + (lane & 15))];
          F[t][2][b] = D.B[0][kr][wide_m(kr, wn * 64 + b * 16 + (lane & 15))];
          F[t][3][b] = D.B[1][kr][wide_m(kr, wn * 64 + b * 16 + (lane & 15))];
        }
      }
    };
    auto mma = [&](const FragF& F) {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        float nbi[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) nbi[j] = -F[t][3][j];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const float ar = F[t][0][i], ai = F[t][1][i];
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            cr[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, F[t][2][j], cr[i][j], 0, 0, 0);
            ci[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, F[t][3][j], ci[i][j], 0, 0, 0);
          }
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            cr[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai, nbi[j], cr[i][j], 0, 0, 0);
            ci[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai, F[t][2][j], ci[i][j], 0, 0, 0);
          }
        }
      }
    };
    // the stage schedule of the split-BF16 path below, in halves of 16 k
    FragF F0, F1;
    auto step = [&](uint32_t s, auto issue_ahead, auto read_next) {
      load(S[s & 1], 1, F1);
      mma(F0);
#pragma unroll
      for (int g = 0; g < 64; ++g) {
        __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);
        __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
      }
      __builtin_amdgcn_sched_group_barrier(0x008, 128, 0);
      __builtin_amdgcn_sched_barrier(0);
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      __builtin_amdgcn_sched_barrier(0);
      if constexpr (decltype(read_next)::value) load(S[(s + 1) & 1], 0, F0);
      if constexpr (decltype(issue_ahead)::value) issue((s + 2) * HK, S[s & 1]);
      mma(F1);
      if constexpr (decltype(read_next)::value) {
#pragma unroll
        for (int g = 0; g < 64; ++g) {
          __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);
          __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
        }
      }
      if constexpr (decltype(issue_ahead)::value) {
#pragma unroll
        for (int g = 0; g < 16; ++g) {
          __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);
          __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);
        }
      }
      __builtin_amdgcn_sched_barrier(0);
    };
    using yes = std::true_type;
    using no = std::false_type;
    issue(0, S[0]);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    load(S[0], 0, F0);
    if (ns > 1) issue(HK, S[1]);
    uint32_t s = 0;
    for (; s + 2 < ns; ++s) step(s, yes{}, yes{});
    if (s + 1 < ns) step(s++, no{}, yes{});
    step(s, no{}, no{});
    // C: lane l holds, per block (i, j), rows 4 (l / 16) + v and column l % 16
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const uint32_t m = m0 + wm * 64 + i * 16 + 4 * (lane >> 4) + v;
        const uint64_t cm = cb + ix(tab, op.c_m, m);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const uint32_t n = n0 + wn * 64 + j * 16 + (lane & 15);
          arena[cm + ix(tab, op.c_n, n)] = make_float2(cr[i][j][v], ci[i][j][v]);
        }
      }
  } else {
    // 32 x 32 x 16 blocks, 2 x 2 per wave; a stage is two k steps of 16.
    // Fragment of a block at k step q: lane l holds row (A) or column (B)
    // l % 32 and k 16 q + 8 (l / 32) .. + 7, one 16-byte LDS chunk.
    f16 cr[2][2], ci[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          cr[i][j][v] = 0.f;
          ci[i][j][v] = 0.f;
        }
    typedef bf8 Frag[2][2][2][2];  // [A/B][block][re/im][hi/lo]
    const int fr = lane & 31;
    auto load = [&](const Smem& D, int q, Frag& F) {
      const int kc = wide_chunk(fr, 16 * q + 8 * (lane >> 5));
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            F[0][b][c][h] = *reinterpret_cast<const bf8*>(&D.A[c][h][wm * 64 + b * 32 + fr][kc]);
            F[1][b][c][h] = *reinterpret_cast<const bf8*>(&D.B[c][h][wn * 64 + b * 32 + fr][kc]);
          }
    };
    // Cr += Ar Br - Ai Bi and Ci += Ar Bi + Ai Br, each real product as
    // hi hi + hi lo + lo hi; the term loop is outermost, so that eight
    // independent accumulations separate two into the same register block
    auto mma = [&](const Frag& F) {
      bf8 na[2][2];  // -(A's imaginary part) [block][hi/lo]
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        na[i][0] = neg_bf8(F[0][i][1][0]);
        na[i][1] = neg_bf8(F[0][i][1][1]);
      }
#pragma unroll
      for (int t = 0; t < 6; ++t) {
        // terms 0..2 take A's real part (Cr: Ar Br, Ci: Ar Bi), terms
        // 3..5 its imaginary part (Cr: -Ai Bi, Ci: Ai Br); within each
        // three, (hi, hi), (hi, lo), (lo, hi)
        const int ah = (t % 3 == 2) ? 1 : 0;
        const int bh = (t % 3 == 1) ? 1 : 0;
        const bool imag = t >= 3;
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) {
            const bf8& xr = imag ? na[i][ah] : F[0][i][0][ah];
            const bf8& xi = imag ? F[0][i][1][ah] : F[0][i][0][ah];
            const bf8& yr = imag ? F[1][j][1][bh] : F[1][j][0][bh];
            const bf8& yi = imag ? F[1][j][0][bh] : F[1][j][1][bh];
            cr[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xr, yr, cr[i][j], 0, 0, 0);
            ci[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xi, yi, ci[i][j], 0, 0, 0);
          }
      }
    };
    // F0 and F1 hold the two k steps of the current stage.  The barrier in
    // the middle of stage s (after the MFMAs of k step 0) is the one point
    // where a wave waits: for the direct loads of stage s + 1, issued a
    // whole stage earlier, and for its reads of stage s, after which no
    // wave reads that buffer again, so the loads of stage s + 2 go into it
    // at once.  The reads of a k step's fragments are spread over the MFMAs
    // of the k step before it (sched_group_barrier: mask 8 = MFMA, 0x100 =
    // LDS read, 0x20 = global load); the last two stages are peeled so that
    // every step is straight-line code.
    Frag F0, F1;
    auto step = [&](uint32_t s, auto issue_ahead, auto read_next) {
      load(S[s & 1], 1, F1);
      mma(F0);
#pragma unroll
      for (int g = 0; g < 16; ++g) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
        __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
      }
      __builtin_amdgcn_sched_group_barrier(0x008, 32, 0);
      __builtin_amdgcn_sched_barrier(0);
      __builtin_amdgcn_s_waitcnt(0);  // direct loads of stage s + 1, reads of stage s
      __syncthreads();
      __builtin_amdgcn_sched_barrier(0);
      if constexpr (decltype(read_next)::value) load(S[(s + 1) & 1], 0, F0);
      if constexpr (decltype(issue_ahead)::value) issue((s + 2) * HK, S[s & 1]);
      mma(F1);
      if constexpr (decltype(read_next)::value) {
#pragma unroll
        for (int g = 0; g < 16; ++g) {
          __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
          __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
        }
      }
      if constexpr (decltype(issue_ahead)::value) {
#pragma unroll
        for (int g = 0; g < 16; ++g) {
          __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
          __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);
        }
      }
      __builtin_amdgcn_sched_barrier(0);
    };
    using yes = std::true_type;
    using no = std::false_type;
    issue(0, S[0]);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    load(S[0], 0, F0);
    if (ns > 1) issue(HK, S[1]);
    uint32_t s = 0;
    for (; s + 2 < ns; ++s) step(s, yes{}, yes{});
    if (s + 1 < ns) step(s++, no{}, yes{});
    step(s, no{}, no{});
    // C: lane l holds, per block (i, j), rows 8 (v / 4) + 4 (l / 32) + v % 4
    // and column l % 32
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const uint32_t m = m0 + wm * 64 + i * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        const uint64_t cm = cb + ix(tab, op.c_m, m);
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const uint32_t n = n0 + wn * 64 + j * 32 + fr;
          arena[cm + ix(tab, op.c_n, n)] = make_float2(cr[i][j][v], ci[i][j][v]);
        }
      }
  }
}

}  // namespace tcx
