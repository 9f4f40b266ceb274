// Gate-tensor entries and their angle derivatives, evaluated on the device
// from fp32 angles.
//
// Paper, section "Circuits and gates": gates are small tensors; exp1-type
// gates exp(i t G) with G^2 = I.  Rotations here are R_G(t) = exp(-i t G/2)
// (so G-rotations with G in {X, Y, Z, XX, YY, ZZ}).  Square roots of
// Pauli-like gates are ((1+i)/2) I + ((1-i)/2) G with W = (X+Y)/sqrt 2, and
// fSim(t, p) follows Foxen et al. (2020).  Section "Very large circuit
// simulation" splits two-qubit gates into two three-leg factors: here
// R_GG(t) = sum_k (G^k) (x) (c_k G^k) with c_0 = cos(t/2),
// c_1 = -i sin(t/2), and CNOT / CZ = sum_k |k><k| (x) X^k / Z^k.
//
// Leaf element index e follows the leaf's legs, first leg most significant:
//   one-qubit gate (out, in)            e = 2 o + i
//   two-qubit gate (o0, o1, i0, i1)     e = 4 (2 o0 + o1) + (2 i0 + i1)
//   split factor (bond, out, in)        e = 4 k + 2 o + i
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/tcx.h"
#include "ops.h"

namespace tcx {

struct c32 {
  float re, im;
};

__device__ __forceinline__ c32 cx(float r, float i) { return c32{r, i}; }

#define TCX_RSQRT2 0.70710678118654752f

// Pauli G^k entries, G in {X=1, Y=2, Z=3}; k = 0 gives the identity.
__device__ __forceinline__ c32 pauli_entry(int g, int o, int i) {
  switch (g) {
    case 1: return cx(o != i ? 1.f : 0.f, 0.f);
    case 2:
      if (o == i) return cx(0.f, 0.f);
      return o == 0 ? cx(0.f, -1.f) : cx(0.f, 1.f);
    case 3: return cx(o == i ? (o == 0 ? 1.f : -1.f) : 0.f, 0.f);
    default: return cx(o == i ? 1.f : 0.f, 0.f);
  }
}

// The operator a status selects (float32 cuts, in the order the header
// gives): DEPOL -> Pauli 0..3, RSWITCH -> TC_GATE_RX / RY / RZ.
__device__ __forceinline__ int depol_choice(float status, const float* p) {
  const float p0 = ((1.f - p[0]) - p[1]) - p[2];
  const float c1 = p0 + p[0], c2 = c1 + p[1];
  return status < p0 ? 0 : status < c1 ? 1 : status < c2 ? 2 : 3;
}
__device__ __forceinline__ int rswitch_choice(float status) {
  return status < 1.f / 3.f ? TC_GATE_RX : status < 2.f / 3.f ? TC_GATE_RY : TC_GATE_RZ;
}

// one-qubit gate entry G[o][i] (t, t1: the gate's angles)
__device__ __forceinline__ c32 gate1(int kind, int o, int i, float t, float t1,
                                     const float* mat) {
  if (kind == TC_GATE_DEPOL) return pauli_entry(depol_choice(t, mat), o, i);
  if (kind == TC_GATE_RSWITCH) kind = rswitch_choice(t1);
  switch (kind) {
    case TC_GATE_H: return cx((o & i) ? -TCX_RSQRT2 : TCX_RSQRT2, 0.f);
    case TC_GATE_X: return pauli_entry(1, o, i);
    case TC_GATE_Y: return pauli_entry(2, o, i);
    case TC_GATE_Z: return pauli_entry(3, o, i);
    case TC_GATE_S:
      if (o != i) return cx(0.f, 0.f);
      return o == 0 ? cx(1.f, 0.f) : cx(0.f, 1.f);
    case TC_GATE_SQRT_X:
    case TC_GATE_SQRT_Y: {
      if (o == i) return cx(0.5f, 0.5f);
      c32 g = pauli_entry(kind == TC_GATE_SQRT_X ? 1 : 2, o, i);
      // (1 - i)/2 * g
      return cx(0.5f * (g.re + g.im), 0.5f * (g.im - g.re));
    }
    case TC_GATE_SQRT_W:
      if (o == i) return cx(0.5f, 0.5f);
      return o == 0 ? cx(0.f, -TCX_RSQRT2) : cx(TCX_RSQRT2, 0.f);
    case TC_GATE_RX: {
      float s, c;
      sincosf(0.5f * t, &s, &c);
      return o == i ? cx(c, 0.f) : cx(0.f, -s);
    }
    case TC_GATE_RY: {
      float s, c;
      sincosf(0.5f * t, &s, &c);
      if (o == i) return cx(c, 0.f);
      return o == 0 ? cx(-s, 0.f) : cx(s, 0.f);
    }
    case TC_GATE_RZ: {
      float s, c;
      sincosf(0.5f * t, &s, &c);
      if (o != i) return cx(0.f, 0.f);
      return o == 0 ? cx(c, -s) : cx(c, s);
    }
    case TC_GATE_U1: {
      int e = 2 * o + i;
      return cx(mat[2 * e], mat[2 * e + 1]);
    }
  }
  return cx(0.f, 0.f);
}

__device__ __forceinline__ c32 dgate1(int kind, int o, int i, float t, float t1) {
  if (kind == TC_GATE_RSWITCH) kind = rswitch_choice(t1);  // (a DEPOL status: 0)
  float s, c;
  sincosf(0.5f * t, &s, &c);
  switch (kind) {
    case TC_GATE_RX: return o == i ? cx(-0.5f * s, 0.f) : cx(0.f, -0.5f * c);
    case TC_GATE_RY:
      if (o == i) return cx(-0.5f * s, 0.f);
      return o == 0 ? cx(-0.5f * c, 0.f) : cx(0.5f * c, 0.f);
    case TC_GATE_RZ:
      if (o != i) return cx(0.f, 0.f);
      // d/dt exp(-+ i t/2) = -+ (i/2) exp(-+ i t/2)
      return o == 0 ? cx(-0.5f * s, -0.5f * c) : cx(-0.5f * s, 0.5f * c);
  }
  return cx(0.f, 0.f);
}

// Pauli generator of a two-qubit rotation (1 X, 2 Y, 3 Z), 0 otherwise
__device__ __forceinline__ int rot2_pauli(int kind) {
  return kind == TC_GATE_RXX ? 1 : kind == TC_GATE_RYY ? 2 : kind == TC_GATE_RZZ ? 3 : 0;
}

__device__ __forceinline__ c32 cmulc(c32 a, c32 b) {
  return cx(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}

// (G (x) G)[row][col] for a Pauli G
__device__ __forceinline__ c32 pauli2(int g, int row, int col) {
  return cmulc(pauli_entry(g, row >> 1, col >> 1), pauli_entry(g, row & 1, col & 1));
}

// whole two-qubit gate entry M[row][col]
__device__ __forceinline__ c32 gate2(int kind, int row, int col, float t0,
                                     float t1, const float* mat) {
  switch (kind) {
    case TC_GATE_CNOT:
      if (row < 2) return cx(row == col ? 1.f : 0.f, 0.f);
      return cx(col == (row ^ 1) ? 1.f : 0.f, 0.f);
    case TC_GATE_CZ:
      return cx(row == col ? (row == 3 ? -1.f : 1.f) : 0.f, 0.f);
    case TC_GATE_RZZ:
    case TC_GATE_RXX:
    case TC_GATE_RYY: {
      float s, c;
      sincosf(0.5f * t0, &s, &c);
      c32 p = pauli2(rot2_pauli(kind), row, col);
      float id = row == col ? c : 0.f;
      // c I - i s P
      return cx(id + s * p.im, -s * p.re);
    }
    case TC_GATE_FSIM: {
      if (row == 0 && col == 0) return cx(1.f, 0.f);
      if (row == 3 && col == 3) {
        float s, c;
        sincosf(t1, &s, &c);
        return cx(c, -s);
      }
      if ((row == 1 || row == 2) && (col == 1 || col == 2)) {
        float s, c;
        sincosf(t0, &s, &c);
        return row == col ? cx(c, 0.f) : cx(0.f, -s);
      }
      return cx(0.f, 0.f);
    }
    case TC_GATE_U2: {
      int e = 4 * row + col;
      return cx(mat[2 * e], mat[2 * e + 1]);
    }
  }
  return cx(0.f, 0.f);
}

__device__ __forceinline__ c32 dgate2(int kind, int row, int col, float t0,
                                      float t1, int which) {
  switch (kind) {
    case TC_GATE_RZZ:
    case TC_GATE_RXX:
    case TC_GATE_RYY: {
      float s, c;
      sincosf(0.5f * t0, &s, &c);
      c32 p = pauli2(rot2_pauli(kind), row, col);
      float id = row == col ? -0.5f * s : 0.f;
      // -s/2 I - i c/2 P
      return cx(id + 0.5f * c * p.im, -0.5f * c * p.re);
    }
    case TC_GATE_FSIM:
      if (which == 0) {
        if ((row == 1 || row == 2) && (col == 1 || col == 2)) {
          float s, c;
          sincosf(t0, &s, &c);
          return row == col ? cx(-s, 0.f) : cx(0.f, -c);
        }
        return cx(0.f, 0.f);
      } else {
        if (row == 3 && col == 3) {
          float s, c;
          sincosf(t1, &s, &c);
          // d/dp exp(-i p) = -i exp(-i p)
          return cx(-s, -c);
        }
        return cx(0.f, 0.f);
      }
  }
  return cx(0.f, 0.f);
}

// split factors: e = 4 k + 2 o + i
__device__ __forceinline__ c32 split_entry(int kind, int part, int k, int o, int i,
                                           float t) {
  if (kind == TC_GATE_CNOT || kind == TC_GATE_CZ) {
    if (part == 1) return cx((o == k && i == k) ? 1.f : 0.f, 0.f);
    return pauli_entry(k ? (kind == TC_GATE_CNOT ? 1 : 3) : 0, o, i);
  }
  int g = rot2_pauli(kind);
  c32 p = pauli_entry(k ? g : 0, o, i);
  if (part == 1) return p;
  float s, c;
  sincosf(0.5f * t, &s, &c);
  c32 ck = k ? cx(0.f, -s) : cx(c, 0.f);
  return cmulc(ck, p);
}

__device__ __forceinline__ c32 dsplit_entry(int kind, int part, int k, int o, int i,
                                            float t) {
  if (part != 2 || !rot2_pauli(kind)) return cx(0.f, 0.f);
  c32 p = pauli_entry(k ? rot2_pauli(kind) : 0, o, i);
  float s, c;
  sincosf(0.5f * t, &s, &c);
  c32 dk = k ? cx(0.f, -0.5f * c) : cx(-0.5f * s, 0.f);
  return cmulc(dk, p);
}

__device__ __forceinline__ c32 leaf_entry(const DevLeaf& L, int e, float t0, float t1,
                                          const float* ftab) {
  c32 v;
  switch (L.kind) {
    case DLEAF_KET0: v = cx(e == 0 ? 1.f : 0.f, 0.f); break;
    case DLEAF_BRA: v = cx(e == L.value ? 1.f : 0.f, 0.f); break;
    case DLEAF_PAULI: v = pauli_entry(L.value, e >> 1, e & 1); break;
    case DLEAF_MPO: v = cx(ftab[L.mat + 2 * e], ftab[L.mat + 2 * e + 1]); break;
    default:
      if (L.part == 0) {
        if (L.rank == 2)
          v = gate1(L.gkind, e >> 1, e & 1, t0, t1, ftab + L.mat);
        else
          v = gate2(L.gkind, e >> 2, e & 3, t0, t1, ftab + L.mat);
      } else {
        v = split_entry(L.gkind, L.part, e >> 2, (e >> 1) & 1, e & 1, t0);
      }
  }
  if (L.conj) v.im = -v.im;
  return v;
}

__device__ __forceinline__ c32 dleaf_entry(const DevLeaf& L, int e, float t0, float t1,
                                           int which) {
  c32 v;
  if (L.part == 0) {
    if (L.rank == 2)
      v = which == 0 ? dgate1(L.gkind, e >> 1, e & 1, t0, t1) : cx(0.f, 0.f);
    else
      v = dgate2(L.gkind, e >> 2, e & 3, t0, t1, which);
  } else {
    v = dsplit_entry(L.gkind, L.part, e >> 2, (e >> 1) & 1, e & 1, t0);
  }
  if (L.conj) v.im = -v.im;
  return v;
}

}  // namespace tcx
