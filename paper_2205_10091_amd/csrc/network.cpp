// Circuit intake and circuit -> tensor-network translation.
//
// Paper, section "Tensor network engine": the circuit diagram is read as a
// tensor network of gate tensors and product-state boundary vectors.  An
// amplitude <bits|U|0..0> is one network; an expectation <psi|P|psi> is one
// network per Pauli term (the reuse=False form of section "Custom
// contraction settings"), built from the ket, the Pauli matrices and the
// entrywise-conjugated ket standing for the bra.  Two-qubit Pauli rotations,
// CNOT and CZ can be split into two three-leg factors joined by a bond of
// dimension 2 (section "Very large circuit simulation", gate split; the
// split here is the exact closed form, no SVD).  Gates outside a Pauli
// term's backward light cone cancel against their mirror images and are
// dropped.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "internal.h"

namespace tcx {

int gate_qubits(int kind) {
  switch (kind) {
    case TC_GATE_H: case TC_GATE_X: case TC_GATE_Y: case TC_GATE_Z:
    case TC_GATE_S: case TC_GATE_SQRT_X: case TC_GATE_SQRT_Y:
    case TC_GATE_SQRT_W: case TC_GATE_RX: case TC_GATE_RY: case TC_GATE_RZ:
    case TC_GATE_U1: case TC_GATE_DEPOL: case TC_GATE_RSWITCH:
      return 1;
    case TC_GATE_CNOT: case TC_GATE_CZ: case TC_GATE_RZZ: case TC_GATE_RXX:
    case TC_GATE_RYY: case TC_GATE_FSIM: case TC_GATE_U2:
      return 2;
    default:
      return 0;
  }
}

int gate_angles(int kind) {
  switch (kind) {
    case TC_GATE_RX: case TC_GATE_RY: case TC_GATE_RZ: case TC_GATE_RZZ:
    case TC_GATE_RXX: case TC_GATE_RYY: case TC_GATE_DEPOL:
      return 1;
    case TC_GATE_FSIM: case TC_GATE_RSWITCH:
      return 2;
    default:
      return 0;
  }
}

bool gate_angle_differentiable(int kind, int a) {
  // a status chooses an operator: piecewise constant
  return !(kind == TC_GATE_DEPOL && a == 0) && !(kind == TC_GATE_RSWITCH && a == 1);
}

bool gate_diagonal(int kind) {
  return kind == TC_GATE_Z || kind == TC_GATE_S || kind == TC_GATE_RZ ||
         kind == TC_GATE_CZ || kind == TC_GATE_RZZ;
}

bool gate_splittable(int kind) {
  return kind == TC_GATE_RZZ || kind == TC_GATE_RXX || kind == TC_GATE_RYY ||
         kind == TC_GATE_CNOT || kind == TC_GATE_CZ;
}

uint64_t hash_mix(uint64_t h, uint64_t v) {
  // splitmix64 finaliser over the running hash
  h ^= v + 0x9e3779b97f4a7c15ULL + (h << 6) + (h >> 2);
  h ^= h >> 30;
  h *= 0xbf58476d1ce4e5b9ULL;
  h ^= h >> 27;
  h *= 0x94d049bb133111ebULL;
  h ^= h >> 31;
  return h;
}

bool leaf_param_dependent(const Network& net, const Leaf& lf) {
  if (lf.kind != LEAF_GATE) return false;
  const GateRec& g = net.gates[lf.gate];
  if (lf.part == 1) return false;  // first split factor is P_k, constant
  for (int a = 0; a < g.n_angles; ++a)
    if (g.param[a] >= 0) return true;
  return false;
}

namespace {

std::vector<GateRec> intake(const tc_circuit* c) {
  if (!c) fail(TC_ERR_INVALID_ARG, "circuit is NULL");
  if (c->n_qubits < 1 || c->n_qubits > 4096)
    fail(TC_ERR_INVALID_ARG, "n_qubits must be in 1..4096");
  if (c->n_params < 0) fail(TC_ERR_INVALID_ARG, "n_params < 0");
  if (c->n_gates < 0) fail(TC_ERR_INVALID_ARG, "n_gates < 0");
  if (c->n_gates > 0 && !c->gates) fail(TC_ERR_INVALID_ARG, "gates is NULL");
  std::vector<GateRec> out;
  out.reserve(c->n_gates);
  for (int i = 0; i < c->n_gates; ++i) {
    const tc_gate& g = c->gates[i];
    GateRec r;
    r.kind = g.kind;
    r.nq = gate_qubits(g.kind);
    if (r.nq == 0)
      fail(TC_ERR_UNSUPPORTED, "gate " + std::to_string(i) + ": unknown kind " +
                                   std::to_string(g.kind));
    r.n_angles = gate_angles(g.kind);
    for (int k = 0; k < r.nq; ++k) {
      if (g.q[k] < 0 || g.q[k] >= c->n_qubits)
        fail(TC_ERR_INVALID_ARG, "gate " + std::to_string(i) + ": qubit out of range");
      r.q[k] = g.q[k];
    }
    if (r.nq == 2 && r.q[0] == r.q[1])
      fail(TC_ERR_INVALID_ARG, "gate " + std::to_string(i) + ": repeated qubit");
    for (int a = 0; a < r.n_angles; ++a) {
      if (g.param[a] < -1 || g.param[a] >= c->n_params)
        fail(TC_ERR_INVALID_ARG, "gate " + std::to_string(i) + ": param slot out of range");
      r.param[a] = g.param[a];
      r.fixed[a] = g.fixed[a];
      if (r.param[a] < 0 && !std::isfinite(r.fixed[a]))
        fail(TC_ERR_INVALID_ARG, "gate " + std::to_string(i) + ": non-finite angle");
    }
    if (g.kind == TC_GATE_DEPOL) {
      if (!g.matrix) fail(TC_ERR_INVALID_ARG, "gate " + std::to_string(i) + ": probabilities are NULL");
      double sum = 0;
      for (int k = 0; k < 3; ++k) {
        if (!std::isfinite(g.matrix[k]) || g.matrix[k] < 0)
          fail(TC_ERR_INVALID_ARG, "gate " + std::to_string(i) + ": bad probability");
        r.mat[k] = g.matrix[k];
        sum += g.matrix[k];
      }
      if (sum > 1.0) fail(TC_ERR_INVALID_ARG, "gate " + std::to_string(i) + ": probabilities exceed 1");
    }
    if (g.kind == TC_GATE_U1 || g.kind == TC_GATE_U2) {
      if (!g.matrix) fail(TC_ERR_INVALID_ARG, "gate " + std::to_string(i) + ": matrix is NULL");
      int n = g.kind == TC_GATE_U1 ? 8 : 32;
      for (int k = 0; k < n; ++k) {
        if (!std::isfinite(g.matrix[k]))
          fail(TC_ERR_INVALID_ARG, "gate " + std::to_string(i) + ": non-finite matrix entry");
        r.mat[k] = g.matrix[k];
      }
    }
    out.push_back(r);
  }
  return out;
}

struct TermBuilder {
  const Network& net;
  Term term;
  int32_t next = 0;
  explicit TermBuilder(const Network& n) : net(n) {}
  int32_t label() { return next++; }
  void leaf(int32_t kind, int32_t gate, int32_t part, int32_t conj,
            const std::vector<int32_t>& legs, int32_t qubit) {
    if ((int)legs.size() > MAX_LEAF_RANK) fail(TC_ERR_INVALID_ARG, "internal: leaf rank");
    Leaf lf;
    lf.kind = kind;
    lf.gate = gate;
    lf.part = part;
    lf.conj = conj;
    lf.qubit = qubit;
    lf.rank = 0;
    for (int32_t l : legs) lf.legs[lf.rank++] = l;
    term.leaves.push_back(lf);
  }

  // Adds the (possibly conjugated) ket: |0> vectors on `active` qubits and
  // the kept gates.  If `final_labels` is given, the last segment of each
  // active wire takes that label.  Returns the open label of each qubit.
  std::vector<int32_t> ket(const std::vector<char>& active,
                           const std::vector<char>& keep, int conj,
                           const std::vector<int32_t>* final_labels) {
    const int n = net.n_qubits;
    std::vector<int32_t> last_use(n, -1);
    for (size_t gi = 0; gi < net.gates.size(); ++gi) {
      if (!keep[gi]) continue;
      const GateRec& g = net.gates[gi];
      for (int k = 0; k < g.nq; ++k) last_use[g.q[k]] = (int32_t)gi;
    }
    std::vector<int32_t> cur(n, -1);
    for (int q = 0; q < n; ++q) {
      if (!active[q]) continue;
      cur[q] = (final_labels && last_use[q] < 0) ? (*final_labels)[q] : label();
      leaf(LEAF_KET0, 0, 0, conj, {cur[q]}, q);
    }
    for (size_t gi = 0; gi < net.gates.size(); ++gi) {
      if (!keep[gi]) continue;
      const GateRec& g = net.gates[gi];
      int32_t out[2];
      for (int k = 0; k < g.nq; ++k)
        out[k] = (final_labels && last_use[g.q[k]] == (int32_t)gi)
                     ? (*final_labels)[g.q[k]]
                     : label();
      if (g.nq == 1) {
        leaf(LEAF_GATE, (int32_t)gi, 0, conj, {out[0], cur[g.q[0]]}, g.q[0]);
      } else if (net.opts.split_2q && gate_splittable(g.kind)) {
        int32_t bond = label();
        leaf(LEAF_GATE, (int32_t)gi, 1, conj, {bond, out[0], cur[g.q[0]]}, g.q[0]);
        leaf(LEAF_GATE, (int32_t)gi, 2, conj, {bond, out[1], cur[g.q[1]]}, g.q[1]);
      } else {
        leaf(LEAF_GATE, (int32_t)gi, 0, conj,
             {out[0], out[1], cur[g.q[0]], cur[g.q[1]]}, std::max(g.q[0], g.q[1]));
      }
      for (int k = 0; k < g.nq; ++k) cur[g.q[k]] = out[k];
    }
    return cur;
  }
};

}  // namespace

Network build_network(const tc_circuit* c, const tc_observable* o,
                      const tc_build_opts* opts) {
  Network net;
  net.gates = intake(c);
  net.n_qubits = c->n_qubits;
  net.n_params = c->n_params;
  if (opts) net.opts = *opts;
  if (!o) fail(TC_ERR_INVALID_ARG, "observable is NULL");
  net.obs_kind = o->kind;
  const int n = net.n_qubits;

  uint64_t h = hash_mix(0x5443u, (uint64_t)n);
  h = hash_mix(h, (uint64_t)net.n_params);
  h = hash_mix(h, (uint64_t)o->kind);
  h = hash_mix(h, (uint64_t)(net.opts.split_2q * 4 + net.opts.lightcone * 2 +
                             net.opts.absorb_1q));
  for (const GateRec& g : net.gates) {
    h = hash_mix(h, (uint64_t)g.kind);
    for (int k = 0; k < g.nq; ++k) h = hash_mix(h, (uint64_t)g.q[k]);
    for (int a = 0; a < g.n_angles; ++a) {
      h = hash_mix(h, (uint64_t)(int64_t)g.param[a]);
      uint64_t bits;
      std::memcpy(&bits, &g.fixed[a], 8);
      if (g.param[a] < 0) h = hash_mix(h, bits);
    }
    if (g.kind == TC_GATE_U1 || g.kind == TC_GATE_U2 || g.kind == TC_GATE_DEPOL)
      for (int k = 0; k < 32; ++k) {
        uint64_t bits;
        std::memcpy(&bits, &g.mat[k], 8);
        h = hash_mix(h, bits);
      }
  }

  std::vector<char> all_active(n, 1), all_keep(net.gates.size(), 1);
  if (o->kind == TC_OBS_AMPLITUDE) {
    TermBuilder tb(net);
    std::vector<int32_t> fin = tb.ket(all_active, all_keep, 0, nullptr);
    for (int q = 0; q < n; ++q) {
      int32_t b = o->bits ? o->bits[q] : 0;
      if (b != 0 && b != 1) fail(TC_ERR_INVALID_ARG, "bits must be 0 or 1");
      tb.leaf(LEAF_BRA, b, 0, 0, {fin[q]}, q);
      h = hash_mix(h, (uint64_t)b);
    }
    tb.term.n_labels = tb.next;
    tb.term.weight = 1.0;
    net.terms.push_back(std::move(tb.term));
  } else if (o->kind == TC_OBS_PAULI_SUM) {
    if (o->n_terms < 1) fail(TC_ERR_INVALID_ARG, "n_terms must be >= 1");
    if (!o->structures || !o->weights)
      fail(TC_ERR_INVALID_ARG, "structures/weights are NULL");
    for (int j = 0; j < o->n_terms; ++j) {
      const uint8_t* s = o->structures + (size_t)j * n;
      double w = o->weights[j];
      if (!std::isfinite(w)) fail(TC_ERR_INVALID_ARG, "non-finite weight");
      for (int q = 0; q < n; ++q) {
        if (s[q] > 3) fail(TC_ERR_INVALID_ARG, "structure values must be 0..3");
        h = hash_mix(h, (uint64_t)s[q]);
      }
      uint64_t wb;
      std::memcpy(&wb, &w, 8);
      h = hash_mix(h, wb);
      // backward light cone of P_j
      std::vector<char> keep(net.gates.size(), 1), active(n, 0);
      for (int q = 0; q < n; ++q) active[q] = s[q] != 0;
      if (net.opts.lightcone) {
        // Reverse sweep.  A maximal run of consecutive diagonal gates is one
        // commuting block D = D_touch * D_rest, where D_rest acts outside the
        // current support S and therefore commutes with the conjugated
        // operator O and with D_touch: D^dagger O D = D_touch^dagger O
        // D_touch.  So the support grows only by the gates touching S at the
        // block's entry, not by a cascade through the block.
        int gi = (int)net.gates.size() - 1;
        std::vector<int> added;
        while (gi >= 0) {
          int end = gi;
          int start = gi;
          if (gate_diagonal(net.gates[gi].kind))
            while (start > 0 && gate_diagonal(net.gates[start - 1].kind)) --start;
          added.clear();
          for (int x = end; x >= start; --x) {
            const GateRec& g = net.gates[x];
            bool touch = false;
            for (int k = 0; k < g.nq; ++k) touch |= active[g.q[k]] != 0;
            // caller matrices may be non-unitary (G^dagger G != I): never drop
            touch |= g.kind == TC_GATE_U1 || g.kind == TC_GATE_U2;
            if (touch) {
              for (int k = 0; k < g.nq; ++k) added.push_back(g.q[k]);
            } else {
              keep[x] = 0;
            }
          }
          for (int q : added) active[q] = 1;
          gi = start - 1;
        }
      } else {
        for (int q = 0; q < n; ++q) active[q] = 1;
      }
      TermBuilder tb(net);
      std::vector<int32_t> ket_out = tb.ket(active, keep, 0, nullptr);
      std::vector<int32_t> bra_out = ket_out;
      for (int q = 0; q < n; ++q) {
        if (!active[q] || s[q] == 0) continue;
        int32_t ol = tb.label();
        tb.leaf(LEAF_PAULI, s[q], 0, 0, {ol, ket_out[q]}, q);
        bra_out[q] = ol;
      }
      tb.ket(active, keep, 1, &bra_out);
      tb.term.n_labels = tb.next;
      tb.term.weight = w;
      net.terms.push_back(std::move(tb.term));
    }
  } else if (o->kind == TC_OBS_STATE) {
    // <psi|psi>: the conjugated ket's wires end on the ket's open legs
    TermBuilder tb(net);
    std::vector<int32_t> ket_out = tb.ket(all_active, all_keep, 0, nullptr);
    tb.ket(all_active, all_keep, 1, &ket_out);
    tb.term.n_labels = tb.next;
    tb.term.weight = 1.0;
    net.terms.push_back(std::move(tb.term));
  } else if (o->kind == TC_OBS_MPO) {
    // one network: ket, the MPO sites (out leg to the bra, in leg from the
    // ket, bond legs between neighbours), conjugated ket
    if (n > 1 && !o->mpo_bonds) fail(TC_ERR_INVALID_ARG, "mpo_bonds is NULL");
    if (!o->mpo) fail(TC_ERR_INVALID_ARG, "mpo is NULL");
    std::vector<int32_t> dim(n + 1, 1);
    for (int k = 1; k < n; ++k) {
      dim[k] = o->mpo_bonds[k - 1];
      if (dim[k] < 1 || dim[k] > 8) fail(TC_ERR_INVALID_ARG, "MPO bond dimensions must be 1..8");
      h = hash_mix(h, (uint64_t)dim[k]);
    }
    auto bits_of = [](int32_t d) {
      int32_t b = 0;
      while ((1 << b) < d) ++b;
      return b;
    };
    TermBuilder tb(net);
    std::vector<int32_t> ket_out = tb.ket(all_active, all_keep, 0, nullptr);
    std::vector<int32_t> bra_out(n);
    std::vector<int32_t> left;  // legs of the bond to the left of site k
    const double* src = o->mpo;
    net.mpo.resize(n);
    for (int k = 0; k < n; ++k) {
      MpoSite& site = net.mpo[k];
      site.lbits = bits_of(dim[k]);
      site.rbits = bits_of(dim[k + 1]);
      std::vector<int32_t> right;
      for (int b = 0; b < site.rbits; ++b) right.push_back(tb.label());
      bra_out[k] = tb.label();
      std::vector<int32_t> legs = left;
      legs.insert(legs.end(), right.begin(), right.end());
      legs.push_back(bra_out[k]);
      legs.push_back(ket_out[k]);
      const int32_t pr = 1 << site.rbits;
      site.entries.assign((size_t)2 << (site.lbits + site.rbits + 2), 0.0);
      for (int32_t l = 0; l < dim[k]; ++l)
        for (int32_t r = 0; r < dim[k + 1]; ++r)
          for (int oi = 0; oi < 4; ++oi) {
            const double re = *src++, im = *src++;
            if (!std::isfinite(re) || !std::isfinite(im))
              fail(TC_ERR_INVALID_ARG, "non-finite MPO entry");
            const size_t e = ((size_t)(l * pr + r) << 2) | (size_t)oi;
            site.entries[2 * e] = re;
            site.entries[2 * e + 1] = im;
            uint64_t b;
            std::memcpy(&b, &re, 8);
            h = hash_mix(h, b);
            std::memcpy(&b, &im, 8);
            h = hash_mix(h, b);
          }
      tb.leaf(LEAF_MPO, k, 0, 0, legs, k);
      left = right;
    }
    tb.ket(all_active, all_keep, 1, &bra_out);
    tb.term.n_labels = tb.next;
    tb.term.weight = 1.0;
    net.terms.push_back(std::move(tb.term));
  } else {
    fail(TC_ERR_INVALID_ARG, "unknown observable kind");
  }
  net.structure_hash = h;
  return net;
}

}  // namespace tcx
