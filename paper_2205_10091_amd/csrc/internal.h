// Internal host-side structures of the contraction executor.
#pragma once

#include <cstdint>
#include <string>
#include <utility>
#include <vector>

#include "../../include/tcx.h"

namespace tcx {

// ---------------------------------------------------------------- errors
void set_error(const std::string& msg);
struct Error {
  tc_status status;
  std::string msg;
};
[[noreturn]] void fail(tc_status s, const std::string& msg);

// ---------------------------------------------------------------- circuit
struct GateRec {
  int32_t kind = 0;
  int32_t nq = 1;
  int32_t q[2] = {0, 0};
  int32_t param[2] = {-1, -1};
  double fixed[2] = {0.0, 0.0};
  int32_t n_angles = 0;
  double mat[32] = {0};  // U1/U2 entries (re, im) row-major
};

int gate_qubits(int kind);   // 1 or 2; 0 for unknown kinds
int gate_angles(int kind);   // number of angle arguments
bool gate_splittable(int kind);
bool gate_angle_differentiable(int kind, int angle);
bool gate_diagonal(int kind);   // diagonal in the computational basis

// ---------------------------------------------------------------- network
enum LeafKind : int32_t { LEAF_GATE = 0, LEAF_KET0 = 1, LEAF_BRA = 2, LEAF_PAULI = 3,
                          LEAF_MPO = 4 };
constexpr int MAX_LEAF_RANK = 8;

struct Leaf {
  int32_t kind = LEAF_GATE;
  int32_t gate = 0;   // gate index, bit / Pauli value, or MPO site
  int32_t part = 0;   // 0 whole, 1 / 2 split factors
  int32_t conj = 0;
  int32_t rank = 0;
  int32_t legs[MAX_LEAF_RANK] = {-1, -1, -1, -1, -1, -1, -1, -1};
  int32_t qubit = 0;  // the wire it sits on (a whole two-qubit gate: the later one)
};

// An MPO site as a leaf tensor: legs (left bond bits, right bond bits, out,
// in), entries (re, im) with the bonds padded to powers of two.
struct MpoSite {
  int32_t lbits = 0, rbits = 0;
  std::vector<double> entries;   // 2 * 2^(lbits + rbits + 2)
};

struct Term {
  std::vector<Leaf> leaves;
  int32_t n_labels = 0;
  double weight = 1.0;
};

struct Network {
  int32_t n_qubits = 0;
  int32_t n_params = 0;
  int32_t obs_kind = TC_OBS_AMPLITUDE;
  tc_build_opts opts{1, 1, 1};
  std::vector<GateRec> gates;
  std::vector<Term> terms;
  std::vector<MpoSite> mpo;   // MPO observable: one per qubit
  // identifies the circuit + observable structure (for plan caches)
  uint64_t structure_hash = 0;
};

// True iff leaf values depend on the parameter vector.
bool leaf_param_dependent(const Network& net, const Leaf& lf);

Network build_network(const tc_circuit* c, const tc_observable* o,
                      const tc_build_opts* opts);

// ---------------------------------------------------------------- path
struct TermPath {
  int32_t n_leaves = 0;
  std::vector<std::pair<int32_t, int32_t>> pairs;  // SSA
};

struct Path {
  std::vector<TermPath> terms;
  tc_path_opts opts{};
  int32_t depth_cap = 0;  // the tree depth cap used (0 = none)
};

struct TreeStats {
  double flops = 0, write = 0, size = 0;
  int32_t depth = 0;
};

Path greedy_path(const Network& net, const tc_path_opts& opts);
TreeStats tree_stats(const Term& term, const TermPath& tp);
void validate_term_path(const Term& term, const TermPath& tp);

// legs of every SSA tensor of a term (leaves, then one per step)
std::vector<std::vector<int32_t>> ssa_legs(const Term& term, const TermPath& tp);

uint64_t hash_mix(uint64_t h, uint64_t v);

// Slicing (slice.cpp): every term whose tree has an intermediate above
// 2^max_log2 elements becomes 2^s terms with s bond labels fixed, and the
// path of each is the original tree; max_sliced receives the largest s.
void slice_network(const Network& net, const Path& path, int32_t max_log2, int32_t max_labels,
                   Network& out_net, Path& out_path, int32_t& max_sliced);

}  // namespace tcx
