// Slicing: one network contracted as a sum of smaller ones.
//
// Paper, section "Outlook and concluding remarks": slicing (fixing some
// bond indices and summing the resulting networks) is named as the way to
// contract networks whose intermediates exceed memory, and as a way to
// spread one contraction over devices.  The sum over a bond index is
// written out: for a sliced label l joining leaves A and B and a value k,
// the bond is cut into l (kept by A) and a new label l' (given to B), and
// each end is capped by the basis vector e_k (a <k| leaf).  A term with s
// sliced labels becomes 2^s terms of the same weight, so the root sum adds
// the slices and the gradient sums over them.
//
// Labels are chosen on the term's existing tree: while the largest
// intermediate (legs minus the sliced ones) exceeds 2^max_log2, slice the
// label carried by the most of the largest intermediates (ties: the most
// elements summed over all intermediates holding it, then the smaller
// label).  The sliced term's path is that same tree: every cap is first
// absorbed into its leaf, then the original pairs follow, so each
// intermediate is the original one without the sliced legs.
#include <algorithm>
#include <cmath>

#include "internal.h"

namespace tcx {

void slice_network(const Network& net, const Path& path, int32_t max_log2, int32_t max_labels,
                   Network& out_net, Path& out_path, int32_t& max_sliced) {
  if (path.terms.size() != net.terms.size()) fail(TC_ERR_INVALID_ARG, "path does not match network");
  if (max_log2 < 0 || max_log2 > 31) fail(TC_ERR_INVALID_ARG, "max_log2_size must be 0..31");
  if (max_labels < 0 || max_labels > 16) fail(TC_ERR_INVALID_ARG, "max_labels must be 0..16");
  out_net = net;
  out_net.terms.clear();
  out_path = Path();
  out_path.opts = path.opts;
  max_sliced = 0;
  uint64_t h = net.structure_hash;
  for (size_t t = 0; t < net.terms.size(); ++t) {
    const Term& term = net.terms[t];
    const TermPath& tp = path.terms[t];
    validate_term_path(term, tp);
    const int32_t nl = (int32_t)term.leaves.size();
    const std::vector<std::vector<int32_t>> legs = ssa_legs(term, tp);
    std::vector<char> sliced(term.n_labels, 0);
    std::vector<int32_t> chosen;
    for (;;) {
      int peak = 0;
      for (size_t x = nl; x < legs.size(); ++x) {
        int r = 0;
        for (int32_t l : legs[x]) r += !sliced[l];
        peak = std::max(peak, r);
      }
      if (peak <= max_log2) break;
      if ((int32_t)chosen.size() >= max_labels)
        fail(TC_ERR_TOO_LARGE, "more than " + std::to_string(max_labels) +
                                   " sliced labels needed to reach 2^" + std::to_string(max_log2));
      std::vector<int32_t> at_peak(term.n_labels, 0);
      std::vector<double> weight(term.n_labels, 0.0);
      for (size_t x = nl; x < legs.size(); ++x) {
        int r = 0;
        for (int32_t l : legs[x]) r += !sliced[l];
        for (int32_t l : legs[x]) {
          if (sliced[l]) continue;
          weight[l] += std::ldexp(1.0, r);
          if (r == peak) ++at_peak[l];
        }
      }
      int32_t best = -1;
      for (int32_t l = 0; l < term.n_labels; ++l) {
        if (sliced[l] || !at_peak[l]) continue;
        if (best < 0 || at_peak[l] > at_peak[best] ||
            (at_peak[l] == at_peak[best] && weight[l] > weight[best]))
          best = l;
      }
      sliced[best] = 1;
      chosen.push_back(best);
    }
    const int32_t s = (int32_t)chosen.size();
    max_sliced = std::max(max_sliced, s);
    // the two leaves of every chosen label
    std::vector<std::pair<int32_t, int32_t>> ends(s, {-1, -1});
    for (int32_t j = 0; j < s; ++j)
      for (int32_t i = 0; i < nl; ++i)
        for (int r = 0; r < term.leaves[i].rank; ++r)
          if (term.leaves[i].legs[r] == chosen[j])
            (ends[j].first < 0 ? ends[j].first : ends[j].second) = i;
    for (int32_t j = 0; j < s; ++j) {
      if (ends[j].first < 0 || ends[j].second < 0)
        fail(TC_ERR_INVALID_ARG, "internal: a sliced label must join two leaves");
      h = hash_mix(h, (uint64_t)(t * 131 + chosen[j]));
    }
    for (uint32_t v = 0; v < (1u << s); ++v) {
      Term st = term;
      int32_t next = term.n_labels;
      TermPath sp;
      std::vector<int32_t> cur(nl);  // current SSA id of each original leaf
      for (int32_t i = 0; i < nl; ++i) cur[i] = i;
      std::vector<std::pair<int32_t, int32_t>> caps;  // (leaf, cap leaf)
      for (int32_t j = 0; j < s; ++j) {
        const int32_t bit = (int32_t)((v >> (s - 1 - j)) & 1);
        const int32_t a = ends[j].first, b = ends[j].second;
        const int32_t lb = next++;
        Leaf& B = st.leaves[b];
        for (int r = 0; r < B.rank; ++r)
          if (B.legs[r] == chosen[j]) B.legs[r] = lb;
        for (auto [leaf, label] : {std::pair<int32_t, int32_t>{a, chosen[j]}, {b, lb}}) {
          Leaf cap;
          cap.kind = LEAF_BRA;
          cap.gate = bit;
          cap.rank = 1;
          cap.legs[0] = label;
          cap.qubit = st.leaves[leaf].qubit;
          caps.push_back({leaf, (int32_t)st.leaves.size()});
          st.leaves.push_back(cap);
        }
      }
      st.n_labels = next;
      sp.n_leaves = (int32_t)st.leaves.size();
      const int32_t nl2 = sp.n_leaves;
      for (auto [leaf, cap] : caps) {
        sp.pairs.push_back({cur[leaf], cap});
        cur[leaf] = nl2 + (int32_t)sp.pairs.size() - 1;
      }
      std::vector<int32_t> id(nl + tp.pairs.size());
      for (int32_t i = 0; i < nl; ++i) id[i] = cur[i];
      for (size_t k = 0; k < tp.pairs.size(); ++k) {
        sp.pairs.push_back({id[tp.pairs[k].first], id[tp.pairs[k].second]});
        id[nl + k] = nl2 + (int32_t)sp.pairs.size() - 1;
      }
      if (nl == 1 && s == 0) sp.pairs.clear();
      validate_term_path(st, sp);
      out_net.terms.push_back(std::move(st));
      out_path.terms.push_back(std::move(sp));
    }
  }
  out_net.structure_hash = hash_mix(h, 0x51ce5);
}

}  // namespace tcx
