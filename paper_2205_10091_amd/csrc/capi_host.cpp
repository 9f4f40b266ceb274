// C ABI entry points for errors, networks and paths (host only).
#include <cmath>
#include <cstring>
#include <new>

#include "internal.h"

struct tc_network {
  tcx::Network net;
};
struct tc_path {
  tcx::Path path;
  // leg structure of each term, kept for stats and validation
  std::vector<tcx::Term> terms;
};

namespace tcx {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

void fail(tc_status s, const std::string& msg) { throw Error{s, msg}; }

}  // namespace tcx

using tcx::Error;

#define TC_GUARD_BEGIN try {
#define TC_GUARD_END                                   \
  }                                                    \
  catch (const Error& e) {                             \
    tcx::set_error(e.msg);                             \
    return e.status;                                   \
  }                                                    \
  catch (const std::bad_alloc&) {                      \
    tcx::set_error("host allocation failed");          \
    return TC_ERR_OUT_OF_MEMORY;                       \
  }                                                    \
  catch (const std::exception& e) {                    \
    tcx::set_error(std::string("internal error: ") + e.what()); \
    return TC_ERR_INVALID_ARG;                         \
  }

extern "C" {

const char* tc_status_string(tc_status s) {
  switch (s) {
    case TC_OK: return "ok";
    case TC_ERR_INVALID_ARG: return "invalid argument";
    case TC_ERR_UNSUPPORTED: return "unsupported";
    case TC_ERR_OUT_OF_MEMORY: return "out of memory";
    case TC_ERR_TOO_LARGE: return "too large";
    case TC_ERR_DEVICE: return "device error";
    case TC_ERR_BUSY: return "busy";
    case TC_ERR_STATE: return "invalid state";
  }
  return "unknown status";
}

const char* tc_last_error(void) { return tcx::g_last_error.c_str(); }

int32_t tc_version(void) { return 100; }

tc_status tc_build_network(const tc_circuit* circuit,
                           const tc_observable* observable,
                           const tc_build_opts* opts, tc_network** out) {
  TC_GUARD_BEGIN
  if (!out) tcx::fail(TC_ERR_INVALID_ARG, "out is NULL");
  auto* n = new tc_network{tcx::build_network(circuit, observable, opts)};
  *out = n;
  return TC_OK;
  TC_GUARD_END
}

void tc_network_free(tc_network* net) { delete net; }

tc_status tc_network_info_get(const tc_network* net, tc_network_info* out) {
  TC_GUARD_BEGIN
  if (!net || !out) tcx::fail(TC_ERR_INVALID_ARG, "NULL argument");
  tc_network_info info{};
  info.n_qubits = net->net.n_qubits;
  info.n_params = net->net.n_params;
  info.n_terms = (int32_t)net->net.terms.size();
  for (const auto& t : net->net.terms) {
    info.max_leaves = std::max(info.max_leaves, (int32_t)t.leaves.size());
    info.total_leaves += (int64_t)t.leaves.size();
  }
  *out = info;
  return TC_OK;
  TC_GUARD_END
}

tc_status tc_network_term_leaves(const tc_network* net, int32_t term,
                                 int32_t* n_leaves, int32_t* kind,
                                 int32_t* gate, int32_t* part, int32_t* conj,
                                 int32_t* rank, int32_t* legs) {
  TC_GUARD_BEGIN
  if (!net || !n_leaves) tcx::fail(TC_ERR_INVALID_ARG, "NULL argument");
  if (term < 0 || term >= (int32_t)net->net.terms.size())
    tcx::fail(TC_ERR_INVALID_ARG, "term out of range");
  const auto& t = net->net.terms[term];
  *n_leaves = (int32_t)t.leaves.size();
  for (size_t i = 0; i < t.leaves.size(); ++i) {
    const auto& lf = t.leaves[i];
    if (kind) kind[i] = lf.kind;
    if (gate) gate[i] = lf.gate;
    if (part) part[i] = lf.part;
    if (conj) conj[i] = lf.conj;
    if (rank) rank[i] = lf.rank;
    if (legs)
      for (int r = 0; r < tcx::MAX_LEAF_RANK; ++r)
        legs[tcx::MAX_LEAF_RANK * i + r] = lf.legs[r];
  }
  return TC_OK;
  TC_GUARD_END
}

tc_status tc_greedy_path(const tc_network* net, const tc_path_opts* opts,
                         tc_path** out) {
  TC_GUARD_BEGIN
  if (!net || !out) tcx::fail(TC_ERR_INVALID_ARG, "NULL argument");
  tc_path_opts o{0, 1, TC_SCORE_COMBO, 0.1, 0, 0};
  if (opts) o = *opts;
  if (o.n_trials < 1) tcx::fail(TC_ERR_INVALID_ARG, "n_trials must be >= 1");
  if (o.score < 0 || o.score > 4) tcx::fail(TC_ERR_INVALID_ARG, "unknown score");
  if (o.reconf_k < 0 || o.reconf_k > 10) tcx::fail(TC_ERR_INVALID_ARG, "reconf_k must be 0..10");
  if (o.max_depth < -1) tcx::fail(TC_ERR_INVALID_ARG, "max_depth must be -1, 0 or a depth");
  auto* p = new tc_path;
  p->path = tcx::greedy_path(net->net, o);
  p->terms = net->net.terms;
  *out = p;
  return TC_OK;
  TC_GUARD_END
}

tc_status tc_path_replace_term(tc_path* base, int32_t term,
                               const int32_t* pairs, int32_t n_steps) {
  TC_GUARD_BEGIN
  if (!base || (n_steps > 0 && !pairs)) tcx::fail(TC_ERR_INVALID_ARG, "NULL argument");
  if (term < 0 || term >= (int32_t)base->terms.size())
    tcx::fail(TC_ERR_INVALID_ARG, "term out of range");
  tcx::TermPath tp;
  tp.n_leaves = (int32_t)base->terms[term].leaves.size();
  for (int32_t s = 0; s < n_steps; ++s) tp.pairs.emplace_back(pairs[2 * s], pairs[2 * s + 1]);
  tcx::validate_term_path(base->terms[term], tp);
  base->path.terms[term] = std::move(tp);
  return TC_OK;
  TC_GUARD_END
}

void tc_path_free(tc_path* path) { delete path; }

tc_status tc_slice(const tc_network* net, const tc_path* path, int32_t max_log2_size,
                   int32_t max_labels, tc_network** out_net, tc_path** out_path,
                   int32_t* n_sliced_labels) {
  TC_GUARD_BEGIN
  if (!net || !path || !out_net || !out_path) tcx::fail(TC_ERR_INVALID_ARG, "NULL argument");
  auto* n = new tc_network;
  auto* p = new tc_path;
  int32_t s = 0;
  try {
    tcx::slice_network(net->net, path->path, max_log2_size, max_labels, n->net, p->path, s);
  } catch (...) {
    delete n;
    delete p;
    throw;
  }
  p->terms = n->net.terms;
  *out_net = n;
  *out_path = p;
  if (n_sliced_labels) *n_sliced_labels = s;
  return TC_OK;
  TC_GUARD_END
}

tc_status tc_path_stats_get(const tc_path* path, int32_t term, tc_path_stats* out) {
  TC_GUARD_BEGIN
  if (!path || !out) tcx::fail(TC_ERR_INVALID_ARG, "NULL argument");
  if (term < -1 || term >= (int32_t)path->terms.size())
    tcx::fail(TC_ERR_INVALID_ARG, "term out of range");
  tc_path_stats st{};
  for (size_t t = 0; t < path->terms.size(); ++t) {
    if (term >= 0 && (int32_t)t != term) continue;
    tcx::TreeStats s = tcx::tree_stats(path->terms[t], path->path.terms[t]);
    st.flops += s.flops;
    st.write += s.write;
    st.size = std::max(st.size, s.size);
    st.n_steps += (int32_t)path->path.terms[t].pairs.size();
    st.max_depth = std::max(st.max_depth, s.depth);
  }
  st.log10_flops = st.flops > 0 ? std::log10(st.flops) : 0;
  st.log2_write = st.write > 0 ? std::log2(st.write) : 0;
  st.log2_size = st.size > 0 ? std::log2(st.size) : 0;
  *out = st;
  return TC_OK;
  TC_GUARD_END
}

tc_status tc_path_term_pairs(const tc_path* path, int32_t term, int32_t* pairs,
                             int32_t* n_steps) {
  TC_GUARD_BEGIN
  if (!path || !n_steps) tcx::fail(TC_ERR_INVALID_ARG, "NULL argument");
  if (term < 0 || term >= (int32_t)path->terms.size())
    tcx::fail(TC_ERR_INVALID_ARG, "term out of range");
  const auto& tp = path->path.terms[term];
  *n_steps = (int32_t)tp.pairs.size();
  if (pairs)
    for (size_t s = 0; s < tp.pairs.size(); ++s) {
      pairs[2 * s] = tp.pairs[s].first;
      pairs[2 * s + 1] = tp.pairs[s].second;
    }
  return TC_OK;
  TC_GUARD_END
}

}  // extern "C"

namespace tcx {
// Accessors for the other translation units.
const Network& network_of(const tc_network* n) { return n->net; }
const Path& path_of(const tc_path* p) { return p->path; }
}  // namespace tcx
