// Host-side contraction path: preprocessing by absorption, then a pairwise
// greedy search, per term.
//
// Paper, section "Custom contraction settings": the default path finder is a
// pairwise greedy; preprocessing absorbs single-qubit gates into two-qubit
// gates before the search; path quality is measured by FLOPs, WRITE (all
// elements written, intermediates included) and SIZE (largest
// intermediate); the contractor table combines flops and write as
// flops + 64 * write.  The greedy rule used here is the size-reduction rule
// of Gray & Kourtis (Quantum 5, 410 (2021), cited in section "Tensor network
// engine"): contract the connected pair minimising
// size(out) - size(a) - size(b).
#include <algorithm>
#include <array>
#include <functional>
#include <atomic>
#include <exception>
#include <mutex>
#include <thread>
#include <cmath>
#include <queue>
#include <random>
#include <unordered_map>

#include "internal.h"

namespace tcx {

namespace {

// legs of a contraction result: symmetric difference, keeping a's order
// then b's order
std::vector<int32_t> result_legs(const std::vector<int32_t>& a,
                                 const std::vector<int32_t>& b) {
  std::vector<int32_t> out;
  out.reserve(a.size() + b.size());
  for (int32_t l : a)
    if (std::find(b.begin(), b.end(), l) == b.end()) out.push_back(l);
  for (int32_t l : b)
    if (std::find(a.begin(), a.end(), l) == a.end()) out.push_back(l);
  return out;
}

int union_rank(const std::vector<int32_t>& a, const std::vector<int32_t>& b) {
  int shared = 0;
  for (int32_t l : a)
    if (std::find(b.begin(), b.end(), l) != b.end()) ++shared;
  return (int)(a.size() + b.size()) - shared;
}

struct Cand {
  double cost;
  double flops;
  int32_t i, j;
};
struct CandCmp {
  bool operator()(const Cand& x, const Cand& y) const {
    if (x.cost != y.cost) return x.cost > y.cost;
    if (x.flops != y.flops) return x.flops > y.flops;
    if (x.i != y.i) return x.i > y.i;
    return x.j > y.j;
  }
};

struct Search {
  std::vector<std::vector<int32_t>> legs;  // per SSA id
  std::vector<char> alive;
  std::unordered_map<int32_t, std::pair<int32_t, int32_t>> owner;  // leg -> ids
  std::vector<std::pair<int32_t, int32_t>> pairs;
  int32_t n_alive = 0;

  void init(const Term& t) {
    for (const Leaf& lf : t.leaves) {
      legs.emplace_back(lf.legs, lf.legs + lf.rank);
      alive.push_back(1);
    }
    n_alive = (int32_t)legs.size();
    for (int32_t id = 0; id < (int32_t)legs.size(); ++id)
      for (int32_t l : legs[id]) {
        auto it = owner.find(l);
        if (it == owner.end())
          owner[l] = {id, -1};
        else
          it->second.second = id;
      }
  }

  int32_t other(int32_t leg, int32_t id) const {
    auto it = owner.find(leg);
    if (it == owner.end()) return -1;
    if (it->second.first == id) return it->second.second;
    return it->second.first;
  }

  int32_t contract(int32_t i, int32_t j) {
    int32_t k = (int32_t)legs.size();
    std::vector<int32_t> out = result_legs(legs[i], legs[j]);
    for (int32_t l : legs[i])
      if (std::find(out.begin(), out.end(), l) == out.end()) owner.erase(l);
    for (int32_t l : out) {
      auto& o = owner[l];
      if (o.first == i || o.first == j) o.first = k;
      if (o.second == i || o.second == j) o.second = k;
    }
    legs.push_back(std::move(out));
    alive.push_back(1);
    alive[i] = alive[j] = 0;
    --n_alive;
    pairs.emplace_back(i, j);
    return k;
  }

  std::vector<int32_t> neighbours(int32_t id) const {
    std::vector<int32_t> nb;
    for (int32_t l : legs[id]) {
      int32_t o = other(l, id);
      if (o >= 0 && std::find(nb.begin(), nb.end(), o) == nb.end()) nb.push_back(o);
    }
    return nb;
  }

  // preprocessing: tensors of rank <= 2 go into their largest neighbour
  void absorb_small() {
    bool changed = true;
    while (changed) {
      changed = false;
      for (int32_t id = 0; id < (int32_t)legs.size(); ++id) {
        if (!alive[id] || legs[id].size() > 2) continue;
        std::vector<int32_t> nb = neighbours(id);
        if (nb.empty()) continue;
        int32_t best = nb[0];
        for (int32_t x : nb)
          if (legs[x].size() > legs[best].size() ||
              (legs[x].size() == legs[best].size() && x < best))
            best = x;
        int32_t a = std::min(id, best), b = std::max(id, best);
        contract(a, b);
        changed = true;
      }
    }
  }

  double costmod = 1.0;

  Cand cand(int32_t i, int32_t j) const {
    int ra = (int)legs[i].size(), rb = (int)legs[j].size();
    int ru = union_rank(legs[i], legs[j]);
    int shared = ra + rb - ru;
    int rc = ra + rb - 2 * shared;
    double cost = std::ldexp(1.0, rc) -
                  costmod * (std::ldexp(1.0, ra) + std::ldexp(1.0, rb));
    double flops = 8.0 * std::ldexp(1.0, ru);
    return Cand{cost, flops, std::min(i, j), std::max(i, j)};
  }

  void greedy(std::mt19937_64* rng, double temperature) {
    std::priority_queue<Cand, std::vector<Cand>, CandCmp> heap;
    for (int32_t id = 0; id < (int32_t)legs.size(); ++id) {
      if (!alive[id]) continue;
      for (int32_t o : neighbours(id))
        if (o > id && alive[o]) heap.push(cand(id, o));
    }
    std::uniform_real_distribution<double> U(1e-12, 1.0);
    while (!heap.empty()) {
      Cand c = heap.top();
      heap.pop();
      if (!alive[c.i] || !alive[c.j]) continue;
      if (rng && temperature > 0) {
        // thermal choice among up to 8 live candidates
        std::vector<Cand> pool{c};
        while (!heap.empty() && pool.size() < 8) {
          Cand d = heap.top();
          heap.pop();
          if (alive[d.i] && alive[d.j]) pool.push_back(d);
        }
        double c0 = pool[0].cost;
        double scale = temperature * std::max(std::fabs(c0), 1.0);
        size_t pick = 0;
        double best = 0;
        for (size_t k = 0; k < pool.size(); ++k) {
          // Gumbel-max sampling of exp(-(cost - c0) / scale)
          double g = -std::log(-std::log(U(*rng)));
          double v = -(pool[k].cost - c0) / scale + g;
          if (k == 0 || v > best) {
            best = v;
            pick = k;
          }
        }
        for (size_t k = 0; k < pool.size(); ++k)
          if (k != pick) heap.push(pool[k]);
        c = pool[pick];
      }
      int32_t k = contract(c.i, c.j);
      for (int32_t o : neighbours(k))
        if (alive[o]) heap.push(cand(k, o));
    }
    // disconnected pieces (scalars, separate components): join by id
    std::vector<int32_t> rest;
    for (int32_t id = 0; id < (int32_t)legs.size(); ++id)
      if (alive[id]) rest.push_back(id);
    while (rest.size() > 1) {
      int32_t a = rest[0], b = rest[1];
      int32_t k = contract(a, b);
      rest.erase(rest.begin(), rest.begin() + 2);
      rest.insert(rest.begin(), k);
    }
  }
};

double score_of(const TreeStats& s, int score) {
  switch (score) {
    case TC_SCORE_FLOPS: return s.flops;
    case TC_SCORE_WRITE: return s.write;
    case TC_SCORE_SIZE: return s.size * 1e6 + s.flops * 1e-12;
    case TC_SCORE_TIME:
      // seconds: flops at 10 TFLOP/s, written elements (8 B) at 2 TB/s,
      // and one dependent launch of about 6 us per tree level
      return s.flops * 1e-13 + s.write * 8.0 / 2e12 + s.depth * 6e-6;
    default: return s.flops / 8.0 + 64.0 * s.write;
  }
}

std::vector<std::vector<int32_t>> ssa_legs_of(const Term& term, const TermPath& tp) {
  std::vector<std::vector<int32_t>> legs;
  for (const Leaf& lf : term.leaves) legs.emplace_back(lf.legs, lf.legs + lf.rank);
  for (auto& p : tp.pairs) legs.push_back(result_legs(legs[p.first], legs[p.second]));
  return legs;
}

// ---- subtree reconfiguration
//
// Section "Custom contraction settings" compares path finders by FLOPs,
// WRITE and SIZE (the contractor table, where reconfigured trees from the
// hyper-optimising finder it cites do best).  Here, from scratch: for each
// internal node of a tree, its subtree is opened up to a frontier of at
// most k inputs (expanding the frontier's largest internal node first);
// the cheapest binary tree over those inputs that yields the node's legs is
// found exactly by dynamic programming over input subsets (cost of a step:
// 2^|union of its operands' legs| + 64 * 2^|its result's legs|, i.e.
// flops / 8 + 64 * write), and replaces the subtree when cheaper.  Legs are
// tracked as bitsets over the frontier's labels.
struct RNode {
  int32_t a = -1, b = -1;        // children (-1: a leaf)
  std::vector<int32_t> legs;
};

using Bits = std::array<uint64_t, 8>;  // up to 512 labels in one frontier

inline int bits_count(const Bits& x) {
  int c = 0;
  for (uint64_t w : x) c += __builtin_popcountll(w);
  return c;
}

double rstep(int union_legs, int out_legs) {
  return std::ldexp(1.0, union_legs) + 64.0 * std::ldexp(1.0, out_legs);
}

// Re-optimises the region of `v` (a node with children); true if changed.
bool reconf_node(std::vector<RNode>& nodes, int32_t v, int k) {
  std::vector<int32_t> front{nodes[v].a, nodes[v].b};
  std::vector<int32_t> inner{v};
  while ((int)front.size() < k) {
    int best = -1;
    for (int i = 0; i < (int)front.size(); ++i)
      if (nodes[front[i]].a >= 0 &&
          (best < 0 || nodes[front[i]].legs.size() > nodes[front[best]].legs.size()))
        best = i;
    if (best < 0) break;
    const int32_t x = front[best];
    inner.push_back(x);
    front[best] = nodes[x].a;
    front.push_back(nodes[x].b);
  }
  const int m = (int)front.size();
  if (m < 3) return false;
  // local labels
  std::vector<int32_t> labels;
  for (int32_t f : front)
    for (int32_t l : nodes[f].legs)
      if (std::find(labels.begin(), labels.end(), l) == labels.end()) labels.push_back(l);
  if (labels.size() > 512) return false;
  auto idx = [&](int32_t l) { return (int)(std::find(labels.begin(), labels.end(), l) - labels.begin()); };
  std::vector<Bits> in(m, Bits{});
  for (int i = 0; i < m; ++i)
    for (int32_t l : nodes[front[i]].legs) {
      const int j = idx(l);
      in[i][j >> 6] |= uint64_t(1) << (j & 63);
    }
  Bits out{};
  for (int32_t l : nodes[v].legs) {
    const int j = idx(l);
    if (j < (int)labels.size()) out[j >> 6] |= uint64_t(1) << (j & 63);
  }
  // legs of every subset: a label stays open if it is an output label or
  // also touches an input outside the subset
  const uint32_t full = (1u << m) - 1;
  std::vector<Bits> lg(full + 1, Bits{});
  for (uint32_t S = 1; S <= full; ++S) {
    Bits touch{}, outside{};
    for (int i = 0; i < m; ++i)
      for (int w = 0; w < 8; ++w) (((S >> i) & 1) ? touch : outside)[w] |= in[i][w];
    for (int w = 0; w < 8; ++w) lg[S][w] = touch[w] & (outside[w] | out[w]);
  }
  std::vector<double> cost(full + 1, 0.0);
  std::vector<uint32_t> split(full + 1, 0);
  for (uint32_t S = 1; S <= full; ++S) {
    if (!(S & (S - 1))) continue;
    const uint32_t low = S & (~S + 1);
    double best = -1;
    // A holds the lowest input (each split once)
    for (uint32_t A = (S - 1) & S; A; A = (A - 1) & S) {
      if (!(A & low)) continue;
      const uint32_t Bs = S ^ A;
      Bits u;
      for (int w = 0; w < 8; ++w) u[w] = lg[A][w] | lg[Bs][w];
      const double c = cost[A] + cost[Bs] + rstep(bits_count(u), bits_count(lg[S]));
      if (best < 0 || c < best) {
        best = c;
        split[S] = A;
      }
    }
    cost[S] = best;
  }
  // the region's current cost
  double now = 0;
  for (int32_t x : inner) {
    const RNode& n = nodes[x];
    std::vector<int32_t> u = nodes[n.a].legs;
    for (int32_t l : nodes[n.b].legs)
      if (std::find(u.begin(), u.end(), l) == u.end()) u.push_back(l);
    now += rstep((int)u.size(), (int)n.legs.size());
  }
  if (cost[full] >= now * (1.0 - 1e-9)) return false;
  // rebuild: the region's inner nodes are reused for the new internal
  // nodes (m - 1 of them, the same count), v stays the region's top
  std::vector<int32_t> pool(inner.begin() + 1, inner.end());
  std::function<int32_t(uint32_t, int32_t)> build = [&](uint32_t S, int32_t at) -> int32_t {
    if (!(S & (S - 1))) return front[__builtin_ctz(S)];
    int32_t id = at;
    if (id < 0) {
      id = pool.back();
      pool.pop_back();
    }
    const uint32_t A = split[S];
    const int32_t ca = build(A, -1), cb = build(S ^ A, -1);
    nodes[id].a = ca;
    nodes[id].b = cb;
    nodes[id].legs.clear();
    for (int j = 0; j < (int)labels.size(); ++j)
      if ((lg[S][j >> 6] >> (j & 63)) & 1) nodes[id].legs.push_back(labels[j]);
    return id;
  };
  std::vector<int32_t> keep_legs = nodes[v].legs;
  build(full, v);
  nodes[v].legs = keep_legs;  // (the same set; keep the original order)
  return true;
}

TermPath reconfigure(const Term& term, const TermPath& tp, int k, int passes) {
  const int32_t nl = (int32_t)term.leaves.size();
  if ((int32_t)tp.pairs.size() < 2) return tp;
  std::vector<std::vector<int32_t>> legs = ssa_legs_of(term, tp);
  std::vector<RNode> nodes(legs.size());
  for (size_t i = 0; i < legs.size(); ++i) nodes[i].legs = legs[i];
  for (size_t s = 0; s < tp.pairs.size(); ++s) {
    nodes[nl + s].a = tp.pairs[s].first;
    nodes[nl + s].b = tp.pairs[s].second;
  }
  const int32_t root = nl + (int32_t)tp.pairs.size() - 1;
  for (int p = 0; p < passes; ++p) {
    // internal nodes, children before parents
    std::vector<int32_t> order;
    std::vector<int32_t> st{root};
    while (!st.empty()) {
      const int32_t x = st.back();
      st.pop_back();
      if (nodes[x].a < 0) continue;
      order.push_back(x);
      st.push_back(nodes[x].a);
      st.push_back(nodes[x].b);
    }
    std::reverse(order.begin(), order.end());
    bool changed = false;
    for (int32_t x : order) changed |= reconf_node(nodes, x, k);
    if (!changed) break;
  }
  // SSA pairs in post order
  TermPath out;
  out.n_leaves = nl;
  std::vector<int32_t> ssa(nodes.size(), -1);
  for (int32_t i = 0; i < nl; ++i) ssa[i] = i;
  std::vector<std::pair<int32_t, bool>> st{{root, false}};
  while (!st.empty()) {
    auto [x, done] = st.back();
    st.pop_back();
    if (nodes[x].a < 0) continue;
    if (!done) {
      st.push_back({x, true});
      st.push_back({nodes[x].b, false});
      st.push_back({nodes[x].a, false});
    } else {
      out.pairs.push_back({ssa[nodes[x].a], ssa[nodes[x].b]});
      ssa[x] = nl + (int32_t)out.pairs.size() - 1;
    }
  }
  return out;
}

}  // namespace

std::vector<std::vector<int32_t>> ssa_legs(const Term& term, const TermPath& tp) {
  std::vector<std::vector<int32_t>> legs;
  for (const Leaf& lf : term.leaves) legs.emplace_back(lf.legs, lf.legs + lf.rank);
  for (auto& p : tp.pairs) legs.push_back(result_legs(legs[p.first], legs[p.second]));
  return legs;
}

void validate_term_path(const Term& term, const TermPath& tp) {
  int32_t n = (int32_t)term.leaves.size();
  if (tp.n_leaves != n) fail(TC_ERR_INVALID_ARG, "path does not match the network");
  if (n == 0) {
    if (!tp.pairs.empty()) fail(TC_ERR_INVALID_ARG, "path has steps for an empty term");
    return;
  }
  if ((int32_t)tp.pairs.size() != n - 1)
    fail(TC_ERR_INVALID_ARG, "path must have n_leaves - 1 steps");
  std::vector<char> used(2 * n, 0);
  for (size_t s = 0; s < tp.pairs.size(); ++s) {
    int32_t a = tp.pairs[s].first, b = tp.pairs[s].second;
    int32_t limit = n + (int32_t)s;
    if (a < 0 || b < 0 || a >= limit || b >= limit || a == b)
      fail(TC_ERR_INVALID_ARG, "path step refers to a tensor that does not exist yet");
    if (used[a] || used[b]) fail(TC_ERR_INVALID_ARG, "path uses a tensor twice");
    used[a] = used[b] = 1;
  }
}

TreeStats tree_stats(const Term& term, const TermPath& tp) {
  TreeStats st;
  std::vector<std::vector<int32_t>> legs = ssa_legs(term, tp);
  int32_t n = (int32_t)term.leaves.size();
  std::vector<int32_t> depth(legs.size(), 0);
  for (size_t s = 0; s < tp.pairs.size(); ++s) {
    int32_t a = tp.pairs[s].first, b = tp.pairs[s].second;
    int ru = union_rank(legs[a], legs[b]);
    st.flops += 8.0 * std::ldexp(1.0, ru);
    double sz = std::ldexp(1.0, (int)legs[n + s].size());
    st.write += sz;
    st.size = std::max(st.size, sz);
    depth[n + s] = 1 + std::max(depth[a], depth[b]);
    st.depth = std::max(st.depth, depth[n + s]);
  }
  return st;
}

// Depth choice (tc_path_opts.max_depth = -1).  A plan runs one dependent
// launch per tree level of its deepest term (twice with the reverse
// sweep), and each costs about LEVEL_SECONDS whatever its size, while the
// small gather nodes of such trees run at about 1 / FLOP_SECONDS flop/s:
// the cap D minimises D LEVEL_SECONDS + flops(D) FLOP_SECONDS over the
// depths the candidates offer (measured on the 20-qubit chain of the VQE
// workload: removing a level saved about 4 us per pass, extra flops cost
// about 0.45 ps each).
constexpr double LEVEL_SECONDS = 4e-6, FLOP_SECONDS = 4.5e-13;

namespace {

// One term's candidates: the best tree found at each depth, with the offer
// order (ties go to the earlier offer, as with a single running best).
struct TreeCand {
  double score = 0, flops = 0, size = 0;
  int32_t depth = 0;
  int64_t seq = 0;
  TermPath tp;
};

// candidate x beats y under the cap (cap <= 0: no cap): within the cap
// first, then the shallower, then the score, then the earlier offer
bool beats(const TreeCand& x, const TreeCand& y, int32_t cap) {
  if (cap > 0) {
    const bool ok = x.depth <= cap, yok = y.depth <= cap;
    if (ok != yok) return ok;
    if (!ok && x.depth != y.depth) return x.depth < y.depth;
  }
  if (x.score != y.score) return x.score < y.score;
  return x.seq < y.seq;
}

const TreeCand& pick(const std::vector<TreeCand>& front, int32_t cap) {
  size_t b = 0;
  for (size_t i = 1; i < front.size(); ++i)
    if (beats(front[i], front[b], cap)) b = i;
  return front[b];
}

}  // namespace

Path greedy_path(const Network& net, const tc_path_opts& opts) {
  Path path;
  path.opts = opts;
  int trials = std::max(1, opts.n_trials);
  std::vector<std::vector<TreeCand>> fronts(net.terms.size());
  for (size_t t = 0; t < net.terms.size(); ++t) {
    const Term& term = net.terms[t];
    std::vector<TreeCand>& front = fronts[t];
    int64_t seq = 0;
    // keeps tp if it is the best so far at its depth
    auto offer = [&](TermPath&& tp, const TreeStats& st, double sc) {
      TreeCand c;
      c.score = sc;
      c.flops = st.flops;
      c.size = st.size;
      c.depth = st.depth;
      c.seq = seq++;
      for (TreeCand& f : front)
        if (f.depth == c.depth) {
          if (c.score < f.score) {
            c.tp = std::move(tp);
            f = std::move(c);
          }
          return;
        }
      c.tp = std::move(tp);
      front.push_back(std::move(c));
    };
    // the trials are independent (each seeds its own generator from the
    // seed, the term and the trial number): they run on up to 16 host
    // threads and are offered in trial order, so the result does not
    // depend on the thread count
    std::vector<TermPath> found(trials);
    std::vector<TreeStats> tstat(trials);
    auto run_trial = [&](int trial) {
      Search s;
      s.init(term);
      if (net.opts.absorb_1q) s.absorb_small();
      std::mt19937_64 rng(hash_mix(opts.seed, (uint64_t)(t * 1000003u + trial)));
      if (trial == 0) {
        s.greedy(nullptr, 0.0);
      } else {
        // later trials: random cost modifier alpha in size(ab) - alpha *
        // (size(a) + size(b)), log-uniform in [1/4, 4], and Boltzmann
        // choices at the given temperature
        std::uniform_real_distribution<double> u(-2.0, 2.0);
        s.costmod = std::exp2(u(rng));
        s.greedy(&rng, opts.temperature > 0 ? opts.temperature : 0.1);
      }
      TermPath& tp = found[trial];
      tp.n_leaves = (int32_t)term.leaves.size();
      tp.pairs = std::move(s.pairs);
      tstat[trial] = tree_stats(term, tp);
    };
    const int n_threads =
        std::min(trials, std::max(1, std::min(16, (int)std::thread::hardware_concurrency())));
    if (n_threads <= 1 || trials < 4) {
      for (int trial = 0; trial < trials; ++trial) run_trial(trial);
    } else {
      std::atomic<int> next{0};
      std::vector<std::thread> pool;
      std::exception_ptr err;
      std::mutex err_mu;
      for (int w = 0; w < n_threads; ++w)
        pool.emplace_back([&]() {
          for (int trial = next++; trial < trials; trial = next++) {
            try {
              run_trial(trial);
            } catch (...) {
              std::lock_guard<std::mutex> g(err_mu);
              if (!err) err = std::current_exception();
            }
          }
        });
      for (auto& th : pool) th.join();
      if (err) std::rethrow_exception(err);
    }
    for (int trial = 0; trial < trials; ++trial)
      offer(std::move(found[trial]), tstat[trial], score_of(tstat[trial], opts.score));
    // One more candidate: the time-ordered sweep of a state-vector
    // simulation.  The unconjugated leaves (boundary vectors, gates in
    // circuit order, Pauli matrices or output bras) are absorbed one by one
    // into a single growing tensor, then the conjugated copy from its last
    // gate back to its boundary vectors, so the tensor never holds more
    // than the light cone's open wires (plus a split gate's bond).  On
    // two-dimensional circuits, where greedy merging of the doubled network
    // can open far more legs, this bounds the largest intermediate by
    // 2^(qubits in the light cone).
    if (term.leaves.size() > 1) {
      std::vector<int32_t> order;
      for (int32_t i = 0; i < (int32_t)term.leaves.size(); ++i)
        if (!term.leaves[i].conj) order.push_back(i);
      for (int32_t i = (int32_t)term.leaves.size() - 1; i >= 0; --i)
        if (term.leaves[i].conj) order.push_back(i);
      TermPath tp;
      tp.n_leaves = (int32_t)term.leaves.size();
      int32_t cur = order[0];
      for (size_t k = 1; k < order.size(); ++k) {
        tp.pairs.push_back({cur, order[k]});
        cur = tp.n_leaves + (int32_t)tp.pairs.size() - 1;
      }
      const TreeStats st = tree_stats(term, tp);
      offer(std::move(tp), st, score_of(st, opts.score));
    }
    // Two spatial candidates, wire by wire (on each wire: ket gates in time
    // order, the observable's leaves, the conjugated gates from the last
    // back): (a) every leaf absorbed in that order into one growing tensor,
    // which holds one boundary of open bonds; (b) each wire's leaves folded
    // into a column tensor, all wires independently, then the columns
    // merged as a balanced binary tree over wire order, whose blocks hold
    // two boundaries but whose depth is log2 of the wire count (for wide
    // shallow circuits: far fewer dependent launches).
    // They are scored under the time score, or when the best path so far
    // has an intermediate above 2^28 elements (other plans stay as found).
    if (term.leaves.size() > 2 &&
        (opts.score == TC_SCORE_TIME || pick(front, 0).size > std::ldexp(1.0, 28))) {
      const int32_t nl = (int32_t)term.leaves.size();
      int32_t max_q = 0;
      for (const Leaf& lf : term.leaves) max_q = std::max(max_q, lf.qubit);
      std::vector<std::vector<int32_t>> col(max_q + 1);
      std::vector<int32_t> ord(nl);
      for (int32_t i = 0; i < nl; ++i) ord[i] = i;
      auto side = [&](const Leaf& lf) {
        if (lf.conj) return 2;
        return (lf.kind == LEAF_KET0 || lf.kind == LEAF_GATE) ? 0 : 1;
      };
      std::stable_sort(ord.begin(), ord.end(), [&](int32_t x, int32_t y) {
        const Leaf &a = term.leaves[x], &b = term.leaves[y];
        const int sa = side(a), sb = side(b);
        if (sa != sb) return sa < sb;
        return sa == 2 ? x > y : x < y;  // conjugated gates from the last back
      });
      for (int32_t i : ord) col[term.leaves[i].qubit].push_back(i);
      TermPath base;
      base.n_leaves = nl;
      std::vector<int32_t> heads;  // one tensor per non-empty wire, in wire order
      for (const auto& c : col) {
        if (c.empty()) continue;
        int32_t cur = c[0];
        for (size_t k = 1; k < c.size(); ++k) {
          base.pairs.push_back({cur, c[k]});
          cur = nl + (int32_t)base.pairs.size() - 1;
        }
        heads.push_back(cur);
      }
      for (int variant = 0; variant < 2; ++variant) {
        TermPath tp;
        std::vector<int32_t> level = heads;
        if (variant == 0) {
          // every leaf straight into one growing tensor, wire by wire
          tp.n_leaves = nl;
          int32_t cur = -1;
          for (const auto& c : col)
            for (int32_t i : c) {
              if (cur < 0) {
                cur = i;
                continue;
              }
              tp.pairs.push_back({cur, i});
              cur = nl + (int32_t)tp.pairs.size() - 1;
            }
        } else {
          tp = base;
          while (level.size() > 1) {
            std::vector<int32_t> next;
            for (size_t k = 0; k + 1 < level.size(); k += 2) {
              tp.pairs.push_back({level[k], level[k + 1]});
              next.push_back(nl + (int32_t)tp.pairs.size() - 1);
            }
            if (level.size() % 2) next.push_back(level.back());
            level = std::move(next);
          }
        }
        const TreeStats st = tree_stats(term, tp);
        // (a candidate whose largest intermediate the executor cannot hold
        // is never kept)
        if (st.size <= std::ldexp(1.0, 31)) offer(std::move(tp), st, score_of(st, opts.score));
      }
    }
  }
  // the depth cap: as given, or the one the time model prefers
  int32_t cap = opts.max_depth;
  if (cap < 0) {
    std::vector<int32_t> depths;
    for (const auto& front : fronts)
      for (const TreeCand& c : front) depths.push_back(c.depth);
    std::sort(depths.begin(), depths.end());
    depths.erase(std::unique(depths.begin(), depths.end()), depths.end());
    double best_t = 0;
    cap = 0;
    for (auto it = depths.rbegin(); it != depths.rend(); ++it) {
      double flops = 0;
      int32_t levels = 0;
      for (const auto& front : fronts) {
        if (front.empty()) continue;
        const TreeCand& c = pick(front, *it);
        flops += c.flops;
        levels = std::max(levels, c.depth);
      }
      const double tm = levels * LEVEL_SECONDS + flops * FLOP_SECONDS;
      if (cap == 0 || tm < best_t) {
        best_t = tm;
        cap = *it;
      }
    }
  }
  path.depth_cap = cap;
  for (size_t t = 0; t < net.terms.size(); ++t) {
    const Term& term = net.terms[t];
    if (fronts[t].empty()) {  // a network without leaves
      TermPath tp;
      tp.n_leaves = (int32_t)term.leaves.size();
      path.terms.push_back(std::move(tp));
      continue;
    }
    TreeCand best = pick(fronts[t], cap);
    if (opts.reconf_k >= 3 && best.tp.pairs.size() >= 2) {
      TreeCand r;
      r.tp = reconfigure(term, best.tp, std::min(opts.reconf_k, 10), 4);
      const TreeStats st = tree_stats(term, r.tp);
      r.score = score_of(st, opts.score);
      r.depth = st.depth;
      r.seq = -1;  // ties: the reconfigured tree stays out
      if (st.size <= std::ldexp(1.0, 31) && beats(r, best, cap) && r.score < best.score)
        best = std::move(r);
      else if (st.size <= std::ldexp(1.0, 31) && cap > 0 && best.depth > cap && r.depth < best.depth)
        best = std::move(r);
    }
    path.terms.push_back(std::move(best.tp));
  }
  return path;
}

}  // namespace tcx
