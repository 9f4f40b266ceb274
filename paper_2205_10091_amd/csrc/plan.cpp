// Plan compilation (host only): contraction trees -> level-ordered batched
// launches, index tables, leaf / root / gradient tables, and a
// liveness-based arena.
//
// Paper: section "Tensor network engine" (the contraction itself is a
// sequence of pairwise einsum/matmul steps chosen by the path), section
// "Gradients, optimization and variational algorithms" (reverse-mode
// gradient; section "Custom contraction settings" notes that AD keeps every
// intermediate, which is why WRITE rather than SIZE bounds its memory), and
// section "vmap and vectorized_value_and_grad" (one compiled plan evaluated
// for a batch of parameter vectors).
//
// Execution model.  Tree nodes of all terms are grouped by level (longest
// path from the leaves); each level is one launch.  The reverse sweep seeds
// each term's root with its weight alpha_j; for a node C = A.B it computes
// dA = dC.B and dB = dC.A with the same contraction kernels (the network is
// holomorphic in its leaf entries, so no conjugation appears; bra leaves
// already hold conjugated entries).  Adjoint launches visit the forward
// levels from the top down.  Leaf adjoints are written in their leaf's leg
// order and dotted with dLeaf/dangle in FP64.
//
// Checkpointing.  With segment length c, forward levels are cut into
// segments of c levels.  A node's value is kept for the reverse sweep only
// if its consumer lies in another segment; the others are freed after the
// forward pass.  The reverse sweep handles segments from the top: it first
// recomputes the segment's dropped values from kept ones (a second forward
// pass over that segment), then runs the segment's adjoint launches.
#include <algorithm>
#include <cmath>
#include <map>
#include <set>
#include <string>
#include <unordered_map>

#include "plan.h"

namespace tcx {

namespace {

struct PT {                       // a tensor of the plan
  std::vector<int32_t> legs;      // storage order, most significant first
  bool batched = false;
  uint64_t elems = 1;
  int64_t off = -1;
  int32_t first = 0, last = 0;    // timeline steps of production / last use
  bool fixed = false;             // preallocated constant (seeds)
  int32_t term = -1;              // owning term
  // resident term launches: an LDS copy at lds_off serves the reads up to
  // step lds_last; `global` says whether the global copy at off is kept
  // (read later, or by the root and gradient kernels)
  int64_t lds_off = -1;
  int32_t lds_last = -1;
  bool global = true;
};

// offset of index i under descriptor d (see ops.h)
uint64_t ix_host(const std::vector<uint32_t>& tabs, uint32_t d, uint64_t i) {
  if (d & IX_TABLE) return tabs[(d & ~IX_TABLE) + i];
  uint64_t off = 0;
  uint32_t src = 0;
  for (int r = 0; r < IX_RUNS; ++r) {
    const uint32_t f = (d >> (10 * r)) & 0x3ffu;
    const uint32_t len = f & 31, dst = f >> 5;
    off |= ((i >> src) & ((uint64_t(1) << len) - 1)) << dst;
    src += len;
  }
  return off;
}

struct Tables {
  std::vector<uint32_t>& tabs;
  std::unordered_map<std::string, uint32_t> memo;
  std::unordered_map<uint32_t, uint32_t> maxv;  // table base -> largest entry
  uint64_t n_runs = 0, n_tables = 0;            // descriptors of each kind
  explicit Tables(std::vector<uint32_t>& t) : tabs(t) {}

  // Descriptor of the offsets of index i over the ordered sub-legs `sub` of
  // a rank-r tensor whose leg l sits at position pos[l]:
  // sum_j bit_j(i) * 2^(r-1-pos[sub[j]]), sub[0] most significant.
  uint32_t gather(const std::vector<int8_t>& pos, int r, const std::vector<int32_t>& sub) {
    uint32_t stride[32];
    char sh[32];
    const size_t nb = sub.size();
    for (size_t j = 0; j < nb; ++j) {
      const int idx = pos[sub[j]];
      if (idx < 0) fail(TC_ERR_INVALID_ARG, "internal: leg missing from tensor");
      sh[j] = (char)(r - 1 - idx);
      stride[j] = 1u << (r - 1 - idx);
    }
    // runs: maximal stretches of legs on consecutive, descending tensor
    // bits, found from the most significant index bit down and stored from
    // the least significant up
    {
      uint32_t len[IX_RUNS + 1], dst[IX_RUNS + 1];
      int runs = 0;
      size_t j = 0;
      while (j < nb && runs <= IX_RUNS) {
        size_t e = j + 1;
        while (e < nb && sh[e] == sh[e - 1] - 1) ++e;
        len[runs] = (uint32_t)(e - j);
        dst[runs] = (uint32_t)sh[e - 1];  // lowest tensor bit of the run
        ++runs;
        j = e;
      }
      if (j == nb && runs <= IX_RUNS) {
        uint32_t d = 0;
        for (int q = 0; q < runs; ++q)
          d |= (len[runs - 1 - q] | (dst[runs - 1 - q] << 5)) << (10 * q);
        ++n_runs;
        return d;
      }
    }
    ++n_tables;
    std::string key(sh, nb);
    auto it = memo.find(key);
    if (it != memo.end()) return IX_TABLE | it->second;
    const uint64_t n = 1ull << nb;
    // checked before building: a plan whose tables would pass the budget is
    // rejected at once instead of after filling them
    if (tabs.size() + n > TABLE_MAX_ENTRIES)
      fail(TC_ERR_TOO_LARGE, "index tables would exceed 2^27 entries (512 MiB)");
    uint32_t base = (uint32_t)tabs.size();
    tabs.resize(tabs.size() + n);
    // entry i = entry(i without its lowest set bit) + stride of that bit
    tabs[base] = 0;
    uint32_t mx = 0;
    for (uint64_t i = 1; i < n; ++i) {
      const int low = __builtin_ctzll(i);
      const uint32_t v = tabs[base + (i & (i - 1))] + stride[nb - 1 - low];
      tabs[base + i] = v;
      mx = std::max(mx, v);
    }
    memo.emplace(key, base);
    maxv.emplace(base, mx);
    return IX_TABLE | base;
  }
  // largest offset over the group's 2^nb indices
  uint64_t max_of(uint32_t d, uint32_t n) const {
    if (d & IX_TABLE) return maxv.at(d & ~IX_TABLE);
    return n ? ix_host(tabs, d, n - 1) : 0;  // all index bits set
  }
};

// Best-fit allocator over element offsets: free blocks indexed both by
// offset (to coalesce neighbours) and by size (to find the best fit).
struct Arena {
  std::map<uint64_t, uint64_t> free_;             // offset -> size (elements)
  std::set<std::pair<uint64_t, uint64_t>> by_size_;  // (size, offset)
  uint64_t top = 0;
  static uint64_t align(uint64_t x) { return (x + 31) & ~uint64_t(31); }  // 256 B
  void add_free(uint64_t off, uint64_t n) {
    free_[off] = n;
    by_size_.emplace(n, off);
  }
  void drop_free(std::map<uint64_t, uint64_t>::iterator it) {
    by_size_.erase({it->second, it->first});
    free_.erase(it);
  }
  uint64_t alloc(uint64_t n) {
    n = align(std::max<uint64_t>(n, 1));
    auto b = by_size_.lower_bound({n, 0});
    if (b != by_size_.end()) {
      uint64_t sz = b->first, off = b->second;
      by_size_.erase(b);
      free_.erase(off);
      if (sz > n) add_free(off + n, sz - n);
      return off;
    }
    uint64_t off = top;
    top += n;
    return off;
  }
  void release(uint64_t off, uint64_t n) {
    n = align(std::max<uint64_t>(n, 1));
    auto nx = free_.lower_bound(off);
    if (nx != free_.end() && off + n == nx->first) {  // merge the next block
      n += nx->second;
      auto tmp = nx++;
      drop_free(tmp);
    }
    if (nx != free_.begin()) {                        // merge the previous block
      auto pv = std::prev(nx);
      if (pv->first + pv->second == off) {
        off = pv->first;
        n += pv->second;
        drop_free(pv);
      }
    }
    if (off + n == top)
      top = off;
    else
      add_free(off, n);
  }
};

// Gather layout of a node: k-split S = 2^ls lanes per output group (long
// sums of small nodes, while a lane keeps more than min_steps k-steps and
// the node stays within `lanes` lanes; further while a lane would hold more
// than 256), else V = 2^lv outputs per thread along n.  Level launches
// spread a node over the whole chip (65536 lanes); term mode over one
// 1024-thread workgroup.
void gather_shape(uint32_t M, uint32_t N, uint32_t K, uint32_t rows, uint64_t lanes,
                  uint32_t& ls, uint32_t& lv, uint32_t min_steps = 4) {
  const uint64_t outs = (uint64_t)rows * M * N;
  ls = 0;
  while (ls < 6 && (K >> ls) > min_steps && (outs << (ls + 1)) <= lanes) ++ls;
  while (ls < 6 && (K >> ls) > 256) ++ls;
  lv = 0;
  if (ls == 0) lv = N >= 4 ? 2 : (N == 2 ? 1 : 0);
}

uint64_t gather_items(uint32_t M, uint32_t N, uint32_t K, uint32_t rows, uint64_t lanes) {
  uint32_t ls, lv;
  gather_shape(M, N, K, rows, lanes, ls, lv);
  uint64_t items = ((uint64_t)rows * M * (N >> lv)) << ls;
  return ls ? (items + 63) & ~uint64_t(63) : items;
}

struct PendingOp {
  int32_t a, b, c;   // tensor ids
  int32_t step;
  int32_t term;
  bool bwd;          // part of the reverse-sweep launch list
  bool recompute;    // forward op re-run by checkpointing
};

struct TermInfo {
  std::vector<int32_t> tid;     // SSA id -> tensor id
  std::vector<int32_t> level;   // SSA id -> forward level
  std::vector<int32_t> parent;  // SSA id -> SSA id of consumer (-1 root)
  std::vector<char> needs;      // subtree holds a parameter-dependent leaf
  int32_t root = -1;
};

struct Schedule {
  std::vector<PT> T;
  std::vector<PendingOp> pend;
  std::vector<TermInfo> ti;
  std::vector<std::pair<int32_t, int32_t>> leaf_adj;      // (leaf tensor, adj tensor)
  std::vector<std::pair<size_t, int32_t>> leaf_adj_term;  // (term, leaf index)
  int32_t max_level = 0, root_step = 0, grad_step = 0;
  uint64_t seed_elems = 0, arena_elems = 0, peak_tensor_elems = 0;
  // term groups: group g's steps are (g span, (g + 1) span]; live elements
  // at the busiest step of each group, and after the leaves are placed
  int32_t span = 0;
  std::vector<uint64_t> group_peak;
  uint64_t base_live = 0;
};

// Builds tensors, ops with their steps, lifetimes and arena offsets.
// ckpt = 0: keep every intermediate for the reverse sweep; ckpt >= 2:
// checkpoint segments of that many levels.
// A node that runs as 64 x 64 GEMM tiles (the level launch's block tiles).
bool block_gemm_node(const Plan& plan, uint32_t M, uint32_t N, uint32_t K, uint32_t rows) {
  return K >= (uint32_t)plan.gemm_min_k && M >= (uint32_t)plan.gemm_min_mn &&
         N >= (uint32_t)plan.gemm_min_mn && (uint64_t)rows * M * N * K >= plan.gemm_min_macs &&
         M >= (uint32_t)plan.block_tile_min_mn && N >= (uint32_t)plan.block_tile_min_mn &&
         K >= (uint32_t)plan.block_tile_min_k;
}

// Term groups (grp: term -> group, G groups; nullptr = one group): the
// terms of a group advance level by level together, and group g runs its
// whole forward pass and reverse sweep before group g + 1 starts, so only
// one group's intermediates are live at a time.  The root sum and the
// gradient sum follow the last group.
void schedule(Schedule& S, const Plan& plan, const Network& net, const Path& path, int B,
              bool grad, int ckpt, bool per_term_arena,
              const std::vector<int32_t>* grp = nullptr, int32_t G = 1) {
  std::vector<PT>& T = S.T;
  S.ti.assign(net.terms.size(), TermInfo{});

  // seeds: one rank-0 constant per term, value alpha_j (arena offset t)
  for (size_t t = 0; t < net.terms.size(); ++t) {
    PT s;
    s.fixed = true;
    s.off = (int64_t)t;
    T.push_back(s);
  }
  S.seed_elems = Arena::align(net.terms.size());

  // ---- forward structure
  for (size_t t = 0; t < net.terms.size(); ++t) {
    const Term& term = net.terms[t];
    const TermPath& tp = path.terms[t];
    validate_term_path(term, tp);
    TermInfo& I = S.ti[t];
    const int32_t nl = (int32_t)term.leaves.size();
    const int32_t ns = nl + (int32_t)tp.pairs.size();
    I.tid.assign(ns, -1);
    I.level.assign(ns, 0);
    I.parent.assign(ns, -1);
    I.needs.assign(ns, 0);
    std::vector<std::vector<int32_t>> legs = ssa_legs(term, tp);
    for (int32_t i = 0; i < nl; ++i) {
      PT x;
      x.legs = legs[i];
      x.elems = 1ull << x.legs.size();
      const bool pd = leaf_param_dependent(net, term.leaves[i]);
      // geometric tensor: the ket's parameter leaves differ per row (each
      // row differentiates one gate use); the reverse sweep runs toward
      // the bra's parameter leaves only
      x.batched = plan.qgt ? pd && !term.leaves[i].conj : pd;
      x.term = (int32_t)t;
      I.needs[i] = plan.qgt ? pd && term.leaves[i].conj : pd;
      x.first = 0;
      I.tid[i] = (int32_t)T.size();
      T.push_back(x);
    }
    for (size_t s = 0; s < tp.pairs.size(); ++s) {
      int32_t a = tp.pairs[s].first, b = tp.pairs[s].second, c = nl + (int32_t)s;
      PT x;
      x.legs = legs[c];
      if (x.legs.size() > 31) fail(TC_ERR_TOO_LARGE, "intermediate of rank > 31");
      x.elems = 1ull << x.legs.size();
      x.batched = T[I.tid[a]].batched || T[I.tid[b]].batched;
      x.term = (int32_t)t;
      I.needs[c] = I.needs[a] || I.needs[b];
      I.level[c] = 1 + std::max(I.level[a], I.level[b]);
      x.first = I.level[c];
      I.parent[a] = I.parent[b] = c;
      I.tid[c] = (int32_t)T.size();
      T.push_back(x);
      S.max_level = std::max(S.max_level, I.level[c]);
    }
    // Storage order of intermediates.  The leg order of an intermediate is
    // free (its node writes it through index descriptors), and each has one
    // consumer; one that feeds a GEMM-tile node is stored the way that node
    // reads contiguously: as operand A its free legs, then the contracted
    // ones (k fastest); as operand B the contracted legs, then its free ones
    // (n fastest); the contracted legs in the same order on both sides (a
    // leaf operand's order, whose layout is fixed).  Every other tensor
    // keeps its legs in contraction order.
    for (size_t s = 0; s < tp.pairs.size(); ++s) {
      const int32_t a = tp.pairs[s].first, b = tp.pairs[s].second;
      if (a < nl && b < nl) continue;
      PT& A = T[I.tid[a]];
      PT& Bt = T[I.tid[b]];
      auto in = [](const std::vector<int32_t>& v, int32_t l) {
        return std::find(v.begin(), v.end(), l) != v.end();
      };
      std::vector<int32_t> sh, fa, fb;
      for (int32_t l : A.legs) (in(Bt.legs, l) ? sh : fa).push_back(l);
      for (int32_t l : Bt.legs)
        if (!in(A.legs, l)) fb.push_back(l);
      const uint32_t rows = (A.batched || Bt.batched) && B > 1 ? (uint32_t)B : 1u;
      if (!block_gemm_node(plan, 1u << fa.size(), 1u << fb.size(), 1u << sh.size(), rows)) continue;
      if (a >= nl && b < nl) {  // B's order of the contracted legs
        sh.clear();
        for (int32_t l : Bt.legs)
          if (in(A.legs, l)) sh.push_back(l);
      }
      if (a >= nl) {
        A.legs = fa;
        A.legs.insert(A.legs.end(), sh.begin(), sh.end());
      }
      if (b >= nl) {
        Bt.legs = sh;
        Bt.legs.insert(Bt.legs.end(), fb.begin(), fb.end());
      }
    }
    if (ns > 0) {
      I.root = ns - 1;
      if (!T[I.tid[I.root]].legs.empty()) fail(TC_ERR_INVALID_ARG, "network is not closed");
    }
  }
  const int32_t Lf = S.max_level;
  const bool ck = grad && ckpt >= 2;
  auto seg_of = [&](int32_t level) { return level <= 0 ? -1 : (level - 1) / ckpt; };

  // ---- timeline of one group: forward levels 1..Lf, one empty step, then
  // for each checkpoint segment from the top its recompute steps (ascending
  // levels) and its adjoint steps (descending); groups follow each other,
  // then the root sum and the gradient sum
  const int32_t nseg = ck ? seg_of(Lf) + 1 : 1;
  std::vector<int32_t> recompute_step(Lf + 2, -1), adjoint_step(Lf + 2, -1);
  S.span = Lf;
  if (grad) {
    int32_t st = Lf + 2;
    for (int32_t sg = nseg - 1; sg >= 0; --sg) {
      const int32_t lo = ck ? sg * ckpt + 1 : 1;
      const int32_t hi = ck ? std::min((sg + 1) * ckpt, Lf) : Lf;
      if (ck)
        for (int32_t l = lo; l < hi; ++l) recompute_step[l] = st++;
      for (int32_t l = hi; l >= lo; --l) adjoint_step[l] = st++;
    }
    S.span = st - 1;
  }
  if (G < 1 || (G > 1 && (!grp || grp->size() != net.terms.size())))
    fail(TC_ERR_INVALID_ARG, "internal: term groups");
  S.root_step = G * S.span + 1;
  S.grad_step = S.root_step + 1;
  auto goff = [&](size_t t) { return G > 1 ? (*grp)[t] * S.span : 0; };

  // ---- forward ops and last uses
  for (size_t t = 0; t < net.terms.size(); ++t) {
    const TermPath& tp = path.terms[t];
    TermInfo& I = S.ti[t];
    const int32_t nl = (int32_t)net.terms[t].leaves.size();
    for (size_t s = 0; s < tp.pairs.size(); ++s) {
      int32_t a = tp.pairs[s].first, b = tp.pairs[s].second, c = nl + (int32_t)s;
      int32_t step = goff(t) + I.level[c];
      T[I.tid[c]].first = step;
      S.pend.push_back({I.tid[a], I.tid[b], I.tid[c], step, (int32_t)t, false, false});
      T[I.tid[a]].last = std::max(T[I.tid[a]].last, step);
      T[I.tid[b]].last = std::max(T[I.tid[b]].last, step);
    }
    if (I.root >= 0) T[I.tid[I.root]].last = S.root_step;
  }
  if (grad) {
    for (size_t t = 0; t < net.terms.size(); ++t) {
      const TermPath& tp = path.terms[t];
      TermInfo& I = S.ti[t];
      if (I.root < 0 || !I.needs[I.root]) continue;
      const int32_t nl = (int32_t)net.terms[t].leaves.size();
      const int32_t ns = (int32_t)I.tid.size();
      // value instance used by the reverse sweep for each SSA id
      std::vector<int32_t> val(ns);
      for (int32_t x = 0; x < ns; ++x) val[x] = I.tid[x];
      if (ck) {
        // dropped: a node whose consumer sits in the same segment
        std::vector<char> dropped(ns, 0);
        for (int32_t x = nl; x < ns; ++x)
          if (I.parent[x] >= 0 && seg_of(I.level[x]) == seg_of(I.level[I.parent[x]]))
            dropped[x] = 1;
        // recompute dropped nodes whose subtree matters for the gradient
        // (their values are operands of adjoint ops), in level order
        std::vector<int32_t> order;
        for (int32_t x = nl; x < ns; ++x)
          if (dropped[x]) order.push_back(x);
        std::stable_sort(order.begin(), order.end(),
                         [&](int32_t u, int32_t v) { return I.level[u] < I.level[v]; });
        for (int32_t x : order) {
          int32_t a = tp.pairs[x - nl].first, b = tp.pairs[x - nl].second;
          int32_t step = goff(t) + recompute_step[I.level[x]];
          PT r = T[I.tid[x]];
          r.off = -1;
          r.first = step;
          r.last = step;
          int32_t rid = (int32_t)T.size();
          T.push_back(r);
          S.pend.push_back({val[a], val[b], rid, step, (int32_t)t, true, true});
          T[val[a]].last = std::max(T[val[a]].last, step);
          T[val[b]].last = std::max(T[val[b]].last, step);
          val[x] = rid;
        }
      }
      std::vector<int32_t> adj(ns, -1);
      adj[I.root] = (int32_t)t;  // seed tensor
      for (int32_t c = ns - 1; c >= nl; --c) {
        if (adj[c] < 0) continue;
        int32_t a = tp.pairs[c - nl].first, b = tp.pairs[c - nl].second;
        int32_t step = goff(t) + adjoint_step[I.level[c]];
        for (int side = 0; side < 2; ++side) {
          int32_t x = side == 0 ? a : b, other = side == 0 ? b : a;
          if (!I.needs[x]) continue;
          const int32_t ov = val[other];
          PT d;
          // the adjoint keeps its tensor's leg order (a leaf's for the
          // gradient dot): later adjoint ops then meet operands whose shared
          // legs sit in the same order, which keeps their index groups in a
          // few bit-field runs
          d.legs = T[I.tid[x]].legs;
          d.elems = 1ull << d.legs.size();
          d.term = (int32_t)t;
          d.batched = T[adj[c]].batched || T[ov].batched;
          d.first = step;
          d.last = step;  // extended when consumed
          int32_t did = (int32_t)T.size();
          T.push_back(d);
          S.pend.push_back({adj[c], ov, did, step, (int32_t)t, true, false});
          T[adj[c]].last = std::max(T[adj[c]].last, step);
          T[ov].last = std::max(T[ov].last, step);
          adj[x] = did;
          if (x < nl) {
            S.leaf_adj.push_back({I.tid[x], did});
            S.leaf_adj_term.push_back({t, x});
          }
        }
      }
    }
  }
  for (auto& la : S.leaf_adj) T[la.second].last = S.grad_step;

  // ---- arena: allocate in step order, release after last use.  One arena
  // over all terms (level-synchronous launches order every term's steps), or
  // one region per term when terms run independently (term mode).
  const int32_t n_steps = S.grad_step + 1;
  std::vector<std::vector<int32_t>> members(per_term_arena ? net.terms.size() : 1);
  for (int32_t i = 0; i < (int32_t)T.size(); ++i)
    if (!T[i].fixed) members[per_term_arena ? T[i].term : 0].push_back(i);
  uint64_t base = S.seed_elems;
  S.group_peak.assign(G, 0);
  for (const auto& mem : members) {
    Arena ar;
    ar.top = base;
    uint64_t top = base;
    uint64_t live = 0;
    std::vector<std::vector<int32_t>> born(n_steps + 1), dies(n_steps + 2);
    for (int32_t i : mem) {
      born[T[i].first].push_back(i);
      dies[std::max(T[i].last, T[i].first) + 1].push_back(i);
    }
    for (int32_t s = 0; s < n_steps; ++s) {
      for (int32_t i : dies[s]) {
        uint64_t n = T[i].elems * (T[i].batched ? (uint64_t)B : 1);
        ar.release((uint64_t)T[i].off, n);
        live -= Arena::align(std::max<uint64_t>(n, 1));
      }
      // big tensors first keeps the best-fit layout compact
      std::sort(born[s].begin(), born[s].end(),
                [&](int32_t x, int32_t y) { return T[x].elems > T[y].elems; });
      for (int32_t i : born[s]) {
        uint64_t n = T[i].elems * (T[i].batched ? (uint64_t)B : 1);
        T[i].off = (int64_t)ar.alloc(n);
        top = std::max(top, ar.top);
        S.peak_tensor_elems = std::max(S.peak_tensor_elems, n);
        live += Arena::align(std::max<uint64_t>(n, 1));
      }
      if (s == 0) S.base_live = std::max(S.base_live, live);
      if (!per_term_arena && s >= 1 && s <= G * S.span) {
        uint64_t& gp = S.group_peak[(s - 1) / S.span];
        gp = std::max(gp, live);
      }
    }
    base = Arena::align(top);
  }
  S.arena_elems = std::max(base, S.seed_elems);
}

// LDS placement of a resident plan, term by term (each term's workgroup
// has the whole LDS arena of `cap` elements to itself).  A tensor whose
// reads all come within RES_LDS_WINDOW steps of its production (and that
// neither the root sum nor the gradient sum reads) lives in LDS alone; any
// other keeps its global copy and, where space allows, gets an LDS copy
// that serves its first reading step, so a forward value feeds the next
// node from LDS and the reverse sweep from global memory.  Short LDS
// lifetimes are placed first (they return their space soonest), each at
// the lowest offset clear of every placed tensor whose lifetime overlaps
// its own; lifetimes are inclusive step ranges, so a node's operands and
// its result never share space.
// A window [s0, s1] restricts the placement to one run of steps (a light
// run of the automatic mode): only tensors produced in it (and the leaves,
// when it materialises them) are candidates, an LDS copy serves only reads
// inside it, and a tensor read after it keeps its global copy.
constexpr int32_t RES_LDS_WINDOW = 6;

void place_lds(std::vector<PT>& T, const std::vector<PendingOp>& pend, int32_t root_step,
               uint64_t cap, size_t n_terms, int32_t s0 = 0, int32_t s1 = INT32_MAX,
               bool leaves = true) {
  std::vector<int32_t> u1(T.size(), INT32_MAX);
  for (const PendingOp& q : pend) {
    u1[q.a] = std::min(u1[q.a], q.step);
    u1[q.b] = std::min(u1[q.b], q.step);
  }
  std::vector<std::vector<int32_t>> by_term(n_terms);
  for (int32_t i = 0; i < (int32_t)T.size(); ++i)
    if (!T[i].fixed && T[i].term >= 0 && (size_t)T[i].term < n_terms) by_term[T[i].term].push_back(i);
  struct Cand {
    int32_t id, lo, hi;
    uint64_t size;
    bool keep;  // the global copy stays
  };
  struct Placed {
    uint64_t off, size;
    int32_t lo, hi;
  };
  std::vector<Cand> cs;
  std::vector<Placed> pl;
  std::vector<std::pair<uint64_t, uint64_t>> busy;
  for (const auto& ids : by_term) {
    cs.clear();
    pl.clear();
    for (int32_t id : ids) {
      const PT& x = T[id];
      if (x.elems > cap || u1[id] == INT32_MAX || u1[id] > s1) continue;
      if (x.first == 0 ? !leaves : (x.first < s0 || x.first > s1)) continue;
      const bool keep = x.last >= root_step || x.last > s1 || x.last - x.first > RES_LDS_WINDOW;
      cs.push_back({id, x.first, keep ? u1[id] : x.last, (x.elems + 7) & ~uint64_t(7), keep});
    }
    std::sort(cs.begin(), cs.end(), [](const Cand& p, const Cand& q) {
      if (p.hi - p.lo != q.hi - q.lo) return p.hi - p.lo < q.hi - q.lo;
      if (p.size != q.size) return p.size > q.size;
      return p.id < q.id;
    });
    for (const Cand& c : cs) {
      busy.clear();
      for (const Placed& p : pl)
        if (p.lo <= c.hi && c.lo <= p.hi) busy.push_back({p.off, p.off + p.size});
      std::sort(busy.begin(), busy.end());
      uint64_t off = 0;
      for (const auto& b : busy) {
        if (b.first >= off + c.size) break;
        off = std::max(off, b.second);
      }
      if (off + c.size > cap) continue;
      pl.push_back({off, c.size, c.lo, c.hi});
      PT& x = T[c.id];
      x.lds_off = (int64_t)off;
      x.lds_last = c.hi;
      x.global = c.keep;
    }
  }
}

}  // namespace

WorkspaceLayout workspace_layout(const Plan& p) {
  auto al = [](uint64_t x) { return (x + 255) & ~uint64_t(255); };
  WorkspaceLayout w{};
  uint64_t o = 0;
  w.ops = o; o = al(o + p.ops.size() * sizeof(DevOp));
  w.tabs = o; o = al(o + p.tabs.size() * sizeof(uint32_t));
  w.item_op = o; o = al(o + p.item_op.size() * sizeof(uint32_t));
  w.leaves = o; o = al(o + p.leaves.size() * sizeof(DevLeaf));
  w.ftab = o; o = al(o + p.ftab.size() * sizeof(float));
  w.uses = o; o = al(o + p.uses.size() * sizeof(DevGradUse));
  w.slot_begin = o; o = al(o + p.slot_begin.size() * sizeof(uint32_t));
  w.roots = o; o = al(o + p.roots.size() * sizeof(DevRoot));
  w.terms = o; o = al(o + p.terms.size() * sizeof(DevTerm));
  w.groups = o; o = al(o + p.groups.size() * sizeof(DevGroup));
  w.ranges = o; o = al(o + p.ranges.size() * sizeof(DevRange));
  w.rops = o; o = al(o + p.rops.size() * sizeof(DevROp));
  w.split = o; o = al(o + p.split_floats * sizeof(float));
  w.sunits = o; o = al(o + p.split_units.size() * sizeof(DevSplitUnit));
  w.gsunits = o; o = al(o + p.gsplit_units.size() * sizeof(DevSplitUnit));
  w.qslot = o; o = al(o + p.qslot_begin.size() * sizeof(uint32_t));
  w.qrows = o; o = al(o + p.qrows.size() * sizeof(uint32_t));
  const uint64_t np = (uint64_t)std::max(p.n_params, 1);
  w.params = o; o = al(o + (p.qgt ? 1 : (uint64_t)p.batch) * np * sizeof(float));
  w.value = o; o = al(o + (uint64_t)p.batch * 2 * sizeof(double));
  // (geometric tensor: complex adjoint sums per row and slot)
  w.grad = o; o = al(o + (uint64_t)p.batch * np * (p.qgt ? 2 : 1) * sizeof(double));
  w.qgt = o; o = al(o + (p.qgt ? 2 * np * np : 0) * sizeof(double));
  w.arena = o; o = al(o + p.arena_elems * 8);
  w.total = o;
  return w;
}

std::vector<const Launch*> launch_order(const Plan& p, bool with_grad) {
  std::vector<const Launch*> seq;
  seq.reserve(p.fwd.size() + (with_grad ? p.bwd.size() : 0));
  size_t i = 0, j = 0;
  while (i < p.fwd.size() || (with_grad && j < p.bwd.size())) {
    const bool take_fwd = i < p.fwd.size() &&
                          (!with_grad || j >= p.bwd.size() || p.fwd[i].step <= p.bwd[j].step);
    const Launch* L = take_fwd ? &p.fwd[i++] : &p.bwd[j++];
    // a resident plan's forward-only launch gives way to the launch that
    // runs both the forward pass and the reverse sweep
    if (with_grad && L->resident == 1) continue;
    seq.push_back(L);
  }
  return seq;
}

void build_plan(Plan& plan, const Network& net, const Path& path) {
  if (plan.qgt) {
    // one row per gate use of a parameter on the ket side
    if (net.obs_kind != TC_OBS_STATE)
      fail(TC_ERR_INVALID_ARG, "the geometric tensor needs a network built for TC_OBS_STATE");
    if (plan.batch != 1)
      fail(TC_ERR_INVALID_ARG, "geometric tensor plans take one parameter vector (batch 1)");
    int32_t u = 0;
    for (const Term& term : net.terms)
      for (const Leaf& lf : term.leaves)
        if (lf.kind == LEAF_GATE && !lf.conj && leaf_param_dependent(net, lf)) {
          const GateRec& g = net.gates[lf.gate];
          for (int a = 0; a < g.n_angles; ++a)
            u += g.param[a] >= 0 && gate_angle_differentiable(g.kind, a);
        }
    plan.qgt_rows = u;
    plan.batch = std::max(u, 1);
    plan.want_grad = 1;
  }
  const int B = plan.batch;
  const bool grad = plan.want_grad != 0;
  plan.n_params = net.n_params;
  plan.n_terms = (int32_t)net.terms.size();
  if (path.terms.size() != net.terms.size()) fail(TC_ERR_INVALID_ARG, "path does not match network");

  // ---- schedule under the memory budget: all terms level by level; if
  // their live intermediates do not fit, terms in groups run one group
  // after another; with a gradient, then checkpointed segments (which
  // recompute forward values), alone or with groups
  Schedule S;
  int ckpt = plan.checkpoint > 0 ? plan.checkpoint : 0;
  std::vector<int32_t> grp;
  int32_t G = 1;
  schedule(S, plan, net, path, B, grad, ckpt, false);
  // bytes of the op records and per-item op tables (an upper estimate:
  // every gather item of every op), which share the budget with the arena
  uint64_t tab_est = 0;
  if (plan.budget) {
    int32_t nlab = 0;
    for (const Term& term : net.terms) nlab = std::max(nlab, term.n_labels);
    std::vector<char> inb(nlab, 0);
    double items = 0;
    for (const PendingOp& q : S.pend) {
      const PT& A = S.T[q.a];
      const PT& Bt = S.T[q.b];
      for (int32_t l : Bt.legs) inb[l] = 1;
      uint32_t sh = 0;
      for (int32_t l : A.legs) sh += inb[l];
      for (int32_t l : Bt.legs) inb[l] = 0;
      const uint32_t K = 1u << sh, M = 1u << (A.legs.size() - sh), N = 1u << (Bt.legs.size() - sh);
      const uint32_t rows = (A.batched || Bt.batched) && B > 1 ? (uint32_t)B : 1u;
      items += (double)std::min<uint64_t>(gather_items(M, N, K, rows, LEVEL_LANES), ITEM_TABLE_MAX);
    }
    const double b = (double)S.pend.size() * sizeof(DevOp) +
                     4.0 * std::min(items, (double)ITEM_TABLES_TOTAL_MAX);
    // plus the split-K partial tiles, held to a sixteenth of the budget
    tab_est = (uint64_t)(1.25 * b) + (uint64_t(1) << 16) + plan.budget / 16;
  }
  auto over = [&](const Schedule& x) {
    return plan.budget && x.arena_elems * 8 + tab_est > plan.budget;
  };
  const size_t nt = net.terms.size();
  // groups of consecutive terms whose live intermediates (estimated from
  // each term's peak when run alone) fit 80 % of the budget, the rest
  // being left for tables and split regions; fewer terms per group until
  // the arena fits
  uint64_t single_term_bytes = ~uint64_t(0);  // arena with one term at a time, if tried
  auto try_groups = [&](int c) {
    if (nt < 2 || plan.exec_mode == 2) return false;
    std::vector<int32_t> one(nt);
    for (size_t t = 0; t < nt; ++t) one[t] = (int32_t)t;
    Schedule s1;
    schedule(s1, plan, net, path, B, grad, c, false, &one, (int32_t)nt);
    single_term_bytes = std::min(single_term_bytes, s1.arena_elems * 8);
    if (over(s1)) return false;
    const double cap = 0.9 * (double)(plan.budget - std::min(tab_est, plan.budget)) / 8.0;
    for (double f : {1.0, 0.6, 0.35, 0.0}) {
      std::vector<int32_t> g(nt);
      int32_t ng = 0;
      double acc = 0;
      for (size_t t = 0; t < nt; ++t) {
        const double need = (double)(s1.group_peak[t] > s1.base_live ? s1.group_peak[t] - s1.base_live : 0);
        if (t > 0 && (f == 0.0 || s1.base_live + acc + need > f * cap)) {
          ++ng;
          acc = 0;
        }
        g[t] = ng;
        acc += need;
      }
      ++ng;
      if (ng == (int32_t)nt) {
        S = std::move(s1);
        grp = std::move(one);
        G = ng;
        ckpt = c;
        return true;
      }
      Schedule sg;
      schedule(sg, plan, net, path, B, grad, c, false, &g, ng);
      if (!over(sg)) {
        S = std::move(sg);
        grp = std::move(g);
        G = ng;
        ckpt = c;
        return true;
      }
    }
    return false;
  };
  if (over(S) && !try_groups(ckpt) && grad && plan.checkpoint == 0 && S.max_level >= 4) {
    // smallest arena over a few segment lengths
    Schedule best;
    int best_c = 0;
    // (segments of about sqrt(levels) keep the fewest values for deep
    // trees, so longer segments are tried as well)
    for (int c : {2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64, 96, 128}) {
      if (c > std::max(2, S.max_level / 2)) break;
      Schedule t;
      schedule(t, plan, net, path, B, grad, c, false);
      if (!best_c || t.arena_elems < best.arena_elems) {
        best = std::move(t);
        best_c = c;
      }
    }
    if (best_c && !over(best)) {
      S = std::move(best);
      ckpt = best_c;
    } else if (best_c) {
      if (!try_groups(best_c) && best.arena_elems < S.arena_elems) {
        S = std::move(best);
        ckpt = best_c;
      }
    }
  }
  plan.term_groups = G;
  // leg label -> position in one operand's storage order (-1: absent)
  int32_t n_labels = 0;
  for (const Term& term : net.terms) n_labels = std::max(n_labels, term.n_labels);
  std::vector<int8_t> pa(n_labels, -1), pb(n_labels, -1), pc(n_labels, -1);
  auto mark = [&](std::vector<int8_t>& pos, const std::vector<int32_t>& legs, bool on) {
    for (size_t x = 0; x < legs.size(); ++x) {
      if (legs[x] < 0 || legs[x] >= n_labels) fail(TC_ERR_INVALID_ARG, "internal: leg label out of range");
      pos[legs[x]] = on ? (int8_t)x : (int8_t)-1;
    }
  };
  auto gemm_node = [&](uint32_t M, uint32_t N, uint32_t K, uint32_t rows) {
    return K >= (uint32_t)plan.gemm_min_k && M >= (uint32_t)plan.gemm_min_mn &&
           N >= (uint32_t)plan.gemm_min_mn && (uint64_t)rows * M * N * K >= plan.gemm_min_macs;
  };

  // ---- execution mode, step by step.  A step runs either as a level
  // launch (all terms' nodes at that step, k_gemm + k_gather over the whole
  // chip) or inside a term launch: one workgroup per term runs the term's
  // nodes of a run of consecutive steps with workgroup barriers in between,
  // so a run of k steps costs one kernel instead of k.  A workgroup is one
  // CU, so only light steps go to term launches: at batch 1, no node for the
  // GEMM path and no term with more gather items than two per thread; and
  // only runs of at least two such steps (one step gains nothing).  Terms
  // then advance independently, so each term gets its own arena region.
  std::map<int32_t, bool> light;  // step -> light
  {
    std::map<std::pair<int32_t, int32_t>, uint64_t> items;  // (step, term) -> items
    for (const PendingOp& q : S.pend) {
      bool& l = light.emplace(q.step, true).first->second;
      const PT& A = S.T[q.a];
      const PT& Bt = S.T[q.b];
      mark(pb, Bt.legs, true);
      uint32_t sh = 0;
      for (int32_t x : A.legs) sh += pb[x] >= 0;
      mark(pb, Bt.legs, false);
      const uint32_t K = 1u << sh, M = 1u << (A.legs.size() - sh), N = 1u << (Bt.legs.size() - sh);
      uint64_t& n_items = items[{q.step, q.term}];
      uint32_t ls, lv;
      gather_shape(M, N, K, 1, TERM_LANES, ls, lv);
      if (ls) n_items = (n_items + 63) & ~uint64_t(63);  // k-split ops start on a wavefront
      n_items += gather_items(M, N, K, 1, TERM_LANES);
      // one CU walks the term's sums: light means few items and short sums
      if (B != 1 || gemm_node(M, N, K, 1) || n_items > TERM_MODE_MAX_ITEMS ||
          (K >> ls) > TERM_MODE_MAX_KSTEPS)
        l = false;
    }
  }
  std::map<int32_t, bool> term_step;  // step -> runs inside a term launch
  for (auto it = light.begin(); it != light.end(); ++it) {
    bool t = plan.exec_mode == 2;
    if (plan.exec_mode == 0 && it->second) {
      auto nx = std::next(it);
      const bool prev_light = it != light.begin() && std::prev(it)->first == it->first - 1 &&
                              std::prev(it)->second;
      const bool next_light = nx != light.end() && nx->first == it->first + 1 && nx->second;
      t = prev_light || next_light;
    }
    term_step[it->first] = t;
  }
  if (G > 1)  // groups run level launches only
    for (auto& ts : term_step) ts.second = false;
  // Resident term launches: one workgroup per term runs every step, the
  // leaves first and the reverse sweep after the forward pass, in a single
  // kernel; tensors placed in the workgroup's LDS arena are read and
  // written there, so a step costs a workgroup barrier and LDS traffic
  // instead of a kernel launch and dependent global-memory round trips.
  // Batch 1, one term group, every node on the gather path, and an LDS
  // arena from the device.
  plan.resident = false;
  if (plan.exec_mode == 3 || plan.exec_mode == 0) {
    bool ok = B == 1 && G == 1 && !plan.qgt && plan.lds_elems >= 1024;
    for (size_t k = 0; ok && k < S.pend.size(); ++k) {
      const PT& A = S.T[S.pend[k].a];
      const PT& Bt = S.T[S.pend[k].b];
      mark(pb, Bt.legs, true);
      uint32_t sh = 0;
      for (int32_t x : A.legs) sh += pb[x] >= 0;
      mark(pb, Bt.legs, false);
      if (gemm_node(1u << (A.legs.size() - sh), 1u << (Bt.legs.size() - sh), 1u << sh, 1)) ok = false;
    }
    if (plan.exec_mode == 3 && !ok)
      fail(TC_ERR_UNSUPPORTED, "resident term launches need batch 1, one term group, no node for "
                               "the GEMM path and a device LDS arena");
    plan.resident = ok && plan.exec_mode == 3;
  }
  if (plan.resident)
    for (auto& ts : term_step) ts.second = true;
  bool any_term = false, any_level = false;
  for (const auto& ts : term_step) (ts.second ? any_term : any_level) = true;
  if (any_term) {
    Schedule St;
    schedule(St, plan, net, path, B, grad, ckpt, true);
    // automatic choice: only while the separate regions stay modest
    const bool fits = !plan.budget || St.arena_elems * 8 <= plan.budget;
    const bool modest = St.arena_elems <= std::max<uint64_t>(4 * S.arena_elems, uint64_t(1) << 25);
    if (plan.exec_mode == 2 || plan.exec_mode == 3 || (fits && modest)) {
      S = std::move(St);
    } else {
      for (auto& ts : term_step) ts.second = false;
      any_term = false;
      any_level = true;
      plan.resident = false;
    }
  }
  plan.term_mode = any_term;
  plan.exec_used = plan.resident ? 4 : any_term ? (any_level ? 3 : 2) : 1;
  // automatic mode: the forward runs of light steps become resident runs
  // (their tensors in LDS where they fit, placed run by run) when the
  // device has an LDS arena and the global arena fits 32-bit offsets
  plan.resident_runs = plan.exec_mode == 0 && any_term && B == 1 && !plan.qgt &&
                       plan.lds_elems >= 1024 && S.arena_elems < (uint64_t(1) << 32);
  if (plan.resident) {
    if (S.arena_elems >= (uint64_t(1) << 32))
      fail(TC_ERR_TOO_LARGE, "resident term launches address the global arena with 32-bit offsets");
    place_lds(S.T, S.pend, S.root_step, plan.lds_elems, net.terms.size());
  } else if (plan.resident_runs) {
    // the runs as the op emission below forms them: consecutive term steps
    // (in step order) of one phase
    std::map<int32_t, bool> bwd_step;
    for (const PendingOp& q : S.pend) bwd_step[q.step] = q.bwd;
    int32_t r0 = -1, r1 = -1;
    bool rb = false;
    // (forward runs only: a reverse-sweep run reads mostly forward values
    // kept in global memory, and measured slower as a resident launch
    // than as a plain term launch on the 20-qubit chain, 21 against 11 us)
    auto flush = [&]() {
      if (r0 >= 0 && !rb)
        place_lds(S.T, S.pend, S.root_step, plan.lds_elems, net.terms.size(), r0, r1, r0 == 1);
      r0 = -1;
    };
    for (const auto& ts : term_step) {
      const bool b = bwd_step.at(ts.first);
      if (!ts.second || (r0 >= 0 && b != rb)) flush();
      if (!ts.second) continue;
      if (r0 < 0) {
        r0 = ts.first;
        rb = b;
      }
      r1 = ts.first;
    }
    flush();
  }

  plan.checkpoint_used = grad ? ckpt : 0;
  plan.arena_elems = S.arena_elems;
  plan.peak_tensor_elems = S.peak_tensor_elems;
  // the arena alone already exceeds the budget: stop before building tables
  if (plan.budget && plan.arena_elems * 8 > plan.budget) {
    if (single_term_bytes != ~uint64_t(0) && single_term_bytes > plan.budget)
      fail(TC_ERR_TOO_LARGE, "live intermediates need " + std::to_string(single_term_bytes) +
                                 " bytes even with one term at a time, more than the memory budget");
    fail(TC_ERR_TOO_LARGE, "live intermediates need " + std::to_string(plan.arena_elems * 8) +
                               " bytes, more than the memory budget");
  }
  std::vector<PT>& T = S.T;
  std::vector<PendingOp>& pend = S.pend;
  std::vector<TermInfo>& ti = S.ti;
  const uint64_t seed_elems = S.seed_elems;
  for (size_t t = 0; t < net.terms.size(); ++t) {
    plan.seeds.push_back((float)net.terms[t].weight);
    plan.seeds.push_back(0.0f);
  }
  Tables tables(plan.tabs);

  // ---- contraction ops: a level launch per level step; for a term step,
  // one group per term, collected into the open term launch
  std::stable_sort(pend.begin(), pend.end(), [](const PendingOp& x, const PendingOp& y) {
    return x.step != y.step ? x.step < y.step : x.term < y.term;
  });
  double flops = 0, bytes = 0, gflops = 0, gbytes = 0;
  int32_t n_gemm_nodes = 0;
  plan.terms.assign(net.terms.size(), DevTerm{});
  const uint32_t n_terms = (uint32_t)net.terms.size();
  // the open term launch: its groups start at seg_begin (each tagged with
  // its term in group_term), its phase and algorithmic totals
  bool seg_open = false, seg_bwd = false;
  int32_t seg_first_step = 0;
  size_t seg_begin = 0;
  double seg_flops = 0, seg_bytes = 0, seg_fflops = 0, seg_fbytes = 0;
  std::vector<uint32_t> group_term;
  std::vector<char> group_bwd;
  auto close_segment = [&]() {
    if (!seg_open) return;
    // groups by term (stable: each term's steps stay in order), then one
    // [begin, end) range per term
    std::vector<size_t> ord(plan.groups.size() - seg_begin);
    for (size_t x = 0; x < ord.size(); ++x) ord[x] = seg_begin + x;
    std::stable_sort(ord.begin(), ord.end(),
                     [&](size_t x, size_t y) { return group_term[x] < group_term[y]; });
    std::vector<DevGroup> gs;
    std::vector<uint32_t> gt;
    std::vector<char> gb;
    for (size_t x : ord) {
      gs.push_back(plan.groups[x]);
      gt.push_back(group_term[x]);
      gb.push_back(group_bwd[x]);
    }
    std::copy(gs.begin(), gs.end(), plan.groups.begin() + seg_begin);
    std::copy(gt.begin(), gt.end(), group_term.begin() + seg_begin);
    std::copy(gb.begin(), gb.end(), group_bwd.begin() + seg_begin);
    Launch L;
    L.kind = L_TERM;
    L.step = seg_first_step;
    L.begin = (uint32_t)plan.ranges.size();
    L.with_leaves = seg_first_step == 1;  // the first term launch also materialises the leaves
    L.flops = seg_flops;
    L.bytes = seg_bytes;
    size_t g = seg_begin;
    for (uint32_t t = 0; t < n_terms; ++t) {
      DevRange R{(uint32_t)g, (uint32_t)g};
      while (g < plan.groups.size() && group_term[g] == t) ++g;
      R.g_end = (uint32_t)g;
      plan.ranges.push_back(R);
    }
    if (plan.resident) {
      // one launch holds every step; calls without the gradient run each
      // term's forward groups only (they precede its reverse-sweep groups)
      Launch F = L;
      F.resident = 1;
      F.begin = (uint32_t)plan.ranges.size();
      F.flops = seg_fflops;
      F.bytes = seg_fbytes;
      for (uint32_t t = 0; t < n_terms; ++t) {
        DevRange R = plan.ranges[L.begin + t];
        uint32_t e = R.g_begin;
        while (e < R.g_end && !group_bwd[e]) ++e;
        for (uint32_t x = e; x < R.g_end; ++x)
          if (!group_bwd[x]) fail(TC_ERR_INVALID_ARG, "internal: forward group after the reverse sweep");
        R.g_end = e;
        plan.ranges.push_back(R);
      }
      plan.fwd.push_back(F);
      if (grad) {
        L.resident = 2;
        plan.bwd.push_back(L);
      }
    } else {
      if (plan.resident_runs && !seg_bwd) L.resident = 3;
      (seg_bwd ? plan.bwd : plan.fwd).push_back(L);
    }
    seg_open = false;
  };
  std::vector<int32_t> Sh, FA, FB;
  size_t i = 0;
  while (i < pend.size()) {
    const bool tstep = term_step.at(pend[i].step);
    if (!tstep || (seg_open && !plan.resident && seg_bwd != pend[i].bwd)) close_segment();
    if (tstep && !seg_open) {
      seg_open = true;
      seg_bwd = pend[i].bwd;
      seg_first_step = pend[i].step;
      seg_begin = plan.groups.size();
      seg_flops = seg_bytes = seg_fflops = seg_fbytes = 0;
    }
    // a level step takes every term's ops at the step, a term step one term's
    size_t j = i;
    while (j < pend.size() && pend[j].step == pend[i].step &&
           (!tstep || pend[j].term == pend[i].term))
      ++j;
    const bool term_mode = tstep;
    // a level with more gather items than two chip-fulls (at 4 k-steps per
    // lane) splits its sums half as far: fewer, longer items in one pass
    uint32_t min_steps = 4;
    if (!term_mode) {
      uint64_t li = 0;
      for (size_t k = i; k < j; ++k) {
        const PT& A = T[pend[k].a];
        const PT& Bt = T[pend[k].b];
        mark(pb, Bt.legs, true);
        uint32_t sh = 0;
        for (int32_t x : A.legs) sh += pb[x] >= 0;
        mark(pb, Bt.legs, false);
        const uint32_t K = 1u << sh, M = 1u << (A.legs.size() - sh), N = 1u << (Bt.legs.size() - sh);
        const uint32_t rows = (A.batched || Bt.batched) && B > 1 ? (uint32_t)B : 1u;
        li += gather_items(M, N, K, rows, LEVEL_LANES);
      }
      if (li > LEVEL_SHORT_SPLIT_ITEMS) min_steps = 8;
    }
    std::vector<DevOp> gc, gm, wv, wd, rt;
    std::vector<DevROp> gcr;  // resident plans: gc's nodes as resident records
    double lf = 0, lb = 0, gf = 0, gb = 0, wf = 0, wb = 0, rtf = 0, rtby = 0, sgf = 0, sgby = 0;
    for (size_t k = i; k < j; ++k) {
      const PT& A = T[pend[k].a];
      const PT& Bt = T[pend[k].b];
      const PT& C = T[pend[k].c];
      mark(pa, A.legs, true);
      mark(pb, Bt.legs, true);
      mark(pc, C.legs, true);
      Sh.clear();
      FA.clear();
      FB.clear();
      for (int32_t l : A.legs) (pb[l] >= 0 ? Sh : FA).push_back(l);
      for (int32_t l : Bt.legs)
        if (pa[l] < 0) FB.push_back(l);
      // Coalescing: an operand reads contiguously along m (n) when its
      // fastest leg is free and along k when its fastest leg is the last
      // contracted index.  A's fastest leg is one or the other; when it is
      // free, the contracted legs follow B's order so that B's fastest leg,
      // if contracted, becomes the last contracted index.
      if (!A.legs.empty() && pb[A.legs.back()] < 0)
        std::sort(Sh.begin(), Sh.end(), [&](int32_t x, int32_t y) { return pb[x] < pb[y]; });
      DevOp op{};
      op.ksplit = 1;
      op.a = (uint64_t)A.off;
      op.b = (uint64_t)Bt.off;
      op.c = (uint64_t)C.off;
      op.M = 1u << FA.size();
      op.N = 1u << FB.size();
      op.K = 1u << Sh.size();
      const int ra = (int)A.legs.size(), rb = (int)Bt.legs.size(), rc = (int)C.legs.size();
      op.a_m = tables.gather(pa, ra, FA);
      op.a_k = tables.gather(pa, ra, Sh);
      op.b_k = tables.gather(pb, rb, Sh);
      op.b_n = tables.gather(pb, rb, FB);
      op.c_m = tables.gather(pc, rc, FA);
      op.c_n = tables.gather(pc, rc, FB);
      mark(pa, A.legs, false);
      mark(pb, Bt.legs, false);
      mark(pc, C.legs, false);
      bool rowsB = (A.batched || Bt.batched) && B > 1;
      op.rows = rowsB ? (uint32_t)B : 1u;
      op.a_bs = (A.batched && B > 1) ? (uint32_t)A.elems : 0u;
      op.b_bs = (Bt.batched && B > 1) ? (uint32_t)Bt.elems : 0u;
      op.c_bs = rowsB ? (uint32_t)C.elems : 0u;
      double f = 8.0 * op.M * op.N * op.K * op.rows;
      double by = 8.0 * (A.elems * (A.batched ? op.rows : 1) +
                         Bt.elems * (Bt.batched ? op.rows : 1) + C.elems * op.rows);
      if (pend[k].bwd) {
        gflops += f;
        gbytes += by;
      } else {
        flops += f;
        bytes += by;
      }
      lf += f;
      lb += by;
      const bool to_gemm = !term_mode && gemm_node(op.M, op.N, op.K, op.rows);
      // batched nodes too narrow for the GEMM rule (a small block absorbed
      // into every batch row) take masked wave tiles: one wavefront reads a
      // row's operands once, where gather items read them once per output
      // group.  Below 8 in M, N or K a tile's fixed costs outweigh that
      // (measured on the 1024-row VQE sweep: 23.1 ms per evaluation with
      // this rule, 26.5 ms without masked tiles, 40 ms with every node of
      // M, N >= 2 and K >= 4 on them).
      const bool small_wave = !term_mode && !to_gemm && op.rows >= SMALL_WAVE_MIN_ROWS &&
                              op.K >= 8 && op.M >= 8 && op.N >= 8;
      if (to_gemm || small_wave) {
        gf += f;
        gb += by;
      }
      // k-contiguity of the operands picks the GEMM's load pattern
      if (op.K > 1 && ix_host(plan.tabs, op.a_k, 1) == 1) op.flags |= 1u;
      if (op.K > 1 && ix_host(plan.tabs, op.b_k, 1) == 1) op.flags |= 2u;
      const bool block_tile = op.M >= (uint32_t)plan.block_tile_min_mn &&
                              op.N >= (uint32_t)plan.block_tile_min_mn &&
                              op.K >= (uint32_t)plan.block_tile_min_k;
      // wide tiles: dense operands, A as [m][k] and B as [k][n] (element
      // offsets even, for 16-byte loads), and at least one 128 x 128 tile
      // per CU of the 256
      const uint32_t lm = __builtin_ctz(op.M), ln = __builtin_ctz(op.N), lk = __builtin_ctz(op.K);
      const bool dense = op.a_k == lk && op.a_m == (lm | (lk << 5)) && op.b_n == ln &&
                         op.b_k == (lk | (ln << 5)) && op.a % 2 == 0 && op.b % 2 == 0 &&
                         op.a_bs % 2 == 0 && op.b_bs % 2 == 0;
      // (split BF16: the operands' BF16 planes take 8 bytes per element of
      // workspace, which must fit the memory budget)
      const uint64_t planes_bytes =
          8 * ((A.batched && B > 1 ? op.rows : 1) * (uint64_t)op.M * op.K +
               (Bt.batched && B > 1 ? op.rows : 1) * (uint64_t)op.N * op.K);
      const bool planes_fit = !plan.budget ||
                              plan.arena_elems * 8 + planes_bytes <= plan.budget;
      const bool wide = to_gemm && block_tile && plan.wide_tiles && dense && op.M >= 128 &&
                        op.N >= 128 && op.K >= 32 && planes_fit &&
                        (plan.wide_tiles == 2 || (uint64_t)op.rows * (op.M / 128) * (op.N / 128) >= 256);
      if (wide) {
        wf += f;
        wb += by;
        op.tiles_m = op.M / 128;
        op.tiles_n = op.N / 128;
        op.flags |= OPF_WIDE;
        wd.push_back(op);
        if (!pend[k].bwd) ++n_gemm_nodes;
      } else if (to_gemm && block_tile) {
        op.tiles_m = (op.M + 63) / 64;
        op.tiles_n = (op.N + 63) / 64;
        gm.push_back(op);
        if (!pend[k].bwd) ++n_gemm_nodes;
      } else if ((to_gemm && op.K >= 4) || small_wave) {
        // one wavefront per (16 BI) x (16 BJ) block of one row (M or N
        // below 16: one block, rows or columns past the edge masked)
        const uint32_t bi = op.M >= 32 ? 2 : 1, bj = op.N >= 32 ? 2 : 1;
        op.tiles_m = std::max(1u, op.M / (16 * bi));
        op.tiles_n = std::max(1u, op.N / (16 * bj));
        op.flags |= ((bi - 1) << 12) | ((bj - 1) << 13);
        {
          const uint32_t lk2 = __builtin_ctz(op.K);
          const bool tabs = ((op.a_m | op.a_k | op.b_k | op.b_n | op.c_m | op.c_n) & IX_TABLE) != 0;
          if (!tabs && op.K >= 16 && op.a_k == lk2 && op.a % 2 == 0 && op.a_bs % 2 == 0)
            op.flags |= OPF_AVEC;
        }
        wv.push_back(op);
        if (!pend[k].bwd) ++n_gemm_nodes;
      } else if (!term_mode && op.rows >= SMALL_WAVE_MIN_ROWS &&
                 (uint64_t)op.M * op.K + (uint64_t)op.K * op.N <= ROW_TILE_ELEMS) {
        // row tiles: a batched node small per row (a gate absorbed into
        // every row): a workgroup copies RPB whole rows of both operands
        // into LDS once (coalesced: a row of a batched tensor is one block)
        // and computes their outputs from there, where gather items would
        // re-read the shared operand once per output group.  RPB (in
        // tiles_m) is the largest power of two <= ROW_TILE_ROWS whose rows
        // fit ROW_TILE_LDS.
        const uint64_t per_row = (uint64_t)op.M * op.K + (uint64_t)op.K * op.N;
        uint32_t rpb = 1;
        while (rpb < ROW_TILE_ROWS && 2 * rpb * per_row <= ROW_TILE_LDS) rpb *= 2;
        op.tiles_m = rpb;
        op.tiles_n = (op.rows + rpb - 1) / rpb;
        rt.push_back(op);
        rtf += f;
        rtby += by;
      } else {
        // gather: split long sums over up to 64 lanes while the op is small,
        // else 4 outputs per thread along n
        uint32_t ls, lv;
        gather_shape(op.M, op.N, op.K, op.rows, term_mode ? TERM_LANES : LEVEL_LANES, ls, lv, min_steps);
        op.flags |= (ls << 4) | (lv << 8);
        // a sum too long even for 64 lanes (few outputs, huge K: a final
        // inner product) is cut into slices reduced afterwards, as split-K
        if (!term_mode && (op.K >> ls) > 256) {
          // (partial sums of one op: at most a sixteenth of a memory budget)
          const uint64_t outs = (uint64_t)op.rows * op.M * (op.N >> lv);
          uint32_t P = 1;
          while (P < 65536 && (op.K >> ls) / P > 256 &&
                 (!plan.budget || outs * 2 * P * 2 * 4 <= plan.budget / 16))
            P *= 2;
          op.ksplit = P;
          if (P > 1) {
            sgf += f;
            sgby += by;
          }
        }
        gc.push_back(op);
        if (plan.resident || (plan.resident_runs && term_mode && !pend[k].bwd)) {
          // where each operand is read at this step, and where C goes
          const int32_t st = pend[k].step;
          DevROp r{};
          uint32_t shape = (uint32_t)__builtin_ctz(op.M) | ((uint32_t)__builtin_ctz(op.N) << 5) |
                           ((uint32_t)__builtin_ctz(op.K) << 10) | (ls << 15) | (lv << 18);
          auto src = [&](const PT& x, uint32_t flag) -> uint32_t {
            if (x.lds_off >= 0 && st <= x.lds_last) {
              shape |= flag;
              return (uint32_t)x.lds_off;
            }
            if (!x.global || x.off < 0) fail(TC_ERR_INVALID_ARG, "internal: resident operand has no copy");
            return (uint32_t)x.off;
          };
          r.a = src(A, RES_A_LDS);
          r.b = src(Bt, RES_B_LDS);
          if (C.lds_off >= 0) {
            shape |= RES_C_LDS;
            r.c = (uint32_t)C.lds_off;
            if (C.global) {
              shape |= RES_C2;
              r.c2 = (uint32_t)C.off;
            }
          } else {
            r.c = (uint32_t)C.off;
          }
          r.a_m = op.a_m;
          r.a_k = op.a_k;
          r.b_k = op.b_k;
          r.b_n = op.b_n;
          r.c_m = op.c_m;
          r.c_n = op.c_n;
          for (uint32_t d : {op.a_m, op.a_k, op.b_k, op.b_n, op.c_m, op.c_n})
            if (d & IX_TABLE) shape |= RES_TABLES;
          r.shape = shape;
          gcr.push_back(r);
        }
      }
    }
    Launch L;
    L.kind = L_LEVEL;
    L.step = pend[i].step;
    L.flops = lf;
    L.bytes = lb;
    L.gemm_flops = gf;
    L.gemm_bytes = gb;
    L.wide_flops = wf;
    L.wide_bytes = wb;
    L.rt_flops = rtf;
    L.rt_bytes = rtby;
    L.gs_flops = sgf;
    L.gs_bytes = sgby;
    // split-K: a GEMM node with too few output tiles to fill the chip (256
    // CUs) cuts K into slices of at least 64; each slice writes a partial
    // tile and the level's reduction kernel adds them in slice order.  The
    // partial tiles of one level reuse the region of every other level's
    // (levels never overlap).
    // Under a memory budget the partial tiles of a level get at most a
    // sixteenth of it (fewer slices; the result does not change).
    uint64_t part = 0;
    L.gbegin = (uint32_t)plan.ops.size();
    L.sbegin = (uint32_t)plan.split_units.size();
    auto split = [&](DevOp& op, uint64_t target_units, uint64_t floats_per_tile) {
      const uint64_t base = (uint64_t)op.rows * op.tiles_m * op.tiles_n;
      uint32_t P = 1;
      while (P < 64 && base * P < target_units && op.K / (2 * P) >= 64 &&
             (!plan.budget || (part + base * 2 * P * floats_per_tile) * 4 <= plan.budget / 16))
        P *= 2;
      op.ksplit = P;
      if (P > 1) {
        op.part = part;
        part += base * P * floats_per_tile;
        const uint32_t rel = (uint32_t)(plan.ops.size() - L.gbegin);  // op's index in the level
        for (uint64_t t = 0; t < base; ++t) plan.split_units.push_back({rel, (uint32_t)t});
      }
      return base * P;
    };
    uint64_t tiles = 0;
    for (DevOp& op : gm) {
      op.work0 = tiles;
      tiles += split(op, 512, 32 * 256);  // 32 accumulators per thread, 256 threads
      plan.ops.push_back(op);
    }
    L.gend = (uint32_t)plan.ops.size();
    L.tiles = tiles;
    L.wbegin = (uint32_t)plan.ops.size();
    uint64_t wtiles = 0;
    for (DevOp& op : wv) {
      op.work0 = wtiles;
      const uint64_t blocks = (uint64_t)((op.flags >> 12) & 1u ? 2 : 1) * ((op.flags >> 13) & 1u ? 2 : 1);
      wtiles += split(op, 2048, 8 * blocks * 64);  // 8 accumulators per 16x16 block and lane
      plan.ops.push_back(op);
    }
    plan.split_floats = std::max(plan.split_floats, part);
    L.send = (uint32_t)plan.split_units.size();
    L.wend = (uint32_t)plan.ops.size();
    L.wtiles = wtiles;
    if (wtiles && wtiles <= WAVE_TABLE_MAX &&
        plan.item_op.size() + wtiles <= ITEM_TABLES_TOTAL_MAX) {
      // wave tile -> op (relative to L.wbegin): one load instead of a search
      L.wunit_begin = plan.item_op.size();
      plan.item_op.resize(plan.item_op.size() + wtiles);
      uint32_t* it = plan.item_op.data() + L.wunit_begin;
      for (uint32_t o = L.wbegin; o < L.wend; ++o) {
        const uint64_t lo = plan.ops[o].work0;
        const uint64_t hi = o + 1 < L.wend ? plan.ops[o + 1].work0 : wtiles;
        for (uint64_t x = lo; x < hi; ++x) it[x] = o - L.wbegin;
      }
    }
    // wide tiles read their operands as planes written by the level's split
    // pass into the split region (FP32: re and im planes, k-major; split
    // BF16: re-hi, re-lo, im-hi, im-lo planes interleaved by stage, each
    // row's 32-k stage one 256-byte block of the four planes' 64 bytes;
    // 8 bytes per element either way), A's planes then B's from op.part.
    L.hbegin = (uint32_t)plan.ops.size();
    for (DevOp& op : wd) {
      op.work0 = L.htiles;
      L.htiles += (uint64_t)op.rows * op.tiles_m * op.tiles_n;
      {
        part = (part + 63) & ~uint64_t(63);
        op.part = part;
        const uint64_t ra = op.a_bs ? op.rows : 1, rb = op.b_bs ? op.rows : 1;
        const uint64_t chunks = (ra * op.M + rb * op.N) * (op.K / 8);
        part += chunks * 16;  // 64 bytes per 8 elements, in either precision
        L.wchunks += chunks;
      }
      plan.ops.push_back(op);
    }
    L.hend = (uint32_t)plan.ops.size();
    // gather ops: the split ones last, in a work space and a kernel of
    // their own (their partial sums go to the split region, slice-major,
    // and a reduction over 256-output chunks adds them)
    std::stable_partition(gc.begin(), gc.end(), [](const DevOp& op) { return op.ksplit == 1; });
    const bool res_step = plan.resident || (plan.resident_runs && term_mode && !pend[i].bwd);
    if (res_step && (gcr.size() != gc.size() || !gm.empty() || !wv.empty() || !wd.empty() ||
                     !rt.empty()))
      fail(TC_ERR_INVALID_ARG, "internal: resident step with non-gather nodes");
    L.begin = (uint32_t)plan.ops.size();
    uint64_t w = 0;
    L.gsbegin = (uint32_t)plan.gsplit_units.size();
    bool in_split = false;
    for (DevOp& op : gc) {
      const uint32_t ls = (op.flags >> 4) & 7u, lv = (op.flags >> 8) & 3u;
      const uint64_t groups = (uint64_t)op.rows * op.M * (op.N >> lv);
      if (op.ksplit > 1 && !in_split) {  // first split op
        in_split = true;
        L.xbegin = (uint32_t)plan.ops.size();
        L.work = (w + 63) & ~uint64_t(63);
        w = 0;
      }
      uint64_t items = (groups * op.ksplit) << ls;
      // whole wavefronts (aligned start, padded length): ops that split
      // their sums over lanes, and every op of a level launch, whose
      // wavefronts then each hold one op (found through a per-wavefront
      // table, 4 bytes per 64 items)
      if (ls || !term_mode) {
        w = (w + 63) & ~uint64_t(63);
        items = (items + 63) & ~uint64_t(63);
      }
      op.work0 = w;
      w += items;
      if (res_step) {
        if (op.ksplit != 1 || w >= (uint64_t(1) << 32))
          fail(TC_ERR_INVALID_ARG, "internal: resident node items");
        DevROp r = gcr[plan.ops.size() - L.begin];
        r.work0 = (uint32_t)op.work0;
        plan.rops.push_back(r);
      }
      if (op.ksplit > 1) {
        op.part = part;
        part += groups * op.ksplit * 2;
        const uint32_t rel = (uint32_t)(plan.ops.size() - L.xbegin);
        for (uint64_t ch = 0; ch < (groups + 255) / 256; ++ch)
          plan.gsplit_units.push_back({rel, (uint32_t)ch});
      }
      plan.ops.push_back(op);
    }
    L.gsend = (uint32_t)plan.gsplit_units.size();
    {
      // k-steps per item, averaged over the level's unsplit gather items:
      // long sums (8 or more) take the deep unroll (bandwidth bound: the
      // sweeps of wide chains, 2^22-element boundaries absorbing gates),
      // short ones the short unroll with more wavefronts (latency bound)
      double it = 0, ks = 0;
      for (uint32_t o = L.begin; o < plan.ops.size(); ++o) {
        const DevOp& op = plan.ops[o];
        if (op.ksplit != 1) continue;
        const uint32_t ls = (op.flags >> 4) & 7u, lv = (op.flags >> 8) & 3u;
        const double items = (double)(((uint64_t)op.rows * op.M * (op.N >> lv)) << ls);
        it += items;
        ks += items * (double)(op.K >> ls);
      }
      L.deep_gather = it > 0 && ks >= 8.0 * it;
    }
    plan.split_floats = std::max(plan.split_floats, part);
    L.end = (uint32_t)plan.ops.size();
    L.rbegin = L.end;
    for (DevOp& op : rt) {
      op.work0 = L.rblocks;
      L.rblocks += op.tiles_n;
      plan.ops.push_back(op);
    }
    L.rend = (uint32_t)plan.ops.size();
    // (resident runs: the level steps' ops get empty resident records, so
    // that the records stay indexed like the ops)
    if (plan.resident_runs) {
      if (res_step && plan.rops.size() != plan.ops.size())
        fail(TC_ERR_INVALID_ARG, "internal: resident records out of step with the ops");
      plan.rops.resize(plan.ops.size());
    }
    if (L.rblocks && L.rblocks <= WAVE_TABLE_MAX &&
        plan.item_op.size() + L.rblocks <= ITEM_TABLES_TOTAL_MAX) {
      // row-tile workgroup -> op (relative to L.rbegin): one load instead of
      // a search over the level's (often thousands of) row-tile ops
      L.rtunit_begin = plan.item_op.size();
      plan.item_op.resize(plan.item_op.size() + L.rblocks);
      uint32_t* it = plan.item_op.data() + L.rtunit_begin;
      for (uint32_t o = L.rbegin; o < L.rend; ++o)
        for (uint64_t x = plan.ops[o].work0; x < plan.ops[o].work0 + plan.ops[o].tiles_n; ++x)
          it[x] = o - L.rbegin;
    }
    if (!in_split) {
      L.xbegin = L.end;
      L.work = (w + 63) & ~uint64_t(63);
    } else {
      L.xwork = (w + 63) & ~uint64_t(63);
    }
    // item -> op (relative to L.begin) for a term step's group, wavefront
    // -> op for a level launch (its ops start on wavefronts); pad items map
    // to the op before them
    const uint64_t per = term_mode ? 1 : 64, n_entries = L.work / per;
    if (L.xbegin > L.begin && n_entries <= ITEM_TABLE_MAX &&
        plan.item_op.size() + n_entries <= ITEM_TABLES_TOTAL_MAX) {
      L.item_begin = plan.item_op.size();
      plan.item_op.resize(plan.item_op.size() + n_entries);
      uint32_t* it = plan.item_op.data() + L.item_begin;
      for (uint32_t o = L.begin; o < L.xbegin; ++o) {
        const uint64_t lo = plan.ops[o].work0;
        const uint64_t hi = o + 1 < L.xbegin ? plan.ops[o + 1].work0 : L.work;
        for (uint64_t x = lo / per; x < hi / per; ++x) it[x] = o - L.begin;
      }
    }
    if (term_mode) {
      // one group of the term: its ops at this step
      DevGroup G{};
      G.op_begin = L.begin;
      G.op_end = L.end;
      G.items = L.work;
      G.item_base = L.item_begin;
      plan.groups.push_back(G);
      group_term.push_back((uint32_t)pend[i].term);
      group_bwd.push_back(pend[i].bwd ? 1 : 0);
      seg_flops += lf;
      seg_bytes += lb;
      if (!pend[i].bwd) {
        seg_fflops += lf;
        seg_fbytes += lb;
      }
    } else {
      (pend[i].bwd ? plan.bwd : plan.fwd).push_back(L);
    }
    i = j;
  }
  close_segment();
  // leaves: inside the first term launch when it starts at the first level,
  // else a launch of their own
  if (plan.fwd.empty() || plan.fwd[0].kind != L_TERM || !plan.fwd[0].with_leaves) {
    Launch L;
    L.kind = L_LEAF;
    plan.fwd.insert(plan.fwd.begin(), L);  // leaf work filled below
  }

  // ---- leaves
  uint64_t lw = 0;
  std::vector<int32_t> qrow_slot;  // geometric tensor: the slot of each row
  for (size_t t = 0; t < net.terms.size(); ++t) {
    const Term& term = net.terms[t];
    plan.terms[t].leaf_begin = (uint32_t)plan.leaves.size();
    plan.terms[t].leaf_work0 = lw;
    for (size_t li = 0; li < term.leaves.size(); ++li) {
      const Leaf& lf = term.leaves[li];
      const PT& x = T[ti[t].tid[li]];
      DevLeaf d{};
      d.out = (uint64_t)x.off;
      d.where = 1;
      if ((plan.resident || plan.resident_runs) && x.lds_off >= 0) {
        d.lds_out = (uint32_t)x.lds_off;
        d.where = (x.global ? 1u : 0u) | 2u;
      }
      d.work0 = lw;
      d.kind = lf.kind;
      d.part = lf.part;
      d.conj = lf.conj;
      d.rank = lf.rank;
      d.rows = (x.batched && B > 1) ? (uint32_t)B : 1u;
      d.param[0] = d.param[1] = -1;
      d.dsel[0] = d.dsel[1] = -1;
      if (lf.kind == LEAF_GATE) {
        const GateRec& g = net.gates[lf.gate];
        d.gkind = g.kind;
        for (int a = 0; a < g.n_angles; ++a) {
          d.param[a] = g.param[a];
          d.fixed[a] = (float)g.fixed[a];
          if (plan.qgt && !lf.conj && leaf_param_dependent(net, lf) && g.param[a] >= 0 &&
              gate_angle_differentiable(g.kind, a)) {
            d.dsel[a] = (int32_t)qrow_slot.size();  // this use's row
            qrow_slot.push_back(g.param[a]);
          }
        }
        if (g.kind == TC_GATE_U1 || g.kind == TC_GATE_U2) {
          d.mat = (uint32_t)plan.ftab.size();
          for (int k = 0; k < 32; ++k) plan.ftab.push_back((float)g.mat[k]);
        } else if (g.kind == TC_GATE_DEPOL) {
          d.mat = (uint32_t)plan.ftab.size();  // px, py, pz
          for (int k = 0; k < 3; ++k) plan.ftab.push_back((float)g.mat[k]);
        }
      } else if (lf.kind == LEAF_MPO) {
        // a constant tensor: its (padded) entries in the float table
        const MpoSite& site = net.mpo.at((size_t)lf.gate);
        if (site.entries.size() != (size_t)2 << lf.rank)
          fail(TC_ERR_INVALID_ARG, "internal: MPO site size");
        d.mat = (uint32_t)plan.ftab.size();
        for (double x : site.entries) plan.ftab.push_back((float)x);
      } else {
        d.value = lf.gate;
      }
      lw += (uint64_t)d.rows << lf.rank;
      plan.leaves.push_back(d);
    }
    plan.terms[t].leaf_end = (uint32_t)plan.leaves.size();
    plan.terms[t].leaf_work_end = lw;
  }
  if (!plan.term_mode) plan.terms.clear();
  plan.leaf_work = lw;
  if (plan.qgt) {
    if ((int32_t)qrow_slot.size() != plan.qgt_rows) fail(TC_ERR_INVALID_ARG, "internal: qgt rows");
    plan.qslot_begin.assign(net.n_params + 1, 0);
    for (int32_t s : qrow_slot) plan.qslot_begin[s + 1]++;
    for (int p2 = 0; p2 < net.n_params; ++p2) plan.qslot_begin[p2 + 1] += plan.qslot_begin[p2];
    plan.qrows.assign(qrow_slot.size(), 0);
    std::vector<uint32_t> fill(plan.qslot_begin.begin(), plan.qslot_begin.end() - 1);
    for (size_t r = 0; r < qrow_slot.size(); ++r) plan.qrows[fill[qrow_slot[r]]++] = (uint32_t)r;
  }
  plan.fwd[0].work = lw;
  if (lw > 0 && lw <= ITEM_TABLE_MAX) {  // leaf entry -> leaf index
    plan.fwd[0].item_begin = plan.item_op.size();
    plan.item_op.reserve(plan.item_op.size() + lw);
    for (uint32_t i = 0; i < (uint32_t)plan.leaves.size(); ++i) {
      const DevLeaf& d = plan.leaves[i];
      plan.item_op.insert(plan.item_op.end(), (uint64_t)d.rows << d.rank, i);
    }
  }
  plan.fwd[0].bytes += 8.0 * (double)lw;  // every leaf entry written once
  for (Launch& L : plan.bwd)  // a resident plan's launch with the reverse sweep
    if (L.resident == 2) {
      L.work = plan.fwd[0].work;
      L.item_begin = plan.fwd[0].item_begin;
      L.bytes += 8.0 * (double)lw;
    }

  // ---- roots
  for (size_t t = 0; t < net.terms.size(); ++t) {
    DevRoot r{};
    r.weight = net.terms[t].weight;
    if (ti[t].root >= 0) {
      const PT& x = T[ti[t].tid[ti[t].root]];
      r.present = 1;
      r.val = (uint64_t)x.off;
      r.bs = (x.batched && B > 1) ? 1u : 0u;
    }
    plan.roots.push_back(r);
  }
  {
    Launch L;
    L.kind = L_ROOT;
    L.step = S.root_step;
    L.work = (uint64_t)B;
    plan.fwd.push_back(L);
  }

  // ---- gradient uses, sorted by slot then creation order
  if (grad) {
    std::vector<uint32_t> leaf_base(net.terms.size() + 1, 0);
    for (size_t t = 0; t < net.terms.size(); ++t)
      leaf_base[t + 1] = leaf_base[t] + (uint32_t)net.terms[t].leaves.size();
    std::vector<DevGradUse> uses;
    for (size_t u = 0; u < S.leaf_adj.size(); ++u) {
      size_t t = S.leaf_adj_term[u].first;
      int32_t li = S.leaf_adj_term[u].second;
      const Leaf& lf = net.terms[t].leaves[li];
      const GateRec& g = net.gates[lf.gate];
      const PT& d = T[S.leaf_adj[u].second];
      for (int a = 0; a < g.n_angles; ++a) {
        if (g.param[a] < 0 || !gate_angle_differentiable(g.kind, a)) continue;
        DevGradUse gu{};
        gu.adj = (uint64_t)d.off;
        gu.adj_bs = (d.batched && B > 1) ? (uint32_t)d.elems : 0u;
        gu.leaf = leaf_base[t] + (uint32_t)li;
        gu.which = a;
        gu.slot = g.param[a];
        uses.push_back(gu);
      }
    }
    std::stable_sort(uses.begin(), uses.end(),
                     [](const DevGradUse& x, const DevGradUse& y) { return x.slot < y.slot; });
    plan.uses = uses;
    plan.slot_begin.assign(net.n_params + 1, 0);
    for (const auto& gu : uses) plan.slot_begin[gu.slot + 1]++;
    for (int p = 0; p < net.n_params; ++p) plan.slot_begin[p + 1] += plan.slot_begin[p];
    if (net.n_params > 0) {
      Launch L;
      L.kind = L_GRAD;
      L.step = S.grad_step;
      L.work = (uint64_t)B * net.n_params;
      plan.bwd.push_back(L);
    }
    if (plan.qgt && net.n_params > 0) {
      Launch L;
      L.kind = L_QGT;
      L.step = S.grad_step + 1;
      L.work = (uint64_t)net.n_params * net.n_params;
      plan.bwd.push_back(L);
    }
  }

  // ---- every device access in bounds (checked here, before any launch)
  {
    const uint64_t AE = plan.arena_elems;
    const uint64_t NT = plan.tabs.size();
    auto tmax = [&](uint32_t d, uint32_t n) {
      if ((d & IX_TABLE) && (uint64_t)(d & ~IX_TABLE) + n > NT)
        fail(TC_ERR_INVALID_ARG, "internal: table out of range");
      return tables.max_of(d, n);  // a group of n = 2^b indices
    };
    for (const DevOp& op : plan.ops) {
      uint64_t r1 = op.rows - 1;
      uint64_t a_end = op.a + r1 * op.a_bs + tmax(op.a_m, op.M) + tmax(op.a_k, op.K);
      uint64_t b_end = op.b + r1 * op.b_bs + tmax(op.b_k, op.K) + tmax(op.b_n, op.N);
      uint64_t c_end = op.c + r1 * op.c_bs + tmax(op.c_m, op.M) + tmax(op.c_n, op.N);
      if (a_end >= AE || b_end >= AE || c_end >= AE)
        fail(TC_ERR_INVALID_ARG, "internal: contraction op out of the arena");
      if (op.c < seed_elems) fail(TC_ERR_INVALID_ARG, "internal: op writes over the seeds");
    }
    for (const DevLeaf& d : plan.leaves) {
      if (d.out + ((uint64_t)d.rows << d.rank) > AE || d.out < seed_elems ||
          (d.param[0] >= plan.n_params) || (d.param[1] >= plan.n_params) ||
          d.rank > MAX_LEAF_RANK)
        fail(TC_ERR_INVALID_ARG, "internal: leaf out of range");
      const uint64_t nf = d.kind == DLEAF_MPO ? (uint64_t)2 << d.rank
                          : (d.kind == DLEAF_GATE && (d.gkind == TC_GATE_U1 || d.gkind == TC_GATE_U2)) ? 32
                          : (d.kind == DLEAF_GATE && d.gkind == TC_GATE_DEPOL) ? 3 : 0;
      if (nf && (uint64_t)d.mat + nf > plan.ftab.size())
        fail(TC_ERR_INVALID_ARG, "internal: leaf table out of range");
    }
    for (const DevGradUse& u : plan.uses)
      if (u.leaf >= plan.leaves.size() ||
          u.adj + (uint64_t)(B - 1) * u.adj_bs + (1ull << plan.leaves[u.leaf].rank) > AE)
        fail(TC_ERR_INVALID_ARG, "internal: gradient use out of range");
    for (uint32_t r : plan.qrows)
      if (r >= (uint32_t)B) fail(TC_ERR_INVALID_ARG, "internal: qgt row out of range");
    for (const DevLeaf& d : plan.leaves)
      for (int a = 0; a < 2; ++a)
        if (d.dsel[a] >= B || (d.dsel[a] >= 0 && d.rows != (uint32_t)B))
          fail(TC_ERR_INVALID_ARG, "internal: derivative row out of range");
    for (const DevRoot& r : plan.roots)
      if (r.present && r.val + (uint64_t)(B - 1) * r.bs >= AE)
        fail(TC_ERR_INVALID_ARG, "internal: root out of range");
    // GEMM ops: tile grids that cover M x N, split-K partial tiles and
    // counters inside their regions
    for (const auto* seq : {&plan.fwd, &plan.bwd})
      for (const Launch& L : *seq) {
        if (L.kind != L_LEVEL) continue;
        for (uint32_t o = L.gbegin; o < L.wend; ++o) {
          const DevOp& op = plan.ops[o];
          const bool wave = o >= L.wbegin;
          const uint64_t bi = (op.flags >> 12) & 1u ? 2 : 1, bj = (op.flags >> 13) & 1u ? 2 : 1;
          const uint64_t fpt = wave ? 8 * bi * bj * 64 : 32 * 256;
          const bool cover = wave ? ((uint64_t)op.tiles_m * 16 * bi == op.M ||
                                     (op.M < 16 && op.tiles_m == 1 && bi == 1)) &&
                                        ((uint64_t)op.tiles_n * 16 * bj == op.N ||
                                         (op.N < 16 && op.tiles_n == 1 && bj == 1)) &&
                                        op.K >= 4
                                  : (uint64_t)op.tiles_m * 64 >= op.M && (uint64_t)op.tiles_n * 64 >= op.N;
          if (!cover || op.ksplit < 1 || op.K % op.ksplit != 0)
            fail(TC_ERR_INVALID_ARG, "internal: GEMM tile grid does not match the node");
          if (op.ksplit == 1) continue;
          const uint64_t base = (uint64_t)op.rows * op.tiles_m * op.tiles_n;
          if (op.part + base * op.ksplit * fpt > plan.split_floats ||
              (wave && (op.K / op.ksplit) % 4 != 0))
            fail(TC_ERR_INVALID_ARG, "internal: split-K tiles out of range");
        }
        // wide tiles: dense operands, whole 128 x 128 tiles, no split
        if (L.hbegin != L.wend || L.hend < L.hbegin || L.begin != L.hend)
          fail(TC_ERR_INVALID_ARG, "internal: wide op range");
        // row tiles: whole rows of both operands within the LDS budget
        if (L.rbegin != L.end || L.rend < L.rbegin)
          fail(TC_ERR_INVALID_ARG, "internal: row-tile op range");
        for (uint32_t o = L.rbegin; o < L.rend; ++o) {
          const DevOp& op = plan.ops[o];
          const uint64_t rpb = op.tiles_m;
          if (rpb < 1 || rpb > ROW_TILE_ROWS || (rpb & (rpb - 1)) || op.rows < 1 ||
              rpb * ((uint64_t)op.M * op.K + (uint64_t)op.K * op.N) > ROW_TILE_LDS ||
              op.K > ROW_TILE_LDS / 2 ||
              op.tiles_n != (op.rows + rpb - 1) / rpb || op.ksplit != 1 ||
              op.work0 != (o == L.rbegin ? 0 : plan.ops[o - 1].work0 + plan.ops[o - 1].tiles_n))
            fail(TC_ERR_INVALID_ARG, "internal: row-tile op");
        }
        for (uint32_t o = L.hbegin; o < L.hend; ++o) {
          const DevOp& op = plan.ops[o];
          const uint32_t lm = __builtin_ctz(op.M), ln = __builtin_ctz(op.N), lk = __builtin_ctz(op.K);
          const uint64_t chunks =
              ((op.a_bs ? op.rows : 1) * (uint64_t)op.M + (op.b_bs ? op.rows : 1) * (uint64_t)op.N) *
              (op.K / 8);
          if (op.part % 64 || op.part + chunks * 16 > plan.split_floats)
            fail(TC_ERR_INVALID_ARG, "internal: wide op BF16 planes out of range");
          if (!(op.flags & OPF_WIDE) || op.ksplit != 1 || op.M % 128 || op.N % 128 || op.K % 32 ||
              op.tiles_m * 128 != op.M || op.tiles_n * 128 != op.N || op.a_k != lk ||
              op.a_m != (lm | (lk << 5)) || op.b_n != ln || op.b_k != (lk | (ln << 5)) ||
              op.a % 2 || op.b % 2 || op.a_bs % 2 || op.b_bs % 2 ||
              (o > L.hbegin && op.work0 != plan.ops[o - 1].work0 + (uint64_t)plan.ops[o - 1].rows *
                                                              plan.ops[o - 1].tiles_m * plan.ops[o - 1].tiles_n))
            fail(TC_ERR_INVALID_ARG, "internal: wide GEMM op");
        }
        if (L.sbegin > L.send || L.send > plan.split_units.size() || L.gsbegin > L.gsend ||
            L.gsend > plan.gsplit_units.size())
          fail(TC_ERR_INVALID_ARG, "internal: split-K units out of range");
        // gather ops: unsplit in [begin, xbegin) over `work` items, split
        // (V == 1, K a multiple of the slices) in [xbegin, end) over `xwork`
        if (L.xbegin < L.begin || L.xbegin > L.end)
          fail(TC_ERR_INVALID_ARG, "internal: split gather range");
        for (uint32_t o = L.begin; o < L.end; ++o) {
          const DevOp& op = plan.ops[o];
          const bool sp = o >= L.xbegin;
          const uint32_t ls = (op.flags >> 4) & 7u, lv = (op.flags >> 8) & 3u;
          const uint64_t groups = (uint64_t)op.rows * op.M * (op.N >> lv);
          const uint64_t items = (groups * op.ksplit) << ls;
          if ((sp ? op.ksplit < 2 || lv != 0 : op.ksplit != 1) || op.work0 + items > (sp ? L.xwork : L.work) ||
              (o > L.begin && o != L.xbegin && op.work0 < plan.ops[o - 1].work0))
            fail(TC_ERR_INVALID_ARG, "internal: gather items do not cover the ops");
          if (sp && (op.K % op.ksplit != 0 || op.part + groups * op.ksplit * 2 > plan.split_floats))
            fail(TC_ERR_INVALID_ARG, "internal: gather split out of range");
        }
        for (uint32_t u = L.gsbegin; u < L.gsend; ++u) {
          const DevSplitUnit su = plan.gsplit_units[u];
          if (su.op >= L.end - L.xbegin) fail(TC_ERR_INVALID_ARG, "internal: gather split unit op");
          const DevOp& op = plan.ops[L.xbegin + su.op];
          const uint64_t groups = (uint64_t)op.rows * op.M * (op.N >> ((op.flags >> 8) & 3u));
          if (op.ksplit < 2 || (uint64_t)su.tile * 256 >= groups)
            fail(TC_ERR_INVALID_ARG, "internal: gather split unit chunk");
        }
        for (uint32_t u = L.sbegin; u < L.send; ++u) {
          const DevSplitUnit su = plan.split_units[u];
          if (su.op >= L.wend - L.gbegin) fail(TC_ERR_INVALID_ARG, "internal: split unit op");
          const DevOp& op = plan.ops[L.gbegin + su.op];
          if (op.ksplit < 2 || su.tile >= (uint64_t)op.rows * op.tiles_m * op.tiles_n)
            fail(TC_ERR_INVALID_ARG, "internal: split unit tile");
        }
      }
    // term mode: groups name contiguous op ranges whose items cover the ops,
    // terms name group and leaf ranges
    for (const DevGroup& G : plan.groups) {
      if (G.op_begin >= G.op_end || G.op_end > plan.ops.size() || (G.items & 63) != 0)
        fail(TC_ERR_INVALID_ARG, "internal: bad group");
      for (uint32_t o = G.op_begin; o < G.op_end; ++o) {
        const DevOp& op = plan.ops[o];
        const uint32_t ls = (op.flags >> 4) & 7u, lv = (op.flags >> 8) & 3u;
        const uint64_t items = ((uint64_t)op.rows * op.M * (op.N >> lv)) << ls;
        if (op.work0 + items > G.items || (o > G.op_begin && op.work0 < plan.ops[o - 1].work0))
          fail(TC_ERR_INVALID_ARG, "internal: group items do not cover its ops");
      }
      if (G.item_base != NO_ITEMS) {
        if (G.item_base + G.items > plan.item_op.size())
          fail(TC_ERR_INVALID_ARG, "internal: item table out of range");
        for (uint64_t x = 0; x < G.items; ++x)
          if (plan.item_op[G.item_base + x] >= G.op_end - G.op_begin)
            fail(TC_ERR_INVALID_ARG, "internal: item table names a missing op");
      }
    }
    // resident plans: one record per gather op with the same shape, every
    // operand inside the LDS arena or the global arena it names
    if (plan.resident || plan.resident_runs) {
      const uint64_t LE = plan.lds_elems;
      if (plan.rops.size() != plan.ops.size() || !LE)
        fail(TC_ERR_INVALID_ARG, "internal: resident op records");
      // the ops that resident term launches run
      std::vector<char> used(plan.ops.size(), 0);
      for (const auto* seq : {&plan.fwd, &plan.bwd})
        for (const Launch& L : *seq) {
          if (L.kind != L_TERM || !L.resident) continue;
          for (size_t t = 0; t < plan.terms.size(); ++t) {
            const DevRange& R = plan.ranges.at(L.begin + t);
            for (uint32_t g = R.g_begin; g < R.g_end; ++g)
              for (uint32_t o = plan.groups.at(g).op_begin; o < plan.groups.at(g).op_end; ++o) used.at(o) = 1;
          }
        }
      for (size_t o = 0; o < plan.rops.size(); ++o) {
        if (!used[o]) continue;
        const DevROp& r = plan.rops[o];
        const DevOp& op = plan.ops[o];
        const uint32_t sh = r.shape;
        if ((1u << (sh & 31)) != op.M || (1u << ((sh >> 5) & 31)) != op.N ||
            (1u << ((sh >> 10) & 31)) != op.K || ((sh >> 15) & 7) != ((op.flags >> 4) & 7u) ||
            ((sh >> 18) & 3) != ((op.flags >> 8) & 3u) || r.work0 != op.work0 || op.rows != 1 ||
            op.ksplit != 1 || r.a_m != op.a_m || r.a_k != op.a_k || r.b_k != op.b_k ||
            r.b_n != op.b_n || r.c_m != op.c_m || r.c_n != op.c_n)
          fail(TC_ERR_INVALID_ARG, "internal: resident record does not match its op");
        const uint64_t a_end = (uint64_t)r.a + tmax(r.a_m, op.M) + tmax(r.a_k, op.K);
        const uint64_t b_end = (uint64_t)r.b + tmax(r.b_k, op.K) + tmax(r.b_n, op.N);
        const uint64_t c_ext = tmax(r.c_m, op.M) + tmax(r.c_n, op.N);
        if (a_end >= ((sh & RES_A_LDS) ? LE : AE) || b_end >= ((sh & RES_B_LDS) ? LE : AE) ||
            (uint64_t)r.c + c_ext >= ((sh & RES_C_LDS) ? LE : AE) ||
            ((sh & RES_C2) && (!(sh & RES_C_LDS) || (uint64_t)r.c2 + c_ext >= AE)) ||
            (!(sh & RES_C_LDS) && r.c < seed_elems) || ((sh & RES_C2) && r.c2 < seed_elems))
          fail(TC_ERR_INVALID_ARG, "internal: resident op out of its arena");
      }
      for (const DevLeaf& d : plan.leaves)
        if (!(d.where & 3u) || d.where > 3u ||
            ((d.where & 2u) && (uint64_t)d.lds_out + (1ull << d.rank) > LE) || d.rows != 1)
          fail(TC_ERR_INVALID_ARG, "internal: resident leaf out of the LDS arena");
      // leaves held in LDS are written by the resident launch that runs first
      bool lds_leaves = false;
      for (const DevLeaf& d : plan.leaves) lds_leaves = lds_leaves || d.where != 1u;
      if (lds_leaves && (plan.fwd.empty() || plan.fwd[0].kind != L_TERM || !plan.fwd[0].with_leaves ||
                         !plan.fwd[0].resident))
        fail(TC_ERR_INVALID_ARG, "internal: leaves in LDS without a resident launch writing them");
    } else if (!plan.rops.empty()) {
      fail(TC_ERR_INVALID_ARG, "internal: resident records in a plan without resident launches");
    }
    for (const auto* seq : {&plan.fwd, &plan.bwd})
      for (const Launch& L : *seq)
        if (L.resident && (L.kind != L_TERM || !(plan.resident || plan.resident_runs)))
          fail(TC_ERR_INVALID_ARG, "internal: resident launch in a plan without resident records");
    for (const DevTerm& D : plan.terms)
      if (D.leaf_begin > D.leaf_end || D.leaf_end > plan.leaves.size() ||
          D.leaf_work_end > plan.leaf_work || D.leaf_work0 > D.leaf_work_end)
        fail(TC_ERR_INVALID_ARG, "internal: bad term leaf range");
    for (const DevRange& R : plan.ranges)
      if (R.g_begin > R.g_end || R.g_end > plan.groups.size())
        fail(TC_ERR_INVALID_ARG, "internal: bad term group range");
    for (const auto* seq : {&plan.fwd, &plan.bwd})
      for (const Launch& L : *seq)
        if (L.kind == L_TERM &&
            ((uint64_t)L.begin + plan.terms.size() > plan.ranges.size() || plan.terms.empty()))
          fail(TC_ERR_INVALID_ARG, "internal: term launch without ranges");
    // per-wave-tile tables, and tile grids and slices in powers of two (the
    // kernels decode tiles with shifts)
    for (const auto* seq : {&plan.fwd, &plan.bwd})
      for (const Launch& L : *seq) {
        if (L.kind != L_LEVEL) continue;
        for (uint32_t o = L.gbegin; o < L.hend; ++o) {
          const DevOp& op = plan.ops[o];
          auto pow2 = [](uint64_t v) { return v && !(v & (v - 1)); };
          if (!pow2(op.tiles_m) || !pow2(op.tiles_n) || !pow2(op.ksplit))
            fail(TC_ERR_INVALID_ARG, "internal: tile grid not in powers of two");
        }
        if (L.rtunit_begin != NO_ITEMS) {
          if (L.rtunit_begin + L.rblocks > plan.item_op.size())
            fail(TC_ERR_INVALID_ARG, "internal: row-tile table out of range");
          for (uint64_t x = 0; x < L.rblocks; ++x) {
            const uint32_t o = plan.item_op[L.rtunit_begin + x];
            if (o >= L.rend - L.rbegin) fail(TC_ERR_INVALID_ARG, "internal: row-tile table names a missing op");
            const DevOp& op = plan.ops[L.rbegin + o];
            if (x < op.work0 || x >= op.work0 + op.tiles_n)
              fail(TC_ERR_INVALID_ARG, "internal: row-tile table entry outside its op");
          }
        }
        if (L.wunit_begin == NO_ITEMS) continue;
        if (L.wunit_begin + L.wtiles > plan.item_op.size())
          fail(TC_ERR_INVALID_ARG, "internal: wave tile table out of range");
        for (uint64_t x = 0; x < L.wtiles; ++x) {
          const uint32_t o = plan.item_op[L.wunit_begin + x];
          if (o >= L.wend - L.wbegin) fail(TC_ERR_INVALID_ARG, "internal: wave tile table names a missing op");
          const DevOp& op = plan.ops[L.wbegin + o];
          if (x < op.work0 || x >= op.work0 + (uint64_t)op.rows * op.tiles_m * op.tiles_n * op.ksplit)
            fail(TC_ERR_INVALID_ARG, "internal: wave tile table entry outside its op");
        }
      }
    // per-item tables: one entry per work item, naming an item of the launch
    for (const auto* seq : {&plan.fwd, &plan.bwd})
      for (const Launch& L : *seq) {
        if (L.item_begin == NO_ITEMS) continue;
        const uint64_t n_items =
            (L.kind == L_LEAF || L.kind == L_TERM) ? plan.leaves.size() : L.xbegin - L.begin;
        // a level launch's table has one entry per wavefront of 64 items,
        // each naming the op whose (padded) items hold that wavefront
        const uint64_t per = L.kind == L_LEVEL ? 64 : 1;
        if (L.kind == L_LEVEL && L.work % 64)
          fail(TC_ERR_INVALID_ARG, "internal: level items not whole wavefronts");
        if (L.item_begin + L.work / per > plan.item_op.size())
          fail(TC_ERR_INVALID_ARG, "internal: item table out of range");
        for (uint64_t x = 0; x < L.work / per; ++x) {
          const uint32_t o = plan.item_op[L.item_begin + x];
          if (o >= n_items) fail(TC_ERR_INVALID_ARG, "internal: item table names a missing op");
          if (L.kind == L_LEVEL) {
            const uint64_t lo = plan.ops[L.begin + o].work0;
            const uint64_t hi = L.begin + o + 1 < L.xbegin ? plan.ops[L.begin + o + 1].work0 : L.work;
            if (lo % 64 || x * 64 < lo || x * 64 + 64 > hi)
              fail(TC_ERR_INVALID_ARG, "internal: wavefront table entry outside its op");
          }
        }
      }
  }

  // ---- info
  tc_plan_info& info = plan.info;
  info = tc_plan_info{};
  info.n_gemm_nodes = n_gemm_nodes;
  info.flops = flops;
  info.alg_bytes = bytes;
  info.grad_flops = gflops;
  info.grad_alg_bytes = gbytes;
  info.workspace_bytes = workspace_layout(plan).total;
  info.peak_tensor_bytes = plan.peak_tensor_elems * 8;
  int32_t nn = 0;
  for (const auto& p : pend)
    if (!p.bwd) ++nn;
  info.n_nodes = nn;
  info.n_levels = S.max_level;
  info.n_launches = (int32_t)plan.fwd.size();
  info.n_grad_launches = (int32_t)plan.bwd.size();
  info.batch = plan.qgt ? 1 : B;   // the caller's parameter vectors
  info.n_params = net.n_params;
  info.n_qgt_rows = plan.qgt_rows;
  info.n_terms = plan.n_terms;
  info.checkpoint_every = plan.checkpoint_used;
  info.n_term_groups = plan.term_groups;
  info.exec_mode = plan.exec_used;
  for (const auto* seq : {&plan.fwd, &plan.bwd})
    for (const Launch& L : *seq)
      if (L.kind == L_LEVEL) {
        for (uint32_t o = L.gbegin; o < L.wend; ++o) info.n_split_nodes += plan.ops[o].ksplit > 1;
        info.n_split_sums += (int32_t)(L.end - L.xbegin);
        info.n_wide_nodes += (int32_t)(L.hend - L.hbegin);
      }
  if (plan.budget && info.workspace_bytes > plan.budget) {
    const WorkspaceLayout w = workspace_layout(plan);
    fail(TC_ERR_TOO_LARGE, "workspace of " + std::to_string(info.workspace_bytes) +
                               " bytes (intermediates " + std::to_string(w.total - w.arena) +
                               ", split partial sums and operand planes " +
                               std::to_string(w.sunits - w.split) + ", tables and the rest " +
                               std::to_string(w.arena - (w.sunits - w.split)) +
                               ") exceeds the memory budget");
  }
}

}  // namespace tcx
