// Host-side check driver for sanitizer builds (no GPU): runs the network
// builder, the path finder (trials, reconfiguration, spatial candidates),
// slicing and the planner (budgets, term groups, checkpointing, batches,
// MPO and state observables, geometric tensor plans, channel gates) over a
// spread of circuits, plus the error paths, so that AddressSanitizer and
// UndefinedBehaviorSanitizer see every host code path the library takes
// before a kernel is launched.  Prints "host check ok" and exits 0 when
// every call behaves as documented.
//
//   g++ -std=c++17 -g -O1 -fsanitize=address,undefined -fno-omit-frame-pointer \
//       -I include paper_2205_10091_amd/csrc/{network,path,plan,slice,capi_host,host_check}.cpp
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "plan.h"

struct tc_network;
struct tc_path;
namespace tcx {
const Network& network_of(const tc_network* n);
const Path& path_of(const tc_path* p);
}  // namespace tcx

namespace {

int failures = 0;
int resident_checked = 0;
int runs_checked = 0;

void expect(bool ok, const std::string& what) {
  if (!ok) {
    std::fprintf(stderr, "FAILED: %s (%s)\n", what.c_str(), tc_last_error());
    ++failures;
  }
}

struct Circ {
  int n = 0, n_params = 0;
  std::vector<tc_gate> gates;
  std::vector<std::vector<double>> mats;  // caller matrices / probabilities
  std::vector<int> mat_of;                // per gate: index into mats, or -1
  void add(int kind, int q0, int q1 = -1, int p0 = -1, int p1 = -1,
           const std::vector<double>& m = {}) {
    tc_gate g{};
    g.kind = kind;
    g.q[0] = q0;
    g.q[1] = q1 < 0 ? 0 : q1;
    g.param[0] = p0;
    g.param[1] = p1;
    g.fixed[0] = 0.3;
    g.fixed[1] = 0.7;
    gates.push_back(g);
    mat_of.push_back(m.empty() ? -1 : (int)mats.size());
    if (!m.empty()) mats.push_back(m);
  }
  tc_circuit c() {
    for (size_t i = 0; i < gates.size(); ++i)
      gates[i].matrix = mat_of[i] < 0 ? nullptr : mats[mat_of[i]].data();
    return tc_circuit{n, n_params, (int32_t)gates.size(), gates.data()};
  }
};

Circ ladder(int n, int layers) {
  Circ c;
  c.n = n;
  c.n_params = layers * 2 * n;
  for (int l = 0; l < layers; ++l) {
    for (int i = 0; i + 1 < n; ++i) c.add(TC_GATE_RZZ, i, i + 1, (l * 2) * n + i);
    for (int i = 0; i < n; ++i) c.add(TC_GATE_RX, i, -1, (l * 2 + 1) * n + i);
  }
  return c;
}

Circ grid(int r, int cols, int layers) {
  Circ c;
  c.n = r * cols;
  int s = 0;
  for (int l = 0; l < layers; ++l) {
    for (int a = 0; a < r; ++a)
      for (int b = 0; b + 1 < cols; ++b) c.add(TC_GATE_RZZ, a * cols + b, a * cols + b + 1, s++);
    for (int a = 0; a + 1 < r; ++a)
      for (int b = 0; b < cols; ++b) c.add(TC_GATE_RZZ, a * cols + b, (a + 1) * cols + b, s++);
    for (int q = 0; q < c.n; ++q) c.add(TC_GATE_FSIM, q, (q + 1) % c.n, s, s + 1), s += 2;
  }
  c.n_params = s;
  return c;
}

Circ all_kinds(int n, int seed) {
  Circ c;
  c.n = n;
  std::srand(seed);
  int s = 0;
  for (int k = 0; k < 60; ++k) {
    int kind = std::rand() % 21;
    int q0 = std::rand() % n, q1 = (q0 + 1 + std::rand() % (n - 1)) % n;
    switch (kind) {
      case TC_GATE_U1: c.add(kind, q0, -1, -1, -1, std::vector<double>(8, 0.25)); break;
      case TC_GATE_U2: c.add(kind, q0, q1, -1, -1, std::vector<double>(32, 0.1)); break;
      case TC_GATE_DEPOL: c.add(kind, q0, -1, s++, -1, {0.1, 0.2, 0.3}); break;
      case TC_GATE_RSWITCH: c.add(kind, q0, -1, s, s + 1), s += 2; break;
      case TC_GATE_FSIM: c.add(kind, q0, q1, s, s + 1), s += 2; break;
      case TC_GATE_RX: case TC_GATE_RY: case TC_GATE_RZ: c.add(kind, q0, -1, s++); break;
      case TC_GATE_RZZ: case TC_GATE_RXX: case TC_GATE_RYY: c.add(kind, q0, q1, s++); break;
      case TC_GATE_CNOT: case TC_GATE_CZ: c.add(kind, q0, q1); break;
      default: c.add(kind, q0); break;
    }
  }
  c.n_params = s;
  return c;
}

struct Obs {
  std::vector<uint8_t> st;
  std::vector<double> w;
  std::vector<int32_t> bonds;
  std::vector<double> mpo;
  tc_observable o{};
};

Obs tfim(int n) {
  Obs x;
  for (int i = 0; i + 1 < n; ++i) {
    std::vector<uint8_t> s(n, 0);
    s[i] = s[i + 1] = 3;
    x.st.insert(x.st.end(), s.begin(), s.end());
    x.w.push_back(1.0);
  }
  for (int i = 0; i < n; ++i) {
    std::vector<uint8_t> s(n, 0);
    s[i] = 1;
    x.st.insert(x.st.end(), s.begin(), s.end());
    x.w.push_back(0.8);
  }
  x.o = tc_observable{TC_OBS_PAULI_SUM, nullptr, (int32_t)x.w.size(), x.st.data(), x.w.data(),
                      nullptr, nullptr};
  return x;
}

Obs mpo_random(int n) {
  Obs x;
  std::vector<int32_t> d(n + 1, 1);
  for (int k = 1; k < n; ++k) d[k] = 1 + (k * 3) % 8;
  for (int k = 1; k < n; ++k) x.bonds.push_back(d[k]);
  for (int k = 0; k < n; ++k)
    for (int e = 0; e < d[k] * d[k + 1] * 4; ++e) {
      x.mpo.push_back(std::sin(0.3 * e + k));
      x.mpo.push_back(std::cos(0.7 * e - k));
    }
  x.o = tc_observable{TC_OBS_MPO, nullptr, 0, nullptr, nullptr, x.bonds.data(), x.mpo.data()};
  return x;
}

// Resident term launches, executed on the host: every launch of the
// sequence in order, the nodes of resident term launches with operands
// taken from a per-workgroup LDS arena or the global arena as their
// resident records say (`res`), everything else from the global arena
// through the plain op records (the reference).  The arithmetic is the
// contraction's sums of products over the integers modulo the prime
// 2^61 - 1 (exact, no overflow on networks of any length), with leaves and
// seeds hashed from their indices; memory starts as a poison value that
// every product with it keeps, so a read of anything not yet written shows
// in the results.  The nodes of a step run first to last or last to first
// (`rev`), so a node that overwrote another's operand within one step
// would change them.  Returns the term roots and the leaf adjoints the
// gradient reads.
using val = uint64_t;
constexpr val MOD = (uint64_t(1) << 61) - 1, POISON = ~uint64_t(0);

val vmul(val a, val b) {
  if (a == POISON || b == POISON) return POISON;
  const unsigned __int128 x = (unsigned __int128)a * b;
  val r = (val)(x & MOD) + (val)(x >> 61);
  return r >= MOD ? r - MOD : r;
}
val vadd(val a, val b) {
  if (a == POISON || b == POISON) return POISON;
  const val r = a + b;
  return r >= MOD ? r - MOD : r;
}
val vhash(uint64_t a, uint64_t b) {
  uint64_t x = a * 0x9E3779B97F4A7C15ull ^ (b + 0x7F4A7C159E3779B9ull);
  x ^= x >> 31;
  x *= 0xBF58476D1CE4E5B9ull;
  x ^= x >> 29;
  return x % MOD;
}

uint64_t ix_of(const std::vector<uint32_t>& tabs, uint32_t d, uint64_t i) {
  if (d & 0x80000000u) return tabs.at((d & 0x7fffffffu) + i);
  uint64_t off = 0;
  uint32_t src = 0;
  for (int r = 0; r < 3; ++r) {
    const uint32_t f = (d >> (10 * r)) & 0x3ffu, len = f & 31u, dst = f >> 5;
    off |= ((i >> src) & ((uint64_t(1) << len) - 1)) << dst;
    src += len;
  }
  return off;
}

std::vector<val> run_resident(const tcx::Plan& p, bool res, bool grad, bool rev) {
  std::vector<val> G(p.arena_elems, POISON), L;
  for (size_t t = 0; t < p.seeds.size() / 2; ++t) G.at(t) = vhash(1000003 + t, 7);
  auto leaf = [&](uint32_t li, bool use_where) {
    const tcx::DevLeaf& d = p.leaves[li];
    for (uint64_t e = 0; e < (uint64_t(1) << d.rank); ++e) {
      const val v = vhash(li, e);
      if (!use_where || (d.where & 1u)) G.at(d.out + e) = v;
      if (use_where && (d.where & 2u)) L.at(d.lds_out + e) = v;
    }
  };
  auto node = [&](uint32_t o, bool resident) {
    const tcx::DevOp& op = p.ops.at(o);
    uint64_t a = op.a, b = op.b, c = op.c, c2 = 0;
    bool al = false, bl = false, cl = false, two = false;
    if (resident) {
      const tcx::DevROp& r = p.rops.at(o);
      a = r.a, b = r.b, c = r.c, c2 = r.c2;
      al = r.shape & tcx::RES_A_LDS, bl = r.shape & tcx::RES_B_LDS;
      cl = r.shape & tcx::RES_C_LDS, two = r.shape & tcx::RES_C2;
    }
    std::vector<val>& MA = al ? L : G;
    std::vector<val>& MB = bl ? L : G;
    std::vector<val>& MC = cl ? L : G;
    auto offs = [&](uint32_t d, uint64_t n) {
      std::vector<uint64_t> v(n);
      for (uint64_t i = 0; i < n; ++i) v[i] = ix_of(p.tabs, d, i);
      return v;
    };
    const std::vector<uint64_t> am = offs(op.a_m, op.M), ak = offs(op.a_k, op.K),
                                bk = offs(op.b_k, op.K), bn = offs(op.b_n, op.N),
                                cm = offs(op.c_m, op.M), cn = offs(op.c_n, op.N);
    for (uint64_t m = 0; m < op.M; ++m)
      for (uint64_t n = 0; n < op.N; ++n) {
        val acc = 0;
        for (uint64_t k = 0; k < op.K; ++k)
          acc = vadd(acc, vmul(MA.at(a + am[m] + ak[k]), MB.at(b + bk[k] + bn[n])));
        MC.at(c + cm[m] + cn[n]) = acc;
        if (two) G.at(c2 + cm[m] + cn[n]) = acc;
      }
  };
  for (const tcx::Launch* x : tcx::launch_order(p, grad)) {
    if (x->kind == tcx::L_LEAF) {
      for (uint32_t li = 0; li < p.leaves.size(); ++li) leaf(li, false);
    } else if (x->kind == tcx::L_LEVEL) {
      const uint32_t n = x->rend - x->gbegin;
      for (uint32_t q = 0; q < n; ++q) node(rev ? x->rend - 1 - q : x->gbegin + q, false);
    } else if (x->kind == tcx::L_TERM) {
      const bool resident = res && x->resident;
      for (size_t t = 0; t < p.terms.size(); ++t) {
        L.assign(p.lds_elems, POISON);  // each launch's workgroup starts afresh
        if (x->with_leaves)
          for (uint32_t li = p.terms[t].leaf_begin; li < p.terms[t].leaf_end; ++li) leaf(li, resident);
        const tcx::DevRange R = p.ranges.at(x->begin + t);
        for (uint32_t g = R.g_begin; g < R.g_end; ++g) {
          const tcx::DevGroup& grp = p.groups.at(g);
          for (uint32_t q = 0; q < grp.op_end - grp.op_begin; ++q)
            node(rev ? grp.op_end - 1 - q : grp.op_begin + q, resident);
        }
      }
    }
  }
  std::vector<val> out;
  for (const tcx::DevRoot& r : p.roots)
    if (r.present) out.push_back(G.at(r.val));
  if (grad)
    for (const tcx::DevGradUse& u : p.uses)
      for (uint64_t e = 0; e < (uint64_t(1) << p.leaves.at(u.leaf).rank); ++e)
        out.push_back(G.at(u.adj + e));
  return out;
}

bool same(const std::vector<val>& x, const std::vector<val>& y) {
  if (x.size() != y.size() || x.empty()) return false;
  for (size_t i = 0; i < x.size(); ++i)
    if (x[i] != y[i] || x[i] == POISON) return false;
  return true;
}

void run_plans(const tc_network* net, const tc_path* path, bool grad, const char* what) {
  tc_path_stats st{};
  expect(tc_path_stats_get(path, -1, &st) == TC_OK, std::string(what) + ": stats");
  for (int batch : {1, 8})
    for (uint64_t budget : {uint64_t(0), uint64_t(1) << 22})
      for (int exec : {0, 1}) {
        tcx::Plan p;
        p.batch = batch;
        p.want_grad = grad ? 1 : 0;
        p.budget = budget;
        p.exec_mode = exec;
        try {
          tcx::build_plan(p, tcx::network_of(net), tcx::path_of(path));
          const tcx::WorkspaceLayout w = tcx::workspace_layout(p);
          expect(!budget || w.total <= budget, std::string(what) + ": within budget");
          expect(!tcx::launch_order(p, grad).empty(), std::string(what) + ": launches");
        } catch (const tcx::Error& e) {
          expect(e.status == TC_ERR_TOO_LARGE && budget, std::string(what) + ": plan " + e.msg);
        }
      }
  // the automatic mode with an LDS arena: its light runs are resident
  // launches, checked against the same plan's plain records
  for (uint32_t lds : {1024u, 16384u}) {
    tcx::Plan p;
    p.want_grad = grad ? 1 : 0;
    p.lds_elems = lds;
    try {
      tcx::build_plan(p, tcx::network_of(net), tcx::path_of(path));
    } catch (const tcx::Error& e) {
      expect(false, std::string(what) + ": automatic plan with LDS " + e.msg);
      continue;
    }
    if (!p.resident_runs) continue;
    ++runs_checked;
    const std::vector<val> want = run_resident(p, false, grad, false);
    expect(same(run_resident(p, true, grad, false), want), std::string(what) + ": resident runs");
    expect(same(run_resident(p, true, grad, true), want), std::string(what) + ": resident runs, nodes reversed");
  }
  // resident term launches: a small LDS arena (most tensors global) and a
  // large one, each against the same plan's plain records
  for (uint32_t lds : {1024u, 16384u}) {
    tcx::Plan p;
    p.want_grad = grad ? 1 : 0;
    p.exec_mode = 3;
    p.lds_elems = lds;
    try {
      tcx::build_plan(p, tcx::network_of(net), tcx::path_of(path));
    } catch (const tcx::Error& e) {
      // (nodes for the GEMM path rule the mode out)
      expect(e.status == TC_ERR_UNSUPPORTED, std::string(what) + ": resident plan " + e.msg);
      continue;
    }
    expect(p.resident && p.exec_used == 4, std::string(what) + ": resident mode");
    ++resident_checked;
    const std::vector<val> want = run_resident(p, false, grad, false);
    expect(same(run_resident(p, true, grad, false), want), std::string(what) + ": resident values");
    expect(same(run_resident(p, true, grad, true), want), std::string(what) + ": resident values, nodes reversed");
    // a planted misplacement must show: the first node that reads an LDS
    // operand reads it from the wrong place
    if (lds == 16384u)
      for (tcx::DevROp& r : p.rops)
        if (r.shape & tcx::RES_A_LDS) {
          const uint32_t keep = r.a;
          r.a = keep >= 8 ? keep - 8 : keep + 8;
          expect(!same(run_resident(p, true, grad, false), want), std::string(what) + ": planted misplacement seen");
          r.a = keep;
          break;
        }
    if (grad) {
      // the forward-only launch gives the same roots
      std::vector<val> fw = run_resident(p, true, false, false), ref = run_resident(p, false, false, false);
      expect(same(fw, ref), std::string(what) + ": resident forward launch");
    }
  }
}

void one(Circ& c, tc_observable* o, bool grad, const char* what, int reconf, int score) {
  tc_circuit cc = c.c();
  tc_network* net = nullptr;
  if (tc_build_network(&cc, o, nullptr, &net) != TC_OK) {
    expect(false, std::string(what) + ": network");
    return;
  }
  tc_path_opts po{7, 4, score, 0.1, reconf, reconf ? 12 : 0};
  tc_path* path = nullptr;
  expect(tc_greedy_path(net, &po, &path) == TC_OK, std::string(what) + ": path");
  if (path) {
    run_plans(net, path, grad, what);
    tc_path_stats st{};
    tc_path_stats_get(path, -1, &st);
    tc_network* snet = nullptr;
    tc_path* spath = nullptr;
    int32_t s = 0;
    const int target = std::max(2, (int)std::lround(st.log2_size) - 2);
    const tc_status rs = tc_slice(net, path, target, 16, &snet, &spath, &s);
    expect(rs == TC_OK || rs == TC_ERR_TOO_LARGE, std::string(what) + ": slice");
    if (rs == TC_OK) {
      tc_path_stats ss{};
      expect(tc_path_stats_get(spath, -1, &ss) == TC_OK && ss.log2_size <= target + 1e-9,
             std::string(what) + ": sliced size");
      run_plans(snet, spath, grad, what);
      tc_path_free(spath);
      tc_network_free(snet);
    }
    tc_path_free(path);
  }
  tc_network_free(net);
}

}  // namespace

int main() {
  {
    Circ c = ladder(10, 3);
    Obs o = tfim(10);
    one(c, &o.o, true, "ladder tfim", 0, TC_SCORE_COMBO);
    one(c, &o.o, true, "ladder tfim reconf", 8, TC_SCORE_TIME);
    Obs m = mpo_random(10);
    one(c, &m.o, true, "ladder mpo", 6, TC_SCORE_TIME);
  }
  {
    Circ c = grid(3, 3, 2);
    Obs o = tfim(9);
    one(c, &o.o, true, "grid fsim tfim", 8, TC_SCORE_COMBO);
    std::vector<uint8_t> bits(9, 1);
    tc_observable amp{TC_OBS_AMPLITUDE, bits.data(), 0, nullptr, nullptr, nullptr, nullptr};
    one(c, &amp, false, "grid amplitude", 8, TC_SCORE_COMBO);
  }
  for (int seed = 0; seed < 3; ++seed) {
    Circ c = all_kinds(6, seed);
    Obs o = tfim(6);
    one(c, &o.o, true, "all kinds", seed % 2 ? 6 : 0, seed % 2 ? TC_SCORE_TIME : TC_SCORE_COMBO);
  }
  {
    // geometric tensor plan on the state network
    Circ c = all_kinds(6, 9);
    tc_circuit cc = c.c();
    tc_observable st{TC_OBS_STATE, nullptr, 0, nullptr, nullptr, nullptr, nullptr};
    tc_network* net = nullptr;
    expect(tc_build_network(&cc, &st, nullptr, &net) == TC_OK, "state network");
    tc_path_opts po{3, 2, TC_SCORE_COMBO, 0.1, 0, 0};
    tc_path* path = nullptr;
    expect(tc_greedy_path(net, &po, &path) == TC_OK, "state path");
    tcx::Plan p;
    p.qgt = 1;
    try {
      tcx::build_plan(p, tcx::network_of(net), tcx::path_of(path));
      expect(p.qgt_rows > 0 && p.batch == p.qgt_rows, "qgt rows");
    } catch (const tcx::Error& e) {
      expect(false, "qgt plan: " + e.msg);
    }
    tc_path_free(path);
    tc_network_free(net);
  }
  {
    // documented errors
    Circ c = ladder(4, 1);
    c.gates[0].q[1] = 9;  // qubit out of range
    tc_circuit cc = c.c();
    Obs o = tfim(4);
    tc_network* net = nullptr;
    expect(tc_build_network(&cc, &o.o, nullptr, &net) == TC_ERR_INVALID_ARG, "bad qubit");
    Circ d;
    d.n = 1;
    d.n_params = 1;
    d.add(TC_GATE_DEPOL, 0, -1, 0, -1, {0.5, 0.4, 0.3});  // sum > 1
    tc_circuit dc = d.c();
    Obs one_q = tfim(1);
    expect(tc_build_network(&dc, &one_q.o, nullptr, &net) == TC_ERR_INVALID_ARG, "bad probabilities");
    Obs bad = tfim(4);
    bad.st[0] = 7;
    Circ e = ladder(4, 1);
    tc_circuit ec = e.c();
    expect(tc_build_network(&ec, &bad.o, nullptr, &net) == TC_ERR_INVALID_ARG, "bad structure");
  }
  if (failures) {
    std::fprintf(stderr, "%d failures\n", failures);
    return 1;
  }
  expect(resident_checked >= 8, "resident plans checked");
  expect(runs_checked >= 4, "plans with resident runs checked");
  std::printf("host check ok (%d resident plans, %d plans with resident runs simulated)\n",
              resident_checked, runs_checked);
  return 0;
}
