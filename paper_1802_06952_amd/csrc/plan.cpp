// Host planner of the qs library.
//
// Partition (Sec. 2.1; Supp. A): the CZ gates with one endpoint in each half
// are the cut gates E_int; each becomes P_b on its upper endpoint and Z^b on
// its lower endpoint (Eq. 1), giving 2^c copies of two independent halves.
//
// Copy tree of one half (the prefix reuse of Sec. 2.3.2, taken further): a
// cut factor is diagonal, so it commutes with every gate except a
// non-diagonal gate on its own qubit.  An operation depends on cut j when a
// chain of non-commuting operations leads from the cut factor to it; every
// operation that depends on no undecided cut runs once for all copies that
// share the decided bits.  Cuts are decided in the order of their first
// dependent operation; a level of the tree holds the cuts decided together
// and the operations that become runnable.  A cut with no dependent operation
// is only applied to the output amplitudes.
//
// Levels up to a chosen depth are materialised as full half states by
// passes over register tiles of one wavefront (LDS tiles for small halves);
// a pass may descend several levels at once.  The deeper levels are evaluated
// only at the requested half values, on the subspace spanned by the
// non-diagonal targets of those levels (the light cone), which these levels
// leave invariant.
#include "plan.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <map>
#include <sstream>

namespace qs {

static inline int popc64(uint64_t x) { return __builtin_popcountll(x); }

bool build_partition(const Circuit& c, uint64_t upper_mask, std::vector<Cut>& cuts, Side& up,
                     Side& lo, std::string& err) {
  const int n = c.n;
  const uint64_t full = (n == 64) ? ~0ULL : ((1ULL << n) - 1);
  if (upper_mask == 0 || (upper_mask & ~full) != 0 || (upper_mask & full) == full) {
    err = "upper_mask must be a non-empty proper subset of the circuit's qubits";
    return false;
  }
  const uint64_t lower_mask = full & ~upper_mask;
  cuts.clear();
  std::vector<std::tuple<int, int, int>> raw;
  for (const Gate& g : c.gates) {
    if (g.kind != G_CZ) continue;
    bool ua = (upper_mask >> g.q0) & 1, ub = (upper_mask >> g.q1) & 1;
    if (ua != ub) raw.emplace_back(g.cycle, ua ? g.q0 : g.q1, ua ? g.q1 : g.q0);
  }
  std::sort(raw.begin(), raw.end());
  for (size_t j = 0; j < raw.size(); ++j)
    cuts.push_back(Cut{(int)j, std::get<0>(raw[j]), std::get<1>(raw[j]), std::get<2>(raw[j])});
  std::map<std::pair<int, int>, int> cut_of;  // (cycle, endpoint) -> cut
  for (const Cut& k : cuts) {
    cut_of[{k.cycle, k.upper}] = k.index;
    cut_of[{k.cycle, k.lower}] = k.index;
  }
  build_side(c, upper_mask, true, cut_of, up);
  build_side(c, lower_mask, false, cut_of, lo);
  return true;
}

void build_side(const Circuit& c, uint64_t mask, bool upper,
                const std::map<std::pair<int, int>, int>& cut_of, Side& s) {
  const int n = c.n;
  {
    s = Side();
    s.upper = upper;
    std::vector<int> loc(n, -1);
    for (int q = 0; q < n; ++q)
      if ((mask >> q) & 1) {
        loc[q] = (int)s.qubits.size();
        s.qubits.push_back(q);
      }
    s.n = (int)s.qubits.size();
    std::vector<HOp> ops;
    for (const Gate& g : c.gates) {
      if (g.kind == G_CZ) {
        int a = loc[g.q0], b = loc[g.q1];
        if (a >= 0 && b >= 0) ops.push_back(HOp{OP_CZ, a, b, -1, 0, g.cycle});
        else if (a >= 0 || b >= 0) {
          int q = a >= 0 ? g.q0 : g.q1;
          ops.push_back(HOp{OP_CUT, loc[q], -1, cut_of.at({g.cycle, q}), 0, g.cycle});
        }
      } else {
        int a = loc[g.q0];
        if (a < 0) continue;
        if (g.kind == G_T) ops.push_back(HOp{OP_T, a, -1, -1, g.pw, g.cycle});
        else ops.push_back(HOp{OP_MAT, a, -1, -1, g.kind == G_H ? 0 : (g.kind == G_SX ? 1 : 2), g.cycle});
      }
    }
    // fold each qubit's leading H into the initial product state
    std::vector<bool> touched(s.n, false);
    for (const HOp& o : ops) {
      bool fold = false;
      if (o.kind == OP_MAT && o.mat == 0 && !touched[o.q0]) {
        fold = true;
        s.hinit |= 1ULL << o.q0;
      }
      touched[o.q0] = true;
      if (o.q1 >= 0) touched[o.q1] = true;
      if (!fold) s.ops.push_back(o);
    }
  }
}

Tree build_tree(const Side& s, int c, const Block& blk) {
  Tree t;
  t.fixed.assign(c, -1);
  for (int j = 0; j < blk.p && j < c; ++j) t.fixed[j] = (int)((blk.k0 >> (c - 1 - j)) & 1);
  const int nops = (int)s.ops.size();
  auto is_free_cut = [&](const HOp& o) { return o.kind == OP_CUT && t.fixed[o.cut] < 0; };
  // dependency masks over cuts
  std::vector<uint64_t> dep(nops, 0);
  std::vector<uint64_t> acc_all(s.n, 0), acc_nd(s.n, 0);
  for (int i = 0; i < nops; ++i) {
    const HOp& o = s.ops[i];
    bool nd = o.kind == OP_MAT;
    uint64_t d = 0;
    int qs[2] = {o.q0, o.q1};
    for (int k = 0; k < 2; ++k) {
      if (qs[k] < 0) continue;
      d |= nd ? acc_all[qs[k]] : acc_nd[qs[k]];
    }
    dep[i] = d;
    uint64_t own = d | (is_free_cut(o) ? (1ULL << o.cut) : 0);
    for (int k = 0; k < 2; ++k) {
      if (qs[k] < 0) continue;
      acc_all[qs[k]] |= own;
      if (nd) acc_nd[qs[k]] |= own;
    }
  }
  // order free cuts by first dependent op
  std::vector<int> first(c, -1);
  for (int i = 0; i < nops; ++i) {
    if (is_free_cut(s.ops[i])) continue;
    for (int j = 0; j < c; ++j)
      if (((dep[i] >> j) & 1) && first[j] < 0) first[j] = i;
  }
  std::vector<int> order;
  for (int j = 0; j < c; ++j)
    if (t.fixed[j] < 0) {
      if (first[j] >= 0) order.push_back(j);
      else t.end_cuts.push_back(j);
    }
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return first[a] < first[b]; });
  std::vector<bool> done(nops, false);
  uint64_t D = 0;
  auto take = [&]() {
    std::vector<int> lst;
    for (int i = 0; i < nops; ++i) {
      if (done[i] || is_free_cut(s.ops[i])) continue;
      if ((dep[i] & ~D) == 0) {
        done[i] = true;
        lst.push_back(i);
      }
    }
    return lst;
  };
  t.levels.push_back(Level{{}, take()});
  std::vector<int> pend;
  for (size_t a = 0; a < order.size(); ++a) {
    pend.push_back(order[a]);
    D |= 1ULL << order[a];
    std::vector<int> lst = take();
    if (!lst.empty() || (int)pend.size() == kMaxBranch || a + 1 == order.size()) {
      t.levels.push_back(Level{pend, lst});
      pend.clear();
    }
  }
  for (const Level& L : t.levels)
    for (int j : L.cuts) t.order.push_back(j);
  for (int j : t.end_cuts) t.order.push_back(j);
  return t;
}

namespace {

// Greedy pass packing: take ops in order while their non-diagonal targets fit
// in the tile and the pass holds fewer than `budget` ops; an op that does not
// fit is deferred together with every later op that does not commute with a
// deferred one.
void absorb(const Side& s, const std::vector<int>& P, std::vector<int>& S, int tmax,
            std::vector<int>& taken, std::vector<int>& deferred, bool one_op, int& budget) {
  std::vector<char> nd_def(s.n, 0), any_def(s.n, 0);
  taken.clear();
  deferred.clear();
  for (int i : P) {
    if ((one_op && !taken.empty()) || budget <= 0) {
      deferred.push_back(i);
      continue;
    }
    const HOp& o = s.ops[i];
    bool nd = o.kind == OP_MAT;
    bool conflict = false;
    if (nd) conflict = any_def[o.q0];
    else {
      conflict = nd_def[o.q0] || (o.q1 >= 0 && nd_def[o.q1]);
    }
    if (!conflict && nd && std::find(S.begin(), S.end(), o.q0) == S.end()) {
      if ((int)S.size() < tmax) S.push_back(o.q0);
      else conflict = true;
    }
    if (conflict) {
      deferred.push_back(i);
      any_def[o.q0] = 1;
      if (o.q1 >= 0) any_def[o.q1] = 1;
      if (nd) nd_def[o.q0] = 1;
    } else {
      taken.push_back(i);
      --budget;
    }
  }
}

}  // namespace

namespace {

// Cost units: bytes moved at HBM speed (8 TB/s); arithmetic is converted at the
// VALU rate of the chip without packed FP32 (one wave64 instruction per cycle
// per compute unit: about 39 T lane-operations per second, i.e. 0.2 byte per
// lane-operation), and every launch costs about 10 us.
constexpr double kBytesPerLaneOp = 8.0e12 / 39.3e12;
constexpr double kLaunchBytes = 8.0e12 * 10e-6;

double op_cost(const Side& s, const std::vector<int>& ops) {
  // lane-operations per amplitude: a 2x2 gate about 10, a fused diagonal run about 16
  double c = 0;
  bool in_diag = false;
  for (int i : ops) {
    if (s.ops[i].kind == OP_MAT) {
      c += 10;
      in_diag = false;
    } else if (!in_diag) {
      c += 16;
      in_diag = true;
    }
  }
  return c;
}

// Cost-model price and peak live states of one pass.
void price_pass(const Side& s, const PassPlan& pp, const std::vector<uint64_t>& nodes,
                double& cost, size_t& peak) {
  const double B = std::ldexp(8.0, s.n);
  const double N = std::ldexp(1.0, s.n);
  const double nin = (double)nodes[pp.level_in];
  double bytes, alu;
  if (pp.branch()) {
    const double nout = (double)nodes[pp.level_out()];
    bytes = (pp.init ? 0 : B * nin) + B * nout;
    alu = op_cost(s, pp.ops_in);
    for (size_t st = 0; st < pp.stages.size(); ++st)
      alu += ((double)nodes[pp.level_in + st + 1] / nin) * (op_cost(s, pp.stages[st]) + 6);
    alu *= N * nin;
    peak = std::max<size_t>(peak, nodes[pp.level_in] + nodes[pp.level_out()]);
  } else {
    bytes = (pp.init ? 1 : 2) * B * nin;
    alu = N * nin * (op_cost(s, pp.ops_in) + 4);
    peak = std::max<size_t>(peak, nodes[pp.level_in]);
  }
  cost += std::max(bytes, alu * kBytesPerLaneOp) + kLaunchBytes;
}

// Packing of the materialised levels 0..ls into passes.  Inside a level the
// pending ops go greedily into passes of at most t tile bits; the pass that
// takes the last of them branches, and descends 1 .. max_stages levels at
// once (each further stage only if the previous level's ops all fitted), so
// the levels in between never reach memory.  The number of stages of every
// branch pass is chosen for the lowest total cost (a search over the levels
// where the passes land; the state after a branch pass is its landing level
// and the ops of that level still pending).
struct PassPacker {
  const Side& s;
  const Tree& tree;
  int ls, t, tmin, b, max_stages;
  bool one_op;
  const std::vector<uint64_t>& nodes;
  bool exchange;
  struct Res {
    double cost = 0;
    size_t peak = 1;
    std::vector<PassPlan> passes;
  };
  std::map<std::pair<int, std::vector<int>>, Res> memo;

  Res solve(int cur, std::vector<int> P, bool first) {
    const auto key = std::make_pair(first ? -1 - cur : cur, P);
    auto it = memo.find(key);
    if (it != memo.end()) return it->second;
    Res r;
    for (int guard = 0; guard < 100000; ++guard) {
      if (cur == ls && P.empty() && !first) break;  // landed on the last level with nothing left
      PassPlan pp;
      pp.level_in = cur;
      pp.init = first;
      first = false;
      std::vector<int> S;
      for (int q = 0; q < b; ++q) S.push_back(q);
      std::vector<int> deferred;
      int budget = kMaxPassOps;
      absorb(s, P, S, t, pp.ops_in, deferred, one_op, budget);
      if (!deferred.empty() && try_group(pp, P, r)) continue;
      P = deferred;
      const bool open = deferred.empty() && !(one_op && !pp.ops_in.empty());
      if (!open || cur == ls) {
        finish(pp, S);
        price_pass(s, pp, nodes, r.cost, r.peak);
        r.passes.push_back(pp);
        if (cur == ls && P.empty()) break;
        continue;
      }
      // branch: try every feasible number of stages
      Res best;
      bool have = false;
      PassPlan bp = pp;
      std::vector<int> BS = S;
      int bud = budget;
      for (int ns = 1; ns <= max_stages && cur + ns <= ls; ++ns) {
        std::vector<int> taken, d2;
        absorb(s, tree.levels[cur + ns].ops, BS, t, taken, d2, one_op, bud);
        bp.stages.push_back(taken);
        PassPlan fin = bp;
        finish(fin, BS);
        Res cand;
        price_pass(s, fin, nodes, cand.cost, cand.peak);
        Res rest = solve(cur + ns, d2, false);
        cand.cost += rest.cost;
        cand.peak = std::max(cand.peak, rest.peak);
        cand.passes.push_back(fin);
        cand.passes.insert(cand.passes.end(), rest.passes.begin(), rest.passes.end());
        if (!have || cand.cost < best.cost) {
          best = std::move(cand);
          have = true;
        }
        if (!d2.empty() || bud <= 0) break;  // a further stage needs all of this level's ops
      }
      r.cost += best.cost;
      r.peak = std::max(r.peak, best.peak);
      r.passes.insert(r.passes.end(), best.passes.begin(), best.passes.end());
      break;
    }
    memo[key] = r;
    return r;
  }

  // Exchange group instead of the pass pp: gates are taken into a workgroup
  // tile of kXWaveBits more bits (U: its non-lane bits), and the taken
  // sequence splits into phases of at most R = t - 6 non-lane targets each;
  // consecutive phases exchange the tile through LDS (k_xpass), so the group
  // reads and writes the states once.  Used when the wide tile still leaves
  // ops for a later pass (the group never ends a level's schedule) and takes
  // more ops than the plain pass; emits the phases into r and leaves the
  // deferred ops in P.
  bool try_group(const PassPlan& pp, std::vector<int>& P, Res& r) const {
    const int R = t - b;
    if (!exchange || one_op || b != 6 || R < kXMinRegBits || t + kXWaveBits > s.n) return false;
    std::vector<int> SX;
    for (int q = 0; q < b; ++q) SX.push_back(q);
    std::vector<int> taken, def;
    int budget = kMaxPassOps;
    absorb(s, P, SX, t + kXWaveBits, taken, def, one_op, budget);
    if (def.empty() || taken.size() <= pp.ops_in.size()) return false;
    // phases: the longest runs of the taken sequence with at most R non-lane targets
    std::vector<std::vector<int>> ph(1), regs(1);
    for (int i : taken) {
      const HOp& o = s.ops[i];
      if (o.kind == OP_MAT && o.q0 >= b &&
          std::find(regs.back().begin(), regs.back().end(), o.q0) == regs.back().end()) {
        if ((int)regs.back().size() == R) {
          ph.emplace_back();
          regs.emplace_back();
        }
        regs.back().push_back(o.q0);
      }
      ph.back().push_back(i);
    }
    if (ph.size() < 2 || ph.size() > (size_t)kMaxXPhases) return false;
    std::vector<int> U(SX.begin() + b, SX.end());
    for (int q = b; (int)U.size() < R + kXWaveBits && q < s.n; ++q)
      if (std::find(U.begin(), U.end(), q) == U.end()) U.push_back(q);
    std::sort(U.begin(), U.end());
    for (size_t k = 0; k < ph.size(); ++k) {
      PassPlan g;
      g.level_in = pp.level_in;
      g.init = pp.init && k == 0;
      g.ops_in = ph[k];
      std::vector<int> T = regs[k];
      for (int q : U)
        if ((int)T.size() < R && std::find(T.begin(), T.end(), q) == T.end()) T.push_back(q);
      for (int q = 0; q < b; ++q) T.push_back(q);
      std::sort(T.begin(), T.end());
      g.tile = T;
      g.xg = k == 0 ? (int)ph.size() : 0;
      if (k == 0) g.xu = U;
      r.passes.push_back(g);
    }
    // price: one read and one write of the states, the phases' arithmetic
    PassPlan whole = pp;
    whole.ops_in = taken;
    price_pass(s, whole, nodes, r.cost, r.peak);
    P = def;
    return true;
  }

  // fill the tile with the lowest unused qubits up to tmin bits (a tile holds
  // at least the pass's targets; a smaller tile means fewer registers per
  // lane and more wavefronts in flight)
  void finish(PassPlan& pp, std::vector<int> S) const {
    for (int q = 0; (int)S.size() < tmin && q < s.n; ++q)
      if (std::find(S.begin(), S.end(), q) == S.end()) S.push_back(q);
    std::sort(S.begin(), S.end());
    pp.tile = S;
  }
};

void build_passes(const Side& s, const Tree& tree, int ls, int t, int tmin, int b, bool one_op,
                  int max_stages, bool exchange, const std::vector<uint64_t>& nodes,
                  std::vector<PassPlan>& passes, double& cost, size_t& peak) {
  PassPacker pk{s, tree, ls, t, std::min(t, tmin), b,
                one_op ? 1 : std::max(1, std::min(max_stages, kMaxStages)), one_op, nodes, exchange,
                {}};
  PassPacker::Res r = pk.solve(0, tree.levels[0].ops, true);
  passes = std::move(r.passes);
  cost = r.cost;
  peak = r.peak;
}

}  // namespace

bool plan_side(const Side& s, int c, const Block& blk, const PlanKnobs& kn, SidePlan& out,
               std::string& err) {
  Tree tree = build_tree(s, c, blk);
  const int L = (int)tree.levels.size() - 1;
  std::vector<uint64_t> nodes(L + 1, 1);
  for (int l = 1; l <= L; ++l) nodes[l] = nodes[l - 1] << tree.levels[l].cuts.size();
  const double B = std::ldexp(8.0, s.n);
  // states of 7+ qubits use wave tiles: lanes over state bits 0..5 plus up to
  // 5 register bits; smaller states are staged whole in LDS
  int t, tmin, b;
  if (s.n >= 7) {
    t = std::max(7, std::min({kn.tile_bits, s.n, 11}));
    tmin = std::max(7, std::min(kn.min_tile_bits, t));
    b = 6;
  } else {
    t = tmin = s.n;
    b = std::max(0, std::min(kn.coalesce_bits, t - 1));
  }

  bool found = false;
  SidePlan best;
  for (int ls = 0; ls <= L; ++ls) {
    if (kn.force_lstar >= 0 && ls != std::min(kn.force_lstar, L)) continue;
    SidePlan sp;
    sp.tree = tree;
    sp.lstar = ls;
    sp.nodes = nodes;
    // light cone of the levels below ls
    std::vector<int> Q;
    for (int l = ls + 1; l <= L; ++l)
      for (int i : tree.levels[l].ops)
        if (s.ops[i].kind == OP_MAT && std::find(Q.begin(), Q.end(), s.ops[i].q0) == Q.end())
          Q.push_back(s.ops[i].q0);
    std::sort(Q.begin(), Q.end());
    if ((int)Q.size() > kn.tail_max_qubits) continue;
    sp.Q = Q;
    const int q = (int)Q.size();
    const int nlev = L - ls;
    int M = 0;
    for (int l = ls + 1; l <= L; ++l) M += (int)tree.levels[l].cuts.size();
    if (nlev > kMaxTailLevels || M > 16) continue;
    double cost = 0;
    size_t peak = 1;
    build_passes(s, tree, ls, t, tmin, b, kn.one_op_per_pass, kn.max_stages, kn.exchange, nodes,
                 sp.passes, cost, peak);
    // leaf evaluation: the backward rows per requested value (arithmetic and
    // the W round trip), the contiguous gathers of the node amplitudes (the
    // light cone is relabelled onto the lowest state bits), and the per-value
    // GEMM on MFMA
    const double K = std::ldexp(1.0, q), Lam = std::ldexp(1.0, M), Sd = kn.S;
    double rev = 0, paths = 1;
    for (int l = L; l > ls; --l) {
      double nops = 1;
      for (int i : tree.levels[l].ops) nops += s.ops[i].kind == OP_MAT ? 1.0 : 1.5;
      rev += paths * nops * K;
      paths *= std::ldexp(1.0, (int)tree.levels[l].cuts.size());
    }
    cost += Sd * rev * 12.0 * kBytesPerLaneOp;                              // backward rows
    cost += Sd * Lam * K * 16.0;                                            // W written and read
    cost += Sd * std::ceil(Lam / 64.0) * K * (double)nodes[ls] * 8.0;       // gathers
    cost += Sd * Lam * K * (double)nodes[ls] * 8.0 / 80.0e12 * 8.0e12;      // MFMA GEMM
    cost += 2 * kLaunchBytes;
    sp.cost_bytes = cost;
    sp.peak_states = peak;
    if (kn.mem_budget && (double)peak * B > (double)kn.mem_budget) continue;
    if (!found || cost < best.cost_bytes) {
      best = sp;
      found = true;
    }
  }
  if (!found) {
    err = "no feasible schedule: light cone of the leaf levels exceeds the limit or the "
          "materialised states exceed the memory budget";
    return false;
  }
  // relabel the half's qubits so that the light cone sits on the lowest state
  // bits (the leaf evaluation then gathers contiguous runs), and pack the
  // passes again for the relabelled program
  best.perm.assign(s.n, -1);
  int next = 0;
  for (int qq : best.Q) best.perm[qq] = next++;
  for (int qq = 0; qq < s.n; ++qq)
    if (best.perm[qq] < 0) best.perm[qq] = next++;
  Side& r = best.side;
  r = s;
  for (int i = 0; i < s.n; ++i) r.qubits[best.perm[i]] = s.qubits[i];
  r.hinit = 0;
  for (int i = 0; i < s.n; ++i)
    if ((s.hinit >> i) & 1) r.hinit |= 1ULL << best.perm[i];
  for (HOp& o : r.ops) {
    o.q0 = best.perm[o.q0];
    if (o.q1 >= 0) o.q1 = best.perm[o.q1];
  }
  {
    double cost = 0;
    size_t peak = 1;
    build_passes(r, best.tree, best.lstar, t, tmin, b, kn.one_op_per_pass, kn.max_stages,
                 kn.exchange, best.nodes, best.passes, cost, peak);
  }
  out = std::move(best);
  return true;
}

namespace {

struct DiagAcc {
  int w[64] = {0};
  std::map<int, uint64_t> cz;  // distance -> mask of lower endpoints
  uint64_t pmask = 0, pval = 0;
  bool zero = false;
  bool any = false;
  void reset() { *this = DiagAcc(); }
};

// Does the accumulated diagonal act on qubit q?  A 2x2 gate on q commutes
// with every diagonal factor that does not.
bool involves(const DiagAcc& a, int q) {
  if (!a.any) return false;
  if (a.zero || (a.w[q] & 7) || ((a.pmask >> q) & 1)) return true;
  for (const auto& kv : a.cz) {
    if ((kv.second >> q) & 1) return true;
    if (q >= kv.first && ((kv.second >> (q - kv.first)) & 1)) return true;
  }
  return false;
}

void flush(DiagAcc& a, std::vector<DevOp>& out) {
  if (!a.any) return;
  std::vector<std::pair<int, uint64_t>> dl;
  for (auto& kv : a.cz)
    if (kv.second) dl.push_back(kv);
  size_t at = 0;
  bool firstop = true;
  do {
    DevOp op{};
    op.kind = 1;
    if (firstop) {
      for (int q = 0; q < 64; ++q) {
        int w = a.w[q] & 7;
        if (w & 1) op.t0 |= 1ULL << q;
        if (w & 2) op.t1 |= 1ULL << q;
        if (w & 4) op.t2 |= 1ULL << q;
      }
      op.pmask = a.pmask;
      op.pval = a.pval;
      if (a.zero) {
        op.pmask = 1;
        op.pval = 2;
      }
    }
    int k = 0;
    while (at < dl.size() && k < kMaxDiagDist) {
      op.d[k] = dl[at].first;
      op.M[k] = dl[at].second;
      ++k;
      ++at;
    }
    op.nd = k;
    out.push_back(op);
    firstop = false;
  } while (at < dl.size());
  a.reset();
}

void set_mat(DevOp& op, int mat) {
  // the unit-entry part of the gate (the scalar goes to the half's constant)
  if (mat == 0) {  // H = 1/sqrt 2 [[1, 1], [1, -1]]
    const float v[8] = {1, 0, 1, 0, 1, 0, -1, 0};
    std::copy(v, v + 8, op.m);
    op.mk = MK_H;
  } else if (mat == 1) {  // sqrt X = (1+i)/2 [[1, -i], [-i, 1]]
    const float v[8] = {1, 0, 0, -1, 0, -1, 1, 0};
    std::copy(v, v + 8, op.m);
    op.mk = MK_X;
  } else {  // sqrt Y = (1+i)/2 [[1, -1], [1, 1]]
    const float v[8] = {1, 0, -1, 0, 1, 0, 1, 0};
    std::copy(v, v + 8, op.m);
    op.mk = MK_Y;
  }
}

}  // namespace

namespace {

// Register split of a DIAG op for a wave-tile pass (see DevOp).
void split_registers(DevOp& op, const std::vector<int>& rb) {
  const int R = (int)rb.size();
  auto reg_index = [&](int bit) {
    for (int k = 0; k < R; ++k)
      if (rb[k] == bit) return k;
    return -1;
  };
  for (int k = 0; k < R; ++k) {
    const int rho = rb[k];
    op.wl[k] = (int)(((op.t0 >> rho) & 1) + 2 * ((op.t1 >> rho) & 1) + 4 * ((op.t2 >> rho) & 1));
    op.cross[k] = 0;
    op.rr[k] = 0;
  }
  for (int i = 0; i < op.nd; ++i) {
    const int d = op.d[i];
    for (int a = 0; a + d < 64; ++a) {
      if (!((op.M[i] >> a) & 1)) continue;
      const int b = a + d;  // the pair (a, b) of state bits
      const int ka = reg_index(a), kb = reg_index(b);
      if (ka >= 0 && kb >= 0) {
        if (ka < kb) op.rr[kb] |= 1u << ka;
        else op.rr[ka] |= 1u << kb;
      } else if (ka >= 0) {
        op.cross[ka] |= 1u << b;
      } else if (kb >= 0) {
        op.cross[kb] |= 1u << a;
      }
    }
  }
}

}  // namespace

bool encode_ops(const Side& s, const std::vector<int>& ops, const std::vector<int>& fixed_bits,
                const std::vector<int>& work_of, std::vector<DevOp>& out, std::string& err,
                bool transpose, const std::vector<int>* reg_bits) {
  const size_t first_new = out.size();
  DiagAcc acc;
  for (int i : ops) {
    const HOp& o = s.ops[i];
    switch (o.kind) {
      case OP_MAT: {
        // the pending diagonal goes out first only if it touches the gate's
        // qubit; otherwise the gate is moved ahead of it
        if (involves(acc, o.q0)) flush(acc, out);
        int w = work_of[o.q0];
        if (w < 0) {
          err = "internal: non-diagonal gate outside the working bits";
          return false;
        }
        DevOp op{};
        op.kind = 0;
        op.target = w;
        set_mat(op, o.mat);
        if (transpose) {
          std::swap(op.m[2], op.m[4]);
          std::swap(op.m[3], op.m[5]);
          if (op.mk == MK_Y) op.mk = MK_YT;  // X and H are symmetric
        }
        out.push_back(op);
        break;
      }
      case OP_T:
        acc.w[o.q0] += o.mat;  // T^mat
        acc.any = true;
        break;
      case OP_CZ: {
        int lo = std::min(o.q0, o.q1), hi = std::max(o.q0, o.q1);
        acc.cz[hi - lo] ^= 1ULL << lo;
        acc.any = true;
        break;
      }
      case OP_CUT: {
        int bit = fixed_bits[o.cut];
        if (bit < 0) {
          err = "internal: free cut inside an op list";
          return false;
        }
        if (s.upper) {
          uint64_t m = 1ULL << o.q0;
          if ((acc.pmask & m) && (((acc.pval >> o.q0) & 1) != (uint64_t)bit)) acc.zero = true;
          acc.pmask |= m;
          if (bit) acc.pval |= m;
        } else if (bit) {
          acc.w[o.q0] += 4;
        }
        acc.any = true;
        break;
      }
    }
  }
  flush(acc, out);
  if (reg_bits)
    for (size_t i = first_new; i < out.size(); ++i)
      if (out[i].kind == 1) split_registers(out[i], *reg_bits);
  return true;
}

std::string dump_json(const Circuit& c, uint64_t upper_mask, const std::vector<Cut>& cuts,
                      const Side& up, const Side& lo, const SidePlan* pu, const SidePlan* pl) {
  std::ostringstream o;
  o << "{\"n\":" << c.n << ",\"upper_mask\":" << upper_mask << ",\"cuts\":[";
  for (size_t j = 0; j < cuts.size(); ++j)
    o << (j ? "," : "") << "[" << cuts[j].cycle << "," << cuts[j].upper << "," << cuts[j].lower << "]";
  o << "],\"sides\":[";
  for (int k = 0; k < 2; ++k) {
    const Side& s = k == 0 ? up : lo;
    const SidePlan* sp = k == 0 ? pu : pl;
    o << (k ? "," : "") << "{\"upper\":" << (s.upper ? "true" : "false") << ",\"n\":" << s.n
      << ",\"hinit\":" << s.hinit << ",\"qubits\":[";
    for (size_t i = 0; i < s.qubits.size(); ++i) o << (i ? "," : "") << s.qubits[i];
    o << "],\"ops\":[";
    for (size_t i = 0; i < s.ops.size(); ++i) {
      const HOp& h = s.ops[i];
      std::string nm = h.kind == OP_MAT ? (h.mat == 0 ? "h" : h.mat == 1 ? "sx" : "sy")
                       : h.kind == OP_T ? (h.mat == 1 ? "t" : "t" + std::to_string(h.mat))
                       : h.kind == OP_CZ ? "cz" : "cut";
      o << (i ? "," : "") << "[\"" << nm << "\"," << h.q0 << "," << h.q1 << "," << h.cut << ","
        << h.cycle << "]";
    }
    o << "]";
    if (sp) {
      o << ",\"lstar\":" << sp->lstar << ",\"cost_bytes\":" << sp->cost_bytes
        << ",\"peak_states\":" << sp->peak_states << ",\"end_cuts\":[";
      for (size_t i = 0; i < sp->tree.end_cuts.size(); ++i)
        o << (i ? "," : "") << sp->tree.end_cuts[i];
      o << "],\"levels\":[";
      for (size_t l = 0; l < sp->tree.levels.size(); ++l) {
        const Level& L = sp->tree.levels[l];
        o << (l ? "," : "") << "{\"cuts\":[";
        for (size_t i = 0; i < L.cuts.size(); ++i) o << (i ? "," : "") << L.cuts[i];
        o << "],\"ops\":[";
        for (size_t i = 0; i < L.ops.size(); ++i) o << (i ? "," : "") << L.ops[i];
        o << "],\"nodes\":" << sp->nodes[l] << "}";
      }
      o << "],\"passes\":[";
      for (size_t p = 0; p < sp->passes.size(); ++p) {
        const PassPlan& pp = sp->passes[p];
        o << (p ? "," : "") << "{\"level_in\":" << pp.level_in << ",\"init\":" << (pp.init ? 1 : 0)
          << ",\"branch\":" << pp.stages.size() << ",\"xg\":" << pp.xg << ",\"ops_in\":[";
        for (size_t i = 0; i < pp.ops_in.size(); ++i) o << (i ? "," : "") << pp.ops_in[i];
        o << "],\"stages\":[";
        for (size_t st = 0; st < pp.stages.size(); ++st) {
          o << (st ? "," : "") << "[";
          for (size_t i = 0; i < pp.stages[st].size(); ++i) o << (i ? "," : "") << pp.stages[st][i];
          o << "]";
        }
        o << "],\"tile\":[";
        // tiles are printed as local qubit ids of the unrelabelled half
        std::vector<int> inv(sp->perm.size());
        for (size_t i = 0; i < sp->perm.size(); ++i) inv[sp->perm[i]] = (int)i;
        for (size_t i = 0; i < pp.tile.size(); ++i)
          o << (i ? "," : "") << (inv.empty() ? pp.tile[i] : inv[pp.tile[i]]);
        o << "]}";
      }
      o << "],\"Q\":[";
      for (size_t i = 0; i < sp->Q.size(); ++i) o << (i ? "," : "") << sp->Q[i];
      o << "],\"perm\":[";
      for (size_t i = 0; i < sp->perm.size(); ++i) o << (i ? "," : "") << sp->perm[i];
      o << "]";
    }
    o << "}";
  }
  o << "]}";
  return o.str();
}

}  // namespace qs
