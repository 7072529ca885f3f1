// C ABI of the qs library and the executor of the half-circuit plans.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <tuple>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/qs.h"
#include "kernels.h"
#include "plan.h"
#include "qs_internal.h"

using namespace qs;

namespace {

thread_local std::string g_err;

qs_status fail(qs_status s, const std::string& m) {
  g_err = m;
  return s;
}

// Device memory of a plan: the caller's allocator (qs_options.alloc) or
// hipMalloc / hipFree.
struct DevAlloc {
  qs_allocator a{};
  void* get(size_t bytes) {
    if (a.alloc) return a.alloc(bytes, a.ctx);
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    return p;
  }
  void put(void* p) {
    if (!p) return;
    if (a.free) a.free(p, a.ctx);
    else (void)hipFree(p);
  }
};

// Device buffers of a plan, reused across calls.  The two halves of a copy
// block run on two streams; a released buffer is reused only by the stream
// that released it until settle(), called where the streams are ordered by
// events, makes every idle buffer usable by either.
struct Pool {
  struct Ent {
    void* p;
    size_t bytes;
    bool used;
    bool any;      // idle and usable by either stream
    void* owner;   // stream that released it
  };
  std::vector<Ent> ents;
  size_t held = 0;
  DevAlloc* da = nullptr;
  uint64_t frees = 0;  // counts trims (buffers handed back to the allocator)
  void* get(size_t bytes, void* stream) {
    if (bytes == 0) bytes = 256;
    Ent* best = nullptr;
    for (Ent& e : ents)
      if (!e.used && (e.any || e.owner == stream) && e.bytes >= bytes &&
          (!best || e.bytes < best->bytes))
        best = &e;
    if (best && best->bytes <= 2 * bytes + (1 << 20)) {
      best->used = true;
      return best->p;
    }
    void* p = da->get(bytes);
    if (!p) {
      // release idle buffers and retry once
      trim();
      p = da->get(bytes);
      if (!p) return nullptr;
    }
    ents.push_back(Ent{p, bytes, true, false, stream});
    held += bytes;
    return p;
  }
  void put(void* p, void* stream) {
    for (Ent& e : ents)
      if (e.p == p) {
        e.used = false;
        e.any = false;
        e.owner = stream;
      }
  }
  // released outside any stream order: reusable after the next settle()
  void put_unordered(void* p) {
    for (Ent& e : ents)
      if (e.p == p) {
        e.used = false;
        e.any = false;
        e.owner = &ents;  // matches no stream
      }
  }
  void settle() {
    for (Ent& e : ents)
      if (!e.used) e.any = true;
  }
  void trim() {
    // idle buffers may still be read by queued kernels
    (void)hipDeviceSynchronize();
    ++frees;
    std::vector<Ent> keep;
    for (Ent& e : ents) {
      if (e.used) keep.push_back(e);
      else {
        da->put(e.p);
        held -= e.bytes;
      }
    }
    ents.swap(keep);
  }
  void release_all() {
    for (Ent& e : ents) da->put(e.p);
    ents.clear();
    held = 0;
  }
};

struct BlockRes {
  uint64_t k0 = 0, k1 = 0;
  // X[side][s * K_b + nu]: half amplitudes at requested value s; nu runs over
  // the block's copies in the upper half's natural order (the lower half is
  // permuted onto it), so both sides share the contraction index
  float2* X[2] = {nullptr, nullptr};
  std::shared_ptr<std::vector<uint32_t>> nu_to_k;  // copy (block-local) of each nu
  // Lower end cuts folded into the upper operand (ne > 0): Ut[sig][s][nu'] is
  // X[0] transformed over the end bits (positions pos[] of nu), X[1] holds
  // only the lower copies with end bits 0, as rows sorted by sig with columns
  // nu' (nu without the end bits); rows goff[sig] .. goff[sig+1] - 1 of X[1]
  // are the lower values d_rows[...] (original value indices).
  int ne = 0;
  int pos[4] = {0, 0, 0, 0};
  float2* Ut = nullptr;
  const uint32_t* d_rows = nullptr;
  std::vector<int> goff;
  std::shared_ptr<std::vector<uint32_t>> rows, sig;  // host copies (value order, sig per value)
};

}  // namespace

struct qs_circuit {
  Circuit c;
};

// A planned block of one half: schedule, descriptors (host and device).
struct Prepared {
  DevAlloc* da = nullptr;  // owner of dev
  SidePlan sp;
  std::vector<PassDesc> pds;
  std::vector<XPassDesc> xds;  // exchange groups
  std::vector<int> xidx;       // per pass: its group's index in xds (first pass only), or -1
  TailDesc td{};
  char* dev = nullptr;  // descriptors, tail desc, ops, node copy indices (owned)
  size_t o_pd = 0, o_td = 0, o_ops = 0, o_nk = 0, o_lk = 0, o_sv = 0, o_tl = 0, o_xd = 0;
  uint32_t n_list = 0;  // tiles of the last pass that the leaf evaluation reads (0 = all)
  // lower half with end_base: the end-cut bits sig of every requested value,
  // the values sorted by sig (rows) and the group starts (goff); d_rows in the blob
  std::shared_ptr<std::vector<uint32_t>> sig, rows;
  std::vector<int> goff;
  size_t o_rows = 0;
  std::vector<uint64_t> leaf_k;
  std::vector<uint32_t> nu_to_k;  // block-local copy index of each natural position nu
  double pass_bytes = 0;  // algorithmic bytes of the passes
  std::vector<double> pass_bytes_each;  // the same per pass
  // The kernels apply the unit-entry part of every 2x2 gate, and each pass
  // (and the leaf evaluation) multiplies by an exact power of two: the true
  // amplitudes are the computed ones times phi = 2^(-carry/2) omega^A (A the
  // number of sqrt X and sqrt Y gates, carry the odd half power left over).
  double phi_re = 1, phi_im = 0;
  double tail_flops = 0;  // 2x2-gate flops of the leaf evaluation
  ~Prepared() {
    if (dev) da->put(dev);
  }
};

// Per copy block: device table nu_U -> nu_L and the upper half's nu -> copy;
// with lower end cuts folded into the assembly, also their positions in the
// upper half's copy order and the table nu' -> nu0_L.
struct BlockMaps {
  uint32_t* d_perm = nullptr;
  std::shared_ptr<std::vector<uint32_t>> nu_to_k;
  int ne = 0;
  int pos[4] = {0, 0, 0, 0};
  uint32_t* d_colsel = nullptr;
};

struct EvRec {
  int fam;
  int launches;
  hipEvent_t a, b;
};

struct qs_plan {
  Circuit circ;
  uint64_t upper_mask = 0;
  std::vector<Cut> cuts;
  Side side[2];
  qs_options opts{};
  DevAlloc dalloc;
  Pool pool;
  // memory budget of one half's schedule: fixed at the first run, the plan's
  // budget divided by the sides that run at the same time (concurrency)
  size_t side_budget = 0;
  bool budget_set = false;
  int concurrency = 1;
  bool registered = false;
  // qs_plan_reset without keep_bitstrings leaves the registered set here
  // (stale): registering the same set again reuses its tables and block plans
  bool stale = false;
  std::vector<uint64_t> bits;
  std::vector<uint32_t> vals[2];
  std::vector<int> idx[2];
  uint32_t* d_vals[2] = {nullptr, nullptr};
  int* d_idx[2] = {nullptr, nullptr};
  bool list_mode = false;  // bitstrings far from a product set: per-bitstring sums
  bool part_mode = false;  // one part of a chain partition (qs_mplan): side 0 only
  // buffers released by qs_plan_reset wait for the next run to be ordered
  // after their last users (Pool::put_unordered); last_st is the stream of the
  // latest run or assembly
  bool unordered = false;
  hipStream_t last_st = nullptr;
  double phi[2][2] = {{1, 0}, {1, 0}};  // per half: the constant of its unit-entry gates (Prepared)
  std::vector<BlockRes> blocks;
  std::vector<std::pair<uint64_t, uint64_t>> ranges;
  std::map<std::tuple<int, uint64_t, int>, std::unique_ptr<Prepared>> cache;
  // per copy block: device table nu_U -> nu_L and the upper half's nu -> copy
  std::map<std::pair<uint64_t, int>, BlockMaps> perms;
  // the lower half runs on aux, forked from and joined into the caller's stream
  hipStream_t aux = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // qs_run_graph: one captured step and what it was captured for; mem_gen
  // counts every release of device memory the plan holds, so a graph whose
  // buffers may have gone is captured again
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  uint64_t graph_k0 = 0, graph_k1 = 0, graph_gen = 0;
  int graph_prec = -1;
  void* graph_out = nullptr;
  void* graph_sums = nullptr;
  uint64_t mem_gen = 0;
  uint64_t gen() const { return mem_gen + pool.frees; }
  void drop_graph() {
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    if (graph) (void)hipGraphDestroy(graph);
    graph_exec = nullptr;
    graph = nullptr;
  }
  int timing = 0;  // 1: per kernel family; 2: also every full-state pass on its own
  std::vector<EvRec> events;
  struct PassRec {
    int side, pass, level_in, stages, passes;
    uint64_t tiles;
    double bytes;
    hipEvent_t a, b;
  };
  std::vector<PassRec> pass_events;
  std::vector<double> pass_log;  // 8 doubles per timed pass launch (qs_get_pass_timing)
  double tms[4] = {0, 0, 0, 0};
  double counts[4] = {0, 0, 0, 0};
  double pass_bytes = 0, gemm_flops = 0, tail_flops = 0;
  qs_plan() { pool.da = &dalloc; }
  // cached block plans and their copy tables; the caller synchronises first
  void drop_block_plans() {
    ++mem_gen;
    cache.clear();
    for (auto& kv : perms) {
      dalloc.put(kv.second.d_perm);
      dalloc.put(kv.second.d_colsel);
    }
    perms.clear();
  }
  ~qs_plan() {
    (void)hipDeviceSynchronize();
    drop_graph();
    for (EvRec& e : events) {
      (void)hipEventDestroy(e.a);
      (void)hipEventDestroy(e.b);
    }
    for (PassRec& e : pass_events) {
      (void)hipEventDestroy(e.a);
      (void)hipEventDestroy(e.b);
    }
    drop_block_plans();
    pool.release_all();
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (aux) (void)hipStreamDestroy(aux);
  }
};

namespace {

#define HIPCHECK(expr)                                                              \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess) return fail(QS_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

int ctz64(uint64_t x) { return x ? __builtin_ctzll(x) : 64; }

#ifndef QS_PASS_NT_DEFAULT
#define QS_PASS_NT_DEFAULT 1
#endif

// Cached block plans (one per half and copy block) kept at most; the flat
// form plans every copy as a block of its own.
constexpr size_t kMaxCachedSides = 4096;

PlanKnobs knobs_of(qs_plan* p, int S) {
  PlanKnobs k;
  if (p->opts.tile_bits > 0) k.tile_bits = std::min(p->opts.tile_bits, 13);
  if (p->opts.coalesce_bits > 0) k.coalesce_bits = p->opts.coalesce_bits;
  if (p->opts.tail_max_qubits > 0) k.tail_max_qubits = std::min(p->opts.tail_max_qubits, 10);
  k.force_lstar = p->opts.materialize_level;
  if (!p->budget_set) {
    // once per plan, so that the same inputs always give the same schedule
    size_t total = p->opts.mem_budget;
    if (total == 0) {
      size_t fr = 0, tot = 0;
      if (hipMemGetInfo(&fr, &tot) == hipSuccess) total = (size_t)(0.8 * (double)tot);
      else (void)hipGetLastError();
    }
    p->side_budget = total / (size_t)std::max(1, p->concurrency);
    p->budget_set = true;
  }
  k.mem_budget = p->side_budget;
  k.S = S;
  k.one_op_per_pass = p->opts.plain != 0;
  if (p->opts.max_stages > 0) k.max_stages = std::min(p->opts.max_stages, kMaxStages);
  if (p->opts.min_tile_bits > 0) k.min_tile_bits = p->opts.min_tile_bits;
  k.exchange = p->opts.no_exchange == 0;
  return k;
}

// Records a pair of events around a family of launches on the stream; the
// elapsed times are collected by qs_get_timing without blocking the caller.
struct Timer {
  qs_plan* P;
  hipStream_t st;
  int fam;
  int launches = 0;
  hipEvent_t a = nullptr;
  Timer(qs_plan* p, hipStream_t s, int f) : P(p), st(s), fam(f) {
    if (P->timing) {
      (void)hipEventCreate(&a);
      (void)hipEventRecord(a, st);
    }
  }
  ~Timer() {
    if (P->timing) {
      hipEvent_t b = nullptr;
      (void)hipEventCreate(&b);
      (void)hipEventRecord(b, st);
      P->events.push_back(EvRec{fam, launches, a, b});
    }
  }
};

// Plan one half of one block and upload its descriptors (cached per block).
qs_status prepare_side(qs_plan* P, int sidx, const Block& blk, Prepared** out) {
  auto key = std::make_tuple(sidx, blk.k0, blk.p);
  auto it = P->cache.find(key);
  if (it != P->cache.end()) {
    *out = it->second.get();
    P->phi[sidx][0] = (*out)->phi_re;
    P->phi[sidx][1] = (*out)->phi_im;
    return QS_OK;
  }
  const int c = (int)P->cuts.size();
  const int S = (int)P->vals[sidx].size();
  std::unique_ptr<Prepared> pr(new Prepared());
  pr->da = &P->dalloc;
  SidePlan& sp = pr->sp;
  std::string err;
  if (!plan_side(P->side[sidx], c, blk, knobs_of(P, S), sp, err)) return fail(QS_ERR_UNSUPPORTED, err);
  // from here on the half program is the relabelled one: local qubit ids are state bits
  const Side& s = sp.side;
  const Tree& tr = sp.tree;
  const int L = (int)tr.levels.size() - 1;
  if (L - sp.lstar > kMaxTailLevels) return fail(QS_ERR_UNSUPPORTED, "too many leaf levels");
  if ((int)tr.end_cuts.size() > 2 * kMaxBranch) return fail(QS_ERR_UNSUPPORTED, "too many end cuts");
  auto cut_qubit = [&](int j) {
    const Cut& k = P->cuts[j];
    int g = s.upper ? k.upper : k.lower;
    return (int)(std::find(s.qubits.begin(), s.qubits.end(), g) - s.qubits.begin());
  };
  const double SB = std::ldexp(8.0, s.n);
  std::vector<DevOp> ops;
  double last_bytes = 0;
  int carry = 0, n_omega = 0;
  auto mat_counts = [&](const std::vector<int>& lst, int& k, int& w) {
    for (int i : lst)
      if (s.ops[i].kind == OP_MAT) {
        ++k;
        if (s.ops[i].mat == 1 || s.ops[i].mat == 2) ++w;
      }
  };
  for (const PassPlan& pp : sp.passes) {
    PassDesc d{};
    d.wave = s.n >= 7 ? 1 : 0;
    d.n = s.n;
    d.t = (int)pp.tile.size();
    std::vector<int> work_of(s.n, -1);
    for (int i = 0; i < d.t; ++i) {
      d.tbit[i] = pp.tile[i];
      work_of[pp.tile[i]] = i;
    }
    d.n_outer = 0;
    for (int q = 0; q < s.n; ++q)
      if (work_of[q] < 0) d.obit[d.n_outer++] = q;
    d.init = pp.init ? 1 : 0;
    d.hinit = s.hinit;
    d.hamp = (float)std::pow(2.0, -0.5 * __builtin_popcountll(s.hinit));
    std::vector<int> regs;
    if (d.wave)
      for (int i = 6; i < d.t; ++i) regs.push_back(pp.tile[i]);
    const std::vector<int>* rp = d.wave ? &regs : nullptr;
    d.op_in = (int)ops.size();
    if (!encode_ops(s, pp.ops_in, tr.fixed, work_of, ops, err, false, rp))
      return fail(QS_ERR_UNSUPPORTED, err);
    d.n_in = (int)ops.size() - d.op_in;
    d.ns = (int)pp.stages.size();
    if (d.ns > kMaxStages) return fail(QS_ERR_UNSUPPORTED, "internal: too many branch stages");
    for (int st = 0; st < d.ns; ++st) {
      const Level& nx = tr.levels[pp.level_in + 1 + st];
      d.sm[st] = (int)nx.cuts.size();
      for (int i = 0; i < d.sm[st]; ++i) d.sbq[st][i] = cut_qubit(nx.cuts[i]);
      d.sop[st] = (int)ops.size() - d.op_in;
      if (!encode_ops(s, pp.stages[st], tr.fixed, work_of, ops, err, false, rp))
        return fail(QS_ERR_UNSUPPORTED, err);
      d.snops[st] = (int)ops.size() - d.op_in - d.sop[st];
    }
    d.n_all = (int)ops.size() - d.op_in;
    if (d.n_all > kMaxPassOps) return fail(QS_ERR_UNSUPPORTED, "internal: too many ops in a pass");
    const double nin = (double)sp.nodes[pp.level_in];
    if (pp.branch())
      last_bytes = (pp.init ? 0.0 : nin * SB) + (double)sp.nodes[pp.level_out()] * SB;
    else if (pp.xg == 0)
      last_bytes = 0;  // a later phase of an exchange group: its traffic is the group's
    else
      last_bytes = (pp.init ? 1.0 : 2.0) * nin * SB;
    pr->pass_bytes += last_bytes;
    pr->pass_bytes_each.push_back(last_bytes);
    d.upper = s.upper ? 1 : 0;
    d.nt = QS_PASS_NT_DEFAULT;
    {
      int k = 0;
      mat_counts(pp.ops_in, k, n_omega);
      for (const std::vector<int>& so : pp.stages) mat_counts(so, k, n_omega);
      d.scale = std::ldexp(1.0f, -((k + carry) >> 1));
      carry = (k + carry) & 1;
    }
    pr->pds.push_back(d);
  }
  // exchange groups: one descriptor per group, at the group's first pass
  pr->xidx.assign(sp.passes.size(), -1);
  for (size_t pi = 0; pi < sp.passes.size(); ++pi) {
    const PassPlan& pp = sp.passes[pi];
    if (pp.xg < 2) continue;
    XPassDesc x{};
    x.G = pp.xg;
    x.pd0 = (int)pi;
    x.R = (int)pp.tile.size() - 6;
    x.n = s.n;
    x.nu = (int)pp.xu.size();
    if (x.G > kMaxXPhases || pi + x.G > sp.passes.size() || x.nu != x.R + kXWaveBits ||
        x.R < kXMinRegBits || x.R > kMaxRegBits || 6 + x.nu > s.n)
      return fail(QS_ERR_UNSUPPORTED, "internal: exchange group shape");
    std::vector<int> inu(s.n, -1);
    for (int i = 0; i < x.nu; ++i) {
      x.ubit[i] = pp.xu[i];
      if (pp.xu[i] < 6 || pp.xu[i] >= s.n) return fail(QS_ERR_UNSUPPORTED, "internal: exchange bits");
      inu[pp.xu[i]] = i;
    }
    x.n_outer = 0;
    for (int q = 6; q < s.n; ++q)
      if (inu[q] < 0) x.obit[x.n_outer++] = q;
    for (int p = 0; p < x.G; ++p) {
      const PassPlan& ph = sp.passes[pi + p];
      if ((int)ph.tile.size() != 6 + x.R || ph.branch() || (p > 0 && ph.xg != 0))
        return fail(QS_ERR_UNSUPPORTED, "internal: exchange group phase");
      std::vector<char> isreg(x.nu, 0);
      for (int k = 0; k < x.R; ++k) {
        const int q = ph.tile[6 + k];
        if (q < 0 || q >= s.n || inu[q] < 0) return fail(QS_ERR_UNSUPPORTED, "internal: exchange register bit");
        x.rpos[p][k] = inu[q];
        isreg[inu[q]] = 1;
      }
      int j = 0;
      for (int i = 0; i < x.nu; ++i)
        if (!isreg[i]) {
          if (j == kXWaveBits) return fail(QS_ERR_UNSUPPORTED, "internal: exchange wave bits");
          x.wpos[p][j++] = i;
        }
      if (j != kXWaveBits) return fail(QS_ERR_UNSUPPORTED, "internal: exchange wave bits");
    }
    x.init = pp.init ? 1 : 0;
    x.nt = pr->pds[pi + x.G - 1].nt;
    pr->xidx[pi] = (int)pr->xds.size();
    pr->xds.push_back(x);
  }
  TailDesc& td = pr->td;
  td.n = s.n;
  td.q = (int)sp.Q.size();
  std::vector<int> work_q(s.n, -1);
  for (int i = 0; i < td.q; ++i) {
    td.Q[i] = sp.perm[sp.Q[i]];  // = i: the light cone is on the lowest state bits
    work_q[sp.perm[sp.Q[i]]] = i;
  }
  td.nlev = L - sp.lstar;
  td.M = 0;
  for (int l = sp.lstar + 1; l <= L; ++l) td.M += (int)tr.levels[l].cuts.size();
  std::vector<DevOp> tops;
  {
    // the backward rows keep light-cone bits lg..q-1 in registers (lg = min(q, 6)
    // bits across the lanes of a group): the register split of their DIAG ops
    std::vector<int> tail_regs;
    for (int i = std::min(td.q, 6); i < td.q; ++i) tail_regs.push_back(td.Q[i]);
    int shift = td.M;
    for (int l = sp.lstar + 1; l <= L; ++l) {
      TailLevel& tl = td.lev[l - sp.lstar - 1];
      const Level& lv = tr.levels[l];
      tl.m = (int)lv.cuts.size();
      shift -= tl.m;
      tl.shift = shift;
      for (int i = 0; i < tl.m; ++i) {
        tl.bq[i] = cut_qubit(lv.cuts[i]);
        tl.kbit[i] = 1ULL << (c - 1 - lv.cuts[i]);
      }
      std::vector<int> rev(lv.ops.rbegin(), lv.ops.rend());
      tl.bop0 = (int)(ops.size() + tops.size());
      size_t before = tops.size();
      if (!encode_ops(s, rev, tr.fixed, work_q, tops, err, true, &tail_regs))
        return fail(QS_ERR_UNSUPPORTED, err);
      tl.bnops = (int)(tops.size() - before);
      tl.code = 0;
      if (tl.bnops <= 8)
        for (int o = 0; o < tl.bnops; ++o) {
          const DevOp& op = tops[before + o];
          const uint64_t b = op.kind == 1 ? 0x80u : (uint64_t)((op.mk & 7) << 3 | (op.target & 7));
          tl.code |= b << (8 * o);
        }
    }
  }
  {
    int acc = 0;
    for (int l = 0; l < td.nlev; ++l) {
      td.lev[l].pos = acc;
      acc += td.lev[l].m;
    }
  }
  td.n_nodes = (int)sp.nodes[sp.lstar];
  td.fused = tail_fused_ok(td) ? 1 : 0;
  td.ws = td.fused && tail_ws_ok(td) ? 1 : 0;
  // copy-index contribution of each leaf path below the materialised level,
  // indexed the way the leaf evaluation writes its output (lam, the emission
  // index of the fused kernel, or its field-swapped form of the specialised one)
  pr->leaf_k.assign((size_t)1 << td.M, 0);
  for (size_t lam = 0; lam < pr->leaf_k.size(); ++lam) {
    uint64_t k = 0;
    for (int l = 0; l < td.nlev; ++l) {
      const TailLevel& tl = td.lev[l];
      const int at = td.fused ? tl.pos : tl.shift;
      for (int i = 0; i < tl.m; ++i) {
        const int b = at + tl.m - 1 - i;
        if ((lam >> (td.ws ? tail_ws_bit(b, td.M) : b)) & 1) k |= tl.kbit[i];
      }
    }
    pr->leaf_k[lam] = k;
  }
  {
    // algorithmic flops: the per-value GEMM (8 per complex multiply-add) and
    // the backward rows (14 per amplitude per 2x2 gate)
    const double K = std::ldexp(1.0, td.q);
    pr->tail_flops = 8.0 * std::ldexp(1.0, td.M) * K * (double)sp.nodes[sp.lstar] * S;
    double paths = 1;
    for (int l = L; l > sp.lstar; --l) {
      double nmat = 0;
      for (int i : tr.levels[l].ops) nmat += s.ops[i].kind == OP_MAT ? 1 : 0;
      pr->tail_flops += (double)S * paths * 14.0 * nmat * K;
      paths *= std::ldexp(1.0, (int)tr.levels[l].cuts.size());
    }
  }
  {
    int k = 0;
    for (int l = sp.lstar + 1; l <= L; ++l) mat_counts(tr.levels[l].ops, k, n_omega);
    td.tscale = std::ldexp(1.0f, -((k + carry) >> 1));
    carry = (k + carry) & 1;
    const double mag = carry ? std::sqrt(0.5) : 1.0;
    const double ang = (n_omega & 7) * (M_PI / 4.0);
    pr->phi_re = mag * std::cos(ang);
    pr->phi_im = mag * std::sin(ang);
    P->phi[sidx][0] = pr->phi_re;
    P->phi[sidx][1] = pr->phi_im;
  }
  td.n_end = (int)tr.end_cuts.size();
  for (int i = 0; i < td.n_end; ++i) {
    td.eq[i] = cut_qubit(tr.end_cuts[i]);
    td.ekbit[i] = 1ULL << (c - 1 - tr.end_cuts[i]);
  }
  // spread each value's backward rows over up to 8 wavefronts (the first
  // reverse levels' branches) so that a launch has several waves per SIMD
  td.split_levels = 0;
  td.split_bits = 0;
  while (td.split_levels < td.nlev) {
    const int m = td.lev[td.nlev - 1 - td.split_levels].m;
    if (td.split_bits + m > 3) break;
    td.split_bits += m;
    ++td.split_levels;
  }
  td.upper = s.upper ? 1 : 0;
  td.S = S;
  td.ldx = 1 << (c - blk.p);  // row stride of X[s][nu]: the block's copies
  // lower half, product-set assembly: write only the copies with end bits 0
  // (the assembly folds the end cuts' signs into the upper operand)
  td.end_base = (!s.upper && !P->list_mode && !P->opts.plain && !P->part_mode && td.n_end >= 1 &&
                 td.n_end <= 4 &&
                 (td.ldx >> td.n_end) >= 1)
                    ? 1
                    : 0;
  if (td.end_base) td.ldx >>= td.n_end;
  ops.insert(ops.end(), tops.begin(), tops.end());
  // copy-index contribution of each materialised node
  std::vector<int> ncuts;
  for (int l = 1; l <= sp.lstar; ++l)
    for (int j : tr.levels[l].cuts) ncuts.push_back(j);
  std::vector<uint64_t> node_k(sp.nodes[sp.lstar], 0);
  const int nb = (int)ncuts.size();
  for (uint64_t r = 0; r < node_k.size(); ++r) {
    uint64_t k = 0;
    for (int i = 0; i < nb; ++i)
      if ((r >> (nb - 1 - i)) & 1) k |= 1ULL << (c - 1 - ncuts[i]);
    node_k[r] = k;
  }
  {
    // natural order nu = ((node << M) + lam) << n_end | end bits
    const size_t Kb = (size_t)1 << (c - blk.p);
    const int ne = td.n_end;
    pr->nu_to_k.assign(Kb, 0);
    for (size_t r = 0; r < node_k.size(); ++r)
      for (size_t lam = 0; lam < pr->leaf_k.size(); ++lam)
        for (int e = 0; e < (1 << ne); ++e) {
          uint64_t k = node_k[r] | pr->leaf_k[lam];
          for (int i = 0; i < ne; ++i)
            if ((e >> (ne - 1 - i)) & 1) k |= td.ekbit[i];
          const size_t nu = (((r << td.M) + lam) << ne) | (size_t)e;
          if (nu < Kb) pr->nu_to_k[nu] = (uint32_t)k;
        }
  }
  const size_t b_pd = pr->pds.size() * sizeof(PassDesc);
  const size_t b_td = sizeof(TailDesc);
  const size_t b_ops = std::max<size_t>(1, ops.size()) * sizeof(DevOp);
  const size_t b_nk = node_k.size() * sizeof(uint64_t);
  const size_t b_lk = pr->leaf_k.size() * sizeof(uint64_t);
  // requested half values in the relabelled bit order
  std::vector<uint32_t> sv(S);
  for (int i = 0; i < S; ++i) {
    const uint32_t v = P->vals[sidx][i];
    uint32_t w = 0;
    for (int qq = 0; qq < s.n; ++qq)
      if ((v >> qq) & 1) w |= 1u << sp.perm[qq];
    sv[i] = w;
  }
  const size_t b_sv = (size_t)S * sizeof(uint32_t);
  std::vector<uint32_t> rows_v;
  if (td.end_base) {
    auto sig = std::make_shared<std::vector<uint32_t>>(S);
    for (int i = 0; i < S; ++i) {
      uint32_t g = 0;
      for (int e = 0; e < td.n_end; ++e) g |= ((sv[i] >> td.eq[e]) & 1u) << e;
      (*sig)[i] = g;
    }
    rows_v.resize(S);
    for (int i = 0; i < S; ++i) rows_v[i] = (uint32_t)i;
    std::stable_sort(rows_v.begin(), rows_v.end(),
                     [&](uint32_t a, uint32_t b) { return (*sig)[a] < (*sig)[b]; });
    pr->goff.assign((1 << td.n_end) + 1, 0);
    for (int i = 0; i < S; ++i) ++pr->goff[(*sig)[i] + 1];
    for (int g = 0; g < (1 << td.n_end); ++g) pr->goff[g + 1] += pr->goff[g];
    pr->sig = sig;
    pr->rows = std::make_shared<std::vector<uint32_t>>(rows_v);
  }
  if (td.end_base)
    for (int g : pr->goff) rows_v.push_back((uint32_t)g);  // the group starts follow the rows
  const size_t b_rows = rows_v.size() * sizeof(uint32_t);
  // The leaf evaluation reads the last materialised states only at the
  // requested values with their light-cone bits free, so the last pass need
  // only produce the tiles whose outer bits agree with some requested value
  // (outer bits inside the light cone take both values).
  std::vector<uint32_t> tl;
  if (!P->opts.plain && !pr->pds.empty() && pr->pds.back().wave) {
    const PassDesc& d = pr->pds.back();
    uint32_t qmask = 0;
    for (int i = 0; i < td.q; ++i) qmask |= 1u << td.Q[i];
    std::vector<int> fixed_j, free_j;
    for (int j = 0; j < d.n_outer; ++j) ((qmask >> d.obit[j]) & 1 ? free_j : fixed_j).push_back(j);
    const int nf = (int)free_j.size();
    if (d.n_outer > 0 && nf <= 6) {
      tl.reserve((size_t)S << nf);
      for (int i = 0; i < S; ++i) {
        uint32_t t0 = 0;
        for (int j : fixed_j) t0 |= ((sv[i] >> d.obit[j]) & 1u) << j;
        for (int f = 0; f < (1 << nf); ++f) {
          uint32_t t = t0;
          for (int b = 0; b < nf; ++b) t |= (uint32_t)((f >> b) & 1) << free_j[b];
          tl.push_back(t);
        }
      }
      std::sort(tl.begin(), tl.end());
      tl.erase(std::unique(tl.begin(), tl.end()), tl.end());
      const double frac = (double)tl.size() / std::ldexp(1.0, d.n_outer);
      if (frac > 0.75) {
        tl.clear();
      } else {
        pr->pass_bytes -= last_bytes * (1.0 - frac);
        pr->pass_bytes_each.back() *= frac;
      }
    }
  }
  pr->n_list = (uint32_t)tl.size();
  const size_t b_tl = tl.size() * sizeof(uint32_t);
  const size_t b_xd = pr->xds.size() * sizeof(XPassDesc);
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t total = al(b_pd) + al(b_td) + al(b_ops) + al(b_nk) + al(b_lk) + al(b_sv) +
                       al(b_tl) + al(b_rows) + al(b_xd);
  std::vector<char> host(total, 0);
  pr->o_pd = 0;
  pr->o_td = al(b_pd);
  pr->o_ops = pr->o_td + al(b_td);
  pr->o_nk = pr->o_ops + al(b_ops);
  pr->o_lk = pr->o_nk + al(b_nk);
  pr->o_sv = pr->o_lk + al(b_lk);
  pr->o_tl = pr->o_sv + al(b_sv);
  pr->o_rows = pr->o_tl + al(b_tl);
  pr->o_xd = pr->o_rows + al(b_rows);
  if (b_pd) std::memcpy(host.data() + pr->o_pd, pr->pds.data(), b_pd);
  std::memcpy(host.data() + pr->o_td, &td, b_td);
  if (!ops.empty()) std::memcpy(host.data() + pr->o_ops, ops.data(), ops.size() * sizeof(DevOp));
  std::memcpy(host.data() + pr->o_nk, node_k.data(), b_nk);
  std::memcpy(host.data() + pr->o_lk, pr->leaf_k.data(), b_lk);
  std::memcpy(host.data() + pr->o_sv, sv.data(), b_sv);
  if (b_tl) std::memcpy(host.data() + pr->o_tl, tl.data(), b_tl);
  if (b_rows) std::memcpy(host.data() + pr->o_rows, rows_v.data(), b_rows);
  if (b_xd) std::memcpy(host.data() + pr->o_xd, pr->xds.data(), b_xd);
  pr->dev = (char*)P->dalloc.get(total);
  if (!pr->dev) return fail(QS_ERR_OOM, "descriptor buffer");
  HIPCHECK(hipMemcpy(pr->dev, host.data(), total, hipMemcpyHostToDevice));
  *out = pr.get();
  P->cache[key] = std::move(pr);
  return QS_OK;
}

// Run one half of one block: passes for the materialised levels, then the
// leaf evaluation into X[k][s].  Asynchronous on st.
qs_status run_side(qs_plan* P, int sidx, const Prepared& pr, float2* X, hipStream_t st) {
  const Side& s = P->side[sidx];
  const SidePlan& sp = pr.sp;
  const size_t SB = (size_t)8 << s.n;
  float2* cur = nullptr;
  uint64_t cur_nodes = 0;
  const DevOp* d_ops = (const DevOp*)(pr.dev + pr.o_ops);
  {
    Timer tm(P, st, 0);
    for (size_t pi = 0; pi < sp.passes.size(); ++pi) {
      const PassPlan& pp = sp.passes[pi];
      if (pp.xg == 0) continue;  // a later phase of the exchange group launched before
      const PassDesc* dd = (const PassDesc*)(pr.dev + pr.o_pd) + pi;
      const bool last = pi + 1 == sp.passes.size() && pr.n_list > 0;
      const uint32_t* tl = last ? (const uint32_t*)(pr.dev + pr.o_tl) : nullptr;
      const uint32_t nl = last ? pr.n_list : 0;
      if (pp.init) {
        cur_nodes = 1;
        cur = (float2*)P->pool.get(SB, st);
        if (!cur) return fail(QS_ERR_OOM, "root state");
      }
      hipEvent_t ea = nullptr;
      if (P->timing >= 2) {
        HIPCHECK(hipEventCreate(&ea));
        HIPCHECK(hipEventRecord(ea, st));
      }
      if (pp.xg >= 2) {
        const int xi = pr.xidx[pi];
        if (xi < 0) return fail(QS_ERR_UNSUPPORTED, "internal: exchange group descriptor");
        HIPCHECK(launch_xpass(pr.xds[xi], (const XPassDesc*)(pr.dev + pr.o_xd) + xi,
                              (const PassDesc*)(pr.dev + pr.o_pd), d_ops, cur, cur_nodes, st));
      } else if (pp.branch()) {
        const uint64_t on = sp.nodes[pp.level_out()];
        float2* nxt = (float2*)P->pool.get(SB * on, st);
        if (!nxt) return fail(QS_ERR_OOM, "tree level states");
        HIPCHECK(launch_pass(pr.pds[pi], dd, d_ops, cur, nxt, cur_nodes, tl, nl, st));
        P->pool.put(cur, st);
        cur = nxt;
        cur_nodes = on;
      } else {
        HIPCHECK(launch_pass(pr.pds[pi], dd, d_ops, cur, cur, cur_nodes, tl, nl, st));
      }
      if (P->timing >= 2) {
        hipEvent_t eb = nullptr;
        HIPCHECK(hipEventCreate(&eb));
        HIPCHECK(hipEventRecord(eb, st));
        const PassDesc& h = pr.pds[pi];
        const uint64_t nin = pp.init ? 1 : sp.nodes[pp.level_in];
        const uint64_t tiles = tl ? nin * nl : (nin << h.n_outer);
        P->pass_events.push_back(qs_plan::PassRec{sidx, (int)pi, pp.level_in, (int)pp.stages.size(),
                                                  std::max(1, pp.xg),
                                                  tiles, pr.pass_bytes_each[pi], ea, eb});
      }
      ++tm.launches;
    }
    if (P->timing) P->pass_bytes += pr.pass_bytes;
  }
  {
    Timer tm(P, st, 1);
    const int S = (int)P->vals[sidx].size();
    const size_t per_s = tail_w_bytes(pr.td, 1);
    int chunk = pr.td.fused ? S : (int)std::max<size_t>(1, ((size_t)512 << 20) / per_s);
    chunk = std::min({chunk, S, 65535});
    float2* W = nullptr;  // the fused leaf evaluation keeps its rows on chip
    if (!pr.td.fused) {
      W = (float2*)P->pool.get(per_s * chunk, st);
      if (!W) return fail(QS_ERR_OOM, "leaf rows");
    }
    for (int s0 = 0; s0 < S; s0 += chunk) {
      const int ns = std::min(chunk, S - s0);
      HIPCHECK(launch_tail(pr.td, (const TailDesc*)(pr.dev + pr.o_td), d_ops, cur,
                           (const uint32_t*)(pr.dev + pr.o_sv), s0, ns, W, X, st));
      tm.launches += pr.td.fused ? 1 : 2;
    }
    if (W) P->pool.put(W, st);
    if (P->timing) P->tail_flops += pr.tail_flops;
  }
  // later users of these buffers are ordered after the kernels above by the stream
  P->pool.put(cur, st);
  return QS_OK;
}

qs_status register_bits(qs_plan* P, const uint64_t* bits, size_t m) {
  const int n = P->circ.n;
  const uint64_t full = n == 64 ? ~0ULL : ((1ULL << n) - 1);
  if (P->registered) {
    if (bits == nullptr && m == 0) return QS_OK;
    if (!bits || m != P->bits.size() || std::memcmp(bits, P->bits.data(), m * 8) != 0)
      return fail(QS_ERR_STATE, "bitstrings differ from the registered set");
    return QS_OK;
  }
  if (!bits || m == 0) return fail(QS_ERR_ARG, "no bitstrings registered yet");
  if (P->stale) {
    if (m == P->bits.size() && std::memcmp(bits, P->bits.data(), m * 8) == 0) {
      // the set registered before the last reset: its value tables and
      // cached block plans still hold
      P->stale = false;
      P->registered = true;
      return QS_OK;
    }
    for (int k = 0; k < 2; ++k) {
      if (P->d_vals[k]) P->pool.put_unordered(P->d_vals[k]);
      if (P->d_idx[k]) P->pool.put_unordered(P->d_idx[k]);
      P->d_vals[k] = nullptr;
      P->d_idx[k] = nullptr;
    }
    ++P->mem_gen;  // a captured step read the old tables
    P->stale = false;
  }
  for (size_t t = 0; t < m; ++t)
    if (bits[t] & ~full) return fail(QS_ERR_ARG, "bitstring has bits set beyond the qubit count");
  std::vector<uint32_t> vals[2];
  std::vector<int> idx[2];
  for (int sidx = 0; sidx < 2; ++sidx) {
    const Side& s = P->side[sidx];
    std::vector<uint32_t> hv(m);
    for (size_t t = 0; t < m; ++t) {
      uint32_t v = 0;
      for (int i = 0; i < s.n; ++i) v |= (uint32_t)((bits[t] >> s.qubits[i]) & 1) << i;
      hv[t] = v;
    }
    std::vector<uint32_t> u = hv;
    std::sort(u.begin(), u.end());
    u.erase(std::unique(u.begin(), u.end()), u.end());
    idx[sidx].resize(m);
    for (size_t t = 0; t < m; ++t)
      idx[sidx][t] = (int)(std::lower_bound(u.begin(), u.end(), hv[t]) - u.begin());
    vals[sidx] = std::move(u);
  }
  const double prod = (double)vals[0].size() * (double)vals[1].size();
  P->list_mode = prod > 4.0 * (double)m + 1024.0;
  // every queued kernel is done before buffers change hands here
  (void)hipDeviceSynchronize();
  P->pool.settle();
  for (int sidx = 0; sidx < 2; ++sidx) {
    const size_t bytes = vals[sidx].size() * sizeof(uint32_t);
    uint32_t* dv = (uint32_t*)P->pool.get(bytes, nullptr);
    int* di = (int*)P->pool.get(m * sizeof(int), nullptr);
    if (!dv || !di) return fail(QS_ERR_OOM, "value tables");
    HIPCHECK(hipMemcpy(dv, vals[sidx].data(), bytes, hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(di, idx[sidx].data(), m * sizeof(int), hipMemcpyHostToDevice));
    P->d_vals[sidx] = dv;
    P->d_idx[sidx] = di;
    P->vals[sidx] = std::move(vals[sidx]);
    P->idx[sidx] = std::move(idx[sidx]);
  }
  P->bits.assign(bits, bits + m);
  // a new value set changes the leaf evaluation (and, through the cost model,
  // possibly the trees): drop cached block plans and copy tables
  (void)hipDeviceSynchronize();
  P->drop_block_plans();
  P->registered = true;
  return QS_OK;
}

// Assembly of every run block into C, then the amplitudes of the registered
// bitstrings into d_amps and their FP64 sums into d_sums.  Asynchronous.
// The product of the two halves' constants (see Prepared::phi).
float2 phi_of(const qs_plan* plan) {
  const double a = plan->phi[0][0], b = plan->phi[0][1], c = plan->phi[1][0], d = plan->phi[1][1];
  return make_float2((float)(a * c - b * d), (float)(a * d + b * c));
}

// Temporary device buffers of one assembly: from the plan's pool, or (static
// form) carved in call order from a caller-given region.  Every request is
// 256-byte aligned; release() returns the region to a mark (the stream orders
// the next user after the previous one).
struct Scratch {
  qs_plan* P;
  hipStream_t st;
  char* base = nullptr;  // static region (nullptr: the pool)
  size_t cap = 0, used = 0;
  bool measure = false;  // only add up the bytes the requests need
  void* get(size_t bytes) {
    if (!base && !measure) return P->pool.get(bytes, st);
    const size_t off = (used + 255) & ~(size_t)255;
    if (!measure && off + bytes > cap) return nullptr;
    used = off + bytes;
    return measure ? (void*)(uintptr_t)256 : (void*)(base + off);  // measure: never dereferenced
  }
  void put(void* p) {
    if (!base && !measure) P->pool.put(p, st);
  }
  size_t mark() const { return used; }
  void release(size_t m) {
    if (base || measure) used = m;
  }
};

// Assembly of every run block into C, then the amplitudes of the registered
// bitstrings into d_amps and their FP64 sums into d_sums.  Asynchronous.
// sc.measure: no launch, only the scratch bytes (sc.used afterwards).
qs_status assemble(qs_plan* plan, qs_precision prec, float2* d_amps, double* d_sums, Scratch& sc) {
  hipStream_t st = sc.st;
  const bool run = !sc.measure;
  if (run) plan->last_st = st;
  const int M = (int)plan->vals[0].size(), N = (int)plan->vals[1].size();
  const size_t m = plan->bits.size();
  const int nb = prob_partial_blocks(m);
  double* d_part = (double*)sc.get((2 * (size_t)nb + 2) * sizeof(double));
  if (!d_part) return fail(QS_ERR_OOM, "assembly buffers");
  bool sums_done = false;  // the product path gathers and sums in one kernel
  if (plan->list_mode) {
    // the bitstrings are far from a product set: one sum over the copies per
    // bitstring (FP32 accumulation for either precision)
    if (run) {
      Timer tm(plan, st, 2);
      bool first = true;
      for (BlockRes& b : plan->blocks) {
        const int K = (int)(b.k1 - b.k0);
        HIPCHECK(launch_gathered_dot(K, b.X[0], K, b.X[1], K, plan->d_idx[0], plan->d_idx[1], m,
                                     d_amps, first ? 0 : 1, phi_of(plan), st));
        ++tm.launches;
        if (plan->timing) plan->gemm_flops += 8.0 * (double)m * (double)K;
        first = false;
      }
    }
  } else {
    float2* C = (float2*)sc.get((size_t)M * N * sizeof(float2));
    if (!C) return fail(QS_ERR_OOM, "assembly buffers");
    {
      std::unique_ptr<Timer> tm(run ? new Timer(plan, st, 2) : nullptr);
      bool first = true;
      for (BlockRes& b : plan->blocks) {
        const int K = (int)(b.k1 - b.k0);
        const size_t mk = sc.mark();
        if (b.ne > 0) {
          // one product per end-cut pattern sig over K >> ne copies (the
          // transformed upper operand for sig against the lower values with
          // that pattern, scattered to their columns of C), all in one
          // launch; split-BF16 splits both operands once for all patterns
          const int K0 = K >> b.ne, ng = 1 << b.ne;
          int maxn = 1;
          for (int g = 0; g < ng; ++g) maxn = std::max(maxn, b.goff[g + 1] - b.goff[g]);
          const bool f32 = prec == QS_PREC_FP32;
          const size_t wb = f32 ? zgemm_grouped_workspace_bytes(M, N, maxn, K0, ng)
                                : zgemm_grouped_bf16_workspace_bytes(M, N, maxn, K0, ng);
          void* work = sc.get(wb);
          if (!work) return fail(QS_ERR_OOM, "assembly workspace");
          if (run) {
            if (f32)
              HIPCHECK(launch_zgemm_grouped(M, N, maxn, K0, ng, (const int*)(b.d_rows + N), b.Ut,
                                            (size_t)M * K0, b.X[1], C, N, first ? 0 : 1, work, st,
                                            b.d_rows));
            else
              HIPCHECK(launch_zgemm_grouped_bf16(M, N, maxn, K0, ng, (const int*)(b.d_rows + N),
                                                 b.Ut, b.X[1], C, N, first ? 0 : 1, work, st,
                                                 b.d_rows));
            tm->launches += f32 ? 2 : 4;
            if (plan->timing) plan->gemm_flops += 8.0 * M * N * (double)K0;
          }
          sc.put(work);
        } else {
          const size_t wb = zgemm_workspace_bytes((int)prec, M, N, K);
          void* work = sc.get(wb);
          if (!work) return fail(QS_ERR_OOM, "assembly workspace");
          if (run) {
            HIPCHECK(launch_zgemm_tn((int)prec, M, N, K, b.X[0], K, b.X[1], K, C, N,
                                     first ? 0 : 1, work, st));
            tm->launches += prec == QS_PREC_FP32 ? 2 : 4;
            if (plan->timing) plan->gemm_flops += 8.0 * M * N * (double)K;
          }
          sc.put(work);
        }
        sc.release(mk);  // the next block's workspace reuses this one's
        first = false;
      }
    }
    if (run) {
      Timer tm(plan, st, 3);
      HIPCHECK(launch_gather_prob_sums(C, N, plan->d_idx[0], plan->d_idx[1], m, d_amps,
                                       phi_of(plan), d_part, d_sums ? d_sums : d_part + 2 * nb,
                                       st));
      tm.launches += 2;
    }
    sums_done = true;
    sc.put(C);
  }
  if (run && !sums_done) {
    Timer tm(plan, st, 3);
    HIPCHECK(launch_prob_sums(d_amps, m, d_part, d_sums ? d_sums : d_part + 2 * nb, st));
    tm.launches += 2;
  }
  sc.put(d_part);
  return QS_OK;
}

PlanKnobs dump_knobs(const qs_plan* plan, int k) {
  PlanKnobs kn;
  if (plan->opts.tile_bits > 0) kn.tile_bits = std::min(plan->opts.tile_bits, 13);
  if (plan->opts.coalesce_bits > 0) kn.coalesce_bits = plan->opts.coalesce_bits;
  if (plan->opts.tail_max_qubits > 0) kn.tail_max_qubits = std::min(plan->opts.tail_max_qubits, 10);
  kn.force_lstar = plan->opts.materialize_level;
  kn.mem_budget = plan->opts.mem_budget;
  kn.S = plan->registered ? (int)plan->vals[k].size() : 1024;
  kn.one_op_per_pass = plan->opts.plain != 0;
  if (plan->opts.max_stages > 0) kn.max_stages = std::min(plan->opts.max_stages, kMaxStages);
  if (plan->opts.min_tile_bits > 0) kn.min_tile_bits = plan->opts.min_tile_bits;
  kn.exchange = plan->opts.no_exchange == 0;
  return kn;
}

}  // namespace

extern "C" {

const char* qs_last_error(void) { return g_err.c_str(); }

qs_status qs_load_circuit(const char* text, size_t len, qs_circuit** out) {
  if (!text || !out) return fail(QS_ERR_ARG, "null pointer");
  auto* c = new (std::nothrow) qs_circuit();
  if (!c) return fail(QS_ERR_OOM, "host allocation");
  std::string err;
  if (!parse_circuit(text, len, c->c, err)) {
    delete c;
    return fail(QS_ERR_PARSE, err);
  }
  *out = c;
  return QS_OK;
}

qs_status qs_circuit_info(const qs_circuit* circ, int* n_qubits, int* n_gates) {
  if (!circ) return fail(QS_ERR_ARG, "null circuit");
  if (n_qubits) *n_qubits = circ->c.n;
  if (n_gates) {
    int k = 0;
    for (const Gate& g : circ->c.gates) k += g.aux ? 0 : 1;
    *n_gates = k;
  }
  return QS_OK;
}

void qs_circuit_free(qs_circuit* circ) { delete circ; }

qs_status qs_partition(const qs_circuit* circ, uint64_t upper_mask, const qs_options* opts,
                       qs_plan** out) {
  if (!circ || !out) return fail(QS_ERR_ARG, "null pointer");
  std::unique_ptr<qs_plan> p(new (std::nothrow) qs_plan());
  if (!p) return fail(QS_ERR_OOM, "host allocation");
  p->circ = circ->c;
  p->upper_mask = upper_mask;
  if (opts) p->opts = *opts;
  else {
    p->opts = qs_options{};
    p->opts.materialize_level = -1;
  }
  if (p->opts.tile_bits < 0 || p->opts.coalesce_bits < 0 || p->opts.tail_max_qubits < 0 ||
      p->opts.max_stages < 0 || p->opts.min_tile_bits < 0 || p->opts.no_exchange < 0)
    return fail(QS_ERR_ARG, "negative option");
  if ((p->opts.alloc.alloc == nullptr) != (p->opts.alloc.free == nullptr))
    return fail(QS_ERR_ARG, "allocator needs both alloc and free");
  if (p->opts.copies_per_launch & (p->opts.copies_per_launch - 1))
    return fail(QS_ERR_ARG, "copies_per_launch must be a power of two");
  p->dalloc.a = p->opts.alloc;
  p->concurrency = (p->opts.one_stream || p->opts.plain) ? 1 : 2;
  std::string err;
  if (!build_partition(p->circ, upper_mask, p->cuts, p->side[0], p->side[1], err))
    return fail(QS_ERR_ARG, err);
  if (p->side[0].n > 32 || p->side[1].n > 32) return fail(QS_ERR_ARG, "a half has more than 32 qubits");
  if (p->cuts.size() > 40) return fail(QS_ERR_UNSUPPORTED, "more than 40 cut gates");
  *out = p.release();
  return QS_OK;
}

namespace {

qs_status score_cut(const Circuit& circ, uint64_t upper_mask, int n_values, qs_cut_score& sc) {
  std::vector<Cut> cuts;
  Side up, lo;
  std::string err;
  if (!build_partition(circ, upper_mask, cuts, up, lo, err)) return fail(QS_ERR_ARG, err);
  if (up.n > 32 || lo.n > 32) return fail(QS_ERR_ARG, "a half has more than 32 qubits");
  const int c = (int)cuts.size();
  if (c > 40) return fail(QS_ERR_UNSUPPORTED, "more than 40 cut gates");
  // written gates touching each half (a cut two-qubit gate touches both)
  double g[2] = {0, 0};
  for (const Gate& gt : circ.gates) {
    if (gt.aux) continue;
    const bool u0 = (upper_mask >> gt.q0) & 1;
    g[u0 ? 0 : 1] += 1;
    if (gt.q1 >= 0) {
      const bool u1 = (upper_mask >> gt.q1) & 1;
      if (u1 != u0) g[u1 ? 0 : 1] += 1;
    }
  }
  sc.n_cuts = c;
  sc.n_upper = up.n;
  sc.n_lower = lo.n;
  sc.equivalent_qubits = std::max(up.n, lo.n) + c + 1;
  sc.flat_updates = std::ldexp(g[0], c + up.n) + std::ldexp(g[1], c + lo.n);
  PlanKnobs kn;
  kn.S = n_values;
  Block blk;
  double cost = 0;
  int ne_lower = 0;
  for (const Side* sd : {&up, &lo}) {
    SidePlan sp;
    if (!plan_side(*sd, c, blk, kn, sp, err)) return fail(QS_ERR_UNSUPPORTED, err);
    cost += sp.cost_bytes;
    if (!sd->upper) ne_lower = std::min(4, (int)sp.tree.end_cuts.size());
  }
  // assembly over n_values x n_values values: three real products per complex
  // one over 2^c copies (2^(c - ne) with the lower end cuts folded), priced
  // at the FP32 MFMA rate in HBM byte-equivalents (8 TB/s against 157.3 TFLOP/s)
  const double flops = 6.0 * (double)n_values * (double)n_values * std::ldexp(1.0, c - ne_lower);
  cost += flops * (8.0 / 157.3);
  sc.plan_cost = cost;
  return QS_OK;
}

}  // namespace

qs_status qs_score_cut(const qs_circuit* circ, uint64_t upper_mask, int n_values,
                       qs_cut_score* out) {
  if (!circ || !out) return fail(QS_ERR_ARG, "null pointer");
  if (n_values < 1) return fail(QS_ERR_ARG, "n_values must be at least 1");
  qs_cut_score sc{};
  const qs_status s = score_cut(circ->c, upper_mask, n_values, sc);
  if (s != QS_OK) return s;
  *out = sc;
  return QS_OK;
}

qs_status qs_choose_cut(const qs_circuit* circ, const uint64_t* masks, size_t n_masks,
                        int n_values, int criterion, size_t* best, qs_cut_score* best_score) {
  if (!circ || !masks || !best) return fail(QS_ERR_ARG, "null pointer");
  if (n_masks == 0) return fail(QS_ERR_ARG, "no candidate masks");
  if (n_values < 1) return fail(QS_ERR_ARG, "n_values must be at least 1");
  if (criterion != 0 && criterion != 1) return fail(QS_ERR_ARG, "unknown criterion");
  bool found = false;
  size_t bi = 0;
  qs_cut_score bs{};
  for (size_t i = 0; i < n_masks; ++i) {
    qs_cut_score sc{};
    if (score_cut(circ->c, masks[i], n_values, sc) != QS_OK) continue;
    const double v = criterion == 0 ? sc.flat_updates : sc.plan_cost;
    const double bv = criterion == 0 ? bs.flat_updates : bs.plan_cost;
    if (!found || v < bv) {
      found = true;
      bi = i;
      bs = sc;
    }
  }
  if (!found) return fail(QS_ERR_UNSUPPORTED, "no candidate mask can be scored");
  *best = bi;
  if (best_score) *best_score = bs;
  return QS_OK;
}

qs_status qs_plan_info(const qs_plan* plan, int* n_upper, int* n_lower, int* n_cuts) {
  if (!plan) return fail(QS_ERR_ARG, "null plan");
  if (n_upper) *n_upper = plan->side[0].n;
  if (n_lower) *n_lower = plan->side[1].n;
  if (n_cuts) *n_cuts = (int)plan->cuts.size();
  return QS_OK;
}

qs_status qs_plan_dump(const qs_plan* plan, uint64_t copy_begin, uint64_t copy_end, char* buf,
                       size_t cap, size_t* needed) {
  if (!plan || (!buf && cap)) return fail(QS_ERR_ARG, "null pointer");
  const int c = (int)plan->cuts.size();
  if (copy_begin >= copy_end || copy_end > (1ULL << c)) return fail(QS_ERR_ARG, "copy range outside [0, 2^c)");
  // the first block of the range, as qs_run_halves would split it
  int sz = std::min(ctz64(copy_begin), c);
  while (sz > 0 && (copy_begin + (1ULL << sz) > copy_end ||
                    (plan->opts.copies_per_launch && (1ULL << sz) > plan->opts.copies_per_launch)))
    --sz;
  if (plan->opts.plain) sz = 0;
  Block blk;
  blk.k0 = copy_begin;
  blk.p = c - sz;
  SidePlan sp[2];
  bool ok[2];
  std::string err;
  for (int k = 0; k < 2; ++k) ok[k] = plan_side(plan->side[k], c, blk, dump_knobs(plan, k), sp[k], err);
  std::string js = dump_json(plan->circ, plan->upper_mask, plan->cuts, plan->side[0],
                             plan->side[1], ok[0] ? &sp[0] : nullptr, ok[1] ? &sp[1] : nullptr);
  js.pop_back();  // closing brace
  js += ",\"block\":{\"k0\":" + std::to_string(blk.k0) + ",\"p\":" + std::to_string(blk.p) + "}";
  if (!ok[0] || !ok[1]) js += ",\"error\":\"" + err + "\"";
  js += "}";
  if (needed) *needed = js.size() + 1;
  if (cap) {
    size_t nb = std::min(cap - 1, js.size());
    std::memcpy(buf, js.data(), nb);
    buf[nb] = '\0';
  }
  return QS_OK;
}

void qs_plan_free(qs_plan* plan) { delete plan; }

qs_status qs_plan_reset(qs_plan* plan, int keep_bitstrings) {
  if (!plan) return fail(QS_ERR_ARG, "null plan");
  for (BlockRes& b : plan->blocks) {
    for (int k = 0; k < 2; ++k) plan->pool.put_unordered(b.X[k]);
    if (b.Ut) plan->pool.put_unordered(b.Ut);
    if (b.d_rows) plan->pool.put_unordered((void*)b.d_rows);
  }
  plan->blocks.clear();
  plan->ranges.clear();
  plan->unordered = true;
  if (!keep_bitstrings && plan->registered) {
    // the tables stay (stale) until a different set is registered
    plan->registered = false;
    plan->stale = true;
  }
  return QS_OK;
}

qs_status qs_run_halves(qs_plan* plan, uint64_t copy_begin, uint64_t copy_end,
                        const uint64_t* bitstrings, size_t m, void* hip_stream) {
  if (!plan) return fail(QS_ERR_ARG, "null plan");
  if ((bitstrings == nullptr) != (m == 0)) return fail(QS_ERR_ARG, "bitstrings and m disagree");
  const int c = (int)plan->cuts.size();
  const uint64_t total = 1ULL << c;
  if (copy_begin >= copy_end || copy_end > total) return fail(QS_ERR_ARG, "copy range outside [0, 2^c)");
  for (auto& r : plan->ranges)
    if (copy_begin < r.second && r.first < copy_end) return fail(QS_ERR_STATE, "copy range already run");
  qs_status s = register_bits(plan, bitstrings, m);
  if (s != QS_OK) return s;
  hipStream_t st = (hipStream_t)hip_stream;
  if (plan->unordered) {
    // the blocks below settle the pool after their fork, which orders reuse on
    // both streams after the released buffers' last users when those ran on
    // this stream (and on aux, joined into it); after a change of stream, wait
    // for them first
    if (st != plan->last_st) HIPCHECK(hipDeviceSynchronize());
    plan->pool.settle();
    plan->unordered = false;
  }
  plan->last_st = st;
  uint64_t k = copy_begin;
  while (k < copy_end) {
    int sz = std::min(ctz64(k), c);
    while (sz > 0 && (k + (1ULL << sz) > copy_end ||
                      (plan->opts.copies_per_launch && (1ULL << sz) > plan->opts.copies_per_launch)))
      --sz;
    if (plan->opts.plain) sz = 0;  // the flat form runs every copy on its own
    Block blk;
    blk.k0 = k;
    blk.p = c - sz;
    BlockRes br;
    br.k0 = k;
    br.k1 = k + (1ULL << sz);
    const uint64_t Kb = 1ULL << sz;
    if (plan->cache.size() + 2 > kMaxCachedSides &&
        plan->cache.find(std::make_tuple(0, blk.k0, blk.p)) == plan->cache.end()) {
      // bound the host and device memory of cached block plans (the flat
      // form plans every copy as a block of its own): drop them all, with
      // their copy tables, before this block plans either side, once no
      // queued kernel reads their descriptors
      HIPCHECK(hipDeviceSynchronize());
      plan->drop_block_plans();
    }
    Prepared* prs[2] = {nullptr, nullptr};
    for (int sidx = 0; sidx < 2; ++sidx) {
      s = prepare_side(plan, sidx, blk, &prs[sidx]);
      if (s != QS_OK) return s;
    }
    // the lower half's natural order mapped onto the upper half's (cached per block)
    auto pkey = std::make_pair(blk.k0, blk.p);
    auto pit = plan->perms.find(pkey);
    if (pit == plan->perms.end()) {
      const std::vector<uint32_t>& ku = prs[0]->nu_to_k;
      const std::vector<uint32_t>& kl = prs[1]->nu_to_k;
      std::vector<uint32_t> inv(Kb), perm(Kb);
      for (uint64_t nu = 0; nu < Kb; ++nu) inv[kl[nu]] = (uint32_t)nu;
      for (uint64_t nu = 0; nu < Kb; ++nu) perm[nu] = inv[ku[nu]];
      BlockMaps bm;
      // the tables go to the cache at the end; a failure on the way frees them
      struct Guard {
        DevAlloc* da;
        BlockMaps* bm;
        bool keep = false;
        ~Guard() {
          if (!keep) {
            da->put(bm->d_perm);
            da->put(bm->d_colsel);
          }
        }
      } guard{&plan->dalloc, &bm};
      bm.d_perm = (uint32_t*)plan->dalloc.get(Kb * sizeof(uint32_t));
      if (!bm.d_perm) return fail(QS_ERR_OOM, "copy permutation");
      HIPCHECK(hipMemcpy(bm.d_perm, perm.data(), Kb * sizeof(uint32_t), hipMemcpyHostToDevice));
      bm.nu_to_k = std::make_shared<std::vector<uint32_t>>(ku);
      const TailDesc& tl = prs[1]->td;
      if (tl.end_base) {
        // nu_U -> copy is linear in the bits of nu: find the bit of each lower
        // end cut, then nu' (nu without those bits) -> the lower copy with end bits 0
        bm.ne = tl.n_end;
        for (int i = 0; i < bm.ne; ++i) {
          bm.pos[i] = -1;
          for (int b = 0; (1ULL << b) < Kb; ++b)
            if ((uint64_t)ku[(size_t)1 << b] == tl.ekbit[i]) bm.pos[i] = b;
          if (bm.pos[i] < 0) return fail(QS_ERR_UNSUPPORTED, "internal: end cut outside the copy order");
        }
        std::vector<int> asc(bm.pos, bm.pos + bm.ne);
        std::sort(asc.begin(), asc.end());
        const uint64_t K0 = Kb >> bm.ne;
        std::vector<uint32_t> colsel(K0);
        for (uint64_t v = 0; v < K0; ++v) {
          uint64_t nu = v;
          for (int p : asc) nu = ((nu >> p) << (p + 1)) | (nu & ((1ULL << p) - 1));
          const uint32_t nl = inv[ku[nu]];
          if (nl & ((1u << bm.ne) - 1)) return fail(QS_ERR_UNSUPPORTED, "internal: end bits do not match");
          colsel[v] = nl >> bm.ne;
        }
        bm.d_colsel = (uint32_t*)plan->dalloc.get(K0 * sizeof(uint32_t));
        if (!bm.d_colsel) return fail(QS_ERR_OOM, "copy permutation");
        HIPCHECK(hipMemcpy(bm.d_colsel, colsel.data(), K0 * sizeof(uint32_t), hipMemcpyHostToDevice));
      }
      pit = plan->perms.emplace(pkey, bm).first;
      guard.keep = true;
    }
    br.nu_to_k = pit->second.nu_to_k;
    const BlockMaps& bmap = pit->second;
    // the halves are independent until the assembly: the upper one runs on
    // the caller's stream, the lower one on the plan's second stream, forked
    // after the work already queued on st and joined back before the permute
    hipStream_t ss[2] = {st, st};
    if (!plan->opts.one_stream && !plan->opts.plain) {
      if (!plan->aux) {
        HIPCHECK(hipStreamCreateWithFlags(&plan->aux, hipStreamNonBlocking));
        HIPCHECK(hipEventCreateWithFlags(&plan->ev_fork, hipEventDisableTiming));
        HIPCHECK(hipEventCreateWithFlags(&plan->ev_join, hipEventDisableTiming));
      }
      ss[1] = plan->aux;
      HIPCHECK(hipEventRecord(plan->ev_fork, st));
      HIPCHECK(hipStreamWaitEvent(plan->aux, plan->ev_fork, 0));
    }
    plan->pool.settle();
    const int ne = bmap.ne;
    const uint64_t K0 = Kb >> ne;
    const int NL = (int)plan->vals[1].size();
    // the lower rows' order with folded end cuts (rows, then group starts),
    // copied ahead of the lower half's passes: off the path from its leaf
    // evaluation to the product
    uint32_t* dr = nullptr;
    if (ne > 0) {
      const size_t nr = (size_t)NL + (1u << ne) + 1;
      dr = (uint32_t*)plan->pool.get(nr * sizeof(uint32_t), ss[1]);
      if (!dr) return fail(QS_ERR_OOM, "row order");
      HIPCHECK(hipMemcpyAsync(dr, prs[1]->dev + prs[1]->o_rows, nr * sizeof(uint32_t),
                              hipMemcpyDeviceToDevice, ss[1]));
    }
    for (int sidx = 0; sidx < 2; ++sidx) {
      const size_t bytes = (sidx == 1 ? K0 : Kb) * plan->vals[sidx].size() * sizeof(float2);
      br.X[sidx] = (float2*)plan->pool.get(bytes, ss[sidx]);
      if (!br.X[sidx]) return fail(QS_ERR_OOM, "gathered half amplitudes");
      s = run_side(plan, sidx, *prs[sidx], br.X[sidx], ss[sidx]);
      if (s != QS_OK) return s;
    }
    {
      // the lower half's columns onto the upper half's copy order, still on
      // the lower half's stream (with folded end cuts: rows sorted by their
      // end-cut bits, columns nu')
      const size_t bytes = K0 * NL * sizeof(float2);
      float2* XL = (float2*)plan->pool.get(bytes, ss[1]);
      if (!XL) return fail(QS_ERR_OOM, "gathered half amplitudes");
      Timer tm(plan, ss[1], 3);
      if (ne > 0) {
        HIPCHECK(launch_gather_rows_cols(br.X[1], XL, dr, bmap.d_colsel, NL, (int)K0, (int)K0,
                                         ss[1]));
        br.d_rows = dr;
        br.ne = ne;
        for (int i = 0; i < ne; ++i) br.pos[i] = bmap.pos[i];
        br.goff = prs[1]->goff;
        br.rows = prs[1]->rows;
        br.sig = prs[1]->sig;
      } else {
        HIPCHECK(launch_permute_cols(br.X[1], XL, bmap.d_perm, NL, (int)Kb, ss[1]));
      }
      ++tm.launches;
      plan->pool.put(br.X[1], ss[1]);
      br.X[1] = XL;
    }
    if (ne > 0) {
      // the upper operand transformed over the lower end cuts' bits
      const int MU = (int)plan->vals[0].size();
      br.Ut = (float2*)plan->pool.get(Kb * MU * sizeof(float2), st);
      if (!br.Ut) return fail(QS_ERR_OOM, "transformed upper amplitudes");
      Timer tm(plan, st, 3);
      HIPCHECK(launch_end_wht(br.X[0], MU, (int)Kb, ne, br.pos, br.Ut, st));
      ++tm.launches;
    }
    if (ss[1] != st) {
      HIPCHECK(hipEventRecord(plan->ev_join, ss[1]));
      HIPCHECK(hipStreamWaitEvent(st, plan->ev_join, 0));
    }
    plan->pool.settle();
    plan->blocks.push_back(br);
    k = br.k1;
  }
  plan->ranges.emplace_back(copy_begin, copy_end);
  return QS_OK;
}

qs_status qs_amplitudes(qs_plan* plan, const uint64_t* bitstrings, size_t m, qs_precision prec,
                        float* out_c64, double* out_stats, void* hip_stream) {
  if (!plan || !bitstrings || !out_c64) return fail(QS_ERR_ARG, "null pointer");
  if (m == 0) return fail(QS_ERR_ARG, "no bitstrings");
  if (prec != QS_PREC_FP32 && prec != QS_PREC_SPLIT_BF16) return fail(QS_ERR_ARG, "unknown precision");
  hipStream_t st = (hipStream_t)hip_stream;
  if (plan->registered &&
      (m != plan->bits.size() || std::memcmp(bitstrings, plan->bits.data(), m * 8) != 0))
    return fail(QS_ERR_STATE, "bitstrings differ from the registered set");
  if (!plan->registered || plan->blocks.empty()) {
    qs_status s = qs_run_halves(plan, 0, 1ULL << plan->cuts.size(), bitstrings, m, hip_stream);
    if (s != QS_OK) return s;
  }
  float2* amps = (float2*)plan->pool.get(m * sizeof(float2), st);
  double* sums = (double*)plan->pool.get(2 * sizeof(double), st);
  if (!amps || !sums) return fail(QS_ERR_OOM, "output buffers");
  Scratch sc{plan, st};
  qs_status s = assemble(plan, prec, amps, sums, sc);
  if (s != QS_OK) return s;
  // staged on the host: the caller's arrays are written only on success
  std::vector<float2> ha(m);
  double h[2];
  HIPCHECK(hipMemcpyAsync(ha.data(), amps, m * sizeof(float2), hipMemcpyDeviceToHost, st));
  HIPCHECK(hipMemcpyAsync(h, sums, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHECK(hipStreamSynchronize(st));
  plan->pool.put(amps, st);
  plan->pool.put(sums, st);
  std::memcpy(out_c64, ha.data(), m * sizeof(float2));
  if (out_stats) {
    const double n = plan->circ.n;
    out_stats[0] = h[0];
    out_stats[1] = std::ldexp(h[0] / (double)m, (int)n);
    out_stats[2] = std::ldexp(h[1] / (double)m, (int)(2 * n));
  }
  return QS_OK;
}

static qs_status assemble_on(qs_plan* plan, qs_precision prec, float* d_out_c64,
                             double* d_out_sums, hipStream_t st) {
  if (!plan->registered || plan->blocks.empty()) return fail(QS_ERR_STATE, "no copies run");
  Scratch sc{plan, st};
  return assemble(plan, prec, (float2*)d_out_c64, d_out_sums, sc);
}

qs_status qs_amplitudes_device(qs_plan* plan, qs_precision prec, float* d_out_c64,
                               double* d_out_sums, void* hip_stream) {
  if (!plan || !d_out_c64) return fail(QS_ERR_ARG, "null pointer");
  if (prec != QS_PREC_FP32 && prec != QS_PREC_SPLIT_BF16) return fail(QS_ERR_ARG, "unknown precision");
  if (!plan->registered || plan->blocks.empty()) return fail(QS_ERR_STATE, "no copies run");
  Scratch sc{plan, (hipStream_t)hip_stream};
  return assemble(plan, prec, (float2*)d_out_c64, d_out_sums, sc);
}

qs_status qs_amplitudes_device_static(qs_plan* plan, qs_precision prec, float* d_out_c64,
                                      double* d_out_sums, void* hip_stream) {
  if (!plan || !d_out_c64) return fail(QS_ERR_ARG, "null pointer");
  if (prec != QS_PREC_FP32 && prec != QS_PREC_SPLIT_BF16) return fail(QS_ERR_ARG, "unknown precision");
  if (!plan->registered || plan->blocks.empty()) return fail(QS_ERR_STATE, "no copies run");
  // the scratch bytes this assembly needs, before anything is launched
  Scratch need{plan, (hipStream_t)hip_stream};
  need.measure = true;
  qs_status s = assemble(plan, prec, nullptr, nullptr, need);
  if (s != QS_OK) return s;
  if (need.used > static_scratch_capacity())
    return fail(QS_ERR_UNSUPPORTED, "the assembly needs " + std::to_string(need.used) +
                                        " bytes of scratch, more than the static region's " +
                                        std::to_string(static_scratch_capacity()));
  void* base = nullptr;
  HIPCHECK(static_scratch(&base));
  Scratch sc{plan, (hipStream_t)hip_stream};
  sc.base = (char*)base;
  sc.cap = static_scratch_capacity();
  // no timing events either (creating one is an allocation of the runtime)
  const bool timing = plan->timing;
  plan->timing = false;
  s = assemble(plan, prec, (float2*)d_out_c64, d_out_sums, sc);
  plan->timing = timing;
  return s;
}

qs_status qs_run_graph(qs_plan* plan, uint64_t copy_begin, uint64_t copy_end, qs_precision prec,
                       float* d_out_c64, double* d_out_sums, void* hip_stream) {
  if (!plan || !d_out_c64) return fail(QS_ERR_ARG, "null pointer");
  if (prec != QS_PREC_FP32 && prec != QS_PREC_SPLIT_BF16) return fail(QS_ERR_ARG, "unknown precision");
  const uint64_t total = 1ULL << plan->cuts.size();
  if (copy_begin >= copy_end || copy_end > total) return fail(QS_ERR_ARG, "copy range outside [0, 2^c)");
  if (!plan->registered) return fail(QS_ERR_STATE, "no bitstrings registered");
  hipStream_t st = (hipStream_t)hip_stream;
  if (!st) return fail(QS_ERR_ARG, "a graph is captured on a stream other than the null stream");
  auto step = [&]() -> qs_status {
    qs_status s = qs_plan_reset(plan, 1);
    if (s == QS_OK) s = qs_run_halves(plan, copy_begin, copy_end, nullptr, 0, hip_stream);
    if (s == QS_OK) s = assemble_on(plan, prec, d_out_c64, d_out_sums, st);
    return s;
  };
  const bool same = plan->graph_exec && plan->graph_k0 == copy_begin &&
                    plan->graph_k1 == copy_end && plan->graph_prec == (int)prec &&
                    plan->graph_out == (void*)d_out_c64 && plan->graph_sums == (void*)d_out_sums &&
                    plan->graph_gen == plan->gen() && plan->last_st == st;
  if (same) {
    HIPCHECK(hipGraphLaunch(plan->graph_exec, st));
    return QS_OK;
  }
  plan->drop_graph();
  // an eager step first: it plans and uploads whatever is not cached yet and
  // leaves in the plan's pool every buffer a step takes, so that the captured
  // step below makes no allocation, no copy from the host and no
  // synchronisation
  const int timing = plan->timing;
  plan->timing = 0;  // no events inside the graph
  qs_status s = step();
  if (s != QS_OK) {
    plan->timing = timing;
    return s;
  }
  const uint64_t g0 = plan->gen();
  HIPCHECK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  s = step();
  hipGraph_t g = nullptr;
  const hipError_t ec = hipStreamEndCapture(st, &g);
  plan->timing = timing;
  if (s != QS_OK) {
    if (g) (void)hipGraphDestroy(g);
    return s;
  }
  if (ec != hipSuccess) return fail(QS_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(ec));
  if (plan->gen() != g0) {
    // the captured step released memory (it had to make room): not replayable
    (void)hipGraphDestroy(g);
    return fail(QS_ERR_OOM, "the step does not fit the device without releasing buffers");
  }
  hipGraphExec_t ex = nullptr;
  const hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  if (ei != hipSuccess) {
    (void)hipGraphDestroy(g);
    return fail(QS_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
  }
  plan->graph = g;
  plan->graph_exec = ex;
  plan->graph_k0 = copy_begin;
  plan->graph_k1 = copy_end;
  plan->graph_prec = (int)prec;
  plan->graph_out = d_out_c64;
  plan->graph_sums = d_out_sums;
  plan->graph_gen = g0;
  HIPCHECK(hipGraphLaunch(ex, st));
  return QS_OK;
}

qs_status qs_half_amplitudes(qs_plan* plan, int side, uint64_t copy_begin, uint64_t copy_end,
                             float* out_c64, size_t cap, size_t* n_values, void* hip_stream) {
  if (!plan || !out_c64 || !n_values) return fail(QS_ERR_ARG, "null pointer");
  if (side != 0 && side != 1) return fail(QS_ERR_ARG, "side must be 0 or 1");
  const BlockRes* hit = nullptr;
  for (const BlockRes& b : plan->blocks)
    if (b.k0 == copy_begin && b.k1 == copy_end) hit = &b;
  if (!hit) return fail(QS_ERR_STATE, "copy range was not run as one block");
  const size_t S = plan->vals[side].size();
  const size_t cnt = (size_t)(copy_end - copy_begin) * S;
  if (cap < cnt) return fail(QS_ERR_ARG, "output capacity too small");
  hipStream_t st = (hipStream_t)hip_stream;
  const size_t Kb = (size_t)(copy_end - copy_begin);
  const std::vector<uint32_t>& nk = *hit->nu_to_k;
  float2* o = (float2*)out_c64;
  const double pr_ = plan->phi[side][0], pi_ = plan->phi[side][1];
  auto ph = [&](float2 a) {
    return make_float2((float)(a.x * pr_ - a.y * pi_), (float)(a.x * pi_ + a.y * pr_));
  };
  if (side == 1 && hit->ne > 0) {
    // stored: rows sorted by end-cut pattern, the copies with end bits 0 in
    // the order nu'; the copy with end bits e is that one times (-1)^popc(e & sig)
    const int ne = hit->ne;
    const size_t K0 = Kb >> ne;
    std::vector<float2> tmp(S * K0);
    HIPCHECK(hipMemcpyAsync(tmp.data(), hit->X[1], tmp.size() * sizeof(float2),
                            hipMemcpyDeviceToHost, st));
    HIPCHECK(hipStreamSynchronize(st));
    std::vector<int> asc(hit->pos, hit->pos + ne);
    std::sort(asc.begin(), asc.end());
    const std::vector<uint32_t>& rows = *hit->rows;
    const std::vector<uint32_t>& sig = *hit->sig;
    for (size_t r = 0; r < S; ++r) {
      const uint32_t l = rows[r];
      for (size_t nu = 0; nu < Kb; ++nu) {
        uint32_t e = 0;
        for (int i = 0; i < ne; ++i) e |= (uint32_t)((nu >> hit->pos[i]) & 1) << i;
        size_t v = 0, vb = 0;
        for (int b = 0; (1ULL << b) < Kb; ++b) {
          if (std::find(asc.begin(), asc.end(), b) != asc.end()) continue;
          v |= ((nu >> b) & 1) << vb++;
        }
        float2 a = tmp[r * K0 + v];
        if (__builtin_popcount(e & sig[l]) & 1) a = make_float2(-a.x, -a.y);
        o[(size_t)nk[nu] * S + l] = ph(a);
      }
    }
    *n_values = S;
    return QS_OK;
  }
  std::vector<float2> tmp(cnt);
  HIPCHECK(hipMemcpyAsync(tmp.data(), hit->X[side], cnt * sizeof(float2), hipMemcpyDeviceToHost, st));
  HIPCHECK(hipStreamSynchronize(st));
  // stored as [s][nu] in the upper half's natural copy order; returned as [k][s]
  for (size_t si = 0; si < S; ++si)
    for (size_t nu = 0; nu < Kb; ++nu) o[(size_t)nk[nu] * S + si] = ph(tmp[si * Kb + nu]);
  *n_values = S;
  return QS_OK;
}

qs_status qs_get_timing(qs_plan* plan, double* out10) {
  if (!plan || !out10) return fail(QS_ERR_ARG, "null pointer");
  // out10 holds 11 doubles (see qs.h)
  for (EvRec& e : plan->events) {
    HIPCHECK(hipEventSynchronize(e.b));
    float ms = 0;
    HIPCHECK(hipEventElapsedTime(&ms, e.a, e.b));
    plan->tms[e.fam] += ms;
    plan->counts[e.fam] += e.launches;
    (void)hipEventDestroy(e.a);
    (void)hipEventDestroy(e.b);
  }
  plan->events.clear();
  for (qs_plan::PassRec& e : plan->pass_events) {
    HIPCHECK(hipEventSynchronize(e.b));
    float ms = 0;
    HIPCHECK(hipEventElapsedTime(&ms, e.a, e.b));
    const double rec[8] = {(double)e.side, (double)e.pass, (double)e.level_in, (double)e.stages,
                           (double)e.tiles, e.bytes, (double)ms, (double)e.passes};
    plan->pass_log.insert(plan->pass_log.end(), rec, rec + 8);
    (void)hipEventDestroy(e.a);
    (void)hipEventDestroy(e.b);
  }
  plan->pass_events.clear();
  for (int i = 0; i < 4; ++i) {
    out10[i] = plan->tms[i];
    out10[4 + i] = plan->counts[i];
  }
  out10[8] = plan->pass_bytes;
  out10[9] = plan->gemm_flops;
  out10[10] = plan->tail_flops;
  return QS_OK;
}

qs_status qs_set_timing(qs_plan* plan, int enable) {
  if (!plan) return fail(QS_ERR_ARG, "null plan");
  double dummy[11];
  (void)qs_get_timing(plan, dummy);
  if (enable < 0 || enable > 2) return fail(QS_ERR_ARG, "timing mode must be 0, 1 or 2");
  plan->timing = enable;
  plan->pass_log.clear();
  for (int i = 0; i < 4; ++i) plan->tms[i] = plan->counts[i] = 0;
  plan->pass_bytes = plan->gemm_flops = plan->tail_flops = 0;
  return QS_OK;
}

qs_status qs_get_pass_timing(qs_plan* plan, double* out, size_t cap_records, size_t* n_records) {
  if (!plan || !n_records || (!out && cap_records)) return fail(QS_ERR_ARG, "null pointer");
  double fam[11];
  const qs_status st = qs_get_timing(plan, fam);
  if (st != QS_OK) return st;
  const size_t n = plan->pass_log.size() / 8;
  const size_t k = std::min(n, cap_records);
  if (k) std::memcpy(out, plan->pass_log.data(), k * 8 * sizeof(double));
  *n_records = n;
  return QS_OK;
}

}  // extern "C"

// ------------------------------------------------------------ chain partitions
//
// t parts whose cut gates each join parts i and i+1 (Sec. 3, Fig. 3).  A cut
// CZ puts P_b on its endpoint in the even-numbered part and Z^b on the one in
// the odd-numbered part, so every part carries one kind of cut factor and
// runs as side 0 of a one-sided plan over its own cuts (numbered in cut
// order).  With k_i the bits of link i's cuts, the sum over copies is a
// chain of t - 1 products contracted from both ends towards a split part s
// (chosen at registration for the fewest flops):
//   left,  p < s:  T_p[(v_0..v_p)][k_p] = sum_{k_{p-1}} T_{p-1}[(v_0..v_{p-1})][k_{p-1}]
//                                            X_p[v_p][k_p][k_{p-1}]      (T_0 = X_0)
//   right, p >= s: R_p[(v_{t-1}..v_p)][k_{p-1}] = sum_{k_p} R_{p+1}[(v_{t-1}..v_{p+1})][k_p]
//                                            X_p[v_p][k_{p-1}][k_p]      (R_{t-1} = X_{t-1})
//   amp[(v_0..v_{s-1})][(v_{t-1}..v_s)] = sum_k T_{s-1}[..][k] R_s[..][k].
// Part p's output X_p[v][k] (value v, local copy k) is first permuted to the
// column order its side of the chain needs.

struct qs_mplan {
  Circuit circ;
  int t = 0;
  std::vector<uint64_t> masks;
  std::vector<int> link_c;                       // cuts of link i (parts i, i+1)
  std::vector<std::unique_ptr<qs_plan>> parts;   // one-sided plans
  std::vector<std::vector<int>> link_of;         // per part, per local cut: its link
  DevAlloc dalloc;
  Pool pool;
  bool registered = false;
  std::vector<uint64_t> bits;
  std::vector<int> nvals;
  int* d_iu = nullptr;   // grid row of each bitstring (values of parts 0..t-2)
  int* d_il = nullptr;   // value index in the last part
  std::vector<uint32_t*> d_perm;  // per part: natural column of each ordered column
  int split = 1;  // parts [0, split) contract from the left end, [split, t) from the right
  hipEvent_t ev_fork = nullptr;   // the parts run on their plans' streams (qs_plan::aux)
  qs_mplan() { pool.da = &dalloc; }
  ~qs_mplan() {
    (void)hipDeviceSynchronize();
    for (uint32_t* q : d_perm) dalloc.put(q);
    pool.release_all();
    if (ev_fork) (void)hipEventDestroy(ev_fork);
  }
};

extern "C" {

qs_status qs_partition_chain(const qs_circuit* circ, const uint64_t* part_masks, int t,
                             const qs_options* opts, qs_mplan** out) {
  if (!circ || !part_masks || !out) return fail(QS_ERR_ARG, "null pointer");
  if (t < 2 || t > 8) return fail(QS_ERR_ARG, "t must be 2..8 parts");
  const Circuit& c = circ->c;
  const int n = c.n;
  const uint64_t full = n == 64 ? ~0ULL : ((1ULL << n) - 1);
  std::vector<int> owner(n, -1);
  uint64_t seen = 0;
  for (int p = 0; p < t; ++p) {
    const uint64_t m = part_masks[p];
    if (m == 0 || (m & ~full) || (m & seen)) return fail(QS_ERR_ARG, "parts must be non-empty and disjoint");
    if (__builtin_popcountll(m) > 32) return fail(QS_ERR_ARG, "a part has more than 32 qubits");
    seen |= m;
    for (int q = 0; q < n; ++q)
      if ((m >> q) & 1) owner[q] = p;
  }
  if (seen != full) return fail(QS_ERR_ARG, "the parts must cover every qubit");
  // cut gates in cut order: (cycle, endpoint in the lower-numbered part)
  std::vector<std::tuple<int, int, int, int>> raw;  // cycle, q_lo, q_hi, link
  for (const Gate& g : c.gates) {
    if (g.kind != G_CZ || owner[g.q0] == owner[g.q1]) continue;
    int a = g.q0, b = g.q1;
    if (owner[a] > owner[b]) std::swap(a, b);
    if (owner[b] != owner[a] + 1)
      return fail(QS_ERR_UNSUPPORTED, "the parts do not form a chain (a cut gate skips a part)");
    raw.emplace_back(g.cycle, a, b, owner[a]);
  }
  std::sort(raw.begin(), raw.end());
  if (opts && (opts->alloc.alloc == nullptr) != (opts->alloc.free == nullptr))
    return fail(QS_ERR_ARG, "allocator needs both alloc and free");
  std::unique_ptr<qs_mplan> mp(new (std::nothrow) qs_mplan());
  if (!mp) return fail(QS_ERR_OOM, "host allocation");
  if (opts) mp->dalloc.a = opts->alloc;
  mp->circ = c;
  mp->t = t;
  mp->masks.assign(part_masks, part_masks + t);
  mp->link_c.assign(t - 1, 0);
  for (auto& r : raw) ++mp->link_c[std::get<3>(r)];
  mp->link_of.resize(t);
  mp->d_perm.assign(t, nullptr);
  for (int p = 0; p < t; ++p) {
    std::unique_ptr<qs_plan> pp(new (std::nothrow) qs_plan());
    if (!pp) return fail(QS_ERR_OOM, "host allocation");
    pp->circ = c;
    pp->upper_mask = part_masks[p];
    pp->part_mode = true;
    if (opts) pp->opts = *opts;
    else {
      pp->opts = qs_options{};
      pp->opts.materialize_level = -1;
    }
    pp->opts.one_stream = 1;
    pp->dalloc.a = pp->opts.alloc;
    pp->concurrency = t;  // the parts run at the same time
    std::map<std::pair<int, int>, int> cut_of;
    for (auto& r : raw) {
      const int link = std::get<3>(r);
      if (link != p && link != p - 1) continue;
      const int q = link == p ? std::get<1>(r) : std::get<2>(r);  // this part's endpoint
      const int j = (int)pp->cuts.size();
      pp->cuts.push_back(Cut{j, std::get<0>(r), q, q});
      cut_of[{std::get<0>(r), q}] = j;
      mp->link_of[p].push_back(link);
    }
    // all of a part's copies run as one block: X_p holds values x 2^c_p amplitudes
    if (pp->cuts.size() > 30) return fail(QS_ERR_UNSUPPORTED, "more than 30 cut gates touch one part");
    build_side(c, part_masks[p], p % 2 == 0, cut_of, pp->side[0]);
    pp->side[1] = Side();
    pp->side[1].upper = false;
    mp->parts.push_back(std::move(pp));
  }
  *out = mp.release();
  return QS_OK;
}

qs_status qs_chain_info(const qs_mplan* mp, int* t, int* part_qubits, int* link_cuts) {
  if (!mp) return fail(QS_ERR_ARG, "null plan");
  if (t) *t = mp->t;
  for (int p = 0; p < mp->t; ++p) {
    if (part_qubits) part_qubits[p] = mp->parts[p]->side[0].n;
    if (link_cuts && p + 1 < mp->t) link_cuts[p] = mp->link_c[p];
  }
  return QS_OK;
}

void qs_chain_free(qs_mplan* mp) { delete mp; }

qs_status qs_chain_register(qs_mplan* mp, const uint64_t* bits, size_t m) {
  if (!mp || !bits || m == 0) return fail(QS_ERR_ARG, "no bitstrings");
  if (mp->registered) {
    if (m == mp->bits.size() && std::memcmp(bits, mp->bits.data(), m * 8) == 0) return QS_OK;
    return fail(QS_ERR_STATE, "bitstrings differ from the registered set");
  }
  const int t = mp->t;
  const int n = mp->circ.n;
  const uint64_t full = n == 64 ? ~0ULL : ((1ULL << n) - 1);
  for (size_t i = 0; i < m; ++i)
    if (bits[i] & ~full) return fail(QS_ERR_ARG, "bitstring has bits set beyond the qubit count");
  std::vector<std::vector<int>> idx(t, std::vector<int>(m));
  mp->nvals.assign(t, 0);
  double grid = 1;
  for (int p = 0; p < t; ++p) {
    const Side& s = mp->parts[p]->side[0];
    std::vector<uint32_t> hv(m);
    for (size_t i = 0; i < m; ++i) {
      uint32_t v = 0;
      for (int q = 0; q < s.n; ++q) v |= (uint32_t)((bits[i] >> s.qubits[q]) & 1) << q;
      hv[i] = v;
    }
    std::vector<uint32_t> u(hv);
    std::sort(u.begin(), u.end());
    u.erase(std::unique(u.begin(), u.end()), u.end());
    for (size_t i = 0; i < m; ++i)
      idx[p][i] = (int)(std::lower_bound(u.begin(), u.end(), hv[i]) - u.begin());
    mp->nvals[p] = (int)u.size();
    mp->parts[p]->vals[0] = std::move(u);
    grid *= mp->nvals[p];
  }
  // the products run over the whole grid of part values
  if (grid > (double)(1u << 28))
    return fail(QS_ERR_UNSUPPORTED, "the part values span a grid above 2^28 amplitudes");
  // split part: the fewest flops over both partial chains and the last product
  {
    const std::vector<int>& nv = mp->nvals;
    const std::vector<int>& lc = mp->link_c;
    double best = -1;
    for (int sp = 1; sp < t; ++sp) {
      double f = 0, big = 0, rows = nv[0];
      for (int p = 1; p < sp; ++p) {  // left products
        const double out = rows * nv[p] * std::ldexp(1.0, lc[p]);
        f += out * std::ldexp(1.0, lc[p - 1]);
        big = std::max(big, out);
        rows *= nv[p];
      }
      double rr = nv[t - 1];
      for (int p = t - 2; p >= sp; --p) {  // right products
        const double out = rr * nv[p] * std::ldexp(1.0, lc[p - 1]);
        f += out * std::ldexp(1.0, lc[p]);
        big = std::max(big, out);
        rr *= nv[p];
      }
      f += rows * rr * std::ldexp(1.0, lc[sp - 1]);
      if (big > (double)(1u << 28)) continue;
      if (best < 0 || f < best) {
        best = f;
        mp->split = sp;
      }
    }
    if (best < 0) return fail(QS_ERR_UNSUPPORTED, "a partial product would exceed 2^28 amplitudes");
  }
  std::vector<int> iu(m), il(m);
  for (size_t i = 0; i < m; ++i) {
    size_t r = 0, c = 0;
    for (int p = 0; p < mp->split; ++p) r = r * mp->nvals[p] + idx[p][i];
    for (int p = t - 1; p >= mp->split; --p) c = c * mp->nvals[p] + idx[p][i];
    iu[i] = (int)r;
    il[i] = (int)c;
  }
  (void)hipDeviceSynchronize();
  mp->pool.settle();
  int* a = (int*)mp->pool.get(m * sizeof(int), nullptr);
  int* b = (int*)mp->pool.get(m * sizeof(int), nullptr);
  if (!a || !b) return fail(QS_ERR_OOM, "value tables");
  HIPCHECK(hipMemcpy(a, iu.data(), m * sizeof(int), hipMemcpyHostToDevice));
  HIPCHECK(hipMemcpy(b, il.data(), m * sizeof(int), hipMemcpyHostToDevice));
  mp->d_iu = a;
  mp->d_il = b;
  mp->bits.assign(bits, bits + m);
  mp->registered = true;
  return QS_OK;
}

qs_status qs_chain_amplitudes_device(qs_mplan* mp, float* d_out_c64, double* d_out_sums,
                                     void* hip_stream) {
  if (!mp || !d_out_c64) return fail(QS_ERR_ARG, "null pointer");
  if (!mp->registered) return fail(QS_ERR_STATE, "no bitstrings registered");
  hipStream_t st = (hipStream_t)hip_stream;
  const int t = mp->t;
  std::vector<float2*> Y(t, nullptr);
  double ph_re = 1, ph_im = 0;  // product of the parts' constants (Prepared::phi)
  // the parts are independent until the products: each runs on a stream of
  // its own (default priority), forked from the caller's stream after the
  // work already queued there and joined back before the products.  Their
  // buffers return to the part streams, whose later work always starts after
  // such a fork, so after the products that read them.
  if (!mp->ev_fork) HIPCHECK(hipEventCreateWithFlags(&mp->ev_fork, hipEventDisableTiming));
  HIPCHECK(hipEventRecord(mp->ev_fork, st));
  for (int p = 0; p < t; ++p) {
    qs_plan* pp = mp->parts[p].get();
    if (!pp->aux) {
      HIPCHECK(hipStreamCreateWithFlags(&pp->aux, hipStreamNonBlocking));
      HIPCHECK(hipEventCreateWithFlags(&pp->ev_join, hipEventDisableTiming));
    }
    HIPCHECK(hipStreamWaitEvent(pp->aux, mp->ev_fork, 0));
  }
  for (int p = 0; p < t; ++p) {
    qs_plan* pp = mp->parts[p].get();
    hipStream_t ps = pp->aux;
    const int cp = (int)pp->cuts.size();
    const size_t K = (size_t)1 << cp;
    const int S = mp->nvals[p];
    Prepared* pr = nullptr;
    qs_status s = prepare_side(pp, 0, Block{}, &pr);
    if (s != QS_OK) return s;
    const double a = pp->phi[0][0], b = pp->phi[0][1];
    const double r0 = ph_re * a - ph_im * b, i0 = ph_re * b + ph_im * a;
    ph_re = r0;
    ph_im = i0;
    float2* X = (float2*)pp->pool.get((size_t)S * K * sizeof(float2), ps);
    float2* O = (float2*)mp->pool.get((size_t)S * K * sizeof(float2), ps);
    if (!X || !O) return fail(QS_ERR_OOM, "part amplitudes");
    s = run_side(pp, 0, *pr, X, ps);
    if (s != QS_OK) return s;
    if (!mp->d_perm[p]) {
      // ordered column of every natural column nu: left of the split the
      // later link's bits are major, from the split on the earlier link's
      const std::vector<int>& lk = mp->link_of[p];
      const bool left = p < mp->split;
      std::vector<uint32_t> perm(K);
      for (size_t nu = 0; nu < K; ++nu) {
        const uint32_t k = pr->nu_to_k[nu];
        uint32_t later = 0, earlier = 0;
        for (int j = 0; j < cp; ++j) {
          const uint32_t bit = (k >> (cp - 1 - j)) & 1;
          if (lk[j] == p) later = (later << 1) | bit;
          else earlier = (earlier << 1) | bit;
        }
        const int ne_ = p > 0 ? mp->link_c[p - 1] : 0;
        const int nl_ = p + 1 < t ? mp->link_c[p] : 0;
        const size_t col = left ? ((size_t)later << ne_) | earlier : ((size_t)earlier << nl_) | later;
        perm[col] = (uint32_t)nu;
      }
      uint32_t* d = (uint32_t*)mp->dalloc.get(K * sizeof(uint32_t));
      if (!d) return fail(QS_ERR_OOM, "part column order");
      mp->d_perm[p] = d;
      HIPCHECK(hipMemcpy(d, perm.data(), K * sizeof(uint32_t), hipMemcpyHostToDevice));
    }
    HIPCHECK(launch_permute_cols(X, O, mp->d_perm[p], S, (int)K, ps));
    pp->pool.put(X, ps);
    Y[p] = O;
    HIPCHECK(hipEventRecord(pp->ev_join, ps));
    HIPCHECK(hipStreamWaitEvent(st, pp->ev_join, 0));
  }
  // the two partial chains, then their product; a part's buffer returns to
  // its stream, a product's to the caller's
  auto product = [&](const float2* A, const float2* B, size_t M, size_t N, int kbits,
                     float2** C) -> qs_status {
    const int Kc = 1 << kbits;
    *C = (float2*)mp->pool.get(M * N * sizeof(float2), st);
    void* work = mp->pool.get(std::max<size_t>(256, zgemm_workspace_bytes(0, (int)M, (int)N, Kc)), st);
    if (!*C || !work) return fail(QS_ERR_OOM, "chain products");
    HIPCHECK(launch_zgemm_tn(0, (int)M, (int)N, Kc, A, Kc, B, Kc, *C, (int)N, 0, work, st));
    mp->pool.put(work, st);
    return QS_OK;
  };
  auto release = [&](float2* buf, int part) {  // part < 0: a product
    mp->pool.put(buf, part < 0 ? st : mp->parts[part]->aux);
  };
  const int sp = mp->split;
  float2* T = Y[0];
  int t_part = 0;
  size_t R = (size_t)mp->nvals[0];
  for (int p = 1; p < sp; ++p) {
    float2* C = nullptr;
    qs_status s = product(T, Y[p], R, (size_t)mp->nvals[p] << mp->link_c[p], mp->link_c[p - 1], &C);
    if (s != QS_OK) return s;
    release(T, t_part);
    release(Y[p], p);
    T = C;
    t_part = -1;
    R *= (size_t)mp->nvals[p];
  }
  float2* U = Y[t - 1];
  int u_part = t - 1;
  size_t Rr = (size_t)mp->nvals[t - 1];
  for (int p = t - 2; p >= sp; --p) {
    float2* C = nullptr;
    qs_status s = product(U, Y[p], Rr, (size_t)mp->nvals[p] << mp->link_c[p - 1], mp->link_c[p], &C);
    if (s != QS_OK) return s;
    release(U, u_part);
    release(Y[p], p);
    U = C;
    u_part = -1;
    Rr *= (size_t)mp->nvals[p];
  }
  float2* G = nullptr;
  {
    qs_status s = product(T, U, R, Rr, mp->link_c[sp - 1], &G);
    if (s != QS_OK) return s;
    release(T, t_part);
    release(U, u_part);
  }
  const size_t m = mp->bits.size();
  const int nb = prob_partial_blocks(m);
  double* part = (double*)mp->pool.get((2 * (size_t)nb + 2) * sizeof(double), st);
  if (!part) return fail(QS_ERR_OOM, "probability sums");
  HIPCHECK(launch_gather_prob_sums(G, (int)Rr, mp->d_iu, mp->d_il, m, (float2*)d_out_c64,
                                   make_float2((float)ph_re, (float)ph_im), part,
                                   d_out_sums ? d_out_sums : part + 2 * nb, st));
  mp->pool.put(part, st);
  mp->pool.put(G, st);
  return QS_OK;
}

qs_status qs_chain_amplitudes(qs_mplan* mp, const uint64_t* bits, size_t m, float* out_c64,
                              double* out_stats, void* hip_stream) {
  if (!mp || !bits || !out_c64) return fail(QS_ERR_ARG, "null pointer");
  qs_status s = qs_chain_register(mp, bits, m);
  if (s != QS_OK) return s;
  hipStream_t st = (hipStream_t)hip_stream;
  float2* amps = (float2*)mp->pool.get(m * sizeof(float2), st);
  double* sums = (double*)mp->pool.get(2 * sizeof(double), st);
  if (!amps || !sums) return fail(QS_ERR_OOM, "output buffers");
  s = qs_chain_amplitudes_device(mp, (float*)amps, sums, hip_stream);
  if (s != QS_OK) return s;
  // staged on the host: the caller's arrays are written only on success
  std::vector<float2> ha(m);
  double h[2];
  HIPCHECK(hipMemcpyAsync(ha.data(), amps, m * sizeof(float2), hipMemcpyDeviceToHost, st));
  HIPCHECK(hipMemcpyAsync(h, sums, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHECK(hipStreamSynchronize(st));
  mp->pool.put(amps, st);
  mp->pool.put(sums, st);
  std::memcpy(out_c64, ha.data(), m * sizeof(float2));
  if (out_stats) {
    const int n = mp->circ.n;
    out_stats[0] = h[0];
    out_stats[1] = std::ldexp(h[0] / (double)m, n);
    out_stats[2] = std::ldexp(h[1] / (double)m, 2 * n);
  }
  return QS_OK;
}

}  // extern "C"
