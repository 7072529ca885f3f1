// C ABI of the qs library and the executor of the half-circuit plans.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
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

// Device buffers of a plan, recycled between calls of the same size.
struct Pool {
  struct Ent {
    void* p;
    size_t bytes;
    bool used;
  };
  std::vector<Ent> ents;
  size_t held = 0;
  void* get(size_t bytes) {
    if (bytes == 0) bytes = 256;
    Ent* best = nullptr;
    for (Ent& e : ents)
      if (!e.used && e.bytes >= bytes && (!best || e.bytes < best->bytes)) best = &e;
    if (best && best->bytes <= 2 * bytes + (1 << 20)) {
      best->used = true;
      return best->p;
    }
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      // release idle buffers and retry once
      trim();
      if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
      }
    }
    ents.push_back(Ent{p, bytes, true});
    held += bytes;
    return p;
  }
  void put(void* p) {
    for (Ent& e : ents)
      if (e.p == p) e.used = false;
  }
  void trim() {
    std::vector<Ent> keep;
    for (Ent& e : ents) {
      if (e.used) keep.push_back(e);
      else {
        (void)hipFree(e.p);
        held -= e.bytes;
      }
    }
    ents.swap(keep);
  }
  void release_all() {
    for (Ent& e : ents) (void)hipFree(e.p);
    ents.clear();
    held = 0;
  }
};

struct BlockRes {
  uint64_t k0 = 0, k1 = 0;
  float2* X[2] = {nullptr, nullptr};  // [K_b][S_side]
};

}  // namespace

struct qs_circuit {
  Circuit c;
};

struct qs_plan {
  Circuit circ;
  uint64_t upper_mask = 0;
  std::vector<Cut> cuts;
  Side side[2];
  qs_options opts{};
  Pool pool;
  bool registered = false;
  std::vector<uint64_t> bits;
  std::vector<uint32_t> vals[2];
  std::vector<int> idx[2];
  uint32_t* d_vals[2] = {nullptr, nullptr};
  std::vector<BlockRes> blocks;
  std::vector<std::pair<uint64_t, uint64_t>> ranges;
  bool timing = false;
  double tms[4] = {0, 0, 0, 0};
  ~qs_plan() { pool.release_all(); }
};

namespace {

#define HIPCHECK(expr)                                                              \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess) return fail(QS_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

int ctz64(uint64_t x) { return x ? __builtin_ctzll(x) : 64; }

PlanKnobs knobs_of(const qs_plan* p, int S) {
  PlanKnobs k;
  if (p->opts.tile_bits > 0) k.tile_bits = std::min(p->opts.tile_bits, 13);
  if (p->opts.coalesce_bits > 0) k.coalesce_bits = p->opts.coalesce_bits;
  if (p->opts.tail_max_qubits > 0) k.tail_max_qubits = std::min(p->opts.tail_max_qubits, 10);
  k.force_lstar = p->opts.materialize_level;
  k.mem_budget = p->opts.mem_budget;
  if (k.mem_budget == 0) {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) == hipSuccess) k.mem_budget = (size_t)(0.85 * (double)fr);
  }
  k.S = S;
  return k;
}

struct Timer {
  bool on;
  hipStream_t st;
  hipEvent_t a = nullptr, b = nullptr;
  double* slot;
  Timer(bool on_, hipStream_t s, double* sl) : on(on_), st(s), slot(sl) {
    if (on) {
      (void)hipEventCreate(&a);
      (void)hipEventCreate(&b);
      (void)hipEventRecord(a, st);
    }
  }
  ~Timer() {
    if (on) {
      (void)hipEventRecord(b, st);
      (void)hipEventSynchronize(b);
      float ms = 0;
      (void)hipEventElapsedTime(&ms, a, b);
      *slot += ms;
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
    }
  }
};

// Run one side of one block: passes for the materialised levels, then the
// leaf evaluation into X[k][s].
qs_status run_side(qs_plan* P, int sidx, const Block& blk, float2* X, hipStream_t st) {
  const Side& s = P->side[sidx];
  const int c = (int)P->cuts.size();
  const int S = (int)P->vals[sidx].size();
  SidePlan sp;
  std::string err;
  if (!plan_side(s, c, blk, knobs_of(P, S), sp, err)) return fail(QS_ERR_UNSUPPORTED, err);
  const Tree& tr = sp.tree;
  const int L = (int)tr.levels.size() - 1;
  if (L - sp.lstar > kMaxTailLevels) return fail(QS_ERR_UNSUPPORTED, "too many leaf levels");
  if ((int)tr.end_cuts.size() > 2 * kMaxBranch) return fail(QS_ERR_UNSUPPORTED, "too many end cuts");
  auto cut_qubit = [&](int j) {
    const Cut& k = P->cuts[j];
    int g = s.upper ? k.upper : k.lower;
    return (int)(std::find(s.qubits.begin(), s.qubits.end(), g) - s.qubits.begin());
  };
  // ---- descriptors
  std::vector<PassDesc> pds;
  std::vector<DevOp> ops;
  for (const PassPlan& pp : sp.passes) {
    PassDesc d{};
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
    d.op_in = (int)ops.size();
    if (!encode_ops(s, pp.ops_in, tr.fixed, work_of, ops, err)) return fail(QS_ERR_UNSUPPORTED, err);
    d.n_in = (int)ops.size() - d.op_in;
    d.op_out = (int)ops.size();
    if (!encode_ops(s, pp.ops_out, tr.fixed, work_of, ops, err)) return fail(QS_ERR_UNSUPPORTED, err);
    d.n_out = (int)ops.size() - d.op_out;
    d.m = 0;
    if (pp.branch) {
      const Level& nx = tr.levels[pp.level_in + 1];
      d.m = (int)nx.cuts.size();
      for (int i = 0; i < d.m; ++i) d.bq[i] = cut_qubit(nx.cuts[i]);
    }
    d.upper = s.upper ? 1 : 0;
    pds.push_back(d);
  }
  TailDesc td{};
  td.n = s.n;
  td.q = (int)sp.Q.size();
  std::vector<int> work_q(s.n, -1);
  for (int i = 0; i < td.q; ++i) {
    td.Q[i] = sp.Q[i];
    work_q[sp.Q[i]] = i;
  }
  td.nlev = L - sp.lstar;
  std::vector<DevOp> tops;
  for (int l = sp.lstar + 1; l <= L; ++l) {
    TailLevel& tl = td.lev[l - sp.lstar - 1];
    const Level& lv = tr.levels[l];
    tl.m = (int)lv.cuts.size();
    for (int i = 0; i < tl.m; ++i) {
      tl.bq[i] = cut_qubit(lv.cuts[i]);
      tl.kbit[i] = 1ULL << (c - 1 - lv.cuts[i]);
    }
    tl.op0 = (int)(ops.size() + tops.size());
    size_t before = tops.size();
    if (!encode_ops(s, lv.ops, tr.fixed, work_q, tops, err)) return fail(QS_ERR_UNSUPPORTED, err);
    tl.nops = (int)(tops.size() - before);
  }
  td.n_end = (int)tr.end_cuts.size();
  for (int i = 0; i < td.n_end; ++i) {
    td.eq[i] = cut_qubit(tr.end_cuts[i]);
    td.ekbit[i] = 1ULL << (c - 1 - tr.end_cuts[i]);
  }
  td.upper = s.upper ? 1 : 0;
  td.n_nodes = (int)sp.nodes[sp.lstar];
  td.S = S;
  td.ldx = S;
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
  // ---- upload (one buffer)
  const size_t b_pd = pds.size() * sizeof(PassDesc);
  const size_t b_td = sizeof(TailDesc);
  const size_t b_ops = std::max<size_t>(1, ops.size()) * sizeof(DevOp);
  const size_t b_nk = node_k.size() * sizeof(uint64_t);
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t total = al(b_pd) + al(b_td) + al(b_ops) + al(b_nk);
  std::vector<char> host(total, 0);
  size_t o_pd = 0, o_td = al(b_pd), o_ops = o_td + al(b_td), o_nk = o_ops + al(b_ops);
  if (b_pd) std::memcpy(host.data() + o_pd, pds.data(), b_pd);
  std::memcpy(host.data() + o_td, &td, b_td);
  if (!ops.empty()) std::memcpy(host.data() + o_ops, ops.data(), ops.size() * sizeof(DevOp));
  std::memcpy(host.data() + o_nk, node_k.data(), b_nk);
  char* dev = (char*)P->pool.get(total);
  if (!dev) return fail(QS_ERR_OOM, "descriptor buffer");
  HIPCHECK(hipMemcpyAsync(dev, host.data(), total, hipMemcpyHostToDevice, st));
  HIPCHECK(hipStreamSynchronize(st));
  // ---- passes
  const size_t SB = (size_t)8 << s.n;
  float2* cur = nullptr;
  uint64_t cur_nodes = 0;
  {
    Timer tm(P->timing, st, &P->tms[0]);
    for (size_t pi = 0; pi < sp.passes.size(); ++pi) {
      const PassPlan& pp = sp.passes[pi];
      const PassDesc* dd = (const PassDesc*)(dev + o_pd) + pi;
      if (pp.init) {
        cur_nodes = 1;
        cur = (float2*)P->pool.get(SB);
        if (!cur) return fail(QS_ERR_OOM, "root state");
      }
      if (pp.branch) {
        const uint64_t on = sp.nodes[pp.level_in + 1];
        float2* nxt = (float2*)P->pool.get(SB * on);
        if (!nxt) return fail(QS_ERR_OOM, "tree level states");
        HIPCHECK(launch_pass(pds[pi], dd, (const DevOp*)(dev + o_ops), cur, nxt, cur_nodes, st));
        P->pool.put(cur);
        cur = nxt;
        cur_nodes = on;
      } else {
        HIPCHECK(launch_pass(pds[pi], dd, (const DevOp*)(dev + o_ops), cur, cur, cur_nodes, st));
      }
    }
  }
  {
    Timer tm(P->timing, st, &P->tms[1]);
    HIPCHECK(launch_tail(td, (const TailDesc*)(dev + o_td), (const DevOp*)(dev + o_ops), cur,
                         P->d_vals[sidx], (const uint64_t*)(dev + o_nk), X, st));
  }
  // the stream orders later users of these buffers after the kernels above
  P->pool.put(cur);
  P->pool.put(dev);
  return QS_OK;
}

qs_status register_bits(qs_plan* P, const uint64_t* bits, size_t m) {
  const int n = P->circ.n;
  const uint64_t full = n == 64 ? ~0ULL : ((1ULL << n) - 1);
  for (size_t t = 0; t < m; ++t)
    if (bits[t] & ~full) return fail(QS_ERR_ARG, "bitstring has bits set beyond the qubit count");
  if (P->registered) {
    if (m != P->bits.size() || std::memcmp(bits, P->bits.data(), m * 8) != 0)
      return fail(QS_ERR_STATE, "bitstrings differ from the registered set");
    return QS_OK;
  }
  P->bits.assign(bits, bits + m);
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
    P->vals[sidx] = u;
    P->idx[sidx].resize(m);
    for (size_t t = 0; t < m; ++t)
      P->idx[sidx][t] = (int)(std::lower_bound(u.begin(), u.end(), hv[t]) - u.begin());
  }
  const double prod = (double)P->vals[0].size() * (double)P->vals[1].size();
  if (prod > 4.0 * (double)m + 1024.0)
    return fail(QS_ERR_UNSUPPORTED, "bitstrings are not close to a product set of upper x lower values");
  for (int sidx = 0; sidx < 2; ++sidx) {
    const size_t bytes = P->vals[sidx].size() * sizeof(uint32_t);
    P->d_vals[sidx] = (uint32_t*)P->pool.get(bytes);
    if (!P->d_vals[sidx]) return fail(QS_ERR_OOM, "value table");
    HIPCHECK(hipMemcpy(P->d_vals[sidx], P->vals[sidx].data(), bytes, hipMemcpyHostToDevice));
  }
  P->registered = true;
  return QS_OK;
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
  if (n_gates) *n_gates = (int)circ->c.gates.size();
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
  std::string err;
  if (!build_partition(p->circ, upper_mask, p->cuts, p->side[0], p->side[1], err))
    return fail(QS_ERR_ARG, err);
  if (p->side[0].n > 32 || p->side[1].n > 32) return fail(QS_ERR_ARG, "a half has more than 32 qubits");
  if (p->cuts.size() > 40) return fail(QS_ERR_UNSUPPORTED, "more than 40 cut gates");
  *out = p.release();
  return QS_OK;
}

qs_status qs_plan_info(const qs_plan* plan, int* n_upper, int* n_lower, int* n_cuts) {
  if (!plan) return fail(QS_ERR_ARG, "null plan");
  if (n_upper) *n_upper = plan->side[0].n;
  if (n_lower) *n_lower = plan->side[1].n;
  if (n_cuts) *n_cuts = (int)plan->cuts.size();
  return QS_OK;
}

qs_status qs_plan_dump(const qs_plan* plan, char* buf, size_t cap, size_t* needed) {
  if (!plan || (!buf && cap)) return fail(QS_ERR_ARG, "null pointer");
  const int c = (int)plan->cuts.size();
  Block blk;
  SidePlan sp[2];
  bool ok[2];
  std::string err;
  for (int k = 0; k < 2; ++k) {
    PlanKnobs kn;
    if (plan->opts.tile_bits > 0) kn.tile_bits = std::min(plan->opts.tile_bits, 13);
    if (plan->opts.coalesce_bits > 0) kn.coalesce_bits = plan->opts.coalesce_bits;
    if (plan->opts.tail_max_qubits > 0) kn.tail_max_qubits = std::min(plan->opts.tail_max_qubits, 10);
    kn.force_lstar = plan->opts.materialize_level;
    kn.mem_budget = plan->opts.mem_budget;
    kn.S = plan->registered ? (int)plan->vals[k].size() : 1024;
    ok[k] = plan_side(plan->side[k], c, blk, kn, sp[k], err);
  }
  std::string js = dump_json(plan->circ, plan->upper_mask, plan->cuts, plan->side[0],
                             plan->side[1], ok[0] ? &sp[0] : nullptr, ok[1] ? &sp[1] : nullptr);
  if (needed) *needed = js.size() + 1;
  if (cap) {
    size_t nb = std::min(cap - 1, js.size());
    std::memcpy(buf, js.data(), nb);
    buf[nb] = '\0';
  }
  return QS_OK;
}

void qs_plan_free(qs_plan* plan) { delete plan; }

qs_status qs_plan_reset(qs_plan* plan) {
  if (!plan) return fail(QS_ERR_ARG, "null plan");
  (void)hipDeviceSynchronize();
  for (BlockRes& b : plan->blocks)
    for (int k = 0; k < 2; ++k) plan->pool.put(b.X[k]);
  plan->blocks.clear();
  plan->ranges.clear();
  for (int k = 0; k < 2; ++k) {
    if (plan->d_vals[k]) plan->pool.put(plan->d_vals[k]);
    plan->d_vals[k] = nullptr;
    plan->vals[k].clear();
    plan->idx[k].clear();
  }
  plan->bits.clear();
  plan->registered = false;
  return QS_OK;
}

qs_status qs_run_halves(qs_plan* plan, uint64_t copy_begin, uint64_t copy_end,
                        const uint64_t* bitstrings, size_t m, void* hip_stream) {
  if (!plan || !bitstrings) return fail(QS_ERR_ARG, "null pointer");
  if (m == 0) return fail(QS_ERR_ARG, "no bitstrings");
  const int c = (int)plan->cuts.size();
  const uint64_t total = 1ULL << c;
  if (copy_begin >= copy_end || copy_end > total) return fail(QS_ERR_ARG, "copy range outside [0, 2^c)");
  for (auto& r : plan->ranges)
    if (copy_begin < r.second && r.first < copy_end) return fail(QS_ERR_STATE, "copy range already run");
  qs_status s = register_bits(plan, bitstrings, m);
  if (s != QS_OK) return s;
  hipStream_t st = (hipStream_t)hip_stream;
  uint64_t k = copy_begin;
  while (k < copy_end) {
    int sz = std::min(ctz64(k), c);
    while (sz > 0 && k + (1ULL << sz) > copy_end) --sz;
    Block blk;
    blk.k0 = k;
    blk.p = c - sz;
    BlockRes br;
    br.k0 = k;
    br.k1 = k + (1ULL << sz);
    const uint64_t Kb = 1ULL << sz;
    for (int sidx = 0; sidx < 2; ++sidx) {
      const size_t bytes = Kb * plan->vals[sidx].size() * sizeof(float2);
      br.X[sidx] = (float2*)plan->pool.get(bytes);
      if (!br.X[sidx]) return fail(QS_ERR_OOM, "gathered half amplitudes");
      s = run_side(plan, sidx, blk, br.X[sidx], st);
      if (s != QS_OK) return s;
    }
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
  if (!plan->registered || plan->blocks.empty()) {
    if (plan->registered && (m != plan->bits.size() || std::memcmp(bitstrings, plan->bits.data(), m * 8)))
      return fail(QS_ERR_STATE, "bitstrings differ from the registered set");
    qs_status s = qs_run_halves(plan, 0, 1ULL << plan->cuts.size(), bitstrings, m, hip_stream);
    if (s != QS_OK) return s;
  } else {
    if (m != plan->bits.size() || std::memcmp(bitstrings, plan->bits.data(), m * 8) != 0)
      return fail(QS_ERR_STATE, "bitstrings differ from the registered set");
  }
  const int M = (int)plan->vals[0].size(), N = (int)plan->vals[1].size();
  float2* C = (float2*)plan->pool.get((size_t)M * N * sizeof(float2));
  float2* amps = (float2*)plan->pool.get(m * sizeof(float2));
  int* d_iu = (int*)plan->pool.get(m * sizeof(int));
  int* d_il = (int*)plan->pool.get(m * sizeof(int));
  const int nb = prob_partial_blocks(m);
  double* d_part = (double*)plan->pool.get((2 * (size_t)nb + 2) * sizeof(double));
  if (!C || !amps || !d_iu || !d_il || !d_part) return fail(QS_ERR_OOM, "assembly buffers");
  HIPCHECK(hipMemcpyAsync(d_iu, plan->idx[0].data(), m * sizeof(int), hipMemcpyHostToDevice, st));
  HIPCHECK(hipMemcpyAsync(d_il, plan->idx[1].data(), m * sizeof(int), hipMemcpyHostToDevice, st));
  {
    Timer tm(plan->timing, st, &plan->tms[2]);
    void* work = nullptr;
    bool first = true;
    for (BlockRes& b : plan->blocks) {
      const int K = (int)(b.k1 - b.k0);
      if (prec == QS_PREC_FP32) {
        HIPCHECK(launch_zgemm_tn_f32(M, N, K, b.X[0], M, b.X[1], N, C, N, first ? 0 : 1, st));
      } else {
        const size_t wb = split_bf16_workspace_bytes(M, N, K);
        work = plan->pool.get(wb);
        if (!work) return fail(QS_ERR_OOM, "split-bf16 workspace");
        HIPCHECK(launch_zgemm_tn_split_bf16(M, N, K, b.X[0], M, b.X[1], N, C, N, first ? 0 : 1, work, st));
        plan->pool.put(work);
      }
      first = false;
    }
  }
  {
    Timer tm(plan->timing, st, &plan->tms[3]);
    HIPCHECK(launch_gather_amps(C, N, d_iu, d_il, m, amps, st));
    HIPCHECK(launch_prob_sums(amps, m, d_part, d_part + 2 * nb, st));
  }
  HIPCHECK(hipMemcpyAsync(out_c64, amps, m * sizeof(float2), hipMemcpyDeviceToHost, st));
  double sums[2];
  HIPCHECK(hipMemcpyAsync(sums, d_part + 2 * nb, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHECK(hipStreamSynchronize(st));
  if (out_stats) {
    const double n = plan->circ.n;
    out_stats[0] = sums[0];
    out_stats[1] = std::ldexp(sums[0] / (double)m, (int)n);
    out_stats[2] = std::ldexp(sums[1] / (double)m, (int)(2 * n));
  }
  plan->pool.put(C);
  plan->pool.put(amps);
  plan->pool.put(d_iu);
  plan->pool.put(d_il);
  plan->pool.put(d_part);
  return QS_OK;
}

qs_status qs_get_timing(const qs_plan* plan, double* out4) {
  if (!plan || !out4) return fail(QS_ERR_ARG, "null pointer");
  for (int i = 0; i < 4; ++i) out4[i] = plan->tms[i];
  return QS_OK;
}

qs_status qs_set_timing(qs_plan* plan, int enable) {
  if (!plan) return fail(QS_ERR_ARG, "null plan");
  plan->timing = enable != 0;
  for (int i = 0; i < 4; ++i) plan->tms[i] = 0;
  return QS_OK;
}

}  // extern "C"
