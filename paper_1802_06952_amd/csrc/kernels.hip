// HIP kernels of the qs library (gfx950, wave64).
//
//  k_pass      full-state pass over LDS tiles: gates of a tree level, branch
//              into the children of a cut level (Sec. 2.1, Eq. 1; Sec. 2.3.2),
//              diagonal gates folded into one phase multiply (Sec. 2.4, Eq. 3-6).
//  k_tail      leaf levels evaluated at the requested half values only.
//  k_zgemm_*   amplitude assembly: amp(u, l) = sum_k U_k[u] L_k[l] (Sec. 2.3.1).
//  k_prob_*    FP64 sums of |amp|^2 and |amp|^4 (the statistics of Sec. 3, Eq. 7).
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <algorithm>
#include <map>
#include <mutex>

#include "kernels.h"

namespace qs {

typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// omega^e with omega = (1+i)/sqrt 2, e taken mod 8.
__device__ __forceinline__ float2 omega_pow(int e) {
  const float r = 0.70710678118654752f;
  const bool odd = e & 1;
  float x = odd ? r : 1.0f, y = odd ? r : 0.0f;
  const int q = (e >> 1) & 3;
  float xr = x, yr = y;
  if (q == 1) { xr = -y; yr = x; }
  if (q == 2) { xr = -x; yr = -y; }
  if (q == 3) { xr = y; yr = -x; }
  return make_float2(xr, yr);
}

// Fused diagonal factor of a DIAG op at state index x (halves have <= 32 qubits).
__device__ __forceinline__ float2 diag_apply(const DevOp& op, uint32_t x, float2 v) {
  int e = __popc(x & (uint32_t)op.t0) + 2 * __popc(x & (uint32_t)op.t1) +
          4 * __popc(x & (uint32_t)op.t2);
  int par = 0;
  for (int i = 0; i < op.nd; ++i) par += __popc(x & (x >> op.d[i]) & (uint32_t)op.M[i]);
  e += 4 * par;
  if ((x & (uint32_t)op.pmask) != (uint32_t)op.pval) return make_float2(0.f, 0.f);
  if ((e & 7) == 0) return v;
  return cmul(v, omega_pow(e));
}

__device__ __forceinline__ void mat_apply(const float* m, float2 a, float2 b, float2& oa, float2& ob) {
  oa = make_float2(m[0] * a.x - m[1] * a.y + m[2] * b.x - m[3] * b.y,
                   m[0] * a.y + m[1] * a.x + m[2] * b.y + m[3] * b.x);
  ob = make_float2(m[4] * a.x - m[5] * a.y + m[6] * b.x - m[7] * b.y,
                   m[4] * a.y + m[5] * a.x + m[6] * b.y + m[7] * b.x);
}

// The unit-entry gates (MatKind) on a pair (a0, a1) = amplitudes with the
// target bit 0 and 1: out0 = m00 a0 + m01 a1, out1 = m10 a0 + m11 a1, all
// entries 0, +-1, +-i, so additions only.
template <int MK>
__device__ __forceinline__ void unit_pair(float2& a0, float2& a1) {
  const float2 x = a0, y = a1;
  if constexpr (MK == MK_X) {  // [[1, -i], [-i, 1]]
    a0 = make_float2(x.x + y.y, x.y - y.x);
    a1 = make_float2(x.y + y.x, y.y - x.x);
  } else if constexpr (MK == MK_Y) {  // [[1, -1], [1, 1]]
    a0 = make_float2(x.x - y.x, x.y - y.y);
    a1 = make_float2(x.x + y.x, x.y + y.y);
  } else if constexpr (MK == MK_YT) {  // [[1, 1], [-1, 1]]
    a0 = make_float2(x.x + y.x, x.y + y.y);
    a1 = make_float2(y.x - x.x, y.y - x.y);
  } else {  // MK_H: [[1, 1], [1, -1]]
    a0 = make_float2(x.x + y.x, x.y + y.y);
    a1 = make_float2(x.x - y.x, x.y - y.y);
  }
}

// Register-pair 2x2 gate: pairs (r, r | 2^rb) of a per-lane register array.
template <int R>
__device__ __forceinline__ void tail_mat_reg_m(float2 (&v)[R], const float* m, int rb) {
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if (r & (1 << rb)) continue;
    const int r1 = r | (1 << rb);
    float2 oa, ob;
    mat_apply(m, v[r], v[r1], oa, ob);
    v[r] = oa;
    v[r1] = ob;
  }
}

template <int R, int MK>
__device__ __forceinline__ void tail_mat_reg_u(float2 (&v)[R], int rb) {
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if (r & (1 << rb)) continue;
    unit_pair<MK>(v[r], v[r | (1 << rb)]);
  }
}

template <int R>
__device__ __forceinline__ void tail_mat_reg(float2 (&v)[R], const DevOp& op, int rb) {
  switch (__builtin_amdgcn_readfirstlane(op.mk)) {
    case MK_X: tail_mat_reg_u<R, MK_X>(v, rb); break;
    case MK_Y: tail_mat_reg_u<R, MK_Y>(v, rb); break;
    case MK_YT: tail_mat_reg_u<R, MK_YT>(v, rb); break;
    case MK_H: tail_mat_reg_u<R, MK_H>(v, rb); break;
    default: tail_mat_reg_m<R>(v, op.m, rb); break;
  }
}

// ------------------------------------------------------------------ full-state pass

constexpr int kPassThreads = 256;

__device__ __forceinline__ uint32_t deposit_tile(uint32_t i, const int* tbit, int t) {
  uint32_t x = 0;
  for (int k = 0; k < t; ++k) x |= ((i >> k) & 1u) << tbit[k];
  return x;
}

__device__ void lds_apply_ops(float2* L, const DevOp* __restrict__ ops, int nops, int t,
                              const int* tbit, uint32_t outer) {
  const int size = 1 << t;
  for (int o = 0; o < nops; ++o) {
    const DevOp& op = ops[o];
    if (op.kind == 0) {
      const int j = op.target;
      const uint32_t lowm = (1u << j) - 1;
      for (int p = threadIdx.x; p < size / 2; p += kPassThreads) {
        const uint32_t i0 = ((p & ~lowm) << 1) | (p & lowm);
        const uint32_t i1 = i0 | (1u << j);
        float2 a = L[i0], b = L[i1], oa, ob;
        mat_apply(op.m, a, b, oa, ob);
        L[i0] = oa;
        L[i1] = ob;
      }
    } else {
      for (int i = threadIdx.x; i < size; i += kPassThreads) {
        const uint32_t x = outer | deposit_tile(i, tbit, t);
        L[i] = diag_apply(op, x, L[i]);
      }
    }
    __syncthreads();
  }
}

// Child tile of an LDS pass: dst = the cut factors of branch b (m cut bits on
// state bits bq, MSB first) applied to src.
__device__ void lds_child(float2* dst, const float2* src, const int* bq, int m, int b, int upper,
                          int t, const int* tbit, uint32_t outer) {
  const int size = 1 << t;
  for (int i = threadIdx.x; i < size; i += kPassThreads) {
    const uint32_t x = outer | deposit_tile(i, tbit, t);
    float2 v = src[i];
    for (int k = 0; k < m; ++k) {
      const uint32_t want = (b >> (m - 1 - k)) & 1;
      const uint32_t xb = (x >> bq[k]) & 1;
      if (upper) {
        if (xb != want) v = make_float2(0.f, 0.f);
      } else if (want & xb) {
        v = make_float2(-v.x, -v.y);
      }
    }
    dst[i] = v;
  }
  __syncthreads();
}

__device__ void lds_store(float2* dst, const float2* L, float sc, int t, const int* tbit,
                          uint32_t outer) {
  for (int i = threadIdx.x; i < (1 << t); i += kPassThreads) {
    const uint32_t x = outer | deposit_tile(i, tbit, t);
    dst[x] = make_float2(L[i].x * sc, L[i].y * sc);
  }
  __syncthreads();
}

__global__ void __launch_bounds__(kPassThreads)
k_pass(const PassDesc* __restrict__ pdp, const DevOp* __restrict__ ops,
       const float2* __restrict__ in, float2* __restrict__ out) {
  extern __shared__ float2 smem[];  // 1 + ns tiles
  __shared__ int tbit[kMaxTileBits];
  const PassDesc& P = *pdp;
  const int t = P.t;
  const int size = 1 << t;
  if (threadIdx.x < kMaxTileBits) tbit[threadIdx.x] = P.tbit[threadIdx.x];
  const uint64_t blk = blockIdx.x;
  const uint64_t tile = blk & ((1ull << P.n_outer) - 1);
  const uint64_t node = blk >> P.n_outer;
  uint32_t outer = 0;
  for (int j = 0; j < P.n_outer; ++j) outer |= (uint32_t)((tile >> j) & 1) << P.obit[j];
  const uint64_t N = 1ull << P.n;
  __syncthreads();
  float2* A = smem;
  for (int i = threadIdx.x; i < size; i += kPassThreads) {
    const uint32_t x = outer | deposit_tile(i, tbit, t);
    float2 v;
    if (P.init) {
      v = ((x & ~(uint32_t)P.hinit) == 0) ? make_float2(P.hamp, 0.f) : make_float2(0.f, 0.f);
    } else {
      v = in[node * N + x];
    }
    A[i] = v;
  }
  __syncthreads();
  const DevOp* pops = ops + P.op_in;
  lds_apply_ops(A, pops, P.n_in, t, tbit, outer);
  const float sc = P.scale;
  const int ns = P.ns;
  if (ns == 0) {
    lds_store(out + node * N, A, sc, t, tbit, outer);
    return;
  }
  const int m1 = P.sm[0];
  const int m2 = ns > 1 ? P.sm[1] : 0;
  float2* B1 = smem + size;
  float2* B2 = smem + 2 * size;
  for (int b1 = 0; b1 < (1 << m1); ++b1) {
    lds_child(B1, A, P.sbq[0], m1, b1, P.upper, t, tbit, outer);
    lds_apply_ops(B1, pops + P.sop[0], P.snops[0], t, tbit, outer);
    const uint64_t c1 = (node << m1) | (uint64_t)b1;
    if (ns == 1) {
      lds_store(out + c1 * N, B1, sc, t, tbit, outer);
      continue;
    }
    for (int b2 = 0; b2 < (1 << m2); ++b2) {
      lds_child(B2, B1, P.sbq[1], m2, b2, P.upper, t, tbit, outer);
      lds_apply_ops(B2, pops + P.sop[1], P.snops[1], t, tbit, outer);
      lds_store(out + ((c1 << m2) | (uint64_t)b2) * N, B2, sc, t, tbit, outer);
    }
  }
}

// Cut factors of branch b over m cut bits (bit k of the branch = (b >> (m-1-k)) & 1
// acts on state bit bq[k]): an amplitude x survives iff (x & cmask) == cval and
// is negated iff popc(x & zmask) is odd.  Upper half: P_b on each cut qubit;
// two cuts on one qubit with different bits give P0 P1 = 0 (cval gets a bit
// outside cmask, so nothing survives).  Lower half: Z^b, and Z^b0 Z^b1 on one
// qubit is Z^(b0 xor b1).
__device__ __forceinline__ void cut_factors(const int* bq, int m, int b, int upper,
                                            uint32_t& cmask, uint32_t& cval, uint32_t& zmask) {
  cmask = 0;
  cval = 0;
  zmask = 0;
  bool never = false;
  for (int k = 0; k < m; ++k) {
    const uint32_t want = (b >> (m - 1 - k)) & 1;
    const uint32_t qb = 1u << bq[k];
    if (upper) {
      if ((cmask & qb) && (((cval & qb) != 0) != (want != 0))) never = true;
      cmask |= qb;
      if (want) cval |= qb;
    } else if (want) {
      zmask ^= qb;
    }
  }
  if (never) {
    cmask = 0;
    cval = 1;  // (x & 0) == 1 never holds
  }
}

// ------------------------------------------------------------------ wave-tile pass
//
// One wavefront owns a tile of 64 x 2^R amplitudes: lane l holds the state
// bits 0..5 = l (so every register load or store is one contiguous 512-byte
// run), register r holds the R state bits tbit[6..6+R-1] = bits of r.  Gates
// on state bits 0..5 exchange partners with lane shuffles; gates on register
// bits stay inside the lane; diagonal ops need only the index.  No LDS and
// no barriers.

constexpr int kWaveThreads = 256;

// omega^e for e = 0..7 at entry e, and 0 at entry 8, in LDS: a DIAG op reads
// its factor at byte offset 8 (e mod 8), or 64 where the projector fails.
constexpr int kPhaseEntries = 9;

__device__ __forceinline__ void init_phase_table(float2* tab) {
  if (threadIdx.x == 0) {
    const float r = 0.70710678118654752f;
    tab[0] = make_float2(1.f, 0.f);
    tab[1] = make_float2(r, r);
    tab[2] = make_float2(0.f, 1.f);
    tab[3] = make_float2(-r, r);
    tab[4] = make_float2(-1.f, 0.f);
    tab[5] = make_float2(-r, -r);
    tab[6] = make_float2(0.f, -1.f);
    tab[7] = make_float2(r, -r);
    tab[8] = make_float2(0.f, 0.f);
  }
  __syncthreads();
}

__device__ __forceinline__ float uniform_f(float x) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}

// Lane-pair 2x2 gate from the matrix entries m[] (any 2x2 matrix).
template <int R>
__device__ __forceinline__ void lane_mat_m(float2 (&v)[R], const DevOp& op, int w, bool bit) {
  float m[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) m[i] = uniform_f(op.m[i]);
  const float sr = bit ? m[6] : m[0], si = bit ? m[7] : m[1];
  const float pr = bit ? m[4] : m[2], pi = bit ? m[5] : m[3];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const float px = __shfl_xor(v[r].x, 1 << w);
    const float py = __shfl_xor(v[r].y, 1 << w);
    const float2 a = v[r];
    v[r] = make_float2(sr * a.x - si * a.y + pr * px - pi * py,
                       sr * a.y + si * a.x + pr * py + pi * px);
  }
}

// Lane-pair 2x2 gate on lane bit w: bit = this lane's value of the target
// bit, p = the partner lane's amplitude.  Unit-entry kinds: X gives
// a - i p on both sides; Y gives a -+ p; its transpose a +- p; H +-a + p.
template <int R>
__device__ __forceinline__ void lane_mat(float2 (&v)[R], const DevOp& op, int w, bool bit) {
  const int mk = __builtin_amdgcn_readfirstlane(op.mk);
  if (mk == MK_X) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const float px = __shfl_xor(v[r].x, 1 << w);
      const float py = __shfl_xor(v[r].y, 1 << w);
      v[r] = make_float2(v[r].x + py, v[r].y - px);
    }
  } else if (mk == MK_Y || mk == MK_YT) {
    const float sg = (bit == (mk == MK_Y)) ? 1.f : -1.f;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const float px = __shfl_xor(v[r].x, 1 << w);
      const float py = __shfl_xor(v[r].y, 1 << w);
      v[r] = make_float2(fmaf(sg, px, v[r].x), fmaf(sg, py, v[r].y));
    }
  } else if (mk == MK_H) {
    const float sg = bit ? -1.f : 1.f;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const float px = __shfl_xor(v[r].x, 1 << w);
      const float py = __shfl_xor(v[r].y, 1 << w);
      v[r] = make_float2(fmaf(sg, v[r].x, px), fmaf(sg, v[r].y, py));
    }
  } else {
    lane_mat_m<R>(v, op, w, bit);
  }
}

template <int R>
__device__ __forceinline__ uint32_t reg_index(int r, const uint32_t (&RB)[R]) {
  uint32_t d = 0;
#pragma unroll
  for (int k = 0; k < R; ++k)
    if ((r >> k) & 1) d |= RB[k];
  return d;
}

// A DIAG op on the 2^NB registers of a lane: index of register r is
// F | sum_k r_k RB[k], with F fixed per lane.  The exponent of F is taken
// once, then each register's by adding one register bit at a time (the
// register split of the op); it is kept as 8 e, the byte offset of omega^e in
// the phase table, where a failed projector points at the zero entry.
template <int NB>
__device__ __forceinline__ void diag_offsets(uint32_t (&off)[1 << NB], const DevOp& op, uint32_t F,
                                             const uint32_t (&RB)[NB > 0 ? NB : 1]) {
  constexpr int E = 1 << NB;
  // every field of the op is the same in all lanes: read into scalar registers
  const auto su = [](uint32_t x) { return (uint32_t)__builtin_amdgcn_readfirstlane(x); };
  // (the masks used once per op stay in vector registers: moving each into a
  // scalar register would cost one more vector instruction than it saves)
  int eF = __popc(F & (uint32_t)op.t0) + 2 * __popc(F & (uint32_t)op.t1) +
           4 * __popc(F & (uint32_t)op.t2);
  const int nd = __builtin_amdgcn_readfirstlane(op.nd);
  for (int i = 0; i < nd; ++i)
    eF += 4 * __popc(F & (F >> (uint32_t)op.d[i]) & (uint32_t)op.M[i]);
  int ex[E];
  ex[0] = eF << 3;
  if constexpr (NB > 0) {
    int wk[NB];
    uint32_t rr[NB];
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      wk[k] = (op.wl[k] + 4 * __popc(F & op.cross[k])) << 3;
      rr[k] = su(op.rr[k]);
    }
#pragma unroll
    for (int r = 1; r < E; ++r) {
      const int top = 31 - __builtin_clz((unsigned)r);
      const int low = r ^ (1 << top);
      ex[r] = ex[low] + wk[top] + 32 * __popc(rr[top] & (uint32_t)low);
    }
  }
#pragma unroll
  for (int r = 0; r < E; ++r) off[r] = (uint32_t)ex[r] & 56u;
  if (__builtin_amdgcn_readfirstlane((uint32_t)op.pmask) != 0) {
    // (x & pm) == pv splits into the lane's fixed bits and the register bits,
    // whose part is the same in every lane
    const uint32_t pm = su((uint32_t)op.pmask), pv = su((uint32_t)op.pval);
    uint32_t rbm = 0;
#pragma unroll
    for (int k = 0; k < NB; ++k) rbm |= RB[k];
    const bool lane_ok = (F & pm) == (pv & ~rbm);
#pragma unroll
    for (int r = 0; r < E; ++r) {
      uint32_t ri = 0;
#pragma unroll
      for (int k = 0; k < NB; ++k)
        if ((r >> k) & 1) ri |= RB[k];
      const bool reg_ok = (ri & pm) == (pv & rbm);
      if (!(lane_ok && reg_ok)) off[r] = 8u * (kPhaseEntries - 1);
    }
  }
}

template <int NB>
__device__ __forceinline__ void diag_regs(float2 (&v)[1 << NB], const DevOp& op, uint32_t F,
                                          const uint32_t (&RB)[NB > 0 ? NB : 1],
                                          const float2* tab) {
  constexpr int E = 1 << NB;
  uint32_t off[E];
  diag_offsets<NB>(off, op, F, RB);
#pragma unroll
  for (int r = 0; r < E; ++r) v[r] = cmul(v[r], *(const float2*)((const char*)tab + off[r]));
}

template <int R>
__device__ __forceinline__ void wave_apply_ops(float2 (&v)[1 << R], const DevOp* __restrict__ ops,
                                               int nops, uint32_t F, const uint32_t (&RB)[R],
                                               int lane, const float2* tab) {
  constexpr int E = 1 << R;
  for (int o = 0; o < nops; ++o) {
    const DevOp& op = ops[o];
    if (__builtin_amdgcn_readfirstlane(op.kind) == 0) {
      const int w = __builtin_amdgcn_readfirstlane(op.target);
      if (w < 6) {
        lane_mat<E>(v, op, w, (lane >> w) & 1);
      } else {
        const int k = w - 6;
        if constexpr (R >= 1) { if (k == 0) tail_mat_reg<E>(v, op, 0); }
        if constexpr (R >= 2) { if (k == 1) tail_mat_reg<E>(v, op, 1); }
        if constexpr (R >= 3) { if (k == 2) tail_mat_reg<E>(v, op, 2); }
        if constexpr (R >= 4) { if (k == 3) tail_mat_reg<E>(v, op, 3); }
        if constexpr (R >= 5) { if (k == 4) tail_mat_reg<E>(v, op, 4); }
      }
    } else {
      diag_regs<R>(v, op, F, RB, tab);
    }
  }
}

// Index bits of a wave tile: lane l holds the state bits F = xo | l (xo, the
// tile's outer bits, is the same in every lane of the wave) and register r
// adds the bits O_r = sum_k r_k RB[k].  Everything but the lane part is
// wave-uniform, so the address of register r is a scalar base plus 8 l: the
// loads and stores take the base in scalar registers and share one vector
// offset, and conditions on an index split into a lane part and a uniform
// register part.

// Child of a wave tile: the cut factors of branch b (m cut bits on state bits
// bq, MSB first) applied to v.
template <int R>
__device__ __forceinline__ void wave_child(float2 (&w)[1 << R], const float2 (&v)[1 << R],
                                           const int* bq, int m, int b, int upper, uint32_t F,
                                           const uint32_t (&RB)[R]) {
  uint32_t cmask, cval, zmask;
  cut_factors(bq, m, b, upper, cmask, cval, zmask);
  uint32_t rbm = 0;
#pragma unroll
  for (int k = 0; k < R; ++k) rbm |= RB[k];
  // (x & cmask) == cval for x = F | O_r: the lane bits and the register bits separately
  const bool lane_ok = (F & cmask) == (cval & ~rbm);
  const bool lane_neg = __popc(F & zmask) & 1;
#pragma unroll
  for (int r = 0; r < (1 << R); ++r) {
    const uint32_t o = reg_index<R>(r, RB);
    const bool reg_ok = (o & cmask) == (cval & rbm);
    const bool neg = lane_neg != (bool)(__popc(o & zmask) & 1);
    float2 a = v[r];
    if (!(lane_ok && reg_ok)) a = make_float2(0.f, 0.f);
    if (neg) a = make_float2(-a.x, -a.y);
    w[r] = a;
  }
}

// Store of a wave tile, scaled by sc, at row + xo + O_r + lane; nt: streaming
// stores that bypass the caches (the outputs are read again only by the next
// pass or the leaf stage).
template <int R>
__device__ __forceinline__ void wave_store(float2* row, const float2 (&v)[1 << R], float sc,
                                           uint32_t xo, uint32_t lane, const uint32_t (&RB)[R],
                                           int nt) {
  typedef float f32x2 __attribute__((ext_vector_type(2)));
  if (nt) {
#pragma unroll
    for (int r = 0; r < (1 << R); ++r) {
      const f32x2 a = {v[r].x * sc, v[r].y * sc};
      float2* base = row + (xo | reg_index<R>(r, RB));
      __builtin_nontemporal_store(a, (f32x2*)(base + lane));
    }
  } else {
#pragma unroll
    for (int r = 0; r < (1 << R); ++r) {
      float2* base = row + (xo | reg_index<R>(r, RB));
      base[lane] = make_float2(v[r].x * sc, v[r].y * sc);
    }
  }
}

// S = number of branch stages (P.ns).  The pass's ops (n_all of them from
// op_in) are staged in LDS first, so that every wave reads its op stream from
// LDS instead of waiting on a chain of scalar loads per op.
template <int R, int S>
__global__ void __launch_bounds__(kWaveThreads)
k_wpass(const PassDesc* __restrict__ pdp, const DevOp* __restrict__ ops, const float2* in,
        float2* out, uint64_t total_tiles, const uint32_t* __restrict__ tlist, uint32_t n_list) {
  constexpr int E = 1 << R;
  extern __shared__ uint2 wp_ops[];
  __shared__ float2 tab[kPhaseEntries];
  const PassDesc& P = *pdp;
  const uint32_t lane = threadIdx.x & 63;
  const uint64_t wt = (uint64_t)blockIdx.x * (kWaveThreads / 64) +
                      (uint64_t)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const bool active = wt < total_tiles;
  // the tile: its node, its outer bits (the same in every lane of the wave)
  // and its register bits
  const int nouter = P.n_outer;
  uint64_t node = 0, tile = 0;
  if (active) {
    if (tlist) {
      // only the listed tiles of every node (the rest is never read)
      node = wt / n_list;
      tile = tlist[wt - node * n_list];
    } else {
      node = wt >> nouter;
      tile = wt & ((1ull << nouter) - 1);
    }
  }
  uint32_t xo = 0;
  for (int j = 0; j < nouter; ++j) xo |= (uint32_t)((tile >> j) & 1) << P.obit[j];
  xo = __builtin_amdgcn_readfirstlane(xo);
  node = ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(node >> 32)) << 32) |
         (uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)node);
  uint32_t RB[R];
#pragma unroll
  for (int k = 0; k < R; ++k) RB[k] = 1u << P.tbit[6 + k];
  const uint32_t F = xo | lane;
  const uint64_t N = 1ull << P.n;
  // the tile's loads go out first, so that their latency overlaps the
  // staging of the ops below
  float2 v[E];
  if (P.init) {
    const uint32_t hmask = ~(uint32_t)P.hinit;
    const float h = P.hamp;
    const bool lane_ok = (F & hmask) == 0;
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const bool ok = lane_ok && (reg_index<R>(r, RB) & hmask) == 0;
      v[r] = ok ? make_float2(h, 0.f) : make_float2(0.f, 0.f);
    }
  } else if (active) {
    const float2* row = in + node * N;
#pragma unroll
    for (int r = 0; r < E; ++r) v[r] = (row + (xo | reg_index<R>(r, RB)))[lane];
  }
  {
    const uint2* src = (const uint2*)(ops + P.op_in);
    const int nw = P.n_all * (int)(sizeof(DevOp) / sizeof(uint2));
    for (int i = threadIdx.x; i < nw; i += kWaveThreads) wp_ops[i] = src[i];
  }
  init_phase_table(tab);  // and the barrier after the staging
  if (!active) return;
  const DevOp* sops = (const DevOp*)wp_ops;
  wave_apply_ops<R>(v, sops, P.n_in, F, RB, (int)lane, tab);
  const float sc = P.scale;
  const int nt = P.nt;
  if constexpr (S == 0) {
    wave_store<R>(out + node * N, v, sc, xo, lane, RB, nt);
  } else {
    const int m1 = P.sm[0];
    for (int b1 = 0; b1 < (1 << m1); ++b1) {
      float2 w[E];
      wave_child<R>(w, v, P.sbq[0], m1, b1, P.upper, F, RB);
      wave_apply_ops<R>(w, sops + P.sop[0], P.snops[0], F, RB, (int)lane, tab);
      const uint64_t c1 = (node << m1) | (uint64_t)b1;
      if constexpr (S == 1) {
        wave_store<R>(out + c1 * N, w, sc, xo, lane, RB, nt);
      } else {
        const int m2 = P.sm[1];
        for (int b2 = 0; b2 < (1 << m2); ++b2) {
          float2 u[E];
          wave_child<R>(u, w, P.sbq[1], m2, b2, P.upper, F, RB);
          wave_apply_ops<R>(u, sops + P.sop[1], P.snops[1], F, RB, (int)lane, tab);
          wave_store<R>(out + ((c1 << m2) | (uint64_t)b2) * N, u, sc, xo, lane, RB, nt);
        }
      }
    }
  }
}

// ------------------------------------------------------------------ exchange group
//
// k_xpass: the passes of an exchange group (XPassDesc) as phases of one
// launch.  A workgroup of kXWaves waves owns the amplitudes of one node whose
// bits outside the lanes and U are fixed (2^(6 + R + kXWaveBits) of them).  In
// phase p each wave holds a wave tile of that pass (lanes: state bits 0..5,
// registers: the pass's R register bits) at its own combination of the other
// bits of U, applies the pass's ops, and writes the tile to LDS at position
// (bits of U, compressed) 64 + lane; after a barrier the next phase reads it
// back in its own split.  Phase 0 reads HBM (or starts from the product
// state), the last phase writes HBM: one read and one write for the group.
// Each phase's op list is staged in LDS when it fits.
constexpr int kXWaves = 1 << kXWaveBits;
constexpr int kXThreads = 64 * kXWaves;
constexpr int kXOpsBytes = 14 * 1024;

template <int R>
__global__ void __launch_bounds__(kXThreads)
k_xpass(const XPassDesc* __restrict__ xdp, const PassDesc* __restrict__ pds,
        const DevOp* __restrict__ ops, float2* state) {
  constexpr int E = 1 << R;
  constexpr int T = 6 + R + kXWaveBits;
  __shared__ __attribute__((aligned(16))) float2 xt[1 << T];
  __shared__ __attribute__((aligned(16))) uint2 xops[kXOpsBytes / sizeof(uint2)];
  __shared__ float2 tab[kPhaseEntries];
  const XPassDesc& X = *xdp;
  const uint32_t lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint64_t wt = blockIdx.x;
  const int nouter = X.n_outer;
  const uint64_t node = wt >> nouter;
  const uint64_t tile = wt & ((1ull << nouter) - 1);
  uint32_t xo = 0;
  for (int j = 0; j < nouter; ++j) xo |= (uint32_t)((tile >> j) & 1) << X.obit[j];
  xo = __builtin_amdgcn_readfirstlane(xo);
  float2* row = state + node * (1ull << X.n);
  float2 v[E];
  for (int p = 0; p < X.G; ++p) {
    const PassDesc& P = pds[X.pd0 + p];
    uint32_t RB[R];
#pragma unroll
    for (int k = 0; k < R; ++k) RB[k] = 1u << P.tbit[6 + k];
    // this wave's bits of U outside the pass's registers, and its LDS offset
    uint32_t wb = 0, wpos = 0;
#pragma unroll
    for (int j = 0; j < kXWaveBits; ++j)
      if ((wave >> j) & 1) {
        wb |= 1u << X.ubit[X.wpos[p][j]];
        wpos |= 1u << X.wpos[p][j];
      }
    const uint32_t F = xo | wb | lane;
    // the phase's ops: staged in LDS when they fit
    const int nw = P.n_in * (int)(sizeof(DevOp) / sizeof(uint2));
    const bool staged = nw <= (int)(kXOpsBytes / sizeof(uint2));
    if (staged) {
      const uint2* src = (const uint2*)(ops + P.op_in);
      for (int i = threadIdx.x; i < nw; i += kXThreads) xops[i] = src[i];
    }
    if (p == 0) {
      if (X.init) {
        const uint32_t hmask = ~(uint32_t)P.hinit;
        const float h = P.hamp;
        const bool lane_ok = (F & hmask) == 0;
#pragma unroll
        for (int r = 0; r < E; ++r) {
          const bool ok = lane_ok && (reg_index<R>(r, RB) & hmask) == 0;
          v[r] = ok ? make_float2(h, 0.f) : make_float2(0.f, 0.f);
        }
      } else {
#pragma unroll
        for (int r = 0; r < E; ++r) v[r] = (row + (xo | wb | reg_index<R>(r, RB)))[lane];
      }
      init_phase_table(tab);  // and the barrier after the staging
    } else {
#pragma unroll
      for (int r = 0; r < E; ++r) {
        uint32_t u = wpos;
#pragma unroll
        for (int k = 0; k < R; ++k)
          if ((r >> k) & 1) u |= 1u << X.rpos[p][k];
        v[r] = xt[(u << 6) | lane];
      }
      __syncthreads();  // ops staged, and every wave has read its tile
    }
    wave_apply_ops<R>(v, staged ? (const DevOp*)xops : ops + P.op_in, P.n_in, F, RB, (int)lane,
                      tab);
    const float sc = P.scale;
    if (p + 1 < X.G) {
#pragma unroll
      for (int r = 0; r < E; ++r) {
        uint32_t u = wpos;
#pragma unroll
        for (int k = 0; k < R; ++k)
          if ((r >> k) & 1) u |= 1u << X.rpos[p][k];
        xt[(u << 6) | lane] = make_float2(v[r].x * sc, v[r].y * sc);
      }
      __syncthreads();  // the tile is in LDS, and every wave is done with the staged ops
    } else {
      wave_store<R>(row, v, sc, xo | wb, lane, RB, X.nt);
    }
  }
}

hipError_t launch_xpass(const XPassDesc& h, const XPassDesc* d_desc, const PassDesc* d_pds,
                        const DevOp* d_ops, float2* state, uint64_t nodes, hipStream_t st) {
  if (h.G < 2 || h.G > kMaxXPhases || h.nu != h.R + kXWaveBits || 6 + h.nu + h.n_outer != h.n)
    return hipErrorInvalidValue;
  const uint64_t blocks = nodes << h.n_outer;
  if (blocks == 0 || blocks > 0x7fffffffull) return hipErrorInvalidValue;
  dim3 g((unsigned)blocks), b(kXThreads);
  switch (h.R) {
    case 3: hipLaunchKernelGGL(k_xpass<3>, g, b, 0, st, d_desc, d_pds, d_ops, state); break;
    case 4: hipLaunchKernelGGL(k_xpass<4>, g, b, 0, st, d_desc, d_pds, d_ops, state); break;
    case 5: hipLaunchKernelGGL(k_xpass<5>, g, b, 0, st, d_desc, d_pds, d_ops, state); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int R>
static hipError_t launch_wpass_r(int S, dim3 g, dim3 b, size_t lds, hipStream_t st,
                                 const PassDesc* d_desc, const DevOp* d_ops, const float2* in,
                                 float2* out, uint64_t tiles, const uint32_t* tlist,
                                 uint32_t n_list) {
  switch (S) {
    case 0:
      hipLaunchKernelGGL((k_wpass<R, 0>), g, b, lds, st, d_desc, d_ops, in, out, tiles, tlist, n_list);
      break;
    case 1:
      hipLaunchKernelGGL((k_wpass<R, 1>), g, b, lds, st, d_desc, d_ops, in, out, tiles, tlist, n_list);
      break;
    case 2:
      hipLaunchKernelGGL((k_wpass<R, 2>), g, b, lds, st, d_desc, d_ops, in, out, tiles, tlist, n_list);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_pass(const PassDesc& h, const PassDesc* d_desc, const DevOp* d_ops,
                       const float2* in, float2* out, uint64_t n_in_nodes, const uint32_t* tlist,
                       uint32_t n_list, hipStream_t st) {
  static_assert(kMaxStages == 2, "k_wpass and k_pass are written for at most two stages");
  if (tlist && (!h.wave || n_list == 0)) return hipErrorInvalidValue;
  if (h.ns < 0 || h.ns > kMaxStages || h.n_all < 0 || h.n_all > kMaxPassOps)
    return hipErrorInvalidValue;
  if (h.wave) {
    const int R = h.t - 6;
    const uint64_t tiles = tlist ? n_in_nodes * n_list : n_in_nodes << h.n_outer;
    const uint64_t blocks = (tiles + (kWaveThreads / 64) - 1) / (kWaveThreads / 64);
    if (blocks == 0 || blocks > 0x7fffffffull) return hipErrorInvalidValue;
    dim3 g((unsigned)blocks), b(kWaveThreads);
    const size_t lds = (size_t)h.n_all * sizeof(DevOp);
    switch (R) {
      case 1: return launch_wpass_r<1>(h.ns, g, b, lds, st, d_desc, d_ops, in, out, tiles, tlist, n_list);
      case 2: return launch_wpass_r<2>(h.ns, g, b, lds, st, d_desc, d_ops, in, out, tiles, tlist, n_list);
      case 3: return launch_wpass_r<3>(h.ns, g, b, lds, st, d_desc, d_ops, in, out, tiles, tlist, n_list);
      case 4: return launch_wpass_r<4>(h.ns, g, b, lds, st, d_desc, d_ops, in, out, tiles, tlist, n_list);
      case 5: return launch_wpass_r<5>(h.ns, g, b, lds, st, d_desc, d_ops, in, out, tiles, tlist, n_list);
      default: return hipErrorInvalidValue;
    }
  }
  const uint64_t blocks = n_in_nodes << h.n_outer;
  if (blocks == 0 || blocks > 0x7fffffffull) return hipErrorInvalidValue;
  const size_t lds = (size_t)(1 + h.ns) * ((size_t)8 << h.t);
  hipLaunchKernelGGL(k_pass, dim3((unsigned)blocks), dim3(kPassThreads), lds, st, d_desc, d_ops,
                     in, out);
  return hipGetLastError();
}

// ------------------------------------------------------------------ leaf evaluation
//
// k_tail_bwd: per requested value s, the rows w_{s,lam} of every leaf path's
// operator, by running the transposed leaf levels backwards from the unit
// vector at s (the paths share their suffixes, so the backward traversal is a
// tree too).  One group of G = min(64, 2^q) lanes per s; each lane holds
// 2^q / G amplitudes.  Output W[s][lam][y].
//
// k_tail_mm: A[node, lam] at s = sum_y W[s][lam][y] v_node[x(s, y)], a complex
// GEMM per s on FP32 MFMA; the result is written to X[k][s] for every copy k
// the (node, lam) pair stands for (times the factors of the end cuts).

constexpr int kTailThreads = 256;

constexpr int ilog2(int x) { return x <= 1 ? 0 : 1 + ilog2(x / 2); }

template <int R>
struct TailCtx {
  static constexpr int NB = ilog2(R);
  uint32_t xs[R];
  uint32_t RB[NB > 0 ? NB : 1];  // state bit of each register bit (light-cone bits lg..q-1)
  int g;       // lane inside the group
  int lg;      // log2 of the group width
  int sub;     // this wavefront's branches of the first reverse levels
  const float2* tab;  // phase table (LDS)
};

template <int R>
__device__ __forceinline__ void tail_apply_ops(float2 (&v)[R], const TailCtx<R>& c,
                                               const DevOp* __restrict__ ops, int nops) {
  for (int o = 0; o < nops; ++o) {
    const DevOp& op = ops[o];
    if (__builtin_amdgcn_readfirstlane(op.kind) == 0) {
      const int w = __builtin_amdgcn_readfirstlane(op.target);
      // the general form: one code path per gate keeps the unrolled leaf
      // kernels small (a branch per gate kind there costs more than it saves)
      if (w < c.lg) {
        lane_mat_m<R>(v, op, w, (c.g >> w) & 1);
      } else {
        const int rb = w - c.lg;
        if constexpr (R >= 2) { if (rb == 0) tail_mat_reg_m<R>(v, op.m, 0); }
        if constexpr (R >= 4) { if (rb == 1) tail_mat_reg_m<R>(v, op.m, 1); }
        if constexpr (R >= 8) { if (rb == 2) tail_mat_reg_m<R>(v, op.m, 2); }
        if constexpr (R >= 16) { if (rb == 3) tail_mat_reg_m<R>(v, op.m, 3); }
      }
    } else {
      diag_regs<TailCtx<R>::NB>(v, op, c.xs[0], c.RB, c.tab);
    }
  }
}

// Backward traversal: level index runs from the last leaf level to the first.
template <int R, int D>
__device__ __forceinline__ void tail_bwd_rec(const float2 (&v)[R], const TailCtx<R>& c,
                                             const TailDesc& T, const DevOp* __restrict__ ops,
                                             uint32_t lam, float2* __restrict__ Wrow) {
  if constexpr (D < kMaxTailLevels) {
    const int l = T.nlev - 1 - D;
    const TailLevel& L = T.lev[l];
    float2 u[R];
#pragma unroll
    for (int r = 0; r < R; ++r) u[r] = v[r];
    tail_apply_ops<R>(u, c, ops + L.bop0, L.bnops);
    const int m = L.m;
    const int G = 1 << c.lg;
    int b_lo = 0, b_hi = 1 << m;
    if (D < T.split_levels) {
      // only the branch this wavefront owns
      int sh = 0;
      for (int d2 = D + 1; d2 < T.split_levels; ++d2) sh += T.lev[T.nlev - 1 - d2].m;
      b_lo = (c.sub >> sh) & ((1 << m) - 1);
      b_hi = b_lo + 1;
    }
    for (int b = b_lo; b < b_hi; ++b) {
      uint32_t cmask, cval, zmask;
      cut_factors(L.bq, m, b, T.upper, cmask, cval, zmask);
      float2 w[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        float2 a = u[r];
        if ((c.xs[r] & cmask) != cval) a = make_float2(0.f, 0.f);
        if (__popc(c.xs[r] & zmask) & 1) a = make_float2(-a.x, -a.y);
        w[r] = a;
      }
      const uint32_t lam2 = lam | ((uint32_t)b << L.shift);
      if (l == 0) {
        float2* dst = Wrow + (size_t)lam2 * ((size_t)G * R);
#pragma unroll
        for (int r = 0; r < R; ++r) dst[c.g + (r << c.lg)] = w[r];
      } else {
        tail_bwd_rec<R, D + 1>(w, c, T, ops, lam2, Wrow);
      }
    }
  }
}

template <int R>
__global__ void __launch_bounds__(kTailThreads)
k_tail_bwd(const TailDesc* __restrict__ tdp, const DevOp* __restrict__ ops,
           const uint32_t* __restrict__ svals, int s0, int ns, float2* __restrict__ W) {
  __shared__ float2 tab[kPhaseEntries];
  init_phase_table(tab);
  const TailDesc& T = *tdp;
  const int lg = T.q < 6 ? T.q : 6;
  const int G = 1 << lg;
  const uint64_t gtid = (uint64_t)blockIdx.x * kTailThreads + threadIdx.x;
  const uint64_t grp = gtid >> lg;
  if (grp >= ((uint64_t)ns << T.split_bits)) return;
  const uint64_t gid = grp >> T.split_bits;
  TailCtx<R> c;
  c.g = (int)(gtid & (G - 1));
  c.lg = lg;
  c.sub = (int)(grp & ((1u << T.split_bits) - 1));
  c.tab = tab;
#pragma unroll
  for (int k = 0; k < TailCtx<R>::NB; ++k) c.RB[k] = 1u << T.Q[lg + k];
  const uint32_t s = svals[s0 + gid];
  uint32_t qmask = 0, ys = 0;
  for (int i = 0; i < T.q; ++i) {
    qmask |= 1u << T.Q[i];
    ys |= ((s >> T.Q[i]) & 1u) << i;
  }
  const uint32_t base = s & ~qmask;
  float2 v[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const uint32_t y = (uint32_t)(c.g + (r << lg));
    uint32_t x = base;
    for (int i = 0; i < T.q; ++i) x |= ((y >> i) & 1u) << T.Q[i];
    c.xs[r] = x;
    v[r] = (y == ys) ? make_float2(T.tscale, 0.f) : make_float2(0.f, 0.f);
  }
  const size_t K = (size_t)G * R;
  float2* Wrow = W + gid * ((size_t)1 << T.M) * K;
  if (T.nlev == 0) {
#pragma unroll
    for (int r = 0; r < R; ++r) Wrow[c.g + (r << lg)] = v[r];  // split_bits is 0 here
    return;
  }
  tail_bwd_rec<R, 0>(v, c, T, ops, 0u, Wrow);
}

constexpr int kTM = 64, kTN = 64, kTK = 16;

// Per requested value s: C[node][lam] = sum_y v_node[x(s, y)] W[s][lam][y] on
// v_mfma_f32_16x16x4f32 with three real products per complex one
// (Ar Br, Ai Bi, (Ar + Ai)(Br + Bi)); rows are materialised nodes, columns leaf
// paths, so consecutive lanes of a store hold consecutive leaf paths and the
// row X[s][nu] of the output is written in contiguous runs.  nu is the half's
// natural copy order ((node * 2^M + lam) * 2^n_end + end bits).
__global__ void __launch_bounds__(kTailThreads)
k_tail_mm(const TailDesc* __restrict__ tdp, const float2* __restrict__ W,
          const float2* __restrict__ states, const uint32_t* __restrict__ svals, int s0,
          float2* __restrict__ X) {
  __shared__ float2 As[kTK][kTM + 1];   // [y][node]
  __shared__ float2 Bs[kTK][kTN + 1];   // [y][lam]
  __shared__ uint32_t xy[kTK];
  const TailDesc& T = *tdp;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int sl = blockIdx.z;
  const int si = s0 + sl;
  const uint32_t s = svals[si];
  const int K = 1 << T.q;
  const int Lam = 1 << T.M;
  const int Nn = T.n_nodes;
  const int r0 = blockIdx.y * kTM, lam0 = blockIdx.x * kTN;
  uint32_t qmask = 0;
  for (int i = 0; i < T.q; ++i) qmask |= 1u << T.Q[i];
  const uint32_t base = s & ~qmask;
  const float2* Ws = W + (size_t)sl * Lam * K;
  const size_t N = (size_t)1 << T.n;
  const int wi = (wave >> 1) * 32, wj = (wave & 1) * 32;
  floatx4 p1[2][2], p2[2][2], p3[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      p1[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};
      p2[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};
      p3[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};
    }
  for (int y0 = 0; y0 < K; y0 += kTK) {
    if (tid < kTK) {
      const uint32_t y = (uint32_t)(y0 + tid);
      uint32_t x = base;
      for (int i = 0; i < T.q; ++i) x |= ((y >> i) & 1u) << T.Q[i];
      xy[tid] = x;
    }
    __syncthreads();
    for (int e = tid; e < kTK * kTM; e += kTailThreads) {
      const int kk = e % kTK, ii = e / kTK;
      const int y = y0 + kk;
      const int rr = r0 + ii, lam = lam0 + ii;
      As[kk][ii] = (y < K && rr < Nn) ? states[(size_t)rr * N + xy[kk]] : make_float2(0.f, 0.f);
      Bs[kk][ii] = (y < K && lam < Lam) ? Ws[(size_t)lam * K + y] : make_float2(0.f, 0.f);
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kTK; kk += 4) {
      float2 av[2], bv[2];
      for (int a = 0; a < 2; ++a) av[a] = As[kk + (lane >> 4)][wi + a * 16 + (lane & 15)];
      for (int b = 0; b < 2; ++b) bv[b] = Bs[kk + (lane >> 4)][wj + b * 16 + (lane & 15)];
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
          p1[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a].x, bv[b].x, p1[a][b], 0, 0, 0);
          p2[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a].y, bv[b].y, p2[a][b], 0, 0, 0);
          p3[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a].x + av[a].y, bv[b].x + bv[b].y,
                                                          p3[a][b], 0, 0, 0);
        }
    }
    __syncthreads();
  }
  const int ne = T.n_end;
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int e4 = 0; e4 < 4; ++e4) {
        const int rr = r0 + wi + a * 16 + 4 * (lane >> 4) + e4;
        const int lam = lam0 + wj + b * 16 + (lane & 15);
        if (lam >= Lam || rr >= Nn) continue;
        const float re = p1[a][b][e4] - p2[a][b][e4];
        const float im = p3[a][b][e4] - p1[a][b][e4] - p2[a][b][e4];
        if (T.end_base) {
          X[(size_t)si * T.ldx + (((size_t)rr << T.M) + lam)] = make_float2(re, im);
          continue;
        }
        float2* dst = X + (size_t)si * T.ldx + ((((size_t)rr << T.M) + lam) << ne);
        for (int e = 0; e < (1 << ne); ++e) {
          float2 f = make_float2(re, im);
          for (int i = 0; i < ne; ++i) {
            const uint32_t eb = (e >> (ne - 1 - i)) & 1;
            const uint32_t sb = (s >> T.eq[i]) & 1;
            if (T.upper) {
              if (eb != sb) f = make_float2(0.f, 0.f);
            } else if (eb & sb) {
              f = make_float2(-f.x, -f.y);
            }
          }
          dst[e] = f;
        }
      }
}

// Workgroup barrier that orders LDS accesses only: it waits for this wave's
// LDS operations but not for its global stores (a __syncthreads waits for
// those as well, and the leaf kernels' output stores need no ordering with
// the other waves).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// k_tail_fused: the rows and the contraction of one requested value s in one
// workgroup, without the rows passing through HBM.  The 2^M leaf paths are
// taken in emission order j (the digit of level l at bit pos(l) =
// sum_{l' < l} m_l'); wave w owns j in [w 2^M/4, (w+1) 2^M/4) and walks it as
// a depth-first traversal whose stack (u_D: the vector after depth D's ops,
// before its cut factor) stays in registers, so consecutive paths redo only
// the levels whose digit changed.  Every chunk of kFusedRows rows (8 per
// wave) goes to LDS, then the four waves contract it with the materialised
// node states on FP32 MFMA (three real products per complex one).  The
// light cone must be on state bits 0..q-1 (x(s, y) = base + y).

constexpr int kFusedRows = 32;  // 16 or 32
constexpr int kFusedWaves = 4;  // waves per workgroup (4 or 8)
constexpr int kFusedThreads = 64 * kFusedWaves;
constexpr int kFusedDepth = 8;
constexpr int kFusedPadQ = 2;    // complex padding after each quarter of a row
constexpr int kFusedPadRow = 28; // more padding per row (row stride = 4 mod 32 complex)

__host__ __device__ constexpr int fused_row_stride(int K) {
  return 4 * (K / 4 + kFusedPadQ) + kFusedPadRow;
}

// The leaf amplitude of node rn, emission path j at value s, from the three
// real products of the contraction (re = p1 - p2, im = p3 - p1 - p2), stored
// at every copy it stands for: Xs[((rn << M) + j) << ne | e] (Xs = X[s], the
// value's output row, whose length ldx fits an int) times the end cuts'
// factors at s (upper: the projector on bit e, lower: the sign), or only at
// e = 0 without factors when the end cuts are folded into the assembly.
__device__ __forceinline__ void tail_store(const TailDesc& T, int end_base, float2* __restrict__ Xs,
                                           uint32_t s, int rn, int M, int ne, uint32_t j,
                                           float p1, float p2, float p3) {
  const float re = p1 - p2;
  const float im = p3 - p1 - p2;
  const uint32_t o = ((uint32_t)rn << M) + j;
  if (end_base) {
    Xs[o] = make_float2(re, im);
    return;
  }
  float2* dst = Xs + (o << ne);
  for (int e = 0; e < (1 << ne); ++e) {
    float2 f = make_float2(re, im);
    for (int i = 0; i < ne; ++i) {
      const uint32_t eb = (e >> (ne - 1 - i)) & 1;
      const uint32_t sb = (s >> T.eq[i]) & 1;
      if (T.upper) {
        if (eb != sb) f = make_float2(0.f, 0.f);
      } else if (eb & sb) {
        f = make_float2(-f.x, -f.y);
      }
    }
    dst[e] = f;
  }
}

// One contraction unit of k_tail_fused: node tile `at` (16 nodes) against
// NBT column tiles of the chunk starting at tile b0.  Lane group gq = lane/16
// takes y in [gq K/4, (gq+1) K/4) as the MFMA k index; the node amplitudes
// come from global memory (L2) in double-buffered batches of 4 x 16 bytes.
// Nodes past the last one read a valid row and are not written.
template <int R, int NBT>
__device__ __forceinline__ void fused_unit(const TailDesc& T, const float2* __restrict__ states,
                                           uint32_t base, const float2* wl, int at, int b0, int ch,
                                           uint32_t J4, int si, uint32_t s,
                                           float2* __restrict__ X) {
  constexpr int K = 64 * R, KQ = K / 4, RS = fused_row_stride(K);
  constexpr int TB = KQ / 2 < 4 ? KQ / 2 : 4;  // float4 (two y) per batch
  constexpr int NBATCH = KQ / 2 / TB;
  const int lane = threadIdx.x & 63, gq = lane >> 4, li = lane & 15;
  const int Nn = T.n_nodes, M = T.M, ne = T.n_end;
  const size_t N = (size_t)1 << T.n;
  const int node = at * 16 + li;
  const float4* arow =
      (const float4*)(states + (size_t)min(node, Nn - 1) * N + base + gq * KQ);
  const float2* brow[NBT];
#pragma unroll
  for (int bb = 0; bb < NBT; ++bb) brow[bb] = wl + ((b0 + bb) * 16 + li) * RS + gq * (KQ + kFusedPadQ);
  floatx4 p1[NBT], p2[NBT], p3[NBT];
#pragma unroll
  for (int bb = 0; bb < NBT; ++bb) {
    p1[bb] = floatx4{0.f, 0.f, 0.f, 0.f};
    p2[bb] = floatx4{0.f, 0.f, 0.f, 0.f};
    p3[bb] = floatx4{0.f, 0.f, 0.f, 0.f};
  }
  float4 a0[TB], a1[TB];
  auto load = [&](float4 (&dst)[TB], int bt) {
#pragma unroll
    for (int i = 0; i < TB; ++i) dst[i] = arow[bt * TB + i];
  };
  auto mma = [&](const float4 (&src)[TB], int bt) {
#pragma unroll
    for (int i = 0; i < TB; ++i) {
      const float4 av = src[i];
      const int t = 2 * (bt * TB + i);
#pragma unroll
      for (int bb = 0; bb < NBT; ++bb) {
        const float4 bv = *(const float4*)(brow[bb] + t);
        p1[bb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.x, bv.x, p1[bb], 0, 0, 0);
        p2[bb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.y, bv.y, p2[bb], 0, 0, 0);
        p3[bb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.x + av.y, bv.x + bv.y, p3[bb], 0, 0, 0);
        p1[bb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.z, bv.z, p1[bb], 0, 0, 0);
        p2[bb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.w, bv.w, p2[bb], 0, 0, 0);
        p3[bb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.z + av.w, bv.z + bv.w, p3[bb], 0, 0, 0);
      }
    }
  };
  // batches alternate between a0 and a1: the next batch loads while the
  // current one feeds the MFMAs
  // (the scheduling barriers keep each prefetch ahead of the MFMAs it overlaps)
  // (the last pair prefetches batch 0 again, unused, to keep the loop branch-free)
  static_assert(NBATCH % 2 == 0, "batches come in pairs");
  load(a0, 0);
#pragma unroll 1
  for (int bt = 0; bt < NBATCH; bt += 2) {
    load(a1, bt + 1);
    __builtin_amdgcn_sched_barrier(0);
    mma(a0, bt);
    __builtin_amdgcn_sched_barrier(0);
    load(a0, bt + 2 < NBATCH ? bt + 2 : 0);
    __builtin_amdgcn_sched_barrier(0);
    mma(a1, bt + 1);
    __builtin_amdgcn_sched_barrier(0);
  }
#pragma unroll
  for (int bb = 0; bb < NBT; ++bb) {
    // LDS row col = w RW + ci kSt + st (RW = rows per wave, kSt = steps of a
    // chain per chunk) holds path w J4 + ci J4/2 + ch kSt + st (J4: paths per wave)
    constexpr int RW = kFusedRows / kFusedWaves, kSt = RW / 2;
    const int col = (b0 + bb) * 16 + li;
    const uint32_t j = (uint32_t)(col / RW) * J4 + (uint32_t)((col % RW) / kSt) * (J4 / 2) +
                       (uint32_t)(ch * kSt + col % kSt);
#pragma unroll
    for (int e4 = 0; e4 < 4; ++e4) {
      const int rn = at * 16 + 4 * gq + e4;
      if (rn >= Nn) continue;
      tail_store(T, T.end_base, X + (size_t)si * T.ldx, s, rn, M, ne, j, p1[bb][e4], p2[bb][e4],
                 p3[bb][e4]);
    }
  }
}

bool tail_fused_ok(const TailDesc& h) {
  if (h.q < 6 || h.q > 8 || h.nlev < 1 || h.nlev > kFusedDepth || h.M < 5) return false;
  for (int i = 0; i < h.q; ++i)
    if (h.Q[i] != i) return false;
  return true;
}

template <int R>
__global__ void __launch_bounds__(kFusedThreads)
k_tail_fused(const TailDesc* __restrict__ tdp, const DevOp* __restrict__ ops,
             const float2* __restrict__ states, const uint32_t* __restrict__ svals, int s0,
             float2* __restrict__ X) {
  constexpr int K = 64 * R, KQ = K / 4;
  constexpr int RS = fused_row_stride(K);
  __shared__ __attribute__((aligned(16))) float2 wl[kFusedRows * RS];  // rows of the chunk
  __shared__ float2 tab[kPhaseEntries];
  init_phase_table(tab);
  const TailDesc& T = *tdp;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int si = s0 + blockIdx.x;
  const uint32_t s = svals[si];
  const uint32_t qmask = (1u << T.q) - 1u;
  const uint32_t base = s & ~qmask, ys = s & qmask;
  // Two traversal chains per wave, over the first and the second half of the
  // wave's paths, advance in lockstep: they redo the same depths at the same
  // time, so every op is applied to both at once (the chain index acts as one
  // more register bit that no op touches: state bit mask 0, no phase terms).
  constexpr int C = 2, RC = R * C;
  TailCtx<RC> c;
  c.g = lane;
  c.lg = 6;
  c.sub = 0;
  c.tab = tab;
#pragma unroll
  for (int k = 0; k < TailCtx<RC>::NB; ++k) c.RB[k] = k < TailCtx<R>::NB ? 1u << (6 + k) : 0u;
#pragma unroll
  for (int r = 0; r < RC; ++r) c.xs[r] = base | (uint32_t)(lane + 64 * (r % R));
  const int nlev = T.nlev, M = T.M;
  const uint32_t J4 = (1u << M) / kFusedWaves;  // paths per wave
  const uint32_t JC = J4 / C;                    // paths per chain
  const uint32_t jw = (uint32_t)wave * J4;
  constexpr int kSteps = kFusedRows / kFusedWaves / C;  // steps of a chain per chunk
  const int nchunks = (int)(JC / kSteps);
  const int nat = (T.n_nodes + 15) >> 4;
  float2 u[kFusedDepth][RC];
  uint32_t jprev = 0;
  for (int ch = 0; ch < nchunks; ++ch) {
    // ---- rows of this chunk: wave w, chain ci, step st -> LDS row w * rows per wave + ci * kSteps + st
    for (int st = 0; st < kSteps; ++st) {
      const uint32_t jl = (uint32_t)(ch * kSteps + st);  // path index inside a chain
      int d0 = -1;  // u[0..d0] still hold
      if (jl > 0) {
        // chain offsets are multiples of JC > jl: the changed digits are jl's
        const int hb = 31 - __builtin_clz(jl ^ jprev);
        int lh = 0;
        while (lh + 1 < nlev && T.lev[lh + 1].pos <= hb) ++lh;
        d0 = nlev - 1 - lh;
      }
      jprev = jl;
      float2 v[RC];
#pragma unroll
      for (int D = 0; D < kFusedDepth; ++D) {
        if (D < nlev) {
          const int l = nlev - 1 - D;
          if (D > d0) {
            if (D == 0) {
#pragma unroll
              for (int r = 0; r < RC; ++r)
                v[r] = ((uint32_t)(lane + 64 * (r % R)) == ys) ? make_float2(T.tscale, 0.f)
                                                                : make_float2(0.f, 0.f);
            } else {
              const TailLevel& L = T.lev[l + 1];
#pragma unroll
              for (int ci = 0; ci < C; ++ci) {
                const uint32_t j = jw + (uint32_t)ci * JC + jl;
                const int b = (int)((j >> L.pos) & ((1u << L.m) - 1u));
                uint32_t cmask, cval, zmask;
                cut_factors(L.bq, L.m, b, T.upper, cmask, cval, zmask);
#pragma unroll
                for (int r = 0; r < R; ++r) {
                  float2 a = u[D - 1][ci * R + r];
                  if ((c.xs[r] & cmask) != cval) a = make_float2(0.f, 0.f);
                  if (__popc(c.xs[r] & zmask) & 1) a = make_float2(-a.x, -a.y);
                  v[ci * R + r] = a;
                }
              }
            }
#pragma unroll
            for (int r = 0; r < RC; ++r) u[D][r] = v[r];
            tail_apply_ops<RC>(u[D], c, ops + T.lev[l].bop0, T.lev[l].bnops);
          }
          if (D == nlev - 1) {
            const TailLevel& L = T.lev[0];
#pragma unroll
            for (int ci = 0; ci < C; ++ci) {
              const uint32_t j = jw + (uint32_t)ci * JC + jl;
              const int b = (int)((j >> L.pos) & ((1u << L.m) - 1u));
              uint32_t cmask, cval, zmask;
              cut_factors(L.bq, L.m, b, T.upper, cmask, cval, zmask);
              float2* row = wl + (wave * (kFusedRows / kFusedWaves) + ci * kSteps + st) * RS;
#pragma unroll
              for (int r = 0; r < R; ++r) {
                float2 a = u[D][ci * R + r];
                if ((c.xs[r] & cmask) != cval) a = make_float2(0.f, 0.f);
                if (__popc(c.xs[r] & zmask) & 1) a = make_float2(-a.x, -a.y);
                const int y = lane + 64 * r;
                row[(y / KQ) * (KQ + kFusedPadQ) + (y % KQ)] = a;
              }
            }
          }
        }
      }
    }
    lds_barrier();
    // ---- contraction: C[node][col] = sum_y v_node[base + y] W[col][y]; a unit
    // is one 16-node tile with both 16-column tiles (or one, when there are
    // fewer than four node tiles)
    if constexpr (kFusedRows == 16) {
      for (int un = wave; un < nat; un += kFusedWaves)
        fused_unit<R, 1>(T, states, base, wl, un, 0, ch, J4, si, s, X);
    } else if (nat >= kFusedWaves) {
      for (int un = wave; un < nat; un += kFusedWaves)
        fused_unit<R, 2>(T, states, base, wl, un, 0, ch, J4, si, s, X);
    } else {
      for (int un = wave; un < 2 * nat; un += kFusedWaves)
        fused_unit<R, 1>(T, states, base, wl, un >> 1, un & 1, ch, J4, si, s, X);
    }
    lds_barrier();
  }
}

// k_tail_ws: the same leaf evaluation with specialised waves, for at most
// kWsMaxNodes materialised nodes.  Eight producer waves walk the leaf paths
// (one depth-first chain each, its stack in registers as in k_tail_fused) and
// write each chunk of kWsRows rows into one of two LDS buffers; four consumer
// waves each hold one 16-node tile of the value's node amplitudes in
// registers (read from HBM once per value, instead of once per chunk) and
// contract the other buffer's chunk on FP32 MFMA.  One barrier per chunk.
// Waves w, w + 4 and w + 8 share a SIMD, so every SIMD runs two producers and
// one consumer: the producers' vector work and the consumer's MFMAs overlap
// instead of alternating.  The workgroups are persistent: each takes the
// values blockIdx.x, blockIdx.x + gridDim.x, ... and runs one pipeline over
// all their chunks, so the producers start a value while the consumers finish
// the one before (the DIAG offset table is double-buffered for that).
constexpr int kWsProducers = 8;
constexpr int kWsConsumers = 4;
constexpr int kWsThreads = 64 * (kWsProducers + kWsConsumers);
constexpr int kWsRows = 32;                         // rows per chunk
constexpr int kWsSteps = kWsRows / kWsProducers;    // paths per producer per chunk
constexpr int kWsMaxNodes = 16 * kWsConsumers;
constexpr int kWsMaxOps = 32;  // leaf-level ops whose DIAG offsets fit in LDS
// Row stride of the chunk buffers (complex): quarters of K/4 + kFusedPadQ,
// plus 4 so that the stride is 12 mod 32 complex.  A consumer's fragment read
// takes 16 B at one column of 16 rows; with a stride of 24 mod 64 dwords the
// rows of each group of eight start 8 dwords apart modulo 64, on distinct banks.
__host__ __device__ constexpr int ws_row_stride(int K) { return 4 * (K / 4 + kFusedPadQ) + 4; }

bool tail_ws_ok(const TailDesc& h) {
  if (!tail_fused_ok(h) || h.n_nodes < 1 || h.n_nodes > kWsMaxNodes) return false;
  // every producer needs at least one whole chunk: 2^M >= kWsRows
  if ((1 << h.M) < kWsRows) return false;
  // the producers take the first two leaf levels' digits together: one cut bit each
  if (h.nlev < 2 || h.lev[0].m != 1 || h.lev[1].m != 1) return false;
  // ops decoded from the levels' byte codes (targets are light-cone bits 0..7)
  for (int l = 0; l < h.nlev; ++l)
    if (h.lev[l].bnops > 8) return false;
  const int nops = h.lev[h.nlev - 1].bop0 + h.lev[h.nlev - 1].bnops - h.lev[0].bop0;
  return nops <= kWsMaxOps;
}

// Lane-pair 2x2 gate on lane bit w in its unit-entry form, the partner's
// amplitude read by ds_bpermute at lane ^ 2^w (the generic form for other
// matrices).
template <int R>
__device__ __forceinline__ void ws_lane_mat(float2 (&v)[R], const DevOp& op, int mk, int w,
                                            int lane) {
  const int addr = (lane ^ (1 << w)) << 2;
  const bool bit = (lane >> w) & 1;
  const auto sh = [addr](float x) {
    return __int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(x)));
  };
  if (mk == MK_X) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const float px = sh(v[r].x), py = sh(v[r].y);
      v[r] = make_float2(v[r].x + py, v[r].y - px);
    }
  } else if (mk == MK_Y || mk == MK_YT) {
    const float sg = (bit == (mk == MK_Y)) ? 1.f : -1.f;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const float px = sh(v[r].x), py = sh(v[r].y);
      v[r] = make_float2(fmaf(sg, px, v[r].x), fmaf(sg, py, v[r].y));
    }
  } else if (mk == MK_H) {
    const float sg = bit ? -1.f : 1.f;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const float px = sh(v[r].x), py = sh(v[r].y);
      v[r] = make_float2(fmaf(sg, v[r].x, px), fmaf(sg, v[r].y, py));
    }
  } else {
    lane_mat_m<R>(v, op, w, bit);
  }
}

// dst = src times the cut factors of branch b over a level's cut bits (the
// rule of cut_factors) on a producer's 64 x R vector: index F | r 2^6 with F =
// value base | lane.  The condition splits into the lane's part (one test per
// level visit) and the register's part, which is the same in every lane.
template <int R>
__device__ __forceinline__ void ws_cut(float2 (&dst)[R], const float2 (&src)[R],
                                       const TailLevel& L, int b, int upper, uint32_t F) {
  uint32_t cmask, cval, zmask;
  cut_factors(L.bq, L.m, b, upper, cmask, cval, zmask);
  cmask = (uint32_t)__builtin_amdgcn_readfirstlane(cmask);
  cval = (uint32_t)__builtin_amdgcn_readfirstlane(cval);
  zmask = (uint32_t)__builtin_amdgcn_readfirstlane(zmask);
  constexpr uint32_t regm = (uint32_t)(R - 1) << 6;
  const bool lane_ok = (F & cmask & ~regm) == (cval & ~regm);
  const uint32_t lane_sg = (uint32_t)(__popc(F & zmask & ~regm) & 1) << 31;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const uint32_t rb = (uint32_t)r << 6;
    float2 a = src[r];
    if ((rb & cmask) != (cval & regm)) {
      a = make_float2(0.f, 0.f);
    } else {
      if (cmask | cval) a = lane_ok ? a : make_float2(0.f, 0.f);
      if (zmask) {
        const uint32_t sg = lane_sg ^ ((uint32_t)(__popc(rb & zmask) & 1) << 31);
        a = make_float2(__uint_as_float(__float_as_uint(a.x) ^ sg),
                        __uint_as_float(__float_as_uint(a.y) ^ sg));
      }
    }
    dst[r] = a;
  }
}

// Register-pair 2x2 gate on register bit rb with a given matrix kind.
template <int R>
__device__ __forceinline__ void ws_mat_reg(float2 (&v)[R], const DevOp& op, int mk, int rb) {
  switch (mk) {
    case MK_X: tail_mat_reg_u<R, MK_X>(v, rb); break;
    case MK_Y: tail_mat_reg_u<R, MK_Y>(v, rb); break;
    case MK_YT: tail_mat_reg_u<R, MK_YT>(v, rb); break;
    case MK_H: tail_mat_reg_u<R, MK_H>(v, rb); break;
    default: tail_mat_reg_m<R>(v, op.m, rb); break;
  }
}

// The ops [o0, o0 + nops) of a producer of k_tail_ws on its 64 x R vector
// (lanes: working bits 0..5, registers: bits 6..): MATs in their unit-entry
// forms, DIAGs as table lookups at the offsets precomputed for this
// workgroup's value (dof: one word per op and lane, byte r = 8 e of register
// r, op index counted from the first leaf-level op).
template <int R, int C>
__device__ __forceinline__ void ws_apply_ops(float2 (&v)[C * R], const DevOp* __restrict__ ops,
                                             int o0, int nops, uint64_t code, int rel0, int lane,
                                             const uint32_t* dof, const float2* tab) {
  // C vectors side by side: register ci R + r is register r of vector ci (the
  // vector index acts as a register bit that no op touches).  Op o is byte o
  // of the level's code; only a MAT with a general matrix reads its entries.
  for (int o = 0; o < nops; ++o) {
    const uint32_t b = (uint32_t)(code >> (8 * o)) & 0xffu;
    if ((b & 0x80u) == 0) {
      const int w = (int)(b & 7u), mk = (int)((b >> 3) & 7u);
      const DevOp& op = ops[o0 + o];
      if (w < 6) {
        ws_lane_mat<C * R>(v, op, mk, w, lane);
      } else {
        if constexpr (R >= 2) { if (w == 6) ws_mat_reg<C * R>(v, op, mk, 0); }
        if constexpr (R >= 4) { if (w == 7) ws_mat_reg<C * R>(v, op, mk, 1); }
      }
    } else {
      const uint32_t pk = dof[(rel0 + o) * 64 + lane];
#pragma unroll
      for (int r = 0; r < C * R; ++r)
        v[r] = cmul(v[r], *(const float2*)((const char*)tab + ((pk >> (8 * (r % R))) & 0xffu)));
    }
  }
}

template <int R>
__global__ void __launch_bounds__(kWsThreads)
k_tail_ws(const TailDesc* __restrict__ tdp, const DevOp* __restrict__ ops,
          const float2* __restrict__ states, const uint32_t* __restrict__ svals, int s0, int ns,
          float2* __restrict__ X) {
  constexpr int K = 64 * R, KQ = K / 4;
  constexpr int RS = ws_row_stride(K);
  constexpr int NB = ilog2(R);
  __shared__ __attribute__((aligned(16))) float2 wl[2][kWsRows * RS];  // chunk buffers
  __shared__ uint32_t dof[2][kWsMaxOps * 64];  // DIAG table offsets, by value parity
  __shared__ float2 tab[kPhaseEntries];
  const TailDesc& T = *tdp;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int G = (int)gridDim.x;
  const int nv = (ns - (int)blockIdx.x + G - 1) / G;  // values of this workgroup
  const uint32_t qmask = (1u << T.q) - 1u;
  const int nlev = T.nlev, M = T.M;
  const int top0 = T.lev[0].bop0;
  const int ntop = T.lev[nlev - 1].bop0 + T.lev[nlev - 1].bnops - top0;
  // every DIAG op of the leaf levels at value v (index base | lane | register
  // bits, the lane part fixed for the whole value), by the producers
  auto offsets = [&](int v) {
    const uint32_t base = svals[s0 + (int)blockIdx.x + v * G] & ~qmask;
    uint32_t RB[NB > 0 ? NB : 1];
#pragma unroll
    for (int k = 0; k < NB; ++k) RB[k] = 1u << (6 + k);
    if constexpr (NB == 0) RB[0] = 0;
    uint32_t* d = dof[v & 1];
    for (int i = wave; i < ntop; i += kWsProducers) {
      const DevOp& op = ops[top0 + i];
      if (__builtin_amdgcn_readfirstlane(op.kind) == 1) {
        uint32_t off[R];
        diag_offsets<NB>(off, op, base | (uint32_t)lane, RB);
        uint32_t pk = 0;
#pragma unroll
        for (int r = 0; r < R; ++r) pk |= off[r] << (8 * r);
        d[i * 64 + lane] = pk;
      }
    }
  };
  if (wave < kWsProducers && nv > 0) offsets(0);
  init_phase_table(tab);  // and the barrier after the offsets
  const uint32_t JP = (1u << M) / kWsProducers;  // paths per producer
  const int nchunks = (int)(JP / kWsSteps);
  const int total = nv * nchunks;                // chunks of the pipeline
  if (wave < kWsProducers) {
    // ---- producer: paths [wave JP, (wave + 1) JP) of each value, the
    // kWsSteps = 4 paths j = wave JP + 4 ch + 2 b1 + b0 in chunk ch, at LDS row
    // wave 4 + 2 b1 + b0 (b0, b1: the digits of the first two leaf levels, one
    // cut bit each).  The four share the vector above level 1; level 0's ops
    // run on both values of b1 at once (one decode of each op for two vectors).
    static_assert(kWsSteps == 4, "a chunk takes one group of four paths per producer");
    const uint32_t jw = (uint32_t)wave * JP;
    float2 u[kFusedDepth - 1][R];  // the vector after depth D's ops, D < nlev - 1
    uint32_t jprev = 0;
    for (int g = 0; g <= total; ++g) {
      if (g < total) {
        const int v = g / nchunks, ch = g - v * nchunks;
        const uint32_t s = svals[s0 + (int)blockIdx.x + v * G];
        const uint32_t ys = s & qmask;
        const uint32_t F = (s & ~qmask) | (uint32_t)lane;
        const uint32_t* dv = dof[v & 1];
        float2* buf = wl[g & 1];
        const uint32_t jl = (uint32_t)ch * kWsSteps;
        int d0 = -1;  // u[0..d0] still hold (none at a value's first chunk)
        if (jl > 0) {
          // jw is a multiple of JP > jl: the changed digits are jl's (levels 2..)
          const int hb = 31 - __builtin_clz(jl ^ jprev);
          int lh = 0;
          while (lh + 1 < nlev && T.lev[lh + 1].pos <= hb) ++lh;
          d0 = nlev - 1 - lh;
        }
        jprev = jl;
        const uint32_t j = jw + jl;
#pragma unroll
        for (int D = 0; D < kFusedDepth - 1; ++D) {
          if (D < nlev - 1 && D > d0) {
            const int l = nlev - 1 - D;
            float2 x[R];
            if (D == 0) {
#pragma unroll
              for (int r = 0; r < R; ++r)
                x[r] = ((uint32_t)(lane + 64 * r) == ys) ? make_float2(T.tscale, 0.f)
                                                         : make_float2(0.f, 0.f);
            } else {
              const TailLevel& L = T.lev[l + 1];
              const int b = (int)((j >> L.pos) & ((1u << L.m) - 1u));
              ws_cut<R>(x, u[D - 1], L, b, T.upper, F);
            }
#pragma unroll
            for (int r = 0; r < R; ++r) u[D][r] = x[r];
            ws_apply_ops<R, 1>(u[D], ops, T.lev[l].bop0, T.lev[l].bnops, T.lev[l].code,
                               T.lev[l].bop0 - top0, lane, dv, tab);
          }
        }
        // level 0 on the vector above it with level 1's cut factor for b1 = 0
        // and for b1 = 1 (registers ci R + r), then level 0's cut for b0
        float2 w[2 * R];
        {
          float2 top[R];
#pragma unroll
          for (int D = 0; D < kFusedDepth - 1; ++D)
            if (D == nlev - 2) {
#pragma unroll
              for (int r = 0; r < R; ++r) top[r] = u[D][r];
            }
          float2 h[R];
          ws_cut<R>(h, top, T.lev[1], 0, T.upper, F);
#pragma unroll
          for (int r = 0; r < R; ++r) w[r] = h[r];
          ws_cut<R>(h, top, T.lev[1], 1, T.upper, F);
#pragma unroll
          for (int r = 0; r < R; ++r) w[R + r] = h[r];
        }
        ws_apply_ops<R, 2>(w, ops, T.lev[0].bop0, T.lev[0].bnops, T.lev[0].code,
                           T.lev[0].bop0 - top0, lane, dv, tab);
#pragma unroll
        for (int st = 0; st < kWsSteps; ++st) {
          float2 src[R], a[R];
#pragma unroll
          for (int r = 0; r < R; ++r) src[r] = w[(st >> 1) * R + r];
          ws_cut<R>(a, src, T.lev[0], st & 1, T.upper, F);
          float2* row = buf + (wave * kWsSteps + st) * RS;
#pragma unroll
          for (int r = 0; r < R; ++r) {
            const int y = lane + 64 * r;
            row[(y / KQ) * (KQ + kFusedPadQ) + (y % KQ)] = a[r];
          }
        }
        // the next value's offsets, into the other table (its last reader,
        // the value before this one, finished before the previous barrier)
        if (ch == nchunks - 1 && v + 1 < nv) offsets(v + 1);
      }
      lds_barrier();
    }
  } else {
    // ---- consumer: node tile `at` in registers; lane group gq = lane / 16
    // takes y in [gq KQ, (gq + 1) KQ) as the MFMA k index
    const int cw = wave - kWsProducers;
    const int Nn = T.n_nodes, ne = T.n_end;
    const int endb = __builtin_amdgcn_readfirstlane(T.end_base);
    const int ldx = __builtin_amdgcn_readfirstlane(T.ldx);
    const int nat = (Nn + 15) >> 4;
    const int nts = nat >= 3 ? 4 : nat;  // node-tile slots
    const int at = cw % nts;
    const int li = lane & 15, gq = lane >> 4;
    const size_t N = (size_t)1 << T.n;
    // nodes past the last one read a valid row and are not written
    const float2* const arow0 = states + (size_t)min(at * 16 + li, Nn - 1) * N + gq * KQ;
    float4 A[KQ / 2];
    auto load_a = [&](int v) {
      const uint32_t base = svals[s0 + (int)blockIdx.x + v * G] & ~qmask;
      const float4* arow = (const float4*)(arow0 + base);
#pragma unroll
      for (int i = 0; i < KQ / 2; ++i) A[i] = arow[i];
    };
    if (nv > 0) load_a(0);
    lds_barrier();
    for (int g = 0; g < total; ++g) {
      const int v = g / nchunks, ch = g - v * nchunks;
      const int si = s0 + (int)blockIdx.x + v * G;
      const uint32_t s = svals[si];
      float2* const Xs = X + (size_t)si * ldx;
      const float2* buf = wl[g & 1];
      if (at < nat) {
        for (int ct = cw / nts; ct < kWsRows / 16; ct += kWsConsumers / nts) {
          const float2* brow = buf + (ct * 16 + li) * RS + gq * (KQ + kFusedPadQ);
          floatx4 p1 = {0.f, 0.f, 0.f, 0.f}, p2 = p1, p3 = p1;
          // the next fragment is read while this one's products run
          float4 bn = *(const float4*)brow;
#pragma unroll
          for (int i = 0; i < KQ / 2; ++i) {
            const float4 bv = bn;
            if (i + 1 < KQ / 2) bn = *(const float4*)(brow + 2 * i + 2);
            __builtin_amdgcn_sched_barrier(0);
            const float4 av = A[i];
            // the sums first, then the six products in a fixed order
            const float sa0 = av.x + av.y, sb0 = bv.x + bv.y, sa1 = av.z + av.w, sb1 = bv.z + bv.w;
            __builtin_amdgcn_sched_barrier(0);
            p1 = __builtin_amdgcn_mfma_f32_16x16x4f32(av.x, bv.x, p1, 0, 0, 0);
            p2 = __builtin_amdgcn_mfma_f32_16x16x4f32(av.y, bv.y, p2, 0, 0, 0);
            p3 = __builtin_amdgcn_mfma_f32_16x16x4f32(sa0, sb0, p3, 0, 0, 0);
            p1 = __builtin_amdgcn_mfma_f32_16x16x4f32(av.z, bv.z, p1, 0, 0, 0);
            p2 = __builtin_amdgcn_mfma_f32_16x16x4f32(av.w, bv.w, p2, 0, 0, 0);
            p3 = __builtin_amdgcn_mfma_f32_16x16x4f32(sa1, sb1, p3, 0, 0, 0);
            __builtin_amdgcn_sched_barrier(0);
          }
          // column col = ct 16 + li is producer col / kWsSteps, step col % kWsSteps:
          // emission index (col / 4) JP + 4 ch + col % 4, written at 32 ch + col
          // (tail_ws_bit), so that a chunk fills 32 consecutive copies of a node
          static_assert(kWsRows == 32 && kWsSteps == 4 && kWsProducers == 8,
                        "the output index of tail_ws_bit");
          const int col = ct * 16 + li;
          const uint32_t j = (uint32_t)ch * kWsRows + (uint32_t)col;
#pragma unroll
          for (int e4 = 0; e4 < 4; ++e4) {
            const int rn = at * 16 + 4 * gq + e4;
            if (rn < Nn) tail_store(T, endb, Xs, s, rn, M, ne, j, p1[e4], p2[e4], p3[e4]);
          }
        }
      }
      // the next value's node tile, once this value's products have read A
      if (ch == nchunks - 1 && v + 1 < nv) load_a(v + 1);
      lds_barrier();
    }
  }
}

// Compute units of the current device (cached per device; 0 on error).
static int device_cus() {
  static int cus[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return 0;
  if (dev >= 64) {
    int n = 0;
    return hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess ? n : 0;
  }
  if (cus[dev] == 0) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    cus[dev] = n;
  }
  return cus[dev];
}

size_t tail_w_bytes(const TailDesc& h, int ns) {
  return (size_t)ns * ((size_t)1 << h.M) * ((size_t)1 << h.q) * sizeof(float2);
}

hipError_t launch_tail(const TailDesc& h, const TailDesc* d_desc, const DevOp* d_ops,
                       const float2* states, const uint32_t* svals, int s0, int ns, float2* W,
                       float2* X, hipStream_t st) {
  if (ns <= 0) return hipSuccess;
  if (h.fused) {
    const int R = 1 << (h.q - 6);
    if (!tail_fused_ok(h)) return hipErrorInvalidValue;
    dim3 g((unsigned)ns);
    if (h.ws) {
      if (!tail_ws_ok(h)) return hipErrorInvalidValue;
      // persistent workgroups: one per compute unit (the LDS holds one), each
      // taking every G-th value
      const int G = std::min(ns, device_cus());
      if (G <= 0) return hipErrorInvalidValue;
      dim3 gw((unsigned)G), b(kWsThreads);
      switch (R) {
        case 1: hipLaunchKernelGGL(k_tail_ws<1>, gw, b, 0, st, d_desc, d_ops, states, svals, s0, ns, X); break;
        case 2: hipLaunchKernelGGL(k_tail_ws<2>, gw, b, 0, st, d_desc, d_ops, states, svals, s0, ns, X); break;
        case 4: hipLaunchKernelGGL(k_tail_ws<4>, gw, b, 0, st, d_desc, d_ops, states, svals, s0, ns, X); break;
        default: return hipErrorInvalidValue;
      }
      return hipGetLastError();
    }
    dim3 b(kFusedThreads);
    switch (R) {
      case 1:
        hipLaunchKernelGGL(k_tail_fused<1>, g, b, 0, st, d_desc, d_ops, states, svals, s0, X);
        break;
      case 2:
        hipLaunchKernelGGL(k_tail_fused<2>, g, b, 0, st, d_desc, d_ops, states, svals, s0, X);
        break;
      case 4:
        hipLaunchKernelGGL(k_tail_fused<4>, g, b, 0, st, d_desc, d_ops, states, svals, s0, X);
        break;
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  const int lg = h.q < 6 ? h.q : 6;
  const uint64_t threads = ((uint64_t)ns << h.split_bits) << lg;
  const uint64_t blocks = (threads + kTailThreads - 1) / kTailThreads;
  const int R = h.q <= 6 ? 1 : (1 << (h.q - 6));
  {
    dim3 g((unsigned)blocks), b(kTailThreads);
    switch (R) {
      case 1: hipLaunchKernelGGL(k_tail_bwd<1>, g, b, 0, st, d_desc, d_ops, svals, s0, ns, W); break;
      case 2: hipLaunchKernelGGL(k_tail_bwd<2>, g, b, 0, st, d_desc, d_ops, svals, s0, ns, W); break;
      case 4: hipLaunchKernelGGL(k_tail_bwd<4>, g, b, 0, st, d_desc, d_ops, svals, s0, ns, W); break;
      case 8: hipLaunchKernelGGL(k_tail_bwd<8>, g, b, 0, st, d_desc, d_ops, svals, s0, ns, W); break;
      case 16: hipLaunchKernelGGL(k_tail_bwd<16>, g, b, 0, st, d_desc, d_ops, svals, s0, ns, W); break;
      default: return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  {
    const int Lam = 1 << h.M;
    dim3 g((unsigned)((Lam + kTN - 1) / kTN), (unsigned)((h.n_nodes + kTM - 1) / kTM), (unsigned)ns);
    if (g.y > 65535 || g.z > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_tail_mm, g, dim3(kTailThreads), 0, st, d_desc, W, states, svals, s0, X);
  }
  return hipGetLastError();
}

// ------------------------------------------------------------------ assembly GEMM
//
// C (M x N) = A B^T over the copy index k, complex64, with both operands stored
// with the copy index contiguous: A[i*lda + k] (upper half amplitudes at value
// i), B[j*ldb + k] (lower half at value j).  Each complex product is taken as
// three real ones: P1 = Ar Br, P2 = Ai Bi, P3 = (Ar + Ai)(Br + Bi), with
// Cre = P1 - P2 and Cim = P3 - P1 - P2.
//
// Workgroup tile 128 x 128 (4 waves of 64 x 64, each 4 x 4 MFMA tiles of
// 16 x 16).  The copy index is split over gridDim.z; each split writes a
// partial tile and k_zgemm_reduce adds the partials in a fixed order (the
// result does not depend on scheduling).

constexpr int kGemmThreads = 256;
constexpr int kGBM = 128, kGBN = 128;

static inline int round_up(int x, int m) { return (x + m - 1) / m * m; }

// FP32 MFMA: v_mfma_f32_16x16x4f32, K step 16 complex, LDS double-buffered.
// Each of the 2 x 2 waves owns TM x TN MFMA tiles (16 x 16 each), so the
// workgroup tile is (32 TM) x (32 TN).
constexpr int kFK = 16;
// Row padding of the staged tiles (complex values): odd, so that the threads
// that store different k of one row (8 or 4 k apart) land on different banks.
constexpr int kFPad = 1;
// Launch shape, measured at 1024 x 1024 outputs over 16384 copies against
// 128 x 64 tiles and other split counts: 128 x 128 tiles (255 VGPRs, two
// waves per SIMD), the split count sized so that every workgroup is resident
// at once (two per CU), and each XCD running whole splits.
constexpr int kF32TN = 4;     // MFMA tiles per wave along N: 2 -> 128 x 64, 4 -> 128 x 128
constexpr int kF32Slots = 2;  // resident workgroups per CU used to size the split count (0: 1024)
constexpr int kXcdMap = 1;    // 1: the workgroups of one split run on one XCD

// Block coordinates; with kXcdMap the linear workgroup id (dispatched to the
// eight XCDs round-robin) is remapped so that XCD g runs splits
// [g nz/8, (g+1) nz/8) and its L2 holds only those splits' copy range.
__device__ __forceinline__ void gemm_block(int& bx, int& by, int& bz) {
  bx = blockIdx.x;
  by = blockIdx.y;
  bz = blockIdx.z;
  if (kXcdMap && gridDim.z % 8 == 0) {
    const int nx = gridDim.x, ny = gridDim.y, nz = gridDim.z;
    const int bid = blockIdx.x + nx * (blockIdx.y + ny * blockIdx.z);
    const int xcd = bid & 7, loc = bid >> 3, per = nx * ny;
    bz = xcd * (nz / 8) + loc / per;
    const int r = loc % per;
    bx = r % nx;
    by = r / nx;
  }
}

template <int TM, int TN>
__global__ void __launch_bounds__(kGemmThreads)
k_zgemm_nt_f32(int M, int N, int K, int kper, const float2* __restrict__ A, int lda,
               const float2* __restrict__ B, int ldb, float2* __restrict__ out, int ldo,
               size_t split_stride, const int* __restrict__ goff, int nsplit, size_t a_gstride) {
  constexpr int BM = 32 * TM, BN = 32 * TN;
  __shared__ float2 As[2][kFK][BM + kFPad];
  __shared__ float2 Bs[2][kFK][BN + kFPad];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  int bx, by, bz;
  gemm_block(bx, by, bz);
  if (goff) {
    // grouped: z = group * nsplit + split; group g multiplies its own A
    // (a_gstride apart) with B rows goff[g] .. goff[g+1]-1 into the same
    // columns of the partial tile
    const int g = bz / nsplit;
    bz -= g * nsplit;
    const int c0 = goff[g];
    N = goff[g + 1] - c0;
    A += (size_t)g * a_gstride;
    B += (size_t)c0 * ldb;
    out += c0;
  }
  if (bx * BN >= N) return;  // a column tile past a group's end (the whole workgroup)
  const int i_blk = by * BM, j_blk = bx * BN;
  const int wi = (wave >> 1) * (16 * TM), wj = (wave & 1) * (16 * TN);
  const int kb = bz * kper;
  const int ke = min(K, kb + kper);
  floatx4 p1[TM][TN], p2[TM][TN], p3[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) {
      p1[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};
      p2[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};
      p3[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};
    }
  // staging: BM (BN) rows of kFK consecutive k; each thread takes VA (VB)
  // consecutive k of one row
  constexpr int VA = BM * kFK / kGemmThreads, VB = BN * kFK / kGemmThreads;
  static_assert(VA >= 1 && VB >= 1 && kFK % VA == 0 && kFK % VB == 0, "staging map");
  float2 ra[VA], rb[VB];
  const int ra_row = tid / (kFK / VA), ra_k = (tid % (kFK / VA)) * VA;
  const int rb_row = tid / (kFK / VB), rb_k = (tid % (kFK / VB)) * VB;
  auto gload = [&](int k0) {
    const int i = i_blk + ra_row, j = j_blk + rb_row;
#pragma unroll
    for (int x = 0; x < VA; ++x) {
      const int k = k0 + ra_k + x;
      ra[x] = (k < ke && i < M) ? A[(size_t)i * lda + k] : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int x = 0; x < VB; ++x) {
      const int k = k0 + rb_k + x;
      rb[x] = (k < ke && j < N) ? B[(size_t)j * ldb + k] : make_float2(0.f, 0.f);
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int x = 0; x < VA; ++x) As[buf][ra_k + x][ra_row] = ra[x];
#pragma unroll
    for (int x = 0; x < VB; ++x) Bs[buf][rb_k + x][rb_row] = rb[x];
  };
  int buf = 0;
  gload(kb);
  sstore(0);
  __syncthreads();
  for (int k0 = kb; k0 < ke; k0 += kFK) {
    const bool more = k0 + kFK < ke;
    if (more) gload(k0 + kFK);
#pragma unroll
    for (int kk = 0; kk < kFK; kk += 4) {
      float2 av[TM], bv[TN];
#pragma unroll
      for (int a = 0; a < TM; ++a) av[a] = As[buf][kk + (lane >> 4)][wi + a * 16 + (lane & 15)];
#pragma unroll
      for (int b = 0; b < TN; ++b) bv[b] = Bs[buf][kk + (lane >> 4)][wj + b * 16 + (lane & 15)];
#pragma unroll
      for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) {
          p1[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a].x, bv[b].x, p1[a][b], 0, 0, 0);
          p2[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a].y, bv[b].y, p2[a][b], 0, 0, 0);
          p3[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a].x + av[a].y, bv[b].x + bv[b].y,
                                                          p3[a][b], 0, 0, 0);
        }
    }
    if (more) {
      sstore(buf ^ 1);
      __syncthreads();
      buf ^= 1;
    }
  }
  float2* o = out + (size_t)bz * split_stride;
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int i = i_blk + wi + a * 16 + 4 * (lane >> 4) + e;
        const int j = j_blk + wj + b * 16 + (lane & 15);
        if (i < M && j < N)
          o[(size_t)i * ldo + j] = make_float2(p1[a][b][e] - p2[a][b][e],
                                               p3[a][b][e] - p1[a][b][e] - p2[a][b][e]);
      }
}

// s_waitcnt immediates (gfx9 encoding: vmcnt in bits 3:0 and 15:14, expcnt in
// 6:4, lgkmcnt in 11:8): wait until at most n vector memory operations of this
// wave are outstanding, whatever the other counters.  Issued through the
// builtin, so that the compiler's own wait insertion knows they happened.
constexpr int waitcnt_vm(int n) { return (n & 15) | ((n >> 4) << 14) | (7 << 4) | (15 << 8); }

// k_zgemm_nt_f32d: the same FP32 product with the operand tiles copied from
// HBM straight into a ring of kF32Stages LDS buffers (global_load_lds_dwordx4,
// no staging registers), so that the loads of step k + 2 are in flight while
// step k is multiplied.  A tile is row-major over the copy index (kFK complex
// values, 128 bytes a row); 16-byte chunk c of row r (copies 2c, 2c + 1) sits
// at position c ^ ((r >> 1) & 7), so that the sixteen rows of a fragment read
// fall on different banks.  A lane reads one chunk per tile row it feeds and
// uses its two copies in two MFMA steps (lane group g takes copies 2g and
// 2g + 1 of each eight-copy block).  Even K only (16-byte loads of complex
// pairs); grouped and plain forms as k_zgemm_nt_f32.
constexpr int kF32Stages = 3;
constexpr int kFRowBytes = kFK * 8;

__device__ __forceinline__ int f32_pos(int row, int c) { return c ^ ((row >> 1) & 7); }

// Rows row0 .. row0 + ROWS - 1 of src (rows of length K; rows past `rows` read
// the last row), copies k0 .. k0 + kFK - 1 (chunks past K read the row's first
// chunk: valid addresses, zeroed when the fragments are read).  Instruction j
// of wave w fills the 1 KB segment j * 4 + w (eight rows).
template <int ROWS>
__device__ __forceinline__ void f32_stage(const float2* __restrict__ src, size_t ld, int row0,
                                          int rows, int k0, int K, char* tile, int wave,
                                          int lane) {
  constexpr int PER = ROWS * (kFRowBytes / 16) / kGemmThreads;
  static_assert(PER >= 1 && ROWS * (kFRowBytes / 16) % kGemmThreads == 0, "staging map");
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int seg = j * (kGemmThreads / 64) + wave;
    const int r = seg * 8 + (lane >> 3);
    const int c = f32_pos(r, lane & 7);
    const int gr = min(row0 + r, rows - 1);
    const int k = k0 + 2 * c + 1 < K ? k0 + 2 * c : 0;
    __builtin_amdgcn_global_load_lds(src + (size_t)gr * ld + k,
                                     (__attribute__((address_space(3))) void*)(tile + seg * 1024),
                                     16, 0, 0);
  }
}

template <int TM, int TN>
__global__ void __launch_bounds__(kGemmThreads)
k_zgemm_nt_f32d(int M, int N, int K, int kper, const float2* __restrict__ A, int lda,
                const float2* __restrict__ B, int ldb, float2* __restrict__ out, int ldo,
                size_t split_stride, const int* __restrict__ goff, int nsplit, size_t a_gstride) {
  constexpr int BM = 32 * TM, BN = 32 * TN;
  constexpr int ABYTES = BM * kFRowBytes, BBYTES = BN * kFRowBytes;
  // loads per thread per step: one 16-byte chunk each
  constexpr int LPT = (BM + BN) * (kFRowBytes / 16) / kGemmThreads;
  static_assert(LPT == 6, "the wait count below assumes six loads per step");
  // one array per stage, so that the compiler can tell a stage's reads from
  // the other stages' loads in flight
  __shared__ __attribute__((aligned(16))) char ring0[ABYTES + BBYTES];
  __shared__ __attribute__((aligned(16))) char ring1[ABYTES + BBYTES];
  __shared__ __attribute__((aligned(16))) char ring2[ABYTES + BBYTES];
  static_assert(kF32Stages == 3, "three stage arrays");
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  int bx, by, bz;
  gemm_block(bx, by, bz);
  if (goff) {
    const int g = bz / nsplit;
    bz -= g * nsplit;
    const int c0 = goff[g];
    N = goff[g + 1] - c0;
    A += (size_t)g * a_gstride;
    B += (size_t)c0 * ldb;
    out += c0;
  }
  if (bx * BN >= N) return;  // a column tile past a group's end (the whole workgroup)
  const int i_blk = by * BM, j_blk = bx * BN;
  const int wi = (wave >> 1) * (16 * TM), wj = (wave & 1) * (16 * TN);
  const int kb = bz * kper;
  const int ke = min(K, kb + kper);
  const int nk = ke > kb ? (ke - kb + kFK - 1) / kFK : 0;
  floatx4 p1[TM][TN], p2[TM][TN], p3[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) {
      p1[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};
      p2[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};
      p3[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};
    }
  auto issue = [&](int t, char* buf) {
    f32_stage<BM>(A, (size_t)lda, i_blk, M, kb + t * kFK, K, buf, wave, lane);
    f32_stage<BN>(B, (size_t)ldb, j_blk, N, kb + t * kFK, K, buf + ABYTES, wave, lane);
  };
  if (nk > 0) issue(0, ring0);
  if (nk > 1) issue(1, ring1);
  const int g = lane >> 4, li = lane & 15;
  auto step = [&](int t, const char* buf, char* nxt) {
    // this step's chunks have landed: this wave's (at most the next step's
    // loads still in flight), then every wave's.  A bare s_barrier: the
    // workgroup has no LDS writes of its own to order, and every wave's reads
    // of the stage that the next loads overwrite were consumed before it got
    // here (a fenced barrier would also wait for the next step's loads).
    if (t + 1 < nk)
      __builtin_amdgcn_s_waitcnt(waitcnt_vm(LPT));
    else
      __builtin_amdgcn_s_waitcnt(waitcnt_vm(0));
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    if (t + 2 < nk) issue(t + 2, nxt);
    const int kvalid = min(kFK, ke - (kb + t * kFK));
#pragma unroll
    for (int kk = 0; kk < kFK; kk += 8) {
      float4 av[TM], bv[TN];
      const int c = kk / 2 + g;
#pragma unroll
      for (int a = 0; a < TM; ++a) {
        const int r = wi + a * 16 + li;
        av[a] = *(const float4*)(buf + r * kFRowBytes + 16 * f32_pos(r, c));
      }
#pragma unroll
      for (int b = 0; b < TN; ++b) {
        const int r = wj + b * 16 + li;
        bv[b] = *(const float4*)(buf + ABYTES + r * kFRowBytes + 16 * f32_pos(r, c));
      }
      if (kvalid < kFK) {
        // copies past this split's end (or past K) are zero
        const int k = kk + 2 * g;
        const bool z0 = k >= kvalid, z1 = k + 1 >= kvalid;
#pragma unroll
        for (int a = 0; a < TM; ++a) {
          if (z0) av[a].x = av[a].y = 0.f;
          if (z1) av[a].z = av[a].w = 0.f;
        }
#pragma unroll
        for (int b = 0; b < TN; ++b) {
          if (z0) bv[b].x = bv[b].y = 0.f;
          if (z1) bv[b].z = bv[b].w = 0.f;
        }
      }
#pragma unroll
      for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) {
          p1[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a].x, bv[b].x, p1[a][b], 0, 0, 0);
          p2[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a].y, bv[b].y, p2[a][b], 0, 0, 0);
          p3[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a].x + av[a].y, bv[b].x + bv[b].y,
                                                          p3[a][b], 0, 0, 0);
        }
#pragma unroll
      for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) {
          p1[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a].z, bv[b].z, p1[a][b], 0, 0, 0);
          p2[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a].w, bv[b].w, p2[a][b], 0, 0, 0);
          p3[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a].z + av[a].w, bv[b].z + bv[b].w,
                                                          p3[a][b], 0, 0, 0);
        }
    }
  };
  for (int t = 0; t < nk; t += 3) {
    step(t, ring0, ring2);
    if (t + 1 < nk) step(t + 1, ring1, ring0);
    if (t + 2 < nk) step(t + 2, ring2, ring1);
  }
  float2* o = out + (size_t)bz * split_stride;
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int i = i_blk + wi + a * 16 + 4 * (lane >> 4) + e;
        const int j = j_blk + wj + b * 16 + (lane & 15);
        if (i < M && j < N)
          o[(size_t)i * ldo + j] = make_float2(p1[a][b][e] - p2[a][b][e],
                                               p3[a][b][e] - p1[a][b][e] - p2[a][b][e]);
      }
}

// C[i][j] = (accumulate ? C[i][j] : 0) + sum over splits of P[z][i][j], in split order.
// (column j goes to C column cmap[j] when cmap is given)
// Thread jj of column block x takes column jj of rows y, y + gridDim.y, ...
__global__ void k_zgemm_reduce(int M, int N, int splits, const float2* __restrict__ P,
                               size_t split_stride, float2* __restrict__ C, int ldc, int accumulate,
                               const uint32_t* __restrict__ cmap) {
  const int jj = blockIdx.x * blockDim.x + threadIdx.x;
  if (jj >= N) return;
  const int j = cmap ? (int)cmap[jj] : jj;
  for (int i = blockIdx.y; i < M; i += gridDim.y) {
    float2 acc = accumulate ? C[(size_t)i * ldc + j] : make_float2(0.f, 0.f);
    for (int z = 0; z < splits; ++z) {
      const float2 p = P[(size_t)z * split_stride + (size_t)i * N + jj];
      acc.x += p.x;
      acc.y += p.y;
    }
    C[(size_t)i * ldc + j] = acc;
  }
}

static dim3 reduce_grid(int M, int N) {
  return dim3((unsigned)((N + 255) / 256), (unsigned)std::max(1, std::min(M, 65535)));
}

// Split-BF16: each FP32 value a is split as hi = bf16(a) (round to nearest
// even) and lo = bf16(a - hi); a product a*b is taken as
// hi_a hi_b + hi_a lo_b + lo_a hi_b (the dropped lo_a lo_b is below 2^-16
// relative), accumulated in FP32 on v_mfma_f32_16x16x32_bf16.  The operands
// are read as FP32 complex values (both with the copy index contiguous, as for
// the FP32 product) and split while they are staged: LDS holds four planes
// (re hi, re lo, im hi, im lo), each row-major over the M (or N) index with
// the copy index contiguous, so that a lane's eight consecutive k values are
// one 16-byte read.

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int kBK = 32;

__device__ __forceinline__ bf16x8 bf_neg(bf16x8 v) {
  u32x4 u = __builtin_bit_cast(u32x4, v);
  u ^= 0x80008000u;
  return __builtin_bit_cast(bf16x8, u);
}

// hi and lo bf16 halves of two FP32 values, packed (element 0 in the low half);
// conversions round to nearest even.
__device__ __forceinline__ void split2(float a, float b, uint32_t& hi, uint32_t& lo) {
  typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
  typedef float f32x2 __attribute__((ext_vector_type(2)));
  const f32x2 x = {a, b};
  const bf16x2 h = __builtin_convertvector(x, bf16x2);
  const bf16x2 l = __builtin_convertvector(x - __builtin_convertvector(h, f32x2), bf16x2);
  hi = __builtin_bit_cast(uint32_t, h);
  lo = __builtin_bit_cast(uint32_t, l);
}

// Staged operand tiles: 128 rows of kBK complex FP32 values (256 bytes per
// row, 32 KB per tile), written by direct global-to-LDS loads.  Inside a row
// the 16-byte chunks (two complex values each) are stored at position
// chunk ^ (row & 15), so that the sixteen rows a fragment read touches fall
// on sixteen different bank groups.
constexpr int kRowBytes = kBK * 8;
constexpr int kTileBytes = kGBM * kRowBytes;
// Waves of the split-BF16 product: 2 x 4 waves of 64 x 32 outputs each, two
// waves per SIMD (a 64 x 64 wave tile needs more than 256 registers)
constexpr int kBfWaves = 8;
constexpr int kBfThreads = 64 * kBfWaves;

__device__ __forceinline__ int chunk_pos(int row, int chunk) { return chunk ^ (row & 15); }

// One operand tile, rows row0 .. row0 + 127 of src (row length K), copy
// indices k0 .. k0 + kBK - 1.  Wave w of the product's kBfWaves loads tile rows
// 16 w .. 16 w + 15, four rows per instruction (64 lanes x 16 bytes: lane l
// covers row 4 j + l / 16 at position l % 16).  Rows past `rows` read the last row and chunks past K the
// row's first chunk (valid addresses; the first give outputs that are not
// stored, the second are zeroed when the fragments are read).
__device__ __forceinline__ void stage_tile(const float2* __restrict__ src, size_t ld, int row0,
                                           int rows, int k0, int K, char* tile, int wave,
                                           int lane) {
  const int pos = lane & 15;
  constexpr int RW = kGBM / kBfWaves;  // rows per wave
#pragma unroll
  for (int j = 0; j < RW / 4; ++j) {
    const int r = RW * wave + 4 * j + (lane >> 4);
    const int gr = min(row0 + r, rows - 1);
    const int c = pos ^ (r & 15);
    const int k = k0 + 2 * c + 1 < K ? k0 + 2 * c : 0;
    const float2* g = src + (size_t)gr * ld + k;
    char* l = tile + (RW * wave + 4 * j) * kRowBytes;
    __builtin_amdgcn_global_load_lds(g, (__attribute__((address_space(3))) void*)l, 16, 0, 0);
  }
}

// The four bf16 planes (re hi, re lo, im hi, im lo) of one MFMA fragment: row
// `row` of a staged tile, copy indices 8 g .. 8 g + 7; indices at or past kvalid
// are zero.
__device__ __forceinline__ void frag_planes(const char* tile, int row, int g, int kvalid,
                                            bf16x8 (&pl)[4]) {
  float4 v[4];
#pragma unroll
  for (int j = 0; j < 4; ++j)
    v[j] = *(const float4*)(tile + row * kRowBytes + 16 * chunk_pos(row, 4 * g + j));
  if (kvalid < kBK) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int k = 8 * g + 2 * j;
      if (k >= kvalid) v[j].x = v[j].y = 0.f;
      if (k + 1 >= kvalid) v[j].z = v[j].w = 0.f;
    }
  }
  u32x4 rh, rl, ih, il;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    uint32_t h, l;
    split2(v[j].x, v[j].z, h, l);
    rh[j] = h;
    rl[j] = l;
    split2(v[j].y, v[j].w, h, l);
    ih[j] = h;
    il[j] = l;
  }
  pl[0] = __builtin_bit_cast(bf16x8, rh);
  pl[1] = __builtin_bit_cast(bf16x8, rl);
  pl[2] = __builtin_bit_cast(bf16x8, ih);
  pl[3] = __builtin_bit_cast(bf16x8, il);
}

// C (M x N) = A B^T over the copy index, split-BF16: A[(a_row0 + i) * lda + k],
// B[j * ldb + k], both FP32 complex.  Tiles of 128 x 128 (eight waves of
// 64 x 32), k in steps of kBK, the copy index split over blockIdx.z as for the
// FP32 product (partials reduced by k_zgemm_reduce).  The next step's tiles
// load into the second LDS buffer while the MFMAs consume the current one.
// Grouped form (goff != nullptr): blockIdx.z = group * nsplit + split; group
// g takes the columns goff[g] .. goff[g+1]-1 (B rows, and the columns of the
// partial product) and A rows g * a_grows .. (its M rows); blockIdx.x counts
// the group's column tiles.  Plain form: blockIdx.z is the split.
__global__ void __launch_bounds__(kBfThreads)
k_zgemm_nt_bf16x3(int M, int N, int K, int kper, const float2* __restrict__ A, int lda,
                  const float2* __restrict__ B, int ldb, float2* __restrict__ out, int ldo,
                  size_t split_stride, const int* __restrict__ goff, int nsplit, int a_grows) {
  // [A, B] of each buffer, one array per buffer: the compiler then keeps the
  // next step's loads in flight while this step's tiles are read
  __shared__ __attribute__((aligned(16))) char tA0[kTileBytes];
  __shared__ __attribute__((aligned(16))) char tB0[kTileBytes];
  __shared__ __attribute__((aligned(16))) char tA1[kTileBytes];
  __shared__ __attribute__((aligned(16))) char tB1[kTileBytes];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  int bx, by, bz;
  gemm_block(bx, by, bz);  // an XCD runs whole splits: their operand tiles share its L2
  int split = bz, j_blk = bx * kGBN, jend = N, a_row0 = 0;
  if (goff) {
    const int g = bz / nsplit;
    split = bz - g * nsplit;
    j_blk = goff[g] + bx * kGBN;
    jend = goff[g + 1];
    if (j_blk >= jend) return;  // the whole tile lies past the group (uniform per block)
    a_row0 = g * a_grows;
  }
  const int i_blk = by * kGBM;
  const int wi = (wave >> 2) * 64, wj = (wave & 3) * 32;
  const int kb = split * kper;
  const int ke = min(K, kb + kper);
  const float2* Ag = A + (size_t)a_row0 * lda;
  floatx4 ar[4][2], ai[4][2];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      ar[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};
      ai[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};
    }
  auto issue = [&](int k0, char* ta, char* tb) {
    stage_tile(Ag, (size_t)lda, i_blk, M, k0, K, ta, wave, lane);
    stage_tile(B, (size_t)ldb, j_blk, jend, k0, K, tb, wave, lane);
  };
  const int g = lane >> 4, lr = lane & 15;
  auto step = [&](int k0, const char* ca, const char* cb, char* na, char* nb) {
    // this step's tiles have landed (this wave's loads, then every wave's).
    // A bare s_barrier: the workgroup writes LDS only through these loads, and
    // every wave consumed its reads of the buffer the next loads overwrite
    // before it got here.
    __builtin_amdgcn_s_waitcnt(waitcnt_vm(0));
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    if (k0 + kBK < ke) issue(k0 + kBK, na, nb);
    const int kvalid = min(kBK, ke - k0);
    bf16x8 fa[4][4];  // [a tile][plane]
#pragma unroll
    for (int a = 0; a < 4; ++a) frag_planes(ca, wi + a * 16 + lr, g, kvalid, fa[a]);
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      bf16x8 fb[4];
      frag_planes(cb, wj + b * 16 + lr, g, kvalid, fb);
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        floatx4 r = ar[a][b], im = ai[a][b];
        const bf16x8 nih = bf_neg(fa[a][2]), nil = bf_neg(fa[a][3]);
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[a][0], fb[0], r, 0, 0, 0);
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[a][0], fb[1], r, 0, 0, 0);
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[a][1], fb[0], r, 0, 0, 0);
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nih, fb[2], r, 0, 0, 0);
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nih, fb[3], r, 0, 0, 0);
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nil, fb[2], r, 0, 0, 0);
        im = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[a][0], fb[2], im, 0, 0, 0);
        im = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[a][0], fb[3], im, 0, 0, 0);
        im = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[a][1], fb[2], im, 0, 0, 0);
        im = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[a][2], fb[0], im, 0, 0, 0);
        im = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[a][2], fb[1], im, 0, 0, 0);
        im = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[a][3], fb[0], im, 0, 0, 0);
        ar[a][b] = r;
        ai[a][b] = im;
      }
    }
  };
  if (kb < ke) issue(kb, tA0, tB0);
  for (int k0 = kb; k0 < ke; k0 += 2 * kBK) {
    step(k0, tA0, tB0, tA1, tB1);
    if (k0 + kBK < ke) step(k0 + kBK, tA1, tB1, tA0, tB0);
  }
  float2* o = out + (size_t)split * split_stride;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int i = i_blk + wi + a * 16 + 4 * (lane >> 4) + e;
        const int j = j_blk + wj + b * 16 + (lane & 15);
        if (i < M && j < jend) o[(size_t)i * ldo + j] = make_float2(ar[a][b][e], ai[a][b][e]);
      }
}

// Eight consecutive complex values of one operand row (k .. k+7), split into
// the four planes of that row in LDS; values past the operand (row >= rows or
// k >= K) are zero.
__device__ __forceinline__ void stage_split8(const float2* __restrict__ src, size_t ld, int row,
                                             int rows, int k, int K,
                                             __hip_bfloat16 (*plane)[kGBM][kBK + 8], int lrow,
                                             int lk) {
  float4 v[4];
  const float2* r = src + (size_t)row * ld;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int kk = k + 2 * i;
    const float2 a = (row < rows && kk < K) ? r[kk] : make_float2(0.f, 0.f);
    const float2 b = (row < rows && kk + 1 < K) ? r[kk + 1] : make_float2(0.f, 0.f);
    v[i] = make_float4(a.x, a.y, b.x, b.y);
  }
  u32x4 rh, rl, ih, il;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    uint32_t h, l;
    split2(v[i].x, v[i].z, h, l);
    rh[i] = h;
    rl[i] = l;
    split2(v[i].y, v[i].w, h, l);
    ih[i] = h;
    il[i] = l;
  }
  *(u32x4*)(&plane[0][lrow][lk]) = rh;
  *(u32x4*)(&plane[1][lrow][lk]) = rl;
  *(u32x4*)(&plane[2][lrow][lk]) = ih;
  *(u32x4*)(&plane[3][lrow][lk]) = il;
}

// The same product with the operands staged through registers, value by
// value: for an odd copy count (a single copy), where the 16-byte direct
// loads of k_zgemm_nt_bf16x3 would run past a row.
__global__ void __launch_bounds__(kGemmThreads)
k_zgemm_nt_bf16x3_reg(int M, int N, int K, int kper, const float2* __restrict__ A, int lda,
                  const float2* __restrict__ B, int ldb, float2* __restrict__ out, int ldo,
                  size_t split_stride, const int* __restrict__ goff, int nsplit, int a_grows) {
  // LDS: [plane][row][k] with rows of kBK bf16 (64 bytes) plus 16 bytes of padding
  constexpr int RS = kBK + 8;
  __shared__ __attribute__((aligned(16))) __hip_bfloat16 As[4][kGBM][RS];
  __shared__ __attribute__((aligned(16))) __hip_bfloat16 Bs[4][kGBN][RS];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  int split = blockIdx.z, j_blk = blockIdx.x * kGBN, jend = N, a_row0 = 0;
  if (goff) {
    const int g = blockIdx.z / nsplit;
    split = blockIdx.z - g * nsplit;
    j_blk = goff[g] + blockIdx.x * kGBN;
    jend = goff[g + 1];
    if (j_blk >= jend) return;  // the whole tile lies past the group (uniform per block)
    a_row0 = g * a_grows;
  }
  const int i_blk = blockIdx.y * kGBM;
  const int wi = (wave >> 1) * 64, wj = (wave & 1) * 64;
  const int kb = split * kper;
  const int ke = min(K, kb + kper);
  const float2* Ag = A + (size_t)a_row0 * lda;
  floatx4 ar[4][4], ai[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      ar[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};
      ai[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};
    }
  for (int k0 = kb; k0 < ke; k0 += kBK) {
    // stage: 128 rows x 4 runs of 8 k per operand = 512 runs; 2 per thread
#pragma unroll
    for (int x = 0; x < 2; ++x) {
      const int c = tid + x * kGemmThreads;  // 0..511
      const int row = c >> 2, q = c & 3;
      stage_split8(Ag, (size_t)lda, i_blk + row, M, k0 + q * 8, ke, As, row, q * 8);
      stage_split8(B, (size_t)ldb, j_blk + row, jend, k0 + q * 8, ke, Bs, row, q * 8);
    }
    __syncthreads();
    bf16x8 fa[4][4];  // [a tile][plane]
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int p = 0; p < 4; ++p)
        fa[a][p] = *(const bf16x8*)(&As[p][wi + a * 16 + (lane & 15)][8 * (lane >> 4)]);
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      bf16x8 fb[4];
#pragma unroll
      for (int p = 0; p < 4; ++p)
        fb[p] = *(const bf16x8*)(&Bs[p][wj + b * 16 + (lane & 15)][8 * (lane >> 4)]);
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        floatx4 r = ar[a][b], im = ai[a][b];
        const bf16x8 nih = bf_neg(fa[a][2]), nil = bf_neg(fa[a][3]);
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[a][0], fb[0], r, 0, 0, 0);
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[a][0], fb[1], r, 0, 0, 0);
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[a][1], fb[0], r, 0, 0, 0);
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nih, fb[2], r, 0, 0, 0);
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nih, fb[3], r, 0, 0, 0);
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nil, fb[2], r, 0, 0, 0);
        im = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[a][0], fb[2], im, 0, 0, 0);
        im = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[a][0], fb[3], im, 0, 0, 0);
        im = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[a][1], fb[2], im, 0, 0, 0);
        im = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[a][2], fb[0], im, 0, 0, 0);
        im = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[a][2], fb[1], im, 0, 0, 0);
        im = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[a][3], fb[0], im, 0, 0, 0);
        ar[a][b] = r;
        ai[a][b] = im;
      }
    }
    __syncthreads();
  }
  float2* o = out + (size_t)split * split_stride;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int i = i_blk + wi + a * 16 + 4 * (lane >> 4) + e;
        const int j = j_blk + wj + b * 16 + (lane & 15);
        if (i < M && j < jend) o[(size_t)i * ldo + j] = make_float2(ar[a][b][e], ai[a][b][e]);
      }
}

namespace {

struct GemmShape {
  int bm, bn, tiles, splits, kper;
};

// Enough workgroups to fill the 256 compute units a few times over.
GemmShape gemm_shape(int prec, int M, int N, int K, int kstep) {
  GemmShape g;
  g.bm = 128;
  g.bn = prec == 0 ? 32 * kF32TN : 128;
  g.tiles = ((M + g.bm - 1) / g.bm) * ((N + g.bn - 1) / g.bn);
  const int wgs = prec == 0 && kF32Slots > 0 ? 256 * kF32Slots : 1024;
  const int want = std::max(1, wgs / std::max(1, g.tiles));
  const int maxsplit = std::max(1, K / (4 * kstep));
  g.splits = std::max(1, std::min({want, maxsplit, 64}));
  g.kper = round_up((K + g.splits - 1) / g.splits, kstep);
  g.splits = (K + g.kper - 1) / g.kper;
  return g;
}

}  // namespace

size_t zgemm_workspace_bytes(int prec, int M, int N, int K) {
  const int kstep = prec == 0 ? kFK : kBK;
  const int Kp = prec == 0 ? K : round_up(K, kBK);
  const GemmShape g = gemm_shape(prec, M, N, Kp, kstep);
  return (size_t)g.splits * M * N * sizeof(float2);
}

hipError_t launch_zgemm_tn(int prec, int M, int N, int K, const float2* A, int lda,
                           const float2* B, int ldb, float2* C, int ldc, int accumulate,
                           void* work, hipStream_t st, const uint32_t* cmap) {
  if (M <= 0 || N <= 0 || K <= 0) return hipErrorInvalidValue;
  const int kstep = prec == 0 ? kFK : kBK;
  const int Kp = prec == 0 ? K : round_up(K, kBK);
  const GemmShape g = gemm_shape(prec, M, N, Kp, kstep);
  const size_t ss = (size_t)M * N;
  float2* P = (float2*)work;
  dim3 grid((N + g.bn - 1) / g.bn, (M + g.bm - 1) / g.bm, g.splits);
  if (prec == 0) {
    hipLaunchKernelGGL((k_zgemm_nt_f32<4, kF32TN>), grid, dim3(kGemmThreads), 0, st, M, N, K, g.kper,
                       A, lda, B, ldb, P, N, ss, (const int*)nullptr, 1, (size_t)0);
  } else {
    if (K & 1)
      hipLaunchKernelGGL(k_zgemm_nt_bf16x3_reg, grid, dim3(kGemmThreads), 0, st, M, N, K, g.kper, A,
                         lda, B, ldb, P, N, ss, (const int*)nullptr, g.splits, 0);
    else
      hipLaunchKernelGGL(k_zgemm_nt_bf16x3, grid, dim3(kBfThreads), 0, st, M, N, K, g.kper, A, lda,
                         B, ldb, P, N, ss, (const int*)nullptr, g.splits, 0);
  }
  hipLaunchKernelGGL(k_zgemm_reduce, reduce_grid(M, N), dim3(256), 0, st, M, N,
                     g.splits, P, ss, C, ldc, accumulate, cmap);
  return hipGetLastError();
}

namespace {

// Groups hold about N / ngroups columns each, a few more or fewer: 64-wide
// column tiles waste less on the last, partly filled tile of a group than
// 128-wide ones (three resident workgroups per CU at this tile size).
constexpr int kGroupTN = 2;

GemmShape grouped_shape(int M, int maxn, int K, int ngroups) {
  GemmShape g;
  g.bm = 128;
  g.bn = 32 * kGroupTN;
  g.tiles = ((M + g.bm - 1) / g.bm) * ((maxn + g.bn - 1) / g.bn) * ngroups;
  const int wgs = 256 * 3;
  const int want = std::max(1, wgs / std::max(1, g.tiles));
  const int maxsplit = std::max(1, K / (4 * kFK));
  g.splits = std::max(1, std::min({want, maxsplit, 64}));
  g.kper = round_up((K + g.splits - 1) / g.splits, kFK);
  g.splits = (K + g.kper - 1) / g.kper;
  return g;
}

}  // namespace

size_t zgemm_grouped_workspace_bytes(int M, int Ntot, int maxn, int K, int ngroups) {
  const GemmShape g = grouped_shape(M, maxn, K, ngroups);
  return (size_t)g.splits * M * Ntot * sizeof(float2);
}

hipError_t launch_zgemm_grouped(int M, int Ntot, int maxn, int K, int ngroups, const int* d_goff,
                                const float2* A, size_t a_gstride, const float2* B, float2* C,
                                int ldc, int accumulate, void* work, hipStream_t st,
                                const uint32_t* cmap) {
  if (M <= 0 || Ntot <= 0 || K <= 0 || ngroups <= 0 || maxn <= 0) return hipErrorInvalidValue;
  const GemmShape g = grouped_shape(M, maxn, K, ngroups);
  const size_t ss = (size_t)M * Ntot;
  float2* P = (float2*)work;
  dim3 grid((maxn + g.bn - 1) / g.bn, (M + g.bm - 1) / g.bm, ngroups * g.splits);
  if (grid.z > 65535) return hipErrorInvalidValue;
  if (K & 1)
    hipLaunchKernelGGL((k_zgemm_nt_f32<4, kGroupTN>), grid, dim3(kGemmThreads), 0, st, M, Ntot, K,
                       g.kper, A, K, B, K, P, Ntot, ss, d_goff, g.splits, a_gstride);
  else
    hipLaunchKernelGGL((k_zgemm_nt_f32d<4, kGroupTN>), grid, dim3(kGemmThreads), 0, st, M, Ntot, K,
                       g.kper, A, K, B, K, P, Ntot, ss, d_goff, g.splits, a_gstride);
  hipLaunchKernelGGL(k_zgemm_reduce, reduce_grid(M, Ntot), dim3(256), 0, st, M, Ntot,
                     g.splits, P, ss, C, ldc, accumulate, cmap);
  return hipGetLastError();
}

// Grouped split-BF16 product: as launch_zgemm_grouped, one launch of
// k_zgemm_nt_bf16x3 over every group's column tiles (A holds ngroups * M rows
// of K, group g's M rows at row g * M; B Ntot rows of K).
struct GroupedBf16Shape {
  int tpg, mt, splits, kper;
};

GroupedBf16Shape grouped_bf16_shape(int M, int maxn, int K, int ngroups) {
  GroupedBf16Shape g;
  const int Kp = round_up(K, kBK);
  g.tpg = (maxn + kGBN - 1) / kGBN;
  g.mt = (M + kGBM - 1) / kGBM;
  const int tiles = std::max(1, g.tpg * g.mt * ngroups);
  const int want = std::max(1, 256 / tiles);  // longer k loops, fewer partials
  const int maxsplit = std::max(1, Kp / (4 * kBK));
  g.splits = std::max(1, std::min({want, maxsplit, 64}));
  g.kper = round_up((Kp + g.splits - 1) / g.splits, kBK);
  g.splits = (Kp + g.kper - 1) / g.kper;
  return g;
}

size_t zgemm_grouped_bf16_workspace_bytes(int M, int Ntot, int maxn, int K, int ngroups) {
  const GroupedBf16Shape g = grouped_bf16_shape(M, maxn, K, ngroups);
  return (size_t)g.splits * M * Ntot * sizeof(float2);
}

hipError_t launch_zgemm_grouped_bf16(int M, int Ntot, int maxn, int K, int ngroups,
                                     const int* d_goff, const float2* A, const float2* B,
                                     float2* C, int ldc, int accumulate, void* work,
                                     hipStream_t st, const uint32_t* cmap) {
  if (M <= 0 || Ntot <= 0 || K <= 0 || ngroups <= 0 || maxn <= 0) return hipErrorInvalidValue;
  const GroupedBf16Shape g = grouped_bf16_shape(M, maxn, K, ngroups);
  if ((size_t)ngroups * g.splits > 65535) return hipErrorInvalidValue;
  const size_t ss = (size_t)M * Ntot;
  float2* P = (float2*)work;
  dim3 grid(g.tpg, g.mt, ngroups * g.splits);
  if (K & 1)
    hipLaunchKernelGGL(k_zgemm_nt_bf16x3_reg, grid, dim3(kGemmThreads), 0, st, M, Ntot, K, g.kper, A,
                       K, B, K, P, Ntot, ss, d_goff, g.splits, M);
  else
    hipLaunchKernelGGL(k_zgemm_nt_bf16x3, grid, dim3(kBfThreads), 0, st, M, Ntot, K, g.kper, A, K,
                       B, K, P, Ntot, ss, d_goff, g.splits, M);
  hipLaunchKernelGGL(k_zgemm_reduce, reduce_grid(M, Ntot), dim3(256), 0, st, M, Ntot,
                     g.splits, P, ss, C, ldc, accumulate, cmap);
  return hipGetLastError();
}

// ------------------------------------------------------------------ small kernels

// out[row][j] = in[row][perm[j]] for every row (K columns): brings the lower
// half's copy order onto the upper half's.
__global__ void k_permute_cols(const float2* __restrict__ in, float2* __restrict__ out,
                               const uint32_t* __restrict__ perm, int rows, int K) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= K) return;
  const uint32_t pj = perm[j];
  for (int r = blockIdx.y; r < rows; r += gridDim.y)
    out[(size_t)r * K + j] = in[(size_t)r * K + pj];
}

// out[r][j] = in[rowsel[r]][colsel[j]] (in: rows of Kin, out: rows of Kout).
// Thread j of column block x takes column j of rows y, y + gridDim.y, ... (no
// index division per element).
__global__ void k_gather_rows_cols(const float2* __restrict__ in, float2* __restrict__ out,
                                   const uint32_t* __restrict__ rowsel,
                                   const uint32_t* __restrict__ colsel, int rows, int Kin,
                                   int Kout) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= Kout) return;
  const uint32_t cj = colsel[j];
  for (int r = blockIdx.y; r < rows; r += gridDim.y)
    out[(size_t)r * Kout + j] = in[(size_t)rowsel[r] * Kin + cj];
}

hipError_t launch_gather_rows_cols(const float2* in, float2* out, const uint32_t* rowsel,
                                   const uint32_t* colsel, int rows, int Kin, int Kout,
                                   hipStream_t st) {
  if (rows <= 0 || Kout <= 0) return hipSuccess;
  const dim3 g((unsigned)((Kout + 255) / 256), (unsigned)std::min(rows, 65535));
  hipLaunchKernelGGL(k_gather_rows_cols, g, dim3(256), 0, st, in, out, rowsel, colsel, rows, Kin,
                     Kout);
  return hipGetLastError();
}

// Walsh-Hadamard transform of the upper operand over the lower half's end
// cuts: out[sig][u][nu'] = sum_e (-1)^popc(e & sig) X[u][nu(nu', e)], where
// nu(nu', e) puts bit i of e at copy-order position pos[i] and the bits of
// nu' at the other positions (ascending).  The lower half's copy (nu', e) is
// its copy (nu', 0) times (-1)^popc(e & sig(l)), sig(l) = the lower value's
// bits on the end cuts' qubits, so the sum over copies becomes, for each sig,
// a product over nu' alone.
template <int NE>
__global__ void k_end_wht(const float2* __restrict__ X, int rows, int K, uint32_t pos_packed,
                          float2* __restrict__ out) {
  constexpr int E = 1 << NE;
  const int K0 = K >> NE;
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (size_t)rows * K0) return;
  const size_t u = t / K0;
  const uint32_t v0 = (uint32_t)(t % K0);
  int pos[NE];
#pragma unroll
  for (int i = 0; i < NE; ++i) pos[i] = (int)((pos_packed >> (5 * i)) & 31);
  // nu' -> nu with zeros at the end positions, taken in ascending order
  uint32_t nu = v0;
#pragma unroll
  for (int a = 0; a < NE; ++a) {
    int p = 32;  // a-th smallest position
#pragma unroll
    for (int i = 0; i < NE; ++i) {
      int rank = 0;
#pragma unroll
      for (int i2 = 0; i2 < NE; ++i2) rank += pos[i2] < pos[i] ? 1 : 0;
      if (rank == a) p = pos[i];
    }
    nu = ((nu >> p) << (p + 1)) | (nu & ((1u << p) - 1u));
  }
  float2 x[E];
  const float2* row = X + u * (size_t)K;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    uint32_t o = nu;
#pragma unroll
    for (int i = 0; i < NE; ++i)
      if ((e >> i) & 1) o |= 1u << pos[i];
    x[e] = row[o];
  }
#pragma unroll
  for (int h = 1; h < E; h <<= 1)
#pragma unroll
    for (int e = 0; e < E; ++e)
      if (!(e & h)) {
        const float2 a = x[e], b = x[e | h];
        x[e] = make_float2(a.x + b.x, a.y + b.y);
        x[e | h] = make_float2(a.x - b.x, a.y - b.y);
      }
  const size_t plane = (size_t)rows * K0;
#pragma unroll
  for (int e = 0; e < E; ++e) out[(size_t)e * plane + t] = x[e];
}

hipError_t launch_end_wht(const float2* X, int rows, int K, int ne, const int* pos, float2* out,
                          hipStream_t st) {
  if (ne < 1 || ne > 4 || (K >> ne) < 1) return hipErrorInvalidValue;
  uint32_t pk = 0;
  for (int i = 0; i < ne; ++i) {
    if (pos[i] < 0 || pos[i] > 30) return hipErrorInvalidValue;
    pk |= (uint32_t)pos[i] << (5 * i);
  }
  const size_t tot = (size_t)rows * (size_t)(K >> ne);
  if (tot == 0) return hipSuccess;
  dim3 g((unsigned)((tot + 255) / 256)), b(256);
  switch (ne) {
    case 1: hipLaunchKernelGGL(k_end_wht<1>, g, b, 0, st, X, rows, K, pk, out); break;
    case 2: hipLaunchKernelGGL(k_end_wht<2>, g, b, 0, st, X, rows, K, pk, out); break;
    case 3: hipLaunchKernelGGL(k_end_wht<3>, g, b, 0, st, X, rows, K, pk, out); break;
    case 4: hipLaunchKernelGGL(k_end_wht<4>, g, b, 0, st, X, rows, K, pk, out); break;
  }
  return hipGetLastError();
}

hipError_t launch_permute_cols(const float2* in, float2* out, const uint32_t* perm, int rows,
                               int K, hipStream_t st) {
  if (rows <= 0 || K <= 0) return hipSuccess;
  const dim3 g((unsigned)((K + 255) / 256), (unsigned)std::min(rows, 65535));
  hipLaunchKernelGGL(k_permute_cols, g, dim3(256), 0, st, in, out, perm, rows, K);
  return hipGetLastError();
}

// Sum over copies for one bitstring per wavefront; lanes stride over k, then
// a fixed-order butterfly reduction.
__global__ void __launch_bounds__(256)
k_gathered_dot(int K, const float2* __restrict__ A, int lda, const float2* __restrict__ B, int ldb,
               const int* __restrict__ iu, const int* __restrict__ il, size_t m,
               float2* __restrict__ amps, int accumulate, float2 phi) {
  const size_t t = ((size_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (t >= m) return;
  const int u = iu[t], l = il[t];
  float re = 0.f, im = 0.f;
  for (int k = lane; k < K; k += 64) {
    const float2 a = A[(size_t)u * lda + k], b = B[(size_t)l * ldb + k];
    re += a.x * b.x - a.y * b.y;
    im += a.x * b.y + a.y * b.x;
  }
  for (int w = 32; w > 0; w >>= 1) {
    re += __shfl_xor(re, w);
    im += __shfl_xor(im, w);
  }
  if (lane == 0) {
    float2 o = cmul(make_float2(re, im), phi);
    if (accumulate) {
      o.x += amps[t].x;
      o.y += amps[t].y;
    }
    amps[t] = o;
  }
}

hipError_t launch_gathered_dot(int K, const float2* A, int lda, const float2* B, int ldb,
                               const int* iu, const int* il, size_t m, float2* amps,
                               int accumulate, float2 phi, hipStream_t st) {
  if (m == 0 || K <= 0) return hipSuccess;
  const size_t blocks = (m * 64 + 255) / 256;
  hipLaunchKernelGGL(k_gathered_dot, dim3((unsigned)blocks), dim3(256), 0, st, K, A, lda, B, ldb,
                     iu, il, m, amps, accumulate, phi);
  return hipGetLastError();
}

constexpr int kProbThreads = 256;
constexpr int kProbPerBlock = 1024;

int prob_partial_blocks(size_t m) { return (int)((m + kProbPerBlock - 1) / kProbPerBlock); }

__global__ void __launch_bounds__(kProbThreads)
k_prob_partial(const float2* __restrict__ amps, size_t m, double* __restrict__ partial) {
  __shared__ double s1[kProbThreads], s2[kProbThreads];
  const size_t base = (size_t)blockIdx.x * kProbPerBlock;
  double a1 = 0, a2 = 0;
  for (int i = threadIdx.x; i < kProbPerBlock; i += kProbThreads) {
    const size_t t = base + i;
    if (t < m) {
      const double re = amps[t].x, im = amps[t].y;
      const double p = re * re + im * im;
      a1 += p;
      a2 += p * p;
    }
  }
  s1[threadIdx.x] = a1;
  s2[threadIdx.x] = a2;
  __syncthreads();
  for (int w = kProbThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      s1[threadIdx.x] += s1[threadIdx.x + w];
      s2[threadIdx.x] += s2[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = s1[0];
    partial[2 * blockIdx.x + 1] = s2[0];
  }
}

// One workgroup: thread t sums partials t, t + 256, ... in order, then a
// fixed tree over the threads (the order does not depend on scheduling).
__global__ void __launch_bounds__(kProbThreads)
k_prob_final(const double* __restrict__ partial, int nb, double* __restrict__ out) {
  __shared__ double s1[kProbThreads], s2[kProbThreads];
  double a1 = 0, a2 = 0;
  for (int b = threadIdx.x; b < nb; b += kProbThreads) {
    a1 += partial[2 * b];
    a2 += partial[2 * b + 1];
  }
  s1[threadIdx.x] = a1;
  s2[threadIdx.x] = a2;
  __syncthreads();
  for (int w = kProbThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      s1[threadIdx.x] += s1[threadIdx.x + w];
      s2[threadIdx.x] += s2[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = s1[0];
    out[1] = s2[0];
  }
}

// The output amplitudes amps[t] = phi C[iu[t] ldc + il[t]] and their FP64
// partial sums in one pass: each workgroup gathers its kProbPerBlock
// amplitudes, writes them, and sums them in the same order as k_prob_partial
// does over stored amplitudes.
__global__ void __launch_bounds__(kProbThreads)
k_gather_prob_partial(const float2* __restrict__ C, int ldc, const int* __restrict__ iu,
                      const int* __restrict__ il, size_t m, float2* __restrict__ amps, float2 phi,
                      double* __restrict__ partial) {
  __shared__ double s1[kProbThreads], s2[kProbThreads];
  const size_t base = (size_t)blockIdx.x * kProbPerBlock;
  double a1 = 0, a2 = 0;
  for (int i = threadIdx.x; i < kProbPerBlock; i += kProbThreads) {
    const size_t t = base + i;
    if (t < m) {
      const float2 a = cmul(C[(size_t)iu[t] * ldc + il[t]], phi);
      amps[t] = a;
      const double re = a.x, im = a.y;
      const double p = re * re + im * im;
      a1 += p;
      a2 += p * p;
    }
  }
  s1[threadIdx.x] = a1;
  s2[threadIdx.x] = a2;
  __syncthreads();
  for (int w = kProbThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      s1[threadIdx.x] += s1[threadIdx.x + w];
      s2[threadIdx.x] += s2[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = s1[0];
    partial[2 * blockIdx.x + 1] = s2[0];
  }
}

hipError_t launch_gather_prob_sums(const float2* C, int ldc, const int* iu, const int* il,
                                   size_t m, float2* amps, float2 phi, double* partial,
                                   double* out, hipStream_t st) {
  const int nb = prob_partial_blocks(m);
  if (nb == 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_gather_prob_partial, dim3(nb), dim3(kProbThreads), 0, st, C, ldc, iu, il,
                     m, amps, phi, partial);
  hipLaunchKernelGGL(k_prob_final, dim3(1), dim3(kProbThreads), 0, st, partial, nb, out);
  return hipGetLastError();
}

hipError_t launch_prob_sums(const float2* amps, size_t m, double* partial, double* out,
                            hipStream_t st) {
  const int nb = prob_partial_blocks(m);
  if (nb == 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_prob_partial, dim3(nb), dim3(kProbThreads), 0, st, amps, m, partial);
  hipLaunchKernelGGL(k_prob_final, dim3(1), dim3(kProbThreads), 0, st, partial, nb, out);
  return hipGetLastError();
}

// ------------------------------------------------------------------ static scratch
//
// Scratch of the allocation-free assembly (qs_amplitudes_device_static): the
// value grid C, the split-K partial products, the split-BF16 operand planes
// and the FP64 partial sums, carved from one region per device that lives as
// long as the process.  In host code the array's name is not a device
// address: the address comes from hipGetSymbolAddress, once per device.

constexpr size_t kStaticScratchBytes = (size_t)256 << 20;
static __device__ __align__(256) char assembly_scratch[kStaticScratchBytes];

size_t static_scratch_capacity() { return kStaticScratchBytes; }

hipError_t static_scratch(void** base) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  static std::mutex mu;
  static std::map<int, void*> addr;  // device -> address of its copy of assembly_scratch
  std::lock_guard<std::mutex> lock(mu);
  auto it = addr.find(dev);
  if (it == addr.end()) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(assembly_scratch));
    if (e != hipSuccess) return e;
    if (p == nullptr) return hipErrorInvalidSymbol;
    it = addr.emplace(dev, p).first;
  }
  *base = it->second;
  return hipSuccess;
}

__global__ void k_fill_zero(uint32_t* __restrict__ p, size_t words) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t k = i; k < words; k += stride) p[k] = 0u;
}

hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t st) {
  const size_t words = bytes / 4;
  if (words == 0) return hipSuccess;
  size_t blocks = (words + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)blocks), dim3(256), 0, st, (uint32_t*)p, words);
  return hipGetLastError();
}

}  // namespace qs
