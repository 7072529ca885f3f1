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

__global__ void __launch_bounds__(kPassThreads)
k_pass(const PassDesc* __restrict__ pdp, const DevOp* __restrict__ ops,
       const float2* __restrict__ in, float2* __restrict__ out) {
  extern __shared__ float2 smem[];
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
  lds_apply_ops(A, ops + P.op_in, P.n_in, t, tbit, outer);
  if (P.m == 0) {
    for (int i = threadIdx.x; i < size; i += kPassThreads) {
      const uint32_t x = outer | deposit_tile(i, tbit, t);
      out[node * N + x] = A[i];
    }
    return;
  }
  float2* Bb = smem + size;
  const int m = P.m;
  for (int b = 0; b < (1 << m); ++b) {
    for (int i = threadIdx.x; i < size; i += kPassThreads) {
      const uint32_t x = outer | deposit_tile(i, tbit, t);
      float2 v = A[i];
      for (int k = 0; k < m; ++k) {
        const uint32_t want = (b >> (m - 1 - k)) & 1;
        const uint32_t xb = (x >> P.bq[k]) & 1;
        if (P.upper) {
          if (xb != want) v = make_float2(0.f, 0.f);
        } else if (want & xb) {
          v = make_float2(-v.x, -v.y);
        }
      }
      Bb[i] = v;
    }
    __syncthreads();
    lds_apply_ops(Bb, ops + P.op_out, P.n_out, t, tbit, outer);
    const uint64_t child = (node << m) | (uint64_t)b;
    for (int i = threadIdx.x; i < size; i += kPassThreads) {
      const uint32_t x = outer | deposit_tile(i, tbit, t);
      out[child * N + x] = Bb[i];
    }
    __syncthreads();
  }
}

hipError_t launch_pass(const PassDesc& h, const PassDesc* d_desc, const DevOp* d_ops,
                       const float2* in, float2* out, uint64_t n_in_nodes, hipStream_t st) {
  const uint64_t blocks = n_in_nodes << h.n_outer;
  if (blocks == 0 || blocks > 0x7fffffffull) return hipErrorInvalidValue;
  const size_t lds = (size_t)(h.m > 0 ? 2 : 1) * ((size_t)8 << h.t);
  hipLaunchKernelGGL(k_pass, dim3((unsigned)blocks), dim3(kPassThreads), lds, st, d_desc, d_ops,
                     in, out);
  return hipGetLastError();
}

// ------------------------------------------------------------------ leaf evaluation

constexpr int kTailThreads = 256;

template <int R>
struct TailCtx {
  uint32_t xs[R];
  int g;       // lane inside the group
  int lg;      // log2 of the group width
  uint32_t s;  // requested half value
  int si;      // its index
};

template <int R>
__device__ __forceinline__ void tail_mat_reg(float2 (&v)[R], const float* m, int rb) {
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

template <int R>
__device__ __forceinline__ void tail_apply_ops(float2 (&v)[R], const TailCtx<R>& c,
                                               const DevOp* __restrict__ ops, int nops) {
  for (int o = 0; o < nops; ++o) {
    const DevOp& op = ops[o];
    if (op.kind == 0) {
      const int w = op.target;
      if (w < c.lg) {
        const int bit = (c.g >> w) & 1;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          float2 p;
          p.x = __shfl_xor(v[r].x, 1 << w);
          p.y = __shfl_xor(v[r].y, 1 << w);
          float2 oa, ob;
          if (bit) mat_apply(op.m, p, v[r], oa, ob), v[r] = ob;
          else mat_apply(op.m, v[r], p, oa, ob), v[r] = oa;
        }
      } else {
        const int rb = w - c.lg;
        if constexpr (R >= 2) { if (rb == 0) tail_mat_reg<R>(v, op.m, 0); }
        if constexpr (R >= 4) { if (rb == 1) tail_mat_reg<R>(v, op.m, 1); }
        if constexpr (R >= 8) { if (rb == 2) tail_mat_reg<R>(v, op.m, 2); }
        if constexpr (R >= 16) { if (rb == 3) tail_mat_reg<R>(v, op.m, 3); }
      }
    } else {
#pragma unroll
      for (int r = 0; r < R; ++r) v[r] = diag_apply(op, c.xs[r], v[r]);
    }
  }
}

template <int R>
__device__ __forceinline__ void tail_emit(const float2 (&v)[R], const TailCtx<R>& c,
                                          const TailDesc& T, uint64_t kap, float2* __restrict__ X) {
  // the requested index s sits at working index ys
  uint32_t ys = 0;
  for (int i = 0; i < T.q; ++i) ys |= ((c.s >> T.Q[i]) & 1u) << i;
  const int G = 1 << c.lg;
  if ((int)(ys & (G - 1)) != c.g) return;
  const int rr = ys >> c.lg;
  float2 val = v[0];
#pragma unroll
  for (int r = 1; r < R; ++r)
    if (r == rr) val = v[r];
  const int ne = T.n_end;
  for (int e = 0; e < (1 << ne); ++e) {
    float2 f = val;
    uint64_t k = kap;
    for (int i = 0; i < ne; ++i) {
      const uint32_t eb = (e >> (ne - 1 - i)) & 1;
      const uint32_t sb = (c.s >> T.eq[i]) & 1;
      if (eb) k |= T.ekbit[i];
      if (T.upper) {
        if (eb != sb) f = make_float2(0.f, 0.f);
      } else if (eb & sb) {
        f = make_float2(-f.x, -f.y);
      }
    }
    X[k * (uint64_t)T.ldx + c.si] = f;
  }
}

template <int R, int D>
__device__ __forceinline__ void tail_rec(const float2 (&v)[R], const TailCtx<R>& c,
                                         const TailDesc& T, const DevOp* __restrict__ ops,
                                         uint64_t kap, float2* __restrict__ X) {
  if constexpr (D >= kMaxTailLevels) {
    tail_emit<R>(v, c, T, kap, X);
  } else {
    if (D == T.nlev) {
      tail_emit<R>(v, c, T, kap, X);
      return;
    }
    const TailLevel& L = T.lev[D];
    const int m = L.m;
    for (int b = 0; b < (1 << m); ++b) {
      float2 w[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        float2 a = v[r];
        for (int k = 0; k < m; ++k) {
          const uint32_t want = (b >> (m - 1 - k)) & 1;
          const uint32_t xb = (c.xs[r] >> L.bq[k]) & 1;
          if (T.upper) {
            if (xb != want) a = make_float2(0.f, 0.f);
          } else if (want & xb) {
            a = make_float2(-a.x, -a.y);
          }
        }
        w[r] = a;
      }
      tail_apply_ops<R>(w, c, ops + L.op0, L.nops);
      uint64_t k2 = kap;
      for (int k = 0; k < m; ++k)
        if ((b >> (m - 1 - k)) & 1) k2 |= L.kbit[k];
      tail_rec<R, D + 1>(w, c, T, ops, k2, X);
    }
  }
}

template <int R>
__global__ void __launch_bounds__(kTailThreads)
k_tail(const TailDesc* __restrict__ tdp, const DevOp* __restrict__ ops,
       const float2* __restrict__ states, const uint32_t* __restrict__ svals,
       const uint64_t* __restrict__ node_k, float2* __restrict__ X) {
  const TailDesc& T = *tdp;
  const int lg = T.q < 6 ? T.q : 6;
  const int G = 1 << lg;
  const uint64_t gtid = (uint64_t)blockIdx.x * kTailThreads + threadIdx.x;
  const uint64_t gid = gtid >> lg;
  const uint64_t total = (uint64_t)T.n_nodes * (uint64_t)T.S;
  if (gid >= total) return;
  TailCtx<R> c;
  c.g = (int)(gtid & (G - 1));
  c.lg = lg;
  const uint64_t node = gid / (uint64_t)T.S;
  c.si = (int)(gid % (uint64_t)T.S);
  c.s = svals[c.si];
  uint32_t qmask = 0;
  for (int i = 0; i < T.q; ++i) qmask |= 1u << T.Q[i];
  const uint32_t base = c.s & ~qmask;
  const float2* st = states + node * (1ull << T.n);
  float2 v[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const uint32_t y = (uint32_t)(c.g + (r << lg));
    uint32_t x = base;
    for (int i = 0; i < T.q; ++i) x |= ((y >> i) & 1u) << T.Q[i];
    c.xs[r] = x;
    v[r] = st[x];
  }
  tail_rec<R, 0>(v, c, T, ops, node_k[node], X);
}

hipError_t launch_tail(const TailDesc& h, const TailDesc* d_desc, const DevOp* d_ops,
                       const float2* states, const uint32_t* svals, const uint64_t* node_k,
                       float2* X, hipStream_t st) {
  const int lg = h.q < 6 ? h.q : 6;
  const uint64_t groups = (uint64_t)h.n_nodes * (uint64_t)h.S;
  const uint64_t threads = groups << lg;
  const uint64_t blocks = (threads + kTailThreads - 1) / kTailThreads;
  if (blocks == 0 || blocks > 0x7fffffffull) return hipErrorInvalidValue;
  const int R = h.q <= 6 ? 1 : (1 << (h.q - 6));
  dim3 g((unsigned)blocks), b(kTailThreads);
  switch (R) {
    case 1: hipLaunchKernelGGL(k_tail<1>, g, b, 0, st, d_desc, d_ops, states, svals, node_k, X); break;
    case 2: hipLaunchKernelGGL(k_tail<2>, g, b, 0, st, d_desc, d_ops, states, svals, node_k, X); break;
    case 4: hipLaunchKernelGGL(k_tail<4>, g, b, 0, st, d_desc, d_ops, states, svals, node_k, X); break;
    case 8: hipLaunchKernelGGL(k_tail<8>, g, b, 0, st, d_desc, d_ops, states, svals, node_k, X); break;
    case 16: hipLaunchKernelGGL(k_tail<16>, g, b, 0, st, d_desc, d_ops, states, svals, node_k, X); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ------------------------------------------------------------------ assembly GEMM (FP32 MFMA)
//
// C (M x N) = A^T B with A stored k-major (A[k*lda + i]) and B stored k-major
// (B[k*ldb + j]), complex64.  Real form: Cre = Are Bre - Aim Bim,
// Cim = Are Bim + Aim Bre, each product on v_mfma_f32_16x16x4f32.

constexpr int kGemmThreads = 256;
constexpr int kGBM = 64, kGBN = 64, kGBK = 16;

__global__ void __launch_bounds__(kGemmThreads)
k_zgemm_tn_f32(int M, int N, int K, const float2* __restrict__ A, int lda,
               const float2* __restrict__ B, int ldb, float2* __restrict__ C, int ldc,
               int accumulate) {
  __shared__ float2 As[kGBK][kGBM];
  __shared__ float2 Bs[kGBK][kGBN];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int i_blk = blockIdx.y * kGBM, j_blk = blockIdx.x * kGBN;
  const int wi = (wave >> 1) * 32, wj = (wave & 1) * 32;
  floatx4 acc_re[2][2], acc_im[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      acc_re[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};
      acc_im[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};
    }
  for (int k0 = 0; k0 < K; k0 += kGBK) {
    for (int e = tid; e < kGBK * kGBM; e += kGemmThreads) {
      const int kk = e / kGBM, ii = e % kGBM;
      const int k = k0 + kk;
      As[kk][ii] = (k < K && i_blk + ii < M) ? A[(size_t)k * lda + i_blk + ii] : make_float2(0.f, 0.f);
      Bs[kk][ii] = (k < K && j_blk + ii < N) ? B[(size_t)k * ldb + j_blk + ii] : make_float2(0.f, 0.f);
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kGBK; kk += 4) {
      float2 av[2], bv[2];
      for (int a = 0; a < 2; ++a) av[a] = As[kk + (lane >> 4)][wi + a * 16 + (lane & 15)];
      for (int b = 0; b < 2; ++b) bv[b] = Bs[kk + (lane >> 4)][wj + b * 16 + (lane & 15)];
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
          acc_re[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a].x, bv[b].x, acc_re[a][b], 0, 0, 0);
          acc_re[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(-av[a].y, bv[b].y, acc_re[a][b], 0, 0, 0);
          acc_im[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a].x, bv[b].y, acc_im[a][b], 0, 0, 0);
          acc_im[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a].y, bv[b].x, acc_im[a][b], 0, 0, 0);
        }
    }
    __syncthreads();
  }
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int e = 0; e < 4; ++e) {
        const int i = i_blk + wi + a * 16 + 4 * (lane >> 4) + e;
        const int j = j_blk + wj + b * 16 + (lane & 15);
        if (i < M && j < N) {
          float2 r = make_float2(acc_re[a][b][e], acc_im[a][b][e]);
          float2* p = C + (size_t)i * ldc + j;
          if (accumulate) {
            float2 o = *p;
            r.x += o.x;
            r.y += o.y;
          }
          *p = r;
        }
      }
}

hipError_t launch_zgemm_tn_f32(int M, int N, int K, const float2* A, int lda, const float2* B,
                               int ldb, float2* C, int ldc, int accumulate, hipStream_t st) {
  if (M <= 0 || N <= 0 || K <= 0) return hipErrorInvalidValue;
  dim3 g((N + kGBN - 1) / kGBN, (M + kGBM - 1) / kGBM);
  hipLaunchKernelGGL(k_zgemm_tn_f32, g, dim3(kGemmThreads), 0, st, M, N, K, A, lda, B, ldb, C,
                     ldc, accumulate);
  return hipGetLastError();
}

// ------------------------------------------------------------------ split-BF16 assembly
//
// Each FP32 value a is split as hi = bf16(a) (round to nearest even) and
// lo = bf16(a - hi).  A product a*b is taken as hi_a hi_b + hi_a lo_b + lo_a hi_b
// (the lo*lo term, below 2^-16 relative, is dropped), accumulated in FP32 on
// v_mfma_f32_16x16x32_bf16.  The split operands are staged in planar form
// [k][i] per component (re, im) and part (hi, lo).

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__global__ void k_split_bf16(const float2* __restrict__ src, int ld, int rows, int cols,
                             int cols_pad, __hip_bfloat16* __restrict__ dst) {
  // dst planes: [4][rows_pad][cols_pad] = re_hi, re_lo, im_hi, im_lo; rows_pad = rows rounded to 32
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int rows_pad = (rows + 31) & ~31;
  const size_t plane = (size_t)rows_pad * cols_pad;
  if (idx >= plane) return;
  const int k = (int)(idx / cols_pad), i = (int)(idx % cols_pad);
  float2 v = (k < rows && i < cols) ? src[(size_t)k * ld + i] : make_float2(0.f, 0.f);
  __hip_bfloat16 rh = __float2bfloat16(v.x);
  __hip_bfloat16 rl = __float2bfloat16(v.x - __bfloat162float(rh));
  __hip_bfloat16 ih = __float2bfloat16(v.y);
  __hip_bfloat16 il = __float2bfloat16(v.y - __bfloat162float(ih));
  dst[idx] = rh;
  dst[plane + idx] = rl;
  dst[2 * plane + idx] = ih;
  dst[3 * plane + idx] = il;
}

constexpr int kBBM = 64, kBBN = 64, kBBK = 32;

__global__ void __launch_bounds__(kGemmThreads)
k_zgemm_tn_bf16x3(int M, int N, int Kp, const __hip_bfloat16* __restrict__ Ap, int ldap,
                  const __hip_bfloat16* __restrict__ Bp, int ldbp, float2* __restrict__ C, int ldc,
                  int accumulate) {
  // planes: Ap[p * Kp * ldap + k * ldap + i], p = 0 re_hi, 1 re_lo, 2 im_hi, 3 im_lo
  __shared__ __hip_bfloat16 As[4][kBBK][kBBM];
  __shared__ __hip_bfloat16 Bs[4][kBBK][kBBN];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int i_blk = blockIdx.y * kBBM, j_blk = blockIdx.x * kBBN;
  const int wi = (wave >> 1) * 32, wj = (wave & 1) * 32;
  const size_t pa = (size_t)Kp * ldap, pb = (size_t)Kp * ldbp;
  floatx4 acc_re[2][2], acc_im[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      acc_re[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};
      acc_im[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};
    }
  for (int k0 = 0; k0 < Kp; k0 += kBBK) {
    for (int e = tid; e < kBBK * kBBM; e += kGemmThreads) {
      const int kk = e / kBBM, ii = e % kBBM;
      const size_t ka = (size_t)(k0 + kk) * ldap, kb = (size_t)(k0 + kk) * ldbp;
      for (int p = 0; p < 4; ++p) {
        As[p][kk][ii] = Ap[p * pa + ka + i_blk + ii];
        Bs[p][kk][ii] = Bp[p * pb + kb + j_blk + ii];
      }
    }
    __syncthreads();
    // lane holds A[row = lane & 15][k = 8 * (lane >> 4) + 0..7]
    bf16x8 a_[2][4], b_[2][4];
    for (int a = 0; a < 2; ++a)
      for (int p = 0; p < 4; ++p)
        for (int x = 0; x < 8; ++x) {
          a_[a][p][x] = (__bf16)As[p][8 * (lane >> 4) + x][wi + a * 16 + (lane & 15)];
          b_[a][p][x] = (__bf16)Bs[p][8 * (lane >> 4) + x][wj + a * 16 + (lane & 15)];
        }
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) {
        // negated imaginary parts of A for the Aim*Bim term
        bf16x8 nih = -a_[a][2], nil = -a_[a][3];
        floatx4 r = acc_re[a][b], im = acc_im[a][b];
        // re += Are*Bre
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_[a][0], b_[b][0], r, 0, 0, 0);
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_[a][0], b_[b][1], r, 0, 0, 0);
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_[a][1], b_[b][0], r, 0, 0, 0);
        // re -= Aim*Bim
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nih, b_[b][2], r, 0, 0, 0);
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nih, b_[b][3], r, 0, 0, 0);
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nil, b_[b][2], r, 0, 0, 0);
        // im += Are*Bim
        im = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_[a][0], b_[b][2], im, 0, 0, 0);
        im = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_[a][0], b_[b][3], im, 0, 0, 0);
        im = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_[a][1], b_[b][2], im, 0, 0, 0);
        // im += Aim*Bre
        im = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_[a][2], b_[b][0], im, 0, 0, 0);
        im = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_[a][2], b_[b][1], im, 0, 0, 0);
        im = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_[a][3], b_[b][0], im, 0, 0, 0);
        acc_re[a][b] = r;
        acc_im[a][b] = im;
      }
    __syncthreads();
  }
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int e = 0; e < 4; ++e) {
        const int i = i_blk + wi + a * 16 + 4 * (lane >> 4) + e;
        const int j = j_blk + wj + b * 16 + (lane & 15);
        if (i < M && j < N) {
          float2 r = make_float2(acc_re[a][b][e], acc_im[a][b][e]);
          float2* p = C + (size_t)i * ldc + j;
          if (accumulate) {
            float2 o = *p;
            r.x += o.x;
            r.y += o.y;
          }
          *p = r;
        }
      }
}

static inline int round_up(int x, int m) { return (x + m - 1) / m * m; }

size_t split_bf16_workspace_bytes(int M, int N, int K) {
  const size_t Kp = (size_t)round_up(K, 32);
  return 4 * Kp * (size_t)(round_up(M, kBBM) + round_up(N, kBBN)) * sizeof(__hip_bfloat16);
}

hipError_t launch_zgemm_tn_split_bf16(int M, int N, int K, const float2* A, int lda,
                                      const float2* B, int ldb, float2* C, int ldc,
                                      int accumulate, void* work, hipStream_t st) {
  if (M <= 0 || N <= 0 || K <= 0) return hipErrorInvalidValue;
  const int Kp = round_up(K, 32);
  const int Mp = round_up(M, kBBM), Np = round_up(N, kBBN);
  __hip_bfloat16* Ap = (__hip_bfloat16*)work;
  __hip_bfloat16* Bp = Ap + 4 * (size_t)Kp * Mp;
  {
    const size_t tot = (size_t)Kp * Mp;
    hipLaunchKernelGGL(k_split_bf16, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, A, lda,
                       K, M, Mp, Ap);
  }
  {
    const size_t tot = (size_t)Kp * Np;
    hipLaunchKernelGGL(k_split_bf16, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, B, ldb,
                       K, N, Np, Bp);
  }
  dim3 g(Np / kBBN, Mp / kBBM);
  hipLaunchKernelGGL(k_zgemm_tn_bf16x3, g, dim3(kGemmThreads), 0, st, M, N, Kp, Ap, Mp, Bp, Np, C,
                     ldc, accumulate);
  return hipGetLastError();
}

// ------------------------------------------------------------------ small kernels

__global__ void k_gather_amps(const float2* __restrict__ C, int ldc, const int* __restrict__ iu,
                              const int* __restrict__ il, size_t m, float2* __restrict__ amps) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < m) amps[t] = C[(size_t)iu[t] * ldc + il[t]];
}

hipError_t launch_gather_amps(const float2* C, int ldc, const int* iu, const int* il, size_t m,
                              float2* amps, hipStream_t st) {
  if (m == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_amps, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, C, ldc,
                     iu, il, m, amps);
  return hipGetLastError();
}

constexpr int kProbThreads = 256;
constexpr int kProbPerBlock = 4096;

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

__global__ void k_prob_final(const double* __restrict__ partial, int nb, double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double a1 = 0, a2 = 0;
  for (int b = 0; b < nb; ++b) {
    a1 += partial[2 * b];
    a2 += partial[2 * b + 1];
  }
  out[0] = a1;
  out[1] = a2;
}

hipError_t launch_prob_sums(const float2* amps, size_t m, double* partial, double* out,
                            hipStream_t st) {
  const int nb = prob_partial_blocks(m);
  if (nb == 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_prob_partial, dim3(nb), dim3(kProbThreads), 0, st, amps, m, partial);
  hipLaunchKernelGGL(k_prob_final, dim3(1), dim3(64), 0, st, partial, nb, out);
  return hipGetLastError();
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
