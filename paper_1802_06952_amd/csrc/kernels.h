// Launch wrappers of the HIP kernels (implemented in kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "qs_internal.h"

namespace qs {

// Full-state pass over all tiles of `n_in_nodes` input states (or 1 when the
// pass starts from the initial product state).  d_desc / d_ops live in device
// memory; h_desc is the same descriptor on the host (for the launch shape).
// tlist (optional, wave-tile passes only): the n_list outer-bit values of
// the tiles to compute in every node; the other tiles of the output are left
// as they are.
hipError_t launch_pass(const PassDesc& h_desc, const PassDesc* d_desc, const DevOp* d_ops,
                       const float2* in, float2* out, uint64_t n_in_nodes, const uint32_t* tlist,
                       uint32_t n_list, hipStream_t st);

// The passes of one exchange group (XPassDesc) in one launch, in place on
// `state` (nodes states of 2^n amplitudes); d_pds points at the plan's
// PassDesc array (the group's passes from h.pd0).
hipError_t launch_xpass(const XPassDesc& h, const XPassDesc* d_desc, const PassDesc* d_pds,
                        const DevOp* d_ops, float2* state, uint64_t nodes, hipStream_t st);

// Light-cone leaf evaluation for the requested values s0 .. s0+ns-1: the
// backward rows into W (tail_w_bytes(h, ns) bytes), then the contraction with
// the materialised node states into X[k * ldx + s_index].
size_t tail_w_bytes(const TailDesc& h, int ns);
// Whether the leaf evaluation of h can run as one fused kernel (rows and
// contraction of a value in one workgroup; then W is not used and the output
// leaf paths come in emission order, see TailDesc::fused).
bool tail_fused_ok(const TailDesc& h);
// Whether the fused leaf evaluation of h can take the specialised-wave kernel
// (see TailDesc::ws).
bool tail_ws_ok(const TailDesc& h);
hipError_t launch_tail(const TailDesc& h_desc, const TailDesc* d_desc, const DevOp* d_ops,
                       const float2* states, const uint32_t* svals, int s0, int ns, float2* W,
                       float2* X, hipStream_t st);

// out[row * K + j] = in[row * K + perm[j]].
hipError_t launch_permute_cols(const float2* in, float2* out, const uint32_t* perm, int rows,
                               int K, hipStream_t st);

// C[i*ldc + j] (+)= sum_k A[i*lda + k] * B[j*ldb + k], complex64.  prec 0:
// FP32 MFMA; prec 1: split-BF16 (three bf16 products, FP32 accumulation).
// `work` must hold zgemm_workspace_bytes(prec, M, N, K) bytes (split-K
// partials and, for prec 1, the split operands).
// cmap (optional): column j of the product goes to column cmap[j] of C.
size_t zgemm_workspace_bytes(int prec, int M, int N, int K);
hipError_t launch_zgemm_tn(int prec, int M, int N, int K, const float2* A, int lda,
                           const float2* B, int ldb, float2* C, int ldc, int accumulate,
                           void* work, hipStream_t st, const uint32_t* cmap = nullptr);

// Grouped FP32 product: for every group g < ngroups, columns
// d_goff[g] .. d_goff[g+1]-1 of C (through cmap) (+)= A_g B_g^T, where A_g =
// A + g a_gstride (M rows of K) and B_g = rows d_goff[g] .. of B (K each);
// maxn bounds the columns of a group.  One launch for all groups.
size_t zgemm_grouped_workspace_bytes(int M, int Ntot, int maxn, int K, int ngroups);
hipError_t launch_zgemm_grouped(int M, int Ntot, int maxn, int K, int ngroups, const int* d_goff,
                                const float2* A, size_t a_gstride, const float2* B, float2* C,
                                int ldc, int accumulate, void* work, hipStream_t st,
                                const uint32_t* cmap);

// The same grouped product in split-BF16 (three bf16 products per real
// product, FP32 accumulation): A holds ngroups * M rows of K (group g's M rows
// at row g * M), B Ntot rows of K; both are split once for all groups.
size_t zgemm_grouped_bf16_workspace_bytes(int M, int Ntot, int maxn, int K, int ngroups);
hipError_t launch_zgemm_grouped_bf16(int M, int Ntot, int maxn, int K, int ngroups,
                                     const int* d_goff, const float2* A, const float2* B,
                                     float2* C, int ldc, int accumulate, void* work,
                                     hipStream_t st, const uint32_t* cmap);

// out[r][j] = in[rowsel[r]][colsel[j]].
hipError_t launch_gather_rows_cols(const float2* in, float2* out, const uint32_t* rowsel,
                                   const uint32_t* colsel, int rows, int Kin, int Kout,
                                   hipStream_t st);

// Walsh-Hadamard transform of X (rows x K) over the ne <= 4 copy-order bit
// positions pos[i]: out[sig][u][nu'] for sig < 2^ne, nu' < K >> ne.
hipError_t launch_end_wht(const float2* X, int rows, int K, int ne, const int* pos, float2* out,
                          hipStream_t st);

// amps[t] (+)= phi * sum_k A[iu[t]*lda + k] * B[il[t]*ldb + k] (one wavefront per t).
hipError_t launch_gathered_dot(int K, const float2* A, int lda, const float2* B, int ldb,
                               const int* iu, const int* il, size_t m, float2* amps,
                               int accumulate, float2 phi, hipStream_t st);

// FP64 sums over m amplitudes: out[0] = sum |a|^2, out[1] = sum |a|^4.
// `partial` must hold 2 * prob_partial_blocks(m) doubles.
int prob_partial_blocks(size_t m);
// amps[t] = phi * C[iu[t] * ldc + il[t]], then launch_prob_sums' sums of
// them, with the gather and the partial sums in one kernel.
hipError_t launch_gather_prob_sums(const float2* C, int ldc, const int* iu, const int* il,
                                   size_t m, float2* amps, float2 phi, double* partial,
                                   double* out, hipStream_t st);
hipError_t launch_prob_sums(const float2* amps, size_t m, double* partial, double* out,
                            hipStream_t st);

hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t st);

// The static scratch region of the allocation-free assembly: its size, and
// its device address on the current device (looked up once per device).
size_t static_scratch_capacity();
hipError_t static_scratch(void** base);

}  // namespace qs
