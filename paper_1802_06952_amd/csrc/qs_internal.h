// Internal structures of the qs library: circuit, half programs, the copy tree
// of one half, and the device descriptors of the kernels.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/qs.h"

namespace qs {

// ---------------------------------------------------------------- circuit

enum GateKind : uint8_t { G_H = 0, G_SX = 1, G_SY = 2, G_T = 3, G_CZ = 4 };

struct Gate {
  int cycle;
  GateKind kind;
  int q0, q1;    // q1 = -1 for one-qubit gates
  int pw = 1;    // G_T: the gate is T^pw (phase omega^pw on |1>)
  bool aux = false;  // a basis change added by the controlled-U rewrite (not a written gate)
};

struct Circuit {
  int n = 0;
  std::vector<Gate> gates;
};

// Parse the text format; on error returns false and fills err.  A controlled-U
// with U = X or Y ("cx c t", "cy c t") is stored as a CZ between basis
// changes on its target: U = V Z V^dagger gives P0 x I + P1 x U (Supp. Eq. 1)
// = (I x V) CZ (I x V^dagger), with V = H for X and V = S H for Y (S = T^2).
// Cutting that CZ puts P_b on its upper endpoint and Z^b on its lower one, so
// a cut controlled-U whose control is in the upper half splits exactly as in
// Supp. Eq. 1 (the target gets V Z^b V^dagger = U^b); with the control in
// the lower half the copies are the mirrored split (V P_b V^dagger on the
// target, Z^b on the control), with the same sum.
bool parse_circuit(const char* text, size_t len, Circuit& out, std::string& err);

// ---------------------------------------------------------------- partition

struct Cut {
  int index;  // position in cut order
  int cycle;
  int upper;  // global qubit id of the upper endpoint (carries P_b)
  int lower;  // global qubit id of the lower endpoint (carries Z^b)
};

// One operation of a half program, on local qubit ids.
enum OpKind : uint8_t {
  OP_MAT = 0,  // non-diagonal 2x2 gate (H, sqrt X, sqrt Y) on q0
  OP_T = 1,    // T on q0
  OP_CZ = 2,   // CZ on (q0, q1), both inside the half
  OP_CUT = 3   // the half's factor of cut gate `cut`: P_b (upper) or Z^b (lower) on q0
};

struct HOp {
  OpKind kind;
  int q0, q1;
  int cut;
  int mat;    // OP_MAT: 0 = H, 1 = sqrt X, 2 = sqrt Y; OP_T: the power of T
  int cycle;
};

struct Side {
  bool upper = true;
  int n = 0;                   // qubits of the half
  std::vector<int> qubits;     // global id of local qubit i (ascending)
  std::vector<HOp> ops;        // program order (after the initial H layer)
  uint64_t hinit = 0;          // local qubits starting in |+> (leading H folded into the init)
};

// ---------------------------------------------------------------- device descriptors

constexpr int kMaxDiagDist = 8;
constexpr int kMaxBranch = 8;
constexpr int kMaxTailLevels = 12;
constexpr int kMaxTileBits = 14;

// One operation as the kernels see it.  DIAG multiplies amplitude x by
//   omega^(popc(x & t0) + 2 popc(x & t1) + 4 popc(x & t2)
//           + 4 * sum_i popc(x & (x >> d[i]) & M[i]))
// and zeroes it unless (x & pmask) == pval (omega = (1+i)/sqrt 2; Eq. 4 and 6
// fused with the cut projectors and Z of Eq. 1).  MAT applies a 2x2 matrix on
// index bit `target` of the kernel's working index space.
constexpr int kMaxRegBits = 5;

// The 2x2 gates of the circuits are a scalar times a matrix of entries 0, +-1,
// +-i: sqrt X = (1+i)/2 [[1,-i],[-i,1]], sqrt Y = (1+i)/2 [[1,-1],[1,1]],
// H = 1/sqrt 2 [[1,1],[1,-1]].  The kernels apply the unit-entry matrix (two
// additions per amplitude); the scalars of all gates of a half multiply to one
// constant, which the passes keep in range by exact powers of two and the
// assembly applies once (see Prepared::phi).
enum MatKind : int {
  MK_GENERIC = 0,  // m[] as given
  MK_X = 1,        // [[1, -i], [-i, 1]]
  MK_Y = 2,        // [[1, -1], [1, 1]]
  MK_YT = 3,       // [[1, 1], [-1, 1]]
  MK_H = 4         // [[1, 1], [1, -1]]
};

struct DevOp {
  int kind;    // 0 = MAT, 1 = DIAG
  int target;  // MAT: working bit
  int nd;      // DIAG: number of (d, M) pairs
  int mk;      // MAT: MatKind (m[] holds the same matrix)
  float m[8];  // MAT: m00 m01 m10 m11 as (re, im)
  uint64_t t0, t1, t2, pmask, pval;
  int d[kMaxDiagDist];
  uint64_t M[kMaxDiagDist];
  // DIAG in a wave-tile pass, split over the pass's register bits rho_k (the
  // other bits F of an index are fixed per lane): the exponent of index
  // F | sum_k r_k 2^rho_k is
  //   e(F) + sum_k r_k (wl[k] + 4 popc(F & cross[k]))
  //        + 4 sum_{k2 < k} r_k r_k2 [bit k2 of rr[k]]   (mod 8).
  int wl[kMaxRegBits];
  uint32_t cross[kMaxRegBits];
  uint32_t rr[kMaxRegBits];
};

// Branch stages of one pass at most: a pass may descend this many tree levels
// at once (a parent tile gives 2^(m_1 + ... + m_S) children without the
// intermediate levels reaching memory).
constexpr int kMaxStages = 2;
// Ops of one pass at most (its ops are staged in LDS).
constexpr int kMaxPassOps = 128;

// A full-state pass: every tile of 2^t amplitudes (the tile bits are state
// bits tbit[0..t-1]) is loaded once and gets `n_in` ops; with ns = 0 it is
// stored.  With ns > 0 stages it branches: stage s decides the m_s cut bits
// of the next tree level, and for each of their 2^m_s values the tile gets
// that child's cut factors and the stage's ops; the last stage's results are
// stored, at child (((node << m_1) | b_1) << m_2) | b_2 ...  wave = 1: one
// wavefront owns a tile; its 64 lanes hold state bits 0..5 (tbit[0..5]) and
// each lane holds 2^(t-6) amplitudes in registers over the state bits
// tbit[6..t-1].  wave = 0: one workgroup stages the tile in LDS (small states).
struct PassDesc {
  int wave;
  int n;             // state qubits
  int t;             // tile bits
  int tbit[kMaxTileBits];
  int n_outer;       // n - t
  int obit[64];      // state bit of outer bit j (ascending)
  int init;          // 1: no input, start from the product state given by hinit
  uint64_t hinit;
  float hamp;        // amplitude of the initial product state
  int op_in, n_in;   // range in the op table; the stages' ops follow it
  int n_all;         // ops of the pass: n_in plus the stages' ops
  int ns;            // branch stages (0 = no branch)
  int sm[kMaxStages];              // cut bits of each stage
  int sbq[kMaxStages][kMaxBranch]; // state bit of the cut qubit of each stage bit (MSB first)
  int sop[kMaxStages];             // first op of each stage, counted from op_in
  int snops[kMaxStages];           // ops of each stage
  int upper;         // 1: P_b factors, 0: Z^b factors
  int nt;            // 1: stores bypass the caches (streaming outputs)
  float scale;       // exact power of two applied at the store (keeps unit-entry gates in range)
};

// Exchange groups of passes (PassPlan::xg): wave bits per workgroup, the
// most passes per group, and the fewest register bits of a grouped pass.
constexpr int kXWaveBits = 3;
constexpr int kMaxXPhases = 8;
constexpr int kXMinRegBits = 3;

// One launch of an exchange group: G consecutive passes (PassDescs pd0 ..
// pd0 + G - 1, no branch stages, R register bits each) on workgroup tiles of
// 6 lane bits and the nu = R + kXWaveBits state bits ubit[] (ascending); the
// other state bits obit[] are fixed per workgroup.  In phase p, register bit k
// of the pass is bit rpos[p][k] of U and wave bit j is bit wpos[p][j] of U.
struct XPassDesc {
  int G;
  int pd0;
  int R;
  int n;
  int nu;
  int ubit[kMaxRegBits + kXWaveBits];
  int n_outer;
  int obit[64];
  int rpos[kMaxXPhases][kMaxRegBits];
  int wpos[kMaxXPhases][kXWaveBits];
  int init;  // phase 0 starts from the product state (PassDesc::init of the first pass)
  int nt;    // streaming stores (the last pass's setting)
};

struct TailLevel {
  int m;                 // cut bits decided at this level
  int bq[kMaxBranch];    // state bit of each cut qubit (bit 0 = MSB of b)
  int bop0, bnops;       // the level's ops reversed, MATs transposed (targets are Q indices)
  int shift;             // position of the level's branch bits in the leaf index
  int pos;               // position of the level's branch bits in the emission index
  uint64_t kbit[kMaxBranch];  // copy-index contribution of each branch bit
  // the level's ops, one byte each (levels of at most 8 ops, else 0):
  // DIAG << 7 | MatKind << 3 | target
  uint64_t code;
};

// Leaf evaluation restricted to the light cone.  Below the materialised
// level every operation is the same linear map for all materialised nodes,
// and its non-diagonal gates touch only the qubits Q: the subspace of indices
// that agree with a requested value s outside Q is invariant.  So the leaf
// amplitude of node r, leaf path lam, at s is  sum_y w_{s,lam}[y] v_{r,s}[y],
// where v_{r,s}[y] is node r's amplitude at s with the Q bits replaced by y and
// w_{s,lam} is row s of the leaf path's operator, obtained by running the
// transposed leaf levels backwards from the unit vector at s (k_tail_bwd).
// The contraction over y is a small complex GEMM per s (k_tail_mm).  Cuts
// with no later non-commuting gate multiply the result by their factor at s.
// Output position of emission bit b of a leaf path under the specialised-wave
// leaf evaluation (M >= 5 path bits; see TailDesc::ws).
inline int tail_ws_bit(int b, int M) {
  if (b < 2) return b;
  if (b < M - 3) return b + 3;
  return b - (M - 5);
}

struct TailDesc {
  int n;
  int q;
  int Q[16];            // state bit of working bit i
  int nlev;
  int M;                // total branch bits of the leaf levels (leaf paths = 2^M)
  int split_levels;     // the backward rows of one value are spread over 2^split_bits
  int split_bits;       //   wavefronts by the branches of the first split_levels reverse levels
  TailLevel lev[kMaxTailLevels];
  int n_end;            // cuts with no later non-commuting gate: applied to the output
  int eq[kMaxBranch * 2];   // state bit of each end cut's qubit (MSB first)
  uint64_t ekbit[kMaxBranch * 2];  // copy-index contribution of each end bit
  int upper;
  int n_nodes;          // materialised nodes
  int S;                // requested values
  int ldx;              // leading dimension (row stride) of the output X[k][s]
  // 1: rows and contraction fused in one kernel; the leaf paths of the output
  // then come in emission order j (the digit of level l at bit sum_{l'<l} m_l')
  // instead of lam (the digit of level l at bit lev[l].shift)
  int fused;
  // 1 (with fused): the leaf evaluation with specialised waves, whose output
  // index swaps two fields of the emission index j so that each chunk of 32
  // paths lands on 32 consecutive copies: with j = st | c << 2 | p << (M - 3)
  // (st: the first two levels' digits, c: the chunk, p: the producer wave) the
  // paths are written at st | p << 2 | c << 5 (tail_ws_index)
  int ws;
  // 1: write only the copies whose end bits are all 0, without end factors,
  // at nu0 = node * 2^M + lam (ldx = copies of the block >> n_end).  Used for
  // lower halves: the other copies differ from these by the signs of the end
  // cuts' Z, which the assembly applies to the upper operand instead.
  int end_base;
  float tscale;         // value of the unit vector the backward rows start from (a power of two)
};

}  // namespace qs
