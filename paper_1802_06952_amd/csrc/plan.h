// Host planner: cut classification, half programs, the copy tree of a half
// (branch points pushed past every gate that commutes with the cut factor),
// grouping of each tree level into full-state passes, and the light-cone leaf
// evaluation of the deepest levels.
#pragma once

#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "qs_internal.h"

namespace qs {

// Cuts of E_int in cut order and the two half programs.
bool build_partition(const Circuit& c, uint64_t upper_mask, std::vector<Cut>& cuts, Side& up,
                     Side& lo, std::string& err);

// The program of the qubits in `mask` (ascending ids are the local qubits):
// gates inside the set as ops, gates with one endpoint inside as OP_CUT ops
// whose cut index is cut_of[(cycle, endpoint)]; `upper` gives the cut
// factors' kind (P_b when true, Z^b when false).  Leading H gates fold into
// the initial product state.
void build_side(const Circuit& c, uint64_t mask, bool upper,
                const std::map<std::pair<int, int>, int>& cut_of, Side& s);

// A block of copies: cut j < p is fixed to bit (k0 >> (c-1-j)) & 1, the rest are free.
struct Block {
  uint64_t k0 = 0;
  int p = 0;
};

struct Level {
  std::vector<int> cuts;  // cuts decided on entering the level (branch order, MSB first)
  std::vector<int> ops;   // indices into Side::ops executed at this level, program order
};

struct Tree {
  std::vector<Level> levels;   // levels[0].cuts is empty
  std::vector<int> end_cuts;   // free cuts with no later non-commuting gate on their qubit
  std::vector<int> fixed;      // per cut: -1 free, else the fixed bit
  std::vector<int> order;      // free cuts in leaf-id order: level cuts, then end cuts
};

Tree build_tree(const Side& s, int c, const Block& blk);

// A pass reads the states of tree level level_in, runs ops_in on them, and
// with stages descends one level per stage: stage s branches on the cuts of
// level level_in + s + 1 and runs stages[s] (ops of that level) on every
// child.  It writes level level_in + stages.size().
struct PassPlan {
  int level_in = 0;
  bool init = false;
  std::vector<int> ops_in;
  std::vector<std::vector<int>> stages;
  std::vector<int> tile;  // local qubits of the tile, ascending
  // Exchange groups: consecutive passes without a branch that run as the
  // phases of one launch on workgroup tiles (group_passes).  xg: passes of the
  // group that starts here (1: a pass of its own, 0: covered by an earlier
  // pass); xu (first pass of a group): the tile's non-lane state bits, ascending.
  int xg = 1;
  std::vector<int> xu;
  bool branch() const { return !stages.empty(); }
  int level_out() const { return level_in + (int)stages.size(); }
};

struct SidePlan {
  Tree tree;
  int lstar = 0;                  // last materialised level
  std::vector<int> Q;             // light-cone qubits of the leaf evaluation (local ids, ascending)
  std::vector<int> perm;          // state bit of each local qubit: the light cone takes bits 0..q-1
  Side side;                      // the half program relabelled by perm (what the kernels run)
  std::vector<PassPlan> passes;   // passes of the relabelled program (tiles are state bits)
  double cost_bytes = 0;          // cost model estimate
  size_t peak_states = 0;         // largest number of live states
  std::vector<uint64_t> nodes;    // nodes per level
};

struct PlanKnobs {
  int tile_bits = 10;      // largest tile of a full-state pass
  int min_tile_bits = 8;   // a pass's tile shrinks to its targets, but not below this
  int coalesce_bits = 5;
  int tail_max_qubits = 10;
  int force_lstar = -1;
  size_t mem_budget = 0;  // bytes; 0 = unlimited
  int S = 1;              // requested values of this half (for the cost model)
  bool one_op_per_pass = false;  // flat comparison form: every half op is its own pass
  int max_stages = kMaxStages;   // tree levels one pass may descend (1 = one level per pass)
  bool exchange = true;          // merge runs of passes into exchange groups
};

bool plan_side(const Side& s, int c, const Block& blk, const PlanKnobs& kn, SidePlan& out,
               std::string& err);

// Encode a sequence of half ops as kernel ops; `work_of` maps a local qubit to
// the working bit of a MAT op (-1 if the qubit is not a working bit, which is
// an error for MAT ops).  Diagonal ops are merged into one DIAG op until a MAT
// acts on a qubit they touch; MATs on other qubits move ahead of them.
// transpose = true encodes the transposed operator of the list: the caller
// passes the ops in reverse order and every 2x2 matrix is transposed.
// reg_bits (optional): the state bits of a wave-tile pass's register bits, for
// the register split of DIAG ops.
bool encode_ops(const Side& s, const std::vector<int>& ops, const std::vector<int>& fixed_bits,
                const std::vector<int>& work_of, std::vector<DevOp>& out, std::string& err,
                bool transpose = false, const std::vector<int>* reg_bits = nullptr);

std::string dump_json(const Circuit& c, uint64_t upper_mask, const std::vector<Cut>& cuts,
                      const Side& up, const Side& lo, const SidePlan* pu, const SidePlan* pl);

}  // namespace qs
