// Host-side validation of a cut description and the contraction plan that
// evaluates the FD term sum as a sequence of pairwise tensor contractions.
//
// The term sum p(x) = 2^-K sum_l prod_c E_c[row_c(l), x_c] is a tensor network:
// every cut label l_e is shared by exactly two subcircuit tensors and every
// output bit belongs to one.  Contracting two tensors X, Y over their shared
// labels S gives Z[(rX, rY), (bX, bY)] = sum_s X[row(s, rX), bX] Y[row(s, rY), bY]
// (a batched GEMM with inner dimension 4^|S|); the last contraction writes the
// 2^n output in global order with the exact 2^-K scale.  The order of
// contractions generalises the greedy smallest-first subcircuit order of
// Section 4.2: at every step the pair whose result is smallest is contracted.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "common.hpp"

namespace cqc {

struct CutInfo {
  int n = 0, nsub = 0, K = 0;
  std::vector<int> f, up, down;
  std::vector<std::vector<int>> inc;     // incident cuts per subcircuit, ascending
  std::vector<std::vector<int>> qubits;  // global qubit of each local bit, MSB first
};

// max_n: CQC_MAX_FD_QUBITS or CQC_MAX_DD_QUBITS
Status validate_cut(const cqc_cut *c, int max_n, CutInfo *out);

struct TensorSpec {
  std::vector<int> labels;  // cut ids of row digits, most significant first
  std::vector<int> bits;    // output-bit ids of columns, most significant first
  int entry = -1;           // >= 0: caller entry tensor; -1: intermediate
  int64_t rows() const { return int64_t(1) << (2 * labels.size()); }
  int64_t cols() const { return int64_t(1) << bits.size(); }
};

// Device row-index map of one operand: row = sum_i digit_i * 4^(n-1-i), where
// digit_i = (src_i ? r : s) >> shift_i & 3.
struct DigitMap {
  int8_t n = 0;
  int8_t src[CQC_MAX_K_SUB + 4] = {};
  int8_t shift[CQC_MAX_K_SUB + 4] = {};
};

struct Step {
  int x = -1, y = -1, z = -1;  // tensor ids; z = result tensor (last step: output)
  std::vector<int> S, RX, RY;  // shared (ascending cut id), rest labels (operand order)
  DigitMap mx, my;
  int logM = 0, logN = 0;      // column bits of X and Y
  int64_t nbatch = 1;          // 4^(|RX|+|RY|)
  // both operands hold at most 2^30 elements (the wide kernel's addressing)
  // and have at least two columns (its paired column loads)
  bool wide_ok() const {
    return 2 * (S.size() + RX.size()) + logM <= 30 && 2 * (S.size() + RY.size()) + logN <= 30 && logM >= 1 &&
           logN >= 1;
  }
};

// A plan over "output bits": for FD the bits are global qubits with output
// position n-1-q; for DD they are the active qubits with their bin position.
struct Plan {
  int nbits = 0;                // output index width
  int K = 0;
  std::vector<TensorSpec> tensors;  // [0, nsub) are the (possibly merged) entries
  std::vector<Step> steps;          // contraction order; last writes the output
  std::vector<int> bitpos;          // bit id -> position in the output index
  bool single = false;              // one tensor, no contraction (K = 0, n_C = 1)
};

// Build a plan from per-subcircuit (labels, column bits) and the position of
// every output bit.  Greedy: smallest intermediate first.
Plan make_plan(const CutInfo &cut, const std::vector<std::vector<int>> &cols,
               const std::vector<int> &bitpos, int nbits);

DigitMap digit_map(const std::vector<int> &labels, const std::vector<int> &S,
                   const std::vector<int> &R);

// Eq. 14 with the greedy subcircuit order, and the multiply-adds of a plan.
double eq14_cost(const CutInfo &cut);
double plan_macs(const Plan &p);

}  // namespace cqc
