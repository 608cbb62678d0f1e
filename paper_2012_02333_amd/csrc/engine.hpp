// Workspace layout and enqueue of a contraction plan (shared by FD and DD).
#pragma once

#include <vector>

#include "kernels.hpp"
#include "plan.hpp"

namespace cqc {

struct NetLayout {
  Plan plan;
  Acc acc = Acc::F32;
  size_t esz = 4;
  std::vector<size_t> t_off;   // intermediates (and unit tensor): byte offset
  std::vector<size_t> f_off;   // row flags of every tensor: byte offset
  std::vector<int> tile;       // per step
  std::vector<int64_t> nblocks;
  size_t partials_off = 0;
  std::vector<size_t> list_off;  // per step: label lists of the wide kernel (SIZE_MAX: none)
  std::vector<size_t> xs_off, ys_off;  // per step: bfloat16 parts of X and Y for a split-form
                                       //   wide step (SIZE_MAX: none)
  size_t bytes = 0;            // end offset (relative to the layout base)
};

// Lay out a plan's workspace starting at byte offset `base`.
NetLayout layout_net(const Plan &plan, Acc acc, size_t base);

// Enqueue the plan.  `entries[c]` are Acc-typed device tensors, flags of the
// entry tensors must already be computed into their f_off slots unless
// compute_entry_flags is set.
// skip_final: run every step but the last (the intermediates the adjoint needs).
// gate / gate_val: an optional device-side predicate stamped on every launch
// (see ContractArgs).
Status run_net(const NetLayout &L, char *ws, const std::vector<const void *> &entries,
               void *out, bool out_double, double *mass, bool compute_entry_flags,
               hipStream_t s, bool skip_final = false, const int32_t *gate = nullptr, int32_t gate_val = 0);

DigitMapDev to_dev(const DigitMap &m);
// Whether any step (all but the last if skip_final) compacts its terms by the
// entry row flags (general and wide kernels; every BF16X6 step).  Without them
// the small kernel keeps every term and the flag pass is skipped.
bool needs_flags(const NetLayout &L, bool skip_final);
// Points a step's arguments at its label-list workspace (wide kernel).
void set_lists(const NetLayout &L, size_t step, char *ws, ContractArgs *a);
// Tile shape and XCD mapping recorded by the autotuner for a step's shape class.
bool tuned_choice(Acc acc, int mode, bool small, int logM, int logN, int nS, bool out_double, int *cfg, int *xcd);
BitPos pack_pos(const std::vector<int> &pos);

inline bool is_blocked(const Plan &p, const Step &st) {
  const auto &X = p.tensors[st.x], &Y = p.tensors[st.y];
  const int nY = (int)Y.bits.size();
  for (int j = 0; j < nY; ++j)
    if (p.bitpos[Y.bits[nY - 1 - j]] != j) return false;
  const int nX = (int)X.bits.size();
  for (int j = 0; j < nX; ++j)
    if (p.bitpos[X.bits[nX - 1 - j]] != nY + j) return false;
  return true;
}

}  // namespace cqc
