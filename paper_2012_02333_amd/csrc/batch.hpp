// Prepared batch of full-definition instances (host handle behind cqc_batch).
#pragma once

#include <vector>

#include "fdplan.hpp"

struct cqc_batch_s {
  std::vector<cqc::FdInstancePlan> plans;
  cqc::Acc acc = cqc::Acc::F32;
  bool in_double = false;
  char *ws = nullptr;
  std::vector<std::vector<const void *>> entry_src;  // caller's entry pointers
  // tables (device addresses inside the workspace)
  const cqc::FlagDesc *flag_descs = nullptr;
  int32_t n_flag = 0;
  int64_t flag_blocks = 0;
  const cqc::MassDesc *mass_descs = nullptr;
  int32_t n_mass = 0;
  unsigned long long *counters = nullptr;
  struct Group {
    int level, mode, cfg;
    bool small;
    bool strip;     // two-tile strips of the FP32 small-term kernel
    int xent;       // final steps of the cross-entropy form: 1 gradient, 2 gradient and loss
    cqc::Acc acc;   // arithmetic of the group's steps
    const cqc::ContractArgs *descs;
    const int64_t *prefix;
    int32_t ndesc;
    int64_t total;
    const int64_t *bprefix;   // wide kernel: first batch entry of each step (label-list pass)
    int64_t btotal;
  };
  std::vector<Group> groups;
};
