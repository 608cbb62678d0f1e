// C ABI: on-device entry construction (cqc_build_entries).
#include <cstdint>
#include <cstring>
#include <vector>

#include "entries.hpp"

using namespace cqc;

extern "C" {

int cqc_build_entries(const cqc_entry_job *jobs, int32_t n_jobs, cqc_dtype in_t, cqc_dtype out_t,
                      hipStream_t stream) {
  if (!jobs) return Status::fail(CQC_ERR_INVALID_ARG, "jobs is NULL").code;
  if (n_jobs < 1) return Status::fail(CQC_ERR_INVALID_ARG, "n_jobs < 1").code;
  if ((in_t != CQC_F32 && in_t != CQC_F64) || (out_t != CQC_F32 && out_t != CQC_F64))
    return Status::fail(CQC_ERR_INVALID_ARG, "unknown dtype").code;
  std::vector<EntryArgs> args(n_jobs);
  for (int32_t j = 0; j < n_jobs; ++j) {
    const cqc_entry_job &J = jobs[j];
    const std::string who = "job " + std::to_string(j) + ": ";
    if (J.f < 0 || J.f > 30) return Status::fail(CQC_ERR_SHAPE, who + "f must be in [0, 30]").code;
    if (J.n_cuts < 0 || (J.n_cuts > 0 && !J.cut_kind))
      return Status::fail(CQC_ERR_INVALID_ARG, who + "bad n_cuts or cut_kind").code;
    if (!J.variants || !J.entries) return Status::fail(CQC_ERR_INVALID_ARG, who + "NULL tensor").code;
    EntryArgs &a = args[j];
    std::memset(&a, 0, sizeof(a));
    int kin = 0, kout = 0;
    for (int t = 0; t < J.n_cuts; ++t) {
      const int kd = J.cut_kind[t];
      if (kd == 0) {
        if (kin == kEntryMaxIn) return Status::fail(CQC_ERR_UNSUPPORTED, who + "more than 3 incoming cuts").code;
        a.in_pos[kin++] = t;
      } else if (kd == 1) {
        if (kout == kEntryMaxOut) return Status::fail(CQC_ERR_UNSUPPORTED, who + "more than 4 outgoing cuts").code;
        a.out_pos[kout++] = t;
      } else {
        return Status::fail(CQC_ERR_INVALID_ARG, who + "cut_kind values must be 0 or 1").code;
      }
    }
    a.V = J.variants;
    a.E = J.entries;
    a.f = J.f;
    a.k_in = kin;
    a.k_out = kout;
    a.k = J.n_cuts;
    a.p3 = 1;
    for (int t = 0; t < kout; ++t) a.p3 *= 3;
    a.vec = in_t == CQC_F32 && (reinterpret_cast<uintptr_t>(J.variants) % 16) == 0 ? 1 : 0;
    if (J.form != CQC_FORM_PAULI && J.form != CQC_FORM_EIGEN)
      return Status::fail(CQC_ERR_INVALID_ARG, who + "form must be CQC_FORM_PAULI or CQC_FORM_EIGEN").code;
    a.eigen = J.form == CQC_FORM_EIGEN ? 1 : 0;
  }
  for (int32_t j = 0; j < n_jobs; ++j) {
    Status st = launch_build_entries(args[j], in_t == CQC_F64, out_t == CQC_F64, stream);
    if (!st.good()) return st.code;
  }
  return CQC_OK;
}

}  // extern "C"
