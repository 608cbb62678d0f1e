// Process-wide runtime state: error details, kernel tracing.
#include <map>
#include <mutex>
#include <string>
#include <vector>
#include <cstring>

#include "common.hpp"

namespace cqc {

static thread_local std::string g_err;
void set_error(const std::string &msg) { g_err = msg; }
const char *error_detail() { return g_err.c_str(); }

namespace {
struct Pending {
  std::string name;
  hipEvent_t start, stop;
};
struct TraceState {
  std::mutex mu;
  bool on = false;
  std::vector<Pending> pending;
  std::map<std::string, std::pair<int, double>> totals;
};
TraceState &trace() {
  static TraceState t;
  return t;
}
}  // namespace

bool trace_on() { return trace().on; }

bool trace_events(hipEvent_t *start, hipEvent_t *stop) {
  *start = *stop = nullptr;
  if (hipEventCreate(start) != hipSuccess) {
    *start = nullptr;
    return false;
  }
  if (hipEventCreate(stop) != hipSuccess) {
    (void)hipEventDestroy(*start);
    *start = *stop = nullptr;
    return false;
  }
  return true;
}

void trace_push(const char *name, hipEvent_t start, hipEvent_t stop) {
  std::lock_guard<std::mutex> g(trace().mu);
  trace().pending.push_back({name, start, stop});
}

static void trace_drain() {
  auto &t = trace();
  for (auto &p : t.pending) {
    (void)hipEventSynchronize(p.stop);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, p.start, p.stop);
    auto &e = t.totals[p.name];
    e.first += 1;
    e.second += ms;
    (void)hipEventDestroy(p.start);
    (void)hipEventDestroy(p.stop);
  }
  t.pending.clear();
}

}  // namespace cqc

extern "C" {

int cqc_trace_enable(int on) {
  auto &t = cqc::trace();
  std::lock_guard<std::mutex> g(t.mu);
  t.on = on != 0;
  return CQC_OK;
}

int cqc_trace_read(char *names, size_t names_len, int32_t *counts, double *ms,
                   int32_t max_kernels, int32_t *n_kernels) {
  auto &t = cqc::trace();
  std::lock_guard<std::mutex> g(t.mu);
  cqc::trace_drain();
  int32_t k = 0;
  std::string joined;
  for (auto &kv : t.totals) {
    if (k < max_kernels) {
      if (counts) counts[k] = kv.second.first;
      if (ms) ms[k] = kv.second.second;
      if (!joined.empty()) joined += "\n";
      joined += kv.first;
    }
    ++k;
  }
  if (n_kernels) *n_kernels = k < max_kernels ? k : max_kernels;
  if (names && names_len) {
    std::strncpy(names, joined.c_str(), names_len - 1);
    names[names_len - 1] = 0;
  }
  t.totals.clear();
  return CQC_OK;
}

const char *cqc_status_string(int status) {
  switch (status) {
    case CQC_OK: return "CQC_OK";
    case CQC_ERR_INVALID_ARG: return "CQC_ERR_INVALID_ARG";
    case CQC_ERR_SHAPE: return "CQC_ERR_SHAPE";
    case CQC_ERR_UNSUPPORTED: return "CQC_ERR_UNSUPPORTED";
    case CQC_ERR_WORKSPACE: return "CQC_ERR_WORKSPACE";
    case CQC_ERR_HIP: return "CQC_ERR_HIP";
    default: return "CQC_ERR_UNKNOWN";
  }
}

const char *cqc_last_error_detail(void) { return cqc::error_detail(); }

int cqc_version(void) { return 100; }

}  // extern "C"
