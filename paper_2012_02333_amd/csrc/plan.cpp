// Cut validation and the greedy contraction planner.
#include "plan.hpp"

#include <algorithm>
#include <cmath>
#include <limits>
#include <sstream>

namespace cqc {

Status validate_cut(const cqc_cut *c, int max_n, CutInfo *out) {
  if (!c) return Status::fail(CQC_ERR_INVALID_ARG, "cut is NULL");
  const int n = c->n_qubits, nsub = c->n_sub, K = c->n_cuts;
  if (nsub < 1 || nsub > CQC_MAX_SUB)
    return Status::fail(CQC_ERR_UNSUPPORTED, "n_sub must be in [1, " + std::to_string(CQC_MAX_SUB) + "]");
  if (K < 0 || K > CQC_MAX_CUTS)
    return Status::fail(CQC_ERR_UNSUPPORTED, "n_cuts must be in [0, " + std::to_string(CQC_MAX_CUTS) + "]");
  if (n < 0) return Status::fail(CQC_ERR_SHAPE, "n_qubits < 0");
  if (n > max_n)
    return Status::fail(CQC_ERR_UNSUPPORTED, "n_qubits " + std::to_string(n) + " exceeds " + std::to_string(max_n));
  if (!c->f || (n > 0 && !c->out_qubit) || (K > 0 && (!c->edge_up || !c->edge_down)))
    return Status::fail(CQC_ERR_INVALID_ARG, "NULL array in cut");
  CutInfo ci;
  ci.n = n;
  ci.nsub = nsub;
  ci.K = K;
  int64_t sum = 0;
  for (int s = 0; s < nsub; ++s) {
    if (c->f[s] < 0) return Status::fail(CQC_ERR_SHAPE, "f[" + std::to_string(s) + "] < 0");
    if (c->f[s] > CQC_MAX_F_SUB)
      return Status::fail(CQC_ERR_UNSUPPORTED, "f[" + std::to_string(s) + "] exceeds " + std::to_string(CQC_MAX_F_SUB));
    ci.f.push_back(c->f[s]);
    sum += c->f[s];
  }
  if (sum != n)
    return Status::fail(CQC_ERR_SHAPE, "sum of f (" + std::to_string(sum) + ") != n_qubits (" + std::to_string(n) + ")");
  ci.inc.assign(nsub, {});
  for (int e = 0; e < K; ++e) {
    int u = c->edge_up[e], d = c->edge_down[e];
    if (u < 0 || u >= nsub || d < 0 || d >= nsub)
      return Status::fail(CQC_ERR_INVALID_ARG, "cut " + std::to_string(e) + " names a subcircuit out of range");
    if (u == d)
      return Status::fail(CQC_ERR_SHAPE, "cut " + std::to_string(e) + " has the same upstream and downstream subcircuit");
    ci.up.push_back(u);
    ci.down.push_back(d);
    ci.inc[u].push_back(e);
    ci.inc[d].push_back(e);
  }
  for (int s = 0; s < nsub; ++s) {
    std::sort(ci.inc[s].begin(), ci.inc[s].end());
    if ((int)ci.inc[s].size() > CQC_MAX_K_SUB)
      return Status::fail(CQC_ERR_UNSUPPORTED, "subcircuit " + std::to_string(s) + " has more than " +
                                                   std::to_string(CQC_MAX_K_SUB) + " incident cuts");
  }
  std::vector<int> seen(n, 0);
  ci.qubits.assign(nsub, {});
  int off = 0;
  for (int s = 0; s < nsub; ++s) {
    for (int j = 0; j < ci.f[s]; ++j) {
      int q = c->out_qubit[off + j];
      if (q < 0 || q >= n) return Status::fail(CQC_ERR_SHAPE, "out_qubit entry out of range");
      if (seen[q]++) return Status::fail(CQC_ERR_SHAPE, "out_qubit is not a permutation (qubit " + std::to_string(q) + " repeats)");
      ci.qubits[s].push_back(q);
    }
    off += ci.f[s];
  }
  *out = std::move(ci);
  return Status::ok();
}

DigitMap digit_map(const std::vector<int> &labels, const std::vector<int> &S,
                   const std::vector<int> &R) {
  DigitMap m;
  m.n = (int8_t)labels.size();
  for (size_t i = 0; i < labels.size(); ++i) {
    auto is = std::find(S.begin(), S.end(), labels[i]);
    if (is != S.end()) {
      int pos = int(is - S.begin());
      m.src[i] = 0;
      m.shift[i] = (int8_t)(2 * ((int)S.size() - 1 - pos));
    } else {
      auto ir = std::find(R.begin(), R.end(), labels[i]);
      int pos = int(ir - R.begin());
      m.src[i] = 1;
      m.shift[i] = (int8_t)(2 * ((int)R.size() - 1 - pos));
    }
  }
  return m;
}

Plan make_plan(const CutInfo &cut, const std::vector<std::vector<int>> &cols,
               const std::vector<int> &bitpos, int nbits) {
  Plan p;
  p.nbits = nbits;
  p.K = cut.K;
  p.bitpos = bitpos;
  for (int s = 0; s < cut.nsub; ++s) {
    TensorSpec t;
    t.labels = cut.inc[s];
    t.bits = cols[s];
    t.entry = s;
    p.tensors.push_back(t);
  }
  if (cut.nsub == 1) {
    // One subcircuit and no cut: the output is row 0 of E_0.  Contract it with
    // a unit tensor (one row, one column, value 1) so the same kernel writes it.
    p.single = true;
    TensorSpec unit;
    unit.entry = -2;
    p.tensors.push_back(unit);
    Step st;
    st.x = 0;
    st.y = 1;
    st.mx = digit_map(p.tensors[0].labels, st.S, st.RX);
    st.my = digit_map(unit.labels, st.S, st.RY);
    st.logM = (int)p.tensors[0].bits.size();
    st.logN = 0;
    TensorSpec Z;
    Z.bits = p.tensors[0].bits;
    p.tensors.push_back(Z);
    st.z = 2;
    p.steps.push_back(st);
    return p;
  }
  auto minpos_desc = [&](const TensorSpec &t) {
    // most significant output position held by the tensor (for orientation)
    int best = -1;
    for (int b : t.bits) best = std::max(best, bitpos[b]);
    return best;
  };
  std::vector<int> live;
  for (int s = 0; s < cut.nsub; ++s) live.push_back(s);
  while (live.size() >= 2) {
    int bi = -1, bj = -1;
    double best_size = std::numeric_limits<double>::infinity(), best_flops = best_size;
    bool any_shared = false;
    for (size_t a = 0; a < live.size(); ++a)
      for (size_t b = a + 1; b < live.size(); ++b) {
        const auto &A = p.tensors[live[a]], &B = p.tensors[live[b]];
        for (int l : A.labels)
          if (std::find(B.labels.begin(), B.labels.end(), l) != B.labels.end()) any_shared = true;
      }
    for (size_t a = 0; a < live.size(); ++a)
      for (size_t b = a + 1; b < live.size(); ++b) {
        const auto &A = p.tensors[live[a]], &B = p.tensors[live[b]];
        int shared = 0;
        for (int l : A.labels)
          if (std::find(B.labels.begin(), B.labels.end(), l) != B.labels.end()) ++shared;
        if (any_shared && shared == 0) continue;
        double lsz = 2.0 * (A.labels.size() + B.labels.size() - 2 * shared) +
                     (double)(A.bits.size() + B.bits.size());
        double lfl = lsz + 2.0 * shared;
        if (lsz < best_size || (lsz == best_size && lfl < best_flops)) {
          best_size = lsz;
          best_flops = lfl;
          bi = (int)a;
          bj = (int)b;
        }
      }
    int ta = live[bi], tb = live[bj];
    const bool last = live.size() == 2;
    // Orientation.  Intermediate: X holds the more significant output bits, so
    // Z's columns (X bits then Y bits) stay in descending significance.  Last
    // step: Y holds the least significant output bit so output stores coalesce.
    int x = ta, y = tb;
    if (minpos_desc(p.tensors[tb]) > minpos_desc(p.tensors[ta])) std::swap(x, y);
    if (last) {
      auto lowest = [&](const TensorSpec &t) {
        int m = 1 << 30;
        for (int b : t.bits) m = std::min(m, bitpos[b]);
        return m;
      };
      x = ta;
      y = tb;
      if (lowest(p.tensors[ta]) < lowest(p.tensors[tb])) std::swap(x, y);
    }
    const TensorSpec X = p.tensors[x], Y = p.tensors[y];
    Step st;
    st.x = x;
    st.y = y;
    for (int l : X.labels)
      if (std::find(Y.labels.begin(), Y.labels.end(), l) != Y.labels.end()) st.S.push_back(l);
    std::sort(st.S.begin(), st.S.end());
    for (int l : X.labels)
      if (std::find(st.S.begin(), st.S.end(), l) == st.S.end()) st.RX.push_back(l);
    for (int l : Y.labels)
      if (std::find(st.S.begin(), st.S.end(), l) == st.S.end()) st.RY.push_back(l);
    st.mx = digit_map(X.labels, st.S, st.RX);
    st.my = digit_map(Y.labels, st.S, st.RY);
    st.logM = (int)X.bits.size();
    st.logN = (int)Y.bits.size();
    st.nbatch = int64_t(1) << (2 * (st.RX.size() + st.RY.size()));
    TensorSpec Z;
    Z.labels = st.RX;
    Z.labels.insert(Z.labels.end(), st.RY.begin(), st.RY.end());
    Z.bits = X.bits;
    Z.bits.insert(Z.bits.end(), Y.bits.begin(), Y.bits.end());
    p.tensors.push_back(Z);
    st.z = (int)p.tensors.size() - 1;
    p.steps.push_back(st);
    live.erase(live.begin() + std::max(bi, bj));
    live.erase(live.begin() + std::min(bi, bj));
    live.push_back(st.z);
  }
  return p;
}

double eq14_cost(const CutInfo &cut) {
  std::vector<int> f = cut.f;
  std::sort(f.begin(), f.end());
  double total = 0.0, prod = 1.0;
  for (size_t c = 0; c < f.size(); ++c) {
    prod *= std::ldexp(1.0, f[c]);
    if (c >= 1) total += prod;
  }
  return std::ldexp(1.0, 2 * cut.K) * total;
}

double plan_macs(const Plan &p) {
  double macs = 0.0;
  for (const auto &st : p.steps) {
    const auto &Z = p.tensors[st.z];
    macs += std::ldexp(1.0, (int)(2 * Z.labels.size() + Z.bits.size() + 2 * st.S.size()));
  }
  return macs;
}

}  // namespace cqc
