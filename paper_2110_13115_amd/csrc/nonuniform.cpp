// Host side of the non-uniform-frequency PCA (Sec. III.A): the frequency set
// built from the zero crossings of a reference template, the cell weights
// of its inner product, and the table that maps the uniform grid onto it
// for linear interpolation.
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "../../include/rbmf.h"
#include "internal.h"
#include "nonuniform.h"

// The set is compared value for value with other implementations of the same
// definition: no contraction of a + m * step into a fused multiply-add.
#pragma clang fp contract(off)

namespace rbmf {

bool nonuniform_set(const double* f, const double* y, int64_t n, int per_bin, double df_min, const double* extra,
                    int64_t n_extra, std::vector<double>& nodes, std::string& err) {
  nodes.clear();
  const double lo = f[0], hi = f[n - 1];
  std::vector<double> edges;
  edges.push_back(lo);
  for (int64_t i = 0; i + 1 < n; ++i) {
    double e;
    if (y[i] == 0.0 && i > 0) e = f[i];
    else if (y[i] * y[i + 1] < 0.0) e = f[i] + (f[i + 1] - f[i]) * (y[i] / (y[i] - y[i + 1]));
    else continue;
    if (e > lo && e < hi) edges.push_back(e);
  }
  edges.push_back(hi);
  for (size_t b = 0; b + 1 < edges.size(); ++b) {
    const double a = edges[b], e = edges[b + 1];
    const double step = (e - a) / per_bin;
    if (step >= df_min) {
      for (int m = 0; m < per_bin; ++m) nodes.push_back(a + m * step);
    } else {
      double kd = std::ceil(a / df_min);
      if (!(kd < 9.0e15)) {
        err = "frequency / df_min too large";
        return false;
      }
      int64_t k = (int64_t)kd;
      while ((double)k * df_min < a) ++k;
      while (k > 0 && (double)(k - 1) * df_min >= a) --k;
      for (; (double)k * df_min < e; ++k) nodes.push_back((double)k * df_min);
    }
  }
  nodes.push_back(hi);
  if (n_extra > 0) {
    for (int64_t i = 0; i < n_extra; ++i)
      if (extra[i] > lo && extra[i] < hi) nodes.push_back(extra[i]);
    std::sort(nodes.begin(), nodes.end());
    nodes.erase(std::unique(nodes.begin(), nodes.end()), nodes.end());
  }
  return true;
}

void cell_weights(const double* x, int64_t n, std::vector<double>& w) {
  w.assign(n, 1.0);
  if (n < 2) return;
  w[0] = x[1] - x[0];
  w[n - 1] = x[n - 1] - x[n - 2];
  for (int64_t i = 1; i + 1 < n; ++i) w[i] = 0.5 * (x[i + 1] - x[i - 1]);
}

void interp_table(const double* x, int64_t nt, int64_t k_lo, int64_t k_hi, double df, std::vector<int32_t>& idx,
                  std::vector<double>& frac) {
  const int64_t nb = k_hi - k_lo + 1;
  idx.resize(nb);
  frac.resize(nb);
  int64_t i = 0;
  for (int64_t k = k_lo; k <= k_hi; ++k) {
    const double fk = (double)k * df;
    while (i + 2 < nt && x[i + 1] <= fk) ++i;   // x[i] <= fk < x[i+1], i <= nt - 2
    idx[k - k_lo] = (int32_t)i;
    double a = (fk - x[i]) / (x[i + 1] - x[i]);
    frac[k - k_lo] = std::min(1.0, std::max(0.0, a));
  }
}

}  // namespace rbmf

using namespace rbmf;

extern "C" rb_status rb_nonuniform_freqs(const double* f, const double* h_re, int64_t n, int32_t per_bin,
                                         double df_min, const double* extra, int64_t n_extra, double* out,
                                         int64_t cap, int64_t* n_out) {
  auto fail = [](const std::string& m) {
    set_error(m);
    return RB_ERR_ARG;
  };
  if (f == nullptr || h_re == nullptr || n_out == nullptr) return fail("NULL argument");
  *n_out = 0;
  if (n < 2) return fail("need at least two reference samples");
  if (per_bin < 1 || per_bin > 1024) return fail("per_bin must be in [1, 1024]");
  if (!(std::isfinite(df_min) && df_min > 0)) return fail("df_min must be finite and > 0");
  if (n_extra < 0 || (n_extra > 0 && extra == nullptr)) return fail("bad extra frequencies");
  if (cap < 0 || (cap > 0 && out == nullptr)) return fail("bad output buffer");
  for (int64_t i = 0; i < n; ++i) {
    if (!std::isfinite(f[i]) || !std::isfinite(h_re[i])) return fail("non-finite reference sample");
    if (i > 0 && !(f[i] > f[i - 1])) return fail("reference frequencies must increase strictly");
  }
  for (int64_t i = 0; i < n_extra; ++i)
    if (!std::isfinite(extra[i])) return fail("non-finite extra frequency");
  std::vector<double> nodes;
  std::string err;
  if (!nonuniform_set(f, h_re, n, per_bin, df_min, extra, n_extra, nodes, err)) return fail(err);
  *n_out = (int64_t)nodes.size();
  if ((int64_t)nodes.size() > cap) {
    set_error("frequency set has " + std::to_string(nodes.size()) + " entries, capacity " + std::to_string(cap));
    return RB_ERR_CAPACITY;
  }
  std::copy(nodes.begin(), nodes.end(), out);
  return RB_OK;
}
