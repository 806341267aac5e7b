// Host helpers of the non-uniform-frequency PCA (Sec. III.A).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace rbmf {

// The frequency set of rb_nonuniform_freqs (arguments already validated).
bool nonuniform_set(const double* f, const double* y, int64_t n, int per_bin, double df_min, const double* extra,
                    int64_t n_extra, std::vector<double>& nodes, std::string& err);

// omega_i: width of node i's cell between the midpoints to its neighbours,
// the end cells mirrored.
void cell_weights(const double* x, int64_t n, std::vector<double>& w);

// For the uniform frequencies k df, k = k_lo..k_hi, inside [x[0], x[nt-1]]:
// idx = i with x[i] <= k df <= x[i+1] (0 <= i <= nt - 2), frac = the linear
// weight of x[i+1] (0 when k df is the node x[i] itself).
void interp_table(const double* x, int64_t nt, int64_t k_lo, int64_t k_hi, double df, std::vector<int32_t>& idx,
                  std::vector<double>& frac);

}  // namespace rbmf
