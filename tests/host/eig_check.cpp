// Host check of the basis construction's Hermitian eigensolver: builds
// A = Q diag(lambda) Q^H from a random unitary Q and a prescribed spectrum,
// and compares the returned eigenvalues (descending) and the residual
// ||A v - lambda v|| of the leading eigenvectors.
// usage: eig_check n log10_min rank   (exit 0 when every check passes)
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "linalg.h"

using cd = std::complex<double>;

int main(int argc, char** argv) {
  const int n = argc > 1 ? std::atoi(argv[1]) : 200;
  const double lo = argc > 2 ? std::atof(argv[2]) : -12;
  const int rk = argc > 3 ? std::atoi(argv[3]) : n;
  std::mt19937_64 rng(7);
  std::normal_distribution<double> nd;
  std::vector<cd> Q((size_t)n * n);
  for (auto& v : Q) v = cd(nd(rng), nd(rng));
  for (int j = 0; j < n; ++j) {   // modified Gram-Schmidt on columns
    for (int k = 0; k < j; ++k) {
      cd s = 0;
      for (int i = 0; i < n; ++i) s += std::conj(Q[(size_t)i * n + k]) * Q[(size_t)i * n + j];
      for (int i = 0; i < n; ++i) Q[(size_t)i * n + j] -= s * Q[(size_t)i * n + k];
    }
    double nr = 0;
    for (int i = 0; i < n; ++i) nr += std::norm(Q[(size_t)i * n + j]);
    nr = std::sqrt(nr);
    for (int i = 0; i < n; ++i) Q[(size_t)i * n + j] /= nr;
  }
  std::vector<double> lam(n, 0.0);
  for (int i = 0; i < rk; ++i) lam[i] = std::pow(10.0, lo * i / (rk > 1 ? rk - 1 : 1));
  std::vector<cd> A((size_t)n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      cd s = 0;
      for (int k = 0; k < rk; ++k) s += Q[(size_t)i * n + k] * lam[k] * std::conj(Q[(size_t)j * n + k]);
      A[(size_t)i * n + j] = s;
    }
  std::vector<double> w;
  std::vector<cd> V;
  const auto t0 = std::chrono::steady_clock::now();
  const bool ok = rbmf::herm_eig_desc(n, A, w, V);
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (!ok) {
    std::printf("n=%d: no convergence\n", n);
    return 1;
  }
  double ev = 0.0, res = 0.0;
  for (int i = 0; i < n; ++i) ev = std::max(ev, std::fabs(w[i] - lam[i]));
  for (int k = 0; k < std::min(n, 10); ++k) {   // residual of the 10 leading pairs (V row-major, column k)
    double r2 = 0.0;
    for (int i = 0; i < n; ++i) {
      cd s = 0;
      for (int j = 0; j < n; ++j) s += A[(size_t)i * n + j] * V[(size_t)j * n + k];
      r2 += std::norm(s - w[k] * V[(size_t)i * n + k]);
    }
    res = std::max(res, std::sqrt(r2));
  }
  for (int i = 1; i < n; ++i)
    if (w[i] > w[i - 1]) {
      std::printf("n=%d: not descending at %d\n", n, i);
      return 1;
    }
  std::printf("n=%d rank=%d min=1e%g: max eigenvalue error %.2e, leading residual %.2e (%.2f s)\n", n, rk, lo, ev,
              res, secs);
  return (ev <= 1e-12 && res <= 1e-12) ? 0 : 1;
}
