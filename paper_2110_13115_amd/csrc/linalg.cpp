// Host FP64 dense linear algebra for the basis construction: eigen-
// decomposition of small complex Hermitian matrices (the Rayleigh-Ritz and
// orthonormalisation problems of size L x L, L ~ rank + oversampling).
//
// Method: unitary Householder reduction to Hermitian tridiagonal form, a
// diagonal phase scaling that makes the tridiagonal real, the implicit QL
// iteration with Wilkinson-type shifts on the real tridiagonal (accumulating
// the plane rotations), and back-transformation of the eigenvectors.
#include "linalg.h"

#include <algorithm>
#include <cmath>
#include <numeric>
#include <thread>

namespace rbmf {

using cd = std::complex<double>;

namespace {

// Splits [0, n) into contiguous blocks run on up to 16 host threads (serially
// when the work is small); f(lo, hi) must touch only its own block.
template <class F>
void par_blocks(int n, int min_block, F&& f) {
  static const int hw = std::max(1, std::min(16, (int)std::thread::hardware_concurrency()));
  const int nt = std::min(hw, n / std::max(1, min_block));
  if (nt <= 1) {
    f(0, n);
    return;
  }
  const int step = (n + nt - 1) / nt;
  std::vector<std::thread> th;
  th.reserve(nt - 1);
  for (int t = 1; t < nt; ++t) th.emplace_back([&, t] { f(t * step, std::min(n, (t + 1) * step)); });
  f(0, std::min(n, step));
  for (auto& x : th) x.join();
}

// Implicit QL on a real symmetric tridiagonal (d: diagonal, e[i] = T[i+1][i],
// e[n-1] unused).  Z (n x n, column-major: Z[i + n*j]) accumulates rotations.
// The published method: the QL algorithm with implicit Wilkinson shifts of
// Bowdler, Martin, Reinsch and Wilkinson (Numer. Math. 11, 293-306, 1968;
// the procedure EISPACK calls tql2), with its own deflation test (below) and
// the plane rotations applied to Z in parallel over rows.
bool tql_implicit(int n, std::vector<double>& d, std::vector<double>& e, std::vector<double>& Z) {
  if (n == 1) return true;
  e[n - 1] = 0.0;
  const double eps = std::numeric_limits<double>::epsilon();
  // Deflation test against the largest |d| + |e| met so far (a norm of the
  // tridiagonal), not only against the neighbouring diagonal: inside a
  // cluster of eigenvalues at round-off level (rank-deficient Gram matrices)
  // both neighbours are themselves round-off and a purely local test never
  // succeeds.  Perturbations below eps times the norm are backward stable.
  double tst = 0.0;
  std::vector<int> rot_i;
  std::vector<double> rot_s, rot_c;
  for (int l = 0; l < n; ++l) {
    int iter = 0;
    int m;
    tst = std::max(tst, std::fabs(d[l]) + std::fabs(e[l]));
    do {
      for (m = l; m < n - 1; ++m) {
        const double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
        if (std::fabs(e[m]) <= eps * dd || std::fabs(e[m]) <= eps * tst) break;
      }
      if (m != l) {
        if (++iter > 100) return false;
        double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
        double r = std::hypot(g, 1.0);
        g = d[m] - d[l] + e[l] / (g + (g >= 0 ? std::fabs(r) : -std::fabs(r)));
        double s = 1.0, c = 1.0, p = 0.0;
        int i;
        bool deflated = false;
        rot_i.clear();
        rot_s.clear();
        rot_c.clear();
        for (i = m - 1; i >= l; --i) {
          double f = s * e[i];
          const double b = c * e[i];
          r = std::hypot(f, g);
          e[i + 1] = r;
          if (r == 0.0) {
            d[i + 1] -= p;
            e[m] = 0.0;
            deflated = true;
            break;
          }
          s = f / r;
          c = g / r;
          g = d[i + 1] - p;
          r = (d[i] - g) * s + 2.0 * c * b;
          p = s * r;
          d[i + 1] = g + p;
          g = c * r - b;
          rot_i.push_back(i);
          rot_s.push_back(s);
          rot_c.push_back(c);
        }
        // the sweep's plane rotations, in order, applied to every row of Z
        // (rows are independent, so blocks of rows run in parallel)
        const int nr = (int)rot_i.size();
        par_blocks(n, 64 * std::max(1, 4096 / std::max(1, nr)), [&](int k0, int k1) {
          for (int t = 0; t < nr; ++t) {
            const int ii = rot_i[t];
            const double st = rot_s[t], ct = rot_c[t];
            double* zi = &Z[(size_t)n * ii];
            double* zi1 = &Z[(size_t)n * (ii + 1)];
            for (int k = k0; k < k1; ++k) {
              const double f = zi1[k];
              zi1[k] = st * zi[k] + ct * f;
              zi[k] = ct * zi[k] - st * f;
            }
          }
        });
        if (deflated) continue;
        d[l] -= p;
        e[l] = g;
        e[m] = 0.0;
      }
    } while (m != l);
  }
  return true;
}

}  // namespace

bool herm_eig_desc(int n, const std::vector<cd>& Ain, std::vector<double>& w, std::vector<cd>& V) {
  // A row-major n x n Hermitian (only the lower triangle is read).
  std::vector<cd> A(Ain);
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) A[(size_t)i * n + j] = std::conj(A[(size_t)j * n + i]);
  for (int i = 0; i < n; ++i) A[(size_t)i * n + i] = cd(A[(size_t)i * n + i].real(), 0.0);

  std::vector<double> d(n), e(n, 0.0);
  std::vector<cd> sub(n, cd(0.0, 0.0));
  std::vector<std::vector<cd>> refl;   // Householder vectors v_k (length n-k-1), H = I - 2 v v^H
  refl.reserve(n > 2 ? n - 2 : 0);
  std::vector<cd> p(n), wv(n);
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;
    // x = A[k+1:, k]
    double xn2 = 0.0;
    for (int i = 0; i < m; ++i) xn2 += std::norm(A[(size_t)(k + 1 + i) * n + k]);
    const double xn = std::sqrt(xn2);
    std::vector<cd> v(m, cd(0.0, 0.0));
    if (xn == 0.0) {
      refl.push_back(v);
      sub[k] = cd(0.0, 0.0);
      continue;
    }
    const cd x0 = A[(size_t)(k + 1) * n + k];
    const cd ph = (std::abs(x0) > 0.0) ? x0 / std::abs(x0) : cd(1.0, 0.0);
    const cd alpha = -ph * xn;
    for (int i = 0; i < m; ++i) v[i] = A[(size_t)(k + 1 + i) * n + k];
    v[0] -= alpha;
    double vn2 = 0.0;
    for (int i = 0; i < m; ++i) vn2 += std::norm(v[i]);
    const double vn = std::sqrt(vn2);
    for (int i = 0; i < m; ++i) v[i] /= vn;
    // p = A22 v ; Kv = v^H p ; w = p - Kv v ; A22 -= 2 (v w^H + w v^H)
    par_blocks(m, 128, [&](int i0, int i1) {
      for (int i = i0; i < i1; ++i) {
        cd s(0.0, 0.0);
        const cd* row = &A[(size_t)(k + 1 + i) * n + (k + 1)];
        for (int j = 0; j < m; ++j) s += row[j] * v[j];
        p[i] = s;
      }
    });
    cd Kv(0.0, 0.0);
    for (int i = 0; i < m; ++i) Kv += std::conj(v[i]) * p[i];
    const double kr = Kv.real();
    for (int i = 0; i < m; ++i) wv[i] = p[i] - kr * v[i];
    par_blocks(m, 128, [&](int i0, int i1) {
      for (int i = i0; i < i1; ++i) {
        cd* row = &A[(size_t)(k + 1 + i) * n + (k + 1)];
        for (int j = 0; j < m; ++j) row[j] -= 2.0 * (v[i] * std::conj(wv[j]) + wv[i] * std::conj(v[j]));
      }
    });
    sub[k] = alpha;
    for (int i = 0; i < m; ++i) {
      A[(size_t)(k + 1 + i) * n + k] = (i == 0) ? alpha : cd(0.0, 0.0);
      A[(size_t)k * n + (k + 1 + i)] = (i == 0) ? std::conj(alpha) : cd(0.0, 0.0);
    }
    refl.push_back(v);
  }
  for (int k = 0; k < n; ++k) d[k] = A[(size_t)k * n + k].real();
  if (n >= 2) sub[n - 2] = A[(size_t)(n - 1) * n + (n - 2)];
  // phase scaling: T = D T' D^H with T' real
  std::vector<cd> delta(n, cd(1.0, 0.0));
  for (int k = 0; k + 1 < n; ++k) {
    const double a = std::abs(sub[k]);
    e[k] = a;
    delta[k + 1] = (a > 0.0) ? delta[k] * (sub[k] / a) : delta[k];
  }
  std::vector<double> Z((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) Z[(size_t)n * i + i] = 1.0;
  if (!tql_implicit(n, d, e, Z)) return false;
  // order descending
  std::vector<int> ord(n);
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return d[a] > d[b]; });
  w.resize(n);
  V.assign((size_t)n * n, cd(0.0, 0.0));   // row-major, column j = eigenvector j
  for (int jj = 0; jj < n; ++jj) {
    const int j = ord[jj];
    w[jj] = d[j];
    for (int i = 0; i < n; ++i) V[(size_t)i * n + jj] = delta[i] * Z[(size_t)n * j + i];
  }
  // back-transform: U = H_0 H_1 ... H_{n-3} Y
  // (blocks of columns in parallel; rows are walked contiguously)
  par_blocks(n, 64, [&](int c0, int c1) {
    std::vector<cd> sc(c1 - c0);
    for (int k = (int)refl.size() - 1; k >= 0; --k) {
      const std::vector<cd>& v = refl[k];
      const int m = (int)v.size();
      std::fill(sc.begin(), sc.end(), cd(0.0, 0.0));
      for (int i = 0; i < m; ++i) {
        const cd cv = std::conj(v[i]);
        const cd* row = &V[(size_t)(k + 1 + i) * n];
        for (int col = c0; col < c1; ++col) sc[col - c0] += cv * row[col];
      }
      for (int i = 0; i < m; ++i) {
        const cd vi = 2.0 * v[i];
        cd* row = &V[(size_t)(k + 1 + i) * n];
        for (int col = c0; col < c1; ++col) row[col] -= vi * sc[col - c0];
      }
    }
  });
  return true;
}

}  // namespace rbmf
