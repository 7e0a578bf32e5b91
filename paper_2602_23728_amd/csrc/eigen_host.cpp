// Gamma-point phonons on the host in FP64: the real symmetric dynamical
// matrix D = sum_l Phi(0, l)/sqrt(m m) (paper: Eq. dynmat, Eq. eigenvalue),
// reduced to tridiagonal form by Householder reflections and diagonalised by
// the implicit QL method with Wilkinson-type shifts; eigenvectors are
// accumulated alongside.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "common.h"

namespace kaldo {

// In-place Householder tridiagonalisation of the symmetric n x n matrix A
// (row-major).  On return d = diagonal, e[k] = T[k+1][k] (e[n-1] = 0), and
// Q (row-major, n x n) holds the orthogonal basis: A_in = Q T Q^T.
static void tridiagonalise(int n, std::vector<double>& A, std::vector<double>& d,
                           std::vector<double>& e, std::vector<double>& Q) {
  Q.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) Q[(size_t)i * n + i] = 1.0;
  std::vector<double> v(n), p(n), w(n);
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;  // length of the column below the diagonal
    double norm = 0.0;
    for (int i = 0; i < m; ++i) {
      double x = A[(size_t)(k + 1 + i) * n + k];
      v[i] = x;
      norm += x * x;
    }
    norm = std::sqrt(norm);
    if (norm == 0.0) continue;
    const double alpha = v[0] > 0 ? -norm : norm;
    v[0] -= alpha;
    double vn = 0.0;
    for (int i = 0; i < m; ++i) vn += v[i] * v[i];
    vn = std::sqrt(vn);
    if (vn == 0.0) continue;
    for (int i = 0; i < m; ++i) v[i] /= vn;
    // p = B v over the trailing block B = A[k+1:, k+1:]
    for (int i = 0; i < m; ++i) {
      const double* row = &A[(size_t)(k + 1 + i) * n + k + 1];
      double s = 0.0;
      for (int j = 0; j < m; ++j) s += row[j] * v[j];
      p[i] = s;
    }
    double K = 0.0;
    for (int i = 0; i < m; ++i) K += v[i] * p[i];
    for (int i = 0; i < m; ++i) w[i] = p[i] - K * v[i];
    // B <- B - 2 (v w^T + w v^T)
    for (int i = 0; i < m; ++i) {
      double* row = &A[(size_t)(k + 1 + i) * n + k + 1];
      const double vi = v[i], wi = w[i];
      for (int j = 0; j < m; ++j) row[j] -= 2.0 * (vi * w[j] + wi * v[j]);
    }
    A[(size_t)(k + 1) * n + k] = alpha;
    A[(size_t)k * n + k + 1] = alpha;
    for (int i = 1; i < m; ++i) {
      A[(size_t)(k + 1 + i) * n + k] = 0.0;
      A[(size_t)k * n + k + 1 + i] = 0.0;
    }
    // Q[:, k+1:] <- Q[:, k+1:] (I - 2 v v^T)
    for (int r = 0; r < n; ++r) {
      double* row = &Q[(size_t)r * n + k + 1];
      double s = 0.0;
      for (int j = 0; j < m; ++j) s += row[j] * v[j];
      s *= 2.0;
      for (int j = 0; j < m; ++j) row[j] -= s * v[j];
    }
  }
  d.resize(n);
  e.assign(n, 0.0);
  for (int i = 0; i < n; ++i) d[i] = A[(size_t)i * n + i];
  for (int i = 0; i + 1 < n; ++i) e[i] = A[(size_t)(i + 1) * n + i];
}

// Implicit QL on the tridiagonal (d, e); Zt holds eigenvectors as rows
// (Zt[j][:] is eigenvector j), initialised with Q^T.  Returns false if an
// eigenvalue needs more than 60 iterations.
static bool tridiagonal_ql(int n, std::vector<double>& d, std::vector<double>& e,
                           std::vector<double>& Zt) {
  // A subdiagonal entry is negligible relative to its neighbours or to the
  // whole matrix (backward-stable either way).
  double tnorm = 0.0;
  for (int i = 0; i < n; ++i) tnorm = std::max(tnorm, std::fabs(d[i]) + std::fabs(e[i]));
  const double abs_tol = 1e-15 * tnorm;
  for (int l = 0; l < n; ++l) {
    int iter = 0;
    while (true) {
      int m = l;
      for (; m < n - 1; ++m) {
        double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
        if (std::fabs(e[m]) <= 1e-16 * dd || std::fabs(e[m]) <= abs_tol) break;
      }
      if (m == l) break;
      if (++iter > 60) return false;
      // shift from the leading 2x2 block
      double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
      double r = std::hypot(g, 1.0);
      g = d[m] - d[l] + e[l] / (g + (g >= 0 ? r : -r));
      double s = 1.0, c = 1.0, p = 0.0;
      int i = m - 1;
      bool deflated = false;
      for (; i >= l; --i) {
        double f = s * e[i], b = c * e[i];
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
        // rotate eigenvector rows i and i+1
        double* zi = &Zt[(size_t)i * n];
        double* zj = &Zt[(size_t)(i + 1) * n];
        for (int k = 0; k < n; ++k) {
          double t = zj[k];
          zj[k] = s * zi[k] + c * t;
          zi[k] = c * zi[k] - s * t;
        }
      }
      if (deflated) continue;
      d[l] -= p;
      e[l] = g;
      e[m] = 0.0;
    }
  }
  return true;
}

}  // namespace kaldo

using namespace kaldo;

extern "C" int kaldo_phonons_gamma(int32_t n_basis, const double* mass, int32_t n_rep,
                                   const double* fc2, double* omega, double* evec) {
  KALDO_REQUIRE(n_basis >= 1 && n_rep >= 1, "kaldo_phonons_gamma: bad sizes");
  KALDO_REQUIRE(mass && fc2 && omega && evec, "kaldo_phonons_gamma: NULL argument");
  const int n = 3 * n_basis;
  for (int i = 0; i < n_basis; ++i)
    KALDO_REQUIRE(std::isfinite(mass[i]) && mass[i] > 0, "kaldo_phonons_gamma: mass <= 0");
  std::vector<double> A((size_t)n * n, 0.0);
  for (int a = 0; a < n; ++a)
    for (int l = 0; l < n_rep; ++l)
      for (int b = 0; b < n; ++b) {
        const double f = fc2[((size_t)a * n_rep + l) * n + b];
        KALDO_REQUIRE(std::isfinite(f), "kaldo_phonons_gamma: non-finite FC2");
        A[(size_t)a * n + b] += f;
      }
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b) A[(size_t)a * n + b] /= std::sqrt(mass[a / 3] * mass[b / 3]);
  for (int a = 0; a < n; ++a)
    for (int b = a + 1; b < n; ++b) {
      double s = 0.5 * (A[(size_t)a * n + b] + A[(size_t)b * n + a]);
      A[(size_t)a * n + b] = A[(size_t)b * n + a] = s;
    }
  std::vector<double> d, e, Q;
  tridiagonalise(n, A, d, e, Q);
  std::vector<double> Zt((size_t)n * n);
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < n; ++k) Zt[(size_t)i * n + k] = Q[(size_t)k * n + i];
  if (!tridiagonal_ql(n, d, e, Zt)) {
    set_error("kaldo_phonons_gamma: QL iteration did not converge");
    return KALDO_ENUMERIC;
  }
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return d[a] < d[b]; });
  for (int j = 0; j < n; ++j) {
    const int src = order[j];
    const double l = d[src];
    omega[j] = l >= 0 ? std::sqrt(l * kU) : -std::sqrt(-l * kU);
    const double* z = &Zt[(size_t)src * n];
    int best = 0;
    for (int k = 1; k < n; ++k)
      if (std::fabs(z[k]) > std::fabs(z[best])) best = k;
    const double sg = z[best] < 0 ? -1.0 : 1.0;
    for (int k = 0; k < n; ++k) evec[(size_t)k * n + j] = sg * z[k];
  }
  return KALDO_OK;
}
