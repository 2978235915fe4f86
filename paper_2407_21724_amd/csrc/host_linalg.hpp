// Small dense FP64 linear algebra for the setup stages: complex LU inverse,
// Cholesky, and the symmetric eigensolver (Householder tridiagonalisation +
// implicit-shift QL) behind the generalized eigenproblems of the static modes.
#pragma once

#include <cmath>
#include <complex>
#include <stdexcept>
#include <vector>

namespace mlfma {

// In-place inverse of an n x n complex matrix (row-major) by LU with partial
// pivoting.  Returns false if the matrix is numerically singular.
inline bool complex_inverse(std::vector<std::complex<double>>& A, int n) {
  using cd = std::complex<double>;
  std::vector<int> piv(n);
  std::vector<cd> LU = A;
  for (int k = 0; k < n; ++k) {
    int p = k;
    double best = std::abs(LU[(size_t)k * n + k]);
    for (int i = k + 1; i < n; ++i) {
      double v = std::abs(LU[(size_t)i * n + k]);
      if (v > best) best = v, p = i;
    }
    if (best == 0.0 || !std::isfinite(best)) return false;
    piv[k] = p;
    if (p != k)
      for (int j = 0; j < n; ++j) std::swap(LU[(size_t)k * n + j], LU[(size_t)p * n + j]);
    cd inv = 1.0 / LU[(size_t)k * n + k];
    for (int i = k + 1; i < n; ++i) {
      cd f = LU[(size_t)i * n + k] * inv;
      LU[(size_t)i * n + k] = f;
      for (int j = k + 1; j < n; ++j) LU[(size_t)i * n + j] -= f * LU[(size_t)k * n + j];
    }
  }
  // solve for each unit vector (apply row swaps to the identity)
  std::vector<cd> X((size_t)n * n, 0.0);
  for (int c = 0; c < n; ++c) {
    std::vector<cd> b(n, 0.0);
    b[c] = 1.0;
    for (int k = 0; k < n; ++k) std::swap(b[k], b[piv[k]]);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < i; ++j) b[i] -= LU[(size_t)i * n + j] * b[j];
    for (int i = n - 1; i >= 0; --i) {
      for (int j = i + 1; j < n; ++j) b[i] -= LU[(size_t)i * n + j] * b[j];
      b[i] /= LU[(size_t)i * n + i];
    }
    for (int i = 0; i < n; ++i) X[(size_t)i * n + c] = b[i];
  }
  A.swap(X);
  return true;
}

// Lower Cholesky factor of a symmetric positive definite matrix (row-major).
inline bool cholesky(std::vector<double>& A, int n) {
  for (int j = 0; j < n; ++j) {
    double s = A[(size_t)j * n + j];
    for (int k = 0; k < j; ++k) s -= A[(size_t)j * n + k] * A[(size_t)j * n + k];
    if (s <= 0.0) return false;
    double ljj = std::sqrt(s);
    A[(size_t)j * n + j] = ljj;
    for (int i = j + 1; i < n; ++i) {
      double t = A[(size_t)i * n + j];
      for (int k = 0; k < j; ++k) t -= A[(size_t)i * n + k] * A[(size_t)j * n + k];
      A[(size_t)i * n + j] = t / ljj;
    }
    for (int k = j + 1; k < n; ++k) A[(size_t)j * n + k] = 0.0;
  }
  return true;
}

// Eigen-decomposition of a real symmetric matrix.  On return `evals` holds
// the eigenvalues (unsorted) and column k of V (row-major n x n) the unit
// eigenvector of evals[k].
inline void symmetric_eigen(const std::vector<double>& Ain, int n, std::vector<double>& evals,
                            std::vector<double>& V) {
  V = Ain;
  std::vector<double> d(n), e(n, 0.0);
  auto at = [&](int i, int j) -> double& { return V[(size_t)i * n + j]; };
  // Householder reduction to tridiagonal form, accumulating the transform.
  for (int i = n - 1; i > 0; --i) {
    int l = i - 1;
    double h = 0.0;
    if (l > 0) {
      double scale = 0.0;
      for (int k = 0; k <= l; ++k) scale += std::fabs(at(i, k));
      if (scale == 0.0) {
        e[i] = at(i, l);
      } else {
        for (int k = 0; k <= l; ++k) {
          at(i, k) /= scale;
          h += at(i, k) * at(i, k);
        }
        double f = at(i, l);
        double g = f >= 0 ? -std::sqrt(h) : std::sqrt(h);
        e[i] = scale * g;
        h -= f * g;
        at(i, l) = f - g;
        f = 0.0;
        for (int j = 0; j <= l; ++j) {
          at(j, i) = at(i, j) / h;
          double gg = 0.0;
          for (int k = 0; k <= j; ++k) gg += at(j, k) * at(i, k);
          for (int k = j + 1; k <= l; ++k) gg += at(k, j) * at(i, k);
          e[j] = gg / h;
          f += e[j] * at(i, j);
        }
        double hh = f / (h + h);
        for (int j = 0; j <= l; ++j) {
          double ff = at(i, j);
          double gg = e[j] - hh * ff;
          e[j] = gg;
          for (int k = 0; k <= j; ++k) at(j, k) -= ff * e[k] + gg * at(i, k);
        }
      }
    } else {
      e[i] = at(i, l);
    }
    d[i] = h;
  }
  d[0] = 0.0;
  e[0] = 0.0;
  for (int i = 0; i < n; ++i) {
    int l = i - 1;
    if (d[i] != 0.0) {
      for (int j = 0; j <= l; ++j) {
        double g = 0.0;
        for (int k = 0; k <= l; ++k) g += at(i, k) * at(k, j);
        for (int k = 0; k <= l; ++k) at(k, j) -= g * at(k, i);
      }
    }
    d[i] = at(i, i);
    at(i, i) = 1.0;
    for (int j = 0; j <= l; ++j) at(j, i) = at(i, j) = 0.0;
  }
  // QL iteration with implicit shifts on the tridiagonal matrix.
  for (int i = 1; i < n; ++i) e[i - 1] = e[i];
  e[n - 1] = 0.0;
  for (int l = 0; l < n; ++l) {
    int iter = 0, m;
    do {
      for (m = l; m < n - 1; ++m) {
        double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
        if (std::fabs(e[m]) <= 1e-15 * dd) break;
      }
      if (m != l) {
        if (++iter > 200) throw std::runtime_error("symmetric_eigen: no convergence");
        double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
        double r = std::hypot(g, 1.0);
        g = d[m] - d[l] + e[l] / (g + (g >= 0 ? std::fabs(r) : -std::fabs(r)));
        double s = 1.0, c = 1.0, p = 0.0;
        int i;
        for (i = m - 1; i >= l; --i) {
          double f = s * e[i], b = c * e[i];
          r = std::hypot(f, g);
          e[i + 1] = r;
          if (r == 0.0) {
            d[i + 1] -= p;
            e[m] = 0.0;
            break;
          }
          s = f / r;
          c = g / r;
          g = d[i + 1] - p;
          r = (d[i] - g) * s + 2.0 * c * b;
          p = s * r;
          d[i + 1] = g + p;
          g = c * r - b;
          for (int k = 0; k < n; ++k) {
            f = at(k, i + 1);
            at(k, i + 1) = s * at(k, i) + c * f;
            at(k, i) = c * at(k, i) - s * f;
          }
        }
        if (r == 0.0 && i >= l) continue;
        d[l] -= p;
        e[l] = g;
        e[m] = 0.0;
      }
    } while (m != l);
  }
  evals = d;
}

// Generalized symmetric-definite eigenproblem A v = g B v.  Columns of the
// returned V (row-major n x n) are B-orthonormal eigenvectors.
inline void generalized_eigen(std::vector<double> A, std::vector<double> B, int n,
                              std::vector<double>& evals, std::vector<double>& Vout) {
  if (!cholesky(B, n)) throw std::runtime_error("generalized_eigen: B not positive definite");
  auto Lij = [&](int i, int j) { return B[(size_t)i * n + j]; };
  // C = L^-1 A L^-T: solve L X = A, then L C^T = X^T
  for (int c = 0; c < n; ++c)
    for (int i = 0; i < n; ++i) {
      double s = A[(size_t)i * n + c];
      for (int k = 0; k < i; ++k) s -= Lij(i, k) * A[(size_t)k * n + c];
      A[(size_t)i * n + c] = s / Lij(i, i);
    }
  std::vector<double> C((size_t)n * n);
  for (int r = 0; r < n; ++r)
    for (int i = 0; i < n; ++i) {
      double s = A[(size_t)r * n + i];
      for (int k = 0; k < i; ++k) s -= Lij(i, k) * C[(size_t)r * n + k];
      C[(size_t)r * n + i] = s / Lij(i, i);
    }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < i; ++j) {
      double s = 0.5 * (C[(size_t)i * n + j] + C[(size_t)j * n + i]);
      C[(size_t)i * n + j] = C[(size_t)j * n + i] = s;
    }
  std::vector<double> U;
  symmetric_eigen(C, n, evals, U);
  // v = L^-T u
  Vout.assign((size_t)n * n, 0.0);
  for (int col = 0; col < n; ++col)
    for (int i = n - 1; i >= 0; --i) {
      double s = U[(size_t)i * n + col];
      for (int k = i + 1; k < n; ++k) s -= Lij(k, i) * Vout[(size_t)k * n + col];
      Vout[(size_t)i * n + col] = s / Lij(i, i);
    }
}

}  // namespace mlfma
