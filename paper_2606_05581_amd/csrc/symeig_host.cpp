// Dense symmetric eigensolver for the small projected (Rayleigh-Ritz)
// problems of the eigen step, FP64 on the host. Two phases, as stated in
// Golub & Van Loan, "Matrix Computations", ch. 8: Householder reduction of
// A to tridiagonal form T = Q^T A Q, then implicit symmetric QR steps with a
// Wilkinson shift (Givens bulge chase) until T is diagonal, with all
// transforms accumulated into the eigenvector matrix.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

namespace msk {

namespace {

// In place: A (n x n, row-major, symmetric) -> tridiagonal (diag d, off e,
// e[i] couples i and i+1); Q accumulates the reflections (A = Q T Q^T).
void tridiagonalise(int n, std::vector<double>& A, std::vector<double>& Q, std::vector<double>& d,
                    std::vector<double>& e) {
  auto a = [&](int i, int j) -> double& { return A[(size_t)i * n + j]; };
  Q.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) Q[(size_t)i * n + i] = 1.0;
  std::vector<double> v(n), p(n), w(n), qv(n);
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;  // length of x = A[k+1:n, k]
    double sigma = 0.0;
    for (int i = 1; i < m; ++i) sigma += a(k + 1 + i, k) * a(k + 1 + i, k);
    const double x0 = a(k + 1, k);
    if (sigma == 0.0) continue;  // already tridiagonal in this column (x0 may be any sign)
    // reflector P = I - beta v v^T with v[0] = 1 and P x = mu e1
    const double mu = std::sqrt(x0 * x0 + sigma);
    const double v0 = x0 <= 0.0 ? x0 - mu : -sigma / (x0 + mu);
    const double beta = 2.0 * v0 * v0 / (sigma + v0 * v0);
    v[0] = 1.0;
    for (int i = 1; i < m; ++i) v[i] = a(k + 1 + i, k) / v0;
    // p = beta * A22 v ; w = p - (beta p^T v / 2) v
    double pv = 0.0;
    for (int i = 0; i < m; ++i) {
      double s = 0.0;
      const double* row = &A[(size_t)(k + 1 + i) * n + (k + 1)];
      for (int j = 0; j < m; ++j) s += row[j] * v[j];
      p[i] = beta * s;
      pv += p[i] * v[i];
    }
    const double half = 0.5 * beta * pv;
    for (int i = 0; i < m; ++i) w[i] = p[i] - half * v[i];
    // A22 -= v w^T + w v^T ; column k becomes mu e1
    for (int i = 0; i < m; ++i) {
      double* row = &A[(size_t)(k + 1 + i) * n + (k + 1)];
      for (int j = 0; j < m; ++j) row[j] -= v[i] * w[j] + w[i] * v[j];
    }
    a(k + 1, k) = a(k, k + 1) = mu;
    for (int i = 1; i < m; ++i) a(k + 1 + i, k) = a(k, k + 1 + i) = 0.0;
    // Q[:, k+1:] = Q[:, k+1:] (I - beta v v^T)
    for (int r = 0; r < n; ++r) {
      double* row = &Q[(size_t)r * n + (k + 1)];
      double s = 0.0;
      for (int j = 0; j < m; ++j) s += row[j] * v[j];
      s *= beta;
      for (int j = 0; j < m; ++j) row[j] -= s * v[j];
    }
  }
  d.assign(n, 0.0);
  e.assign(n, 0.0);
  for (int i = 0; i < n; ++i) d[i] = a(i, i);
  for (int i = 0; i + 1 < n; ++i) e[i] = a(i + 1, i);
}

// Implicit symmetric QR on the unreduced block lo..hi with a Wilkinson shift.
void qr_step(int n, int lo, int hi, std::vector<double>& d, std::vector<double>& e, std::vector<double>& Q) {
  // shift: eigenvalue of the trailing 2x2 closer to d[hi]
  const double dlt = 0.5 * (d[hi - 1] - d[hi]);
  const double b = e[hi - 1];
  const double sg = dlt >= 0.0 ? 1.0 : -1.0;
  const double shift = d[hi] - b * b / (dlt + sg * std::hypot(dlt, b));
  double x = d[lo] - shift, z = e[lo];
  for (int k = lo; k < hi; ++k) {
    const double r = std::hypot(x, z);
    const double c = r == 0.0 ? 1.0 : x / r, s = r == 0.0 ? 0.0 : z / r;
    if (k > lo) e[k - 1] = r;
    const double ak = d[k], bk = e[k], ck = d[k + 1];
    d[k] = c * c * ak + 2.0 * c * s * bk + s * s * ck;
    d[k + 1] = s * s * ak - 2.0 * c * s * bk + c * c * ck;
    e[k] = c * s * (ck - ak) + (c * c - s * s) * bk;
    if (k + 1 < hi) {  // bulge below the band, then chase it
      z = s * e[k + 1];
      e[k + 1] *= c;
      x = e[k];
    }
    for (int r2 = 0; r2 < n; ++r2) {  // columns k, k+1 of Q rotate
      double* row = &Q[(size_t)r2 * n];
      const double qk = row[k], qk1 = row[k + 1];
      row[k] = c * qk + s * qk1;
      row[k + 1] = -s * qk + c * qk1;
    }
  }
}

}  // namespace

// A: n x n symmetric, row-major (destroyed); on return evals ascending and V
// (row-major, column j = eigenvector j). Returns false if QR did not settle.
bool sym_eig(int n, std::vector<double>& A, std::vector<double>& evals, std::vector<double>& V) {
  std::vector<double> d, e, Q;
  tridiagonalise(n, A, Q, d, e);
  const double tol = 4e-16;
  int hi = n - 1;
  long iters = 0;
  while (hi > 0) {
    if (std::fabs(e[hi - 1]) <= tol * (std::fabs(d[hi - 1]) + std::fabs(d[hi]))) {
      e[hi - 1] = 0.0;
      --hi;
      continue;
    }
    int lo = hi - 1;
    while (lo > 0 && std::fabs(e[lo - 1]) > tol * (std::fabs(d[lo - 1]) + std::fabs(d[lo]))) --lo;
    if (lo > 0) e[lo - 1] = 0.0;
    qr_step(n, lo, hi, d, e, Q);
    if (++iters > 60L * n + 100) return false;
  }
  std::vector<int> idx(n);
  std::iota(idx.begin(), idx.end(), 0);
  std::sort(idx.begin(), idx.end(), [&](int x, int y) { return d[x] < d[y]; });
  evals.assign(n, 0.0);
  V.assign((size_t)n * n, 0.0);
  for (int j = 0; j < n; ++j) {
    evals[j] = d[idx[j]];
    for (int r = 0; r < n; ++r) V[(size_t)r * n + j] = Q[(size_t)r * n + idx[j]];
  }
  return true;
}

// Upper Cholesky factor R (A = R^T R) of a small SPD matrix, row-major.
// Returns false if a pivot is not safely positive (rank deficiency).
bool cholesky_upper(int n, const std::vector<double>& A, std::vector<double>& R, double rel_tol) {
  R.assign((size_t)n * n, 0.0);
  double amax = 0.0;
  for (int i = 0; i < n; ++i) amax = std::max(amax, std::fabs(A[(size_t)i * n + i]));
  for (int j = 0; j < n; ++j) {
    double s = A[(size_t)j * n + j];
    for (int k = 0; k < j; ++k) s -= R[(size_t)k * n + j] * R[(size_t)k * n + j];
    if (!(s > rel_tol * amax)) return false;
    const double rjj = std::sqrt(s);
    R[(size_t)j * n + j] = rjj;
    for (int i = j + 1; i < n; ++i) {
      double t = A[(size_t)j * n + i];
      for (int k = 0; k < j; ++k) t -= R[(size_t)k * n + j] * R[(size_t)k * n + i];
      R[(size_t)j * n + i] = t / rjj;
    }
  }
  return true;
}

// Inverse of an upper-triangular matrix (row-major).
void upper_inverse(int n, const std::vector<double>& R, std::vector<double>& Ri) {
  Ri.assign((size_t)n * n, 0.0);
  for (int j = n - 1; j >= 0; --j) {
    Ri[(size_t)j * n + j] = 1.0 / R[(size_t)j * n + j];
    for (int i = j - 1; i >= 0; --i) {
      double s = 0.0;
      for (int k = i + 1; k <= j; ++k) s += R[(size_t)i * n + k] * Ri[(size_t)k * n + j];
      Ri[(size_t)i * n + j] = -s / R[(size_t)i * n + i];
    }
  }
}

}  // namespace msk
