// Dense symmetric eigensolver for the small projected (Rayleigh-Ritz)
// problems of the eigen step, FP64 on the host. Two phases, as stated in
// Golub & Van Loan, "Matrix Computations", ch. 8: Householder reduction of
// A to tridiagonal form T = Q^T A Q, then implicit symmetric QR steps with a
// Wilkinson shift (Givens bulge chase) until T is diagonal, with all
// transforms accumulated into the eigenvector matrix.
#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <cstdint>
#include <cfloat>
#include <cmath>
#include <functional>
#include <mutex>
#include <numeric>
#include <thread>
#include <vector>

namespace msk {

namespace {

// A small persistent pool of host threads for the O(n^3) loops of the
// projected eigenproblem (rows or vectors are independent); the caller is
// worker 0. Workers spin briefly on the job counter before they sleep, so
// the many short parallel loops of one factorisation are cheap to start.
// Calls from several host threads are serialised.
class HostPool {
 public:
  HostPool() {
    const unsigned hc = std::thread::hardware_concurrency();
    n_ = (int)std::max(1u, std::min(16u, hc ? hc : 1u));
    for (int i = 1; i < n_; ++i) th_.emplace_back([this, i] { worker(i); });
  }
  ~HostPool() {
    {
      std::lock_guard<std::mutex> lk(m_);
      stop_.store(true);
      gen_.fetch_add(1);
    }
    cv_.notify_all();
    for (auto& t : th_) t.join();
  }
  int size() const { return n_; }
  // f(w) for w = 0..size()-1, one per worker; returns when all are done
  void run(const std::function<void(int)>& f) {
    std::lock_guard<std::mutex> serial(run_m_);
    if (n_ == 1) {
      f(0);
      return;
    }
    job_ = &f;
    pending_.store(n_ - 1);
    {
      std::lock_guard<std::mutex> lk(m_);
      gen_.fetch_add(1);
    }
    cv_.notify_all();
    f(0);
    while (pending_.load() != 0) std::this_thread::yield();
  }

 private:
  void worker(int id) {
    uint64_t seen = 0;
    while (true) {
      // spin for a while, then sleep until the next job
      for (int k = 0; k < 20000 && gen_.load() == seen; ++k) std::this_thread::yield();
      if (gen_.load() == seen) {
        std::unique_lock<std::mutex> lk(m_);
        cv_.wait(lk, [&] { return gen_.load() != seen; });
      }
      seen = gen_.load();
      if (stop_.load()) return;
      (*job_)(id);
      pending_.fetch_sub(1);
    }
  }
  int n_ = 1;
  std::vector<std::thread> th_;
  std::mutex m_, run_m_;
  std::condition_variable cv_;
  const std::function<void(int)>* job_ = nullptr;
  std::atomic<uint64_t> gen_{0};
  std::atomic<int> pending_{0};
  std::atomic<bool> stop_{false};
};

HostPool& host_pool() {
  static HostPool pool;
  return pool;
}

// body(lo, hi) over [0, n) split across the pool (serially when n is small)
void parallel_rows(int n, int min_per_worker, const std::function<void(int, int)>& body) {
  HostPool& P = host_pool();
  const int w = std::max(1, std::min(P.size(), n / std::max(1, min_per_worker)));
  if (w <= 1) {
    body(0, n);
    return;
  }
  P.run([&](int id) {
    if (id >= w) return;
    const int lo = (int)((int64_t)n * id / w), hi = (int)((int64_t)n * (id + 1) / w);
    if (lo < hi) body(lo, hi);
  });
}

// In place: A (n x n, row-major, symmetric) -> tridiagonal (diag d, off e,
// e[i] couples i and i+1) with A = Q T Q^T. With `accumulate`, Q is formed
// explicitly; otherwise the reflectors are kept (reflector k acts on indices
// k+1..n-1: v = (1, H[k][k+2..n-1]) in row k of H, scale beta[k]).
void tridiagonalise(int n, std::vector<double>& A, std::vector<double>& Q, std::vector<double>& d,
                    std::vector<double>& e, bool accumulate = true, std::vector<double>* H = nullptr,
                    std::vector<double>* betas = nullptr) {
  auto a = [&](int i, int j) -> double& { return A[(size_t)i * n + j]; };
  if (accumulate) {
    Q.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) Q[(size_t)i * n + i] = 1.0;
  } else {
    H->assign((size_t)n * n, 0.0);
    betas->assign(n, 0.0);
  }
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
    parallel_rows(m, 64, [&](int lo, int hi) {
      for (int i = lo; i < hi; ++i) {
        const double* row = &A[(size_t)(k + 1 + i) * n + (k + 1)];
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
        int j = 0;
        for (; j + 3 < m; j += 4) {
          s0 += row[j] * v[j];
          s1 += row[j + 1] * v[j + 1];
          s2 += row[j + 2] * v[j + 2];
          s3 += row[j + 3] * v[j + 3];
        }
        for (; j < m; ++j) s0 += row[j] * v[j];
        p[i] = beta * ((s0 + s1) + (s2 + s3));
      }
    });
    double pv = 0.0;
    for (int i = 0; i < m; ++i) pv += p[i] * v[i];
    const double half = 0.5 * beta * pv;
    for (int i = 0; i < m; ++i) w[i] = p[i] - half * v[i];
    // A22 -= v w^T + w v^T ; column k becomes mu e1
    parallel_rows(m, 64, [&](int lo, int hi) {
      for (int i = lo; i < hi; ++i) {
        double* row = &A[(size_t)(k + 1 + i) * n + (k + 1)];
        const double vi = v[i], wi = w[i];
        for (int j = 0; j < m; ++j) row[j] -= vi * w[j] + wi * v[j];
      }
    });
    a(k + 1, k) = a(k, k + 1) = mu;
    for (int i = 1; i < m; ++i) a(k + 1 + i, k) = a(k, k + 1 + i) = 0.0;
    if (!accumulate) {
      (*betas)[k] = beta;
      for (int i = 1; i < m; ++i) (*H)[(size_t)k * n + k + 1 + i] = v[i];
      continue;
    }
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
    if (Q.empty()) continue;
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

namespace {

// Numbers of eigenvalues of the symmetric tridiagonal (d, e) below each of
// B points x: the negative pivots of the LDL^T factorisation of T - x I
// (Sylvester's law of inertia; Golub & Van Loan 8.4.1), e2[i] = e[i]^2, a
// pivot smaller than pivmin in magnitude replaced by -pivmin. The B
// recurrences are independent; interleaving them hides the divisions'
// latency.
template <int B>
void sturm_counts(int n, const double* d, const double* e2, const double* x, double pivmin, int* c) {
  double q[B];
  for (int b = 0; b < B; ++b) {
    q[b] = d[0] - x[b];
    if (std::fabs(q[b]) < pivmin) q[b] = -pivmin;
    c[b] = q[b] < 0.0;
  }
  for (int i = 1; i < n; ++i) {
    for (int b = 0; b < B; ++b) {
      q[b] = (d[i] - x[b]) - e2[i - 1] / q[b];
      if (std::fabs(q[b]) < pivmin) q[b] = -pivmin;
      c[b] += q[b] < 0.0;
    }
  }
}

// The m smallest eigenvalues of the symmetric tridiagonal (d, e), ascending,
// and the largest, each by bisection on the Sturm count inside the
// Gershgorin interval to an absolute width of 4 eps |T| (eigenvalues are
// independent: four bisections advance together, groups are pool tasks).
}  // namespace

// The bisection's set-up: e2[i] = e[i]^2, the widened Gershgorin interval
// [glo, ghi], the pivot floor and the absolute width at which it stops.
void bisect_setup(int n, const std::vector<double>& d, const std::vector<double>& e, std::vector<double>& e2,
                  double& glo, double& ghi, double& pivmin, double& atol) {
  e2.assign(std::max(n - 1, 1), 0.0);
  glo = INFINITY;
  ghi = -INFINITY;
  double emax2 = 0.0;
  for (int i = 0; i < n; ++i) {
    const double r = (i > 0 ? std::fabs(e[i - 1]) : 0.0) + (i + 1 < n ? std::fabs(e[i]) : 0.0);
    glo = std::min(glo, d[i] - r);
    ghi = std::max(ghi, d[i] + r);
    if (i + 1 < n) {
      e2[i] = e[i] * e[i];
      emax2 = std::max(emax2, e2[i]);
    }
  }
  const double tnorm = std::max(std::fabs(glo), std::fabs(ghi));
  const double eps = std::ldexp(1.0, -52);
  pivmin = DBL_MIN * std::max(1.0, emax2);
  atol = 4.0 * eps * std::max(tnorm, DBL_MIN);
  glo -= 2.0 * atol + pivmin;
  ghi += 2.0 * atol + pivmin;
}

namespace {

void tridiag_smallest(int n, const std::vector<double>& d, const std::vector<double>& e, int m,
                      std::vector<double>& out, double& largest) {
  std::vector<double> e2;
  double glo, ghi, pivmin, atol;
  bisect_setup(n, d, e, e2, glo, ghi, pivmin, atol);
  // targets: indices 0..m-1 and n-1 (the largest), in groups of four
  std::vector<int> idx(m + 1);
  for (int j = 0; j < m; ++j) idx[j] = j;
  idx[m] = n - 1;
  std::vector<double> val(m + 1, 0.0);
  constexpr int kB = 4;
  const int groups = (m + 1 + kB - 1) / kB;
  parallel_rows(groups, 1, [&](int g0, int g1) {
    for (int g = g0; g < g1; ++g) {
      double lo[kB], hi[kB], mid[kB];
      int j[kB], c[kB];
      for (int b = 0; b < kB; ++b) {
        const int t = std::min(g * kB + b, m);  // a short last group repeats the last target
        j[b] = idx[t];
        lo[b] = glo;
        hi[b] = ghi;
      }
      for (int it = 0; it < 200; ++it) {
        bool open = false;
        for (int b = 0; b < kB; ++b) {
          mid[b] = 0.5 * (lo[b] + hi[b]);
          open = open || hi[b] - lo[b] > atol;
        }
        if (!open) break;
        sturm_counts<kB>(n, d.data(), e2.data(), mid, pivmin, c);
        for (int b = 0; b < kB; ++b) {
          if (!(hi[b] - lo[b] > atol)) continue;
          if (c[b] <= j[b])
            lo[b] = mid[b];
          else
            hi[b] = mid[b];
        }
      }
      for (int b = 0; b < kB; ++b)
        if (g * kB + b <= m) val[g * kB + b] = 0.5 * (lo[b] + hi[b]);
    }
  });
  out.assign(val.begin(), val.begin() + m);
  largest = val[m];
  std::sort(out.begin(), out.end());
}

// LU factorisation with partial pivoting of the tridiagonal T - sigma I
// (Golub & Van Loan 4.3.4): row i of U holds u0 (diagonal), u1, u2; l[i] and
// swap[i] record the elimination of row i + 1. Zero pivots are replaced by
// `tiny` (inverse iteration only needs a direction).
struct TriLU {
  std::vector<double> u0, u1, u2, l;
  std::vector<char> swap;
};

void tridiag_lu(int n, const std::vector<double>& d, const std::vector<double>& e, double sigma, double tiny,
                TriLU& f) {
  f.u0.assign(n, 0.0);
  f.u1.assign(n, 0.0);
  f.u2.assign(n, 0.0);
  f.l.assign(n, 0.0);
  f.swap.assign(n, 0);
  double r0 = d[0] - sigma, r1 = n > 1 ? e[0] : 0.0, r2 = 0.0;
  for (int i = 0; i + 1 < n; ++i) {
    const double n0 = e[i], n1 = d[i + 1] - sigma, n2 = i + 2 < n ? e[i + 1] : 0.0;
    double m0, m1;
    if (std::fabs(n0) > std::fabs(r0)) {
      f.swap[i] = 1;
      f.u0[i] = n0; f.u1[i] = n1; f.u2[i] = n2;
      const double mult = r0 / n0;
      f.l[i] = mult;
      m0 = r1 - mult * n1;
      m1 = r2 - mult * n2;
    } else {
      if (r0 == 0.0) r0 = tiny;
      f.u0[i] = r0; f.u1[i] = r1; f.u2[i] = r2;
      const double mult = n0 / r0;
      f.l[i] = mult;
      m0 = n1 - mult * r1;
      m1 = n2 - mult * r2;
    }
    r0 = m0;
    r1 = m1;
    r2 = 0.0;
  }
  f.u0[n - 1] = r0 == 0.0 ? tiny : r0;
}

void tridiag_solve(int n, const TriLU& f, std::vector<double>& y) {
  for (int i = 0; i + 1 < n; ++i) {
    if (f.swap[i]) std::swap(y[i], y[i + 1]);
    y[i + 1] -= f.l[i] * y[i];
  }
  for (int i = n - 1; i >= 0; --i) {
    double t = y[i];
    if (i + 1 < n) t -= f.u1[i] * y[i + 1];
    if (i + 2 < n) t -= f.u2[i] * y[i + 2];
    y[i] = t / f.u0[i];
  }
}

}  // namespace

bool tridiag_vectors(int n, const std::vector<double>& d, const std::vector<double>& e,
                     const std::vector<double>& evals, std::vector<double>& Xc);

// The m smallest eigenpairs of the symmetric tridiagonal (d, e): the
// eigenvalues by Sturm-count bisection (ascending), the vectors by inverse
// iteration (with Gram-Schmidt inside clusters of close eigenvalues, as in
// LAPACK's xSTEIN), vector j at Xc[j n .. j n + n); abs_max (optional)
// receives the largest eigenvalue magnitude.
bool tridiag_smallest_pairs(int n, const std::vector<double>& d, const std::vector<double>& e, int m,
                            std::vector<double>& evals, std::vector<double>& Xc, double* abs_max) {
  if (m > n) m = n;
  double largest = 0.0;
  tridiag_smallest(n, d, e, m, evals, largest);
  if (abs_max) *abs_max = std::max(std::fabs(evals.front()), std::fabs(largest));
  return tridiag_vectors(n, d, e, evals, Xc);
}

// Eigenvectors of the symmetric tridiagonal (d, e) for the ascending
// eigenvalues evals, by inverse iteration, vector j at Xc[j n .. j n + n).
bool tridiag_vectors(int n, const std::vector<double>& d, const std::vector<double>& e,
                     const std::vector<double>& evals, std::vector<double>& Xc) {
  const int m = (int)evals.size();
  double tnorm = 0.0;
  for (int i = 0; i < n; ++i)
    tnorm = std::max(tnorm, std::fabs(d[i]) + (i > 0 ? std::fabs(e[i - 1]) : 0.0) + (i + 1 < n ? std::fabs(e[i]) : 0.0));
  if (tnorm == 0.0) tnorm = 1.0;
  const double eps = std::ldexp(1.0, -52);
  // eigenvalues closer than ortol form a cluster, whose vectors are kept
  // orthogonal by Gram-Schmidt. Outside a cluster, inverse iteration from
  // shifts accurate to about eps |T| leaves a neighbour at gap g >= ortol a
  // component of about eps |T| / g <= 2.2e-10 per step, so the vectors come
  // out orthogonal to that level without it. (LAPACK's xSTEIN takes
  // 1e-3 |T|, which on the densely spaced low end of a Steklov spectrum
  // makes the whole requested range one cluster and the work k^2 n.)
  const double ortol = 1e-6 * tnorm;
  Xc.assign((size_t)n * m, 0.0);  // eigenvectors of T, vector j at Xc[j * n + r]
  // clusters [cs[c], cs[c + 1]): independent of each other, so they are pool
  // tasks; each vector's pseudo-random start depends on its index only
  std::vector<int> cs(1, 0);
  for (int j = 1; j < m; ++j)
    if (evals[j] - evals[j - 1] > ortol) cs.push_back(j);
  cs.push_back(m);
  const int ncl = (int)cs.size() - 1;
  std::atomic<bool> good{true};
  parallel_rows(ncl, 1, [&](int c0, int c1) {
    std::vector<double> y(n), x(n), dots;
    TriLU f;
    for (int cl = c0; cl < c1 && good.load(); ++cl) {
      const int cluster_start = cs[cl];
      double sigma_prev = 0.0;
      for (int j = cluster_start; j < cs[cl + 1]; ++j) {
        // separate equal shifts inside a cluster slightly
        double sigma = evals[j];
        if (j > cluster_start && sigma <= sigma_prev + 10.0 * eps * tnorm) sigma = sigma_prev + 10.0 * eps * tnorm;
        sigma_prev = sigma;
        tridiag_lu(n, d, e, sigma, eps * tnorm, f);
        uint64_t seed = 0x9E3779B97F4A7C15ull * (uint64_t)(j + 1) + 0xD1B54A32D192ED03ull;
        for (int r = 0; r < n; ++r) {  // pseudo-random start (xorshift)
          seed ^= seed << 13; seed ^= seed >> 7; seed ^= seed << 17;
          y[r] = (double)(seed >> 11) * 0x1p-53 - 0.5;
        }
        for (int it = 0; it < 4; ++it) {
          x = y;
          tridiag_solve(n, f, x);
          // classical Gram-Schmidt against the cluster's earlier vectors, twice
          const int nc = j - cluster_start;
          for (int pass = 0; pass < 2 && nc > 0; ++pass) {
            dots.assign(nc, 0.0);
            for (int i = 0; i < nc; ++i) {
              const double* xi = &Xc[(size_t)(cluster_start + i) * n];
              double s0 = 0.0, s1 = 0.0;
              int r = 0;
              for (; r + 1 < n; r += 2) {
                s0 += xi[r] * x[r];
                s1 += xi[r + 1] * x[r + 1];
              }
              for (; r < n; ++r) s0 += xi[r] * x[r];
              dots[i] = s0 + s1;
            }
            for (int i = 0; i < nc; ++i) {
              const double* xi = &Xc[(size_t)(cluster_start + i) * n];
              const double dt = dots[i];
              for (int r = 0; r < n; ++r) x[r] -= dt * xi[r];
            }
          }
          double nrm = 0.0;
          for (double t : x) nrm += t * t;
          nrm = std::sqrt(nrm);
          if (!(nrm > 0.0) || !std::isfinite(nrm)) {
            good.store(false);
            return;
          }
          for (int r = 0; r < n; ++r) y[r] = x[r] / nrm;
        }
        std::copy(y.begin(), y.end(), Xc.begin() + (size_t)j * n);
      }
    }
  });
  return good.load();
}

// The m smallest eigenpairs of a symmetric A (n x n, row-major; destroyed):
// Householder tridiagonalisation, the tridiagonal's m smallest pairs, then
// back through the reflectors. evals ascending; V is n x m row-major;
// abs_max (optional) receives the largest eigenvalue magnitude.
bool sym_eig_smallest(int n, std::vector<double>& A, int m, std::vector<double>& evals, std::vector<double>& V,
                      double* abs_max) {
  if (m > n) m = n;
  std::vector<double> d, e, Qdummy, H, betas, Xc;
  tridiagonalise(n, A, Qdummy, d, e, false, &H, &betas);
  if (!tridiag_smallest_pairs(n, d, e, m, evals, Xc, abs_max)) return false;
  // back-transform each vector: H_0 H_1 ... H_{n-3} x (last reflector first),
  // four vectors at a time: each reflector is read once per four, and the
  // four dot products are independent chains (every vector still sees the
  // same operations in the same order)
  auto apply4 = [&](double* x0, double* x1, double* x2, double* x3) {
    for (int k = n - 3; k >= 0; --k) {
      const double beta = betas[k];
      if (beta == 0.0) continue;
      const double* v = &H[(size_t)k * n];  // v[k+1] = 1, v[k+2..] stored
      double s0 = x0[k + 1], s1 = x1[k + 1], s2 = x2[k + 1], s3 = x3[k + 1];
      for (int r = k + 2; r < n; ++r) {
        const double vr = v[r];
        s0 += vr * x0[r];
        s1 += vr * x1[r];
        s2 += vr * x2[r];
        s3 += vr * x3[r];
      }
      s0 *= beta; s1 *= beta; s2 *= beta; s3 *= beta;
      x0[k + 1] -= s0; x1[k + 1] -= s1; x2[k + 1] -= s2; x3[k + 1] -= s3;
      for (int r = k + 2; r < n; ++r) {
        const double vr = v[r];
        x0[r] -= vr * s0;
        x1[r] -= vr * s1;
        x2[r] -= vr * s2;
        x3[r] -= vr * s3;
      }
    }
  };
  std::vector<double> spare((size_t)3 * n, 0.0);  // stand-ins for a short last group
  parallel_rows((m + 3) / 4, 1, [&](int g0, int g1) {
    for (int g = g0; g < g1; ++g) {
      double* xs[4];
      for (int b = 0; b < 4; ++b) xs[b] = 4 * g + b < m ? &Xc[(size_t)(4 * g + b) * n] : &spare[(size_t)(b - 1) * n];
      apply4(xs[0], xs[1], xs[2], xs[3]);
    }
  });
  std::vector<double> X((size_t)n * m);
  for (int j = 0; j < m; ++j)
    for (int r = 0; r < n; ++r) X[(size_t)r * m + j] = Xc[(size_t)j * n + r];
  V.swap(X);
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
