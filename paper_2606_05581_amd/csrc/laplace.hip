// Mesh-based Galerkin basis on the GPU (Sec. 5.1, mesh-based Galerkin basis):
// the K lowest eigenmodes of the cotangent Laplacian with lumped mass,
// L phi = lambda M phi, phi normalised so that Phi^T M Phi = I.
//
// The stiffness and mass are assembled row by row (one thread per vertex,
// its incident triangles in index order, so every run gives the same bits);
// the generalised problem is turned into the symmetric one
// A x = lambda x, A = M^-1/2 L M^-1/2, x = M^1/2 phi, and solved by
// Chebyshev-filtered subspace iteration (Zhou & Saad, "Self-consistent-field
// calculations using Chebyshev-filtered subspace iteration", 2006, with the
// scaled three-term recurrence of their 2007 paper):
//   Y = p_d(A) X           d sparse products, each fused with the recurrence
//                          (d fixed, or per iteration from the Ritz values)
//   Q = orth(Y)            Cholesky QR twice (Gram matrices on the matrix
//                          cores, the small factorisation on the host)
//   H = Q^T A Q, H = Z Theta Z^T (host), X = Q Z   Rayleigh-Ritz
// until every wanted Ritz pair has ||A x - theta x|| <= tol * b, b the
// Gershgorin bound of A. The filter damps [a, b] (a = the block's largest
// Ritz value, which bounds the (m+1)-th eigenvalue from above) and amplifies
// the low end. All blocks are row-major n x m FP64 (row = vertex, in the
// internal vertex order chosen by the caller for locality).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "laplace.h"

namespace msk {

bool sym_eig(int n, std::vector<double>& A, std::vector<double>& evals, std::vector<double>& V);
bool sym_eig_smallest(int n, std::vector<double>& A, int m, std::vector<double>& evals, std::vector<double>& V,
                      double* abs_max);
bool cholesky_upper(int n, const std::vector<double>& A, std::vector<double>& R, double rel_tol);
void upper_inverse(int n, const std::vector<double>& R, std::vector<double>& Ri);

namespace {

// a triangle enters the matrices only if twice its area exceeds this times
// its longest squared edge
constexpr double kDegenerateRel = 1e-12;
// adaptive filter degree: the K-th Ritz value is amplified about this much
// relative to the damped interval per outer iteration (larger gains make the
// filtered block worse conditioned for the Cholesky QR)
constexpr double kAdaptiveGain = 1e3;
// rows a wavefront of the filter step carries at once
constexpr int kFilterRows = 1;
// the step reads each row's neighbour list at once, kFilterBatch entries
// per round (0: the four-entry batches of cheb_step_kernel)
#ifndef MSK_FILTER_BATCH
#define MSK_FILTER_BATCH 8
#endif
constexpr int kFilterBatch = MSK_FILTER_BATCH;

__device__ __forceinline__ int32_t find_col(const int32_t* __restrict__ col, int32_t lo, int32_t hi, int32_t key) {
  while (lo < hi) {
    const int32_t mid = (lo + hi) >> 1;
    if (col[mid] < key)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// Twice the area and the three corner cotangents of triangle (a, b, c), all
// from the triangle's own corner order (so every vertex of it sees the same
// values); false for a degenerate triangle.
__device__ bool tri_cots(const float* __restrict__ P, int32_t ia, int32_t ib, int32_t ic, double cot[3],
                         double& A2) {
  const double ax = P[3 * (int64_t)ia], ay = P[3 * (int64_t)ia + 1], az = P[3 * (int64_t)ia + 2];
  const double bx = P[3 * (int64_t)ib], by = P[3 * (int64_t)ib + 1], bz = P[3 * (int64_t)ib + 2];
  const double cx = P[3 * (int64_t)ic], cy = P[3 * (int64_t)ic + 1], cz = P[3 * (int64_t)ic + 2];
  const double abx = bx - ax, aby = by - ay, abz = bz - az;
  const double acx = cx - ax, acy = cy - ay, acz = cz - az;
  const double bcx = cx - bx, bcy = cy - by, bcz = cz - bz;
  const double nx = aby * acz - abz * acy, ny = abz * acx - abx * acz, nz = abx * acy - aby * acx;
  A2 = sqrt(nx * nx + ny * ny + nz * nz);
  const double l2 = fmax(fmax(abx * abx + aby * aby + abz * abz, bcx * bcx + bcy * bcy + bcz * bcz),
                         acx * acx + acy * acy + acz * acz);
  if (!(A2 > kDegenerateRel * l2)) return false;
  cot[0] = (abx * acx + aby * acy + abz * acz) / A2;     // at a: (b - a).(c - a)
  cot[1] = (bcx * -abx + bcy * -aby + bcz * -abz) / A2;  // at b: (c - b).(a - b)
  cot[2] = (-acx * -bcx + -acy * -bcy + -acz * -bcz) / A2;  // at c: (a - c).(b - c)
  return true;
}

}  // namespace

// Row i of L and m_i (one thread per vertex): every live incident triangle
// with i at corner c adds -cot/2 at the two edges from i (each edge weighted
// by the cotangent of the corner opposite it), their sum to the diagonal and
// a third of its area to the mass. Degenerate triangles are counted once (by
// their first corner).
__global__ void cotan_rows_kernel(const float* __restrict__ P, const int32_t* __restrict__ F,
                                  const int32_t* __restrict__ vt_ptr, const int32_t* __restrict__ vt_tri,
                                  const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col, int64_t nv,
                                  double* __restrict__ val, double* __restrict__ mass,
                                  unsigned long long* __restrict__ skipped) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nv; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t r0 = rowptr[i], r1 = rowptr[i + 1];
    for (int32_t p = r0; p < r1; ++p) val[p] = 0.0;
    const int32_t di = find_col(col, r0, r1, (int32_t)i);
    double m = 0.0, diag = 0.0;
    for (int32_t q = vt_ptr[i]; q < vt_ptr[i + 1]; ++q) {
      const int32_t t = vt_tri[q];
      const int32_t v[3] = {F[3 * (int64_t)t], F[3 * (int64_t)t + 1], F[3 * (int64_t)t + 2]};
      double cot[3], A2;
      const int c = v[0] == i ? 0 : (v[1] == i ? 1 : 2);
      if (!tri_cots(P, v[0], v[1], v[2], cot, A2)) {
        if (c == 0) atomicAdd(skipped, 1ull);
        continue;
      }
      const int c1 = c == 2 ? 0 : c + 1, c2 = c1 == 2 ? 0 : c1 + 1;
      const double w1 = 0.5 * cot[c2];  // edge (i, v[c1]) lies opposite corner c2
      const double w2 = 0.5 * cot[c1];  // edge (i, v[c2]) lies opposite corner c1
      val[find_col(col, r0, r1, v[c1])] -= w1;
      val[find_col(col, r0, r1, v[c2])] -= w2;
      diag += w1 + w2;
      m += A2 / 6.0;
    }
    val[di] += diag;
    mass[i] = m;
  }
}

__global__ void inv_sqrt_mass_kernel(const double* __restrict__ mass, int64_t nv, double* __restrict__ s,
                                     unsigned long long* __restrict__ active) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nv; i += (int64_t)gridDim.x * blockDim.x) {
    const double m = mass[i];
    s[i] = m > 0.0 ? 1.0 / sqrt(m) : 0.0;
    if (m > 0.0) atomicAdd(active, 1ull);
  }
}

// A = S L S in place (S = diag(s)); per-block maximum of the absolute row
// sums (the Gershgorin bound of the spectrum) into bmax[blockIdx.x].
__global__ void __launch_bounds__(256) scale_rows_kernel(const int32_t* __restrict__ rowptr,
                                                         const int32_t* __restrict__ col,
                                                         const double* __restrict__ s, int64_t nv,
                                                         double* __restrict__ val, double* __restrict__ bmax) {
  __shared__ double red[256];
  double best = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nv; i += (int64_t)gridDim.x * blockDim.x) {
    const double si = s[i];
    double sum = 0.0;
    for (int32_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
      const double a = si * val[p] * s[col[p]];
      val[p] = a;
      sum += fabs(a);
    }
    best = fmax(best, sum);
  }
  red[threadIdx.x] = best;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) bmax[blockIdx.x] = red[0];
}

// One step of the filter: Z = alpha (A Y - shift Y) - beta X on 64 C columns
// of blocks with row stride ld, one wavefront per row, each lane holding C
// of the columns (lane_col); beta == 0
// reads no X. With alpha = 1, shift = beta = 0 it is the plain product A Y.
// The rows are dealt to the eight XCDs in contiguous eighths (workgroup b
// runs on XCD b % 8; the grid is a multiple of 8) and swept in order, so the
// neighbour rows a row gathers, close to it in the vertex order, are read
// through the same L2 while still there. X and Z are streamed past the caches (non-temporal), leaving them to
// the gathered rows of Y.
// Lane l's share of a row of m = 64 C doubles: the pairs
// (128 s + 2 l, 128 s + 2 l + 1), s < C / 2, read as 16-byte loads (each
// load instruction covers 1 KB of the row), and for odd C the last 64
// columns as 128 (C / 2) + l.
template <int C>
__device__ __forceinline__ int lane_col(int t, int lane) {
  if (t < 2 * (C / 2)) return 128 * (t >> 1) + 2 * lane + (t & 1);
  return 128 * (C / 2) + lane;
}

template <int C>
__device__ __forceinline__ void load_lane_row(const double* __restrict__ row, int lane, double v[C]) {
#pragma unroll
  for (int s = 0; s < C / 2; ++s) {
    const double2 q = *reinterpret_cast<const double2*>(row + 128 * s + 2 * lane);
    v[2 * s] = q.x;
    v[2 * s + 1] = q.y;
  }
  if constexpr (C % 2 == 1) v[C - 1] = row[128 * (C / 2) + lane];
}

// Non-temporal forms of the same layout: whole 16-byte pairs per lane, so
// each instruction reads or writes 1 KB of the row in full cache lines.
typedef double lap_d2 __attribute__((ext_vector_type(2)));

template <int C>
__device__ __forceinline__ void load_lane_row_nt(const double* __restrict__ row, int lane, double v[C]) {
#pragma unroll
  for (int s = 0; s < C / 2; ++s) {
    const lap_d2 q = __builtin_nontemporal_load(reinterpret_cast<const lap_d2*>(row + 128 * s + 2 * lane));
    v[2 * s] = q.x;
    v[2 * s + 1] = q.y;
  }
  if constexpr (C % 2 == 1) v[C - 1] = __builtin_nontemporal_load(row + 128 * (C / 2) + lane);
}

template <int C>
__device__ __forceinline__ void store_lane_row_nt(double* __restrict__ row, int lane, const double v[C]) {
#pragma unroll
  for (int s = 0; s < C / 2; ++s) {
    const lap_d2 q = {v[2 * s], v[2 * s + 1]};
    __builtin_nontemporal_store(q, reinterpret_cast<lap_d2*>(row + 128 * s + 2 * lane));
  }
  if constexpr (C % 2 == 1) __builtin_nontemporal_store(v[C - 1], row + 128 * (C / 2) + lane);
}

template <int C, int R>
__global__ void __launch_bounds__(256) cheb_step_kernel(const int32_t* __restrict__ rowptr,
                                                        const int32_t* __restrict__ col,
                                                        const double* __restrict__ val, int64_t nv,
                                                        const double* __restrict__ Y, const double* __restrict__ X,
                                                        double* __restrict__ Z, int64_t ld, double alpha,
                                                        double shift, double beta) {
  const int lane = threadIdx.x & 63;
  const int64_t per_xcd = gridDim.x >> 3, xcd = blockIdx.x & 7, j = blockIdx.x >> 3;
  const int64_t chunk = (nv + 7) >> 3;
  const int64_t lo = xcd * chunk, hi = min(nv, lo + chunk);
  // a wavefront takes R consecutive rows and walks their neighbour lists in
  // step, four entries of each row per batch of loads (more reads in flight);
  // each row's products are added in entry order
  for (int64_t i0 = lo + (j * 4 + (threadIdx.x >> 6)) * R; i0 < hi; i0 += per_xcd * 4 * R) {
    int32_t p[R], e[R];
    double acc[R][C];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const bool ok = i0 + r < hi;
      p[r] = ok ? rowptr[i0 + r] : 0;
      e[r] = ok ? rowptr[i0 + r + 1] : 0;
#pragma unroll
      for (int t = 0; t < C; ++t) acc[r][t] = 0.0;
    }
    while (true) {
      bool any = false;
#pragma unroll
      for (int r = 0; r < R; ++r) any |= p[r] < e[r];
      if (!any) break;
      double v[R][4][C], a[R][4];
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int32_t q = p[r] + u;
          if (q < e[r]) {
            a[r][u] = val[q];
            load_lane_row<C>(Y + (int64_t)col[q] * ld, lane, v[r][u]);
          } else {
            a[r][u] = 0.0;
#pragma unroll
            for (int t = 0; t < C; ++t) v[r][u][t] = 0.0;
          }
        }
#pragma unroll
      for (int r = 0; r < R; ++r) {
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int t = 0; t < C; ++t) acc[r][t] += a[r][u] * v[r][u][t];
        p[r] += 4;
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t i = i0 + r;
      if (i >= hi) break;
      double yv[C];
      load_lane_row<C>(Y + i * ld, lane, yv);
      double* zi = Z + i * ld;
      if (beta != 0.0) {
        const double* xi = X + i * ld;
#pragma unroll
        for (int t = 0; t < C; ++t) {
          const int c = lane_col<C>(t, lane);
          __builtin_nontemporal_store(alpha * (acc[r][t] - shift * yv[t]) - beta * __builtin_nontemporal_load(xi + c),
                                      zi + c);
        }
      } else {
#pragma unroll
        for (int t = 0; t < C; ++t) __builtin_nontemporal_store(alpha * (acc[r][t] - shift * yv[t]), zi + lane_col<C>(t, lane));
      }
    }
  }
}

// The same step with the neighbour list of a row read at once: the
// wavefront's lanes k < U load entries p + k of the list, and the gathers of
// all U entries are issued together (lanes take each entry's column index
// and value from lane k), so a row costs three dependent memory round trips
// (row pointers, list, gathered rows) instead of two per four entries. The
// row's own block row and the row of X, which do not depend on the list, are
// read before it. Products are still added in entry order.
template <int C, int U>
__global__ void __launch_bounds__(256) cheb_gather_kernel(const int32_t* __restrict__ rowptr,
                                                          const int32_t* __restrict__ col,
                                                          const double* __restrict__ val, int64_t nv,
                                                          const double* __restrict__ Y, const double* __restrict__ X,
                                                          double* __restrict__ Z, int64_t ld, double alpha,
                                                          double shift, double beta) {
  static_assert(U >= 1 && U <= 64, "a batch holds at most one entry per lane");
  const int lane = threadIdx.x & 63;
  const int64_t per_xcd = gridDim.x >> 3, xcd = blockIdx.x & 7, j = blockIdx.x >> 3;
  const int64_t chunk = (nv + 7) >> 3;
  const int64_t lo = xcd * chunk, hi = min(nv, lo + chunk);
  for (int64_t i = lo + j * 4 + (threadIdx.x >> 6); i < hi; i += per_xcd * 4) {
    const int32_t p0 = rowptr[i], p1 = rowptr[i + 1];
    double yv[C], xv[C];
    load_lane_row<C>(Y + i * ld, lane, yv);
    if (beta != 0.0) load_lane_row_nt<C>(X + i * ld, lane, xv);
    double acc[C];
#pragma unroll
    for (int t = 0; t < C; ++t) acc[t] = 0.0;
    for (int32_t p = p0; p < p1; p += U) {
      const int32_t q = p + lane;
      const bool mine = lane < U && q < p1;
      const int32_t cq = mine ? col[q] : 0;
      const double aq = mine ? val[q] : 0.0;
      double v[U][C];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int32_t cu = __shfl(cq, u);
        if (p + u < p1) {
          load_lane_row<C>(Y + (int64_t)cu * ld, lane, v[u]);
        } else {
#pragma unroll
          for (int t = 0; t < C; ++t) v[u][t] = 0.0;
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const double au = __shfl(aq, u);
#pragma unroll
        for (int t = 0; t < C; ++t) acc[t] += au * v[u][t];
      }
    }
    double zv[C];
#pragma unroll
    for (int t = 0; t < C; ++t)
      zv[t] = beta != 0.0 ? alpha * (acc[t] - shift * yv[t]) - beta * xv[t] : alpha * (acc[t] - shift * yv[t]);
    store_lane_row_nt<C>(Z + i * ld, lane, zv);
  }
}

// Z = Y T, Y n x m, T m x m (row-major), on the matrix cores: a wavefront
// takes 16 rows and sweeps the columns 64 at a time in four 16 x 16 tiles of
// v_mfma_f64_16x16x4 steps over k (operand A: lane l holds Y[row l % 16][k +
// l / 16]; operand B: T[k + l / 16][column l % 16]; accumulator item v of
// lane l is (row 4 v + l / 16, column l % 16)).
typedef double lap_d4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256) rotate_kernel(const double* __restrict__ Y, int64_t n, int32_t m,
                                                     const double* __restrict__ T, double* __restrict__ Z) {
  const int lane = threadIdx.x & 63;
  const int64_t r0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 16;
  if (r0 >= n) return;
  const int rr = lane & 15, kk = lane >> 4;
  const int64_t ra = r0 + rr;
  const bool ok = ra < n;
  const double* yrow = Y + (ok ? ra : r0) * m;
  for (int32_t c0 = 0; c0 < m; c0 += 64) {
    lap_d4 acc[4];
#pragma unroll
    for (int tj = 0; tj < 4; ++tj) acc[tj] = lap_d4{0.0, 0.0, 0.0, 0.0};
    for (int32_t k0 = 0; k0 < m; k0 += 4) {
      const double a = ok ? yrow[k0 + kk] : 0.0;
      const double* trow = T + (int64_t)(k0 + kk) * m + c0 + rr;
#pragma unroll
      for (int tj = 0; tj < 4; ++tj) acc[tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, trow[16 * tj], acc[tj], 0, 0, 0);
    }
#pragma unroll
    for (int tj = 0; tj < 4; ++tj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = r0 + 4 * v + kk;
        if (row < n) Z[row * m + c0 + 16 * tj + rr] = acc[tj][v];
      }
  }
}

// Per-block partial sums of ||AX_j - theta_j X_j||^2 for the columns j < K
// into part[blockIdx.x * K + j]; wavefronts stride over the rows.
template <int C>
__global__ void __launch_bounds__(256) resid_kernel(const double* __restrict__ AX, const double* __restrict__ X,
                                                    const double* __restrict__ theta, int64_t n, int32_t K,
                                                    double* __restrict__ part) {
  constexpr int m = 64 * C;
  __shared__ double red[4][m];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double acc[C], th[C];
#pragma unroll
  for (int t = 0; t < C; ++t) {
    acc[t] = 0.0;
    th[t] = theta[lane + 64 * t];
  }
  for (int64_t i = (int64_t)blockIdx.x * 4 + wave; i < n; i += (int64_t)gridDim.x * 4) {
#pragma unroll
    for (int t = 0; t < C; ++t) {
      const double r = AX[i * m + lane + 64 * t] - th[t] * X[i * m + lane + 64 * t];
      acc[t] += r * r;
    }
  }
#pragma unroll
  for (int t = 0; t < C; ++t) red[wave][lane + 64 * t] = acc[t];
  __syncthreads();
  for (int j = threadIdx.x; j < K; j += 256) part[(int64_t)blockIdx.x * K + j] = red[0][j] + red[1][j] + red[2][j] + red[3][j];
}

// dst[i][0, L) = src[i][0, L) for n x m blocks
__global__ void copy_cols_kernel(const double* __restrict__ src, double* __restrict__ dst, int64_t n, int32_t m,
                                 int32_t L) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * L; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / L, j = e - (e / L) * L;
    dst[i * m + j] = src[i * m + j];
  }
}

// Start block: uniform values in [-1, 1) from a counter hash of (seed, the
// vertex's original index, column), zero on vertices of zero mass, for the
// columns [c0, m).
__global__ void random_block_kernel(double* __restrict__ X, int64_t n, int32_t m, int32_t c0,
                                    const int32_t* __restrict__ orig, const double* __restrict__ s, uint64_t seed) {
  const int64_t w = m - c0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * w; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / w;
    const int32_t j = c0 + (int32_t)(e - i * w);
    // splitmix64 finaliser of the counter
    uint64_t z = seed + 0x9E3779B97F4A7C15ull * ((uint64_t)orig[i] * 0x100000001B3ull + (uint64_t)j + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    const double u = (double)(z >> 11) * (1.0 / 9007199254740992.0);
    X[i * m + j] = s[i] > 0.0 ? 2.0 * u - 1.0 : 0.0;
  }
}

// phi = M^-1/2 x for the first K columns, written in the original vertex
// order: FP64 into phi (optional) and FP32 into the dense basis table
// (rowptr[v] = v K, col = 0..K-1).
__global__ void basis_out_kernel(const double* __restrict__ X, int64_t n, int32_t m, int32_t K,
                                 const int32_t* __restrict__ orig, const double* __restrict__ s,
                                 double* __restrict__ phi, int32_t* __restrict__ rowptr, int32_t* __restrict__ col,
                                 float* __restrict__ tab) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * K; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / K;
    const int32_t j = (int32_t)(e - i * K);
    const int64_t o = (int64_t)orig[i] * K + j;
    const double v = s[i] * X[i * m + j];
    if (phi) phi[o] = v;
    tab[o] = (float)v;
    col[o] = j;
    if (j == 0) rowptr[orig[i]] = (int32_t)(orig[i] * (int64_t)K);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) rowptr[n] = (int32_t)(n * (int64_t)K);
}

namespace {

int grid_of(int64_t n, int64_t per = 256, int64_t cap = 1 << 20) {
  return (int)std::max<int64_t>(1, std::min<int64_t>((n + per - 1) / per, cap));
}

// The step on columns [c0, m) of the n x m blocks (c0 a multiple of 64).
hipError_t cheb_step(const LaplaceJob& J, const double* Y, const double* X, double* Z, double alpha, double shift,
                     double beta, hipStream_t s, int64_t c0 = 0) {
  if (c0 > 0) {
    Y += c0;
    Z += c0;
    if (X) X += c0;
  }
  const int64_t chunk = (J.n + 7) / 8;
  // one group of 4 kFilterRows rows per workgroup: each XCD's workgroups are
  // dispatched in row order, so its rows are swept in order
  const int64_t per = 4 * (kFilterBatch > 0 ? 1 : kFilterRows);
  const int grid = 8 * (int)std::max<int64_t>(1, std::min<int64_t>((chunk + per - 1) / per, 1 << 27));
  const dim3 b(256);
  switch ((J.m - c0) / 64) {
#define LAP_CASE(c)                                                                                            \
  case c:                                                                                                      \
    if constexpr (kFilterBatch > 0)                                                                            \
      hipLaunchKernelGGL((cheb_gather_kernel<c, (kFilterBatch > 0 ? kFilterBatch : 1)>), dim3(grid), b, 0, s,  \
                         J.rowptr, J.col, J.val, J.n, Y, X, Z, J.m, alpha, shift, beta);                       \
    else                                                                                                       \
      hipLaunchKernelGGL((cheb_step_kernel<c, kFilterRows>), dim3(grid), b, 0, s, J.rowptr, J.col, J.val, J.n, \
                         Y, X, Z, J.m, alpha, shift, beta);                                                    \
    break;
    LAP_CASE(1) LAP_CASE(2) LAP_CASE(3) LAP_CASE(4) LAP_CASE(5) LAP_CASE(6) LAP_CASE(7) LAP_CASE(8)
#undef LAP_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t resid(const LaplaceJob& J, const double* AX, const double* X, const double* theta, int32_t K,
                 int grid, double* part, hipStream_t s) {
  switch (J.m / 64) {
#define LAP_CASE(c)                                                                                           \
  case c:                                                                                                     \
    hipLaunchKernelGGL(resid_kernel<c>, dim3(grid), dim3(256), 0, s, AX, X, theta, J.n, K, part);            \
    break;
    LAP_CASE(1) LAP_CASE(2) LAP_CASE(3) LAP_CASE(4) LAP_CASE(5) LAP_CASE(6) LAP_CASE(7) LAP_CASE(8)
#undef LAP_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

struct Timer {
  hipEvent_t a = nullptr, b = nullptr;
  double ms = 0.0;
  hipStream_t s;
  explicit Timer(hipStream_t st) : s(st) {}
  ~Timer() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
  hipError_t init() {
    hipError_t e = hipEventCreate(&a);
    return e != hipSuccess ? e : hipEventCreate(&b);
  }
  hipError_t start() { return hipEventRecord(a, s); }
  hipError_t stop() {
    hipError_t e = hipEventRecord(b, s);
    if (e != hipSuccess) return e;
    e = hipEventSynchronize(b);
    if (e != hipSuccess) return e;
    float t = 0.f;
    e = hipEventElapsedTime(&t, a, b);
    ms += t;
    return e;
  }
};

}  // namespace

#define LAP_TRY(expr)                                          \
  do {                                                         \
    hipError_t e_ = (expr);                                    \
    if (e_ != hipSuccess) {                                    \
      err = std::string(#expr) + ": " + hipGetErrorString(e_); \
      return 3;                                                \
    }                                                          \
  } while (0)

// Gram matrix G = A^T B (m x m, full, from the upper blocks) to the host.
static int gram_to_host(LaplaceJob& J, const double* A, const double* B, std::vector<double>& G, hipStream_t s,
                        std::string& err) {
  const int64_t nblk = psd_blocks(J.m);
  LAP_TRY(launch_fill_u64(J.slots, J.n_slots * nblk * 4096, 0, s));
  LAP_TRY(launch_gram_upper(A, B, J.n, J.m, J.n_slots / 4, J.slots, s));
  LAP_TRY(launch_psd_reduce(J.slots, J.n_slots, J.m, J.m, J.small, s));
  G.resize((size_t)J.m * J.m);
  LAP_TRY(hipMemcpyAsync(G.data(), J.small, sizeof(double) * G.size(), hipMemcpyDeviceToHost, s));
  LAP_TRY(hipStreamSynchronize(s));
  ++J.info.grams;
  return 0;
}

static int rotate(LaplaceJob& J, const double* Y, const std::vector<double>& T, double* Z, hipStream_t s,
                  std::string& err) {
  LAP_TRY(hipMemcpyAsync(J.small, T.data(), sizeof(double) * T.size(), hipMemcpyHostToDevice, s));
  const int64_t waves = (J.n + 15) / 16;
  hipLaunchKernelGGL(rotate_kernel, dim3(grid_of(waves, 4, 1ll << 30)), dim3(256), 0, s, Y, J.n, J.m, J.small, Z);
  LAP_TRY(hipGetLastError());
  LAP_TRY(hipStreamSynchronize(s));  // J.small is reused by the next transfer
  ++J.info.rotates;
  return 0;
}

// Orthonormalise the columns of Y (Cholesky QR: G = Y^T Y = R^T R,
// Y <- Y R^-1) into Z. Columns that the factorisation cannot keep
// (numerically dependent) are dropped by an eigen-decomposition of the
// scaled Gram matrix instead; `rank` returns how many columns remain (the
// rest of Z is zero).
static int orthonormalise(LaplaceJob& J, const double* Y, double* Z, int& rank, hipStream_t s, std::string& err) {
  const int m = (int)J.m;
  std::vector<double> G, R, Ri;
  int rc = gram_to_host(J, Y, Y, G, s, err);
  if (rc) return rc;
  rank = m;
  std::vector<double> T((size_t)m * m, 0.0);
  if (cholesky_upper(m, G, R, 1e-14)) {
    upper_inverse(m, R, Ri);
    T = Ri;
  } else {
    // scaled eigen-decomposition G~ = D G D = U S U^T; T = D U_k S_k^-1/2
    std::vector<double> d(m), Gs((size_t)m * m), ev, U;
    for (int i = 0; i < m; ++i) d[i] = G[(size_t)i * m + i] > 0.0 ? 1.0 / std::sqrt(G[(size_t)i * m + i]) : 0.0;
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) Gs[(size_t)i * m + j] = d[i] * G[(size_t)i * m + j] * d[j];
    if (!sym_eig(m, Gs, ev, U)) {
      err = "eigen-decomposition of the Gram matrix did not converge";
      return 5;
    }
    const double smax = std::max(ev.back(), 0.0);
    int c = 0;
    for (int j = m - 1; j >= 0; --j) {  // largest first
      if (!(ev[j] > 1e-13 * smax)) break;
      const double f = 1.0 / std::sqrt(ev[j]);
      for (int i = 0; i < m; ++i) T[(size_t)i * m + c] = d[i] * U[(size_t)i * m + j] * f;
      ++c;
    }
    rank = c;
    ++J.info.rank_drops;
  }
  return rotate(J, Y, T, Z, s, err);
}

// Returns 0 when converged, 4 when not converged within max_iters (results
// written), 1 on too few vertices of positive mass, 3 on a device error, 5
// on a non-finite operator or a small eigenproblem that did not settle.
int laplace_basis_device(LaplaceJob& J, std::string& err) {
  hipStream_t s = J.stream;
  const int m = (int)J.m, K = (int)J.K;
  Timer t_all(s), t_filter(s), t_dense(s);
  LAP_TRY(t_all.init());
  LAP_TRY(t_filter.init());
  LAP_TRY(t_dense.init());
  LAP_TRY(t_all.start());

  // ---- assembly: L and M, then A = M^-1/2 L M^-1/2 and its bound
  LAP_TRY(launch_fill_u64(J.counters, 2, 0, s));
  hipLaunchKernelGGL(cotan_rows_kernel, dim3(grid_of(J.n)), dim3(256), 0, s, J.P, J.F, J.vt_ptr, J.vt_tri, J.rowptr,
                     J.col, J.n, J.val, J.mass, J.counters);
  LAP_TRY(hipGetLastError());
  hipLaunchKernelGGL(inv_sqrt_mass_kernel, dim3(grid_of(J.n)), dim3(256), 0, s, J.mass, J.n, J.s, J.counters + 1);
  LAP_TRY(hipGetLastError());
  const int gb = grid_of(J.n, 256, 4096);
  hipLaunchKernelGGL(scale_rows_kernel, dim3(gb), dim3(256), 0, s, J.rowptr, J.col, J.s, J.n, J.val, J.small);
  LAP_TRY(hipGetLastError());
  std::vector<double> bm(gb);
  unsigned long long cnt[2];
  LAP_TRY(hipMemcpyAsync(bm.data(), J.small, sizeof(double) * gb, hipMemcpyDeviceToHost, s));
  LAP_TRY(hipMemcpyAsync(cnt, J.counters, sizeof(cnt), hipMemcpyDeviceToHost, s));
  LAP_TRY(hipStreamSynchronize(s));
  double b = 0.0;
  for (double v : bm) b = std::max(b, v);
  J.info.skipped_faces += (int64_t)cnt[0];
  J.info.active_vertices = (int64_t)cnt[1];
  J.info.bound = b;
  {
    float t = 0.f;
    LAP_TRY(hipEventRecord(t_all.b, s));
    LAP_TRY(hipEventSynchronize(t_all.b));
    LAP_TRY(hipEventElapsedTime(&t, t_all.a, t_all.b));
    J.info.assemble_ms = t;
  }
  if (J.info.active_vertices < K) {
    err = "fewer vertices of positive mass than requested modes";
    return 1;
  }
  if (!(b > 0.0) || !std::isfinite(b)) {
    err = "the assembled operator is zero or not finite";
    return 5;
  }

  double* B0 = J.blk[0];
  double* B1 = J.blk[1];
  double* B2 = J.blk[2];
  hipLaunchKernelGGL(random_block_kernel, dim3(grid_of(J.n * m)), dim3(256), 0, s, B0, J.n, m, 0, J.orig, J.s,
                     J.seed);
  LAP_TRY(hipGetLastError());

  std::vector<double> H, theta;
  std::vector<double> part;
  const int rgrid = 1024;
  double* d_part = J.part;
  double a = 0.0;           // lower end of the damped interval, from the last Rayleigh-Ritz
  int rank = m;
  int locked = 0;  // leading columns left out of the filter
  int it = 0;
  bool converged = false;
  double* X = B0;  // current block
  for (; it <= J.max_iters; ++it) {
    double *Y = X, *F1 = (X == B0) ? B1 : B0, *F2 = (X == B2) ? B1 : B2;
    if (it > 0) {
      // Chebyshev filter of degree d on [a, b], scaled at the spectrum's low end aL
      LAP_TRY(t_filter.start());
      const double aL = std::min(0.0, theta.empty() ? 0.0 : theta[0]);
      const double e = 0.5 * (b - a), c = 0.5 * (b + a);
      int degree = J.degree;
      if (degree <= 0) {  // adaptive: C_d((c - theta_K) / e) ~ kAdaptiveGain
        const double tK = (c - theta[K - 1]) / e;
        degree = J.max_degree;
        if (tK > 1.0) degree = (int)std::ceil(std::acosh(kAdaptiveGain) / std::acosh(tK));
        degree = std::max(8, std::min(degree, J.max_degree));
      }
      J.info.last_degree = degree;
      double sig = e / (aL - c);
      const double tau = 2.0 / sig;
      // soft locking: the leading `locked` columns (converged Ritz vectors)
      // are not filtered; they stay in X's buffer, which the steps below
      // touch only in columns [locked, m)
      double *Z0 = X, *Z1 = F1, *Z2 = F2;
      LAP_TRY(cheb_step(J, Z0, nullptr, Z1, sig / e, c, 0.0, s, locked));
      for (int k = 2; k <= degree; ++k) {
        const double sn = 1.0 / (tau - sig);
        LAP_TRY(cheb_step(J, Z1, Z0, Z2, 2.0 * sn / e, c, sig * sn, s, locked));
        sig = sn;
        double* t0 = Z0;
        Z0 = Z1;
        Z1 = Z2;
        Z2 = t0;
      }
      if (locked > 0 && Z1 != X) {
        hipLaunchKernelGGL(copy_cols_kernel, dim3(grid_of(J.n * locked)), dim3(256), 0, s, X, Z1, J.n, m, locked);
        LAP_TRY(hipGetLastError());
      }
      LAP_TRY(t_filter.stop());
      const double w = (double)(m - locked);
      J.info.filter_bytes += (double)degree * (12.0 * J.nnz + 4.0 * (J.n + 1)) +
                             (3.0 * degree - 1.0) * (double)J.n * w * 8.0;
      J.info.spmm_calls += degree;
      Y = Z1;
      F1 = Z0;
      F2 = Z2;
    }
    LAP_TRY(t_dense.start());
    // Y -> Q (twice), into the two free blocks
    int rc = orthonormalise(J, Y, F1, rank, s, err);
    if (rc) return rc;
    int rank2 = rank;
    rc = orthonormalise(J, F1, F2, rank2, s, err);
    if (rc) return rc;
    rank = std::min(rank, rank2);
    double* Qb = F2;
    double* AQ = F1;
    LAP_TRY(cheb_step(J, Qb, nullptr, AQ, 1.0, 0.0, 0.0, s));
    ++J.info.spmm_calls;
    rc = gram_to_host(J, Qb, AQ, H, s, err);
    if (rc) return rc;
    if (rank < m) {  // restrict the projected problem to the kept columns
      for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j)
          if (i >= rank || j >= rank) H[(size_t)i * m + j] = 0.0;
    }
    std::vector<double> Hr((size_t)rank * rank), ev, U;
    for (int i = 0; i < rank; ++i)
      for (int j = 0; j < rank; ++j)
        Hr[(size_t)i * rank + j] = 0.5 * (H[(size_t)i * m + j] + H[(size_t)j * m + i]);
    // all pairs of the projected matrix: eigenvalues by implicit QR, vectors by
    // inverse iteration on the tridiagonal form (faster than accumulating the
    // QR rotations)
    if (!sym_eig_smallest(rank, Hr, rank, ev, U, nullptr)) {
      err = "eigen-decomposition of the projected matrix did not converge";
      return 5;
    }
    theta.assign(m, b);
    for (int j = 0; j < rank; ++j) theta[j] = ev[j];
    std::vector<double> T((size_t)m * m, 0.0);
    for (int i = 0; i < rank; ++i)
      for (int j = 0; j < rank; ++j) T[(size_t)i * m + j] = U[(size_t)i * rank + j];
    double* Xn = Y;  // Y is free once Q exists
    rc = rotate(J, Qb, T, Xn, s, err);
    if (rc) return rc;
    double* AX = AQ;
    LAP_TRY(cheb_step(J, Xn, nullptr, AX, 1.0, 0.0, 0.0, s));
    ++J.info.spmm_calls;
    LAP_TRY(hipMemcpyAsync(J.small, theta.data(), sizeof(double) * m, hipMemcpyHostToDevice, s));
    LAP_TRY(resid(J, AX, Xn, J.small, K, rgrid, d_part, s));
    part.resize((size_t)rgrid * K);
    LAP_TRY(hipMemcpyAsync(part.data(), d_part, sizeof(double) * part.size(), hipMemcpyDeviceToHost, s));
    LAP_TRY(hipStreamSynchronize(s));
    LAP_TRY(t_dense.stop());
    double rmax = 0.0;
    int nconv = 0;  // leading wanted pairs that meet the target
    bool lead = true;
    for (int j = 0; j < K; ++j) {
      double acc = 0.0;
      for (int g = 0; g < rgrid; ++g) acc += part[(size_t)g * K + j];
      const double r = std::sqrt(acc);
      rmax = std::max(rmax, r);
      lead = lead && r <= J.tol * b;
      if (lead) ++nconv;
    }
    locked = (rank == m && J.lock) ? std::min(nconv / 64 * 64, m - 64) : 0;
    J.info.locked = locked;
    X = Xn;
    J.info.max_residual = rmax / b;
    a = theta[rank - 1];
    J.info.filter_lower = a;
    if (rank >= K && rmax <= J.tol * b) {
      converged = true;
      break;
    }
    if (rank < m) {  // refill dropped columns with fresh random vectors
      hipLaunchKernelGGL(random_block_kernel, dim3(grid_of(J.n * (m - rank))), dim3(256), 0, s, X, J.n, m, rank,
                         J.orig, J.s, J.seed + 0x51ED2701ull * (uint64_t)(it + 1));
      LAP_TRY(hipGetLastError());
    }
    if (!(a < b)) {
      err = "the block spans the whole spectrum but the residuals stay above the target";
      break;
    }
  }
  J.info.iters = it;
  J.info.converged = converged ? 1 : 0;
  for (int j = 0; j < K; ++j) J.evals[j] = theta[j];
  hipLaunchKernelGGL(basis_out_kernel, dim3(grid_of(J.n * K)), dim3(256), 0, s, X, J.n, m, K, J.orig, J.s, J.phi,
                     J.out_rowptr, J.out_col, J.out_val);
  LAP_TRY(hipGetLastError());
  LAP_TRY(t_all.stop());
  J.info.filter_ms = t_filter.ms;
  J.info.dense_ms = t_dense.ms;
  J.info.total_ms = t_all.ms;
  return converged ? 0 : 4;
}

}  // namespace msk
