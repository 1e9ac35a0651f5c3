// PSD estimator (Sec. 3.2, Alg. 2): the rank-one updates of a run of walks
// from tangent balls, summed into a dense K x K matrix.
//
// Per antithetic pair p of row i (sample s_i, weight w_i, tangent-ball
// radius r_i) with walks ending at t_1, t_2, the boxed estimator with s
// stratified over rows and z drawn in proportion to the ball jump kernel
// gives X_p = alpha_i (d_1 d_1^T + d_2 d_2^T) / 2, d = b(s_i) - b(t),
// alpha_i = w_i Z_i / (2 P), Z_i the kernel's mass outside the cap. The sums
// S = sum_p X_p and Q = sum_p X_p * X_p (elementwise, for standard errors)
// are symmetric rank-k updates S += U^T U, Q += V^T V over rows
//   U: sqrt(alpha/2) d_1, sqrt(alpha/2) d_2;
//   V: (alpha/2) d_1*d_1, (alpha/2) d_2*d_2, sqrt(2) (alpha/2) d_1*d_2,
// so each chunk of pairs is gathered into U and V (HBM-bound) and handed to
// a dense FP64 product on the matrix cores.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "msk_internal.h"

namespace msk {

namespace {

inline int grid_for(int64_t n, int bs) { return (int)std::min<int64_t>((n + bs - 1) / bs, 1 << 20); }

// Dense per-vertex table (n_verts x K, zeroed beforehand) from the CSR basis.
__global__ void dense_table_kernel(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                                   const float* __restrict__ val, int64_t nv, int64_t K, double* __restrict__ tab) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += (int64_t)gridDim.x * blockDim.x)
    for (int32_t e = rowptr[v]; e < rowptr[v + 1]; ++e) tab[v * K + col[e]] = (double)val[e];
}

// One workgroup per pair of the chunk [q0, q0 + nq); threads over columns.
__global__ void __launch_bounds__(256) psd_gather_kernel(PsdGather G, int64_t q0, int64_t nq, double* __restrict__ U,
                                                         double* __restrict__ V) {
  const int64_t K = G.K;
  for (int64_t qq = blockIdx.x; qq < nq; qq += gridDim.x) {
    const int64_t q = q0 + qq;
    const int64_t i = q / G.pairs;
    const int64_t j = q - i * G.pairs;
    const double r = (double)G.radius[i];
    const double alpha = r > 0.0 ? G.w[i] * (1.0 / (2.0 * r)) * (1.0 / G.u0 - 1.0) / (2.0 * (double)G.pairs) : 0.0;
    // sample: face and barycentrics of s_i
    const int32_t* fs = G.faces + 3 * (int64_t)G.tri[i];
    const double ls[3] = {G.bary[3 * i], G.bary[3 * i + 1], G.bary[3 * i + 2]};
    // terminal points of the two walks (log: status, triangle, barycentrics of vertices 1 and 2)
    int32_t ft[2][3];
    double lt[2][3];
    for (int a = 0; a < 2; ++a) {
      const int64_t li = i * 2 * G.pairs + 2 * j + a;
      const int32_t st = G.log_status[li], t = G.log_tri[li];
      const bool has_t = st >= 0 && st != kEscaped && t >= 0;
      const double l1 = has_t ? (double)G.log_bary[2 * li] : 0.0, l2 = has_t ? (double)G.log_bary[2 * li + 1] : 0.0;
      lt[a][0] = has_t ? (1.0 - l1) - l2 : 0.0;
      lt[a][1] = l1;
      lt[a][2] = l2;
      for (int c = 0; c < 3; ++c) ft[a][c] = has_t ? G.faces[3 * (int64_t)t + c] : 0;
    }
    const double su = sqrt(0.5 * alpha), sv = 0.5 * alpha, sv2 = sqrt(2.0) * 0.5 * alpha;
    double* u = U + 2 * qq * K;
    double* v = V + 3 * qq * K;
    for (int64_t k = threadIdx.x; k < K; k += blockDim.x) {
      const double bs = ls[0] * G.tab[fs[0] * K + k] + ls[1] * G.tab[fs[1] * K + k] + ls[2] * G.tab[fs[2] * K + k];
      const double b1 = lt[0][0] * G.tab[ft[0][0] * K + k] + lt[0][1] * G.tab[ft[0][1] * K + k] +
                        lt[0][2] * G.tab[ft[0][2] * K + k];
      const double b2 = lt[1][0] * G.tab[ft[1][0] * K + k] + lt[1][1] * G.tab[ft[1][1] * K + k] +
                        lt[1][2] * G.tab[ft[1][2] * K + k];
      const double d1 = bs - b1, d2 = bs - b2;
      u[k] = su * d1;
      u[K + k] = su * d2;
      v[k] = sv * d1 * d1;
      v[K + k] = sv * d2 * d2;
      v[2 * K + k] = sv2 * d1 * d2;
    }
  }
}

// Lower triangle from the upper one (column-major K x K from the symmetric
// rank-k updates), then the standard error of every entry:
// se^2 = (n Q - S^2) / (n - 1) over n pair terms.
__global__ void psd_finish_kernel(double* __restrict__ S, double* __restrict__ Q, int64_t K, double n_pairs,
                                  double* __restrict__ se) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < K * K; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = e % K, colm = e / K;  // column-major: element (row, colm)
    const int64_t src = row <= colm ? e : colm + row * K;
    const double s = S[src], q = Q[src];
    se[e] = sqrt(fmax(0.0, n_pairs * q - s * s) / (n_pairs - 1.0));
    if (row > colm) {
      S[e] = s;
      Q[e] = q;
    }
  }
}

}  // namespace

hipError_t launch_dense_table(const int32_t* rowptr, const int32_t* col, const float* val, int64_t nv, int64_t K,
                              double* tab, hipStream_t s) {
  if (nv <= 0) return hipSuccess;
  hipLaunchKernelGGL(dense_table_kernel, dim3(grid_for(nv, 256)), dim3(256), 0, s, rowptr, col, val, nv, K, tab);
  return hipGetLastError();
}

hipError_t launch_psd_gather(const PsdGather& G, int64_t q0, int64_t nq, double* U, double* V, hipStream_t s) {
  if (nq <= 0) return hipSuccess;
  const int threads = G.K >= 256 ? 256 : (G.K >= 128 ? 128 : 64);
  hipLaunchKernelGGL(psd_gather_kernel, dim3((unsigned)std::min<int64_t>(nq, 1 << 20)), dim3(threads), 0, s, G, q0,
                     nq, U, V);
  return hipGetLastError();
}

hipError_t launch_psd_finish(double* S, double* Q, int64_t K, double n_pairs, double* se, hipStream_t s) {
  hipLaunchKernelGGL(psd_finish_kernel, dim3(grid_for(K * K, 256)), dim3(256), 0, s, S, Q, K, n_pairs, se);
  return hipGetLastError();
}

}  // namespace msk
