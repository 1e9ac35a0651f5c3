// Eigen step of the estimator: smallest Steklov eigenpairs of the
// symmetrised, mass-scaled estimate C = M^-1/2 (S + S^T)/2 M^-1/2 (Alg. 1's
// symmetrisation; Sec. 2 eq. steklov-eigenproblem) by a thick-restarted
// block Krylov (block Lanczos) Rayleigh-Ritz method:
//   - products with C in FP32 on the matrix cores (C stored in FP32),
//   - basis kept in FP64 with full re-orthogonalisation (classical
//     Gram-Schmidt twice + Cholesky QR) on the GPU,
//   - the small projected problem solved in FP64 on the host,
//   - final Rayleigh quotients and residuals with C in FP64.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include "msk_internal.h"
#include "eigen.h"
#include "philox.h"

namespace msk {

bool sym_eig(int n, std::vector<double>& A, std::vector<double>& evals, std::vector<double>& V);
bool sym_eig_smallest(int n, std::vector<double>& A, int m, std::vector<double>& evals, std::vector<double>& V,
                      double* abs_max);
bool cholesky_upper(int n, const std::vector<double>& A, std::vector<double>& R, double rel_tol);
void upper_inverse(int n, const std::vector<double>& R, std::vector<double>& Ri);
bool tridiag_smallest_pairs(int n, const std::vector<double>& d, const std::vector<double>& e, int m,
                            std::vector<double>& evals, std::vector<double>& Xc, double* abs_max);
void bisect_setup(int n, const std::vector<double>& d, const std::vector<double>& e, std::vector<double>& e2,
                  double& glo, double& ghi, double& pivmin, double& atol);
bool tridiag_vectors(int n, const std::vector<double>& d, const std::vector<double>& e,
                     const std::vector<double>& evals, std::vector<double>& Xc);

// ------------------------------------------------------------- kernels

// C[a][b] = 1/2 (S[ka][kb] + S[kb][ka]) m[a] m[b] over the kept rows.
__global__ void assemble_c_kernel(const double* __restrict__ S, int64_t ldS, const int32_t* __restrict__ keep,
                                  const double* __restrict__ m, int64_t n, double* C64, float* C32) {
  const int64_t total = n * n;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t a = idx / n, b = idx - a * n;
    const int64_t ka = keep[a], kb = keep[b];
    const double v = 0.5 * (S[ka * ldS + kb] + S[kb * ldS + ka]) * m[a] * m[b];
    C64[idx] = v;
    C32[idx] = (float)v;
  }
}

__global__ void f64_to_f32_kernel(const double* __restrict__ x, float* y, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (float)x[i];
}

// y[r * ldy + c] = x[r * ldx + c] for an r x c sub-block (strided copies, FP32 -> FP64)
__global__ void copy_block_f32_to_f64_kernel(const float* __restrict__ x, int64_t ldx, double* y, int64_t ldy,
                                             int64_t rows, int64_t cols) {
  const int64_t total = rows * cols;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / cols, c = i - r * cols;
    y[r * ldy + c] = (double)x[r * ldx + c];
  }
}

__global__ void copy_block_f64_kernel(const double* __restrict__ x, int64_t ldx, double* y, int64_t ldy, int64_t rows,
                                      int64_t cols) {
  const int64_t total = rows * cols;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / cols, c = i - r * cols;
    y[r * ldy + c] = x[r * ldx + c];
  }
}

__global__ void copy_block_f64_to_f32_kernel(const double* __restrict__ x, int64_t ldx, float* y, int64_t ldy,
                                             int64_t rows, int64_t cols) {
  const int64_t total = rows * cols;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / cols, c = i - r * cols;
    y[r * ldy + c] = (float)x[r * ldx + c];
  }
}

// Row-major GEMM on the matrix cores: C = alpha op(A) op(B) + beta C, op(A)
// M x K, op(B) K x N; A is M x K (lda) or, transposed, K x M; B is K x N
// (ldb) or N x K. A 256-thread workgroup computes a 64 x 64 tile: each
// wavefront a 32 x 32 quarter as 2 x 2 blocks of the 16 x 16 x 4 MFMA (FP64
// or FP32, accumulating in the same precision), K in steps of 16 staged
// through LDS. The K range may be split over blockIdx.z (the long inner
// dimension of the Gram products Q^T X): each slice then writes its partial
// tile to `part` (splits x M x N) and splitk_reduce_kernel sums them in a
// fixed order.
typedef double mfma_d4 __attribute__((ext_vector_type(4)));
typedef float mfma_f4 __attribute__((ext_vector_type(4)));
template <typename T>
struct Mfma;
// Operands: lane l holds A[l % 16][l / 16] and B[l / 16][l % 16]. Results:
// accumulator item e of lane l is column l % 16 and row 4 e + l / 16 (FP64)
// or row 4 (l / 16) + e (FP32) of the 16 x 16 block (measured on gfx950).
template <>
struct Mfma<double> {
  typedef mfma_d4 V;
  __device__ static V step(double a, double b, V c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  __device__ static int row(int lane, int e) { return 4 * e + (lane >> 4); }
};
template <>
struct Mfma<float> {
  typedef mfma_f4 V;
  __device__ static V step(float a, float b, V c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  __device__ static int row(int lane, int e) { return 4 * (lane >> 4) + e; }
};

template <typename T, bool TA, bool TB>
__global__ void __launch_bounds__(256) gemm_kernel(int64_t M, int64_t N, int64_t K, int64_t kchunk, T alpha,
                                                   const T* __restrict__ A, int64_t lda, const T* __restrict__ B,
                                                   int64_t ldb, T beta, T* Cm, int64_t ldc, T* __restrict__ part) {
  constexpr int BM = 64, BN = 64, BK = 16;
  __shared__ T As[BK][BM + 4];
  __shared__ T Bs[BK][BN + 4];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int64_t m0 = (int64_t)blockIdx.y * BM, n0 = (int64_t)blockIdx.x * BN;
  const int64_t kb = (int64_t)blockIdx.z * kchunk, ke = min(K, kb + kchunk);
  const int wm = 32 * (wv >> 1), wn = 32 * (wv & 1);
  typename Mfma<T>::V acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[i][j][e] = T(0);
  for (int64_t k0 = kb; k0 < ke; k0 += BK) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {  // A tile: BM x BK, 4 elements per thread
      const int e = tid + r * 256;
      int mm, kk;
      if (TA) {  // stored K x M: contiguous along m
        kk = e / BM;
        mm = e % BM;
      } else {  // stored M x K: contiguous along k
        mm = e / BK;
        kk = e % BK;
      }
      const int64_t gm = m0 + mm, gk = k0 + kk;
      T v = T(0);
      if (gm < M && gk < ke) v = TA ? A[gk * lda + gm] : A[gm * lda + gk];
      As[kk][mm] = v;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {  // B tile: BK x BN
      const int e = tid + r * 256;
      int nn, kk;
      if (TB) {  // stored N x K: contiguous along k
        nn = e / BK;
        kk = e % BK;
      } else {  // stored K x N: contiguous along n
        kk = e / BN;
        nn = e % BN;
      }
      const int64_t gn = n0 + nn, gk = k0 + kk;
      T v = T(0);
      if (gn < N && gk < ke) v = TB ? B[gn * ldb + gk] : B[gk * ldb + gn];
      Bs[kk][nn] = v;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      const int kk = ks + (lane >> 4);
      T a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = As[kk][wm + 16 * i + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = Bs[kk][wn + 16 * j + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = Mfma<T>::step(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t gm = m0 + wm + 16 * i + Mfma<T>::row(lane, e), gn = n0 + wn + 16 * j + (lane & 15);
        if (gm >= M || gn >= N) continue;
        if (part) {
          part[((int64_t)blockIdx.z * M + gm) * N + gn] = acc[i][j][e];
        } else {
          T* c = Cm + gm * ldc + gn;
          *c = alpha * acc[i][j][e] + (beta == T(0) ? T(0) : beta * *c);
        }
      }
}

// Tall products of the Krylov steps on the matrix cores: A (M x K, or K x M
// when TA) times B (K x N, row-major) with large M and K. A 128 x 64 output
// tile per workgroup (4 wavefronts of 32 rows, each 2 x 4 blocks of the
// 16x16x4 MFMA); K in steps of 32 (FP32) or 16 (FP64) read with 16-byte
// loads (leading dimensions multiples of 16 bytes, A and B 16-byte aligned);
// the next step's tiles are fetched into registers while the current ones
// are multiplied out of LDS. Output as gemm_kernel's (split-K partials or C).
template <typename T>
struct TallCfg;
template <>
struct TallCfg<float> {
  typedef float4 Vec;  // 16-byte load
  static constexpr int kW = 4, kBK = 32, kPad = 4;
};
template <>
struct TallCfg<double> {
  typedef double2 Vec;
  static constexpr int kW = 2, kBK = 16, kPad = 2;
};

template <typename T>
__device__ __forceinline__ T vec_get(const typename TallCfg<T>::Vec& v, int c);
template <>
__device__ __forceinline__ float vec_get<float>(const float4& v, int c) {
  return c == 0 ? v.x : (c == 1 ? v.y : (c == 2 ? v.z : v.w));
}
template <>
__device__ __forceinline__ double vec_get<double>(const double2& v, int c) {
  return c == 0 ? v.x : v.y;
}

template <typename T, bool TA>
__global__ void __launch_bounds__(256) gemm_tall_kernel(int64_t M, int64_t N, int64_t K, int64_t kchunk, T alpha,
                                                        const T* __restrict__ A, int64_t lda, const T* __restrict__ B,
                                                        int64_t ldb, T beta, T* Cm, int64_t ldc, T* __restrict__ part) {
  typedef typename TallCfg<T>::Vec Vec;
  constexpr int W = TallCfg<T>::kW, BK = TallCfg<T>::kBK, PAD = TallCfg<T>::kPad, BM = 128, BN = 64;
  // per thread: 4 vectors of the A tile (BM x BK) and 2 of the B tile (BK x BN)
  static_assert(BM * BK == 4 * 256 * W && BK * BN == 2 * 256 * W, "tile loads");
  __shared__ __align__(16) T As[BK][BM + PAD];
  __shared__ __align__(16) T Bs[BK][BN + PAD];  // rows a multiple of 16 bytes: vector stores stay aligned
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int64_t m0 = (int64_t)blockIdx.y * BM, n0 = (int64_t)blockIdx.x * BN;
  const int64_t kb = (int64_t)blockIdx.z * kchunk, ke = min(K, kb + kchunk);
  const int wm = 32 * wv;
  typename Mfma<T>::V acc[2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[i][j][e] = T(0);
  Vec ra[4], rb[2];
  // which tile entries a thread's vector r holds
  auto a_pos = [&](int r, int& mm, int& kk) {
    const int idx = tid + 256 * r;
    if (TA) {  // rows of k, BM / W vectors each
      kk = idx / (BM / W);
      mm = W * (idx % (BM / W));
    } else {  // rows of m, BK / W vectors each
      mm = idx / (BK / W);
      kk = W * (idx % (BK / W));
    }
  };
  auto b_pos = [&](int r, int& kk, int& nn) {
    const int idx = tid + 256 * r;
    kk = idx / (BN / W);
    nn = W * (idx % (BN / W));
  };
  auto fetch = [&](int64_t k0) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      int mm, kk;
      a_pos(r, mm, kk);
      const int64_t gm = m0 + mm, gk = k0 + kk;
      T v[W];
      if (TA) {  // W consecutive m of row gk
        if (gk < ke && gm + W - 1 < M) {
          ra[r] = *reinterpret_cast<const Vec*>(A + gk * lda + gm);
          continue;
        }
#pragma unroll
        for (int c = 0; c < W; ++c) v[c] = gk < ke && gm + c < M ? A[gk * lda + gm + c] : T(0);
      } else {  // W consecutive k of row gm
        if (gm < M && gk + W - 1 < ke) {
          ra[r] = *reinterpret_cast<const Vec*>(A + gm * lda + gk);
          continue;
        }
#pragma unroll
        for (int c = 0; c < W; ++c) v[c] = gm < M && gk + c < ke ? A[gm * lda + gk + c] : T(0);
      }
      ra[r] = *reinterpret_cast<const Vec*>(v);
    }
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      int kk, nn;
      b_pos(r, kk, nn);
      const int64_t gk = k0 + kk, gn = n0 + nn;
      if (gk < ke && gn + W - 1 < N) {
        rb[r] = *reinterpret_cast<const Vec*>(B + gk * ldb + gn);
        continue;
      }
      T v[W];
#pragma unroll
      for (int c = 0; c < W; ++c) v[c] = gk < ke && gn + c < N ? B[gk * ldb + gn + c] : T(0);
      rb[r] = *reinterpret_cast<const Vec*>(v);
    }
  };
  if (kb < ke) fetch(kb);
  for (int64_t k0 = kb; k0 < ke; k0 += BK) {
    __syncthreads();  // the previous step's reads of As and Bs are done
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      int mm, kk;
      a_pos(r, mm, kk);
      if (TA) {
        *reinterpret_cast<Vec*>(&As[kk][mm]) = ra[r];
      } else {
#pragma unroll
        for (int c = 0; c < W; ++c) As[kk + c][mm] = vec_get<T>(ra[r], c);
      }
    }
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      int kk, nn;
      b_pos(r, kk, nn);
      *reinterpret_cast<Vec*>(&Bs[kk][nn]) = rb[r];
    }
    __syncthreads();
    if (k0 + BK < ke) fetch(k0 + BK);
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      const int kk = ks + (lane >> 4);
      T a[2], b[4];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = As[kk][wm + 16 * i + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[kk][16 * j + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = Mfma<T>::step(a[i], b[j], acc[i][j]);
    }
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t gm = m0 + wm + 16 * i + Mfma<T>::row(lane, e), gn = n0 + 16 * j + (lane & 15);
        if (gm >= M || gn >= N) continue;
        if (part) {
          part[((int64_t)blockIdx.z * M + gm) * N + gn] = acc[i][j][e];
        } else {
          T* c = Cm + gm * ldc + gn;
          *c = alpha * acc[i][j][e] + (beta == T(0) ? T(0) : beta * *c);
        }
      }
}

// C = alpha sum_z part[z] + beta C (z ascending: a fixed order)
template <typename T>
__global__ void splitk_reduce_kernel(int64_t M, int64_t N, int splits, T alpha, const T* __restrict__ part, T beta,
                                     T* Cm, int64_t ldc) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M * N) return;
  T acc = T(0);
  for (int z = 0; z < splits; ++z) acc += part[(int64_t)z * M * N + i];
  const int64_t r = i / N, c = i % N;
  T* o = Cm + r * ldc + c;
  *o = alpha * acc + (beta == T(0) ? T(0) : beta * *o);
}

// ------------------------------------- projected eigenproblem on the device
// Householder tridiagonalisation (Golub & Van Loan, Alg. 8.3.1) of the
// symmetric n x n row-major A, in place, steps k < n - 2: the reflector
// P = I - beta v v^T (v[0] = 1) with P x = mu e1 for x = A[k+1:, k], then
// p = beta A22 v, w = p - (beta p.v / 2) v and A22 -= v w^T + w v^T on the
// trailing (n-k-1)^2 block, kept in full storage (so row k holds x). Each
// workgroup of a step forms the same v from the same sums in the same order;
// workgroup 0 records v[1:] in row k of H (columns k+2..n-1), beta[k],
// d[k] = A[k][k] and e[k] = mu.
constexpr int kProjMax = 2048;  // largest projected problem solved on the device

// Sum over a 256-thread workgroup; every thread receives the same bits.
__device__ __forceinline__ double block_sum256(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}

// One launch per step: step k's kernel applies step k - 1's rank-2 update
// (w from p_{k-1} and v_{k-1}, formed by every workgroup) to the rows of its
// own block while it computes p_k from them. Row k, the only row of step
// k - 1's block that step k reads beyond its own, is updated on the fly, not
// in memory (rows and columns <= k are not read again); the last update, of
// the final 2 x 2 block, is left to house_tail_kernel. Contraction is off,
// so entries (r, c) and (c, r) of an update get the same bits.
__global__ void __launch_bounds__(256) house_step_kernel(double* __restrict__ A, int n, int k, double* __restrict__ H,
                                                         double* __restrict__ betas, double* __restrict__ d,
                                                         double* __restrict__ e, const double* __restrict__ p_prev,
                                                         double* __restrict__ p_out) {
#pragma clang fp contract(off)
  __shared__ double vp[kProjMax], wp[kProjMax], vs[kProjMax];
  __shared__ double red[4];
  constexpr int S = kProjMax / 256;  // entries per thread of a length-n vector
  const int m = n - k - 1;      // step k's block: rows and columns k+1..n-1
  const int mp = m + 1;         // step k-1's block: k..n-1
  const double bp = k > 0 ? betas[k - 1] : 0.0;
  // every load of the prologue issued at once: row k (x = A[k][k+1..]), and
  // step k-1's v and p over its block (index 0 is row k)
  const double* rk = A + (size_t)k * n + (k + 1);
  double xr[S], hv[S], pv[S];
#pragma unroll
  for (int t = 0; t < S; ++t) {
    const int i = threadIdx.x + 256 * t;
    xr[t] = i < m ? rk[i] : 0.0;
    hv[t] = bp != 0.0 && i < mp ? (i == 0 ? 1.0 : H[(size_t)(k - 1) * n + k + i]) : 0.0;
    pv[t] = bp != 0.0 && i < mp ? p_prev[i] : 0.0;
  }
  // step k-1's w = p - (beta p.v / 2) v
  if (bp != 0.0) {
    double sv = 0.0;
#pragma unroll
    for (int t = 0; t < S; ++t) {
      const int i = threadIdx.x + 256 * t;
      if (i < mp) {
        vp[i] = hv[t];
        sv += pv[t] * hv[t];
      }
    }
    const double half = 0.5 * bp * block_sum256(sv, red);
#pragma unroll
    for (int t = 0; t < S; ++t) {
      const int i = threadIdx.x + 256 * t;
      if (i < mp) wp[i] = pv[t] - half * hv[t];
    }
    __syncthreads();
  }
  // row k after step k-1's update, d[k] = A[k][k]
  double s = 0.0;
#pragma unroll
  for (int t = 0; t < S; ++t) {
    const int i = threadIdx.x + 256 * t;
    if (i < m) {
      double x = xr[t];
      if (bp != 0.0) x -= vp[0] * wp[1 + i] + wp[0] * vp[1 + i];
      vs[i] = x;
      if (i >= 1) s += x * x;
    }
  }
  const double sigma = block_sum256(s, red);  // (its barrier also publishes vs)
  const double x0 = vs[0];
  double beta = 0.0, mu = x0, v0 = 1.0;
  if (sigma != 0.0) {
    mu = sqrt(x0 * x0 + sigma);
    v0 = x0 <= 0.0 ? x0 - mu : -sigma / (x0 + mu);
    beta = 2.0 * v0 * v0 / (sigma + v0 * v0);
  }
  __syncthreads();  // every thread has read vs[0]
  for (int i = threadIdx.x; i < m; i += 256) vs[i] = i == 0 ? 1.0 : (sigma != 0.0 ? vs[i] / v0 : 0.0);
  __syncthreads();
  if (blockIdx.x == 0) {
    if (threadIdx.x == 0) {
      double akk = A[(size_t)k * n + k];
      if (bp != 0.0) akk -= vp[0] * wp[0] + wp[0] * vp[0];
      betas[k] = beta;
      d[k] = akk;
      e[k] = mu;
    }
    for (int i = 1 + (int)threadIdx.x; i < m; i += 256) H[(size_t)k * n + k + 1 + i] = vs[i];
  }
  // rows of step k's block: step k-1's update, then p_k = beta A22 v
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  constexpr int U = 8;  // row entries per lane loaded together
  for (int r = blockIdx.x * 4 + wave; r < m; r += gridDim.x * 4) {
    double* row = A + (size_t)(k + 1 + r) * n + (k + 1);
    double acc = 0.0;
    const double vr = bp != 0.0 ? vp[1 + r] : 0.0, wr = bp != 0.0 ? wp[1 + r] : 0.0;
    for (int c0 = 0; c0 < m; c0 += 64 * U) {
      double a[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int c = c0 + lane + 64 * u;
        a[u] = c < m ? row[c] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int c = c0 + lane + 64 * u;
        if (c < m) {
          if (bp != 0.0) {
            a[u] = a[u] - (vr * wp[1 + c] + wr * vp[1 + c]);
            row[c] = a[u];
          }
          acc += a[u] * vs[c];
        }
      }
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if (lane == 0) p_out[r] = beta * acc;
  }
}

// The last steps in one launch: steps k0 .. n-3 and step n-3's update of the
// final 2 x 2 block with that block's entries, by a single workgroup of 1024 threads
// holding step k0 - 1's block (rows and columns k0..n-1, n - k0 <= kTailMax + 1)
// in LDS, a barrier between steps instead of a kernel boundary. The vector
// work runs on the first 256 threads with house_step_kernel's sums in its
// order, and each row's product is reduced within one wavefront as there, so
// the results are the per-step launches' bit for bit.
constexpr int kTailMax = 84;  // (85^2 + 6 * 85) doubles: under 64 KB of LDS

// block_sum256 over the first 256 threads of a larger workgroup (every
// thread takes part in the barriers and receives the sum).
__device__ __forceinline__ double first256_sum(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  __syncthreads();
  if ((threadIdx.x & 63) == 0 && threadIdx.x < 256) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ void __launch_bounds__(1024) house_tail_kernel(const double* __restrict__ A, int n, int k0,
                                                          double* __restrict__ H, double* __restrict__ betas,
                                                          double* __restrict__ d, double* __restrict__ e,
                                                          const double* __restrict__ p_in) {
#pragma clang fp contract(off)
  constexpr int TB = kTailMax + 1;
  __shared__ double As[TB * TB];
  __shared__ double vq[TB], pq[TB];  // step k-1's v and p over its block (index 0 is row k)
  __shared__ double vp[TB], wp[TB], vs[TB], pc[TB];
  __shared__ double red[4];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int mb = n - k0;  // rows and columns k0..n-1
  for (int i = tid; i < mb * mb; i += 1024) As[i] = A[(size_t)(k0 + i / mb) * n + k0 + i % mb];
  double bp = k0 > 0 ? betas[k0 - 1] : 0.0;
  for (int i = tid; i < mb; i += 1024) {
    vq[i] = bp != 0.0 ? (i == 0 ? 1.0 : H[(size_t)(k0 - 1) * n + k0 + i]) : 0.0;
    pq[i] = bp != 0.0 ? p_in[i] : 0.0;
  }
  __syncthreads();
  double beta = 0.0;
  int k = k0;
  for (; k + 2 < n; ++k) {
    const int m = n - k - 1, mp = m + 1, o = k - k0;  // o: row / column k in As
    // step k-1's w = p - (beta p.v / 2) v (one entry per thread, i = tid)
    if (bp != 0.0) {
      double sv = 0.0;
      if (tid < mp) {
        vp[tid] = vq[tid];
        sv += pq[tid] * vq[tid];
      }
      const double half = 0.5 * bp * first256_sum(sv, red);
      if (tid < mp) wp[tid] = pq[tid] - half * vq[tid];
      __syncthreads();
    }
    // row k after step k-1's update
    double s = 0.0;
    if (tid < m) {
      double x = As[o * mb + o + 1 + tid];
      if (bp != 0.0) x -= vp[0] * wp[1 + tid] + wp[0] * vp[1 + tid];
      vs[tid] = x;
      if (tid >= 1) s += x * x;
    }
    const double sigma = first256_sum(s, red);
    const double x0 = vs[0];
    double mu = x0, v0 = 1.0;
    beta = 0.0;
    if (sigma != 0.0) {
      mu = sqrt(x0 * x0 + sigma);
      v0 = x0 <= 0.0 ? x0 - mu : -sigma / (x0 + mu);
      beta = 2.0 * v0 * v0 / (sigma + v0 * v0);
    }
    __syncthreads();  // every thread has read vs[0]
    if (tid < m) vs[tid] = tid == 0 ? 1.0 : (sigma != 0.0 ? vs[tid] / v0 : 0.0);
    __syncthreads();
    if (tid == 0) {
      double akk = As[o * mb + o];
      if (bp != 0.0) akk -= vp[0] * wp[0] + wp[0] * vp[0];
      betas[k] = beta;
      d[k] = akk;
      e[k] = mu;
    }
    if (tid >= 1 && tid < m) H[(size_t)k * n + k + 1 + tid] = vs[tid];
    // rows of step k's block: step k-1's update, then p_k = beta A22 v
    for (int r = wave; r < m; r += 16) {
      double* row = As + (o + 1 + r) * mb + (o + 1);
      double acc = 0.0;
      const double vr = bp != 0.0 ? vp[1 + r] : 0.0, wr = bp != 0.0 ? wp[1 + r] : 0.0;
      double a[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int c = lane + 64 * u;
        a[u] = c < m ? row[c] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int c = lane + 64 * u;
        if (c < m) {
          if (bp != 0.0) {
            a[u] = a[u] - (vr * wp[1 + c] + wr * vp[1 + c]);
            row[c] = a[u];
          }
          acc += a[u] * vs[c];
        }
      }
      for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
      if (lane == 0) pc[r] = beta * acc;
    }
    __syncthreads();
    if (tid < m) {
      vq[tid] = vs[tid];
      pq[tid] = pc[tid];
    }
    bp = beta;
    __syncthreads();
  }
  // step n-3's update of the final 2 x 2 block, and that block's entries
  if (tid == 0) {
    const int o = n - 2 - k0;
    double a00 = As[o * mb + o], a11 = As[(o + 1) * mb + o + 1];
    double a10 = As[(o + 1) * mb + o];
    if (bp != 0.0) {
      const double v0 = 1.0, v1 = vq[1];
      const double half = 0.5 * bp * (pq[0] * v0 + pq[1] * v1);
      const double w0 = pq[0] - half * v0, w1 = pq[1] - half * v1;
      a00 -= v0 * w0 + w0 * v0;
      a11 -= v1 * w1 + w1 * v1;
      a10 -= v1 * w0 + w1 * v0;
    }
    d[n - 2] = a00;
    d[n - 1] = a11;
    e[n - 2] = a10;
    e[n - 1] = 0.0;
  }
}

// Eigenvalue number j (ascending) of the symmetric tridiagonal (d, e2 = e^2)
// by bisection on the Sturm count (the negative pivots of the LDL^T
// factorisation of T - x I; a pivot below pivmin in magnitude taken as
// -pivmin) until the interval is at most atol wide; targets 0..m-1, and
// target m is the largest (index n - 1). 2^L lanes per target, L levels
// per round: lane k (1 .. 2^L - 1) counts at heap node k's midpoint of the
// next L levels (formed by the sequential loop's operations), then the group
// follows the sequential bisection's path through them, stopping where it
// would. So the result is the host's bisection's, with 1/L of the dependent
// counts.
constexpr int kBisectLevels = 6;  // a wavefront per eigenvalue

template <int L>
__global__ void __launch_bounds__(64) sturm_bisect_kernel(int n, const double* __restrict__ d,
                                                          const double* __restrict__ e2, int m, double glo, double ghi,
                                                          double atol, double pivmin, double* __restrict__ out) {
#pragma clang fp contract(off)
  static_assert(L >= 1 && L <= 6, "a group within one wavefront");
  constexpr int G = 1 << L;
  const int lane = threadIdx.x & 63, sub = lane & (G - 1), gbase = lane & ~(G - 1);
  const int t = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> L);
  const bool valid = t <= m;
  const int j = t < m ? t : n - 1;
  double lo = glo, hi = ghi;
  for (int it = 0; it < 200;) {
    // uniform over the wavefront: every lane takes part in every ballot
    if (__ballot(valid && hi - lo > atol) == 0) break;
    bool res = false;
    if (valid && sub >= 1 && hi - lo > atol) {
      double a = lo, b = hi;
      const int depth = 31 - __clz(sub);
      for (int k = depth - 1; k >= 0; --k) {
        const double mm = 0.5 * (a + b);
        if ((sub >> k) & 1)
          a = mm;
        else
          b = mm;
      }
      const double mid = 0.5 * (a + b);
      double q = d[0] - mid;
      if (fabs(q) < pivmin) q = -pivmin;
      int c = q < 0.0;
      for (int i = 1; i < n; ++i) {
        q = (d[i] - mid) - e2[i - 1] / q;
        if (fabs(q) < pivmin) q = -pivmin;
        c += q < 0.0;
      }
      res = c <= j;  // the sequential step would move lo up to this midpoint
    }
    const unsigned long long mask = __ballot(res);
    int node = 1;
    for (int l = 0; l < L && it < 200 && hi - lo > atol; ++l, ++it) {
      const double mid = 0.5 * (lo + hi);
      const int bit = (int)((mask >> (gbase + node)) & 1ull);
      if (bit)
        lo = mid;
      else
        hi = mid;
      node = 2 * node + bit;
    }
  }
  if (valid && sub == 0) out[t] = 0.5 * (lo + hi);
}

// A block of standard normal numbers for the Krylov start: entry t from
// the Philox block (t lo, t hi, 0, 7 << 24) of the key (seed lo, seed hi),
// its first two words as uniforms of (0, 1) by Box-Muller.
__global__ void normal_block_kernel(double* __restrict__ X, int64_t count, uint32_t seed_lo, uint32_t seed_hi) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < count; t += (int64_t)gridDim.x * blockDim.x) {
    const uint4 r = philox10(make_uint4((uint32_t)t, (uint32_t)((uint64_t)t >> 32), 0u, 7u << 24), seed_lo, seed_hi);
    const double u1 = ((double)r.x + 0.5) * 0x1p-32, u2 = ((double)r.y + 0.5) * 0x1p-32;
    X[t] = sqrt(-2.0 * log(u1)) * cospi(2.0 * u2);
  }
}

// Partial sums of the squared Ritz residuals: part[g][j] = sum over the rows
// r of group g (rows g, g + G, ...) of (CV[r][j] - theta[j] V[r][j])^2, for
// the n x m row-major V and CV; the groups are then added in order.
__global__ void ritz_residual_kernel(const double* __restrict__ V, const double* __restrict__ CV,
                                     const double* __restrict__ theta, int64_t n, int m, double* __restrict__ part) {
  const int g = blockIdx.x, G = gridDim.x;
  for (int j = threadIdx.x; j < m; j += blockDim.x) {
    const double th = theta[j];
    double s = 0.0;
    for (int64_t r = g; r < n; r += G) {
      const double dlt = CV[r * m + j] - th * V[r * m + j];
      s += dlt * dlt;
    }
    part[(int64_t)g * m + j] = s;
  }
}

__global__ void sum_groups_kernel(const double* __restrict__ part, int G, int m, double* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m) return;
  double s = 0.0;
  for (int g = 0; g < G; ++g) s += part[(int64_t)g * m + j];
  out[j] = s;
}

// The restart block: X[r][i] = CV[r][pick[i]] - theta[pick[i]] V[r][pick[i]]
// for i < npick, 0 for npick <= i < b (V, CV n x m; X n x b).
__global__ void restart_block_kernel(const double* __restrict__ V, const double* __restrict__ CV,
                                     const double* __restrict__ theta, const int32_t* __restrict__ pick, int npick,
                                     int64_t n, int m, int b, double* __restrict__ X) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n * b; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = t / b;
    const int i = (int)(t % b);
    double x = 0.0;
    if (i < npick) {
      const int j = pick[i];
      x = CV[r * m + j] - theta[j] * V[r * m + j];
    }
    X[t] = x;
  }
}

// A <- (A + A^T) / 2 for the n x n row-major A.
__global__ void symmetrise_kernel(double* A, int n) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * n) return;
  const int i = (int)(t / n), j = (int)(t % n);
  if (j <= i) return;
  const double a = 0.5 * (A[(size_t)i * n + j] + A[(size_t)j * n + i]);
  A[(size_t)i * n + j] = a;
  A[(size_t)j * n + i] = a;
}

// Y = H_0 H_1 ... H_{n-3} X: one wavefront per vector (X vector-major, vector
// j at X[j n ..]; Y n x m row-major), the reflectors applied last first; the
// vector lives in registers, entry r = lane + 64 t in slot t < T (n <= 64 T).
// The reflectors are loaded C = 64 / T at a time (v zero outside its support
// k+1 .. n-1, so the extra terms add exact zeros and the sums are those of the
// support alone, in the same order): one memory latency per C reflectors.
template <int T>
__global__ void __launch_bounds__(256) house_back_kernel(const double* __restrict__ H,
                                                         const double* __restrict__ betas, int n, int m,
                                                         const double* __restrict__ X, double* __restrict__ Y) {
  static_assert(64 * T <= kProjMax, "at most kProjMax entries per vector");
  constexpr int C = 64 / T;
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (j >= m) return;
  double x[T];
#pragma unroll
  for (int t = 0; t < T; ++t) {
    const int r = lane + 64 * t;
    x[t] = r < n ? X[(size_t)j * n + r] : 0.0;
  }
  for (int k = n - 3; k >= 0; k -= C) {
    double v[C][T], beta[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int kc = k - c;  // v[kc+1] = 1, v[kc+2..n-1] stored in row kc
      beta[c] = kc >= 0 ? betas[kc] : 0.0;
      const double* h = H + (size_t)(kc >= 0 ? kc : 0) * n;
#pragma unroll
      for (int t = 0; t < T; ++t) {
        const int r = lane + 64 * t;
        v[c][t] = kc >= 0 && r >= kc + 2 && r < n ? h[r] : (kc >= 0 && r == kc + 1 ? 1.0 : 0.0);
      }
    }
#pragma unroll
    for (int c = 0; c < C; ++c) {
      if (beta[c] == 0.0) continue;
      double s = 0.0;
#pragma unroll
      for (int t = 0; t < T; ++t) s += v[c][t] * x[t];
      for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
      s *= beta[c];
#pragma unroll
      for (int t = 0; t < T; ++t) x[t] -= v[c][t] * s;
    }
  }
#pragma unroll
  for (int t = 0; t < T; ++t) {
    const int r = lane + 64 * t;
    if (r < n) Y[(size_t)r * m + j] = x[t];
  }
}

namespace {

int blocks_for(int64_t n) { return (int)std::min<int64_t>((n + 255) / 256, 1 << 16); }

// Split-K workspace of the products (device memory owned by the caller) and,
// optionally, event pairs around each product for the per-precision sums of
// kernel time and algorithmic flops.
struct GemmWs {
  void* p = nullptr;
  size_t bytes = 0;
  struct Mark {
    hipEvent_t a, b;
    int fp32;
    double flops;
  };
  // Per-product timings: marks still in flight, events free for reuse and the
  // sums over the marks already read. A mark is read as soon as its end event
  // has completed and its events are reused, because creating an event is a
  // driver call that takes longer than a short product, and the device would
  // wait for it.
  struct Timing {
    std::vector<Mark> live;
    std::vector<hipEvent_t> spare;
    EigGemmTimes sum;
    hipError_t take(hipEvent_t& ev) {
      if (!spare.empty()) {
        ev = spare.back();
        spare.pop_back();
        return hipSuccess;
      }
      return hipEventCreate(&ev);
    }
    // read the completed marks, in order (all of them once the stream is idle)
    hipError_t harvest() {
      size_t i = 0;
      for (; i < live.size(); ++i) {
        const Mark& m = live[i];
        const hipError_t q = hipEventQuery(m.b);
        if (q == hipErrorNotReady) break;
        if (q != hipSuccess) return q;
        float g = 0;
        const hipError_t e = hipEventElapsedTime(&g, m.a, m.b);
        if (e != hipSuccess) return e;
        if (m.fp32) {
          ++sum.fp32_products;
          sum.fp32_ms += g;
          sum.fp32_flops += m.flops;
        } else {
          ++sum.fp64_products;
          sum.fp64_ms += g;
          sum.fp64_flops += m.flops;
        }
        spare.push_back(m.a);
        spare.push_back(m.b);
      }
      live.erase(live.begin(), live.begin() + i);
      return hipSuccess;
    }
    ~Timing() {
      for (auto& m : live) {
        (void)hipEventDestroy(m.a);
        (void)hipEventDestroy(m.b);
      }
      for (auto& ev : spare) (void)hipEventDestroy(ev);
    }
  };
  Timing* timing = nullptr;
};

// Splits the K range over enough slices for about 512 workgroups (two per
// compute unit) when the output has few tiles, within the workspace.
template <typename T, bool TA, bool TB>
hipError_t gemm(hipStream_t s, const GemmWs& ws, int64_t M, int64_t N, int64_t K, T alpha, const T* A, int64_t lda,
                const T* B, int64_t ldb, T beta, T* C, int64_t ldc) {
  if (M <= 0 || N <= 0) return hipSuccess;
  // products with more than one 64-row tile and 16-byte aligned rows: the
  // tall kernel
  constexpr bool kTallType = !TB;
  constexpr int64_t kW = 16 / (int64_t)sizeof(T);
  const bool tall = kTallType && M > 64 && lda % kW == 0 && ldb % kW == 0 && ((uintptr_t)A & 15) == 0 &&
                    ((uintptr_t)B & 15) == 0;
  const int64_t BMx = tall ? 128 : 64;
  const int64_t tiles = ((M + BMx - 1) / BMx) * ((N + 63) / 64);
  int64_t splits = 1;
  if (K >= 512) splits = std::min<int64_t>((512 + tiles - 1) / tiles, (K + 255) / 256);
  splits = std::min<int64_t>(splits, (int64_t)(ws.bytes / (sizeof(T) * (size_t)M * (size_t)N)));
  splits = std::max<int64_t>(1, std::min<int64_t>(splits, 65535));
  int64_t kchunk = ((K + splits - 1) / splits + 31) / 32 * 32;  // a multiple of every kernel's K step
  if (kchunk < 32) kchunk = 32;
  splits = std::max<int64_t>(1, (K + kchunk - 1) / kchunk);
  dim3 grid((unsigned)((N + 63) / 64), (unsigned)((M + BMx - 1) / BMx), (unsigned)splits);
  T* part = splits > 1 ? (T*)ws.p : nullptr;
  GemmWs::Mark mk{nullptr, nullptr, sizeof(T) == 4 ? 1 : 0, 2.0 * (double)M * (double)N * (double)K};
  if (ws.timing) {
    hipError_t e;
    if ((e = ws.timing->harvest()) != hipSuccess) return e;
    if ((e = ws.timing->take(mk.a)) != hipSuccess) return e;
    if ((e = ws.timing->take(mk.b)) != hipSuccess) {
      ws.timing->spare.push_back(mk.a);
      return e;
    }
    ws.timing->live.push_back(mk);
    if ((e = hipEventRecord(mk.a, s)) != hipSuccess) return e;
  }
  if constexpr (kTallType) {
    if (tall)
      hipLaunchKernelGGL((gemm_tall_kernel<T, TA>), grid, dim3(256), 0, s, M, N, std::max<int64_t>(K, 0), kchunk,
                         alpha, A, lda, B, ldb, beta, C, ldc, part);
    else
      hipLaunchKernelGGL((gemm_kernel<T, TA, TB>), grid, dim3(256), 0, s, M, N, std::max<int64_t>(K, 0), kchunk, alpha,
                         A, lda, B, ldb, beta, C, ldc, part);
  } else {
    hipLaunchKernelGGL((gemm_kernel<T, TA, TB>), grid, dim3(256), 0, s, M, N, std::max<int64_t>(K, 0), kchunk, alpha, A,
                       lda, B, ldb, beta, C, ldc, part);
  }
  if (splits > 1) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((splitk_reduce_kernel<T>), dim3((unsigned)((M * N + 255) / 256)), dim3(256), 0, s, M, N,
                       (int)splits, alpha, part, beta, C, ldc);
  }
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && ws.timing) e = hipEventRecord(mk.b, s);
  return e;
}

// Page-locked host memory: copies from and to it are queued without a
// staging pass, so the launch that follows a small upload is not held back.
struct PinBuf {
  void* p = nullptr;
  ~PinBuf() {
    if (p) (void)hipHostFree(p);
  }
};

struct DevBuf {
  void* p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  template <typename T>
  T* as() {
    return (T*)p;
  }
};

#define EIG_TRY(expr)                                             \
  do {                                                            \
    hipError_t e_ = (expr);                                       \
    if (e_ != hipSuccess) {                                       \
      err = std::string(#expr) + ": " + hipGetErrorString(e_);    \
      return 3;                                                   \
    }                                                             \
  } while (0)

}  // namespace

// Returns 0 on success, 4 if not converged (best approximations written),
// 1 on bad arguments, 3 on a device error (message in err).
int steklov_modes_device(hipStream_t s, const double* dS, int64_t n_rows, const std::vector<double>& w,
                         const std::vector<int32_t>& discarded, int k, double* evals, double* evecs, int* iters,
                         int* block_out, double* max_res, double* ms_out, EigGemmTimes* gt, std::string& err) {
  hipEvent_t e0, e1;
  EIG_TRY(hipEventCreate(&e0));
  EIG_TRY(hipEventCreate(&e1));
  EIG_TRY(hipEventRecord(e0, s));
  std::vector<int32_t> keep;
  for (int64_t i = 0; i < n_rows; ++i)
    if (w[i] > 0 && !discarded[i]) keep.push_back((int32_t)i);
  const int64_t n = (int64_t)keep.size();
  if (k < 1 || k > n) {
    err = "k must be in 1..(number of kept rows)";
    return 1;
  }
  std::vector<double> m(n);
  for (int64_t a = 0; a < n; ++a) m[a] = 1.0 / std::sqrt(w[keep[a]]);
  DevBuf dkeep, dm, dC64, dC32;
  EIG_TRY(hipMalloc(&dkeep.p, n * 4));
  EIG_TRY(hipMalloc(&dm.p, n * 8));
  EIG_TRY(hipMalloc(&dC64.p, (size_t)n * n * 8));
  EIG_TRY(hipMalloc(&dC32.p, (size_t)n * n * 4));
  // split-K partial tiles: at most about 1,024 tiles of 64 x 64 FP64
  DevBuf dWs;
  GemmWs ws;
  ws.bytes = (size_t)32 << 20;
  EIG_TRY(hipMalloc(&dWs.p, ws.bytes));
  ws.p = dWs.p;
  GemmWs::Timing timing;
  if (gt) ws.timing = &timing;
  EIG_TRY(hipMemcpyAsync(dkeep.p, keep.data(), n * 4, hipMemcpyHostToDevice, s));
  EIG_TRY(hipMemcpyAsync(dm.p, m.data(), n * 8, hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(assemble_c_kernel, dim3(blocks_for(n * n)), dim3(256), 0, s, dS, n_rows, dkeep.as<int32_t>(),
                     dm.as<double>(), n, dC64.as<double>(), dC32.as<float>());
  EIG_TRY(hipGetLastError());

  std::vector<double> theta, Vk;  // final k eigenvalues / n x k vectors (row-major)
  int status = 0;
  const int dense_max = 512;
  if (n <= dense_max) {
    // the whole space fits the projected problem: solve C itself in FP64
    std::vector<double> C((size_t)n * n), ev, V;
    EIG_TRY(hipMemcpyAsync(C.data(), dC64.p, (size_t)n * n * 8, hipMemcpyDeviceToHost, s));
    EIG_TRY(hipStreamSynchronize(s));
    if (!sym_eig((int)n, C, ev, V)) {
      err = "dense eigensolve did not converge";
      return 4;
    }
    theta.assign(ev.begin(), ev.begin() + k);
    Vk.assign((size_t)n * k, 0.0);
    for (int64_t r = 0; r < n; ++r)
      for (int j = 0; j < k; ++j) Vk[(size_t)r * k + j] = V[(size_t)r * n + j];
    *iters = 1;
    *block_out = (int)n;
  } else {
    // block >= 32: smaller blocks stall on clustered ends of the spectrum;
    // a basis of 8k columns and 3k kept Ritz vectors carry the restarts
    // through the dense, noisy lower edge of a Monte Carlo estimate's spectrum
    const int b = std::min<int>(64, std::max<int>(32, ((k + 7) / 8) * 8));
    const int cap = (int)std::min<int64_t>(n, std::max(dense_max, 8 * k));
    const int keep_n = std::min(cap - 2 * b, std::max(3 * k, k + 2 * b));
    // residual target above the floor of FP32 products with C
    const double tol = std::max(1e-5, 16.0 * std::sqrt((double)n) * std::ldexp(1.0, -24));
    *block_out = b;
    DevBuf dQ, dW, dX, dX32, dY32, dT, dG, dY, dQ2, dW2, dH, dBeta, dD, dE, dP, dXc, dEv, dTh, dPart, dRes, dPick;
    EIG_TRY(hipMalloc(&dQ.p, (size_t)n * cap * 8));
    EIG_TRY(hipMalloc(&dW.p, (size_t)n * cap * 8));
    EIG_TRY(hipMalloc(&dX.p, (size_t)n * b * 8));
    EIG_TRY(hipMalloc(&dX32.p, (size_t)n * b * 4));
    EIG_TRY(hipMalloc(&dY32.p, (size_t)n * b * 4));
    EIG_TRY(hipMalloc(&dT.p, (size_t)cap * cap * 8));
    EIG_TRY(hipMalloc(&dG.p, (size_t)cap * b * 8));
    EIG_TRY(hipMalloc(&dY.p, (size_t)cap * cap * 8));
    EIG_TRY(hipMalloc(&dQ2.p, (size_t)n * cap * 8));
    EIG_TRY(hipMalloc(&dW2.p, (size_t)n * cap * 8));
    if (cap <= kProjMax) {  // the device's projected eigensolve
      EIG_TRY(hipMalloc(&dH.p, (size_t)cap * cap * 8));
      EIG_TRY(hipMalloc(&dBeta.p, (size_t)cap * 8));
      EIG_TRY(hipMalloc(&dD.p, (size_t)cap * 8));
      EIG_TRY(hipMalloc(&dE.p, (size_t)cap * 8));
      EIG_TRY(hipMalloc(&dP.p, (size_t)2 * cap * 8));
      EIG_TRY(hipMalloc(&dXc.p, (size_t)cap * keep_n * 8));
      EIG_TRY(hipMalloc(&dEv.p, (size_t)(keep_n + 1) * 8));
    }
    EIG_TRY(hipMalloc(&dTh.p, (size_t)keep_n * 8));
    EIG_TRY(hipMalloc(&dPart.p, (size_t)256 * keep_n * 8));
    EIG_TRY(hipMalloc(&dRes.p, (size_t)keep_n * 8));
    EIG_TRY(hipMalloc(&dPick.p, (size_t)b * 4));
    PinBuf hGram;  // the b x b Gram matrix down, R^-1 up
    EIG_TRY(hipHostMalloc(&hGram.p, (size_t)2 * b * b * 8, hipHostMallocDefault));
    double* const pinG = (double*)hGram.p;
    double* const pinRi = pinG + (size_t)b * b;
    double* Q = dQ.as<double>();
    double* Wm = dW.as<double>();
    double* X = dX.as<double>();
    int cur = 0;
    // orthonormalise X (n x b) against Q[:, :cur] and itself, append it to Q
    // and its product C X to W; false if the block is (numerically) in span(Q)
    auto add_block = [&](bool& ok) -> int {
      ok = false;
      std::vector<double> G((size_t)b * b), R, Ri;
      for (int pass = 0; pass < 2; ++pass) {
        if (cur > 0) {  // X -= Q (Q^T X)
          EIG_TRY((gemm<double, true, false>(s, ws, cur, b, n, 1.0, Q, cap, X, b, 0.0, dG.as<double>(), b)));
          EIG_TRY((gemm<double, false, false>(s, ws, n, b, cur, -1.0, Q, cap, dG.as<double>(), b, 1.0, X, b)));
        }
        EIG_TRY((gemm<double, true, false>(s, ws, b, b, n, 1.0, X, b, X, b, 0.0, dT.as<double>(), b)));
        EIG_TRY(hipMemcpyAsync(pinG, dT.p, (size_t)b * b * 8, hipMemcpyDeviceToHost, s));
        EIG_TRY(hipStreamSynchronize(s));  // (also ends the previous upload from pinRi)
        std::copy(pinG, pinG + (size_t)b * b, G.begin());
        if (!cholesky_upper(b, G, R, 1e-24)) return 0;
        upper_inverse(b, R, Ri);
        std::copy(Ri.begin(), Ri.begin() + (size_t)b * b, pinRi);
        EIG_TRY(hipMemcpyAsync(dT.p, pinRi, (size_t)b * b * 8, hipMemcpyHostToDevice, s));
        // X = X R^-1 (through a temporary: dQ2's first n*b entries)
        EIG_TRY((gemm<double, false, false>(s, ws, n, b, b, 1.0, X, b, dT.as<double>(), b, 0.0, dQ2.as<double>(), b)));
        EIG_TRY(hipMemcpyAsync(X, dQ2.p, (size_t)n * b * 8, hipMemcpyDeviceToDevice, s));
      }
      // append X to Q, C X (FP32 product) to W
      hipLaunchKernelGGL(copy_block_f64_kernel, dim3(blocks_for(n * b)), dim3(256), 0, s, X, (int64_t)b, Q + cur,
                         (int64_t)cap, n, (int64_t)b);
      hipLaunchKernelGGL(copy_block_f64_to_f32_kernel, dim3(blocks_for(n * b)), dim3(256), 0, s, X, (int64_t)b,
                         dX32.as<float>(), (int64_t)b, n, (int64_t)b);
      EIG_TRY((gemm<float, false, false>(s, ws, n, b, n, 1.0f, dC32.as<float>(), n, dX32.as<float>(), b, 0.0f,
                                         dY32.as<float>(), b)));
      hipLaunchKernelGGL(copy_block_f32_to_f64_kernel, dim3(blocks_for(n * b)), dim3(256), 0, s, dY32.as<float>(),
                         (int64_t)b, Wm + cur, (int64_t)cap, n, (int64_t)b);
      EIG_TRY(hipGetLastError());
      cur += b;
      ok = true;
      return 0;
    };
    // random start block (on the device, fixed seed)
    {
      hipLaunchKernelGGL(normal_block_kernel, dim3(blocks_for(n * b)), dim3(256), 0, s, X, n * (int64_t)b, 12345u, 0u);
      EIG_TRY(hipGetLastError());
      bool ok;
      int rc = add_block(ok);
      if (rc) return rc;
      if (!ok) {
        err = "start block is rank deficient";
        return 4;
      }
    }
    const int max_cycles = 60;
    double cnorm = 0.0, worst = 0.0;
    std::vector<double> T, th, Y, res;
    int cycle;
    for (cycle = 0; cycle < max_cycles; ++cycle) {
      // grow the block Krylov space: next block = C (last block)
      while (cur + b <= cap) {
        hipLaunchKernelGGL(copy_block_f64_kernel, dim3(blocks_for(n * b)), dim3(256), 0, s, Wm + (cur - b),
                           (int64_t)cap, X, (int64_t)b, n, (int64_t)b);
        bool ok;
        int rc = add_block(ok);
        if (rc) return rc;
        if (!ok) break;
      }
      // Rayleigh-Ritz on span(Q[:, :cur])
      EIG_TRY((gemm<double, true, false>(s, ws, cur, cur, n, 1.0, Q, cap, Wm, cap, 0.0, dT.as<double>(), cur)));
      const int kk = std::min(keep_n, cur);
      double tmax = 0.0;
      if (cur >= 3 && cur <= kProjMax) {
        // on the device: symmetrise, tridiagonalise; the tridiagonal's kk
        // smallest pairs on the host; back through the reflectors into dY
        double* A = dT.as<double>();
        hipLaunchKernelGGL(symmetrise_kernel, dim3(blocks_for((int64_t)cur * cur)), dim3(256), 0, s, A, cur);
        double* pb[2] = {dP.as<double>(), dP.as<double>() + cap};  // p_{k-1} and p_k, alternating
        // a launch per step while step kx's block is larger than kTailMax,
        // then the rest in one launch from LDS
        int kx = 0;
        for (; kx + 2 < cur && cur - kx - 1 > kTailMax; ++kx) {
          const int g = std::min(256, (cur - kx - 1 + 3) / 4);
          hipLaunchKernelGGL(house_step_kernel, dim3(g), dim3(256), 0, s, A, cur, kx, dH.as<double>(),
                             dBeta.as<double>(), dD.as<double>(), dE.as<double>(), (const double*)pb[(kx + 1) & 1],
                             pb[kx & 1]);
        }
        hipLaunchKernelGGL(house_tail_kernel, dim3(1), dim3(1024), 0, s, (const double*)A, cur, kx, dH.as<double>(),
                           dBeta.as<double>(), dD.as<double>(), dE.as<double>(), (const double*)pb[(kx + 1) & 1]);
        EIG_TRY(hipGetLastError());
        std::vector<double> td(cur), te(cur), e2, Xc;
        EIG_TRY(hipMemcpyAsync(td.data(), dD.p, (size_t)cur * 8, hipMemcpyDeviceToHost, s));
        EIG_TRY(hipMemcpyAsync(te.data(), dE.p, (size_t)cur * 8, hipMemcpyDeviceToHost, s));
        EIG_TRY(hipStreamSynchronize(s));
        // the kk smallest eigenvalues and the largest: bisection, a wavefront each
        double glo, ghi, pivmin, atol;
        bisect_setup(cur, td, te, e2, glo, ghi, pivmin, atol);
        EIG_TRY(hipMemcpyAsync(dP.p, e2.data(), e2.size() * 8, hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(sturm_bisect_kernel<kBisectLevels>, dim3((((kk + 1) << kBisectLevels) + 63) / 64), dim3(64),
                           0, s, cur,
                           (const double*)dD.as<double>(), (const double*)dP.as<double>(), kk, glo, ghi, atol, pivmin,
                           dEv.as<double>());
        EIG_TRY(hipGetLastError());
        std::vector<double> ev((size_t)kk + 1);
        EIG_TRY(hipMemcpyAsync(ev.data(), dEv.p, ev.size() * 8, hipMemcpyDeviceToHost, s));
        EIG_TRY(hipStreamSynchronize(s));
        th.assign(ev.begin(), ev.begin() + kk);
        std::sort(th.begin(), th.end());
        tmax = std::max(std::fabs(th.front()), std::fabs(ev[kk]));
        if (!tridiag_vectors(cur, td, te, th, Xc)) {
          err = "projected eigensolve did not converge";
          return 4;
        }
        EIG_TRY(hipMemcpyAsync(dXc.p, Xc.data(), Xc.size() * 8, hipMemcpyHostToDevice, s));
        const dim3 gb((kk + 3) / 4);
        const double* Hc = dH.as<double>();
        const double* Bc = dBeta.as<double>();
        const double* Xd = dXc.as<double>();
        if (cur <= 512)
          hipLaunchKernelGGL(house_back_kernel<8>, gb, dim3(256), 0, s, Hc, Bc, cur, kk, Xd, dY.as<double>());
        else if (cur <= 1024)
          hipLaunchKernelGGL(house_back_kernel<16>, gb, dim3(256), 0, s, Hc, Bc, cur, kk, Xd, dY.as<double>());
        else
          hipLaunchKernelGGL(house_back_kernel<32>, gb, dim3(256), 0, s, Hc, Bc, cur, kk, Xd, dY.as<double>());
        EIG_TRY(hipGetLastError());
      } else {
        T.assign((size_t)cur * cur, 0.0);
        EIG_TRY(hipMemcpyAsync(T.data(), dT.p, T.size() * 8, hipMemcpyDeviceToHost, s));
        EIG_TRY(hipStreamSynchronize(s));
        for (int i = 0; i < cur; ++i)
          for (int j = i + 1; j < cur; ++j) T[(size_t)i * cur + j] = T[(size_t)j * cur + i] =
              0.5 * (T[(size_t)i * cur + j] + T[(size_t)j * cur + i]);
        if (!sym_eig_smallest(cur, T, kk, th, Y, &tmax)) {
          err = "projected eigensolve did not converge";
          return 4;
        }
        EIG_TRY(hipMemcpyAsync(dY.p, Y.data(), (size_t)cur * kk * 8, hipMemcpyHostToDevice, s));
      }
      cnorm = std::max(cnorm, tmax);
      // Ritz vectors V = Q Y[:, :kk], CV = W Y[:, :kk] (Y is cur x kk)
      EIG_TRY((gemm<double, false, false>(s, ws, n, kk, cur, 1.0, Q, cap, dY.as<double>(), kk, 0.0, dQ2.as<double>(), kk)));
      EIG_TRY((gemm<double, false, false>(s, ws, n, kk, cur, 1.0, Wm, cap, dY.as<double>(), kk, 0.0, dW2.as<double>(), kk)));
      // squared residual norms of the kk Ritz pairs, |CV_j - theta_j V_j|^2,
      // on the device (the row groups added in a fixed order)
      constexpr int kResGroups = 256;
      EIG_TRY(hipMemcpyAsync(dTh.p, th.data(), (size_t)kk * 8, hipMemcpyHostToDevice, s));
      hipLaunchKernelGGL(ritz_residual_kernel, dim3(kResGroups), dim3(256), 0, s, (const double*)dQ2.as<double>(),
                         (const double*)dW2.as<double>(), (const double*)dTh.as<double>(), n, kk, dPart.as<double>());
      hipLaunchKernelGGL(sum_groups_kernel, dim3((kk + 255) / 256), dim3(256), 0, s, (const double*)dPart.as<double>(),
                         kResGroups, kk, dRes.as<double>());
      EIG_TRY(hipGetLastError());
      res.assign(kk, 0.0);
      EIG_TRY(hipMemcpyAsync(res.data(), dRes.p, (size_t)kk * 8, hipMemcpyDeviceToHost, s));
      EIG_TRY(hipStreamSynchronize(s));
      // the first k Ritz vectors on the host, once the iteration ends
      auto take_vectors = [&]() -> int {
        std::vector<double> V2((size_t)n * kk);
        EIG_TRY(hipMemcpyAsync(V2.data(), dQ2.p, V2.size() * 8, hipMemcpyDeviceToHost, s));
        EIG_TRY(hipStreamSynchronize(s));
        theta.assign(th.begin(), th.begin() + k);
        Vk.assign((size_t)n * k, 0.0);
        for (int64_t r = 0; r < n; ++r)
          for (int j = 0; j < k; ++j) Vk[(size_t)r * k + j] = V2[(size_t)r * kk + j];
        return 0;
      };
      worst = 0.0;
      for (int j = 0; j < k; ++j) worst = std::max(worst, std::sqrt(res[j]) / std::max(cnorm, 1e-300));
      const bool done = worst <= tol || cur >= n;
      if (done || cycle + 1 == max_cycles) {
        if (int rc = take_vectors()) return rc;
        if (!done) status = 4;
        break;
      }
      // thick restart: keep the kk Ritz pairs, continue from the residuals of
      // b of them: the lowest unconverged ones first (converged residuals are
      // rounding noise and would add nothing), then the lowest others
      hipLaunchKernelGGL(copy_block_f64_kernel, dim3(blocks_for(n * kk)), dim3(256), 0, s, dQ2.as<double>(),
                         (int64_t)kk, Q, (int64_t)cap, n, (int64_t)kk);
      hipLaunchKernelGGL(copy_block_f64_kernel, dim3(blocks_for(n * kk)), dim3(256), 0, s, dW2.as<double>(),
                         (int64_t)kk, Wm, (int64_t)cap, n, (int64_t)kk);
      EIG_TRY(hipGetLastError());
      cur = kk;
      std::vector<int> pick;
      for (int j = 0; j < kk && (int)pick.size() < b; ++j)
        if (std::sqrt(res[j]) > tol * cnorm) pick.push_back(j);
      for (int j = 0; j < kk && (int)pick.size() < b; ++j)
        if (!(std::sqrt(res[j]) > tol * cnorm)) pick.push_back(j);
      EIG_TRY(hipMemcpyAsync(dPick.p, pick.data(), pick.size() * 4, hipMemcpyHostToDevice, s));
      hipLaunchKernelGGL(restart_block_kernel, dim3(blocks_for(n * b)), dim3(256), 0, s,
                         (const double*)dQ2.as<double>(), (const double*)dW2.as<double>(),
                         (const double*)dTh.as<double>(), (const int32_t*)dPick.as<int32_t>(), (int)pick.size(), n, kk,
                         b, X);
      EIG_TRY(hipGetLastError());
      bool ok;
      int rc = add_block(ok);
      if (rc) return rc;
      if (!ok) {  // residual block already in the span: cannot improve
        if (int rc2 = take_vectors()) return rc2;
        status = worst <= tol ? 0 : 4;
        break;
      }
    }
    *iters = cycle + 1;
  }
  // FP64 Rayleigh quotients and residuals with C in FP64
  {
    DevBuf dV, dCV;
    EIG_TRY(hipMalloc(&dV.p, (size_t)n * k * 8));
    EIG_TRY(hipMalloc(&dCV.p, (size_t)n * k * 8));
    EIG_TRY(hipMemcpyAsync(dV.p, Vk.data(), Vk.size() * 8, hipMemcpyHostToDevice, s));
    EIG_TRY((gemm<double, false, false>(s, ws, n, k, n, 1.0, dC64.as<double>(), n, dV.as<double>(), k, 0.0,
                                        dCV.as<double>(), k)));
    std::vector<double> CV((size_t)n * k);
    EIG_TRY(hipMemcpyAsync(CV.data(), dCV.p, CV.size() * 8, hipMemcpyDeviceToHost, s));
    EIG_TRY(hipStreamSynchronize(s));
    double cn = 0.0;
    for (double t : theta) cn = std::max(cn, std::fabs(t));
    std::vector<double> num(k, 0.0), den(k, 0.0);
    for (int64_t r = 0; r < n; ++r)
      for (int j = 0; j < k; ++j) {
        num[j] += Vk[(size_t)r * k + j] * CV[(size_t)r * k + j];
        den[j] += Vk[(size_t)r * k + j] * Vk[(size_t)r * k + j];
      }
    for (int j = 0; j < k; ++j) theta[j] = num[j] / den[j];
    double mr = 0.0;
    std::vector<double> rr(k, 0.0);
    for (int64_t r = 0; r < n; ++r)
      for (int j = 0; j < k; ++j) {
        const double d = CV[(size_t)r * k + j] - theta[j] * Vk[(size_t)r * k + j];
        rr[j] += d * d;
      }
    for (int j = 0; j < k; ++j) mr = std::max(mr, std::sqrt(rr[j] / den[j]));
    *max_res = mr / std::max(cn, 1e-300);
  }
  // order, then psi = M^-1/2 v on the kept rows, zero elsewhere
  std::vector<int> ord(k);
  for (int j = 0; j < k; ++j) ord[j] = j;
  std::sort(ord.begin(), ord.end(), [&](int a2, int b2) { return theta[a2] < theta[b2]; });
  for (int j = 0; j < k; ++j) evals[j] = theta[ord[j]];
  if (evecs) {
    std::memset(evecs, 0, sizeof(double) * n_rows * k);
    for (int64_t a = 0; a < n; ++a)
      for (int j = 0; j < k; ++j) evecs[(size_t)keep[a] * k + j] = m[a] * Vk[(size_t)a * k + ord[j]];
  }
  EIG_TRY(hipEventRecord(e1, s));
  EIG_TRY(hipEventSynchronize(e1));
  float f = 0;
  EIG_TRY(hipEventElapsedTime(&f, e0, e1));
  *ms_out = f;
  if (gt) {
    EIG_TRY(timing.harvest());  // the stream is idle: every mark is read
    if (!timing.live.empty()) {
      err = "product timing events still pending after the stream finished";
      return 4;
    }
    *gt = timing.sum;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return status;
}

}  // namespace msk
