// PSD estimator (Sec. 3.2, Alg. 2): the rank-one updates of a run of walks
// from tangent balls, summed into a dense K x K matrix.
//
// Per antithetic pair p of row i (sample s_i, weight w_i, tangent-ball
// radius r_i) with walks ending at t_1, t_2, the boxed estimator with s
// stratified over rows and z drawn in proportion to the ball jump kernel
// gives X_p = alpha_i (d_1 d_1^T + d_2 d_2^T) / 2, d = b(s_i) - b(t),
// alpha_i = w_i Z_i / (2 P), Z_i the kernel's mass outside the cap (the
// exterior estimate in the Kelvin-inverted domain passes its own alpha_i and
// a factor g per walk: X_p = alpha_i (g_1 d_1 d_1^T + g_2 d_2 d_2^T) / 2,
// and the rows below scale accordingly). The sums
// S = sum_p X_p and Q = sum_p X_p * X_p (elementwise, for standard errors)
// are symmetric rank-k updates S += U^T U, Q += V^T V over rows
//   U: sqrt(alpha/2) d_1, sqrt(alpha/2) d_2;
//   V: (alpha/2) d_1*d_1, (alpha/2) d_2*d_2, sqrt(2) (alpha/2) d_1*d_2,
// so each chunk of pairs is gathered into U and V (HBM-bound, rows padded to
// a multiple of 64 columns) and multiplied on the matrix cores in FP64.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "msk_internal.h"
#include "psd.h"
#include "laplace.h"

namespace msk {

namespace {

inline int grid_for(int64_t n, int bs) { return (int)std::min<int64_t>((n + bs - 1) / bs, 1 << 20); }

// Dense per-vertex table (n_verts x K, zeroed beforehand) from the CSR basis:
// one wavefront per vertex, lanes over its entries (coalesced).
__global__ void dense_table_kernel(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                                   const float* __restrict__ val, int64_t nv, int64_t K, float* __restrict__ tab) {
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t v = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); v < nv; v += waves)
    for (int32_t e = rowptr[v] + (int32_t)(threadIdx.x & 63); e < rowptr[v + 1]; e += 64)
      tab[v * K + col[e]] = val[e];
}

// alpha_i of row i: given per row, or w_i Z(r_i) / (2 pairs) (0 for a row
// without a tangent ball).
__device__ __forceinline__ double pair_alpha(const PsdGather& G, int64_t i) {
  if (G.alpha_row) return G.alpha_row[i];
  const double r = (double)G.radius[i];
  return r > 0.0 ? G.w[i] * (1.0 / (2.0 * r)) * (1.0 / G.u0 - 1.0) / (2.0 * (double)G.pairs) : 0.0;
}

// One workgroup per pair of the chunk [q0, q0 + nq); threads over columns.
__global__ void __launch_bounds__(256) psd_gather_kernel(PsdGather G, int64_t q0, int64_t nq, double* __restrict__ U,
                                                         double* __restrict__ V) {
  const int64_t K = G.K, Kp = G.Kp;
  for (int64_t qq = blockIdx.x; qq < nq; qq += gridDim.x) {
    const int64_t q = q0 + qq;
    const int64_t i = q / G.pairs;
    const int64_t j = q - i * G.pairs;
    const double alpha = pair_alpha(G, i);
    const double g1 = G.walk_g ? G.walk_g[i * 2 * G.pairs + 2 * j] : 1.0;
    const double g2 = G.walk_g ? G.walk_g[i * 2 * G.pairs + 2 * j + 1] : 1.0;
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
    const double su1 = sqrt(0.5 * alpha * g1), su2 = sqrt(0.5 * alpha * g2);
    const double sv1 = 0.5 * alpha * g1, sv2 = 0.5 * alpha * g2, sv12 = sqrt(2.0) * 0.5 * alpha * sqrt(g1 * g2);
    double* u = U + 2 * qq * Kp;
    double* v = V + 3 * qq * Kp;
    for (int64_t k = K + threadIdx.x; k < Kp; k += blockDim.x) {  // padding columns
      u[k] = 0.0;
      u[Kp + k] = 0.0;
      v[k] = 0.0;
      v[Kp + k] = 0.0;
      v[2 * Kp + k] = 0.0;
    }
    for (int64_t k = threadIdx.x; k < K; k += blockDim.x) {
      const double bs = ls[0] * G.tab[fs[0] * K + k] + ls[1] * G.tab[fs[1] * K + k] + ls[2] * G.tab[fs[2] * K + k];
      const double b1 = lt[0][0] * G.tab[ft[0][0] * K + k] + lt[0][1] * G.tab[ft[0][1] * K + k] +
                        lt[0][2] * G.tab[ft[0][2] * K + k];
      const double b2 = lt[1][0] * G.tab[ft[1][0] * K + k] + lt[1][1] * G.tab[ft[1][1] * K + k] +
                        lt[1][2] * G.tab[ft[1][2] * K + k];
      const double d1 = bs - b1, d2 = bs - b2;
      u[k] = su1 * d1;
      u[Kp + k] = su2 * d2;
      v[k] = sv1 * d1 * d1;
      v[Kp + k] = sv2 * d2 * d2;
      v[2 * Kp + k] = sv12 * d1 * d2;
    }
  }
}

// ---- symmetric rank-k product on the matrix cores
// Partial sums of A^T B, A and B m x Kp row-major FP64 matrices (Kp a
// multiple of 64; B = A for the symmetric rank-k product), for the 64 x 64
// blocks (I, J), I <= J, of the Kp x Kp result (A^T B symmetric: the lower
// blocks are taken as the mirror of the upper ones). A
// workgroup takes a slice of the rows; its work items are (block, 4-row group
// residue q mod Q), Q = 4 / gcd(nblk, 4), dealt to its 4 wavefronts in turn,
// so every wavefront gets the same number of items and never two of one
// block. A wavefront keeps the block
// in 16 tiles of v_mfma_f64_16x16x4 accumulators (4 doubles per lane each),
// each step taking 4 rows: operand A = the rows' I-block columns of A (lane l:
// row l / 16, column l % 16 of the tile), operand B = their J-block columns of
// B, so tile (ti, tj) gains sum_r A[r][I + 16 ti + i] B[r][J + 16 tj + j] with
// lane l, item v holding (i, j) = (4 v + l / 16, l % 16) (measured on gfx950
// with one-hot operands). At the end it
// adds the block into its own partial slot P[slice * 4 + wave][block]
// (no other wavefront writes there; slots are summed by psd_reduce_kernel).
typedef double mfma_d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void block_of(int32_t b, int32_t nb, int32_t& I, int32_t& J) {
  I = 0;
  while (b >= nb - I) {
    b -= nb - I;
    ++I;
  }
  J = I + b;
}

__global__ void __launch_bounds__(256) syrk_blocks_kernel(const double* __restrict__ A, const double* __restrict__ B,
                                                          int64_t m, int64_t Kp, int64_t rows_per_slice,
                                                          double* __restrict__ P) {
  const int32_t nb = (int32_t)(Kp / 64), nblk = nb * (nb + 1) / 2;
  const int32_t Q = (nblk % 4 == 0) ? 1 : ((nblk % 2 == 0) ? 2 : 4);
  const int32_t wave = (int32_t)(threadIdx.x >> 6), lane = (int32_t)(threadIdx.x & 63);
  const int64_t r_begin = (int64_t)blockIdx.x * rows_per_slice;
  const int64_t r_end = min(m, r_begin + rows_per_slice);
  const int32_t kr = lane >> 4, cl = lane & 15;
  const int64_t slot = (int64_t)blockIdx.x * 4 + wave;
  for (int32_t item = wave; item < nblk * Q; item += 4) {
    const int32_t blk = item / Q, q = item - blk * Q;
    int32_t I, J;
    block_of(blk, nb, I, J);
    mfma_d4 acc[4][4];
#pragma unroll
    for (int ti = 0; ti < 4; ++ti)
#pragma unroll
      for (int tj = 0; tj < 4; ++tj) acc[ti][tj] = mfma_d4{0.0, 0.0, 0.0, 0.0};
    for (int64_t r0 = r_begin + 4 * (int64_t)q; r0 < r_end; r0 += 4 * (int64_t)Q) {
      const int64_t r = r0 + kr;
      const bool ok = r < r_end;
      const double* row = A + (ok ? r : r_begin) * Kp;
      const double* rowb = B + (ok ? r : r_begin) * Kp;
      double a[4], bv[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        a[t] = ok ? row[I * 64 + 16 * t + cl] : 0.0;
        bv[t] = ok ? rowb[J * 64 + 16 * t + cl] : 0.0;
      }
#pragma unroll
      for (int ti = 0; ti < 4; ++ti)
#pragma unroll
        for (int tj = 0; tj < 4; ++tj)
          acc[ti][tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ti], bv[tj], acc[ti][tj], 0, 0, 0);
    }
    double* out = P + (slot * nblk + blk) * 4096;
#pragma unroll
    for (int ti = 0; ti < 4; ++ti)
#pragma unroll
      for (int tj = 0; tj < 4; ++tj)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = 16 * ti + 4 * v + kr, j = 16 * tj + cl;
          out[i * 64 + j] += acc[ti][tj][v];
        }
  }
}

// ---- fused form (K <= 384): the update rows never leave LDS
// A workgroup takes a range of pairs and a group of up to 4 upper blocks;
// its wavefronts are (matrix, block) items: the first half accumulate S
// blocks from U rows, the second half Q blocks from V rows. Per tile of T
// pairs the workgroup gathers the pairs' U and V rows into LDS (row stride
// Kp + 2 doubles), then every wavefront runs its MFMA steps over them; the
// accumulators stay in registers over the whole range and are stored once
// into the workgroup's slot (slot = blockIdx.x; no other workgroup writes it).
struct PairMeta {
  double alpha;
  double g[2];
  double ls[3], lt[2][3];
  int32_t fs[3], ft[2][3];
};

__device__ void pair_meta(const PsdGather& G, int64_t q, PairMeta& m) {
  const int64_t i = q / G.pairs, j = q - (q / G.pairs) * G.pairs;
  m.alpha = pair_alpha(G, i);
  for (int a = 0; a < 2; ++a) m.g[a] = G.walk_g ? G.walk_g[i * 2 * G.pairs + 2 * j + a] : 1.0;
  const int32_t* fs = G.faces + 3 * (int64_t)G.tri[i];
  for (int c = 0; c < 3; ++c) {
    m.fs[c] = fs[c];
    m.ls[c] = G.bary[3 * i + c];
  }
  for (int a = 0; a < 2; ++a) {
    const int64_t li = i * 2 * G.pairs + 2 * j + a;
    const int32_t st = G.log_status[li], t = G.log_tri[li];
    const bool has_t = st >= 0 && st != kEscaped && t >= 0;
    const double l1 = has_t ? (double)G.log_bary[2 * li] : 0.0, l2 = has_t ? (double)G.log_bary[2 * li + 1] : 0.0;
    m.lt[a][0] = has_t ? (1.0 - l1) - l2 : 0.0;
    m.lt[a][1] = l1;
    m.lt[a][2] = l2;
    for (int c = 0; c < 3; ++c) m.ft[a][c] = has_t ? G.faces[3 * (int64_t)t + c] : 0;
  }
}

// (At most 8 wavefronts per workgroup, so each lane may hold 256 registers:
// the 16 accumulator tiles alone take 128.)
template <int T>
__global__ void __launch_bounds__(512) psd_fused_kernel(PsdGather G, int64_t n_pairs, int64_t pairs_per_wg,
                                                         int32_t group_blocks, double* __restrict__ PS,
                                                         double* __restrict__ PQ) {
  extern __shared__ double lds[];
  const int64_t K = G.K, Kp = G.Kp;
  const int stride = (int)Kp + 2;
  double* Ur = lds;                      // 2T rows
  double* Vr = lds + 2 * T * stride;     // 3T rows
  PairMeta* meta = (PairMeta*)(lds + 5 * T * stride);
  const int32_t nb = (int32_t)(Kp / 64), nblk = nb * (nb + 1) / 2;
  const int32_t g0 = (int32_t)blockIdx.y * group_blocks;
  const int32_t gcount = min(group_blocks, nblk - g0);
  const int32_t wave = (int32_t)(threadIdx.x >> 6), lane = (int32_t)(threadIdx.x & 63);
  const bool is_q = wave >= group_blocks;
  const int32_t wi = is_q ? wave - group_blocks : wave;
  const bool active = wi < gcount;
  const int32_t blk = g0 + wi;
  int32_t I = 0, J = 0;
  if (active) block_of(blk, nb, I, J);
  const int32_t kr = lane >> 4, cl = lane & 15;
  mfma_d4 acc[4][4];
#pragma unroll
  for (int ti = 0; ti < 4; ++ti)
#pragma unroll
    for (int tj = 0; tj < 4; ++tj) acc[ti][tj] = mfma_d4{0.0, 0.0, 0.0, 0.0};
  const int64_t p_begin = (int64_t)blockIdx.x * pairs_per_wg;
  const int64_t p_end = min(n_pairs, p_begin + pairs_per_wg);
  for (int64_t p0 = p_begin; p0 < p_end; p0 += T) {
    if (threadIdx.x < T) {
      const int64_t q = p0 + threadIdx.x;
      if (q < p_end) {
        pair_meta(G, q, meta[threadIdx.x]);
      } else {
        PairMeta& m = meta[threadIdx.x];
        m.alpha = 0.0;
        m.g[0] = m.g[1] = 1.0;
        for (int c = 0; c < 3; ++c) {
          m.fs[c] = m.ft[0][c] = m.ft[1][c] = 0;
          m.ls[c] = m.lt[0][c] = m.lt[1][c] = 0.0;
        }
      }
    }
    __syncthreads();
    for (int e = (int)threadIdx.x; e < T * (int)Kp; e += (int)blockDim.x) {
      const int pp = e / (int)Kp, k = e - pp * (int)Kp;
      const PairMeta& m = meta[pp];
      double d1 = 0.0, d2 = 0.0;
      if (k < K) {
        const double bs = m.ls[0] * G.tab[m.fs[0] * K + k] + m.ls[1] * G.tab[m.fs[1] * K + k] +
                          m.ls[2] * G.tab[m.fs[2] * K + k];
        const double b1 = m.lt[0][0] * G.tab[m.ft[0][0] * K + k] + m.lt[0][1] * G.tab[m.ft[0][1] * K + k] +
                          m.lt[0][2] * G.tab[m.ft[0][2] * K + k];
        const double b2 = m.lt[1][0] * G.tab[m.ft[1][0] * K + k] + m.lt[1][1] * G.tab[m.ft[1][1] * K + k] +
                          m.lt[1][2] * G.tab[m.ft[1][2] * K + k];
        d1 = bs - b1;
        d2 = bs - b2;
      }
      const double su1 = sqrt(0.5 * m.alpha * m.g[0]), su2 = sqrt(0.5 * m.alpha * m.g[1]);
      const double sv1 = 0.5 * m.alpha * m.g[0], sv2 = 0.5 * m.alpha * m.g[1];
      const double sv12 = sqrt(2.0) * 0.5 * m.alpha * sqrt(m.g[0] * m.g[1]);
      Ur[(2 * pp) * stride + k] = su1 * d1;
      Ur[(2 * pp + 1) * stride + k] = su2 * d2;
      Vr[(3 * pp) * stride + k] = sv1 * d1 * d1;
      Vr[(3 * pp + 1) * stride + k] = sv2 * d2 * d2;
      Vr[(3 * pp + 2) * stride + k] = sv12 * d1 * d2;
    }
    __syncthreads();
    if (active) {
      const double* R = is_q ? Vr : Ur;
      const int nrows = is_q ? 3 * T : 2 * T;
      for (int s0 = 0; s0 < nrows; s0 += 4) {
        const double* row = R + (s0 + kr) * stride;
        double a[4], bv[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          a[t] = row[I * 64 + 16 * t + cl];
          bv[t] = row[J * 64 + 16 * t + cl];
        }
#pragma unroll
        for (int ti = 0; ti < 4; ++ti)
#pragma unroll
          for (int tj = 0; tj < 4; ++tj)
            acc[ti][tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ti], bv[tj], acc[ti][tj], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  if (active) {
    double* out = (is_q ? PQ : PS) + ((int64_t)blockIdx.x * nblk + blk) * 4096;
#pragma unroll
    for (int ti = 0; ti < 4; ++ti)
#pragma unroll
      for (int tj = 0; tj < 4; ++tj)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = 16 * ti + 4 * v + kr, j = 16 * tj + cl;
          out[i * 64 + j] = acc[ti][tj][v];
        }
  }
}

// C (K x K, row-major) = sum over slots of the partial blocks, the lower
// triangle mirrored from the upper one.
__global__ void psd_reduce_kernel(const double* __restrict__ P, int64_t n_slots, int64_t K, int64_t Kp,
                                  double* __restrict__ C) {
  const int32_t nb = (int32_t)(Kp / 64), nblk = nb * (nb + 1) / 2;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < K * K; e += (int64_t)gridDim.x * blockDim.x) {
    int64_t i = e / K, j = e - (e / K) * K;
    if (i > j) {
      const int64_t t = i;
      i = j;
      j = t;
    }
    const int32_t I = (int32_t)(i / 64), J = (int32_t)(j / 64);
    const int32_t blk = I * nb - I * (I - 1) / 2 + (J - I);
    const int64_t off = (int64_t)blk * 4096 + (i - 64 * I) * 64 + (j - 64 * J);
    double sum = 0.0;
    for (int64_t sl = 0; sl < n_slots; ++sl) sum += P[sl * nblk * 4096 + off];
    C[e] = sum;
  }
}

// Standard error of every entry: se^2 = (n Q - S^2) / (n - 1) over n pair terms.
__global__ void psd_se_kernel(const double* __restrict__ S, const double* __restrict__ Q, int64_t n, double n_pairs,
                              double* __restrict__ se) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    se[e] = sqrt(fmax(0.0, n_pairs * Q[e] - S[e] * S[e]) / (n_pairs - 1.0));
}

}  // namespace

hipError_t launch_dense_table(const int32_t* rowptr, const int32_t* col, const float* val, int64_t nv, int64_t K,
                              float* tab, hipStream_t s) {
  if (nv <= 0) return hipSuccess;
  hipLaunchKernelGGL(dense_table_kernel, dim3(grid_for(nv, 4)), dim3(256), 0, s, rowptr, col, val, nv, K, tab);
  return hipGetLastError();
}

hipError_t launch_psd_gather(const PsdGather& G, int64_t q0, int64_t nq, double* U, double* V, hipStream_t s) {
  if (nq <= 0) return hipSuccess;
  const int threads = G.K >= 256 ? 256 : (G.K >= 128 ? 128 : 64);
  hipLaunchKernelGGL(psd_gather_kernel, dim3((unsigned)std::min<int64_t>(nq, 1 << 20)), dim3(threads), 0, s, G, q0,
                     nq, U, V);
  return hipGetLastError();
}

// pairs per tile of the fused form: 5 T rows of Kp + 2 doubles stay within 64 KB of LDS
static int64_t fused_tile(int64_t Kp) { return Kp <= 192 ? 8 : (Kp <= 384 ? 4 : 0); }

// upper blocks per workgroup of the fused form (two wavefronts each)
static const int64_t kFusedGroup = 4;

int64_t psd_fused_slots(int64_t Kp, int64_t n_pairs) {
  const int64_t nblk = psd_blocks(Kp), gb = std::min<int64_t>(nblk, kFusedGroup), groups = (nblk + gb - 1) / gb;
  const int64_t T = fused_tile(Kp);
  if (T == 0) return 0;
  return std::max<int64_t>(1, std::min<int64_t>((n_pairs + T - 1) / T, 2048 / groups));
}

hipError_t launch_psd_fused(const PsdGather& G, int64_t n_pairs, int64_t n_slots, double* PS, double* PQ,
                            hipStream_t s) {
  if (n_pairs <= 0) return hipSuccess;
  const int64_t Kp = G.Kp, nblk = psd_blocks(Kp), gb = std::min<int64_t>(nblk, kFusedGroup);
  const int64_t groups = (nblk + gb - 1) / gb;
  const int64_t ppw = (n_pairs + n_slots - 1) / n_slots;
  const dim3 grid((unsigned)n_slots, (unsigned)groups), block((unsigned)(128 * gb));
  const int64_t T = fused_tile(Kp);
  if (T == 8) {
    const size_t lds = (size_t)5 * 8 * (Kp + 2) * 8 + 8 * sizeof(PairMeta);
    hipLaunchKernelGGL(psd_fused_kernel<8>, grid, block, lds, s, G, n_pairs, ppw, (int32_t)gb, PS, PQ);
  } else if (T == 4) {
    const size_t lds = (size_t)5 * 4 * (Kp + 2) * 8 + 4 * sizeof(PairMeta);
    hipLaunchKernelGGL(psd_fused_kernel<4>, grid, block, lds, s, G, n_pairs, ppw, (int32_t)gb, PS, PQ);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

int64_t psd_blocks(int64_t Kp) {
  const int64_t nb = Kp / 64;
  return nb * (nb + 1) / 2;
}

hipError_t launch_psd_syrk(const double* A, int64_t m, int64_t Kp, int64_t slices, double* P, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  const int64_t rps = ((m + slices - 1) / slices + 3) / 4 * 4;
  const int64_t grid = (m + rps - 1) / rps;
  hipLaunchKernelGGL(syrk_blocks_kernel, dim3((unsigned)grid), dim3(256), 0, s, A, A, m, Kp, rps, P);
  return hipGetLastError();
}

hipError_t launch_gram_upper(const double* A, const double* B, int64_t m, int64_t Kp, int64_t slices, double* P,
                             hipStream_t s) {
  if (m <= 0) return hipSuccess;
  const int64_t rps = ((m + slices - 1) / slices + 3) / 4 * 4;
  const int64_t grid = (m + rps - 1) / rps;
  hipLaunchKernelGGL(syrk_blocks_kernel, dim3((unsigned)grid), dim3(256), 0, s, A, B, m, Kp, rps, P);
  return hipGetLastError();
}

hipError_t launch_psd_reduce(const double* P, int64_t n_slots, int64_t K, int64_t Kp, double* C, hipStream_t s) {
  hipLaunchKernelGGL(psd_reduce_kernel, dim3(grid_for(K * K, 256)), dim3(256), 0, s, P, n_slots, K, Kp, C);
  return hipGetLastError();
}

hipError_t launch_psd_se(const double* S, const double* Q, int64_t n, double n_pairs, double* se, hipStream_t s) {
  hipLaunchKernelGGL(psd_se_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, S, Q, n, n_pairs, se);
  return hipGetLastError();
}

}  // namespace msk
