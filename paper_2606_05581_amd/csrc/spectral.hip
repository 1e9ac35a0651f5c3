// Steklov heat and heat kernel signatures on the vertices (Sec. 5, eqs.
// steklovHeat and spectralSteklovHeat), from K Steklov eigenpairs given in a
// per-vertex table basis Phi (rows: CSR over the basis functions):
//   psi_k(v) = sum_j Phi_vj C_jk,
//   HKS(v, t) = sum_k exp(-lambda_k t) psi_k(v)^2,
//   u_t(v)    = sum_k exp(-lambda_k t) a_k psi_k(v), a_k = sum_v m_v u0_v psi_k(v).
// One wavefront per vertex, lane l holding the eigenfunctions k = l + 64 s
// (s < C); the weights W[k][t] (exp(-lambda_k t), times a_k for the heat)
// come from the host.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "laplace.h"

namespace msk {

namespace {

template <int C>
__device__ __forceinline__ void psi_row(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                                        const float* __restrict__ val, const double* __restrict__ Cm, int32_t Ke,
                                        int64_t v, int lane, double psi[C]) {
#pragma unroll
  for (int s = 0; s < C; ++s) psi[s] = 0.0;
  for (int32_t p = rowptr[v]; p < rowptr[v + 1]; ++p) {
    const double a = (double)val[p];
    const double* crow = Cm + (int64_t)col[p] * Ke;
#pragma unroll
    for (int s = 0; s < C; ++s) {
      const int k = lane + 64 * s;
      if (k < Ke) psi[s] += a * crow[k];
    }
  }
}

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

}  // namespace

// out[v][t] = sum_k W[k][t] f(psi_k(v)), f = square (signature) or identity (heat)
template <int C>
__global__ void __launch_bounds__(256) spectral_fields_kernel(const int32_t* __restrict__ rowptr,
                                                              const int32_t* __restrict__ col,
                                                              const float* __restrict__ val, int64_t nv,
                                                              const double* __restrict__ Cm, int32_t Ke,
                                                              const double* __restrict__ W, int32_t T, int32_t square,
                                                              double* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  for (int64_t v = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); v < nv; v += (int64_t)gridDim.x * 4) {
    double psi[C];
    psi_row<C>(rowptr, col, val, Cm, Ke, v, lane, psi);
    if (square) {
#pragma unroll
      for (int s = 0; s < C; ++s) psi[s] *= psi[s];
    }
    for (int32_t t = 0; t < T; ++t) {
      double acc = 0.0;
#pragma unroll
      for (int s = 0; s < C; ++s) {
        const int k = lane + 64 * s;
        if (k < Ke) acc += W[(int64_t)k * T + t] * psi[s];
      }
      acc = wave_sum(acc);
      if (lane == 0) out[v * T + t] = acc;
    }
  }
}

// part[blockIdx.x][k] = sum over the block's vertices of m_v u0_v psi_k(v)
template <int C>
__global__ void __launch_bounds__(256) spectral_coeff_kernel(const int32_t* __restrict__ rowptr,
                                                             const int32_t* __restrict__ col,
                                                             const float* __restrict__ val, int64_t nv,
                                                             const double* __restrict__ Cm, int32_t Ke,
                                                             const double* __restrict__ mu0,
                                                             double* __restrict__ part) {
  __shared__ double red[4][64 * C];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double acc[C];
#pragma unroll
  for (int s = 0; s < C; ++s) acc[s] = 0.0;
  for (int64_t v = (int64_t)blockIdx.x * 4 + wave; v < nv; v += (int64_t)gridDim.x * 4) {
    double psi[C];
    psi_row<C>(rowptr, col, val, Cm, Ke, v, lane, psi);
    const double w = mu0[v];
#pragma unroll
    for (int s = 0; s < C; ++s) acc[s] += w * psi[s];
  }
#pragma unroll
  for (int s = 0; s < C; ++s) red[wave][lane + 64 * s] = acc[s];
  __syncthreads();
  for (int k = threadIdx.x; k < Ke; k += 256)
    part[(int64_t)blockIdx.x * Ke + k] = red[0][k] + red[1][k] + red[2][k] + red[3][k];
}

hipError_t launch_spectral_fields(const int32_t* rowptr, const int32_t* col, const float* val, int64_t nv,
                                  const double* Cm, int32_t Ke, const double* W, int32_t T, int32_t square,
                                  double* out, hipStream_t s) {
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((nv + 3) / 4, 1 << 20));
  switch ((Ke + 63) / 64) {
#define SP_CASE(c)                                                                                          \
  case c:                                                                                                   \
    hipLaunchKernelGGL(spectral_fields_kernel<c>, dim3(grid), dim3(256), 0, s, rowptr, col, val, nv, Cm, Ke, \
                       W, T, square, out);                                                                  \
    break;
    SP_CASE(1) SP_CASE(2) SP_CASE(3) SP_CASE(4) SP_CASE(5) SP_CASE(6) SP_CASE(7) SP_CASE(8)
#undef SP_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_spectral_coeff(const int32_t* rowptr, const int32_t* col, const float* val, int64_t nv,
                                 const double* Cm, int32_t Ke, const double* mu0, int32_t grid, double* part,
                                 hipStream_t s) {
  switch ((Ke + 63) / 64) {
#define SP_CASE(c)                                                                                         \
  case c:                                                                                                  \
    hipLaunchKernelGGL(spectral_coeff_kernel<c>, dim3(grid), dim3(256), 0, s, rowptr, col, val, nv, Cm, Ke, \
                       mu0, part);                                                                         \
    break;
    SP_CASE(1) SP_CASE(2) SP_CASE(3) SP_CASE(4) SP_CASE(5) SP_CASE(6) SP_CASE(7) SP_CASE(8)
#undef SP_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace msk
