// Declarations of the mesh Laplacian basis (laplace.hip), of the Gram
// product it shares with the PSD estimator (psd.hip), and of the spectral
// fields built on a basis (spectral.hip).
#pragma once
#include "msk_internal.h"

namespace msk {
// Partial upper blocks of A^T B (A, B: m x Kp row-major, A^T B symmetric) into P, as launch_psd_syrk
hipError_t launch_gram_upper(const double* A, const double* B, int64_t m, int64_t Kp, int64_t slices, double* P,
                             hipStream_t s);

// Mesh-based Galerkin basis (laplace.hip)
struct LaplaceInfo {
  int64_t active_vertices = 0, skipped_faces = 0, spmm_calls = 0;
  int32_t iters = 0, converged = 0, grams = 0, rotates = 0, rank_drops = 0, last_degree = 0, locked = 0;
  double bound = 0.0, filter_lower = 0.0, max_residual = 0.0, filter_bytes = 0.0;
  double assemble_ms = 0.0, filter_ms = 0.0, dense_ms = 0.0, total_ms = 0.0;
};
struct LaplaceJob {
  hipStream_t stream = nullptr;
  int64_t n = 0;           // vertices (internal order)
  int64_t nnz = 0;         // stored entries of L
  int32_t lock = 1;        // leave converged leading columns out of the filter
  int64_t m = 0, K = 0;    // block size (multiple of 64, <= 512), wanted modes
  int32_t degree = 0, max_degree = 0, max_iters = 0;  // degree 0: adaptive, at most max_degree
  double tol = 0.0;
  uint64_t seed = 0;
  const float* P = nullptr;       // positions, n x 3, internal order
  const int32_t* F = nullptr;     // faces in internal vertex ids, n_faces x 3
  const int32_t* vt_ptr = nullptr;  // vertex -> incident faces (ascending), CSR
  const int32_t* vt_tri = nullptr;
  const int32_t* rowptr = nullptr;  // sparsity pattern of L (sorted columns, diagonal included)
  const int32_t* col = nullptr;
  const int32_t* orig = nullptr;    // internal -> original vertex index
  double* val = nullptr;            // nnz
  double* mass = nullptr;           // n
  double* s = nullptr;              // n: M^-1/2 (0 where the mass is 0)
  unsigned long long* counters = nullptr;  // 2: degenerate faces, vertices of positive mass
  double* blk[3] = {nullptr, nullptr, nullptr};  // n x m each
  double* slots = nullptr;          // Gram partial slots, n_slots x psd_blocks(m) x 4096
  int64_t n_slots = 0;              // a multiple of 4
  double* small = nullptr;          // max(m * m, 4096) doubles
  double* part = nullptr;           // residual partials, 1024 x K
  double* evals = nullptr;          // host, K
  double* phi = nullptr;            // device, n x K in original order (optional)
  int32_t* out_rowptr = nullptr;    // dense basis table (n + 1, n K, n K)
  int32_t* out_col = nullptr;
  float* out_val = nullptr;
  LaplaceInfo info;
};
int laplace_basis_device(LaplaceJob& J, std::string& err);

// Steklov heat and heat kernel signatures (spectral.hip)
hipError_t launch_spectral_fields(const int32_t* rowptr, const int32_t* col, const float* val, int64_t nv,
                                  const double* Cm, int32_t Ke, const double* W, int32_t T, int32_t square,
                                  double* out, hipStream_t s);
hipError_t launch_spectral_coeff(const int32_t* rowptr, const int32_t* col, const float* val, int64_t nv,
                                 const double* Cm, int32_t Ke, const double* mu0, int32_t grid, double* part,
                                 hipStream_t s);
}  // namespace msk
