// Declarations of the PSD estimator kernels (psd.hip) used by the host code.
#pragma once
#include "msk_internal.h"

namespace msk {

// PSD estimator (psd.hip): per-pair inputs of the rank-one updates
struct PsdGather {
  const float* tab;         // dense per-vertex basis table, n_verts x K (the basis values, FP32)
  int64_t K;
  int64_t Kp;               // row stride of the gathered update rows (K rounded up to 64)
  int64_t pairs;            // antithetic pairs per row
  const int32_t* faces;     // original faces (n_tris x 3)
  const int32_t* tri;       // sample face per row
  const float* bary;        // sample barycentrics per row (n x 3)
  const double* w;          // row weights
  const float* radius;      // tangent-ball radius per row (0 = dropped)
  double u0;                // sin(theta0 / 2)
  const int32_t* log_status;  // walk log, n_rows x 2 pairs
  const int32_t* log_tri;
  const float* log_bary;
  // optional (null = the interior estimator's): per-row alpha replacing
  // w Z(r) / (2 pairs), and a per-walk factor g of its rank-one update
  // (X_p = alpha (g_1 d_1 d_1^T + g_2 d_2 d_2^T) / 2), both FP64
  const double* alpha_row;
  const double* walk_g;
};
hipError_t launch_dense_table(const int32_t* rowptr, const int32_t* col, const float* val, int64_t nv, int64_t K,
                              float* tab, hipStream_t s);
hipError_t launch_psd_gather(const PsdGather& G, int64_t q0, int64_t nq, double* U, double* V, hipStream_t s);
// Fused gather + products (Kp <= 384): partial slots (one per workgroup column) of S and Q blocks; 0 = not available
int64_t psd_fused_slots(int64_t Kp, int64_t n_pairs);
hipError_t launch_psd_fused(const PsdGather& G, int64_t n_pairs, int64_t n_slots, double* PS, double* PQ,
                            hipStream_t s);
hipError_t launch_psd_se(const double* S, const double* Q, int64_t n, double n_pairs, double* se, hipStream_t s);

}  // namespace msk
