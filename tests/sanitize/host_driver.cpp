// Exercises the library's host-side code that runs without a device, under
// AddressSanitizer and UndefinedBehaviorSanitizer: the binned-SAH BVH build
// and 4-wide collapse (build_bvh_host, build_bvh_boxes; valid meshes, a
// degenerate triangle and rejected inputs) and the dense symmetric
// eigensolvers of the eigen step (sym_eig, sym_eig_smallest,
// cholesky_upper). Exit status 0 when every result checks out.
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>

#include "../../paper_2606_05581_amd/csrc/msk_internal.h"

namespace msk {
bool sym_eig(int n, std::vector<double>& A, std::vector<double>& evals, std::vector<double>& V);
bool sym_eig_smallest(int n, std::vector<double>& A, int m, std::vector<double>& evals, std::vector<double>& V,
                      double* abs_max);
bool cholesky_upper(int n, const std::vector<double>& A, std::vector<double>& R, double rel_tol);
}  // namespace msk

int main() {
  std::mt19937 rng(5);
  std::uniform_real_distribution<float> U(-1.0f, 1.0f);
  // a random soup of 3000 triangles plus a zero-area one
  const int nf = 3001, nv = 3 * nf;
  std::vector<float> V(3 * nv);
  std::vector<int32_t> F(3 * nf);
  for (int i = 0; i < nv; ++i)
    for (int k = 0; k < 3; ++k) V[3 * i + k] = U(rng) + (i / 3 % 7) * 0.5f;
  for (int t = 0; t < nf; ++t)
    for (int j = 0; j < 3; ++j) F[3 * t + j] = 3 * t + j;
  for (int k = 0; k < 3; ++k) V[3 * (nv - 1) + k] = V[3 * (nv - 2) + k];  // repeated vertex: zero area
  for (int leaf = 1; leaf <= 8; ++leaf) {
    msk::HostBvh out;
    std::string err = msk::build_bvh_host(V.data(), nv, F.data(), nf, leaf, out);
    if (!err.empty() || (int)out.tris.size() != nf) {
      std::printf("build failed: %s\n", err.c_str());
      return 1;
    }
  }
  {  // rejected inputs
    msk::HostBvh out;
    std::vector<int32_t> Fb = F;
    Fb[7] = nv + 3;
    if (msk::build_bvh_host(V.data(), nv, Fb.data(), nf, 4, out).empty()) return 2;
    std::vector<float> Vb = V;
    Vb[11] = NAN;
    if (msk::build_bvh_host(Vb.data(), nv, F.data(), nf, 4, out).empty()) return 3;
    if (msk::build_bvh_host(V.data(), nv, F.data(), nf, 9, out).empty()) return 4;
  }
  // symmetric eigenproblems: A = Q diag Q^T with a known spectrum
  const int n = 60;
  std::vector<double> A((size_t)n * n, 0.0), A2, ev, Vv;
  std::normal_distribution<double> G(0.0, 1.0);
  std::vector<double> B((size_t)n * n);
  for (double& x : B) x = G(rng);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double s = 0;
      for (int k = 0; k < n; ++k) s += B[i * n + k] * B[j * n + k];
      A[i * n + j] = s;
    }
  A2 = A;
  if (!msk::sym_eig(n, A2, ev, Vv)) return 5;
  for (int i = 1; i < n; ++i)
    if (ev[i] < ev[i - 1]) return 6;
  A2 = A;
  std::vector<double> ev2, V2;
  double amax = 0;
  if (!msk::sym_eig_smallest(n, A2, 10, ev2, V2, &amax)) return 7;
  for (int i = 0; i < 10; ++i)
    if (std::fabs(ev2[i] - ev[i]) > 1e-8 * std::fabs(ev[n - 1])) return 8;
  std::vector<double> R;
  if (!msk::cholesky_upper(n, A, R, 1e-24)) return 9;
  std::printf("host driver: ok (lambda_min %.6g, lambda_max %.6g)\n", ev[0], ev[n - 1]);
  return 0;
}
