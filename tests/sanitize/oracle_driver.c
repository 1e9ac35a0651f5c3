/* Exercises the oracle's C entry points on small inputs under
 * AddressSanitizer and UndefinedBehaviorSanitizer (CPU only): scene with and
 * without its BVH, nearest queries, walks, the row estimator (interior,
 * exterior, hat and point rows), the PSD estimator and the Kelvin-inverted
 * exterior estimator. Exit status 0 when every call ran; a sanitizer report
 * aborts the program. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void* orc_scene_create(const float* V, int64_t nv, const int32_t* F, int64_t nf, int with_bvh);
void orc_scene_destroy(void* h);
void orc_nearest(const void* h, const double* Q, int64_t nq, int use_bvh, int64_t* tri, double* d2, double* bary);
void orc_walks_from(const void* h, const double* X, int64_t n, double eps, double kappa, double delta,
                    int64_t max_steps, uint64_t seed, int32_t* status, int64_t* tri, double* bary, int64_t* nquery);
void orc_estimate(const void* scene, int mode_start, int exterior, int64_t n_rows, const int32_t* rows_sel,
                  const float* p, const float* nrm, const int32_t* tri, const float* bary, const int32_t* ring_ptr,
                  const int32_t* ring_tri, const double* ring_cum, const float* fn, const int32_t* rowptr,
                  const int32_t* col, const float* val, int64_t K, int64_t W, int64_t w0, double eps, double hin,
                  double kappa, double delta, int64_t max_steps, uint64_t seed, uint32_t mesh, int nthreads,
                  double* acc, double* acc2, int64_t* n_query, int64_t* n_escaped, int64_t* n_capped,
                  int32_t* discarded, int32_t* log_status, int64_t* log_tri, float* log_bary, int64_t* log_nquery,
                  int32_t* log_stri, float* log_sbary, const double* knn_x, const double* knn_n, int64_t knn_N,
                  int knn_k, double knn_sigma, double knn_tau, int jump_only);
void orc_psd_estimate(const void* h, int64_t n_rows, const float* p, const float* nrm, const int32_t* tri,
                      const float* bary, const double* w, const double* tab, int64_t K, int64_t pairs,
                      double theta0, double r_max, int bisect_iters, double eps, double kappa, double delta,
                      int64_t max_steps, uint64_t seed, uint32_t mesh, int nthreads, double* S, double* Q,
                      double* radius, double* Zout, int64_t* n_query, int32_t* log_status, int64_t* log_tri,
                      float* log_bary, int64_t* log_nquery);
void* orc_kelvin_create(const float* V, int64_t nv, const int32_t* F, int64_t nf, const double* centre);
void orc_kelvin_destroy(void* h);
void orc_kelvin_estimate(const void* h, int64_t n_rows, const float* p, const float* nrm, const int32_t* tri,
                         const float* bary, const double* w, const double* tab, int64_t K, int64_t pairs,
                         int64_t kill_walks, double theta0, double r_max, int bisect_iters, double eps, double kappa,
                         double delta, int64_t max_steps, uint64_t seed, uint32_t mesh, int nthreads, double* Sj,
                         double* Qj, double* Sk, double* Qk, double* radius, double* Zout, int64_t* n_query,
                         int64_t* kill_query, int32_t* log_status, int64_t* log_tri, float* log_bary);

/* octahedron refined once: 18 vertices, 32 faces, on the unit sphere */
static int mesh(float* V, int32_t* F) {
  static const float base[6][3] = {{1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};
  static const int faces[8][3] = {{0, 2, 4}, {2, 1, 4}, {1, 3, 4}, {3, 0, 4}, {2, 0, 5}, {1, 2, 5}, {3, 1, 5}, {0, 3, 5}};
  int nv = 6, nf = 0;
  memcpy(V, base, sizeof(base));
  for (int f = 0; f < 8; ++f) {
    int m[3];
    for (int e = 0; e < 3; ++e) {
      int a = faces[f][e], b = faces[f][(e + 1) % 3];
      float x[3];
      for (int k = 0; k < 3; ++k) x[k] = 0.5f * (V[3 * a + k] + V[3 * b + k]);
      float l = sqrtf(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
      int found = -1;
      for (int v = 6; v < nv; ++v)
        if (fabsf(V[3 * v] - x[0] / l) < 1e-6f && fabsf(V[3 * v + 1] - x[1] / l) < 1e-6f &&
            fabsf(V[3 * v + 2] - x[2] / l) < 1e-6f)
          found = v;
      if (found < 0) {
        for (int k = 0; k < 3; ++k) V[3 * nv + k] = x[k] / l;
        found = nv++;
      }
      m[e] = found;
    }
    int t[4][3] = {{faces[f][0], m[0], m[2]}, {m[0], faces[f][1], m[1]}, {m[2], m[1], faces[f][2]}, {m[0], m[1], m[2]}};
    for (int i = 0; i < 4; ++i) memcpy(F + 3 * nf++, t[i], sizeof(t[i]));
  }
  return nv;
}

int main(void) {
  float V[3 * 32];
  int32_t F[3 * 32];
  const int nv = mesh(V, F), nf = 32;
  /* rows: face centres with face normals */
  enum { N = 12, W = 8, K = 4 };
  float p[3 * N], n[3 * N], bary[3 * N];
  int32_t tri[N];
  double w[N];
  for (int i = 0; i < N; ++i) {
    int f = (5 * i) % nf;
    float c[3] = {0, 0, 0};
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k) c[k] += V[3 * F[3 * f + j] + k] / 3.0f;
    float l = sqrtf(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
    for (int k = 0; k < 3; ++k) { p[3 * i + k] = c[k]; n[3 * i + k] = c[k] / l; bary[3 * i + k] = 1.0f / 3.0f; }
    tri[i] = f;
    w[i] = 4.0 * M_PI / N;
  }
  /* table: constant and coordinates */
  int32_t rowptr[33], col[4 * 32];
  float val[4 * 32];
  double tab[32 * K];
  for (int v = 0; v < nv; ++v) {
    rowptr[v] = 4 * v;
    for (int k = 0; k < K; ++k) {
      col[4 * v + k] = k;
      val[4 * v + k] = k == 0 ? 1.0f : V[3 * v + k - 1];
      tab[v * K + k] = val[4 * v + k];
    }
  }
  rowptr[nv] = 4 * nv;
  for (int bvh = 0; bvh < 2; ++bvh) {
    void* s = orc_scene_create(V, nv, F, nf, bvh);
    double Q[9] = {0.1, 0.2, 0.3, 2.0, 0.0, 0.0, 0.5, -0.5, 0.2};
    int64_t t[3];
    double d2[3], b[9];
    orc_nearest(s, Q, 3, bvh, t, d2, b);
    int32_t st[3];
    int64_t nq[3];
    orc_walks_from(s, Q, 3, 1e-3, 1e-6, 1e-7, 1000, 1, st, t, b, nq);
    double acc[N * N], acc2[N * N];
    int64_t q[N], esc[N], cap[N];
    int32_t disc[N], ls[N * W], lst[N * W];
    int64_t lt[N * W], lq[N * W];
    float lb[2 * N * W], lsb[2 * N * W];
    for (int ext = 0; ext < 2; ++ext) /* point rows with the vertex basis, logs on */
      orc_estimate(s, 0, ext, N, NULL, p, n, tri, bary, NULL, NULL, NULL, NULL, rowptr, col, val, K, W, 0, 1e-3,
                   0.05, 1e-6, 1e-7, 64, 2, 0, 2, acc, acc2, q, esc, cap, disc, ls, lt, lb, lq, lst, lsb, NULL, NULL,
                   0, 0, 0.0, 0.0, ext);
    /* hat rows over every vertex: one-ring faces with cumulative areas */
    {
      int32_t ring_ptr[33], ring_tri[96];
      double ring_cum[96];
      float fn[3 * 32];
      int m = 0;
      for (int f = 0; f < nf; ++f) {
        const float* a = V + 3 * F[3 * f]; const float* b = V + 3 * F[3 * f + 1]; const float* c = V + 3 * F[3 * f + 2];
        float e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]}, e2[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
        fn[3 * f] = e1[1] * e2[2] - e1[2] * e2[1];
        fn[3 * f + 1] = e1[2] * e2[0] - e1[0] * e2[2];
        fn[3 * f + 2] = e1[0] * e2[1] - e1[1] * e2[0];
        float l = sqrtf(fn[3 * f] * fn[3 * f] + fn[3 * f + 1] * fn[3 * f + 1] + fn[3 * f + 2] * fn[3 * f + 2]);
        for (int k = 0; k < 3; ++k) fn[3 * f + k] /= l;
      }
      for (int v = 0; v < nv; ++v) {
        ring_ptr[v] = m;
        double cum = 0;
        for (int f = 0; f < nf; ++f)
          if (F[3 * f] == v || F[3 * f + 1] == v || F[3 * f + 2] == v) {
            ring_tri[m] = f;
            cum += 1.0;
            ring_cum[m++] = cum;
          }
      }
      ring_ptr[nv] = m;
      int32_t sel[N];
      for (int i = 0; i < N; ++i) sel[i] = (7 * i) % nv;
      orc_estimate(s, 1, 0, N, sel, NULL, NULL, NULL, NULL, ring_ptr, ring_tri, ring_cum, fn, rowptr, col, val, K,
                   W, 3, 1e-3, 0.05, 1e-6, 1e-7, 64, 2, 0, 2, acc, acc2, q, esc, cap, disc, NULL, NULL, NULL, NULL,
                   NULL, NULL, NULL, NULL, 0, 0, 0.0, 0.0, 0);
      /* point basis: k nearest of the row points with Gaussian weights */
      double kx[3 * N], kn[3 * N];
      for (int i = 0; i < 3 * N; ++i) { kx[i] = p[i]; kn[i] = n[i]; }
      orc_estimate(s, 0, 0, N, NULL, p, n, tri, bary, NULL, NULL, NULL, NULL, NULL, NULL, NULL, N, W, 0, 1e-3,
                   0.05, 1e-6, 1e-7, 64, 2, 0, 2, acc2, acc, q, esc, cap, disc, NULL, NULL, NULL, NULL, NULL, NULL,
                   kx, kn, N, 4, 0.3, 0.5, 0);
    }
    double S[K * K], Qm[K * K], rad[N], Z[N];
    int64_t nqr[N];
    orc_psd_estimate(s, N, p, n, tri, bary, w, tab, K, 4, 2.5 * M_PI / 180, 0.5, 10, 1e-4, 1e-6, 1e-7, 200, 3, 0,
                     2, S, Qm, rad, Z, nqr, NULL, NULL, NULL, NULL);
    orc_scene_destroy(s);
  }
  double centre[3] = {0.05, -0.1, 0.02};
  void* k = orc_kelvin_create(V, nv, F, nf, centre);
  double Sj[K * K], Qj[K * K], Sk[K * K], Qk[K * K], rad[N], Z[N];
  int64_t nqr[N], kq = 0;
  orc_kelvin_estimate(k, N, p, n, tri, bary, w, tab, K, 4, 64, 2.5 * M_PI / 180, 0.4, 10, 1e-4, 1e-6, 1e-7, 200, 3,
                      0, 2, Sj, Qj, Sk, Qk, rad, Z, nqr, &kq, NULL, NULL, NULL);
  orc_kelvin_destroy(k);
  printf("oracle driver: ok (%lld killing-walk queries)\n", (long long)kq);
  return 0;
}
