// Layouts and launchers of the Kelvin-inverted exterior estimate (kelvin.hip).
#pragma once
#include "msk_internal.h"

namespace msk {

// Exterior estimate in the Kelvin-inverted domain (kelvin.hip): an element is
// a mesh triangle given by its vertices relative to the inversion centre
// (FP64), in BVH leaf order, with its original index.
struct KelvinTri {
  double a[3], b[3], c[3];  // vertices relative to the inversion centre
  double n[3];              // unit normal of the triangle's plane n . y = cpl (if has_plane)
  double cpl;
  double M2;                // largest squared vertex norm
  int32_t orig;
  int32_t has_plane;        // 0 for a (numerically) degenerate triangle: arcs only
};
static_assert(sizeof(KelvinTri) == 120, "inverted element record must be 120 bytes");
// The part of an element's distance that does not depend on the query point,
// per edge (a, b), (b, c), (c, a) from P to Q: e = Q - P, ee = |e|^2,
// pqmax = max(|P|^2, |Q|^2), and by kind: 1, an arc (the line misses the
// centre): m the unit normal of the plane (0, P, Q), c and rho the image
// circle's centre and radius; 2, a straight segment (the line through the
// centre): m = image(Q) - image(P), rho = |m|^2; 0, a degenerate edge (its
// end points only).
struct KelvinEdge {
  double e[3];
  double ee;
  double m[3];
  double c[3];
  double rho;
  double pqmax;
  int32_t kind;
  int32_t pad;
};
struct KelvinPre {
  double k[3][3];       // images of the vertices a, b, c
  KelvinEdge edge[3];
};
static_assert(sizeof(KelvinPre) == 384, "prepared element record must be 384 bytes");
struct KelvinDev {
  const Node4* nodes;      // 4-wide hierarchy over boxes containing the inverted elements
  const KelvinTri* tris;
  const KelvinPre* pre;    // prepared records, same order as tris
  int64_t n_tris;
  double radius;           // bound of the inverted domain (max |x~| on its boundary)
  double eps2;             // shell width squared (inverted units)
  double kappa, delta;     // step radius d (1 - kappa) - delta
  int64_t max_steps;
  uint32_t mesh_id, seed_lo, seed_hi;
  // the nearest element of the origin, where every killing walk starts (one
  // query for all of them; near the middle of a round shape every element is
  // almost equally near and that query visits most of the hierarchy)
  int32_t origin_known, origin_orig;
  double origin_d2, origin_q[3], origin_l[3];
};
hipError_t launch_kelvin_tangent(const KelvinDev& K, const double* st, const double* nt, int64_t n_rows, double r_max,
                                 int32_t iters, double tol, double* radius, unsigned long long* queries,
                                 hipStream_t s);
hipError_t launch_kelvin_walks(const KelvinDev& K, const double* st, const double* nt, const double* radius,
                               int64_t n_rows, int64_t pairs, double u0, int64_t n_kill, int32_t* log_status,
                               int32_t* log_tri, float* log_bary, int32_t* log_q, double* g,
                               unsigned long long* row_queries, unsigned long long* kill_queries,
                               unsigned long long* next_walk, unsigned long long* stats, int grid, hipStream_t s);
// stats: null for the timed kernel, else 3 counters that the counting
// instantiation adds its node visits, element tests and FP64 operations to
// Plane of a triangle for its inverted element (unit normal n, offset n . a);
// false for a numerically degenerate triangle.
__host__ __device__ bool kelvin_plane(const double a[3], const double b[3], const double c[3], double n[3],
                                      double& cpl);
// The prepared records of n elements (device arrays, leaf order).
hipError_t launch_kelvin_prepare(const KelvinTri* tris, int64_t n, KelvinPre* pre, hipStream_t s);
hipError_t launch_kelvin_closest(const KelvinDev& K, const double* Q, int64_t nq, int32_t* tri, double* d2,
                                 double* qpt, double* bary, hipStream_t s);

}  // namespace msk
