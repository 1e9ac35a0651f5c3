// The exterior estimate in the Kelvin-inverted domain (Sec. 3.3, The Kelvin
// Transform; eqs. exterior-jump-kernel-final, killing-measure-poisson-kernel,
// main-exterior-estimator; Sec. 4, spherical triangular elements).
//
// Coordinates are relative to an inversion centre inside the shape. The map
// x -> x / |x|^2 sends the unbounded exterior to a bounded domain whose
// boundary is the image of the mesh: each planar triangle becomes a piece of
// a sphere through the origin (or of the plane itself when it passes through
// the centre), bounded by three circular arcs, the images of its edges. Walks
// in that domain always end, so Walk-on-Spheres applies with the exact
// distance to these curved elements. Everything here is FP64: element
// spheres of triangles whose planes pass near the centre have huge radii,
// and the distance is written stably in that limit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "msk_internal.h"
#include "kelvin.h"
#include "philox.h"

// wavefronts per SIMD the persistent walk kernel is compiled for
#ifndef MSK_KELVIN_WAVES_PER_EU
#define MSK_KELVIN_WAVES_PER_EU 4
#endif
// the walks' launch: streaming (one hierarchy node per loop trip, 1) or one
// whole search per loop trip (0)
#ifndef MSK_KELVIN_STREAM
#define MSK_KELVIN_STREAM 1
#endif
// the streaming launch's leaf elements: tested across the wavefront (1) or
// by each lane for its own search (0)
#ifndef MSK_KELVIN_COOP
#define MSK_KELVIN_COOP 1
#endif

namespace msk {

namespace {

// The element distance is evaluated exactly as written, with no fused
// multiply-adds, in these helpers as in the functions that use them: the
// result then does not depend on how the compiler inlines them.
__host__ __device__ __forceinline__ double dot(const double a[3], const double b[3]) {
#pragma clang fp contract(off)
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

__host__ __device__ __forceinline__ void invert(const double x[3], double y[3]) {
#pragma clang fp contract(off)
  const double s = 1.0 / dot(x, x);
  y[0] = x[0] * s; y[1] = x[1] * s; y[2] = x[2] * s;
}

__host__ __device__ __forceinline__ void cross(const double u[3], const double v[3], double o[3]) {
#pragma clang fp contract(off)
  o[0] = u[1] * v[2] - u[2] * v[1];
  o[1] = u[2] * v[0] - u[0] * v[2];
  o[2] = u[0] * v[1] - u[1] * v[0];
}

// Offer a candidate point q at squared distance d2 with barycentrics l.
struct Best {
  double d2;
  double q[3];
  double l[3];
};
__host__ __device__ __forceinline__ void offer(Best& b, double d2, const double q[3], double l0, double l1, double l2) {
  if (d2 < b.d2) {
    b.d2 = d2;
    b.q[0] = q[0]; b.q[1] = q[1]; b.q[2] = q[2];
    b.l[0] = l0; b.l[1] = l1; b.l[2] = l2;
  }
}

// The image of the edge [P, Q] (primal, relative to the centre): end points,
// and the nearest point of the arc. The line through P and Q, at foot point f
// from the centre, maps to the circle through the origin in the plane of
// (0, P, Q) with centre f / (2 |f|^2) and radius 1 / (2 |f|); the circle
// point nearest to x is the radial projection of x's in-plane position, and
// it lies on the edge's arc when its image is between P and Q. A line
// through the centre maps to itself: the arc is then the straight segment
// between the end points' images. Everything that does not depend on x is
// computed once per inverted mesh (edge_prepare, kelvin_prepare_kernel);
// edge_eval does the rest, with the same operations in the same order as
// one function evaluating both would. (ia, ib) are the edge's vertex slots.
__host__ __device__ void edge_prepare(const double P[3], const double Q[3], KelvinEdge& E) {
#pragma clang fp contract(off)
  double kp[3], kq[3];
  invert(P, kp);
  invert(Q, kq);
  for (int k = 0; k < 3; ++k) E.e[k] = Q[k] - P[k];
  E.ee = dot(E.e, E.e);
  E.kind = 0;
  E.pad = 0;
  for (int k = 0; k < 3; ++k) E.m[k] = E.c[k] = 0.0;
  E.rho = 0.0;
  E.pqmax = fmax(dot(P, P), dot(Q, Q));
  if (!(E.ee > 0.0)) return;
  const double tf = -dot(P, E.e) / E.ee;
  const double f[3] = {P[0] + tf * E.e[0], P[1] + tf * E.e[1], P[2] + tf * E.e[2]};
  const double ff = dot(f, f);
  double m[3];
  cross(P, Q, m);
  const double mm = dot(m, m);
  if (ff > 1e-24 * E.pqmax && mm > 0.0) {
    E.kind = 1;
    const double ml = 1.0 / sqrt(mm);
    for (int k = 0; k < 3; ++k) E.m[k] = m[k] * ml;
    for (int k = 0; k < 3; ++k) E.c[k] = f[k] / (2.0 * ff);
    E.rho = 1.0 / (2.0 * sqrt(ff));
  } else {
    E.kind = 2;
    for (int k = 0; k < 3; ++k) E.m[k] = kq[k] - kp[k];  // the segment's direction g
    E.rho = dot(E.m, E.m);                               // |g|^2
  }
}

// FP64 operations are counted (kCount) as additions, multiplications,
// divisions and square roots, one each, up to each exit: dot 5, inversion 9.
template <bool kCount>
__host__ __device__ void edge_eval(const double x[3], const double P[3], const double kp[3], const double kq[3],
                                   const KelvinEdge& E, int ia, int ib, Best& b, uint64_t& ops) {
#pragma clang fp contract(off)
  double d[3];
  double l[3] = {0.0, 0.0, 0.0};
  for (int k = 0; k < 3; ++k) d[k] = x[k] - kp[k];
  l[ia] = 1.0;
  offer(b, dot(d, d), kp, l[0], l[1], l[2]);
  for (int k = 0; k < 3; ++k) d[k] = x[k] - kq[k];
  l[ia] = 0.0; l[ib] = 1.0;
  offer(b, dot(d, d), kq, l[0], l[1], l[2]);
  if constexpr (kCount) ops += 16;
  if (E.kind == 0) return;
  if (E.kind == 1) {
    const double* m = E.m;
    const double* c = E.c;
    const double mx = dot(m, x);
    const double u[3] = {x[0] - mx * m[0] - c[0], x[1] - mx * m[1] - c[1], x[2] - mx * m[2] - c[2]};
    const double ul = sqrt(dot(u, u));
    if constexpr (kCount) ops += 20;
    if (!(ul > 0.0)) return;
    const double pt[3] = {c[0] + E.rho * u[0] / ul, c[1] + E.rho * u[1] / ul, c[2] + E.rho * u[2] / ul};
    // the origin is the image of the line's point at infinity: every point of
    // the segment's image lies at least 1 / max(|P|, |Q|) from it
    if constexpr (kCount) ops += 15;
    if (!(dot(pt, pt) * E.pqmax >= 1.0 - 1e-9)) return;
    double y[3];
    invert(pt, y);
    const double yd[3] = {y[0] - P[0], y[1] - P[1], y[2] - P[2]};
    const double t = dot(yd, E.e) / E.ee;
    if constexpr (kCount) ops += 18;
    if (t >= 0.0 && t <= 1.0) {
      if constexpr (kCount) ops += 9;
      for (int k = 0; k < 3; ++k) d[k] = x[k] - pt[k];
      l[ia] = 1.0 - t; l[ib] = t;
      offer(b, dot(d, d), pt, l[0], l[1], l[2]);
    }
  } else {
    const double* g = E.m;
    const double gg = E.rho;
    double s = gg > 0.0 ? ((x[0] - kp[0]) * g[0] + (x[1] - kp[1]) * g[1] + (x[2] - kp[2]) * g[2]) / gg : 0.0;
    s = fmin(1.0, fmax(0.0, s));
    const double pt[3] = {kp[0] + s * g[0], kp[1] + s * g[1], kp[2] + s * g[2]};
    double y[3];
    invert(pt, y);
    const double yd[3] = {y[0] - P[0], y[1] - P[1], y[2] - P[2]};
    const double t = dot(yd, E.e) / E.ee;
    for (int k = 0; k < 3; ++k) d[k] = x[k] - pt[k];
    l[ia] = 1.0 - t; l[ib] = t;
    offer(b, dot(d, d), pt, l[0], l[1], l[2]);
    if constexpr (kCount) ops += 42;
  }
}

}  // namespace

// The plane of triangle (a, b, c) as used by the distance below: unit normal
// n and offset cpl = n . a, or false for a (numerically) degenerate triangle.
__host__ __device__ bool kelvin_plane(const double a[3], const double b[3], const double c[3], double n[3],
                                      double& cpl) {
#pragma clang fp contract(off)
  double ab[3], ac[3];
  for (int k = 0; k < 3; ++k) {
    ab[k] = b[k] - a[k];
    ac[k] = c[k] - a[k];
  }
  cross(ab, ac, n);
  const double nl = sqrt(dot(n, n));
  if (!(nl > 1e-12 * fmax(dot(ab, ab), dot(ac, ac)))) return false;
  for (int k = 0; k < 3; ++k) n[k] /= nl;
  cpl = dot(n, a);
  return true;
}

// Squared distance from x to the image of triangle T, its nearest point and
// the barycentrics of that point's image in T. The triangle's plane
// n . y = c maps to the sphere through the origin with centre n / (2c) and
// radius 1 / (2|c|); with v = c x - n/2 the signed distance of x to it is
// (|c| |x|^2 - sign(c) n . x) / (|v| + 1/2) and the radial projection moves x
// by that distance along sign(c) v / |v|, which tends to the plane's own
// projection as c -> 0. The projection belongs to the patch when its image
// lies in T; otherwise the nearest point is on the patch's boundary (distance
// to a sphere's points grows with their angle from the radial projection).
// Every point of the patch lies on that sphere (or plane), so its distance
// bounds the patch's from below: when its square exceeds `bound` (with a
// relative margin for rounding) the element cannot come nearer than bound and
// INFINITY is returned without the boundary arcs.
template <bool kCount>
__host__ __device__ double kelvin_tri_d2_t(const double x[3], const KelvinTri& T, const KelvinPre& R, double q[3],
                                           double l[3], double bound, uint64_t& ops, double* skip2 = nullptr) {
#pragma clang fp contract(off)
  if (skip2) *skip2 = -INFINITY;  // no plane: never skipped
  Best b;
  b.d2 = INFINITY;
  if (T.has_plane) {
    const double* n = T.n;
    const double c = T.cpl;
    double p[3];
    if (c != 0.0) {
      const double sg = c > 0.0 ? 1.0 : -1.0;
      const double v[3] = {c * x[0] - 0.5 * n[0], c * x[1] - 0.5 * n[1], c * x[2] - 0.5 * n[2]};
      const double vl = sqrt(dot(v, v));
      const double sd = (fabs(c) * dot(x, x) - sg * dot(n, x)) / (vl + 0.5);
      if constexpr (kCount) ops += 32;
      if (skip2) *skip2 = sd * sd;  // the value compared with the bound
      if (sd * sd > bound * (1.0 + 1e-9)) return INFINITY;
      for (int k = 0; k < 3; ++k) p[k] = x[k] - sd * sg * v[k] / vl;
      if constexpr (kCount) ops += 10;
    } else {
      const double nx = dot(n, x);
      if constexpr (kCount) ops += 7;
      if (skip2) *skip2 = nx * nx;
      if (nx * nx > bound * (1.0 + 1e-9)) return INFINITY;
      for (int k = 0; k < 3; ++k) p[k] = x[k] - nx * n[k];
      if constexpr (kCount) ops += 6;
    }
    if constexpr (kCount) ops += 6;
    if (dot(p, p) * T.M2 >= 1.0 - 1e-9) {  // image points lie at least 1 / max|vertex| from the origin
      double y[3], ay[3], w[3], ab[3], ac[3], nn[3];
      invert(p, y);
      for (int k = 0; k < 3; ++k) {
        ay[k] = y[k] - T.a[k];
        ab[k] = T.b[k] - T.a[k];
        ac[k] = T.c[k] - T.a[k];
      }
      // barycentrics of y's projection on the plane
      cross(ab, ac, nn);
      const double nl = dot(nn, n);
      cross(ay, ac, w);
      const double l1 = dot(w, n) / nl;
      cross(ab, ay, w);
      const double l2 = dot(w, n) / nl;
      const double l0 = 1.0 - l1 - l2;
      if constexpr (kCount) ops += 64;
      if (l0 >= 0.0 && l1 >= 0.0 && l2 >= 0.0) {
        const double d[3] = {x[0] - p[0], x[1] - p[1], x[2] - p[2]};
        offer(b, dot(d, d), p, l0, l1, l2);
        if constexpr (kCount) ops += 8;
      }
    }
  }
  edge_eval<kCount>(x, T.a, R.k[0], R.k[1], R.edge[0], 0, 1, b, ops);
  edge_eval<kCount>(x, T.b, R.k[1], R.k[2], R.edge[1], 1, 2, b, ops);
  edge_eval<kCount>(x, T.c, R.k[2], R.k[0], R.edge[2], 2, 0, b, ops);
  q[0] = b.q[0]; q[1] = b.q[1]; q[2] = b.q[2];
  l[0] = b.l[0]; l[1] = b.l[1]; l[2] = b.l[2];
  return b.d2;
}

__host__ __device__ double kelvin_tri_d2(const double x[3], const KelvinTri& T, const KelvinPre& R, double q[3],
                                         double l[3], double bound) {
  uint64_t none = 0;
  return kelvin_tri_d2_t<false>(x, T, R, q, l, bound, none);
}

// The point-independent part of every element (leaf order): the images of
// its vertices and its edges' constants.
__global__ void kelvin_prepare_kernel(const KelvinTri* __restrict__ tris, int64_t n, KelvinPre* __restrict__ pre) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const KelvinTri& T = tris[s];
  KelvinPre R;
  invert(T.a, R.k[0]);
  invert(T.b, R.k[1]);
  invert(T.c, R.k[2]);
  edge_prepare(T.a, T.b, R.edge[0]);
  edge_prepare(T.b, T.c, R.edge[1]);
  edge_prepare(T.c, T.a, R.edge[2]);
  pre[s] = R;
}

// Work of the counting instantiation of the nearest search.
struct KelvinWork {
  uint64_t nodes = 0, elements = 0, ops = 0;
};

// Exact nearest inverted element: lexicographic minimum of (squared distance,
// original index), depth first over the 4-wide hierarchy of boxes that
// contain the elements (FP32 boxes rounded outward; their FP64 lower bounds
// are within the boxes' own rounding of the true distance, hence the small
// relative margin). `slot` names a candidate element on entry (warm start:
// a walk's previous nearest, tested first so that the search starts with a
// finite bound; -1 for none) and receives the nearest one's slot. The
// minimum, and the element that attains it, do not depend on the candidate.
template <bool kCount>
__host__ __device__ double kelvin_nearest_t(const KelvinDev& K, const double x[3], int32_t& orig, double q[3],
                                            double l[3], KelvinWork& work, int32_t& slot) {
  double best = INFINITY;
  orig = INT_MAX;
  int32_t best_slot = -1;
  if (slot >= 0) {
    const KelvinTri& T = K.tris[slot];
    if constexpr (kCount) ++work.elements;
    best = kelvin_tri_d2_t<kCount>(x, T, K.pre[slot], q, l, best, work.ops);
    orig = T.orig;
    best_slot = slot;
  }
  int32_t stk[kStackDepth];
  double stl[kStackDepth];
  int sp = 0;
  int32_t node = 0;
  while (true) {
    const Node4& N = K.nodes[node];
    double lb[4];
    int32_t cc[4], cn[4];
    if constexpr (kCount) {  // four box lower bounds: 6 differences, 6 maxima, 3 products, 2 sums each
      ++work.nodes;
      work.ops += 4 * 17;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const double gx = fmax(fmax((double)N.lox[k] - x[0], x[0] - (double)N.hix[k]), 0.0);
      const double gy = fmax(fmax((double)N.loy[k] - x[1], x[1] - (double)N.hiy[k]), 0.0);
      const double gz = fmax(fmax((double)N.loz[k] - x[2], x[2] - (double)N.hiz[k]), 0.0);
      lb[k] = gx * gx + gy * gy + gz * gz;
      cc[k] = N.child[k];
      cn[k] = N.count[k];
    }
    // nearest first
#pragma unroll
    for (int i = 1; i < 4; ++i)
      for (int j = i; j > 0 && lb[j] < lb[j - 1]; --j) {
        const double t = lb[j]; lb[j] = lb[j - 1]; lb[j - 1] = t;
        const int32_t a = cc[j]; cc[j] = cc[j - 1]; cc[j - 1] = a;
        const int32_t c = cn[j]; cn[j] = cn[j - 1]; cn[j - 1] = c;
      }
    int32_t next = -1;
    double next_lb = 0.0;
    for (int k = 0; k < 4; ++k) {
      if (!(lb[k] <= best * (1.0 + 1e-12))) continue;
      if (cc[k] < 0 && cn[k] > 0) {
        const int32_t first = -cc[k] - 1;
        for (int32_t s = first; s < first + cn[k]; ++s) {
          const KelvinTri& T = K.tris[s];
          double qq[3], ll[3];
          if constexpr (kCount) ++work.elements;
          const double d = kelvin_tri_d2_t<kCount>(x, T, K.pre[s], qq, ll, best, work.ops);
          if (d < best || (d == best && T.orig < orig)) {
            best = d;
            orig = T.orig;
            best_slot = s;
            q[0] = qq[0]; q[1] = qq[1]; q[2] = qq[2];
            l[0] = ll[0]; l[1] = ll[1]; l[2] = ll[2];
          }
        }
      }
    }
    // the nearest surviving inner child is next, the others wait on the
    // stack (farthest first) with their bounds
    for (int k = 3; k >= 0; --k) {
      if (cc[k] >= 0 && lb[k] <= best * (1.0 + 1e-12)) {
        if (next >= 0 && sp < kStackDepth) {
          stk[sp] = next;
          stl[sp] = next_lb;
          ++sp;
        }
        next = cc[k];
        next_lb = lb[k];
      }
    }
    if (next >= 0) {
      node = next;
      continue;
    }
    node = -1;
    while (sp > 0) {
      --sp;
      if (stl[sp] <= best * (1.0 + 1e-12)) {
        node = stk[sp];
        break;
      }
    }
    if (node < 0) break;
  }
  slot = best_slot;
  return best;
}

__host__ __device__ double kelvin_nearest(const KelvinDev& K, const double x[3], int32_t& orig, double q[3], double l[3]) {
  KelvinWork none;
  int32_t cold = -1;
  return kelvin_nearest_t<false>(K, x, orig, q, l, none, cold);
}


// Whether some inverted element lies nearer to x than t (its distance, the
// square root of the exact squared distance, below t): the decision the
// tangent-ball bisection needs, equal to comparing the nearest element's
// distance with t. Boxes and element spheres farther than t (with a small
// relative margin for their own rounding) are skipped, and the search stops
// at the first element found, so a point far from every element costs a few
// box tests instead of a full nearest search.
__host__ __device__ bool kelvin_any_within(const KelvinDev& K, const double x[3], double t) {
  if (!(t > 0.0)) return false;
  const double t2 = t * t * (1.0 + 1e-9);
  int32_t stk[kStackDepth];
  int sp = 0;
  int32_t node = 0;
  while (true) {
    const Node4& N = K.nodes[node];
    for (int k = 0; k < 4; ++k) {
      const double gx = fmax(fmax((double)N.lox[k] - x[0], x[0] - (double)N.hix[k]), 0.0);
      const double gy = fmax(fmax((double)N.loy[k] - x[1], x[1] - (double)N.hiy[k]), 0.0);
      const double gz = fmax(fmax((double)N.loz[k] - x[2], x[2] - (double)N.hiz[k]), 0.0);
      if (!(gx * gx + gy * gy + gz * gz <= t2)) continue;
      const int32_t cc = N.child[k], cn = N.count[k];
      if (cc < 0) {
        const int32_t first = -cc - 1;
        for (int32_t e = first; e < first + cn; ++e) {
          double qq[3], ll[3];
          const double d2 = kelvin_tri_d2(x, K.tris[e], K.pre[e], qq, ll, t2);
          if (sqrt(d2) < t) return true;
        }
      } else if (sp < kStackDepth) {
        stk[sp++] = cc;
      }
    }
    if (sp == 0) return false;
    node = stk[--sp];
  }
}
namespace {

__device__ __forceinline__ void frame(const double n[3], double e1[3], double e2[3]) {
  const double sg = n[2] >= 0.0 ? 1.0 : -1.0;
  const double a = -1.0 / (sg + n[2]);
  const double b = n[0] * n[1] * a;
  e1[0] = 1.0 + sg * n[0] * n[0] * a; e1[1] = sg * b; e1[2] = -sg * n[0];
  e2[0] = b; e2[1] = sg + n[1] * n[1] * a; e2[2] = -n[1];
}

// The move of step k from x at squared distance d2 to the surface: a uniform
// point of the sphere of radius d (1 - kappa) - delta, drawn from the Philox
// block (row, walk, k, step purpose).
__device__ __forceinline__ void kelvin_move(const KelvinDev& K, uint32_t row, uint32_t walk, int64_t k, double d2,
                                            double x[3]) {
#pragma clang fp contract(off)
  const uint4 u = philox10(make_uint4(row, walk, (uint32_t)k, (kPurposeStep << 24) | (K.mesh_id & 0xFFFFFFu)),
                           K.seed_lo, K.seed_hi);
  const double u0 = unit_f(u.x), u1 = unit_f(u.y);
  const double r = sqrt(d2) * (1.0 - K.kappa) - K.delta;
  const double z = 1.0 - 2.0 * u0;
  const double rxy = 2.0 * sqrt(u0 * (1.0 - u0));
  double sp, cp;
  sincospi(2.0 * u1, &sp, &cp);
  x[0] += r * rxy * cp;
  x[1] += r * rxy * sp;
  x[2] += r * z;
}

// One step of Walk-on-Spheres in the inverted domain at x: the exact
// nearest element; in the eps-shell the walk has hit (true), else x moves to
// a uniform point of the sphere of radius d (1 - kappa) - delta, drawn from
// the Philox block (row, walk, k, step purpose), the oracle's streams.
template <bool kCount>
__device__ bool kelvin_step(const KelvinDev& K, uint32_t row, uint32_t walk, int64_t k, double x[3], int32_t& orig,
                            double q[3], double l[3], bool at_origin, KelvinWork& work, int32_t& warm) {
  double d2;
  if (at_origin) {  // the first step of a killing walk: the shared answer
    d2 = K.origin_d2;
    orig = K.origin_orig;
    for (int c = 0; c < 3; ++c) {
      q[c] = K.origin_q[c];
      l[c] = K.origin_l[c];
    }
  } else {
    d2 = kelvin_nearest_t<kCount>(K, x, orig, q, l, work, warm);
  }
  if (d2 < K.eps2) return true;
  kelvin_move(K, row, walk, k, d2, x);
  return false;
}

}  // namespace

// Largest ball in the inverted domain touching its boundary at s~_i (unit
// normal n~_i pointing out of the domain): bisection over [0, r_max], a
// radius accepted when the centre c = s~ - r n~ is at least r - min(tol,
// r/1024) from the inverted surface and the ball lies within the domain's
// bound. Three levels per round: the eight lanes of a row evaluate the (up
// to) seven midpoints of the next three levels at once (lane k takes heap
// node k of that subtree: node 1 the current midpoint, nodes 2k and 2k + 1
// the midpoints of its halves), then all follow the path the sequential
// bisection takes through them. Every midpoint is formed by the operations of
// the sequential loop, so the radius is that loop's; the rounds of dependent
// searches drop from iters to ceil(iters / 3), and eight lanes per row fill
// the GPU. queries[i] counts the iters decisions.
__global__ void __launch_bounds__(64) kelvin_tangent_kernel(KelvinDev K, const double* __restrict__ st,
                                                            const double* __restrict__ nt, int64_t n_rows,
                                                            double r_max, int32_t iters, double tol,
                                                            double* __restrict__ radius,
                                                            unsigned long long* __restrict__ queries) {
#pragma clang fp contract(off)
  const int lane = threadIdx.x & 63, sub = lane & 7, gbase = lane & ~7;
  // eight rows per 64-lane workgroup; the loop bound is uniform over the
  // workgroup, so every lane takes part in every ballot
  for (int64_t base = (int64_t)blockIdx.x * 8; base < n_rows; base += (int64_t)gridDim.x * 8) {
    const int64_t i = base + (threadIdx.x >> 3);
    const bool valid = i < n_rows;
    double s[3] = {0.0, 0.0, 0.0}, n[3] = {0.0, 0.0, 0.0};
    if (valid)
      for (int c = 0; c < 3; ++c) {
        s[c] = st[3 * i + c];
        n[c] = nt[3 * i + c];
      }
    double lo = 0.0, hi = r_max;
    for (int32_t done = 0; done < iters;) {
      const int levels = min(3, iters - done);
      bool res = false;
      if (valid && sub >= 1 && sub < (1 << levels)) {
        double a = lo, b = hi;
        const int depth = 31 - __clz(sub);  // bits of the node index below its leading one
        for (int j = depth - 1; j >= 0; --j) {
          const double m = 0.5 * (a + b);
          if ((sub >> j) & 1)
            a = m;
          else
            b = m;
        }
        const double mid = 0.5 * (a + b);
        const double c[3] = {s[0] - mid * n[0], s[1] - mid * n[1], s[2] - mid * n[2]};
        const double t = mid - fmin(tol, mid * (1.0 / 1024.0));
        res = sqrt(dot(c, c)) + mid <= K.radius && !kelvin_any_within(K, c, t);
      }
      const unsigned long long mask = __ballot(res);  // every lane of the wavefront takes part
      int node = 1;
      for (int l = 0; l < levels; ++l) {
        const double mid = 0.5 * (lo + hi);
        const int bit = (int)((mask >> (gbase + node)) & 1ull);
        if (bit)
          lo = mid;
        else
          hi = mid;
        node = 2 * node + bit;
      }
      done += levels;
    }
    if (valid && sub == 0) {
      radius[i] = lo;
      queries[i] = (unsigned long long)iters;
    }
  }
}

// Walks [0, n_rows 2 pairs) are the jump term's: walk 2j + a of row i starts
// at point a of antithetic pair j on the row's tangent ball, drawn with
// density proportional to the ball jump kernel outside the cap
// (u = sin(theta/2) with density ~ 1/u^2 on [u0, 1], inverted in closed form;
// azimuth uniform, + pi for the partner). The next n_kill walks are the
// killing term's, from the origin (the image of infinity), with Philox row
// 0xFFFFFFFF and walk index k. The launch is persistent: every lane claims
// walks one at a time from a counter and advances its walk by one step per
// loop trip, so a lane whose walk ends takes the next one at once instead of
// idling until the longest walk of its wavefront ends; each walk's result
// depends on its index only. Each walk logs its status, terminal original
// triangle, the barycentrics of that triangle's vertices 1 and 2 at the
// terminal point's image, its query count, and the factor g = 1/|t~| of its
// rank-one update.
// The counting instantiation (kCount) runs the same walks and adds the
// nearest searches' node visits, element tests and FP64 operations to
// stats[0..2].
template <bool kCount>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MSK_KELVIN_WAVES_PER_EU)))
kelvin_walk_kernel(
    KelvinDev K, const double* __restrict__ st, const double* __restrict__ nt, const double* __restrict__ radius,
    int64_t n_rows, int64_t pairs, double u0, int64_t n_kill, int32_t* __restrict__ log_status,
    int32_t* __restrict__ log_tri, float* __restrict__ log_bary, int32_t* __restrict__ log_q, double* __restrict__ g,
    unsigned long long* __restrict__ row_queries, unsigned long long* kill_queries, unsigned long long* next_walk,
    unsigned long long* __restrict__ stats) {
  const int64_t n_jump = n_rows * 2 * pairs, total = n_jump + n_kill;
  KelvinWork work;
  int32_t warm = -1;  // slot of the walk's previous nearest element
  int64_t id = -1, i = -1, k = 0;
  uint32_t row = 0, walk = 0;
  double x[3] = {0.0, 0.0, 0.0}, q[3] = {0.0, 0.0, 0.0}, l[3] = {0.0, 0.0, 0.0};
  int32_t orig = -1;
  while (true) {
    if (id < 0) {  // claim the next walk
      id = (int64_t)atomicAdd(next_walk, 1ull);
      if (id >= total) break;
      k = 0;
      orig = -1;
      warm = -1;
      if (id < n_jump) {
        i = id / (2 * pairs);
        const int64_t w = id - i * 2 * pairs;
        const double r = radius[i];
        if (!(r > 0.0)) {
          log_status[id] = -1;
          log_tri[id] = -1;
          log_bary[2 * id] = log_bary[2 * id + 1] = 0.0f;
          log_q[id] = 0;
          g[id] = 0.0;
          id = -1;
          continue;
        }
        row = (uint32_t)i;
        walk = (uint32_t)w;
        const uint4 u = philox10(
            make_uint4(row, (uint32_t)(w >> 1), 0u, (kPurposeBall << 24) | (K.mesh_id & 0xFFFFFFu)), K.seed_lo,
            K.seed_hi);
        const double xi = unit_f(u.x), eta = unit_f(u.y);
        const double su = 1.0 / (1.0 / u0 - xi * (1.0 / u0 - 1.0));
        const double ct = 1.0 - 2.0 * su * su, sn = 2.0 * su * sqrt(fmax(0.0, 1.0 - su * su));
        double sp, cp;
        sincospi(2.0 * eta + ((w & 1) ? 1.0 : 0.0), &sp, &cp);
        const double n[3] = {nt[3 * i], nt[3 * i + 1], nt[3 * i + 2]};
        double e1[3], e2[3];
        frame(n, e1, e2);
        for (int c3 = 0; c3 < 3; ++c3) {
          const double c = st[3 * i + c3] - r * n[c3];
          x[c3] = c + r * (ct * n[c3] + sn * (cp * e1[c3] + sp * e2[c3]));
        }
      } else {
        i = -1;
        row = 0xFFFFFFFFu;
        walk = (uint32_t)(id - n_jump);
        x[0] = x[1] = x[2] = 0.0;
      }
    }
    int32_t status = -1, nq = 0;
    if (k < K.max_steps) {
      if (kelvin_step<kCount>(K, row, walk, k, x, orig, q, l, i < 0 && k == 0 && K.origin_known, work, warm)) {
        status = kHit;
        nq = (int32_t)(k + 1);
      } else {
        ++k;
      }
    } else {  // step cap: the nearest point of the last position
      kelvin_nearest_t<kCount>(K, x, orig, q, l, work, warm);
      status = kCapped;
      nq = (int32_t)(K.max_steps + 1);
    }
    if (status >= 0) {
      log_status[id] = status;
      log_tri[id] = orig;
      log_bary[2 * id] = (float)l[1];
      log_bary[2 * id + 1] = (float)l[2];
      log_q[id] = nq;
      g[id] = 1.0 / sqrt(dot(q, q));
      if (i >= 0)
        atomicAdd(row_queries + i, (unsigned long long)nq);
      else
        atomicAdd(kill_queries, (unsigned long long)nq);
      id = -1;
    }
  }
  if constexpr (kCount) {
    atomicAdd(stats, (unsigned long long)work.nodes);
    atomicAdd(stats + 1, (unsigned long long)work.elements);
    atomicAdd(stats + 2, (unsigned long long)work.ops);
  }
}

// The leaf elements a wavefront's searches reach in one loop trip, tested 64
// at a time across its lanes: the list (element slot, owner lane), each
// owner's query point and bound, and each test's result, in LDS.
struct KelvinCoop {
  double x[64][3];
  double bound[64];
  int32_t slot[64];
  int32_t owner[64];
  double rd[64], rk[64];  // distance, and the value its sphere (plane) skip compares with the bound
  int32_t ro[64], rs[64];
  double rq[64][3], rl[64][3];
};

// Orders a wavefront's LDS accesses as written (the hardware executes one
// wavefront's LDS instructions in issue order; only the compiler must not
// move them).
__device__ __forceinline__ void kelvin_lds_order() { __asm__ __volatile__("" ::: "memory"); }

// Exclusive prefix sum over the wavefront of a count below 64 (bit-sliced
// ballots); `total` receives the wavefront's sum.
__device__ __forceinline__ uint32_t kelvin_wave_prefix(uint32_t v, uint32_t& total) {
  const uint32_t lane = __lane_id();
  const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  uint32_t pre = 0, tot = 0;
#pragma unroll
  for (int b = 0; b < 6; ++b) {
    const uint64_t m = __ballot((v >> b) & 1u);
    pre += (uint32_t)__popcll(m & below) << b;
    tot += (uint32_t)__popcll(m) << b;
  }
  total = tot;
  return pre;
}

// Streaming form of the same walks: every loop trip advances each searching
// lane by one node of the hierarchy (the node's leaf elements tested by that
// lane), so a lane whose search is long does not hold the others; a lane
// whose search ends finishes its step at once (or its walk, logged as above,
// and claims the next one). Each search visits the same nodes in the same
// order as kelvin_nearest_t, from the same warm candidate, so walks and logs
// are those of kelvin_walk_kernel.
template <bool kCount>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MSK_KELVIN_WAVES_PER_EU)))
kelvin_stream_kernel(
    KelvinDev K, const double* __restrict__ st, const double* __restrict__ nt, const double* __restrict__ radius,
    int64_t n_rows, int64_t pairs, double u0, int64_t n_kill, int32_t* __restrict__ log_status,
    int32_t* __restrict__ log_tri, float* __restrict__ log_bary, int32_t* __restrict__ log_q, double* __restrict__ g,
    unsigned long long* __restrict__ row_queries, unsigned long long* kill_queries, unsigned long long* next_walk,
    unsigned long long* __restrict__ stats) {
  const int64_t n_jump = n_rows * 2 * pairs, total = n_jump + n_kill;
  __shared__ KelvinCoop coop[4];
  KelvinCoop* C = &coop[threadIdx.x >> 6];
  const uint32_t lane = __lane_id();
  KelvinWork work;
  int64_t id = -1, i = -1, k = 0;
  uint32_t row = 0, walk = 0;
  double x[3] = {0.0, 0.0, 0.0}, q[3] = {0.0, 0.0, 0.0}, l[3] = {0.0, 0.0, 0.0};
  int32_t orig = -1, warm = -1;
  bool done = false;
  // the search in progress (node < 0: none)
  int32_t stk[kStackDepth];
  double stl[kStackDepth];
  int sp = 0;
  int32_t node = -1, best_slot = -1;
  double best = INFINITY;
  auto search_begin = [&]() {
    best = INFINITY;
    orig = INT_MAX;
    best_slot = -1;
    if (warm >= 0) {
      const KelvinTri& T = K.tris[warm];
      if constexpr (kCount) ++work.elements;
      best = kelvin_tri_d2_t<kCount>(x, T, K.pre[warm], q, l, best, work.ops);
      orig = T.orig;
      best_slot = warm;
    }
    sp = 0;
    node = 0;
  };
  auto log_walk = [&](int32_t status, int32_t nq) {
    log_status[id] = status;
    log_tri[id] = orig;
    log_bary[2 * id] = (float)l[1];
    log_bary[2 * id + 1] = (float)l[2];
    log_q[id] = nq;
    g[id] = 1.0 / sqrt(dot(q, q));
    if (i >= 0)
      atomicAdd(row_queries + i, (unsigned long long)nq);
    else
      atomicAdd(kill_queries, (unsigned long long)nq);
    id = -1;
  };
  // the answer of step k's search (squared distance d2): the walk hits, or
  // moves and starts the next search (the step cap's final search at
  // k = max_steps)
  auto step_done = [&](double d2) {
    if (k >= K.max_steps) {  // the cap's search
      log_walk(kCapped, (int32_t)(K.max_steps + 1));
      return;
    }
    if (d2 < K.eps2) {
      log_walk(kHit, (int32_t)(k + 1));
      return;
    }
    kelvin_move(K, row, walk, k, d2, x);
    ++k;
    search_begin();
  };
  while (true) {
    // lanes without a walk claim the next one
    while (id < 0 && !done) {
      id = (int64_t)atomicAdd(next_walk, 1ull);
      if (id >= total) {
        id = -1;
        done = true;
        break;
      }
      k = 0;
      orig = -1;
      warm = -1;
      if (id < n_jump) {
        i = id / (2 * pairs);
        const int64_t w = id - i * 2 * pairs;
        const double r = radius[i];
        if (!(r > 0.0)) {
          log_status[id] = -1;
          log_tri[id] = -1;
          log_bary[2 * id] = log_bary[2 * id + 1] = 0.0f;
          log_q[id] = 0;
          g[id] = 0.0;
          id = -1;
          continue;
        }
        row = (uint32_t)i;
        walk = (uint32_t)w;
        const uint4 u = philox10(
            make_uint4(row, (uint32_t)(w >> 1), 0u, (kPurposeBall << 24) | (K.mesh_id & 0xFFFFFFu)), K.seed_lo,
            K.seed_hi);
        const double xi = unit_f(u.x), eta = unit_f(u.y);
        const double su = 1.0 / (1.0 / u0 - xi * (1.0 / u0 - 1.0));
        const double ct = 1.0 - 2.0 * su * su, sn = 2.0 * su * sqrt(fmax(0.0, 1.0 - su * su));
        double sp2, cp;
        sincospi(2.0 * eta + ((w & 1) ? 1.0 : 0.0), &sp2, &cp);
        const double n[3] = {nt[3 * i], nt[3 * i + 1], nt[3 * i + 2]};
        double e1[3], e2[3];
        frame(n, e1, e2);
        for (int c3 = 0; c3 < 3; ++c3) {
          const double c = st[3 * i + c3] - r * n[c3];
          x[c3] = c + r * (ct * n[c3] + sn * (cp * e1[c3] + sp2 * e2[c3]));
        }
        search_begin();
      } else {
        i = -1;
        row = 0xFFFFFFFFu;
        walk = (uint32_t)(id - n_jump);
        x[0] = x[1] = x[2] = 0.0;
        if (K.origin_known && K.max_steps > 0) {  // the first step's shared answer
          orig = K.origin_orig;
          for (int c = 0; c < 3; ++c) {
            q[c] = K.origin_q[c];
            l[c] = K.origin_l[c];
          }
          best_slot = -1;
          step_done(K.origin_d2);  // logs, or starts step 1's search
        } else {
          search_begin();
        }
      }
    }
    if (__ballot(id >= 0) == 0) break;  // no lane of the wavefront has a walk left
    const bool srch = id >= 0;
    // one node of each searching lane's search: its four child boxes, nearest first
    double lb[4] = {0.0, 0.0, 0.0, 0.0};
    int32_t cc[4] = {0, 0, 0, 0}, cn[4] = {0, 0, 0, 0};
    if (srch) {
      const Node4& N = K.nodes[node];
      if constexpr (kCount) {
        ++work.nodes;
        work.ops += 4 * 17;
      }
#pragma unroll
      for (int c4 = 0; c4 < 4; ++c4) {
        const double gx = fmax(fmax((double)N.lox[c4] - x[0], x[0] - (double)N.hix[c4]), 0.0);
        const double gy = fmax(fmax((double)N.loy[c4] - x[1], x[1] - (double)N.hiy[c4]), 0.0);
        const double gz = fmax(fmax((double)N.loz[c4] - x[2], x[2] - (double)N.hiz[c4]), 0.0);
        lb[c4] = gx * gx + gy * gy + gz * gz;
        cc[c4] = N.child[c4];
        cn[c4] = N.count[c4];
      }
#pragma unroll
      for (int a = 1; a < 4; ++a)
        for (int b = a; b > 0 && lb[b] < lb[b - 1]; --b) {
          const double t = lb[b]; lb[b] = lb[b - 1]; lb[b - 1] = t;
          const int32_t t1 = cc[b]; cc[b] = cc[b - 1]; cc[b - 1] = t1;
          const int32_t t2 = cn[b]; cn[b] = cn[b - 1]; cn[b - 1] = t2;
        }
    }
#if MSK_KELVIN_COOP
    // the leaf elements within the bound (the trip's starting bound: a test
    // that a tighter bound would have cut short cannot win either), listed in
    // the lane's order and tested 64 at a time by the whole wavefront; each
    // owner then folds its results in that order
    {
      // the children listed, fixed before any fold tightens the bound
      uint32_t nu = 0, qmask = 0;
      if (srch)
        for (int c4 = 0; c4 < 4; ++c4)
          if (lb[c4] <= best * (1.0 + 1e-12) && cc[c4] < 0 && cn[c4] > 0) {
            nu += (uint32_t)cn[c4];
            qmask |= 1u << c4;
          }
      uint32_t total;
      const uint32_t pre = kelvin_wave_prefix(nu, total);
      bool child_ok = false;  // the fold's current child (carried over a round boundary)
      if (total > 0) {
        C->x[lane][0] = x[0];
        C->x[lane][1] = x[1];
        C->x[lane][2] = x[2];
        C->bound[lane] = best;
        for (uint32_t base = 0; base < total; base += 64) {
          if (nu > 0) {
            uint32_t pos = pre;
            for (int c4 = 0; c4 < 4; ++c4) {
              if (!((qmask >> c4) & 1u)) continue;
              const int32_t first = -cc[c4] - 1;
              for (int32_t e = first; e < first + cn[c4]; ++e, ++pos)
                if (pos >= base && pos < base + 64) {
                  C->slot[pos - base] = e;
                  C->owner[pos - base] = (int32_t)lane;
                }
            }
          }
          kelvin_lds_order();
          if (base + lane < total) {
            const int32_t e = C->slot[lane];
            const int32_t o = C->owner[lane];
            const double xo[3] = {C->x[o][0], C->x[o][1], C->x[o][2]};
            const KelvinTri& T = K.tris[e];
            double qq[3], ll[3];
            if constexpr (kCount) ++work.elements;
            double k2;
            const double d = kelvin_tri_d2_t<kCount>(xo, T, K.pre[e], qq, ll, C->bound[o], work.ops, &k2);
            C->rd[lane] = d;
            C->rk[lane] = k2;
            C->ro[lane] = T.orig;
            C->rs[lane] = e;
            for (int c = 0; c < 3; ++c) {
              C->rq[lane][c] = qq[c];
              C->rl[lane][c] = ll[c];
            }
          }
          kelvin_lds_order();
          if (nu > 0) {
            // the owner replays its lane-private order on these results: a
            // child is entered only if its box is still within the bound, an
            // element counts only if its sphere (plane) is (the tests ran with
            // the trip's starting bound, which is never tighter), so the
            // updates are exactly those of the lane-private search
            uint32_t pos = pre;
            for (int c4 = 0; c4 < 4; ++c4) {
              if (!((qmask >> c4) & 1u)) continue;
              const int32_t first = -cc[c4] - 1;
              for (int32_t e = first; e < first + cn[c4]; ++e, ++pos) {
                if (pos < base || pos >= base + 64) continue;
                if (e == first) child_ok = lb[c4] <= best * (1.0 + 1e-12);
                if (!child_ok) continue;
                const uint32_t r = pos - base;
                if (C->rk[r] > best * (1.0 + 1e-9)) continue;  // the lane-private test would have returned INFINITY
                const double d = C->rd[r];
                const int32_t o2 = C->ro[r];
                if (d < best || (d == best && o2 < orig)) {
                  best = d;
                  orig = o2;
                  best_slot = C->rs[r];
                  for (int c = 0; c < 3; ++c) {
                    q[c] = C->rq[r][c];
                    l[c] = C->rl[r][c];
                  }
                }
              }
            }
          }
          kelvin_lds_order();
        }
      }
    }
#endif
    if (!srch) continue;
    {
#if !MSK_KELVIN_COOP
      for (int c4 = 0; c4 < 4; ++c4) {
        if (!(lb[c4] <= best * (1.0 + 1e-12))) continue;
        if (cc[c4] < 0 && cn[c4] > 0) {
          const int32_t first = -cc[c4] - 1;
          for (int32_t e = first; e < first + cn[c4]; ++e) {
            const KelvinTri& T = K.tris[e];
            double qq[3], ll[3];
            if constexpr (kCount) ++work.elements;
            const double d = kelvin_tri_d2_t<kCount>(x, T, K.pre[e], qq, ll, best, work.ops);
            if (d < best || (d == best && T.orig < orig)) {
              best = d;
              orig = T.orig;
              best_slot = e;
              q[0] = qq[0]; q[1] = qq[1]; q[2] = qq[2];
              l[0] = ll[0]; l[1] = ll[1]; l[2] = ll[2];
            }
          }
        }
      }
#endif
      int32_t next = -1;
      double next_lb = 0.0;
      for (int c4 = 3; c4 >= 0; --c4) {
        if (cc[c4] >= 0 && lb[c4] <= best * (1.0 + 1e-12)) {
          if (next >= 0 && sp < kStackDepth) {
            stk[sp] = next;
            stl[sp] = next_lb;
            ++sp;
          }
          next = cc[c4];
          next_lb = lb[c4];
        }
      }
      if (next < 0) {
        while (sp > 0) {
          --sp;
          if (stl[sp] <= best * (1.0 + 1e-12)) {
            next = stk[sp];
            break;
          }
        }
      }
      node = next;
    }
    if (node < 0) {  // the search is answered
      warm = best_slot;
      step_done(best);
    }
  }
  if constexpr (kCount) {
    atomicAdd(stats, (unsigned long long)work.nodes);
    atomicAdd(stats + 1, (unsigned long long)work.elements);
    atomicAdd(stats + 2, (unsigned long long)work.ops);
  }
}

// Nearest inverted element of each query point (inverted space, relative to
// the centre).
__global__ void kelvin_closest_kernel(KelvinDev K, const double* __restrict__ Q, int64_t nq, int32_t* __restrict__ tri,
                                      double* __restrict__ d2, double* __restrict__ qpt, double* __restrict__ bary) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nq) return;
  const double x[3] = {Q[3 * i], Q[3 * i + 1], Q[3 * i + 2]};
  int32_t o;
  double q[3], l[3];
  d2[i] = kelvin_nearest(K, x, o, q, l);
  tri[i] = o;
  for (int k = 0; k < 3; ++k) {
    qpt[3 * i + k] = q[k];
    bary[3 * i + k] = l[k];
  }
}

hipError_t launch_kelvin_tangent(const KelvinDev& K, const double* st, const double* nt, int64_t n_rows, double r_max,
                                 int32_t iters, double tol, double* radius, unsigned long long* queries,
                                 hipStream_t s) {
  if (n_rows <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((n_rows + 7) / 8, 1 << 20);  // eight rows per 64-lane workgroup
  hipLaunchKernelGGL(kelvin_tangent_kernel, dim3((unsigned)blocks), dim3(64), 0, s, K, st, nt, n_rows, r_max, iters,
                     tol, radius, queries);
  return hipGetLastError();
}

hipError_t launch_kelvin_walks(const KelvinDev& K, const double* st, const double* nt, const double* radius,
                               int64_t n_rows, int64_t pairs, double u0, int64_t n_kill, int32_t* log_status,
                               int32_t* log_tri, float* log_bary, int32_t* log_q, double* g,
                               unsigned long long* row_queries, unsigned long long* kill_queries,
                               unsigned long long* next_walk, unsigned long long* stats, int grid, hipStream_t s) {
  const int64_t n = n_rows * 2 * pairs + n_kill;
  if (n <= 0) return hipSuccess;
  if (grid < 1) return hipErrorInvalidValue;
  const int64_t blocks = std::min<int64_t>(grid, (n + 255) / 256);
#if MSK_KELVIN_STREAM
  if (stats)
    hipLaunchKernelGGL(kelvin_stream_kernel<true>, dim3((unsigned)blocks), dim3(256), 0, s, K, st, nt, radius, n_rows,
                       pairs, u0, n_kill, log_status, log_tri, log_bary, log_q, g, row_queries, kill_queries,
                       next_walk, stats);
  else
    hipLaunchKernelGGL(kelvin_stream_kernel<false>, dim3((unsigned)blocks), dim3(256), 0, s, K, st, nt, radius,
                       n_rows, pairs, u0, n_kill, log_status, log_tri, log_bary, log_q, g, row_queries, kill_queries,
                       next_walk, stats);
#else
  if (stats)
    hipLaunchKernelGGL(kelvin_walk_kernel<true>, dim3((unsigned)blocks), dim3(256), 0, s, K, st, nt, radius, n_rows,
                       pairs, u0, n_kill, log_status, log_tri, log_bary, log_q, g, row_queries, kill_queries,
                       next_walk, stats);
  else
    hipLaunchKernelGGL(kelvin_walk_kernel<false>, dim3((unsigned)blocks), dim3(256), 0, s, K, st, nt, radius, n_rows,
                       pairs, u0, n_kill, log_status, log_tri, log_bary, log_q, g, row_queries, kill_queries,
                       next_walk, stats);
#endif
  return hipGetLastError();
}

hipError_t launch_kelvin_prepare(const KelvinTri* tris, int64_t n, KelvinPre* pre, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(kelvin_prepare_kernel, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, s, tris, n, pre);
  return hipGetLastError();
}

hipError_t launch_kelvin_closest(const KelvinDev& K, const double* Q, int64_t nq, int32_t* tri, double* d2,
                                 double* qpt, double* bary, hipStream_t s) {
  if (nq <= 0) return hipSuccess;
  hipLaunchKernelGGL(kelvin_closest_kernel, dim3((unsigned)((nq + 255) / 256)), dim3(256), 0, s, K, Q, nq, tri, d2,
                     qpt, bary);
  return hipGetLastError();
}

}  // namespace msk
