/*
 * CPU oracle for the Monte Carlo DtN walk estimator (arXiv 2606.05581).
 *
 * TEST INFRASTRUCTURE ONLY. This file is the plain, slow, FP64 reference that
 * the GPU path is checked against. Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it. It shares no code with the
 * GPU library: its Philox generator, closest-point routine, bounding volume
 * hierarchy and walk loop are written here on their own.
 *
 * What it computes, with the passages it follows:
 *   - Philox4x32-10 counter-based generator, after its published definition
 *     (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2,
 *     3", SC 2011): the walk randomness, keyed by (row, walk, step, purpose).
 *   - Closest point on a triangle (the region-based method of Ericson,
 *     Real-Time Collision Detection, sec. 5.1.5) and the nearest triangle of
 *     a point as the lexicographic minimum of (squared distance, index) over
 *     all triangles: the query that Walk-on-Spheres needs (Sec. 2,
 *     "Walk-on-Spheres": the largest empty ball and the nearest boundary point).
 *   - Walk-on-Spheres from an inset point, stopped in an eps-shell (Sec. 2),
 *     with the exterior's hit-or-escape alternative (Sec. 3.3, "Escape to
 *     Infinity") decided exactly at the scene's bounding sphere.
 *   - The naive finite-difference estimator (Sec. 3.1, Alg. 1; eqs.
 *     finite-difference-estimator and naive-stiffness-matrix): every walk
 *     contributes c = b(s) - b(t) to the row of its sample, b = barycentric
 *     interpolation of a per-vertex basis table (Sec. 3.4), or the point
 *     basis's k-nearest-neighbour interpolation with bilateral weights
 *     (Appendix, point-based k-NN interpolator).
 *   - The PSD estimator of Sec. 3.2 (Alg. 2; eqs. strong-markov-property,
 *     ball-jump-kernel, volume-jump-kernel and the boxed estimator): the
 *     largest tangent ball at each sample by bisection, ball points drawn
 *     with density proportional to the ball's jump kernel outside a small cap
 *     about s, in antithetic pairs, a walk from each, and the rank-one updates
 *     d d^T with d = b(s) - b(t), summed into a K x K matrix.
 * The finalisation (scaling, standard errors), symmetrisation and eigen step
 * live in oracle.py.
 *
 * A second, FP32 closest-point routine reproduces the single-precision
 * decision the GPU takes for the nearest-triangle index, so that index output
 * can be compared bit for bit; it follows the same region method in a fixed
 * operation order with no fused multiply-adds (build with -ffp-contract=off).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- Philox */

static void mulhilo32(uint32_t a, uint32_t b, uint32_t* hi, uint32_t* lo) {
  uint64_t p = (uint64_t)a * (uint64_t)b;
  *hi = (uint32_t)(p >> 32);
  *lo = (uint32_t)p;
}

/* Philox4x32 with 10 rounds: S-box = two 32x32->64 multiplies per round,
 * round keys advanced by the Weyl constants (golden ratio, sqrt(3)-1). */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += W0;
      k1 += W1;
    }
    uint32_t hi0, lo0, hi1, lo1;
    mulhilo32(M0, c0, &hi0, &lo0);
    mulhilo32(M1, c2, &hi1, &lo1);
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    uint32_t n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* 23 random bits mapped to the centre of one of 2^23 equal cells of (0,1):
 * exactly representable in both float and double. */
double orc_uniform(uint32_t r) { return ((double)(r >> 9) + 0.5) * (1.0 / 8388608.0); }

enum { PURPOSE_STEP = 0, PURPOSE_HAT_START = 1, PURPOSE_START_SPLIT = 2, PURPOSE_REENTRY = 3, PURPOSE_BALL = 4 };

static void draw4(uint64_t seed, uint32_t row, uint32_t walk, uint32_t step, uint32_t purpose,
                  uint32_t mesh, double u[4]) {
  uint32_t ctr[4] = {row, walk, step, (purpose << 24) | (mesh & 0xFFFFFFu)};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t o[4];
  orc_philox4x32_10(ctr, key, o);
  for (int i = 0; i < 4; ++i) u[i] = orc_uniform(o[i]);
}

/* ---------------------------------------------------- closest point (FP64) */

static double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

static double seg_closest(const double* p, const double* s0, const double* s1, double* t_out) {
  double e[3] = {s1[0] - s0[0], s1[1] - s0[1], s1[2] - s0[2]};
  double ps[3] = {p[0] - s0[0], p[1] - s0[1], p[2] - s0[2]};
  double ee = dot3(e, e);
  double t = ee > 0 ? dot3(ps, e) / ee : 0.0;
  if (t < 0) t = 0;
  if (t > 1) t = 1;
  double d[3] = {p[0] - (s0[0] + t * e[0]), p[1] - (s0[1] + t * e[1]), p[2] - (s0[2] + t * e[2])};
  *t_out = t;
  return dot3(d, d);
}

static void cross3(const double* u, const double* v, double* o) {
  o[0] = u[1] * v[2] - u[2] * v[1];
  o[1] = u[2] * v[0] - u[0] * v[2];
  o[2] = u[0] * v[1] - u[1] * v[0];
}

/* Squared distance from p to triangle (a,b,c); l[0..2] = barycentrics of the
 * closest point with respect to (a,b,c). Voronoi regions are tested in the
 * order: vertex a, vertex b, edge ab, vertex c, edge ac, edge bc, face. The
 * face-region numerators are written as n.(u x v) with n = ab x ac (Lagrange's
 * identity turns Ericson's 2x2 determinants of dot products into these), and
 * the face distance as (n.ap)^2 / n.n, both accurate for slivers. */
double orc_closest_tri(const double* p, const double* a, const double* b, const double* c, double* l) {
  double ab[3], ac[3], ap[3], bp[3], cp[3], n[3], x[3], q[3];
  for (int k = 0; k < 3; ++k) {
    ab[k] = b[k] - a[k];
    ac[k] = c[k] - a[k];
    ap[k] = p[k] - a[k];
    bp[k] = p[k] - b[k];
    cp[k] = p[k] - c[k];
  }
  double l1, l2;
  double d1 = dot3(ab, ap), d2 = dot3(ac, ap);
  double d3 = dot3(ab, bp), d4 = dot3(ac, bp);
  double d5 = dot3(ab, cp), d6 = dot3(ac, cp);
  cross3(ab, ac, n);
  cross3(ap, bp, x);
  double vc = dot3(n, x);
  cross3(cp, ap, x);
  double vb = dot3(n, x);
  cross3(bp, cp, x);
  double va = dot3(n, x);
  if (d1 <= 0 && d2 <= 0) {
    l1 = 0; l2 = 0;
  } else if (d3 >= 0 && d4 <= d3) {
    l1 = 1; l2 = 0;
  } else if (vc <= 0 && d1 >= 0 && d3 <= 0) {
    l1 = d1 / (d1 - d3); l2 = 0;
  } else if (d6 >= 0 && d5 <= d6) {
    l1 = 0; l2 = 1;
  } else if (vb <= 0 && d2 >= 0 && d6 <= 0) {
    l1 = 0; l2 = d2 / (d2 - d6);
  } else if (va <= 0 && (d4 - d3) >= 0 && (d5 - d6) >= 0) {
    double w = (d4 - d3) / ((d4 - d3) + (d5 - d6));
    l1 = 1 - w; l2 = w;
  } else {
    double den = va + vb + vc;
    if (den > 0) {
      l1 = vb / den; l2 = vc / den;
      l[0] = 1 - l1 - l2; l[1] = l1; l[2] = l2;
      double t = dot3(n, ap);
      return t * t / dot3(n, n);
    } else { /* zero-area triangle: nearest point of its three edges */
      double t, best, dd;
      best = seg_closest(p, a, b, &t); l1 = t; l2 = 0;
      dd = seg_closest(p, a, c, &t);
      if (dd < best) { best = dd; l1 = 0; l2 = t; }
      dd = seg_closest(p, b, c, &t);
      if (dd < best) { best = dd; l1 = 1 - t; l2 = t; }
    }
  }
  for (int k = 0; k < 3; ++k) q[k] = a[k] + l1 * ab[k] + l2 * ac[k];
  l[0] = 1 - l1 - l2; l[1] = l1; l[2] = l2;
  double d[3] = {p[0] - q[0], p[1] - q[1], p[2] - q[2]};
  return dot3(d, d);
}

/* ----------------------------------------- closest point (FP32 decision) */

static float dotf(const float* u, const float* v) {
  float s = u[0] * v[0];
  s = s + u[1] * v[1];
  s = s + u[2] * v[2];
  return s;
}

static void crossf(const float* u, const float* v, float* o) {
  o[0] = u[1] * v[2] - u[2] * v[1];
  o[1] = u[2] * v[0] - u[0] * v[2];
  o[2] = u[0] * v[1] - u[1] * v[0];
}

static float segf(const float* p, const float* s0, const float* s1, float* t_out) {
  float e[3] = {s1[0] - s0[0], s1[1] - s0[1], s1[2] - s0[2]};
  float ps[3] = {p[0] - s0[0], p[1] - s0[1], p[2] - s0[2]};
  float ee = dotf(e, e);
  float t = ee > 0.0f ? dotf(ps, e) / ee : 0.0f;
  if (t < 0.0f) t = 0.0f;
  if (t > 1.0f) t = 1.0f;
  float q[3] = {s0[0] + t * e[0], s0[1] + t * e[1], s0[2] + t * e[2]};
  float d[3] = {p[0] - q[0], p[1] - q[1], p[2] - q[2]};
  *t_out = t;
  return dotf(d, d);
}

/* Single-precision closest point, every operation in a fixed order and
 * rounded separately (no fused multiply-add): the regions of orc_closest_tri
 * evaluated lazily; vertex regions return |p - v|^2, edge regions the squared
 * length of p - (s0 + t e), the face region (n.ap)^2 / (n.n). l12 receives
 * the barycentrics of b and c. */
float orc_closest_tri_f32(const float* p, const float* a, const float* b, const float* c, float* l12) {
  float ab[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
  float ac[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
  float ap[3] = {p[0] - a[0], p[1] - a[1], p[2] - a[2]};
  float q[3], e[3], n[3], x[3];
  float d1 = dotf(ab, ap), d2 = dotf(ac, ap);
  if (d1 <= 0.0f && d2 <= 0.0f) {
    l12[0] = 0.0f; l12[1] = 0.0f;
    return dotf(ap, ap);
  }
  float bp[3] = {p[0] - b[0], p[1] - b[1], p[2] - b[2]};
  float d3 = dotf(ab, bp), d4 = dotf(ac, bp);
  if (d3 >= 0.0f && d4 <= d3) {
    l12[0] = 1.0f; l12[1] = 0.0f;
    return dotf(bp, bp);
  }
  crossf(ab, ac, n);
  crossf(ap, bp, x);
  float vc = dotf(n, x);
  if (vc <= 0.0f && d1 >= 0.0f && d3 <= 0.0f) {
    float v = d1 / (d1 - d3);
    for (int k = 0; k < 3; ++k) q[k] = a[k] + v * ab[k];
    for (int k = 0; k < 3; ++k) e[k] = p[k] - q[k];
    l12[0] = v; l12[1] = 0.0f;
    return dotf(e, e);
  }
  float cp[3] = {p[0] - c[0], p[1] - c[1], p[2] - c[2]};
  float d5 = dotf(ab, cp), d6 = dotf(ac, cp);
  if (d6 >= 0.0f && d5 <= d6) {
    l12[0] = 0.0f; l12[1] = 1.0f;
    return dotf(cp, cp);
  }
  crossf(cp, ap, x);
  float vb = dotf(n, x);
  if (vb <= 0.0f && d2 >= 0.0f && d6 <= 0.0f) {
    float w = d2 / (d2 - d6);
    for (int k = 0; k < 3; ++k) q[k] = a[k] + w * ac[k];
    for (int k = 0; k < 3; ++k) e[k] = p[k] - q[k];
    l12[0] = 0.0f; l12[1] = w;
    return dotf(e, e);
  }
  crossf(bp, cp, x);
  float va = dotf(n, x);
  float e43 = d4 - d3, e56 = d5 - d6;
  if (va <= 0.0f && e43 >= 0.0f && e56 >= 0.0f) {
    float w = e43 / (e43 + e56);
    float bc[3] = {c[0] - b[0], c[1] - b[1], c[2] - b[2]};
    for (int k = 0; k < 3; ++k) q[k] = b[k] + w * bc[k];
    for (int k = 0; k < 3; ++k) e[k] = p[k] - q[k];
    l12[0] = 1.0f - w; l12[1] = w;
    return dotf(e, e);
  }
  float den = (va + vb) + vc;
  if (den > 0.0f) {
    l12[0] = vb / den; l12[1] = vc / den;
    float t = dotf(n, ap);
    return (t * t) / dotf(n, n);
  }
  {
    float t, best, dd, l1, l2;
    best = segf(p, a, b, &t); l1 = t; l2 = 0.0f;
    dd = segf(p, a, c, &t);
    if (dd < best) { best = dd; l1 = 0.0f; l2 = t; }
    dd = segf(p, b, c, &t);
    if (dd < best) { best = dd; l1 = 1.0f - t; l2 = t; }
    l12[0] = l1; l12[1] = l2;
    return best;
  }
}

/* ------------------------------------------------------------------ scene */

typedef struct {
  int64_t lo, hi;   /* node: triangle range [lo,hi) if leaf, else children */
  int64_t left, right;
  double bmin[3], bmax[3];
} OrcNode;

typedef struct {
  int64_t nv, nf;
  double* V;    /* (nv,3) relative to centre */
  int32_t* F;   /* (nf,3) */
  double centre[3];
  double radius; /* bounding-sphere radius about centre, slightly inflated */
  /* optional BVH (acceleration of the brute-force minimum, same result) */
  int64_t nnodes;
  OrcNode* nodes;
  int64_t* order; /* triangle ids in leaf order */
} OrcScene;

/* Scene frame: centre of the FP64 bounding box, radius (1 + 2^-20) max|v - c|. */
void orc_scene_frame(const float* V, int64_t nv, double* centre, double* radius) {
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t i = 0; i < nv; ++i)
    for (int k = 0; k < 3; ++k) {
      double x = V[3 * i + k];
      if (x < lo[k]) lo[k] = x;
      if (x > hi[k]) hi[k] = x;
    }
  for (int k = 0; k < 3; ++k) centre[k] = 0.5 * (lo[k] + hi[k]);
  double r2 = 0;
  for (int64_t i = 0; i < nv; ++i) {
    double d[3] = {V[3 * i] - centre[0], V[3 * i + 1] - centre[1], V[3 * i + 2] - centre[2]};
    double q = dot3(d, d);
    if (q > r2) r2 = q;
  }
  *radius = (1.0 + ldexp(1.0, -20)) * sqrt(r2);
}

static void tri_bounds(const OrcScene* s, int64_t t, double* lo, double* hi, double* cen) {
  for (int k = 0; k < 3; ++k) {
    lo[k] = INFINITY; hi[k] = -INFINITY; cen[k] = 0;
  }
  for (int c = 0; c < 3; ++c) {
    const double* v = s->V + 3 * (int64_t)s->F[3 * t + c];
    for (int k = 0; k < 3; ++k) {
      if (v[k] < lo[k]) lo[k] = v[k];
      if (v[k] > hi[k]) hi[k] = v[k];
      cen[k] += v[k] / 3.0;
    }
  }
}

static double* g_sort_key;
static int cmp_key(const void* a, const void* b) {
  int64_t i = *(const int64_t*)a, j = *(const int64_t*)b;
  double x = g_sort_key[i], y = g_sort_key[j];
  if (x < y) return -1;
  if (x > y) return 1;
  return (i < j) ? -1 : (i > j);
}

/* Median-split binary BVH with exact FP64 boxes, inflated by a tiny margin. */
static int64_t build_rec(OrcScene* s, int64_t lo, int64_t hi, double* cen) {
  int64_t id = s->nnodes++;
  OrcNode* n = &s->nodes[id];
  double blo[3] = {INFINITY, INFINITY, INFINITY}, bhi[3] = {-INFINITY, -INFINITY, -INFINITY};
  double clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t i = lo; i < hi; ++i) {
    double tl[3], th[3], tc[3];
    tri_bounds(s, s->order[i], tl, th, tc);
    for (int k = 0; k < 3; ++k) {
      if (tl[k] < blo[k]) blo[k] = tl[k];
      if (th[k] > bhi[k]) bhi[k] = th[k];
      if (tc[k] < clo[k]) clo[k] = tc[k];
      if (tc[k] > chi[k]) chi[k] = tc[k];
    }
  }
  double margin = 1e-12 * (s->radius + 1.0);
  for (int k = 0; k < 3; ++k) {
    n->bmin[k] = blo[k] - margin;
    n->bmax[k] = bhi[k] + margin;
  }
  n->lo = lo; n->hi = hi; n->left = n->right = -1;
  if (hi - lo <= 4) return id;
  int ax = 0;
  for (int k = 1; k < 3; ++k)
    if (chi[k] - clo[k] > chi[ax] - clo[ax]) ax = k;
  for (int64_t i = lo; i < hi; ++i) cen[s->order[i]] = 0; /* unused slot reset */
  for (int64_t i = lo; i < hi; ++i) {
    double tl[3], th[3], tc[3];
    tri_bounds(s, s->order[i], tl, th, tc);
    cen[s->order[i]] = tc[ax];
  }
  g_sort_key = cen;
  qsort(s->order + lo, (size_t)(hi - lo), sizeof(int64_t), cmp_key);
  int64_t mid = lo + (hi - lo) / 2;
  int64_t l = build_rec(s, lo, mid, cen);
  int64_t r = build_rec(s, mid, hi, cen);
  s->nodes[id].left = l;
  s->nodes[id].right = r;
  return id;
}

void* orc_scene_create(const float* V, int64_t nv, const int32_t* F, int64_t nf, int with_bvh) {
  OrcScene* s = (OrcScene*)calloc(1, sizeof(OrcScene));
  s->nv = nv; s->nf = nf;
  orc_scene_frame(V, nv, s->centre, &s->radius);
  s->V = (double*)malloc(sizeof(double) * 3 * (size_t)(nv > 0 ? nv : 1));
  for (int64_t i = 0; i < nv; ++i)
    for (int k = 0; k < 3; ++k) s->V[3 * i + k] = (double)V[3 * i + k] - s->centre[k];
  s->F = (int32_t*)malloc(sizeof(int32_t) * 3 * (size_t)(nf > 0 ? nf : 1));
  memcpy(s->F, F, sizeof(int32_t) * 3 * (size_t)nf);
  if (with_bvh && nf > 0) {
    s->nodes = (OrcNode*)malloc(sizeof(OrcNode) * (size_t)(2 * nf + 1));
    s->order = (int64_t*)malloc(sizeof(int64_t) * (size_t)nf);
    double* cen = (double*)malloc(sizeof(double) * (size_t)nf);
    for (int64_t i = 0; i < nf; ++i) s->order[i] = i;
    build_rec(s, 0, nf, cen);
    free(cen);
  }
  return s;
}

void orc_scene_destroy(void* h) {
  OrcScene* s = (OrcScene*)h;
  if (!s) return;
  free(s->V); free(s->F); free(s->nodes); free(s->order); free(s);
}

void orc_scene_info(const void* h, double* centre, double* radius) {
  const OrcScene* s = (const OrcScene*)h;
  for (int k = 0; k < 3; ++k) centre[k] = s->centre[k];
  *radius = s->radius;
}

static double tri_d2(const OrcScene* s, int64_t t, const double* p, double* l) {
  const int32_t* f = s->F + 3 * t;
  return orc_closest_tri(p, s->V + 3 * (int64_t)f[0], s->V + 3 * (int64_t)f[1], s->V + 3 * (int64_t)f[2], l);
}

/* Nearest triangle: minimum of (d2, index) over all triangles. */
static double nearest_brute(const OrcScene* s, const double* p, int64_t* tri, double* bary) {
  double best = INFINITY;
  int64_t bi = -1;
  double l[3];
  for (int64_t t = 0; t < s->nf; ++t) {
    double d = tri_d2(s, t, p, l);
    if (d < best || (d == best && t < bi)) {
      best = d; bi = t;
      bary[0] = l[0]; bary[1] = l[1]; bary[2] = l[2];
    }
  }
  *tri = bi;
  return best;
}

static double box_d2(const OrcNode* n, const double* p) {
  double s = 0;
  for (int k = 0; k < 3; ++k) {
    double d = 0;
    if (p[k] < n->bmin[k]) d = n->bmin[k] - p[k];
    else if (p[k] > n->bmax[k]) d = p[k] - n->bmax[k];
    s += d * d;
  }
  return s;
}

/* Same minimum as nearest_brute, visiting only boxes that can hold a
 * triangle at squared distance <= the best so far. */
static double nearest_bvh(const OrcScene* s, const double* p, int64_t* tri, double* bary) {
  double best = INFINITY;
  int64_t bi = -1;
  int64_t stack[256];
  int sp = 0;
  stack[sp++] = 0;
  double l[3];
  while (sp > 0) {
    const OrcNode* n = &s->nodes[stack[--sp]];
    if (box_d2(n, p) > best * (1.0 + 1e-12)) continue;
    if (n->left < 0) {
      for (int64_t i = n->lo; i < n->hi; ++i) {
        int64_t t = s->order[i];
        double d = tri_d2(s, t, p, l);
        if (d < best || (d == best && t < bi)) {
          best = d; bi = t;
          bary[0] = l[0]; bary[1] = l[1]; bary[2] = l[2];
        }
      }
    } else {
      const OrcNode* a = &s->nodes[n->left];
      const OrcNode* b = &s->nodes[n->right];
      double da = box_d2(a, p), db = box_d2(b, p);
      /* push the farther child first so the nearer one is visited first */
      if (da <= db) {
        stack[sp++] = n->right;
        stack[sp++] = n->left;
      } else {
        stack[sp++] = n->left;
        stack[sp++] = n->right;
      }
      if (sp > 250) abort();
    }
  }
  *tri = bi;
  return best;
}

static double nearest(const OrcScene* s, const double* p, int64_t* tri, double* bary) {
  if (s->nodes) return nearest_bvh(s, p, tri, bary);
  return nearest_brute(s, p, tri, bary);
}

/* Batch nearest-triangle query in FP64 (points in world coordinates). */
void orc_nearest(const void* h, const double* Q, int64_t nq, int use_bvh, int64_t* tri, double* d2,
                 double* bary) {
  const OrcScene* s = (const OrcScene*)h;
  for (int64_t i = 0; i < nq; ++i) {
    double p[3] = {Q[3 * i] - s->centre[0], Q[3 * i + 1] - s->centre[1], Q[3 * i + 2] - s->centre[2]};
    d2[i] = (use_bvh && s->nodes) ? nearest_bvh(s, p, &tri[i], bary + 3 * i)
                                  : nearest_brute(s, p, &tri[i], bary + 3 * i);
  }
}

/* Brute-force FP32 nearest triangle. Points and vertices are given as float
 * offsets from the scene centre (the single-precision frame of the GPU). */
void orc_nearest_f32(const float* Vrel, const int32_t* F, int64_t nf, const float* Qrel, int64_t nq,
                     int32_t* tri, float* d2, float* bary12) {
  for (int64_t i = 0; i < nq; ++i) {
    float best = INFINITY;
    int32_t bi = -1;
    float bl[2] = {0, 0};
    for (int64_t t = 0; t < nf; ++t) {
      float l[2];
      const int32_t* f = F + 3 * t;
      float d = orc_closest_tri_f32(Qrel + 3 * i, Vrel + 3 * (int64_t)f[0], Vrel + 3 * (int64_t)f[1],
                                    Vrel + 3 * (int64_t)f[2], l);
      if (d < best || (d == best && (int32_t)t < bi)) {
        best = d; bi = (int32_t)t; bl[0] = l[0]; bl[1] = l[1];
      }
    }
    tri[i] = bi; d2[i] = best; bary12[2 * i] = bl[0]; bary12[2 * i + 1] = bl[1];
  }
}

/* ------------------------------------------------------------------ walks */

enum { ST_HIT = 0, ST_ESCAPED = 1, ST_CAPPED = 2 };

typedef struct {
  double eps, kappa, delta;
  int64_t max_steps;
  uint64_t seed;
  uint32_t mesh;
} OrcWalkParams;

/* Point re-entering the bounding sphere B(0,R) from x with |x| = rho > R:
 * given that Brownian motion from x hits the sphere, its hitting point has
 * density proportional to |x - y|^-3 (exterior Poisson kernel of the ball).
 * With a = rho^2 + R^2, b = 2 rho R and mu = cos(angle(x, y)), inverting the
 * CDF of mu gives 1/|x-y| = 1/(rho+R) + u (1/(rho-R) - 1/(rho+R)). */
double orc_reentry_mu(double rho, double R, double u) {
  double a = rho * rho + R * R, b = 2.0 * rho * R;
  double qinv = 1.0 / (rho + R) + u * (1.0 / (rho - R) - 1.0 / (rho + R));
  double mu = (a - 1.0 / (qinv * qinv)) / b;
  if (mu > 1) mu = 1;
  if (mu < -1) mu = -1;
  return mu;
}

/* Orthonormal frame (e1, e2) completing the unit vector n. */
static void frame(const double* n, double* e1, double* e2) {
  double sgn = n[2] >= 0 ? 1.0 : -1.0;
  double a = -1.0 / (sgn + n[2]);
  double b = n[0] * n[1] * a;
  e1[0] = 1.0 + sgn * n[0] * n[0] * a; e1[1] = sgn * b; e1[2] = -sgn * n[0];
  e2[0] = b; e2[1] = sgn + n[1] * n[1] * a; e2[2] = -n[1];
}

/* One Walk-on-Spheres walk from x (scene-relative). Returns the status; the
 * terminal triangle / barycentrics are written for hits and capped walks. */
static int walk(const OrcScene* s, const OrcWalkParams* P, uint32_t row, uint32_t wk, double* x,
                int64_t* tri, double* bary, int64_t* nquery, int64_t* nstep) {
  double eps2 = P->eps * P->eps;
  int64_t q = 0;
  for (int64_t k = 0; k < P->max_steps; ++k) {
    double u[4];
    draw4(P->seed, row, wk, (uint32_t)k, PURPOSE_STEP, P->mesh, u);
    double rho = sqrt(dot3(x, x));
    if (rho > s->radius) {
      /* outside the bounding sphere: escape for good with prob. 1 - R/rho,
       * otherwise jump to the exact first hitting point of the sphere */
      if (u[2] < 1.0 - s->radius / rho) {
        *nquery = q; *nstep = k + 1; *tri = -1;
        return ST_ESCAPED;
      }
      double mu = orc_reentry_mu(rho, s->radius, u[3]);
      double v[4];
      draw4(P->seed, row, wk, (uint32_t)k, PURPOSE_REENTRY, P->mesh, v);
      double phi = 2.0 * M_PI * v[0];
      double nx[3] = {x[0] / rho, x[1] / rho, x[2] / rho}, e1[3], e2[3];
      frame(nx, e1, e2);
      double st = sqrt(fmax(0.0, 1.0 - mu * mu));
      for (int c = 0; c < 3; ++c)
        x[c] = s->radius * (mu * nx[c] + st * (cos(phi) * e1[c] + sin(phi) * e2[c]));
      /* the re-entry point lies on the sphere: the same step goes on with a
       * distance query from there (u[0], u[1] are still unused) */
    }
    double d2 = nearest(s, x, tri, bary);
    ++q;
    if (d2 < eps2) {
      *nquery = q; *nstep = k + 1;
      return ST_HIT;
    }
    /* any ball inside the domain is a valid step (mean value property); the
     * radius is shrunk by the same relative/absolute guard the GPU uses */
    double r = sqrt(d2) * (1.0 - P->kappa) - P->delta;
    double z = 1.0 - 2.0 * u[0];
    double rxy = 2.0 * sqrt(u[0] * (1.0 - u[0]));
    double phi = 2.0 * M_PI * u[1];
    x[0] += r * rxy * cos(phi);
    x[1] += r * rxy * sin(phi);
    x[2] += r * z;
  }
  nearest(s, x, tri, bary);
  *nquery = q + 1; *nstep = P->max_steps;
  return ST_CAPPED;
}

/* Walks from given world-space points: status, terminal triangle,
 * barycentrics and query counts (used for closed-form checks). */
void orc_walks_from(const void* h, const double* X, int64_t n, double eps, double kappa, double delta,
                    int64_t max_steps, uint64_t seed, int32_t* status, int64_t* tri, double* bary,
                    int64_t* nquery) {
  const OrcScene* s = (const OrcScene*)h;
  OrcWalkParams P = {eps, kappa, delta, max_steps, seed, 0};
  for (int64_t i = 0; i < n; ++i) {
    double x[3] = {X[3 * i] - s->centre[0], X[3 * i + 1] - s->centre[1], X[3 * i + 2] - s->centre[2]};
    int64_t ns;
    status[i] = walk(s, &P, 0, (uint32_t)i, x, &tri[i], bary + 3 * i, &nquery[i], &ns);
  }
}

/* ------------------------------------------------------------- estimator */

typedef struct {
  const int32_t* rowptr;
  const int32_t* col;
  const float* val;
  int64_t K;
} OrcBasis;

/* sparse accumulator for one walk: c = b(s) - b(t) with merged columns */
typedef struct {
  int n;
  int32_t col[256];
  double val[256];
} Sparse;

static void sp_add(Sparse* c, const OrcBasis* B, int64_t vtx, double lam) {
  if (lam == 0.0) return;
  for (int32_t e = B->rowptr[vtx]; e < B->rowptr[vtx + 1]; ++e) {
    int32_t j = B->col[e];
    double v = lam * (double)B->val[e];
    int m;
    for (m = 0; m < c->n; ++m)
      if (c->col[m] == j) break;
    if (m == c->n) {
      if (c->n == 256) abort();
      c->col[m] = j; c->val[m] = 0; c->n++;
    }
    c->val[m] += v;
  }
}

/* Point basis (Appendix, point-based k-NN interpolator): column j is sample
 * point x_j (normal n_j); at a query q with normal n_q the basis values are
 * the bilateral weights of q's k nearest points (Euclidean distance, ties by
 * index), w_j = exp(-|q - x_j|^2 / (2 sigma^2)) exp(-(1 - n_q . n_j) / tau),
 * normalised over the k; all other columns are 0. */
typedef struct {
  const double* x;  /* (N,3) scene-relative */
  const double* n;  /* (N,3) unit normals */
  int64_t N;
  int k;
  double sigma, tau;
} OrcKnn;

/* k nearest points of q: the k smallest (squared distance, index) pairs. */
int orc_knn_query(const double* x, int64_t N, int k, const double* q, int32_t* idx, double* d2) {
  int m = 0;
  for (int64_t j = 0; j < N; ++j) {
    const double d[3] = {x[3 * j] - q[0], x[3 * j + 1] - q[1], x[3 * j + 2] - q[2]};
    const double dd = dot3(d, d);
    if (m == k && !(dd < d2[k - 1])) continue; /* equal distance: the lower index is already kept */
    int pos = m < k ? m++ : k - 1;
    while (pos > 0 && dd < d2[pos - 1]) {
      d2[pos] = d2[pos - 1];
      idx[pos] = idx[pos - 1];
      --pos;
    }
    d2[pos] = dd;
    idx[pos] = (int32_t)j;
  }
  return m;
}

/* Bilateral k-NN weights at q (normal nq): returns the neighbour count. */
int orc_knn_weights(const double* x, const double* n, int64_t N, int k, double sigma, double tau, const double* q,
                    const double* nq, int32_t* idx, double* w) {
  double d2[64];
  int m = orc_knn_query(x, N, k, q, idx, d2);
  double sum = 0.0;
  for (int a = 0; a < m; ++a) {
    const double* nj = n + 3 * (int64_t)idx[a];
    w[a] = exp(-d2[a] / (2.0 * sigma * sigma)) * exp(-(1.0 - dot3(nq, nj)) / tau);
    sum += w[a];
  }
  for (int a = 0; a < m; ++a) w[a] = sum > 0.0 ? w[a] / sum : 1.0 / m; /* all weights underflowed: equal shares */
  return m;
}

static void knn_add(Sparse* c, const OrcKnn* P, const double* q, const double* nq, double sign) {
  int32_t idx[64];
  double w[64];
  int m = orc_knn_weights(P->x, P->n, P->N, P->k, P->sigma, P->tau, q, nq, idx, w);
  for (int a = 0; a < m; ++a) {
    int t;
    for (t = 0; t < c->n; ++t)
      if (c->col[t] == idx[a]) break;
    if (t == c->n) {
      if (c->n == 256) abort();
      c->col[t] = idx[a]; c->val[t] = 0; c->n++;
    }
    c->val[t] += sign * w[a];
  }
}

/* Estimate rows of the naive DtN estimator.
 *
 * mode_start: 0 = point rows (fixed sample s = p_i on face tri_i with
 * barycentrics bary_i, normal n_i); 1 = hat rows (row i = vertex i; each
 * walk draws s ~ phi_i / A_i on the vertex one-ring).
 * exterior: 0 inset x = s - h n (interior), 1 inset x = s + h n.
 * Walk indices are [w0, w0 + W). Outputs (row-major, n_rows x K), added to:
 * acc = sum over walks of c, acc2 = sum of c^2; per-row counters; optional
 * walk log (n_rows x W entries: status, terminal triangle and barycentrics,
 * queries, start triangle and start barycentrics).
 */
void orc_estimate(const void* h, int mode_start, int exterior, int64_t n_rows, const int32_t* rows_sel,
                  /* point rows */ const float* p, const float* nrm, const int32_t* tri, const float* bary,
                  /* hat rows */ const int32_t* ring_ptr, const int32_t* ring_tri, const double* ring_cum,
                  const float* fn,
                  /* basis */ const int32_t* rowptr, const int32_t* col, const float* val, int64_t K,
                  int64_t W, int64_t w0, double eps, double hin, double kappa, double delta, int64_t max_steps,
                  uint64_t seed, uint32_t mesh, int nthreads,
                  double* acc, double* acc2, int64_t* n_query, int64_t* n_escaped, int64_t* n_capped,
                  int32_t* discarded,
                  int32_t* log_status, int64_t* log_tri, float* log_bary, int64_t* log_nquery,
                  int32_t* log_stri, float* log_sbary,
                  /* optional point basis (point rows): points and normals in world coordinates */
                  const double* knn_x, const double* knn_n, int64_t knn_N, int knn_k, double knn_sigma,
                  double knn_tau,
                  /* exterior: 1 drops the killing term (Sec. 3.3, eq. exterior-dtn-beurling-deny-form; the
                     default of Sec. 4): an escaped walk contributes nothing instead of b(s) */
                  int jump_only) {
  const OrcScene* s = (const OrcScene*)h;
  OrcBasis B = {rowptr, col, val, K};
  OrcKnn KN = {NULL, knn_n, knn_N, knn_k, knn_sigma, knn_tau};
  double* xrel = NULL;
  if (knn_x) {
    xrel = (double*)malloc(sizeof(double) * 3 * (size_t)(knn_N > 0 ? knn_N : 1));
    for (int64_t j = 0; j < knn_N; ++j)
      for (int k = 0; k < 3; ++k) xrel[3 * j + k] = knn_x[3 * j + k] - s->centre[k];
    KN.x = xrel;
  }
  OrcWalkParams P = {eps, kappa, delta, max_steps, seed, mesh};
  double sgn = exterior ? 1.0 : -1.0;
  (void)nthreads;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads > 0 ? nthreads : 1)
  for (int64_t ri = 0; ri < n_rows; ++ri) {
    int64_t i = rows_sel ? rows_sel[ri] : ri;
    double* A1 = acc + ri * K;
    double* A2 = acc2 + ri * K;
    discarded[ri] = 0;
    n_query[ri] = 0; n_escaped[ri] = 0; n_capped[ri] = 0;
    if (mode_start == 0) {
      /* discard rows whose inset point is closer than h/2 to the surface */
      double x0[3];
      for (int c = 0; c < 3; ++c) x0[c] = ((double)p[3 * i + c] - s->centre[c]) + sgn * hin * (double)nrm[3 * i + c];
      int64_t tt; double bb[3];
      double d2 = nearest(s, x0, &tt, bb);
      n_query[ri] += 1;
      if (d2 < 0.25 * hin * hin) {
        discarded[ri] = 1;
        continue;
      }
    }
    for (int64_t w = w0; w < w0 + W; ++w) {
      double sp[3], n[3], lam[3];
      int32_t face;
      Sparse c;
      c.n = 0;
      if (mode_start == 0) {
        face = tri[i];
        for (int k = 0; k < 3; ++k) {
          sp[k] = (double)p[3 * i + k] - s->centre[k];
          n[k] = nrm[3 * i + k];
          lam[k] = bary[3 * i + k];
        }
      } else {
        double u[4], v[4];
        draw4(seed, (uint32_t)i, (uint32_t)w, 0, PURPOSE_HAT_START, mesh, u);
        draw4(seed, (uint32_t)i, (uint32_t)w, 0, PURPOSE_START_SPLIT, mesh, v);
        int32_t b0 = ring_ptr[i], b1 = ring_ptr[i + 1];
        double target = u[0] * ring_cum[b1 - 1];
        int32_t e = b0;
        while (e < b1 - 1 && !(ring_cum[e] > target)) ++e;
        face = ring_tri[e];
        /* Beta(2,2) coordinate for vertex i = median of three uniforms */
        double m1 = u[1], m2 = u[2], m3 = u[3];
        double li = fmax(fmin(m1, m2), fmin(fmax(m1, m2), m3));
        int corner = 0;
        for (int k = 0; k < 3; ++k)
          if (s->F[3 * face + k] == (int32_t)i) corner = k;
        int o1 = corner == 0 ? 1 : 0;
        int o2 = corner == 2 ? 1 : 2;
        lam[corner] = li;
        lam[o1] = (1.0 - li) * v[0];
        lam[o2] = (1.0 - li) * (1.0 - v[0]);
        for (int k = 0; k < 3; ++k) {
          sp[k] = 0;
          n[k] = fn[3 * face + k];
        }
        for (int cc = 0; cc < 3; ++cc)
          for (int k = 0; k < 3; ++k) sp[k] += lam[cc] * s->V[3 * (int64_t)s->F[3 * face + cc] + k];
      }
      if (KN.x) {
        double nl = sqrt(dot3(n, n));
        double nu[3] = {n[0] / nl, n[1] / nl, n[2] / nl};
        knn_add(&c, &KN, sp, nu, 1.0);
      } else {
        for (int cc = 0; cc < 3; ++cc) sp_add(&c, &B, s->F[3 * face + cc], lam[cc]);
      }
      double x[3] = {sp[0] + sgn * hin * n[0], sp[1] + sgn * hin * n[1], sp[2] + sgn * hin * n[2]};
      int64_t tt = -1, nq = 0, ns = 0;
      double bt[3] = {0, 0, 0};
      int st = walk(s, &P, (uint32_t)i, (uint32_t)w, x, &tt, bt, &nq, &ns);
      if (st != ST_ESCAPED && KN.x) {
        /* hit point and its face normal */
        const double* va = s->V + 3 * (int64_t)s->F[3 * tt];
        const double* vb = s->V + 3 * (int64_t)s->F[3 * tt + 1];
        const double* vc = s->V + 3 * (int64_t)s->F[3 * tt + 2];
        double q[3], e1[3], e2[3], nt[3];
        for (int k = 0; k < 3; ++k) {
          q[k] = bt[0] * va[k] + bt[1] * vb[k] + bt[2] * vc[k];
          e1[k] = vb[k] - va[k];
          e2[k] = vc[k] - va[k];
        }
        cross3(e1, e2, nt);
        double nl = sqrt(dot3(nt, nt));
        if (nl > 0)
          for (int k = 0; k < 3; ++k) nt[k] /= nl;
        knn_add(&c, &KN, q, nt, -1.0);
      } else if (st != ST_ESCAPED) {
        for (int cc = 0; cc < 3; ++cc) sp_add(&c, &B, s->F[3 * tt + cc], -bt[cc]);
      }
      if (jump_only && st == ST_ESCAPED) c.n = 0;
      for (int m = 0; m < c.n; ++m) {
        A1[c.col[m]] += c.val[m];
        A2[c.col[m]] += c.val[m] * c.val[m];
      }
      n_query[ri] += nq;
      if (st == ST_ESCAPED) n_escaped[ri]++;
      if (st == ST_CAPPED) n_capped[ri]++;
      if (log_status) {
        int64_t li = ri * W + (w - w0);
        log_status[li] = st;
        log_tri[li] = tt;
        log_bary[2 * li] = (float)bt[1];
        log_bary[2 * li + 1] = (float)bt[2];
        log_nquery[li] = nq;
        log_stri[li] = face;
        log_sbary[2 * li] = (float)lam[1];
        log_sbary[2 * li + 1] = (float)lam[2];
      }
    }
  }
  free(xrel);
}

/* ------------------------------------------------- PSD estimator (Sec. 3.2) */

/* Largest ball inside the domain that touches the surface at s, centre
 * c = s - r n (Sec. 3.2; Alg. 2, LargestTangentBall): bisection over
 * r in [0, r_max] for `iters` steps; a radius is accepted when the nearest
 * surface point of c is at least r - min(tol, 2^-10 r) away and the ball lies
 * inside the scene's bounding sphere (as every ball inside the domain does).
 * tol is half the walk's termination shell, so a ball point outside the
 * domain lies within the shell and its walk ends at once; the relative bound
 * keeps small balls (next to edges of a faceted surface) essentially inside.
 * Returns the last accepted radius (0 when none is: the sample is then
 * dropped, Appendix A). s, n are scene-relative, n the outward unit normal. */
#define TANGENT_REL_TOL (1.0 / 1024.0)
double orc_tangent_ball(const void* h, const double* s, const double* n, double r_max, int iters, double tol) {
  const OrcScene* sc = (const OrcScene*)h;
  double lo = 0.0, hi = r_max;
  for (int it = 0; it < iters; ++it) {
    double mid = 0.5 * (lo + hi);
    double c[3] = {s[0] - mid * n[0], s[1] - mid * n[1], s[2] - mid * n[2]};
    int64_t tt;
    double bb[3];
    double d = sqrt(nearest(sc, c, &tt, bb));
    double t = mid - fmin(tol, mid * TANGENT_REL_TOL);
    if (d >= t && sqrt(dot3(c, c)) + mid <= sc->radius)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

/* Normaliser of the ball jump kernel J(s, z) = 1 / (2 pi |s - z|^3)
 * (eq. ball-jump-kernel) over the sphere of radius r through s, without the
 * cap of polar angle theta0 about s (angle at the centre): with
 * u = sin(theta / 2), |s - z| = 2 r u and dz = 8 r^2 u du dphi, so
 * int J dz = (1 / (2 r)) int_{u0}^{1} 2 / u^2 du = (1 / (2 r)) (1 / u0 - 1). */
double orc_ball_jump_mass(double r, double theta0) {
  double u0 = sin(0.5 * theta0);
  return (1.0 / (2.0 * r)) * (1.0 / u0 - 1.0);
}

/* A point z on the tangent ball (centre c, radius r, outward normal n at s =
 * c + r n) with density proportional to J(s, z) outside the cap, and its
 * antithetic partner (azimuth + pi): u = sin(theta / 2) has density
 * proportional to 1 / u^2 on [u0, 1], so 1 / u = 1 / u0 - xi (1 / u0 - 1);
 * the azimuth is uniform. (Sec. 3.2, Implementation: importance sampling by
 * the jump kernel, excluded cap, antithetic sampling.) */
void orc_ball_point(const double* c, double r, const double* n, double theta0, double xi, double eta, int partner,
                    double* z) {
  double u0 = sin(0.5 * theta0);
  double u = 1.0 / (1.0 / u0 - xi * (1.0 / u0 - 1.0));
  double ct = 1.0 - 2.0 * u * u, st = 2.0 * u * sqrt(fmax(0.0, 1.0 - u * u));
  double phi = 2.0 * M_PI * eta + (partner ? M_PI : 0.0);
  double e1[3], e2[3];
  frame(n, e1, e2);
  for (int k = 0; k < 3; ++k) z[k] = c[k] + r * (ct * n[k] + st * (cos(phi) * e1[k] + sin(phi) * e2[k]));
}

/* Alg. 2 over point rows: row i is the sample s_i (face tri_i, barycentrics
 * bary_i, outward normal n_i) standing for the area w_i of the surface.
 * Each row draws `pairs` antithetic pairs of ball points (Philox purpose
 * BALL, walk counter = pair index) and runs a walk from each (step streams
 * of walk 2j and 2j+1). The boxed estimator with s stratified over rows and
 * z importance-sampled gives, per pair p of row i,
 *   X_p = alpha_i (d_1 d_1^T + d_2 d_2^T) / 2,  alpha_i = w_i Z_i / (2 pairs),
 * with Z_i = orc_ball_jump_mass(r_i, theta0) the weight J / density and
 * d = b(s_i) - b(t). The tangent-ball tolerance is min(eps / 2, r / 1024). Outputs: S = sum_p X_p and Q = sum_p X_p * X_p
 * (elementwise), both K x K; per-row radius (0 = dropped) and Z; an optional
 * walk log (n_rows x 2 pairs: status, terminal triangle, its barycentrics of
 * vertices 1 and 2, queries). The basis is a dense per-vertex table tab
 * (n_verts x K). */
void orc_psd_estimate(const void* h, int64_t n_rows, const float* p, const float* nrm, const int32_t* tri,
                      const float* bary, const double* w, const double* tab, int64_t K, int64_t pairs,
                      double theta0, double r_max, int bisect_iters, double eps, double kappa,
                      double delta, int64_t max_steps, uint64_t seed, uint32_t mesh, int nthreads, double* S,
                      double* Q, double* radius, double* Zout, int64_t* n_query, int32_t* log_status,
                      int64_t* log_tri, float* log_bary, int64_t* log_nquery) {
  const OrcScene* sc = (const OrcScene*)h;
  OrcWalkParams P = {eps, kappa, delta, max_steps, seed, mesh};
  memset(S, 0, sizeof(double) * K * K);
  memset(Q, 0, sizeof(double) * K * K);
  (void)nthreads;
  /* rows run in parallel; each row's sums are added to S and Q in the order
   * the rows finish (FP64: the order changes only the last bits) */
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads > 0 ? nthreads : 1)
  for (int64_t i = 0; i < n_rows; ++i) {
    double s[3], n[3];
    for (int k = 0; k < 3; ++k) {
      s[k] = (double)p[3 * i + k] - sc->centre[k];
      n[k] = nrm[3 * i + k];
    }
    double nl = sqrt(dot3(n, n));
    for (int k = 0; k < 3; ++k) n[k] /= nl;
    double r = orc_tangent_ball(h, s, n, r_max, bisect_iters, 0.5 * eps);
    radius[i] = r;
    Zout[i] = r > 0 ? orc_ball_jump_mass(r, theta0) : 0.0;
    n_query[i] = bisect_iters;
    if (r <= 0) continue;
    double c[3] = {s[0] - r * n[0], s[1] - r * n[1], s[2] - r * n[2]};
    double alpha = w[i] * Zout[i] / (2.0 * (double)pairs);
    /* b(s) */
    double* bs = (double*)calloc(K, sizeof(double));
    double* d = (double*)malloc(sizeof(double) * 2 * K);
    double* Si = (double*)calloc(K * K, sizeof(double));
    double* Qi = (double*)calloc(K * K, sizeof(double));
    for (int cc = 0; cc < 3; ++cc) {
      int64_t v = sc->F[3 * (int64_t)tri[i] + cc];
      for (int64_t k = 0; k < K; ++k) bs[k] += (double)bary[3 * i + cc] * tab[v * K + k];
    }
    for (int64_t j = 0; j < pairs; ++j) {
      double u[4];
      draw4(seed, (uint32_t)i, (uint32_t)j, 0, PURPOSE_BALL, mesh, u);
      for (int a = 0; a < 2; ++a) {
        double x[3];
        orc_ball_point(c, r, n, theta0, u[0], u[1], a, x);
        int64_t tt = -1, nq = 0, ns = 0;
        double bt[3] = {0, 0, 0};
        int st = walk(sc, &P, (uint32_t)i, (uint32_t)(2 * j + a), x, &tt, bt, &nq, &ns);
        n_query[i] += nq;
        for (int64_t k = 0; k < K; ++k) {
          double b = 0.0;
          if (st != ST_ESCAPED)
            for (int cc = 0; cc < 3; ++cc) b += bt[cc] * tab[(int64_t)sc->F[3 * tt + cc] * K + k];
          d[a * K + k] = bs[k] - b;
        }
        if (log_status) {
          int64_t li = i * 2 * pairs + 2 * j + a;
          log_status[li] = st;
          log_tri[li] = tt;
          log_bary[2 * li] = (float)bt[1];
          log_bary[2 * li + 1] = (float)bt[2];
          log_nquery[li] = nq;
        }
      }
      for (int64_t k = 0; k < K; ++k)
        for (int64_t l = 0; l < K; ++l) {
          double x = 0.5 * alpha * (d[k] * d[l] + d[K + k] * d[K + l]);
          Si[k * K + l] += x;
          Qi[k * K + l] += x * x;
        }
    }
#pragma omp critical
    {
      for (int64_t e = 0; e < K * K; ++e) {
        S[e] += Si[e];
        Q[e] += Qi[e];
      }
    }
    free(bs);
    free(d);
    free(Si);
    free(Qi);
  }
}

/* ------------------------------------- Kelvin-inverted exterior (Sec. 3.3) */

/* The exterior DtN form of Sec. 3.3 (eq. exterior-dtn-beurling-deny-form) is
 * estimated in the image of the exterior under the Kelvin transform
 * x -> x / |x|^2 about a centre o inside the shape (Sec. 3.3, "The Kelvin
 * Transform"; Appendix, Kelvin transform): a bounded domain whose boundary
 * is the image of the mesh, each planar triangle becoming a piece of a sphere
 * through the origin bounded by three circular arcs (Sec. 4: spherical
 * triangular elements with non-planar distance queries). Coordinates below
 * are relative to o. */

typedef struct {
  int64_t nv, nf;
  double* V;     /* (nv, 3) primal vertices relative to the inversion centre */
  int32_t* F;
  double o[3];   /* inversion centre (world) */
  double lo[3], hi[3]; /* bounding box of the inverted vertices */
  double radius; /* max |x~| over the inverted vertices and arcs (a bound of the inverted domain) */
  /* bounding volume hierarchy over boxes that contain each inverted
   * triangle (an acceleration of the brute-force minimum, same result) */
  double* tlo;   /* (nf, 3) */
  double* thi;
  int64_t nnodes;
  OrcNode* nodes;
  int64_t* order;
} OrcKelvin;

static void kelvin3(const double* x, double* y) {
  double r2 = dot3(x, x);
  y[0] = x[0] / r2; y[1] = x[1] / r2; y[2] = x[2] / r2;
}

/* barycentrics of the projection of y onto the plane of (a, b, c) */
static void plane_bary(const double* y, const double* a, const double* b, const double* c, double* l) {
  double ab[3], ac[3], ay[3], n[3], x[3];
  for (int k = 0; k < 3; ++k) { ab[k] = b[k] - a[k]; ac[k] = c[k] - a[k]; ay[k] = y[k] - a[k]; }
  cross3(ab, ac, n);
  double nn = dot3(n, n);
  cross3(ay, ac, x);
  double l1 = dot3(x, n) / nn;
  cross3(ab, ay, x);
  double l2 = dot3(x, n) / nn;
  l[0] = 1 - l1 - l2; l[1] = l1; l[2] = l2;
}

/* Nearest point of the image of the segment [P0, P1] (relative to the
 * centre, not through it) to p: the image of the line is the circle through
 * the origin in the plane of (0, P0, P1) with diameter from 0 to the image
 * of the line's foot point f, centre f / (2 |f|^2), radius 1 / (2 |f|); the
 * nearest circle point to p is the radial projection of p's in-plane
 * position; it lies on the segment's arc when its image lies between P0 and
 * P1, else an end point is nearest. The origin itself is the image of the
 * line's point at infinity, not of a segment point: every point of the
 * segment's image lies at least 1 / max(|P0|, |P1|) from it, and a
 * projection closer than that is not on the arc. A line through the centre
 * maps to itself. Returns the squared distance, the point q and the segment
 * parameter t of kappa(q) = P0 + t (P1 - P0). */
static double inv_seg_d2(const double* p, const double* P0, const double* P1, double* q, double* t_out) {
  double e[3] = {P1[0] - P0[0], P1[1] - P0[1], P1[2] - P0[2]};
  double ee = dot3(e, e);
  double best = INFINITY, bt = 0;
  double k0[3], k1[3];
  kelvin3(P0, k0);
  kelvin3(P1, k1);
  /* end points */
  double dd0[3] = {p[0] - k0[0], p[1] - k0[1], p[2] - k0[2]};
  double dd1[3] = {p[0] - k1[0], p[1] - k1[1], p[2] - k1[2]};
  if (dot3(dd0, dd0) < best) { best = dot3(dd0, dd0); bt = 0; memcpy(q, k0, sizeof(k0)); }
  if (dot3(dd1, dd1) < best) { best = dot3(dd1, dd1); bt = 1; memcpy(q, k1, sizeof(k1)); }
  if (!(ee > 0)) { *t_out = bt; return best; }
  double tf = -dot3(P0, e) / ee;
  double f[3] = {P0[0] + tf * e[0], P0[1] + tf * e[1], P0[2] + tf * e[2]};
  double ff = dot3(f, f);
  double m[3];
  cross3(P0, P1, m);
  double mm = dot3(m, m);
  double scale = fmax(dot3(P0, P0), dot3(P1, P1));
  if (ff > 1e-24 * scale && mm > 0) {
    double ml = sqrt(mm);
    for (int k = 0; k < 3; ++k) m[k] /= ml;
    double cc[3] = {f[0] / (2 * ff), f[1] / (2 * ff), f[2] / (2 * ff)};
    double rho = 1.0 / (2 * sqrt(ff));
    double mp = dot3(m, p);
    double u[3] = {p[0] - mp * m[0] - cc[0], p[1] - mp * m[1] - cc[1], p[2] - mp * m[2] - cc[2]};
    double ul = sqrt(dot3(u, u));
    if (ul > 0) {
      double e2[3] = {cc[0] + rho * u[0] / ul, cc[1] + rho * u[1] / ul, cc[2] + rho * u[2] / ul};
      double ry = dot3(e2, e2);
      if (ry * scale >= 1.0 - 1e-9) {
        double y[3];
        kelvin3(e2, y);
        double yd[3] = {y[0] - P0[0], y[1] - P0[1], y[2] - P0[2]};
        double t = dot3(yd, e) / ee;
        if (t >= 0 && t <= 1) {
          double d[3] = {p[0] - e2[0], p[1] - e2[1], p[2] - e2[2]};
          double d2 = dot3(d, d);
          if (d2 < best) { best = d2; bt = t; memcpy(q, e2, sizeof(e2)); }
        }
      }
    }
  } else {
    /* the line passes through the centre: the arc is the straight segment
     * between the images of the end points */
    double t;
    double d2 = seg_closest(p, k0, k1, &t);
    if (d2 < best) {
      best = d2;
      for (int k = 0; k < 3; ++k) q[k] = k0[k] + t * (k1[k] - k0[k]);
      double y[3], yd[3];
      kelvin3(q, y);
      for (int k = 0; k < 3; ++k) yd[k] = y[k] - P0[k];
      bt = dot3(yd, e) / ee;
    }
  }
  *t_out = bt;
  return best;
}

/* Squared distance from p (inverted space, relative to the centre) to the
 * image of triangle (A, B, C) (relative to the centre), the nearest point q
 * and the barycentrics l of its image kappa(q) in (A, B, C). The plane
 * n . y = dd of the triangle (unit n) maps to the sphere through the origin
 * with centre n / (2 dd) and radius 1 / (2 |dd|); the nearest sphere point to
 * p is the radial projection, written stably in terms of dd so that a plane
 * through the centre (dd = 0: the image is that plane) is the limit; it
 * belongs to the patch when its image lies in the triangle. Otherwise the
 * nearest point of the patch lies on its boundary, the images of the three
 * edges (the distance to points of a sphere grows with their angle from the
 * radial projection). */
double orc_kelvin_tri_d2(const double* p, const double* A, const double* B, const double* C, double* q, double* l) {
  double best = INFINITY;
  double ab[3], ac[3], n[3];
  for (int k = 0; k < 3; ++k) { ab[k] = B[k] - A[k]; ac[k] = C[k] - A[k]; }
  cross3(ab, ac, n);
  double nl = sqrt(dot3(n, n));
  double scale = fmax(dot3(ab, ab), dot3(ac, ac));
  if (nl > 1e-12 * scale) {
    for (int k = 0; k < 3; ++k) n[k] /= nl;
    double dd = dot3(n, A);
    double qq[3];
    if (dd != 0.0) {
      double sg = dd > 0 ? 1.0 : -1.0, ad = fabs(dd);
      double v[3] = {dd * p[0] - 0.5 * n[0], dd * p[1] - 0.5 * n[1], dd * p[2] - 0.5 * n[2]};
      double vl = sqrt(dot3(v, v));
      double sd = (ad * dot3(p, p) - sg * dot3(n, p)) / (vl + 0.5); /* signed distance to the sphere */
      for (int k = 0; k < 3; ++k) qq[k] = p[k] - sd * sg * v[k] / vl;
    } else {
      double np = dot3(n, p);
      for (int k = 0; k < 3; ++k) qq[k] = p[k] - np * n[k];
    }
    double M2 = fmax(dot3(A, A), fmax(dot3(B, B), dot3(C, C)));
    if (dot3(qq, qq) * M2 >= 1.0 - 1e-9) { /* image points lie at least 1 / max|vertex| from the origin */
      double y[3], lb[3];
      kelvin3(qq, y);
      plane_bary(y, A, B, C, lb);
      if (lb[0] >= 0 && lb[1] >= 0 && lb[2] >= 0) {
        double d[3] = {p[0] - qq[0], p[1] - qq[1], p[2] - qq[2]};
        best = dot3(d, d);
        memcpy(q, qq, sizeof(qq));
        memcpy(l, lb, sizeof(lb));
      }
    }
  }
  const double* P[3] = {A, B, C};
  for (int e = 0; e < 3; ++e) {
    int i0 = e, i1 = (e + 1) % 3;
    double qe[3], t;
    double d2 = inv_seg_d2(p, P[i0], P[i1], qe, &t);
    if (d2 < best) {
      best = d2;
      memcpy(q, qe, sizeof(qe));
      l[0] = l[1] = l[2] = 0;
      l[i0] = 1 - t;
      l[i1] = t;
    }
  }
  return best;
}

/* A box containing the image of triangle t: each coordinate of
 * kappa(y) = y / |y|^2 for y in the triangle is a quotient of a number in the
 * triangle's coordinate range and one in [m2, M2], m2 the squared distance
 * from the centre to the triangle and M2 its largest squared vertex norm. */
static void kelvin_tri_box(const OrcKelvin* s, int64_t t, double* lo, double* hi) {
  const double* P[3] = {s->V + 3 * (int64_t)s->F[3 * t], s->V + 3 * (int64_t)s->F[3 * t + 1],
                        s->V + 3 * (int64_t)s->F[3 * t + 2]};
  double l[3], z[3] = {0, 0, 0};
  double m2 = orc_closest_tri(z, P[0], P[1], P[2], l);
  double M2 = fmax(dot3(P[0], P[0]), fmax(dot3(P[1], P[1]), dot3(P[2], P[2])));
  for (int k = 0; k < 3; ++k) {
    double a = fmin(P[0][k], fmin(P[1][k], P[2][k])), b = fmax(P[0][k], fmax(P[1][k], P[2][k]));
    if (a >= 0) { lo[k] = a / M2; hi[k] = b / m2; }
    else if (b <= 0) { lo[k] = a / m2; hi[k] = b / M2; }
    else { lo[k] = a / m2; hi[k] = b / m2; }
    double pad = 1e-12 * (fabs(lo[k]) + fabs(hi[k]));
    lo[k] -= pad; hi[k] += pad;
  }
}

static int64_t kelvin_build(OrcKelvin* s, int64_t lo, int64_t hi, double* key) {
  int64_t id = s->nnodes++;
  OrcNode* n = &s->nodes[id];
  double clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int k = 0; k < 3; ++k) { n->bmin[k] = INFINITY; n->bmax[k] = -INFINITY; }
  for (int64_t i = lo; i < hi; ++i) {
    int64_t t = s->order[i];
    for (int k = 0; k < 3; ++k) {
      n->bmin[k] = fmin(n->bmin[k], s->tlo[3 * t + k]);
      n->bmax[k] = fmax(n->bmax[k], s->thi[3 * t + k]);
      double c = 0.5 * (s->tlo[3 * t + k] + s->thi[3 * t + k]);
      clo[k] = fmin(clo[k], c); chi[k] = fmax(chi[k], c);
    }
  }
  n->lo = lo; n->hi = hi; n->left = n->right = -1;
  if (hi - lo <= 4) return id;
  int ax = 0;
  for (int k = 1; k < 3; ++k)
    if (chi[k] - clo[k] > chi[ax] - clo[ax]) ax = k;
  for (int64_t i = lo; i < hi; ++i) {
    int64_t t = s->order[i];
    key[t] = 0.5 * (s->tlo[3 * t + ax] + s->thi[3 * t + ax]);
  }
  g_sort_key = key;
  qsort(s->order + lo, (size_t)(hi - lo), sizeof(int64_t), cmp_key);
  int64_t mid = lo + (hi - lo) / 2;
  int64_t l = kelvin_build(s, lo, mid, key);
  int64_t r = kelvin_build(s, mid, hi, key);
  s->nodes[id].left = l;
  s->nodes[id].right = r;
  return id;
}

void* orc_kelvin_create(const float* V, int64_t nv, const int32_t* F, int64_t nf, const double* centre) {
  OrcKelvin* s = (OrcKelvin*)calloc(1, sizeof(OrcKelvin));
  s->nv = nv; s->nf = nf;
  s->V = (double*)malloc(sizeof(double) * 3 * nv);
  s->F = (int32_t*)malloc(sizeof(int32_t) * 3 * nf);
  memcpy(s->F, F, sizeof(int32_t) * 3 * nf);
  for (int k = 0; k < 3; ++k) { s->o[k] = centre[k]; s->lo[k] = INFINITY; s->hi[k] = -INFINITY; }
  double rmax = 0;
  for (int64_t i = 0; i < nv; ++i) {
    double y[3];
    for (int k = 0; k < 3; ++k) s->V[3 * i + k] = (double)V[3 * i + k] - centre[k];
    kelvin3(s->V + 3 * i, y);
    for (int k = 0; k < 3; ++k) { s->lo[k] = fmin(s->lo[k], y[k]); s->hi[k] = fmax(s->hi[k], y[k]); }
    rmax = fmax(rmax, sqrt(dot3(y, y)));
  }
  /* the inverted surface lies within 1 / (distance from the centre to the
   * mesh); the inverted vertices alone may miss bulging patches */
  double dmin = INFINITY;
  for (int64_t t = 0; t < nf; ++t) {
    double l[3], z[3] = {0, 0, 0};
    double d2 = orc_closest_tri(z, s->V + 3 * (int64_t)F[3 * t], s->V + 3 * (int64_t)F[3 * t + 1],
                                s->V + 3 * (int64_t)F[3 * t + 2], l);
    dmin = fmin(dmin, d2);
  }
  s->radius = fmax(rmax, 1.0 / sqrt(dmin));
  s->tlo = (double*)malloc(sizeof(double) * 3 * (size_t)nf);
  s->thi = (double*)malloc(sizeof(double) * 3 * (size_t)nf);
  for (int64_t t = 0; t < nf; ++t) kelvin_tri_box(s, t, s->tlo + 3 * t, s->thi + 3 * t);
  s->nodes = (OrcNode*)malloc(sizeof(OrcNode) * (size_t)(2 * nf + 1));
  s->order = (int64_t*)malloc(sizeof(int64_t) * (size_t)nf);
  double* key = (double*)malloc(sizeof(double) * (size_t)nf);
  for (int64_t i = 0; i < nf; ++i) s->order[i] = i;
  kelvin_build(s, 0, nf, key);
  free(key);
  return s;
}

void orc_kelvin_destroy(void* h) {
  OrcKelvin* s = (OrcKelvin*)h;
  free(s->V); free(s->F); free(s->tlo); free(s->thi); free(s->nodes); free(s->order); free(s);
}

void orc_kelvin_info(const void* h, double* lo, double* hi, double* radius) {
  const OrcKelvin* s = (const OrcKelvin*)h;
  for (int k = 0; k < 3; ++k) { lo[k] = s->lo[k]; hi[k] = s->hi[k]; }
  *radius = s->radius;
}

/* Nearest inverted triangle by brute force: minimum of (squared distance,
 * index) over all triangles; q = nearest point (inverted space), l = primal
 * barycentrics of its image. */
static double kelvin_tri(const OrcKelvin* s, int64_t t, const double* p, double* q, double* l) {
  return orc_kelvin_tri_d2(p, s->V + 3 * (int64_t)s->F[3 * t], s->V + 3 * (int64_t)s->F[3 * t + 1],
                           s->V + 3 * (int64_t)s->F[3 * t + 2], q, l);
}

static double kelvin_nearest_brute(const OrcKelvin* s, const double* p, int64_t* tri, double* q, double* l) {
  double best = INFINITY;
  *tri = -1;
  for (int64_t t = 0; t < s->nf; ++t) {
    double qq[3], ll[3];
    double d2 = kelvin_tri(s, t, p, qq, ll);
    if (d2 < best) {
      best = d2; *tri = t;
      memcpy(q, qq, sizeof(qq));
      memcpy(l, ll, sizeof(ll));
    }
  }
  return best;
}

/* The same minimum, visiting only boxes that can hold a closer image. */
static double kelvin_nearest(const OrcKelvin* s, const double* p, int64_t* tri, double* q, double* l) {
  double best = INFINITY;
  int64_t bi = -1;
  int64_t stack[256];
  int sp = 0;
  stack[sp++] = 0;
  while (sp > 0) {
    const OrcNode* n = &s->nodes[stack[--sp]];
    if (box_d2(n, p) > best * (1.0 + 1e-12)) continue;
    if (n->left < 0) {
      for (int64_t i = n->lo; i < n->hi; ++i) {
        int64_t t = s->order[i];
        double qq[3], ll[3];
        double d = kelvin_tri(s, t, p, qq, ll);
        if (d < best || (d == best && t < bi)) {
          best = d; bi = t;
          memcpy(q, qq, sizeof(qq));
          memcpy(l, ll, sizeof(ll));
        }
      }
    } else {
      double da = box_d2(&s->nodes[n->left], p), db = box_d2(&s->nodes[n->right], p);
      if (da <= db) { stack[sp++] = n->right; stack[sp++] = n->left; }
      else { stack[sp++] = n->left; stack[sp++] = n->right; }
      if (sp > 250) abort();
    }
  }
  *tri = bi;
  return best;
}

void orc_kelvin_nearest(const void* h, const double* Q, int64_t nq, int use_bvh, int64_t* tri, double* d2,
                        double* qpt, double* bary) {
  const OrcKelvin* s = (const OrcKelvin*)h;
  for (int64_t i = 0; i < nq; ++i)
    d2[i] = use_bvh ? kelvin_nearest(s, Q + 3 * i, tri + i, qpt + 3 * i, bary + 3 * i)
                    : kelvin_nearest_brute(s, Q + 3 * i, tri + i, qpt + 3 * i, bary + 3 * i);
}

/* Walk-on-Spheres in the inverted exterior from x (inverted space, relative
 * to the centre): a bounded domain, so every walk ends in the eps-shell (or
 * at the step cap). Same step rule and streams as the primal walks. */
static int kelvin_walk(const OrcKelvin* s, const OrcWalkParams* P, uint32_t row, uint32_t wk, double* x,
                       int64_t* tri, double* q, double* l, int64_t* nquery) {
  double eps2 = P->eps * P->eps;
  for (int64_t k = 0; k < P->max_steps; ++k) {
    double d2 = kelvin_nearest(s, x, tri, q, l);
    if (d2 < eps2) { *nquery = k + 1; return ST_HIT; }
    double u[4];
    draw4(P->seed, row, wk, (uint32_t)k, PURPOSE_STEP, P->mesh, u);
    double r = sqrt(d2) * (1.0 - P->kappa) - P->delta;
    double z = 1.0 - 2.0 * u[0];
    double rxy = 2.0 * sqrt(u[0] * (1.0 - u[0]));
    double phi = 2.0 * M_PI * u[1];
    x[0] += r * rxy * cos(phi);
    x[1] += r * rxy * sin(phi);
    x[2] += r * z;
  }
  kelvin_nearest(s, x, tri, q, l);
  *nquery = P->max_steps + 1;
  return ST_CAPPED;
}

/* Largest ball in the inverted exterior touching the inverted surface at
 * s~ (relative to the centre), with n~ its unit normal pointing out of the
 * inverted exterior: bisection as for the interior balls, a radius accepted
 * when the centre c = s~ - r n~ is at least r - min(tol, r/1024) from the
 * inverted surface and the ball lies within the inverted domain's bound. */
double orc_kelvin_tangent_ball(const void* h, const double* st, const double* nt, double r_max, int iters,
                               double tol) {
  const OrcKelvin* s = (const OrcKelvin*)h;
  double lo = 0.0, hi = r_max;
  for (int it = 0; it < iters; ++it) {
    double mid = 0.5 * (lo + hi);
    double c[3] = {st[0] - mid * nt[0], st[1] - mid * nt[1], st[2] - mid * nt[2]};
    int64_t tt;
    double qq[3], ll[3];
    double d = sqrt(kelvin_nearest(s, c, &tt, qq, ll));
    double t = mid - fmin(tol, mid * TANGENT_REL_TOL);
    if (d >= t && sqrt(dot3(c, c)) + mid <= s->radius) lo = mid;
    else hi = mid;
  }
  return lo;
}

/* The point s~ = kappa(s) and the unit normal n~ there pointing out of the
 * inverted exterior: the Kelvin Jacobian maps n_s to -|s~|^2 n~ (Appendix,
 * normal inversion), and it is |s~|^2 times the reflection H = I - 2 s^ s^T,
 * so n~ = -H n_s (s relative to the centre, n_s the outward unit normal). */
void orc_kelvin_point_normal(const double* s, const double* ns, double* st, double* nt) {
  double r = sqrt(dot3(s, s));
  double sh[3] = {s[0] / r, s[1] / r, s[2] / r};
  double sn = dot3(sh, ns);
  kelvin3(s, st);
  for (int k = 0; k < 3; ++k) nt[k] = -(ns[k] - 2.0 * sn * sh[k]);
}

/* The exterior estimate (Sec. 3.3, eq. main-exterior-estimator) over point
 * rows: row i's sample s_i (primal face, barycentrics, outward normal,
 * weight w_i) maps to s~_i; its tangent ball in the inverted exterior (radius
 * r_i, centre c~_i) gets `pairs` antithetic pairs of ball points drawn
 * proportionally to the ball's jump kernel outside the cap (as for the
 * interior PSD estimator), and a walk from each in the inverted exterior ends
 * at t~, whose image t is a primal surface point with basis values b(t). Per
 * pair p of row i the jump term adds
 *   X_p = alpha_i (d_1 d_1^T / |t~_1| + d_2 d_2^T / |t~_2|) / 2,
 *   alpha_i = w_i |s~_i|^3 Z_i / (2 pairs), d = b(s_i) - b(t),
 * (the exterior jump kernel |s~|^3 |t~|^3 J~(s~, t~), eq.
 * exterior-jump-kernel-final, with the surface element of the inverted
 * boundary |t~|^-4 times the primal one). The killing term (eq.
 * killing-measure-poisson-kernel) runs kill_walks walks from the origin of
 * the inverted space (the image of infinity); walk k (Philox row
 * 0xFFFFFFFF, walk k) ends at t~_0 and adds
 *   Y_k = (4 pi / |t~_0|) b(t_0) b(t_0)^T / kill_walks.
 * Outputs: Sj, Qj (sum of X and of X*X), Sk, Qk (same for Y), K x K each; per
 * row radius and Z; queries per row (bisection and walks) and of the killing
 * walks. */
void orc_kelvin_estimate(const void* h, int64_t n_rows, const float* p, const float* nrm, const int32_t* tri,
                         const float* bary, const double* w, const double* tab, int64_t K, int64_t pairs,
                         int64_t kill_walks, double theta0, double r_max, int bisect_iters, double eps, double kappa,
                         double delta, int64_t max_steps, uint64_t seed, uint32_t mesh, int nthreads, double* Sj,
                         double* Qj, double* Sk, double* Qk, double* radius, double* Zout, int64_t* n_query,
                         int64_t* kill_query, int32_t* log_status, int64_t* log_tri, float* log_bary) {
  const OrcKelvin* sc = (const OrcKelvin*)h;
  OrcWalkParams P = {eps, kappa, delta, max_steps, seed, mesh};
  memset(Sj, 0, sizeof(double) * K * K);
  memset(Qj, 0, sizeof(double) * K * K);
  memset(Sk, 0, sizeof(double) * K * K);
  memset(Qk, 0, sizeof(double) * K * K);
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads > 0 ? nthreads : 1)
  for (int64_t i = 0; i < n_rows; ++i) {
    double s[3], n[3], st[3], nt[3];
    for (int k = 0; k < 3; ++k) {
      s[k] = (double)p[3 * i + k] - sc->o[k];
      n[k] = nrm[3 * i + k];
    }
    double nl = sqrt(dot3(n, n));
    for (int k = 0; k < 3; ++k) n[k] /= nl;
    orc_kelvin_point_normal(s, n, st, nt);
    double r = orc_kelvin_tangent_ball(h, st, nt, r_max, bisect_iters, 0.5 * eps);
    radius[i] = r;
    Zout[i] = r > 0 ? orc_ball_jump_mass(r, theta0) : 0.0;
    n_query[i] = bisect_iters;
    if (r <= 0) continue;
    double c[3] = {st[0] - r * nt[0], st[1] - r * nt[1], st[2] - r * nt[2]};
    double sl = sqrt(dot3(st, st));
    double alpha = w[i] * sl * sl * sl * Zout[i] / (2.0 * (double)pairs);
    double* bs = (double*)calloc(K, sizeof(double));
    double* d = (double*)malloc(sizeof(double) * 2 * K);
    double* Si = (double*)calloc(K * K, sizeof(double));
    double* Qi = (double*)calloc(K * K, sizeof(double));
    for (int cc = 0; cc < 3; ++cc) {
      int64_t v = sc->F[3 * (int64_t)tri[i] + cc];
      for (int64_t k = 0; k < K; ++k) bs[k] += (double)bary[3 * i + cc] * tab[v * K + k];
    }
    for (int64_t j = 0; j < pairs; ++j) {
      double u[4], g[2];
      draw4(seed, (uint32_t)i, (uint32_t)j, 0, PURPOSE_BALL, mesh, u);
      for (int a = 0; a < 2; ++a) {
        double x[3], q[3], l[3];
        orc_ball_point(c, r, nt, theta0, u[0], u[1], a, x);
        int64_t tt = -1, nq = 0;
        int stt = kelvin_walk(sc, &P, (uint32_t)i, (uint32_t)(2 * j + a), x, &tt, q, l, &nq);
        n_query[i] += nq;
        g[a] = 1.0 / sqrt(dot3(q, q));
        for (int64_t k = 0; k < K; ++k) {
          double b = 0.0;
          for (int cc = 0; cc < 3; ++cc) b += l[cc] * tab[(int64_t)sc->F[3 * tt + cc] * K + k];
          d[a * K + k] = bs[k] - b;
        }
        if (log_status) {
          int64_t li = i * 2 * pairs + 2 * j + a;
          log_status[li] = stt;
          log_tri[li] = tt;
          log_bary[2 * li] = (float)l[1];
          log_bary[2 * li + 1] = (float)l[2];
        }
      }
      for (int64_t k = 0; k < K; ++k)
        for (int64_t m = 0; m < K; ++m) {
          double xv = 0.5 * alpha * (g[0] * d[k] * d[m] + g[1] * d[K + k] * d[K + m]);
          Si[k * K + m] += xv;
          Qi[k * K + m] += xv * xv;
        }
    }
#pragma omp critical
    {
      for (int64_t e = 0; e < K * K; ++e) { Sj[e] += Si[e]; Qj[e] += Qi[e]; }
    }
    free(bs); free(d); free(Si); free(Qi);
  }
  /* killing term: walks from the image of infinity */
  int64_t kq = 0;
  if (kill_walks > 0) {
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : 1)
    {
      double* b = (double*)malloc(sizeof(double) * K);
      double* Sl = (double*)calloc(K * K, sizeof(double));
      double* Ql = (double*)calloc(K * K, sizeof(double));
      int64_t ql = 0;
#pragma omp for schedule(dynamic, 64)
      for (int64_t k = 0; k < kill_walks; ++k) {
        double x[3] = {0, 0, 0}, q[3], l[3];
        int64_t tt = -1, nq = 0;
        kelvin_walk(sc, &P, 0xFFFFFFFFu, (uint32_t)k, x, &tt, q, l, &nq);
        ql += nq;
        double g = 4.0 * M_PI / sqrt(dot3(q, q)) / (double)kill_walks;
        for (int64_t a = 0; a < K; ++a) {
          b[a] = 0.0;
          for (int cc = 0; cc < 3; ++cc) b[a] += l[cc] * tab[(int64_t)sc->F[3 * tt + cc] * K + a];
        }
        for (int64_t a = 0; a < K; ++a)
          for (int64_t m = 0; m < K; ++m) {
            double yv = g * b[a] * b[m];
            Sl[a * K + m] += yv;
            Ql[a * K + m] += yv * yv;
          }
      }
#pragma omp critical
      {
        for (int64_t e = 0; e < K * K; ++e) { Sk[e] += Sl[e]; Qk[e] += Ql[e]; }
        kq += ql;
      }
      free(b); free(Sl); free(Ql);
    }
  }
  *kill_query = kq;
}
