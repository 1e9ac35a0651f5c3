// HIP kernels of the Walk-on-Spheres DtN estimator for gfx950.
//
// One wavefront lane carries one walk. Each step asks the BVH for the exact
// nearest triangle (the empty-ball radius, Sec. 2 "Walk-on-Spheres"), stops
// in the eps-shell, and otherwise jumps to a uniform point of the ball. The
// walk's hit is scattered into its row as c = b(s) - b(t) (Sec. 3.1, Alg. 1,
// eq. naive-stiffness-matrix). The persistent form keeps every lane busy by
// refilling finished lanes from a work queue (walks of a wavefront have very
// different lengths), with one queue per XCD over a contiguous, Z-ordered
// range of rows so that each XCD's L2 sees one region of the surface.
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstring>

#include "msk_internal.h"
#include "philox.h"

namespace msk {

__device__ __forceinline__ uint4 draw(const WalkLaunch& L, uint32_t row, uint32_t walk, uint32_t step,
                                      uint32_t purpose, uint32_t mesh) {
  return philox10(make_uint4(row, walk, step, (purpose << 24) | (mesh & 0xFFFFFFu)), L.seed_lo, L.seed_hi);
}

// --------------------------------------------------- FP32 closest point
// Squared distance from p to triangle T, evaluated in a fixed order with
// every product and sum rounded on its own (no contraction into FMA), so
// that it is reproducible bit for bit: Voronoi regions tested in the order
// vertex a, vertex b, edge ab, vertex c, edge ac, edge bc, face; face-region
// numerators n.(u x v) with n = ab x ac; face distance (n.ap)^2 / (n.n).
// (l1, l2) are the barycentric weights of vertices b and c.
//
// In the face region the barycentrics are returned as numerators (l1, l2 =
// vb, vc) over `den` (left unchanged in the other regions); they are divided
// only where a walk's final nearest point is used. A face whose squared
// plane distance exceeds `reject` by a safe margin returns +inf without
// dividing: it cannot beat or tie a current best of `reject`. Distances that
// are returned are exactly the values above.
__host__ __device__ __forceinline__ float tri_dist2(float px, float py, float pz, const TriRec& T, float reject,
                                                   float& l1, float& l2, float& den_out, int& region) {
#pragma clang fp contract(off)
  const float ax = T.a.x, ay = T.a.y, az = T.a.z;
  const float bx = T.b.x, by = T.b.y, bz = T.b.z;
  const float cx = T.c.x, cy = T.c.y, cz = T.c.z;
  const float abx = bx - ax, aby = by - ay, abz = bz - az;
  const float acx = cx - ax, acy = cy - ay, acz = cz - az;
  const float apx = px - ax, apy = py - ay, apz = pz - az;
  float t;
  t = abx * apx; t = t + aby * apy; const float d1 = t + abz * apz;
  t = acx * apx; t = t + acy * apy; const float d2 = t + acz * apz;
  if (d1 <= 0.0f && d2 <= 0.0f) {
    l1 = 0.0f; l2 = 0.0f; region = 0;
    t = apx * apx; t = t + apy * apy; return t + apz * apz;
  }
  const float bpx = px - bx, bpy = py - by, bpz = pz - bz;
  t = abx * bpx; t = t + aby * bpy; const float d3 = t + abz * bpz;
  t = acx * bpx; t = t + acy * bpy; const float d4 = t + acz * bpz;
  if (d3 >= 0.0f && d4 <= d3) {
    l1 = 1.0f; l2 = 0.0f; region = 1;
    t = bpx * bpx; t = t + bpy * bpy; return t + bpz * bpz;
  }
  const float nx = aby * acz - abz * acy;
  const float ny = abz * acx - abx * acz;
  const float nz = abx * acy - aby * acx;
  float xx = apy * bpz - apz * bpy, xy = apz * bpx - apx * bpz, xz = apx * bpy - apy * bpx;
  t = nx * xx; t = t + ny * xy; const float vc = t + nz * xz;
  if (vc <= 0.0f && d1 >= 0.0f && d3 <= 0.0f) {
    const float v = d1 / (d1 - d3);
    const float ex = px - (ax + v * abx), ey = py - (ay + v * aby), ez = pz - (az + v * abz);
    l1 = v; l2 = 0.0f; region = 2;
    t = ex * ex; t = t + ey * ey; return t + ez * ez;
  }
  const float cpx = px - cx, cpy = py - cy, cpz = pz - cz;
  t = abx * cpx; t = t + aby * cpy; const float d5 = t + abz * cpz;
  t = acx * cpx; t = t + acy * cpy; const float d6 = t + acz * cpz;
  if (d6 >= 0.0f && d5 <= d6) {
    l1 = 0.0f; l2 = 1.0f; region = 3;
    t = cpx * cpx; t = t + cpy * cpy; return t + cpz * cpz;
  }
  xx = cpy * apz - cpz * apy; xy = cpz * apx - cpx * apz; xz = cpx * apy - cpy * apx;
  t = nx * xx; t = t + ny * xy; const float vb = t + nz * xz;
  if (vb <= 0.0f && d2 >= 0.0f && d6 <= 0.0f) {
    const float w = d2 / (d2 - d6);
    const float ex = px - (ax + w * acx), ey = py - (ay + w * acy), ez = pz - (az + w * acz);
    l1 = 0.0f; l2 = w; region = 4;
    t = ex * ex; t = t + ey * ey; return t + ez * ez;
  }
  xx = bpy * cpz - bpz * cpy; xy = bpz * cpx - bpx * cpz; xz = bpx * cpy - bpy * cpx;
  t = nx * xx; t = t + ny * xy; const float va = t + nz * xz;
  const float e43 = d4 - d3, e56 = d5 - d6;
  if (va <= 0.0f && e43 >= 0.0f && e56 >= 0.0f) {
    const float w = e43 / (e43 + e56);
    const float bcx = cx - bx, bcy = cy - by, bcz = cz - bz;
    const float ex = px - (bx + w * bcx), ey = py - (by + w * bcy), ez = pz - (bz + w * bcz);
    l1 = 1.0f - w; l2 = w; region = 5;
    t = ex * ex; t = t + ey * ey; return t + ez * ez;
  }
  const float den = (va + vb) + vc;
  if (den > 0.0f) {
    region = 6;
    t = nx * apx; t = t + ny * apy; const float tn = t + nz * apz;
    t = nx * nx; t = t + ny * ny; const float nn = t + nz * nz;
    const float tt = tn * tn;
    // fl(tt / nn) > reject whenever tt > fl(fl(reject nn)(1 + 2^-20))
    if (tt > (reject * nn) * (1.0f + 0x1p-20f)) return INFINITY;
    l1 = vb; l2 = vc; den_out = den;
    return tt / nn;
  }
  // zero-area triangle: nearest point of the three edges, first strict minimum
  float best = INFINITY, bl1 = 0.0f, bl2 = 0.0f;
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    const float s0x = s == 2 ? bx : ax, s0y = s == 2 ? by : ay, s0z = s == 2 ? bz : az;
    const float s1x = s == 0 ? bx : cx, s1y = s == 0 ? by : cy, s1z = s == 0 ? bz : cz;
    const float ex = s1x - s0x, ey = s1y - s0y, ez = s1z - s0z;
    const float qx = px - s0x, qy = py - s0y, qz = pz - s0z;
    t = ex * ex; t = t + ey * ey; const float ee = t + ez * ez;
    t = qx * ex; t = t + qy * ey; const float qe = t + qz * ez;
    float u = ee > 0.0f ? qe / ee : 0.0f;
    if (u < 0.0f) u = 0.0f;
    if (u > 1.0f) u = 1.0f;
    const float rx = px - (s0x + u * ex), ry = py - (s0y + u * ey), rz = pz - (s0z + u * ez);
    t = rx * rx; t = t + ry * ry; const float dd = t + rz * rz;
    if (dd < best) {
      best = dd;
      bl1 = s == 0 ? u : (s == 1 ? 0.0f : 1.0f - u);
      bl2 = s == 0 ? 0.0f : u;
    }
  }
  l1 = bl1; l2 = bl2; region = 7;
  return best;
}

// ------------------------------------------------------- BVH traversal
// Squared-distance bound above which a box cannot hold a triangle whose FP32
// distance is <= best: the FP32 distance of a triangle is at least
// (d_true - slack)^2 (1 - 8u) with slack = 2^-18 (R + |p|_inf), and the FP32
// box distance at most its true value times (1 + 6u).
__host__ __device__ __forceinline__ float prune_bound(float best, float slack) {
  const float s = sqrtf(best) * (1.0f + 0x1p-20f) + slack;
  return s * s * (1.0f + 0x1p-20f);
}

// l1, l2 are the barycentrics of the nearest point, or for a face-region
// result their numerators over `den` (divided by nearest_bary where used).
struct Nearest {
  float d2;
  int32_t slot;
  int32_t orig;
  float l1, l2;
  float den = 1.0f;
};

__host__ __device__ __forceinline__ void nearest_bary(const Nearest& h, float& l1, float& l2) {
  l1 = h.l1;
  l2 = h.l2;
  if (h.den != 1.0f) {
    l1 = h.l1 / h.den;
    l2 = h.l2 / h.den;
  }
}

// FP32 operations of tri_dist2 up to each exit (vertex a, vertex b, edge ab,
// vertex c, edge ac, edge bc, face, zero-area fallback); a box lower bound
// costs 17 (6 subtractions, 6 maxima, 3 products, 2 sums).
constexpr uint32_t kTriFlops[8] = {24, 37, 71, 73, 98, 117, 114, 175};
constexpr uint32_t kBoxFlops = 17;

struct TravCount {
  uint32_t nodes = 0, tris = 0, flops = 0;
};

template <bool kStats>
__host__ __device__ __forceinline__ void test_tri(const TriRec* __restrict__ tris, int32_t s, float px, float py, float pz,
                                         Nearest& h, TravCount& cnt) {
  const TriRec T = tris[s];
  float l1 = 0.0f, l2 = 0.0f, den = 1.0f;
  int region = 0;
  const float d = tri_dist2(px, py, pz, T, h.d2, l1, l2, den, region);
  if (kStats) {
    ++cnt.tris;
    cnt.flops += kTriFlops[region & 7];
  }
  int32_t orig;
  memcpy(&orig, &T.a.w, 4);
  if (d < h.d2 || (d == h.d2 && orig < h.orig)) {
    h.d2 = d; h.slot = s; h.orig = orig; h.l1 = l1; h.l2 = l2;
    h.den = region == 6 ? den : 1.0f;
  }
}

// Exact nearest triangle: lexicographic minimum of (FP32 squared distance,
// original index). `h.slot` may name a candidate triangle on entry (warm
// start: the previous step's nearest), tested first so that the search starts
// with a finite bound. Each node test sorts the four children by box lower
// bound, tests the leaf children's triangles at once (nearest first), keeps
// the nearest surviving inner child in registers as the next node and pushes
// the other inner children farthest first; entries are popped only when the
// current subtree is done, and skipped when their bound no longer reaches the
// best distance. (Measured on gfx950 against a stack that also holds leaves
// and against a loop that defers leaves until every lane of the wavefront
// holds one: this order is the fastest of the three.)
struct StackEntry {
  int32_t node;
  float lb;
};

template <bool kStats, bool kStopBelow = false>
__host__ __device__ void bvh_nearest(const Node4* __restrict__ nodes, const TriRec* __restrict__ tris, const Node4* lds,
                                     int32_t n_lds, float px, float py, float pz, float radius, Nearest& h,
                                     TravCount& cnt, float stop_below = 0.0f) {
  const float slack = 0x1p-18f * (radius + fmaxf(fabsf(px), fmaxf(fabsf(py), fabsf(pz))));
  if (h.slot >= 0) {
    const int32_t s = h.slot;
    h.d2 = INFINITY;
    h.orig = INT_MAX;
    h.slot = -1;
    test_tri<kStats>(tris, s, px, py, pz, h, cnt);
  }
  float thr = prune_bound(h.d2, slack);
  StackEntry stk[kStackDepth];
  int sp = 0;
  int32_t node = 0;
  while (true) {
    float4 lox, loy, loz, hix, hiy, hiz;
    int4 ch, ct;
    if (kStats) {
      ++cnt.nodes;
      cnt.flops += 4 * kBoxFlops;
    }
    if (node < n_lds) {
      const float4* N = (const float4*)&lds[node];
      lox = N[0]; loy = N[1]; loz = N[2]; hix = N[3]; hiy = N[4]; hiz = N[5];
      ch = ((const int4*)N)[6]; ct = ((const int4*)N)[7];
    } else {
      const float4* N = (const float4*)&nodes[node];
      lox = N[0]; loy = N[1]; loz = N[2]; hix = N[3]; hiy = N[4]; hiz = N[5];
      ch = ((const int4*)N)[6]; ct = ((const int4*)N)[7];
    }
    float lb[4];
    int32_t cc[4], cn[4];
    {
      const float lx[4] = {lox.x, lox.y, lox.z, lox.w}, ly[4] = {loy.x, loy.y, loy.z, loy.w},
                  lz[4] = {loz.x, loz.y, loz.z, loz.w};
      const float hx[4] = {hix.x, hix.y, hix.z, hix.w}, hy[4] = {hiy.x, hiy.y, hiy.z, hiy.w},
                  hz[4] = {hiz.x, hiz.y, hiz.z, hiz.w};
      const int32_t c4[4] = {ch.x, ch.y, ch.z, ch.w}, n4[4] = {ct.x, ct.y, ct.z, ct.w};
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const float gx = fmaxf(fmaxf(lx[k] - px, px - hx[k]), 0.0f);
        const float gy = fmaxf(fmaxf(ly[k] - py, py - hy[k]), 0.0f);
        const float gz = fmaxf(fmaxf(lz[k] - pz, pz - hz[k]), 0.0f);
        lb[k] = gx * gx + gy * gy + gz * gz;
        cc[k] = c4[k];
        cn[k] = n4[k];
      }
    }
    // sort the four children by lower bound (5 compare-exchanges)
#define MSK_CX(i, j)                                                        \
  if (lb[j] < lb[i]) {                                                      \
    float tl = lb[i]; lb[i] = lb[j]; lb[j] = tl;                            \
    int32_t tc = cc[i]; cc[i] = cc[j]; cc[j] = tc;                          \
    int32_t tn = cn[i]; cn[i] = cn[j]; cn[j] = tn;                          \
  }
    MSK_CX(0, 1) MSK_CX(2, 3) MSK_CX(0, 2) MSK_CX(1, 3) MSK_CX(1, 2)
#undef MSK_CX
    // leaves, nearest first (an unused slot has count 0)
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (cc[k] < 0 && cn[k] > 0 && lb[k] <= thr) {
        const int32_t first = -cc[k] - 1;
        const float before = h.d2;
        for (int32_t s = first; s < first + cn[k]; ++s) test_tri<kStats>(tris, s, px, py, pz, h, cnt);
        if (h.d2 != before) {
          thr = prune_bound(h.d2, slack);
          // kStopBelow: only whether some triangle lies closer than
          // stop_below is asked, and this one does
          if (kStopBelow && sqrtf(h.d2) < stop_below) return;
        }
      }
    }
    // the nearest surviving inner child is next; the others are pushed
    // farthest first
    int32_t next = -1;
    float next_lb = 0.0f;
#pragma unroll
    for (int k = 3; k >= 0; --k) {
      if (cc[k] >= 0 && lb[k] <= thr) {
        if (next >= 0 && sp < kStackDepth) stk[sp++] = StackEntry{next, next_lb};
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
      if (stk[sp].lb <= thr) {
        node = stk[sp].node;
        break;
      }
    }
    if (node < 0) break;
  }
}

// Wavefront-cooperative leaf tests (same result as the lane-private
// bvh_nearest, bit for bit). All 64 lanes take part; each lane walks its own
// nodes, but the triangles of the leaves it reaches are listed in LDS and
// tested 64 at a time by the whole wavefront, so the long triangle test runs
// with most lanes busy instead of a few. A task's (squared distance, original
// index) goes to its owner through a 64-bit LDS atomic minimum, which
// realises the lexicographic order exactly; the task that holds the minimum
// writes its barycentrics for the owner. Work is listed in units of up to 4
// consecutive triangle slots of one owner (one word: first slot << 6 | owner
// lane, so meshes have fewer than 2^26 triangles); 4 lanes take a unit.
constexpr int kCoopUnits = 64;  // units per listing window (4 passes of 64 lanes)
struct CoopScratch {
  uint32_t unit[kCoopUnits];
  uint8_t ucnt[kCoopUnits];
  unsigned long long key[64];
  float4 pt[64];           // owner's query point and early-reject bound
  const TriRec* tris[64];  // lane's triangle array (batched meshes differ per lane)
  const Node4* nodes[64];  // lane's node array
  int32_t rec_slot[64];
  float rec_l1[64], rec_l2[64], rec_den[64];
  uint32_t flops[64];  // statistics kernels only
};

__device__ __forceinline__ uint32_t mbcnt64(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Orders LDS accesses of a wavefront as written: the hardware executes one
// wavefront's LDS instructions in issue order, so only the compiler must
// not move them (a fence would also wait for all outstanding global and
// scratch accesses).
__device__ __forceinline__ void lds_order() { __asm__ __volatile__("" ::: "memory"); }

// Exclusive prefix sum over the wavefront of a count below 64 (bit-sliced
// ballots); `total` receives the wavefront's sum.
__device__ __forceinline__ uint32_t wave_prefix_small(uint32_t v, uint32_t& total) {
  uint32_t pre = 0, tot = 0;
#pragma unroll
  for (int b = 0; b < 6; ++b) {
    const uint64_t m = __ballot((v >> b) & 1u);
    pre += mbcnt64(m) << b;
    tot += (uint32_t)__popcll(m) << b;
  }
  total = tot;
  return pre;
}

template <bool kStats>
__device__ void coop_unit_round(CoopScratch* W, uint32_t lane, uint32_t nunit) {
  for (uint32_t u0 = 0; u0 < nunit; u0 += 16) {
    const uint32_t u = u0 + (lane >> 2), off = lane & 3u;
    if (u < nunit && off < (uint32_t)W->ucnt[u]) {
      const uint32_t pk = W->unit[u];
      const int32_t s = (int32_t)(pk >> 6) + (int32_t)off;
      const uint32_t o = pk & 63u;
      const float4 q = W->pt[o];
      const TriRec T = W->tris[o][s];
      float l1 = 0.0f, l2 = 0.0f, den = 1.0f;
      int region = 0;
      const float d = tri_dist2(q.x, q.y, q.z, T, q.w, l1, l2, den, region);
      if (kStats) atomicAdd(&W->flops[o], kTriFlops[region & 7]);
      if (d <= q.w) {
        int32_t orig;
        memcpy(&orig, &T.a.w, 4);
        const unsigned long long key = ((unsigned long long)__float_as_uint(d) << 32) | (uint32_t)orig;
        atomicMin(&W->key[o], key);
        lds_order();
        if (W->key[o] == key) {
          W->rec_slot[o] = s;
          W->rec_l1[o] = l1;
          W->rec_l2[o] = l2;
          W->rec_den[o] = den;
        }
      }
    }
    lds_order();
  }
}


// ------------------------------------------------------ walk machinery

struct LaneWalk {
  float x, y, z;
  int32_t row;
  uint32_t walk;
  int32_t mesh;
  int32_t step;
  int32_t queries;
  int32_t slot;  // warm-start triangle slot
  int32_t active;
  TravCount cnt;  // traversal work of this walk (counted in the statistics kernels only)
  int32_t tab;    // wavefront row table of the walk (-1: device atomics)
  uint32_t ux, uy;  // direction uniforms of the current step (drawn before its query)
};

// Orthonormal frame (e1, e2) completing a unit vector n (branchless, after
// Duff et al. 2017).
__device__ __forceinline__ void onb(double nx, double ny, double nz, double e1[3], double e2[3]);

// Start of a walk of the PSD estimator (Sec. 3.2, Alg. 2): a point z on the
// tangent ball of row i's sample s (centre c = s - r n), drawn with density
// proportional to the ball's jump kernel 1 / (2 pi |s - z|^3) outside the cap
// of polar angle theta0 about s: u = sin(theta / 2) has density
// proportional to 1 / u^2 on [sin(theta0 / 2), 1], inverted in closed form,
// and the azimuth is uniform. Walks 2j and 2j + 1 are the antithetic pair j
// (azimuth and azimuth + pi). Returns false if the row has no tangent ball.
__device__ bool ball_start(const WalkLaunch& L, const MeshDev& M, LaneWalk& w, int32_t& face) {
  const double r = (double)M.ball_r[w.row];
  if (!(r > 0.0)) return false;
  face = M.tri[w.row];
  const double sx = M.p[3 * w.row], sy = M.p[3 * w.row + 1], sz = M.p[3 * w.row + 2];
  double nx = M.n[3 * w.row], ny = M.n[3 * w.row + 1], nz = M.n[3 * w.row + 2];
  const double nl = sqrt(nx * nx + ny * ny + nz * nz);
  nx /= nl; ny /= nl; nz /= nl;
  const double cx = sx - r * nx, cy = sy - r * ny, cz = sz - r * nz;
  const uint4 u = draw(L, (uint32_t)w.row, w.walk >> 1, 0, kPurposeBall, (uint32_t)M.mesh_id);
  const double xi = unit_f(u.x), eta = unit_f(u.y);
  const double su = 1.0 / (1.0 / M.ball_u0 - xi * (1.0 / M.ball_u0 - 1.0));
  const double ct = 1.0 - 2.0 * su * su, st = 2.0 * su * sqrt(fmax(0.0, 1.0 - su * su));
  double sp, cp;
  sincospi(2.0 * eta + ((w.walk & 1u) ? 1.0 : 0.0), &sp, &cp);
  double e1[3], e2[3];
  onb(nx, ny, nz, e1, e2);
  w.x = (float)(cx + r * (ct * nx + st * (cp * e1[0] + sp * e2[0])));
  w.y = (float)(cy + r * (ct * ny + st * (cp * e1[1] + sp * e2[1])));
  w.z = (float)(cz + r * (ct * nz + st * (cp * e1[2] + sp * e2[2])));
  w.slot = M.slot_of_tri[face];
  w.step = 0;
  w.queries = 0;
  w.cnt = TravCount();
  return true;
}

// Start of a walk: sample s (point rows: the fixed sample; hat rows:
// s ~ phi_i / A_i on the vertex's one-ring), inset it along the face normal.
// Returns false if the row is discarded.
__device__ bool walk_start(const WalkLaunch& L, const MeshDev& M, LaneWalk& w, int32_t& face, double lam[3]) {
  if (M.ball_r) return ball_start(L, M, w, face);
  const float sgn = M.side ? 1.0f : -1.0f;
  float sx, sy, sz, nx, ny, nz;
  if (M.mode == kRowsPoint) {
    if (M.discarded[w.row]) return false;
    face = M.tri[w.row];
    sx = M.p[3 * w.row]; sy = M.p[3 * w.row + 1]; sz = M.p[3 * w.row + 2];
    nx = M.n[3 * w.row]; ny = M.n[3 * w.row + 1]; nz = M.n[3 * w.row + 2];
    lam[0] = M.bary[3 * w.row]; lam[1] = M.bary[3 * w.row + 1]; lam[2] = M.bary[3 * w.row + 2];
  } else {
    const uint4 u = draw(L, (uint32_t)w.row, w.walk, 0, kPurposeHatStart, (uint32_t)M.mesh_id);
    const uint4 v = draw(L, (uint32_t)w.row, w.walk, 0, kPurposeSplit, (uint32_t)M.mesh_id);
    const int32_t b0 = M.ring_ptr[w.row], b1 = M.ring_ptr[w.row + 1];
    const double target = (double)unit_f(u.x) * M.ring_cum[b1 - 1];
    int32_t e = b0;
    while (e < b1 - 1 && !(M.ring_cum[e] > target)) ++e;
    face = M.ring_tri[e];
    const float m1 = unit_f(u.y), m2 = unit_f(u.z), m3 = unit_f(u.w);
    const float li = fmaxf(fminf(m1, m2), fminf(fmaxf(m1, m2), m3));  // median: Beta(2,2)
    const float sv = unit_f(v.x);
    const int32_t* f = M.faces + 3 * (int64_t)face;
    const int corner = f[0] == w.row ? 0 : (f[1] == w.row ? 1 : 2);
    // products of 24-bit values are exact in FP64: the weights sum to 1
    const double la = (1.0 - (double)li) * (double)sv, lb = (1.0 - (double)li) * (1.0 - (double)sv);
    lam[0] = corner == 0 ? (double)li : la;
    lam[1] = corner == 1 ? (double)li : (corner == 0 ? la : lb);
    lam[2] = corner == 2 ? (double)li : lb;
    const TriRec T = M.tris[M.slot_of_tri[face]];
    const float l0 = (float)lam[0], l1 = (float)lam[1], l2 = (float)lam[2];
    sx = l0 * T.a.x + l1 * T.b.x + l2 * T.c.x;
    sy = l0 * T.a.y + l1 * T.b.y + l2 * T.c.y;
    sz = l0 * T.a.z + l1 * T.b.z + l2 * T.c.z;
    nx = M.face_normals[3 * face]; ny = M.face_normals[3 * face + 1]; nz = M.face_normals[3 * face + 2];
  }
  const float h = M.inset;
  w.x = sx + sgn * h * nx;
  w.y = sy + sgn * h * ny;
  w.z = sz + sgn * h * nz;
  w.slot = M.slot_of_tri[face];
  w.step = 0;
  w.queries = 0;
  w.cnt = TravCount();
  return true;
}

// Sparse merge of up to NH sorted table rows with weights: emits each column
// once with sum_h weight_h * value_h (FP64).
template <int NH, typename Emit>
__device__ __forceinline__ void merge_rows(const MeshDev& M, const int32_t (&vtx)[NH], const double (&wt)[NH],
                                           Emit emit) {
  int32_t p[NH], e[NH];
#pragma unroll
  for (int k = 0; k < NH; ++k) {
    if (vtx[k] >= 0 && wt[k] != 0.0) {
      p[k] = M.b_rowptr[vtx[k]];
      e[k] = M.b_rowptr[vtx[k] + 1];
    } else {
      p[k] = 0;
      e[k] = 0;
    }
  }
  while (true) {
    int32_t cmin = INT_MAX;
    int32_t col[NH];
#pragma unroll
    for (int k = 0; k < NH; ++k) {
      col[k] = p[k] < e[k] ? M.b_col[p[k]] : INT_MAX;
      cmin = min(cmin, col[k]);
    }
    if (cmin == INT_MAX) break;
    double v = 0.0;
#pragma unroll
    for (int k = 0; k < NH; ++k) {
      if (col[k] == cmin) {
        v += wt[k] * (double)M.b_val[p[k]];
        ++p[k];
      }
    }
    emit(cmin, v);
  }
}

// ---- point basis (point-based k-NN interpolator)
// The k nearest sample points of q, as the k smallest (squared FP32 distance,
// index) pairs, searched ring by ring of grid cells around q's cell: after
// ring R every unvisited point lies outside the block of (2R + 1)^3 cells, so
// the search ends once the k-th distance is below the squared distance from q
// to that block's boundary (with a margin for rounding) or the block covers
// the grid. Weights exp(-d^2 / (2 sigma^2)) exp(-(1 - n_q . n_j) / tau),
// normalised (equal shares if all underflow). Returns the neighbour count.
__device__ __noinline__ int knn_eval(const KnnDev& G, float qx, float qy, float qz, double nqx, double nqy,
                                     double nqz, int32_t idx[kMaxKnn], double w[kMaxKnn]) {
#pragma clang fp contract(off)
  const int k = G.k;
  float bd[kMaxKnn];
  int m = 0;
  const float q[3] = {qx, qy, qz};
  int c[3];
  for (int a = 0; a < 3; ++a) {
    int ci = (int)floorf((q[a] - G.lo[a]) / G.cell);
    c[a] = min(max(ci, 0), G.dim[a] - 1);
  }
  for (int R = 0;; ++R) {
    for (int dz = -R; dz <= R; ++dz) {
      const int z = c[2] + dz;
      if (z < 0 || z >= G.dim[2]) continue;
      for (int dy = -R; dy <= R; ++dy) {
        const int y = c[1] + dy;
        if (y < 0 || y >= G.dim[1]) continue;
        const bool face = (dz == -R || dz == R || dy == -R || dy == R);
        for (int dx = -R; dx <= R; dx += (face ? 1 : 2 * R)) {
          const int x = c[0] + dx;
          if (x >= 0 && x < G.dim[0]) {
            const int64_t cid = ((int64_t)z * G.dim[1] + y) * G.dim[0] + x;
            for (int32_t e = G.cell_start[cid]; e < G.cell_start[cid + 1]; ++e) {
              const int32_t j = G.cell_pts[e];
              const float4 pj = G.pts[j];
              const float ex = qx - pj.x, ey = qy - pj.y, ez = qz - pj.z;
              float d2 = ex * ex;
              d2 = d2 + ey * ey;
              d2 = d2 + ez * ez;
              if (m == k && !(d2 < bd[k - 1] || (d2 == bd[k - 1] && j < idx[k - 1]))) continue;
              int pos = m < k ? m++ : k - 1;
              while (pos > 0 && (d2 < bd[pos - 1] || (d2 == bd[pos - 1] && j < idx[pos - 1]))) {
                bd[pos] = bd[pos - 1];
                idx[pos] = idx[pos - 1];
                --pos;
              }
              bd[pos] = d2;
              idx[pos] = j;
            }
          }
          if (R == 0) break;
        }
      }
    }
    bool covers = true;
    float gap = INFINITY;
    for (int a = 0; a < 3; ++a) {
      covers = covers && c[a] - R <= 0 && c[a] + R >= G.dim[a] - 1;
      const float blo = G.lo[a] + (float)(c[a] - R) * G.cell, bhi = G.lo[a] + (float)(c[a] + R + 1) * G.cell;
      gap = fminf(gap, fminf(q[a] - blo, bhi - q[a]));
    }
    if (covers) break;
    if (m == k && gap > 0.0f && bd[k - 1] < (gap * gap) * (1.0f - 0x1p-16f)) break;
  }
  double sum = 0.0;
  for (int a = 0; a < m; ++a) {
    const float4 nj = G.nrm[idx[a]];
    w[a] = exp(-(double)bd[a] * G.inv2s2) * exp(-(1.0 - (nqx * nj.x + nqy * nj.y + nqz * nj.z)) * G.inv_tau);
    sum += w[a];
  }
  for (int a = 0; a < m; ++a) w[a] = sum > 0.0 ? w[a] / sum : 1.0 / m;
  return m;
}

// Hit point and unit face normal of a walk's nearest triangle (FP64 from the
// FP32 vertices and barycentrics), then the point basis there. Not inlined:
// the walk kernels keep their registers for the walk itself.
__device__ __noinline__ int knn_at_hit(const MeshDev& M, const Nearest& hit, int32_t idx[kMaxKnn],
                                       double w[kMaxKnn]) {
  double t[3], n[3];
  const TriRec T = M.tris[hit.slot];
  float b1, b2;
  nearest_bary(hit, b1, b2);
  const double l1 = b1, l2 = b2, l0 = (1.0 - l1) - l2;
  const double a[3] = {T.a.x, T.a.y, T.a.z}, b[3] = {T.b.x, T.b.y, T.b.z}, c[3] = {T.c.x, T.c.y, T.c.z};
  double e1[3], e2[3];
  for (int k = 0; k < 3; ++k) {
    t[k] = l0 * a[k] + l1 * b[k] + l2 * c[k];
    e1[k] = b[k] - a[k];
    e2[k] = c[k] - a[k];
  }
  n[0] = e1[1] * e2[2] - e1[2] * e2[1];
  n[1] = e1[2] * e2[0] - e1[0] * e2[2];
  n[2] = e1[0] * e2[1] - e1[1] * e2[0];
  const double nl = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
  if (nl > 0.0)
    for (int k = 0; k < 3; ++k) n[k] /= nl;
  return knn_eval(M.knn, (float)t[0], (float)t[1], (float)t[2], n[0], n[1], n[2], idx, w);
}

// Contribution of a finished walk to its row, emitted once per column:
// point rows emit b(t) (the start is fixed per row; the finalisation folds
// in b(s)), hat rows emit c = b(s) - b(t). Escaped walks have b(t) = 0.
template <bool kKnn, typename Emit>
__device__ void walk_contrib(const WalkLaunch& L, const MeshDev& M, const LaneWalk& w, bool has_t, const Nearest& hit,
                             Emit emit) {
  if (M.ball_r) return;  // PSD walks: the rank-one updates are formed from the walk log
  if constexpr (kKnn) {  // point basis: b(t) from the hit point's k nearest samples (point rows)
    if (M.knn.k > 0) {
      if (has_t) {
        int32_t idx[kMaxKnn];
        double wk[kMaxKnn];
        const int m = knn_at_hit(M, hit, idx, wk);
        for (int a = 0; a < m; ++a) emit(idx[a], wk[a]);
      }
      return;
    }
  }
  int32_t tv[3] = {-1, -1, -1};
  double tw[3] = {0.0, 0.0, 0.0};
  if (has_t) {
    const int32_t* f = M.faces + 3 * (int64_t)hit.orig;
    tv[0] = f[0]; tv[1] = f[1]; tv[2] = f[2];
    float b1, b2;
    nearest_bary(hit, b1, b2);
    const double l1 = b1, l2 = b2;
    tw[0] = (1.0 - l1) - l2; tw[1] = l1; tw[2] = l2;
  }
  if (M.mode == kRowsPoint) {
    if (has_t) merge_rows<3>(M, tv, tw, emit);
  } else {
    int32_t face;
    double lam[3];
    LaneWalk tmp = w;
    walk_start(L, M, tmp, face, lam);
    const int32_t* f = M.faces + 3 * (int64_t)face;
    const int32_t vv[6] = {f[0], f[1], f[2], tv[0], tv[1], tv[2]};
    const double ww[6] = {lam[0], lam[1], lam[2], -tw[0], -tw[1], -tw[2]};
    merge_rows<6>(M, vv, ww, emit);
  }
}

// Walk log and traversal statistics of a finished walk.
__device__ void walk_record(const WalkLaunch& L, const MeshDev& M, const LaneWalk& w, int32_t status, bool has_t,
                            const Nearest& hit) {
  if (L.stats) {
    atomicAdd(L.stats, (unsigned long long)w.cnt.nodes);
    atomicAdd(L.stats + 1, (unsigned long long)w.cnt.tris);
    atomicAdd(L.stats + 2, (unsigned long long)w.cnt.flops);
  }
  if (M.log_status) {
    const int64_t li = (int64_t)w.row * M.walks_per_row + ((int64_t)w.walk - L.walk_offset);
    M.log_status[li] = status;
    M.log_tri[li] = has_t ? hit.orig : -1;
    float b1, b2;
    nearest_bary(hit, b1, b2);
    M.log_bary[2 * li] = has_t ? b1 : 0.0f;
    M.log_bary[2 * li + 1] = has_t ? b2 : 0.0f;
    M.log_queries[li] = w.queries;
  }
}

__device__ __forceinline__ bool walk_has_t(const MeshDev& M, int32_t status, const Nearest& hit) {
  return status != kEscaped && hit.orig >= 0 && hit.orig < M.n_tris;
}

// Scatter a finished walk straight into its row with FP64 device atomics.
template <bool kKnn = false>
__device__ void walk_finish_global(const WalkLaunch& L, const MeshDev& M, const LaneWalk& w, int32_t status,
                                   const Nearest& hit) {
  const bool has_t = walk_has_t(M, status, hit);
  double* a1 = M.acc1 + (int64_t)w.row * M.K;
  double* a2 = M.acc2 + (int64_t)w.row * M.K;
  walk_contrib<kKnn>(L, M, w, has_t, hit, [&](int32_t j, double v) {
    atomicAdd(a1 + j, v);
    atomicAdd(a2 + j, v * v);
  });
  atomicAdd(M.row_queries + w.row, (unsigned long long)w.queries);
  if (status == kEscaped) atomicAdd(M.row_escaped + w.row, 1ull);
  if (status == kCapped) atomicAdd(M.row_capped + w.row, 1ull);
  walk_record(L, M, w, status, has_t, hit);
}

// ---- wavefront row tables (persistent form)
// Each wavefront owns two small open-addressing tables in LDS, column ->
// (sum v, sum v^2), plus the row's query / escape / cap counts. The walks of
// one queue chunk (one row) add into one table with LDS atomics; when the
// chunk's last walk has finished, the wavefront flushes the table into the
// FP64 row with one device atomic per distinct column. AccT = double keeps
// the partial sums in FP64; AccT = float keeps them in FP32 (a chunk holds at
// most `chunk` walks) and flushes them into the FP64 rows; AccT = CompF32
// keeps them as compensated FP32 pairs.
// Row-table slots per wavefront table (2^bits) and the occupancy the
// persistent kernels are compiled for: with 64 slots, the cooperative leaf
// scratch and 21 LDS-staged top nodes a workgroup holds 29.8 KB of LDS.
// The streaming kernel measured fastest on gfx950 at 4 waves per SIMD (128
// VGPRs, few spills) against 3 (no spills) and 5, 6 (many spills); 32-slot
// tables lost to their extra device atomics and 128 slots gained nothing.
#ifndef MSK_TABLE_SLOT_BITS
#define MSK_TABLE_SLOT_BITS 6
#endif
constexpr int kSlotBits = MSK_TABLE_SLOT_BITS, kSlots = 1 << kSlotBits, kProbes = 8, kWaves = 4;
constexpr int32_t kEmptyKey = -1;

// Compensated FP32 partial sum: the value is hi + lo, a double-float pair.
// An addition of x = xh + xl (the FP64 contribution split into two floats)
// forms s = fl(hi + xh) and its exact rounding error e by Knuth's TwoSum,
// then lo += e + xl; the pair is one 64-bit LDS word replaced by
// compare-and-swap, so concurrent lanes on one slot serialise and none is
// lost. The sum's error is then of order u^2 n max|x| plus u |sum| for the
// final rounding of lo, instead of u n max|x| for a plain FP32 sum (u =
// 2^-24, n terms).
struct CompF32 {
  float hi, lo;
};

template <typename AccT>
__device__ __forceinline__ AccT acc_zero() {
  return (AccT)0;
}
template <>
__device__ __forceinline__ CompF32 acc_zero<CompF32>() {
  return CompF32{0.0f, 0.0f};
}
__device__ __forceinline__ double acc_value(double a) { return a; }
__device__ __forceinline__ double acc_value(float a) { return (double)a; }
__device__ __forceinline__ double acc_value(CompF32 a) { return (double)a.hi + (double)a.lo; }

__device__ __forceinline__ void lds_acc_add(double* p, double v) { atomicAdd(p, v); }
__device__ __forceinline__ void lds_acc_add(float* p, double v) { atomicAdd(p, (float)v); }
__device__ __forceinline__ void lds_acc_add(CompF32* p, double v) {
#pragma clang fp contract(off)
  const float xh = (float)v;
  const float xl = (float)(v - (double)xh);
  unsigned long long* q = reinterpret_cast<unsigned long long*>(p);
  unsigned long long old = __atomic_load_n(q, __ATOMIC_RELAXED), seen;
  do {
    seen = old;
    const float hi = __uint_as_float((uint32_t)seen), lo = __uint_as_float((uint32_t)(seen >> 32));
    const float sum = hi + xh;
    const float bv = sum - hi;
    const float err = (hi - (sum - bv)) + (xh - bv);
    const float nlo = lo + (err + xl);
    const unsigned long long nw =
        (unsigned long long)__float_as_uint(sum) | ((unsigned long long)__float_as_uint(nlo) << 32);
    old = atomicCAS(q, seen, nw);
  } while (old != seen);
}

template <typename AccT>
struct WaveTables {
  int32_t key[kWaves][2][kSlots];
  AccT v1[kWaves][2][kSlots];
  AccT v2[kWaves][2][kSlots];
  unsigned long long cnt[kWaves][2][3];
};

template <typename AccT>
__device__ __forceinline__ void table_add(WaveTables<AccT>& T, int wi, int t, int32_t j, double v, double* g1,
                                          double* g2) {
  const uint32_t h = ((uint32_t)j * 2654435761u) >> (32 - kSlotBits);
#pragma unroll 1
  for (int p = 0; p < kProbes; ++p) {
    const uint32_t si = (h + (uint32_t)p) & (kSlots - 1);
    const int32_t old = atomicCAS(&T.key[wi][t][si], kEmptyKey, j);
    if (old == kEmptyKey || old == j) {
      lds_acc_add(&T.v1[wi][t][si], v);
      lds_acc_add(&T.v2[wi][t][si], v * v);
      return;
    }
  }
  atomicAdd(g1 + j, v);  // table full along this probe sequence
  atomicAdd(g2 + j, v * v);
}

template <typename AccT, bool kKnn = false>
__device__ void walk_finish_table(const WalkLaunch& L, const MeshDev& M, const LaneWalk& w, int32_t status,
                                  const Nearest& hit, WaveTables<AccT>& T, int wi) {
  const bool has_t = walk_has_t(M, status, hit);
  double* a1 = M.acc1 + (int64_t)w.row * M.K;
  double* a2 = M.acc2 + (int64_t)w.row * M.K;
  walk_contrib<kKnn>(L, M, w, has_t, hit, [&](int32_t j, double v) { table_add(T, wi, w.tab, j, v, a1, a2); });
  atomicAdd(&T.cnt[wi][w.tab][0], (unsigned long long)w.queries);
  if (status == kEscaped) atomicAdd(&T.cnt[wi][w.tab][1], 1ull);
  if (status == kCapped) atomicAdd(&T.cnt[wi][w.tab][2], 1ull);
  walk_record(L, M, w, status, has_t, hit);
}

// Wavefront-cooperative flush of table t into row `row` of mesh `mesh`.
template <typename AccT>
__device__ void table_flush(const WalkLaunch& L, WaveTables<AccT>& T, int wi, int t, int32_t mesh, int32_t row) {
  __builtin_amdgcn_wave_barrier();
  const MeshDev& F = L.meshes[mesh];
  double* a1 = F.acc1 + (int64_t)row * F.K;
  double* a2 = F.acc2 + (int64_t)row * F.K;
  for (int i = (int)__lane_id(); i < kSlots; i += 64) {
    const int32_t j = T.key[wi][t][i];
    if (j != kEmptyKey) {
      atomicAdd(a1 + j, acc_value(T.v1[wi][t][i]));
      atomicAdd(a2 + j, acc_value(T.v2[wi][t][i]));
      T.key[wi][t][i] = kEmptyKey;
      T.v1[wi][t][i] = acc_zero<AccT>();
      T.v2[wi][t][i] = acc_zero<AccT>();
    }
  }
  if (__lane_id() == 0) {
    if (T.cnt[wi][t][0]) atomicAdd(F.row_queries + row, T.cnt[wi][t][0]);
    if (T.cnt[wi][t][1]) atomicAdd(F.row_escaped + row, T.cnt[wi][t][1]);
    if (T.cnt[wi][t][2]) atomicAdd(F.row_capped + row, T.cnt[wi][t][2]);
    T.cnt[wi][t][0] = T.cnt[wi][t][1] = T.cnt[wi][t][2] = 0;
  }
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ void onb(double nx, double ny, double nz, double e1[3], double e2[3]) {
  const double sg = nz >= 0 ? 1.0 : -1.0;
  const double a = -1.0 / (sg + nz);
  const double b = nx * ny * a;
  e1[0] = 1.0 + sg * nx * nx * a; e1[1] = sg * b; e1[2] = -sg * nx;
  e2[0] = b; e2[1] = sg + ny * ny * a; e2[2] = -ny;
}

// One step of a live walk. Returns -1 while the walk continues, else its
// final status (hit / escaped / capped) with `hit` set for hits and caps.
// First half of a WoS step (Sec. 2; exterior roulette of Sec. 3.3): the step
// cap, and outside the bounding sphere escape or re-entry. Returns kEscaped
// when the walk ends here, else -1: the walk needs the nearest-triangle
// query at (w.x, w.y, w.z); `capped` marks the query that ends a capped walk.
__device__ int32_t walk_begin(const WalkLaunch& L, const MeshDev& M, LaneWalk& w, bool& capped) {
  capped = w.step >= M.max_steps;
  // step cap: the walk ends at the nearest boundary point of its position
  if (capped) return -1;
  const uint4 u = draw(L, (uint32_t)w.row, w.walk, (uint32_t)w.step, kPurposeStep, (uint32_t)M.mesh_id);
  w.ux = u.x;
  w.uy = u.y;
  const float rho2 = w.x * w.x + w.y * w.y + w.z * w.z;
  const double rho = rho2 > M.radius * M.radius * (1.0f - 0x1p-18f)
                         ? sqrt((double)w.x * w.x + (double)w.y * w.y + (double)w.z * w.z)
                         : 0.0;
  if (rho > M.radius_d) {
    // Outside the bounding sphere: escape with probability 1 - R/rho, else
    // jump to the exact first hitting point of the sphere (density ~
    // |x-y|^-3, inverted in closed form).
    const double R = M.radius_d;
    if ((double)unit_f(u.z) < 1.0 - R / rho) return kEscaped;
    const double a = rho * rho + R * R, b = 2.0 * rho * R;
    const double qi = 1.0 / (rho + R) + (double)unit_f(u.w) * (1.0 / (rho - R) - 1.0 / (rho + R));
    const double mu = fmin(1.0, fmax(-1.0, (a - 1.0 / (qi * qi)) / b));
    const uint4 v = draw(L, (uint32_t)w.row, w.walk, (uint32_t)w.step, kPurposeReentry, (uint32_t)M.mesh_id);
    const double phi = 6.283185307179586 * (double)unit_f(v.x);
    const double nx = w.x / rho, ny = w.y / rho, nz = w.z / rho;
    double e1[3], e2[3];
    onb(nx, ny, nz, e1, e2);
    const double st = sqrt(fmax(0.0, 1.0 - mu * mu));
    double sp, cp;
    sincos(phi, &sp, &cp);
    w.x = (float)(R * (mu * nx + st * (cp * e1[0] + sp * e2[0])));
    w.y = (float)(R * (mu * ny + st * (cp * e1[1] + sp * e2[1])));
    w.z = (float)(R * (mu * nz + st * (cp * e1[2] + sp * e2[2])));
    // the walk goes on from the sphere in this same step (u.x, u.y unused so far)
  }
  return -1;
}

// Second half: with the query's answer in `hit`, stop in the eps-shell or
// take the ball step r (shrunk by the conservative guard) along a uniform
// direction. Returns kCapped / kHit when the walk ends, else -1.
__device__ int32_t walk_end(const MeshDev& M, LaneWalk& w, bool capped, const Nearest& hit) {
  ++w.queries;
  if (capped) return kCapped;
  w.slot = hit.slot;
  if (hit.d2 < M.eps2) return kHit;
  const float r = sqrtf(hit.d2) * (1.0f - M.kappa) - M.delta;
  const float u0 = unit_f(w.ux), u1 = unit_f(w.uy);
  const float z = 1.0f - 2.0f * u0;
  const float rxy = 2.0f * sqrtf(u0 * (1.0f - u0));
  // v_sin/v_cos take the angle in revolutions: sin(2 pi u1), cos(2 pi u1)
  const float sn = __builtin_amdgcn_sinf(u1), cs = __builtin_amdgcn_cosf(u1);
  w.x += r * rxy * cs;
  w.y += r * rxy * sn;
  w.z += r * z;
  ++w.step;
  return -1;
}

// One whole step with a lane-private query (plain kernel).
template <bool kStats>
__device__ int32_t walk_step(const WalkLaunch& L, const MeshDev& M, const Node4* lds, int32_t n_lds, LaneWalk& w,
                             Nearest& hit) {
  bool capped;
  const int32_t st = walk_begin(L, M, w, capped);
  if (st >= 0) return st;
  hit.d2 = INFINITY;
  hit.orig = INT_MAX;
  hit.slot = w.slot;
  bvh_nearest<kStats>(M.nodes, M.tris, lds, n_lds, w.x, w.y, w.z, M.radius, hit, w.cnt);
  return walk_end(M, w, capped, hit);
}

__device__ __forceinline__ void decode_walk(const WalkLaunch& L, uint64_t g, LaneWalk& w) {
  const uint64_t slot = g / (uint64_t)L.walks_per_slot;
  const RowSlot rs = L.slots[slot];
  w.mesh = rs.mesh;
  w.row = rs.row;
  w.walk = (uint32_t)((int64_t)(g - slot * (uint64_t)L.walks_per_slot) + L.walk_offset + rs.walk0);
}

// ------------------------------------------------------------- kernels

// Plain form: one thread per walk, run to completion.
template <bool kStats, bool kKnn = false>
__global__ void __launch_bounds__(256) walk_plain_kernel(WalkLaunch L) {
  const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (uint64_t)L.n_slots * (uint64_t)L.walks_per_slot) return;
  LaneWalk w;
  decode_walk(L, g, w);
  const MeshDev& M = L.meshes[w.mesh];
  int32_t face;
  double lam[3];
  if (!walk_start(L, M, w, face, lam)) return;
  Nearest hit;
  int32_t st;
  do {
    st = walk_step<kStats>(L, M, nullptr, 0, w, hit);
  } while (st < 0);
  walk_finish_global<kKnn>(L, M, w, st, hit);
}

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

#ifndef MSK_LDS_TOP_NODES
#define MSK_LDS_TOP_NODES 21
#endif
// top BVH nodes staged in LDS by the persistent kernel in single-mesh
// launches (at most kMaxTop), in dynamic LDS: batched launches, whose lanes
// work on many meshes at once, reserve none
constexpr int kLdsTop = MSK_LDS_TOP_NODES < kMaxTop ? MSK_LDS_TOP_NODES : kMaxTop;
#ifndef MSK_PERSISTENT_WAVES_PER_EU
#define MSK_PERSISTENT_WAVES_PER_EU 4
#endif
#if MSK_PERSISTENT_WAVES_PER_EU > 0
#define MSK_PERSISTENT_OCCUPANCY __attribute__((amdgpu_waves_per_eu(MSK_PERSISTENT_WAVES_PER_EU)))
#else
#define MSK_PERSISTENT_OCCUPANCY
#endif
// Optional per-phase cycle counts of the streaming kernel (a measurement
// build only: -DMSK_PHASE_TIMING=1); phases are timed by the wavefront's
// shader clock at points every lane passes together.
// lanes with an answered query that trigger the step continuation
#ifndef MSK_STEP_MIN
#define MSK_STEP_MIN 16
#endif
constexpr int kStepMin = MSK_STEP_MIN;
#ifndef MSK_PHASE_TIMING
#define MSK_PHASE_TIMING 0
#endif
#if MSK_PHASE_TIMING
__device__ unsigned long long g_phase_cycles[16];
#define MSK_TICK(var) const uint64_t var = (uint64_t)__builtin_amdgcn_s_memtime()
#define MSK_ACC(i, a, b) ph[i] += (b) - (a)
#else
#define MSK_TICK(var)
#define MSK_ACC(i, a, b)
#endif

// Streaming form of the persistent kernel: every loop trip advances each
// traversing lane by one BVH node (its leaf triangles tested by the whole
// wavefront), so a lane whose query is long does not hold the others: lanes
// whose query is answered wait until enough of them do (L.regen_min), then
// finish their step, start the next one or take a new walk together. The
// walks, their queries and their results are those of the other forms.
template <bool kStats, typename AccT, bool kKnn = false>
__global__ void __launch_bounds__(256) MSK_PERSISTENT_OCCUPANCY walk_stream_kernel(WalkLaunch L) {
  extern __shared__ Node4 top[];  // kLdsTop nodes when L.use_lds_top, else none
  __shared__ WaveTables<AccT> T;
  __shared__ CoopScratch coop[kWaves];
  const int wi = threadIdx.x >> 6;
  CoopScratch* W = &coop[wi];
  for (int i = threadIdx.x; i < kWaves * 2 * kSlots; i += blockDim.x) {
    (&T.key[0][0][0])[i] = kEmptyKey;
    (&T.v1[0][0][0])[i] = acc_zero<AccT>();
    (&T.v2[0][0][0])[i] = acc_zero<AccT>();
  }
  for (int i = threadIdx.x; i < kWaves * 2 * 3; i += blockDim.x) (&T.cnt[0][0][0])[i] = 0;
  int32_t n_lds = 0;
  if (L.use_lds_top) {
    n_lds = min(L.n_top, kLdsTop);
    const int4* src = (const int4*)L.meshes[0].nodes;
    int4* dst = (int4*)top;
    for (int i = threadIdx.x; i < n_lds * 8; i += blockDim.x) dst[i] = src[i];
  }
  __syncthreads();
  const uint32_t lane = __lane_id();
  const int qhome = blockIdx.x & 7;
  int qi = 0;  // queues tried so far (uniform)
  uint64_t cur = 0, cend = 0;
  // wave-uniform table bookkeeping
  int32_t t_used[2] = {0, 0}, t_mesh[2] = {0, 0}, t_row[2] = {0, 0}, t_out[2] = {0, 0};
  int32_t c_tab = -1, c_mesh = -1, c_row = -1;  // current chunk's row and table
  LaneWalk w;
  w.active = 0;
  w.tab = -1;
  Nearest hit;
  hit.d2 = INFINITY;
  hit.orig = INT_MAX;
  hit.slot = -1;
  hit.l1 = hit.l2 = 0.0f;
  // lane's state: mode 0 no walk, 1 traversing, 2 query answered (hit holds
  // it), 3 walk ended (hit and fin_status hold its result until the next
  // bookkeeping pass records it)
  int32_t mode = 0, node = -1, sp = 0, warm = -1, fin_status = -1;
  float thr = INFINITY, slack = 0.0f;
  bool capped = false;
  // traversal stack: its top entry in registers (tn, tl), the rest in
  // private memory; a pop takes the registers and starts reading the next
  // entry, which is not needed before the following pop
  StackEntry stk[kStackDepth];
  int32_t tn = -1;
  float tl = 0.0f;
  bool drained = false;
#if MSK_PHASE_TIMING
  uint64_t ph[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#endif
  auto start_query = [&](const MeshDev& M) {
    hit.d2 = INFINITY;
    hit.orig = INT_MAX;
    hit.slot = -1;
    warm = w.slot;
    node = 0;
    sp = 0;
    tn = -1;
    thr = INFINITY;
    slack = 0x1p-18f * (M.radius + fmaxf(fabsf(w.x), fmaxf(fabsf(w.y), fabsf(w.z))));
    W->nodes[lane] = M.nodes;
    W->tris[lane] = M.tris;
    mode = 1;
  };
  while (true) {
    // ---- bookkeeping, when enough lanes wait or none traverses: ended walks
    // are recorded and idle lanes take new walks
    MSK_TICK(tk0);
    // ---- steps whose query is answered: finish the step and start the next
    // one, once kStepMin lanes wait or none traverses; an ended walk waits
    // for the bookkeeping pass below
    {
      const uint64_t pend = __ballot(mode == 2);
      if (pend != 0 && (__ballot(mode == 1) == 0 || (int)__popcll(pend) >= kStepMin)) {
        if (mode == 2) {
          const MeshDev& M = L.meshes[w.mesh];
          int32_t st = walk_end(M, w, capped, hit);
          if (st < 0) {
            st = walk_begin(L, M, w, capped);
            if (st < 0) start_query(M);
          }
          if (st >= 0) {
            fin_status = st;
            mode = 3;
          }
        }
      }
    }
    MSK_TICK(tk0b);
    MSK_ACC(5, tk0, tk0b);
    const uint64_t trav = __ballot(mode == 1);
    if (trav == 0 || (int)__popcll(__ballot(mode == 0 || mode == 3)) >= L.regen_min) {
#if MSK_PHASE_TIMING
      ph[7] += 1;
#endif
      bool fin = false;
      int32_t fin_tab = -1;
      if (mode == 3) {
        const MeshDev& M = L.meshes[w.mesh];
        if (w.tab >= 0)
          walk_finish_table<AccT, kKnn>(L, M, w, fin_status, hit, T, wi);
        else
          walk_finish_global<kKnn>(L, M, w, fin_status, hit);
        fin = true;
        fin_tab = w.tab;
        w.active = 0;
        w.tab = -1;
        mode = 0;
      }
      for (int t = 0; t < 2; ++t) {
        t_out[t] -= (int32_t)__popcll(__ballot(fin && fin_tab == t));
        // flush once the table's walks are done and its chunk hands out no more
        if (t_used[t] && t_out[t] == 0 && !(t == c_tab && cur < cend)) {
          table_flush(L, T, wi, t, t_mesh[t], t_row[t]);
          t_used[t] = 0;
          if (c_tab == t) c_tab = -1;
        }
      }
      // refill idle lanes from the queue chunks
      uint64_t idle = __ballot(!w.active);
      while (idle != 0 && !drained) {
        if (cur >= cend) {
          uint64_t start = 0;
          if (lane == 0) {
            const int q = (qhome + qi) & 7;
            start = atomicAdd(L.queue_next + q, (unsigned long long)L.chunk);
          }
          start = (uint64_t)__shfl((unsigned long long)start, 0);
          const int q = (qhome + qi) & 7;
          const uint64_t qend = L.queue_end[q];
          if (start >= qend) {
            ++qi;
            if (qi >= 8) drained = true;
            continue;
          }
          cur = start;
          cend = min(start + (uint64_t)L.chunk, qend);
          // the chunk's row takes the table it already has, else a free one
          const RowSlot rs = L.slots[start / (uint64_t)L.walks_per_slot];
          c_mesh = rs.mesh;
          c_row = rs.row;
          c_tab = -1;
          for (int t = 0; t < 2; ++t)
            if (t_used[t] && t_mesh[t] == c_mesh && t_row[t] == c_row) c_tab = t;
          if (c_tab < 0) {
            for (int t = 0; t < 2; ++t)
              if (!t_used[t] && c_tab < 0) {
                c_tab = t;
                t_used[t] = 1;
                t_mesh[t] = c_mesh;
                t_row[t] = c_row;
              }
          }
        }
        const uint32_t rank = __popcll(idle & ((1ull << lane) - 1ull));
        const uint64_t avail = cend - cur;
        const uint32_t take = (uint32_t)min(avail, (uint64_t)__popcll(idle));
        bool fresh = false;
        if (!w.active && rank < take) {
          decode_walk(L, cur + rank, w);
          int32_t face;
          double lam[3];
          const MeshDev& M = L.meshes[w.mesh];
          w.active = walk_start(L, M, w, face, lam) ? 1 : 0;
          w.tab = (w.active && c_tab >= 0 && w.mesh == c_mesh && w.row == c_row) ? c_tab : -1;
          if (w.active) {
            const int32_t s0 = walk_begin(L, M, w, capped);
            if (s0 < 0) {
              start_query(M);
              fresh = w.tab >= 0;
            } else {  // left the bounding sphere at once and escaped
              if (w.tab >= 0)
                walk_finish_table<AccT, kKnn>(L, M, w, s0, hit, T, wi);
              else
                walk_finish_global<kKnn>(L, M, w, s0, hit);
              w.active = 0;
              w.tab = -1;
            }
          }
        }
        if (c_tab >= 0) t_out[c_tab] += (int32_t)__popcll(__ballot(fresh));
        cur += take;
        idle = __ballot(!w.active);
        // lanes whose row was discarded, or whose walk ended at once, stay idle
      }
      if (__ballot(w.active) == 0) {
        if (drained) {
          for (int t = 0; t < 2; ++t)
            if (t_used[t]) {
              table_flush(L, T, wi, t, t_mesh[t], t_row[t]);
              t_used[t] = 0;
            }
          break;
        }
        continue;
      }
    }
    MSK_TICK(tk1);
    MSK_ACC(0, tk0, tk1);
    if (__ballot(mode == 1) == 0) continue;
#if MSK_PHASE_TIMING
    ph[6] += 1;
#endif
    // ---- one node of every traversing lane
    const bool tr = mode == 1;
    float lb[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    int32_t cc[4] = {-1, -1, -1, -1}, cn[4] = {0, 0, 0, 0};
    if (tr) {
      const int32_t nl = w.mesh == 0 ? n_lds : 0;
      float4 lox, loy, loz, hix, hiy, hiz;
      int4 ch, ct;
      if (kStats) {
        ++w.cnt.nodes;
        w.cnt.flops += 4 * kBoxFlops;
      }
      if (node < nl) {
        const float4* N = (const float4*)&top[node];
        lox = N[0]; loy = N[1]; loz = N[2]; hix = N[3]; hiy = N[4]; hiz = N[5];
        ch = ((const int4*)N)[6]; ct = ((const int4*)N)[7];
      } else {
        const float4* N = (const float4*)&W->nodes[lane][node];
        lox = N[0]; loy = N[1]; loz = N[2]; hix = N[3]; hiy = N[4]; hiz = N[5];
        ch = ((const int4*)N)[6]; ct = ((const int4*)N)[7];
      }
      const float lx[4] = {lox.x, lox.y, lox.z, lox.w}, ly[4] = {loy.x, loy.y, loy.z, loy.w},
                  lz[4] = {loz.x, loz.y, loz.z, loz.w};
      const float hx[4] = {hix.x, hix.y, hix.z, hix.w}, hy[4] = {hiy.x, hiy.y, hiy.z, hiy.w},
                  hz[4] = {hiz.x, hiz.y, hiz.z, hiz.w};
      const int32_t c4[4] = {ch.x, ch.y, ch.z, ch.w}, n4[4] = {ct.x, ct.y, ct.z, ct.w};
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const float gx = fmaxf(fmaxf(lx[k] - w.x, w.x - hx[k]), 0.0f);
        const float gy = fmaxf(fmaxf(ly[k] - w.y, w.y - hy[k]), 0.0f);
        const float gz = fmaxf(fmaxf(lz[k] - w.z, w.z - hz[k]), 0.0f);
        lb[k] = gx * gx + gy * gy + gz * gz;
        cc[k] = c4[k];
        cn[k] = n4[k];
      }
#define MSK_CX(i, j)                                                        \
  if (lb[j] < lb[i]) {                                                      \
    float tl = lb[i]; lb[i] = lb[j]; lb[j] = tl;                            \
    int32_t tc = cc[i]; cc[i] = cc[j]; cc[j] = tc;                          \
    int32_t tn = cn[i]; cn[i] = cn[j]; cn[j] = tn;                          \
  }
      MSK_CX(0, 1) MSK_CX(2, 3) MSK_CX(0, 2) MSK_CX(1, 3) MSK_CX(1, 2)
#undef MSK_CX
    }
    MSK_TICK(tk2);
    MSK_ACC(1, tk1, tk2);
    // this lane's triangles: the warm-start candidate of a new query, then
    // the leaf children within the bound
    const int32_t hw = (tr && warm >= 0) ? 1 : 0;
    int32_t nl4[4], tot = hw;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      nl4[k] = (tr && cc[k] < 0 && cn[k] > 0 && lb[k] <= thr) ? cn[k] : 0;
      tot += nl4[k];
    }
    if (__ballot(tot > 0) != 0) {
      W->pt[lane] = make_float4(w.x, w.y, w.z, hit.d2);
      W->key[lane] = ((unsigned long long)__float_as_uint(hit.d2) << 32) | (uint32_t)hit.orig;
      if (kStats) W->flops[lane] = 0;
      // lay the units out by a prefix sum over the lanes, in windows of kCoopUnits
      int32_t nu = hw;
#pragma unroll
      for (int k = 0; k < 4; ++k) nu += (nl4[k] + 3) >> 2;
      uint32_t total;
      const uint32_t pre = wave_prefix_small((uint32_t)nu, total);
      for (uint32_t w0 = 0; w0 < total; w0 += (uint32_t)kCoopUnits) {
        const uint32_t w1 = w0 + (uint32_t)kCoopUnits;
        if (nu > 0 && pre < w1 && pre + (uint32_t)nu > w0) {
          uint32_t pos = pre;
          auto put = [&](uint32_t first, uint32_t cnt) {
            if (pos >= w0 && pos < w1) {
              W->unit[pos - w0] = (first << 6) | lane;
              W->ucnt[pos - w0] = (uint8_t)cnt;
            }
            ++pos;
          };
          if (hw) put((uint32_t)warm, 1u);
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            uint32_t first = (uint32_t)(-cc[k] - 1);
            for (int32_t c = nl4[k]; c > 0; c -= 4, first += 4) put(first, (uint32_t)min(c, 4));
          }
        }
        lds_order();
        MSK_TICK(tr0);
        coop_unit_round<kStats>(W, lane, min(total - w0, (uint32_t)kCoopUnits));
        MSK_TICK(tr1);
        MSK_ACC(3, tr0, tr1);
      }
      if (tot > 0) {
        if (kStats) {
          w.cnt.tris += (uint32_t)tot;
          w.cnt.flops += W->flops[lane];
        }
        const unsigned long long k2 = W->key[lane];
        const float d = __uint_as_float((uint32_t)(k2 >> 32));
        const int32_t orig = (int32_t)(uint32_t)k2;
        if (d < hit.d2 || (d == hit.d2 && orig < hit.orig)) {
          hit.d2 = d;
          hit.orig = orig;
          hit.slot = W->rec_slot[lane];
          hit.l1 = W->rec_l1[lane];
          hit.l2 = W->rec_l2[lane];
          hit.den = W->rec_den[lane];
          thr = prune_bound(hit.d2, slack);
        }
      }
    }
    MSK_TICK(tk3);
    MSK_ACC(2, tk2, tk3);
    if (tr) {
      warm = -1;
      // the nearest surviving inner child is next; the others are pushed
      // farthest first; the query is answered when the stack runs out
      int32_t next = -1;
      float next_lb = 0.0f;
#pragma unroll
      for (int k = 3; k >= 0; --k) {
        if (cc[k] >= 0 && lb[k] <= thr) {
          if (next >= 0) {  // push the farther candidate
            if (tn >= 0 && sp < kStackDepth) stk[sp++] = StackEntry{tn, tl};
            tn = next;
            tl = next_lb;
          }
          next = cc[k];
          next_lb = lb[k];
        }
      }
      if (next >= 0) {
        node = next;
      } else {
        node = -1;
        while (tn >= 0) {
          const int32_t cand = tn;
          const float cl = tl;
          if (sp > 0) {
            --sp;
            tn = stk[sp].node;
            tl = stk[sp].lb;
          } else {
            tn = -1;
          }
          if (cl <= thr) {
            node = cand;
            break;
          }
        }
        if (node < 0) mode = 2;  // query answered
      }
    }
    MSK_TICK(tk4);
    MSK_ACC(4, tk3, tk4);
  }
#if MSK_PHASE_TIMING
  if (lane == 0)
    for (int i = 0; i < 8; ++i) atomicAdd(&g_phase_cycles[i], (unsigned long long)ph[i]);
#endif
}

__global__ void init_queues_kernel(unsigned long long* next, unsigned long long* end, QueueInit q) {
  const int i = threadIdx.x;
  if (i < 8) {
    next[i] = q.begin[i];
    end[i] = q.end[i];
  }
}

__global__ void fill_u64_kernel(unsigned long long* p, int64_t n, unsigned long long v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void fill_u32_kernel(uint32_t* p, int64_t n, uint32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// Point rows whose inset point is closer than h/2 to the surface are
// discarded (the inset left the thin region it should probe).
// Largest ball inside the domain tangent at each point row's sample s, centre
// c = s - r n (Sec. 3.2; Alg. 2, LargestTangentBall): bisection over
// [0, r_max]; a radius is accepted when c's nearest surface point is at
// least t = r - min(tol, 2^-10 r) away and the ball lies inside the scene's
// bounding sphere. 0 = no radius accepted. Each step needs only whether some
// triangle lies closer than t, so its query starts from the bound
// B = t^2 (1 + 2^-20) instead of +inf (when a triangle has sqrt(d2) < t then
// d2 < B) and stops at the first triangle found with sqrt(d2) < t; when none
// lies below B the ball is accepted. Same decisions as comparing the exact
// nearest distance with t, with only the boxes near the ball visited.
// Whether the ball of radius r touching s from the inside is accepted (the
// test of one bisection step).
__device__ bool tangent_ball_inside(const MeshDev& M, float sx, float sy, float sz, double nx, double ny, double nz,
                                    float mid, float tol, uint32_t& issued) {
  const double cxd = sx - mid * nx, cyd = sy - mid * ny, czd = sz - mid * nz;
  const float cx = (float)cxd, cy = (float)cyd, cz = (float)czd;
  const float t = mid - fminf(tol, mid * 0x1p-10f);
  const float bound = t > 0.0f ? (t * t) * (1.0f + 0x1p-20f) : 0.0f;
  Nearest h;
  h.d2 = bound; h.orig = INT_MAX; h.slot = -1;
  TravCount cnt;
  if (t > 0.0f) {
    bvh_nearest<false, true>(M.nodes, M.tris, nullptr, 0, cx, cy, cz, M.radius, h, cnt, t);
    ++issued;
  }
  const bool empty = h.orig == INT_MAX || sqrtf(h.d2) >= t;
  return empty && sqrt(cxd * cxd + cyd * cyd + czd * czd) + mid <= M.radius_d;
}

// The bisection of a row, three levels per round: the eight lanes of a row
// evaluate the (up to) seven midpoints of the next three levels at once (lane
// k takes heap node k of that subtree: node 1 the current midpoint, node 2k
// and 2k + 1 the midpoints of its lower and upper halves), then all follow
// the path the sequential bisection takes through them. Every midpoint is
// formed by the same float operations as in the sequential loop, so the
// radius is the same; the rounds of dependent queries drop from iters to
// ceil(iters / 3), and eight lanes per row fill the GPU with 16,384 rows.
// row_queries counts the bounded queries the lanes issue (up to seven per
// round of three levels, so more than the iters decisions they serve).
__global__ void __launch_bounds__(64) tangent_ball_kernel(MeshDev M, int64_t n_rows, float r_max, int32_t iters,
                                                          float tol, float* radius) {
  const int lane = threadIdx.x & 63, sub = lane & 7, gbase = lane & ~7;
  // eight rows per 64-lane workgroup; the loop bound is uniform over the
  // workgroup, so every lane takes part in every ballot
  for (int64_t base = (int64_t)blockIdx.x * 8; base < n_rows; base += (int64_t)gridDim.x * 8) {
    const int64_t i = base + (threadIdx.x >> 3);
    const bool valid = i < n_rows;
    float sx = 0.f, sy = 0.f, sz = 0.f;
    double nx = 0.0, ny = 0.0, nz = 1.0;
    if (valid) {
      sx = M.p[3 * i]; sy = M.p[3 * i + 1]; sz = M.p[3 * i + 2];
      nx = M.n[3 * i]; ny = M.n[3 * i + 1]; nz = M.n[3 * i + 2];
      const double nl = sqrt(nx * nx + ny * ny + nz * nz);
      nx /= nl; ny /= nl; nz /= nl;
    }
    float lo = 0.0f, hi = r_max;
    uint32_t issued = 0;
    for (int32_t done = 0; done < iters;) {
      const int levels = min(3, iters - done);
      bool res = false;
      if (valid && sub >= 1 && sub < (1 << levels)) {
        float a = lo, b = hi;
        const int depth = 31 - __clz(sub);  // bits of the node index below its leading one
        for (int j = depth - 1; j >= 0; --j) {
          const float m = 0.5f * (a + b);
          if ((sub >> j) & 1)
            a = m;
          else
            b = m;
        }
        res = tangent_ball_inside(M, sx, sy, sz, nx, ny, nz, 0.5f * (a + b), tol, issued);
      }
      const unsigned long long mask = __ballot(res);  // every lane of the wavefront takes part
      int node = 1;
      for (int l = 0; l < levels; ++l) {
        const float mid = 0.5f * (lo + hi);
        const int bit = (int)((mask >> (gbase + node)) & 1ull);
        if (bit)
          lo = mid;
        else
          hi = mid;
        node = 2 * node + bit;
      }
      done += levels;
    }
    if (valid && sub == 0) radius[i] = lo;
    if (valid && issued) atomicAdd(M.row_queries + i, (unsigned long long)issued);
  }
}

__device__ __forceinline__ void discard_row(const MeshDev& M, int64_t i, int32_t* discarded) {
  const float sgn = M.side ? 1.0f : -1.0f;
  const float x = M.p[3 * i] + sgn * M.inset * M.n[3 * i];
  const float y = M.p[3 * i + 1] + sgn * M.inset * M.n[3 * i + 1];
  const float z = M.p[3 * i + 2] + sgn * M.inset * M.n[3 * i + 2];
  Nearest h;
  h.d2 = INFINITY; h.orig = INT_MAX; h.slot = M.slot_of_tri[M.tri[i]];
  TravCount cnt;
  bvh_nearest<false>(M.nodes, M.tris, nullptr, 0, x, y, z, M.radius, h, cnt);
  discarded[i] = h.d2 < 0.25f * M.inset * M.inset ? 1 : 0;
  atomicAdd(M.row_queries + i, 1ull);
}

__global__ void discard_kernel(MeshDev M, int64_t n_rows, int32_t* discarded) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_rows) discard_row(M, i, discarded);
}

// The discard pass over the point rows of several meshes in one launch:
// launch index j belongs to the last range k with R[k].first <= j, as row
// j - R[k].first of mesh R[k].mesh.
__global__ void discard_batch_kernel(const MeshDev* __restrict__ meshes, const RowRange* __restrict__ R,
                                     int32_t n_ranges, int64_t n_total) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n_total) return;
  int32_t lo = 0, hi = n_ranges - 1;
  while (lo < hi) {
    const int32_t mid = (lo + hi + 1) >> 1;
    if (R[mid].first <= j)
      lo = mid;
    else
      hi = mid - 1;
  }
  const RowRange r = R[lo];
  discard_row(meshes[r.mesh], j - r.first, r.discarded);
}

__global__ void knn_eval_kernel(KnnDev G, double cx, double cy, double cz, const float* __restrict__ Q,
                                const float* __restrict__ Nq, int64_t n, int32_t* __restrict__ idx,
                                float* __restrict__ w) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float qx = (float)((double)Q[3 * i] - cx);
  const float qy = (float)((double)Q[3 * i + 1] - cy);
  const float qz = (float)((double)Q[3 * i + 2] - cz);
  double nx = Nq[3 * i], ny = Nq[3 * i + 1], nz = Nq[3 * i + 2];
  const double nl = sqrt(nx * nx + ny * ny + nz * nz);
  if (nl > 0.0) {
    nx /= nl; ny /= nl; nz /= nl;
  }
  int32_t id[kMaxKnn];
  double wk[kMaxKnn];
  const int m = knn_eval(G, qx, qy, qz, nx, ny, nz, id, wk);
  for (int a = 0; a < G.k; ++a) {
    idx[i * G.k + a] = a < m ? id[a] : -1;
    w[i * G.k + a] = a < m ? (float)wk[a] : 0.0f;
  }
}

__global__ void closest_points_kernel(const Node4* __restrict__ nodes, const TriRec* __restrict__ tris, float radius,
                                      double cx, double cy, double cz, const float* __restrict__ Q, int64_t nq,
                                      int32_t* tri, float* d2, float* bary) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nq) return;
  const float x = (float)((double)Q[3 * i] - cx);
  const float y = (float)((double)Q[3 * i + 1] - cy);
  const float z = (float)((double)Q[3 * i + 2] - cz);
  Nearest h;
  h.d2 = INFINITY; h.orig = INT_MAX; h.slot = -1;
  TravCount cnt;
  bvh_nearest<false>(nodes, tris, nullptr, 0, x, y, z, radius, h, cnt);
  tri[i] = h.orig;
  d2[i] = h.d2;
  nearest_bary(h, bary[2 * i], bary[2 * i + 1]);
}

// S_ij = (w_i / h) mean_ij, se_ij = (w_i / h) sqrt(var_ij / W_i), var with
// the unbiased (W-1) normalisation. Point rows hold sums of b(t) here and
// the entries where b(s) != 0 are corrected by finalize_point_fix_kernel.
__global__ void finalize_kernel(MeshDev M, int64_t n_rows, const int64_t* __restrict__ walks,
                                const double* __restrict__ w, double* S, double* se) {
  const int64_t n = n_rows * M.K;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n; idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx / M.K;
    const double Wi = (double)walks[i];
    const double scale = (M.mode == kRowsPoint && M.discarded[i]) ? 0.0 : w[i] / M.inset_d;
    const double s1 = M.mode == kRowsPoint ? -M.acc1[idx] : M.acc1[idx];
    const double mean = s1 / Wi;
    const double var = fmax(0.0, M.acc2[idx] / Wi - mean * mean) * (Wi / (Wi - 1.0));
    S[idx] = scale * mean;
    se[idx] = scale * sqrt(var / Wi);
  }
}

// With jump_only (exterior), the killing term is dropped (Sec. 3.3, exterior
// Beurling-Deny form; the paper's default exterior operator): an escaped
// walk contributes nothing instead of b(s), so b(s) enters once per walk
// that did not escape.
__global__ void finalize_point_fix_kernel(MeshDev M, int64_t n_rows, const int64_t* __restrict__ walks,
                                          const double* __restrict__ w, double* S, double* se, int32_t jump_only) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_rows || M.discarded[i]) return;
  const int32_t* f = M.faces + 3 * (int64_t)M.tri[i];
  const int32_t vv[3] = {f[0], f[1], f[2]};
  const double ww[3] = {(double)M.bary[3 * i], (double)M.bary[3 * i + 1], (double)M.bary[3 * i + 2]};
  const double Wi = (double)walks[i];
  const double Hi = jump_only ? Wi - (double)M.row_escaped[i] : Wi;  // walks that carry b(s)
  const double scale = w[i] / M.inset_d;
  auto fix = [&](int32_t j, double bs) {
    const int64_t idx = i * M.K + j;
    const double t1 = M.acc1[idx], t2 = M.acc2[idx];
    const double s1 = Hi * bs - t1;
    const double s2 = Hi * bs * bs - 2.0 * bs * t1 + t2;
    const double mean = s1 / Wi;
    const double var = fmax(0.0, s2 / Wi - mean * mean) * (Wi / (Wi - 1.0));
    S[idx] = scale * mean;
    se[idx] = scale * sqrt(var / Wi);
  };
  if (M.knn.k > 0) {
    double nx = M.n[3 * i], ny = M.n[3 * i + 1], nz = M.n[3 * i + 2];
    const double nl = sqrt(nx * nx + ny * ny + nz * nz);
    nx /= nl; ny /= nl; nz /= nl;
    int32_t idx[kMaxKnn];
    double wk[kMaxKnn];
    const int m = knn_eval(M.knn, M.p[3 * i], M.p[3 * i + 1], M.p[3 * i + 2], nx, ny, nz, idx, wk);
    for (int a = 0; a < m; ++a) fix(idx[a], wk[a]);
  } else {
    merge_rows<3>(M, vv, ww, fix);
  }
}

}  // namespace msk

// ------------------------------------------------------ launch wrappers

namespace msk {

static inline int blocks_for(int64_t n, int bs) { return (int)std::min<int64_t>((n + bs - 1) / bs, 1 << 20); }

hipError_t launch_walk_plain(const WalkLaunch& L, hipStream_t s) {
  const int64_t n = L.n_slots * L.walks_per_slot;
  if (n <= 0) return hipSuccess;
  const int64_t nb = (n + 255) / 256;
  if (nb > INT32_MAX) return hipErrorInvalidValue;
  if (L.knn && L.stats) return hipErrorInvalidValue;  // the point basis has no counting instantiation
  if (L.knn)
    hipLaunchKernelGGL((walk_plain_kernel<false, true>), dim3((unsigned)nb), dim3(256), 0, s, L);
  else if (L.stats)
    hipLaunchKernelGGL(walk_plain_kernel<true>, dim3((unsigned)nb), dim3(256), 0, s, L);
  else
    hipLaunchKernelGGL(walk_plain_kernel<false>, dim3((unsigned)nb), dim3(256), 0, s, L);
  return hipGetLastError();
}

hipError_t launch_walk_persistent(const WalkLaunch& L, int grid, hipStream_t s) {
  if (L.knn && L.stats) return hipErrorInvalidValue;  // the point basis has no counting instantiation
  if (L.accum < 0 || L.accum > 2) return hipErrorInvalidValue;
  const size_t lds = L.use_lds_top && kLdsTop > 0 ? sizeof(Node4) * kLdsTop : 0;
  if (L.knn) {  // point basis: instantiations carrying the k-NN evaluation
    if (L.accum == 1)
      hipLaunchKernelGGL((walk_stream_kernel<false, float, true>), dim3(grid), dim3(256), lds, s, L);
    else if (L.accum == 2)
      hipLaunchKernelGGL((walk_stream_kernel<false, CompF32, true>), dim3(grid), dim3(256), lds, s, L);
    else
      hipLaunchKernelGGL((walk_stream_kernel<false, double, true>), dim3(grid), dim3(256), lds, s, L);
  } else if (L.accum == 1) {
    if (L.stats)
      hipLaunchKernelGGL((walk_stream_kernel<true, float>), dim3(grid), dim3(256), lds, s, L);
    else
      hipLaunchKernelGGL((walk_stream_kernel<false, float>), dim3(grid), dim3(256), lds, s, L);
  } else if (L.accum == 2) {
    if (L.stats)
      hipLaunchKernelGGL((walk_stream_kernel<true, CompF32>), dim3(grid), dim3(256), lds, s, L);
    else
      hipLaunchKernelGGL((walk_stream_kernel<false, CompF32>), dim3(grid), dim3(256), lds, s, L);
  } else {
    if (L.stats)
      hipLaunchKernelGGL((walk_stream_kernel<true, double>), dim3(grid), dim3(256), lds, s, L);
    else
      hipLaunchKernelGGL((walk_stream_kernel<false, double>), dim3(grid), dim3(256), lds, s, L);
  }
  return hipGetLastError();
}

#if MSK_PHASE_TIMING
extern "C" int msk_debug_phase_cycles(unsigned long long* out, int reset) {
  if (hipMemcpyFromSymbol(out, HIP_SYMBOL(g_phase_cycles), sizeof(unsigned long long) * 8) != hipSuccess) return 1;
  if (reset) {
    unsigned long long z[16] = {0};
    if (hipMemcpyToSymbol(HIP_SYMBOL(g_phase_cycles), z, sizeof(z)) != hipSuccess) return 1;
  }
  return 0;
}
#endif

// Counts the non-finite entries of a (n values) into *count (grid-stride).
__global__ void count_nonfinite_kernel(const double* __restrict__ a, int64_t n, unsigned long long* count) {
  unsigned long long c = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    c += isfinite(a[i]) ? 0ull : 1ull;
  // wavefront sum, one atomic per wavefront with any
  for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
  if (__lane_id() == 0 && c) atomicAdd(count, c);
}

// Per-estimate totals of the per-row counters, one workgroup per estimate:
// out[6 k + 0..5] = queries, escaped walks, capped walks, discarded rows,
// walks of the kept rows, non-finite entries.
__global__ void row_totals_kernel(const RowCounters* __restrict__ sets, unsigned long long* __restrict__ out) {
  const RowCounters C = sets[blockIdx.x];
  __shared__ unsigned long long acc[5];
  if (threadIdx.x < 5) acc[threadIdx.x] = 0;
  __syncthreads();
  unsigned long long v[5] = {0, 0, 0, 0, 0};
  for (int64_t i = threadIdx.x; i < C.n; i += blockDim.x) {
    v[0] += C.queries[i];
    v[1] += C.escaped[i];
    v[2] += C.capped[i];
    const bool dropped = C.discarded[i] != 0;
    v[3] += dropped ? 1ull : 0ull;
    v[4] += dropped ? 0ull : (unsigned long long)C.walks[i];
  }
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off);
    if (__lane_id() == 0 && v[k]) atomicAdd(&acc[k], v[k]);
  }
  __syncthreads();
  if (threadIdx.x < 5) out[6 * blockIdx.x + threadIdx.x] = acc[threadIdx.x];
  if (threadIdx.x == 5) out[6 * blockIdx.x + 5] = *C.nonfinite;
}

hipError_t launch_count_nonfinite(const double* a, int64_t n, unsigned long long* count, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int blocks = (int)std::min<int64_t>(1024, (n + 255) / 256);
  hipLaunchKernelGGL(count_nonfinite_kernel, dim3(blocks), dim3(256), 0, s, a, n, count);
  return hipGetLastError();
}

hipError_t launch_init_queues(unsigned long long* next, unsigned long long* end, const QueueInit& q, hipStream_t s) {
  hipLaunchKernelGGL(init_queues_kernel, dim3(1), dim3(64), 0, s, next, end, q);
  return hipGetLastError();
}

hipError_t launch_fill_u64(void* p, int64_t n, unsigned long long v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_u64_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, (unsigned long long*)p, n, v);
  return hipGetLastError();
}

hipError_t launch_fill_u32(void* p, int64_t n, uint32_t v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_u32_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, (uint32_t*)p, n, v);
  return hipGetLastError();
}

hipError_t launch_discard(const MeshDev& M, int64_t n_rows, int32_t* discarded, hipStream_t s) {
  if (n_rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(discard_kernel, dim3(blocks_for(n_rows, 128)), dim3(128), 0, s, M, n_rows, discarded);
  return hipGetLastError();
}

hipError_t launch_discard_batch(const MeshDev* meshes, const RowRange* ranges, int32_t n_ranges, int64_t n_total,
                                hipStream_t s) {
  if (n_ranges <= 0 || n_total <= 0) return hipSuccess;
  hipLaunchKernelGGL(discard_batch_kernel, dim3(blocks_for(n_total, 128)), dim3(128), 0, s, meshes, ranges, n_ranges,
                     n_total);
  return hipGetLastError();
}

hipError_t launch_row_totals(const RowCounters* sets, int32_t n_sets, unsigned long long* out, hipStream_t s) {
  if (n_sets <= 0) return hipSuccess;
  hipLaunchKernelGGL(row_totals_kernel, dim3(n_sets), dim3(256), 0, s, sets, out);
  return hipGetLastError();
}

hipError_t launch_knn_eval(const KnnDev& G, const double* c, const float* Q, const float* Nq, int64_t n, int32_t* idx,
                           float* w, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(knn_eval_kernel, dim3(blocks_for(n, 128)), dim3(128), 0, s, G, c[0], c[1], c[2], Q, Nq, n, idx,
                     w);
  return hipGetLastError();
}

hipError_t launch_tangent_ball(const MeshDev& M, int64_t n_rows, float r_max, int32_t iters, float tol, float* radius,
                               hipStream_t s) {
  if (n_rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(tangent_ball_kernel, dim3(blocks_for(8 * n_rows, 64)), dim3(64), 0, s, M, n_rows, r_max, iters,
                     tol, radius);
  return hipGetLastError();
}

hipError_t launch_closest_points(const Node4* nodes, const TriRec* tris, float radius, const double* c, const float* Q,
                                 int64_t nq, int32_t* tri, float* d2, float* bary, hipStream_t s) {
  if (nq <= 0) return hipSuccess;
  if ((nq + 127) / 128 > INT32_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(closest_points_kernel, dim3((unsigned)((nq + 127) / 128)), dim3(128), 0, s, nodes, tris, radius,
                     c[0], c[1], c[2], Q, nq, tri, d2, bary);
  return hipGetLastError();
}

hipError_t launch_finalize(const MeshDev& M, int64_t n_rows, const int64_t* walks, const double* w, double* S,
                           double* se, hipStream_t s,
                           int32_t jump_only) {
  if (n_rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(finalize_kernel, dim3(blocks_for(n_rows * M.K, 256)), dim3(256), 0, s, M, n_rows, walks, w, S, se);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || M.mode != kRowsPoint) return e;
  hipLaunchKernelGGL(finalize_point_fix_kernel, dim3(blocks_for(n_rows, 128)), dim3(128), 0, s, M, n_rows, walks, w, S,
                     se, jump_only);
  return hipGetLastError();
}

}  // namespace msk
