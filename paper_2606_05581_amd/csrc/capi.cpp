// C ABI of libmsk (declared in include/msk.h): argument checking, device
// memory, row ordering, work queues and kernel launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/msk.h"
#include "msk_internal.h"
#include "eigen.h"
#include "kelvin.h"
#include "psd.h"
#include "laplace.h"

using namespace msk;

struct msk_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  int n_cu = 256;
  std::string err;
};

struct msk_mesh {
  msk_ctx* ctx = nullptr;
  double centre[3] = {0, 0, 0};
  double radius = 0, area = 0;
  int64_t nv = 0, nf = 0, n_nodes = 0;
  int depth = 0, leaf_size = 4, top_nodes = 85;
  Node4* d_nodes = nullptr;
  TriRec* d_tris = nullptr;
  int32_t* d_slot = nullptr;
  int32_t* d_faces = nullptr;
  std::vector<float> vrel;       // float offsets from the centre (host copy)
  std::vector<int32_t> faces;    // host copy
  std::vector<float> vworld;     // input vertices (host copy, for rebuilds)
};

struct msk_rows {
  msk_ctx* ctx = nullptr;
  const msk_mesh* mesh = nullptr;
  int32_t mode = 0;
  int64_t n = 0;
  std::vector<double> w;
  std::vector<int32_t> order;    // Z-order of the rows
  std::vector<float> p_world, n_world;  // point rows: host copies of the samples and normals
  double* d_w = nullptr;
  float* d_p = nullptr;
  float* d_n = nullptr;
  int32_t* d_tri = nullptr;
  float* d_bary = nullptr;
  int32_t* d_ring_ptr = nullptr;
  int32_t* d_ring_tri = nullptr;
  double* d_ring_cum = nullptr;
  float* d_fn = nullptr;
};

struct msk_basis {
  msk_ctx* ctx = nullptr;
  int64_t nv = 0, K = 0;
  // point basis (k nearest sample points): set for msk_basis_create_knn
  const msk_mesh* knn_mesh = nullptr;
  KnnDev kd{};
  float4* d_kpts = nullptr;
  float4* d_knrm = nullptr;
  int32_t* d_cell_start = nullptr;
  int32_t* d_cell_pts = nullptr;
  int32_t max_row_nnz = 0;  // the walk estimators merge at most kMaxTableNnz entries per vertex
  int32_t* d_rowptr = nullptr;
  int32_t* d_col = nullptr;
  float* d_val = nullptr;
};

struct msk_dtn {
  msk_ctx* ctx = nullptr;
  const msk_rows* rows = nullptr;
  int64_t n = 0, K = 0, W = 0;
  int32_t mode = 0;
  double inset = 0;
  double* d_S = nullptr;
  double* d_se = nullptr;
  double* d_acc1 = nullptr;
  double* d_acc2 = nullptr;
  unsigned long long* d_q = nullptr;
  unsigned long long* d_esc = nullptr;
  unsigned long long* d_cap = nullptr;
  int32_t* d_disc = nullptr;
  int64_t* d_walks = nullptr;
  int32_t* d_log_status = nullptr;
  int32_t* d_log_tri = nullptr;
  float* d_log_bary = nullptr;
  int32_t* d_log_q = nullptr;
  unsigned long long* d_nonfinite = nullptr;  // non-finite entries of S and se
  msk_dtn_info info{};
};

namespace {

msk_status fail(msk_ctx* ctx, msk_status st, const std::string& msg) {
  if (ctx) ctx->err = msg;
  return st;
}

#define HIP_TRY(ctx, expr)                                                                   \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      return fail(ctx, e_ == hipErrorOutOfMemory ? MSK_ERR_OOM : MSK_ERR_DEVICE,             \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                        \
  } while (0)

template <typename T>
hipError_t dalloc(T** p, size_t n) {
  *p = nullptr;
  if (n == 0) n = 1;
  return hipMalloc((void**)p, n * sizeof(T));
}

template <typename T>
hipError_t upload(msk_ctx* ctx, T** p, const T* src, size_t n) {
  hipError_t e = dalloc(p, n);
  if (e != hipSuccess) return e;
  if (n == 0) return hipSuccess;
  e = hipMemcpyAsync(*p, src, n * sizeof(T), hipMemcpyHostToDevice, ctx->stream);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(ctx->stream);
}

template <typename T>
void dfree(T*& p) {
  if (p) (void)hipFree((void*)p);
  p = nullptr;
}

uint64_t spread3(uint64_t x) {
  x &= 0x1FFFFF;
  x = (x | x << 32) & 0x1F00000000FFFFull;
  x = (x | x << 16) & 0x1F0000FF0000FFull;
  x = (x | x << 8) & 0x100F00F00F00F00Full;
  x = (x | x << 4) & 0x10C30C30C30C30C3ull;
  x = (x | x << 2) & 0x1249249249249249ull;
  return x;
}

// Z-order (Morton) permutation of points (Sec. 4: samples sorted along a
// Z-order curve so that neighbouring walks traverse the same BVH region).
std::vector<int32_t> morton_order(const std::vector<float>& P, int64_t n) {
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t i = 0; i < n; ++i)
    for (int k = 0; k < 3; ++k) {
      lo[k] = std::min(lo[k], P[3 * i + k]);
      hi[k] = std::max(hi[k], P[3 * i + k]);
    }
  std::vector<uint64_t> code((size_t)n);
  for (int64_t i = 0; i < n; ++i) {
    uint64_t c = 0;
    for (int k = 0; k < 3; ++k) {
      double ext = std::max(1e-30, (double)hi[k] - (double)lo[k]);
      uint64_t q = (uint64_t)std::min(2097151.0, std::max(0.0, ((double)P[3 * i + k] - lo[k]) / ext * 2097151.0));
      c |= spread3(q) << k;
    }
    code[i] = c;
  }
  std::vector<int32_t> ord((size_t)n);
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) { return code[a] < code[b]; });
  return ord;
}

bool finite3(const float* p) { return std::isfinite(p[0]) && std::isfinite(p[1]) && std::isfinite(p[2]); }

}  // namespace

// ------------------------------------------------------------- context

extern "C" msk_status msk_create(int device, void* hip_stream, msk_ctx** out) {
  if (!out) return MSK_ERR_INVALID_ARG;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return MSK_ERR_INVALID_ARG;
  if (hipSetDevice(device) != hipSuccess) return MSK_ERR_DEVICE;
  msk_ctx* c = new msk_ctx();
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
    c->n_cu = prop.multiProcessorCount;
  // the allocation-free estimate's workspace on this device (looked up once
  // per device; a failure is reported by that entry point, not here)
  (void)msk::noalloc_scratch_init(device);
  *out = c;
  return MSK_OK;
}

extern "C" void msk_destroy(msk_ctx* ctx) { delete ctx; }

extern "C" const char* msk_last_error(const msk_ctx* ctx) { return ctx ? ctx->err.c_str() : "no context"; }

// ---------------------------------------------------------------- mesh

extern "C" msk_status msk_build_bvh(msk_ctx* ctx, const float* V, int64_t n_verts, const int32_t* F, int64_t n_tris,
                                    const msk_bvh_opts* opts, msk_mesh** out) {
  if (!ctx || !out) return MSK_ERR_INVALID_ARG;
  *out = nullptr;
  if (!V || !F) return fail(ctx, MSK_ERR_INVALID_ARG, "null mesh arrays");
  if (n_verts >= INT32_MAX || n_tris >= (1ll << 30)) return fail(ctx, MSK_ERR_INVALID_ARG, "mesh too large");
  int leaf = opts && opts->leaf_size > 0 ? opts->leaf_size : 4;
  int top = opts ? opts->top_nodes : 85;
  if (top < 0 || top > kMaxTop) return fail(ctx, MSK_ERR_INVALID_ARG, "top_nodes must be in 0..85");
  HostBvh B;
  std::string e = build_bvh_host(V, n_verts, F, n_tris, leaf, B);
  if (!e.empty()) return fail(ctx, MSK_ERR_INVALID_ARG, e);
  msk_mesh* m = new msk_mesh();
  m->ctx = ctx;
  std::memcpy(m->centre, B.centre, sizeof(m->centre));
  m->radius = B.radius;
  m->area = B.area;
  m->nv = n_verts;
  m->nf = n_tris;
  m->n_nodes = (int64_t)B.nodes.size();
  m->depth = B.depth;
  m->leaf_size = leaf;
  m->top_nodes = (int)std::min<int64_t>(top, m->n_nodes);
  m->vrel.resize((size_t)n_verts * 3);
  for (int64_t i = 0; i < n_verts; ++i)
    for (int k = 0; k < 3; ++k) m->vrel[3 * i + k] = (float)((double)V[3 * i + k] - B.centre[k]);
  m->faces.assign(F, F + 3 * n_tris);
  m->vworld.assign(V, V + 3 * n_verts);
  hipError_t he;
  if ((he = upload(ctx, &m->d_nodes, B.nodes.data(), B.nodes.size())) != hipSuccess ||
      (he = upload(ctx, &m->d_tris, B.tris.data(), B.tris.size())) != hipSuccess ||
      (he = upload(ctx, &m->d_slot, B.slot_of_tri.data(), B.slot_of_tri.size())) != hipSuccess ||
      (he = upload(ctx, &m->d_faces, F, (size_t)n_tris * 3)) != hipSuccess) {
    msk_mesh_destroy(m);
    return fail(ctx, he == hipErrorOutOfMemory ? MSK_ERR_OOM : MSK_ERR_DEVICE,
                std::string("mesh upload: ") + hipGetErrorString(he));
  }
  *out = m;
  return MSK_OK;
}

extern "C" msk_status msk_mesh_get_info(const msk_mesh* m, msk_mesh_info* info) {
  if (!m || !info) return MSK_ERR_INVALID_ARG;
  std::memcpy(info->centre, m->centre, sizeof(info->centre));
  info->radius = m->radius;
  info->area = m->area;
  info->n_verts = m->nv;
  info->n_tris = m->nf;
  info->n_nodes = m->n_nodes;
  info->node_bytes = m->n_nodes * (int64_t)sizeof(Node4);
  info->tri_bytes = m->nf * (int64_t)sizeof(TriRec);
  info->depth = m->depth;
  info->leaf_size = m->leaf_size;
  return MSK_OK;
}

extern "C" void msk_mesh_destroy(msk_mesh* m) {
  if (!m) return;
  dfree(m->d_nodes);
  dfree(m->d_tris);
  dfree(m->d_slot);
  dfree(m->d_faces);
  delete m;
}

extern "C" msk_status msk_closest_points(msk_ctx* ctx, const msk_mesh* m, const float* Q, int64_t nq, int32_t* tri,
                                         float* d2, float* bary) {
  if (!ctx || !m) return MSK_ERR_INVALID_ARG;
  if (nq < 0 || (nq > 0 && (!Q || !tri || !d2 || !bary))) return fail(ctx, MSK_ERR_INVALID_ARG, "bad query arrays");
  if (nq == 0) return MSK_OK;
  HIP_TRY(ctx, launch_closest_points(m->d_nodes, m->d_tris, (float)m->radius, m->centre, Q, nq, tri, d2, bary,
                                     ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  return MSK_OK;
}

// ------------------------------------------------------ rows and basis

extern "C" msk_status msk_rows_create(msk_ctx* ctx, const msk_mesh* m, const msk_rows_desc* d, msk_rows** out) {
  if (!ctx || !m || !d || !out) return MSK_ERR_INVALID_ARG;
  *out = nullptr;
  const int64_t n = d->n_rows;
  if (n < 1 || n >= INT32_MAX) return fail(ctx, MSK_ERR_INVALID_ARG, "n_rows must be >= 1");
  if (!d->w) return fail(ctx, MSK_ERR_INVALID_ARG, "row weights missing");
  for (int64_t i = 0; i < n; ++i)
    if (!(d->w[i] >= 0) || !std::isfinite(d->w[i])) return fail(ctx, MSK_ERR_INVALID_ARG, "bad row weight");
  msk_rows* r = new msk_rows();
  r->ctx = ctx;
  r->mesh = m;
  r->mode = d->mode;
  r->n = n;
  r->w.assign(d->w, d->w + n);
  std::vector<float> pos((size_t)n * 3);
  hipError_t he = hipSuccess;
  if (d->mode == MSK_ROWS_POINT) {
    if (!d->p || !d->n || !d->tri || !d->bary) {
      delete r;
      return fail(ctx, MSK_ERR_INVALID_ARG, "point rows need p, n, tri, bary");
    }
    for (int64_t i = 0; i < n; ++i) {
      if (!finite3(d->p + 3 * i) || !finite3(d->n + 3 * i) || !finite3(d->bary + 3 * i) || d->tri[i] < 0 ||
          d->tri[i] >= m->nf) {
        delete r;
        return fail(ctx, MSK_ERR_INVALID_ARG, "bad point row " + std::to_string(i));
      }
      for (int k = 0; k < 3; ++k) pos[3 * i + k] = (float)((double)d->p[3 * i + k] - m->centre[k]);
    }
    r->p_world.assign(d->p, d->p + 3 * n);
    r->n_world.assign(d->n, d->n + 3 * n);
    if ((he = upload(ctx, &r->d_p, pos.data(), pos.size())) != hipSuccess ||
        (he = upload(ctx, &r->d_n, d->n, (size_t)n * 3)) != hipSuccess ||
        (he = upload(ctx, &r->d_tri, d->tri, (size_t)n)) != hipSuccess ||
        (he = upload(ctx, &r->d_bary, d->bary, (size_t)n * 3)) != hipSuccess) {
      msk_rows_destroy(r);
      return fail(ctx, MSK_ERR_DEVICE, std::string("rows upload: ") + hipGetErrorString(he));
    }
  } else if (d->mode == MSK_ROWS_HAT_RING) {
    if (n != m->nv || !d->ring_ptr || !d->ring_tri || !d->ring_cum || !d->face_normals) {
      delete r;
      return fail(ctx, MSK_ERR_INVALID_ARG, "hat rows need one row per vertex and the one-ring arrays");
    }
    const int64_t ne = d->ring_ptr[n];
    if (d->ring_ptr[0] != 0 || ne < 0) {
      delete r;
      return fail(ctx, MSK_ERR_INVALID_ARG, "bad ring_ptr");
    }
    for (int64_t i = 0; i < n; ++i) {
      if (d->ring_ptr[i + 1] <= d->ring_ptr[i]) {
        delete r;
        return fail(ctx, MSK_ERR_INVALID_ARG, "vertex " + std::to_string(i) + " has an empty one-ring");
      }
      for (int32_t e = d->ring_ptr[i]; e < d->ring_ptr[i + 1]; ++e) {
        int32_t f = d->ring_tri[e];
        if (f < 0 || f >= m->nf ||
            (m->faces[3 * f] != i && m->faces[3 * f + 1] != i && m->faces[3 * f + 2] != i) ||
            !std::isfinite(d->ring_cum[e])) {
          delete r;
          return fail(ctx, MSK_ERR_INVALID_ARG, "bad one-ring entry of vertex " + std::to_string(i));
        }
      }
      for (int k = 0; k < 3; ++k) pos[3 * i + k] = m->vrel[3 * i + k];
    }
    for (int64_t f = 0; f < m->nf; ++f)
      if (!finite3(d->face_normals + 3 * f)) {
        delete r;
        return fail(ctx, MSK_ERR_INVALID_ARG, "bad face normal");
      }
    if ((he = upload(ctx, &r->d_ring_ptr, d->ring_ptr, (size_t)n + 1)) != hipSuccess ||
        (he = upload(ctx, &r->d_ring_tri, d->ring_tri, (size_t)ne)) != hipSuccess ||
        (he = upload(ctx, &r->d_ring_cum, d->ring_cum, (size_t)ne)) != hipSuccess ||
        (he = upload(ctx, &r->d_fn, d->face_normals, (size_t)m->nf * 3)) != hipSuccess) {
      msk_rows_destroy(r);
      return fail(ctx, MSK_ERR_DEVICE, std::string("rows upload: ") + hipGetErrorString(he));
    }
  } else {
    delete r;
    return fail(ctx, MSK_ERR_INVALID_ARG, "unknown row mode");
  }
  if ((he = upload(ctx, &r->d_w, d->w, (size_t)n)) != hipSuccess) {
    msk_rows_destroy(r);
    return fail(ctx, MSK_ERR_DEVICE, std::string("rows upload: ") + hipGetErrorString(he));
  }
  r->order = morton_order(pos, n);
  *out = r;
  return MSK_OK;
}

extern "C" void msk_rows_destroy(msk_rows* r) {
  if (!r) return;
  dfree(r->d_w);
  dfree(r->d_p);
  dfree(r->d_n);
  dfree(r->d_tri);
  dfree(r->d_bary);
  dfree(r->d_ring_ptr);
  dfree(r->d_ring_tri);
  dfree(r->d_ring_cum);
  dfree(r->d_fn);
  delete r;
}

extern "C" msk_status msk_basis_create(msk_ctx* ctx, const int32_t* rowptr, const int32_t* col, const float* val,
                                       int64_t n_verts, int64_t K, msk_basis** out) {
  if (!ctx || !out) return MSK_ERR_INVALID_ARG;
  *out = nullptr;
  if (!rowptr || n_verts < 1 || K < 1 || K >= INT32_MAX) return fail(ctx, MSK_ERR_INVALID_ARG, "bad basis sizes");
  if (rowptr[0] != 0) return fail(ctx, MSK_ERR_INVALID_ARG, "rowptr[0] must be 0");
  const int64_t nnz = rowptr[n_verts];
  if (nnz > 0 && (!col || !val)) return fail(ctx, MSK_ERR_INVALID_ARG, "basis col/val missing");
  for (int64_t v = 0; v < n_verts; ++v) {
    int32_t a = rowptr[v], b = rowptr[v + 1];
    if (b < a) return fail(ctx, MSK_ERR_INVALID_ARG, "bad basis row " + std::to_string(v));
    for (int32_t e = a; e < b; ++e) {
      if (col[e] < 0 || col[e] >= K || (e > a && col[e] <= col[e - 1]) || !std::isfinite(val[e]))
        return fail(ctx, MSK_ERR_INVALID_ARG, "basis row " + std::to_string(v) + " columns must increase in [0,K)");
    }
  }
  int32_t max_nnz = 0;
  for (int64_t v = 0; v < n_verts; ++v) max_nnz = std::max(max_nnz, rowptr[v + 1] - rowptr[v]);
  msk_basis* b = new msk_basis();
  b->ctx = ctx;
  b->max_row_nnz = max_nnz;
  b->nv = n_verts;
  b->K = K;
  hipError_t he;
  if ((he = upload(ctx, &b->d_rowptr, rowptr, (size_t)n_verts + 1)) != hipSuccess ||
      (he = upload(ctx, &b->d_col, col, (size_t)nnz)) != hipSuccess ||
      (he = upload(ctx, &b->d_val, val, (size_t)nnz)) != hipSuccess) {
    msk_basis_destroy(b);
    return fail(ctx, MSK_ERR_DEVICE, std::string("basis upload: ") + hipGetErrorString(he));
  }
  *out = b;
  return MSK_OK;
}

extern "C" void msk_basis_destroy(msk_basis* b) {
  if (!b) return;
  dfree(b->d_rowptr);
  dfree(b->d_col);
  dfree(b->d_val);
  dfree(b->d_kpts);
  dfree(b->d_knrm);
  dfree(b->d_cell_start);
  dfree(b->d_cell_pts);
  delete b;
}

extern "C" msk_status msk_basis_create_knn(msk_ctx* ctx, const msk_mesh* m, const float* points,
                                           const float* normals, int64_t n_points, int32_t k, double sigma,
                                           double tau_n, msk_basis** out) {
  if (!ctx || !out) return MSK_ERR_INVALID_ARG;
  *out = nullptr;
  if (!m || !points || !normals) return fail(ctx, MSK_ERR_INVALID_ARG, "null mesh or point arrays");
  if (k < 1 || k > kMaxKnn) return fail(ctx, MSK_ERR_INVALID_ARG, "k must be in 1..16");
  if (n_points < k || n_points >= INT32_MAX) return fail(ctx, MSK_ERR_INVALID_ARG, "need k <= n_points < 2^31");
  if (!(sigma > 0) || !(tau_n > 0) || !std::isfinite(sigma) || !std::isfinite(tau_n))
    return fail(ctx, MSK_ERR_INVALID_ARG, "sigma and tau_n must be positive");
  // scene-frame positions and unit normals
  std::vector<float4> P((size_t)n_points), Nn((size_t)n_points);
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t j = 0; j < n_points; ++j) {
    double q[3], nn[3], l2 = 0;
    for (int a = 0; a < 3; ++a) {
      if (!std::isfinite(points[3 * j + a]) || !std::isfinite(normals[3 * j + a]))
        return fail(ctx, MSK_ERR_INVALID_ARG, "non-finite point or normal");
      q[a] = (double)points[3 * j + a] - m->centre[a];
      nn[a] = normals[3 * j + a];
      l2 += nn[a] * nn[a];
    }
    if (!(l2 > 0)) return fail(ctx, MSK_ERR_INVALID_ARG, "zero normal");
    const double il = 1.0 / std::sqrt(l2);
    P[j] = make_float4((float)q[0], (float)q[1], (float)q[2], 0.0f);
    Nn[j] = make_float4((float)(nn[0] * il), (float)(nn[1] * il), (float)(nn[2] * il), 0.0f);
    for (int a = 0; a < 3; ++a) {
      lo[a] = std::min(lo[a], (double)((&P[j].x)[a]));
      hi[a] = std::max(hi[a], (double)((&P[j].x)[a]));
    }
  }
  // uniform grid: cells of about two sample spacings (spacing ~ sqrt(area / N)),
  // at most 2^24 cells
  double cell = 2.0 * std::sqrt(std::max(m->area, 1e-30) / (double)n_points);
  const double ext = std::max(hi[0] - lo[0], std::max(hi[1] - lo[1], hi[2] - lo[2]));
  cell = std::max(cell, ext * 1e-6 + 1e-30);
  int64_t dim[3];
  while (true) {
    for (int a = 0; a < 3; ++a) dim[a] = std::max<int64_t>(1, (int64_t)std::floor((hi[a] - lo[a]) / cell) + 1);
    if (dim[0] * dim[1] * dim[2] <= ((int64_t)1 << 24)) break;
    cell *= 1.25;
  }
  const int64_t nc = dim[0] * dim[1] * dim[2];
  std::vector<int32_t> cs((size_t)nc + 1, 0), cp((size_t)n_points), cid((size_t)n_points);
  for (int64_t j = 0; j < n_points; ++j) {
    int64_t c[3];
    for (int a = 0; a < 3; ++a)
      c[a] = std::min<int64_t>(dim[a] - 1,
                               std::max<int64_t>(0, (int64_t)std::floor(((&P[j].x)[a] - (float)lo[a]) / (float)cell)));
    cid[j] = (int32_t)((c[2] * dim[1] + c[1]) * dim[0] + c[0]);
    ++cs[cid[j] + 1];
  }
  for (int64_t c = 0; c < nc; ++c) cs[c + 1] += cs[c];
  std::vector<int32_t> fill(cs.begin(), cs.end() - 1);
  for (int64_t j = 0; j < n_points; ++j) cp[fill[cid[j]]++] = (int32_t)j;
  msk_basis* b = new msk_basis();
  b->ctx = ctx;
  b->nv = m->nv;
  b->K = n_points;
  b->max_row_nnz = k;
  b->knn_mesh = m;
  hipError_t he;
  if ((he = upload(ctx, &b->d_kpts, P.data(), P.size())) != hipSuccess ||
      (he = upload(ctx, &b->d_knrm, Nn.data(), Nn.size())) != hipSuccess ||
      (he = upload(ctx, &b->d_cell_start, cs.data(), cs.size())) != hipSuccess ||
      (he = upload(ctx, &b->d_cell_pts, cp.data(), cp.size())) != hipSuccess) {
    msk_basis_destroy(b);
    return fail(ctx, he == hipErrorOutOfMemory ? MSK_ERR_OOM : MSK_ERR_DEVICE,
                std::string("point basis upload: ") + hipGetErrorString(he));
  }
  KnnDev& G = b->kd;
  G.pts = b->d_kpts;
  G.nrm = b->d_knrm;
  G.cell_start = b->d_cell_start;
  G.cell_pts = b->d_cell_pts;
  for (int a = 0; a < 3; ++a) {
    G.lo[a] = (float)lo[a];
    G.dim[a] = (int32_t)dim[a];
  }
  G.cell = (float)cell;
  G.k = k;
  G.inv2s2 = 1.0 / (2.0 * sigma * sigma);
  G.inv_tau = 1.0 / tau_n;
  *out = b;
  return MSK_OK;
}

extern "C" msk_status msk_basis_eval_knn(msk_ctx* ctx, const msk_basis* b, const float* Q, const float* Nq,
                                         int64_t n, int32_t* idx, float* w) {
  if (!ctx || !b) return MSK_ERR_INVALID_ARG;
  if (!b->knn_mesh) return fail(ctx, MSK_ERR_INVALID_ARG, "not a point basis");
  if (n < 0 || (n > 0 && (!Q || !Nq || !idx || !w))) return fail(ctx, MSK_ERR_INVALID_ARG, "bad query arrays");
  if (n == 0) return MSK_OK;
  HIP_TRY(ctx, launch_knn_eval(b->kd, b->knn_mesh->centre, Q, Nq, n, idx, w, ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  return MSK_OK;
}

// ------------------------------------------------------------ estimate

extern "C" void msk_dtn_opts_default(msk_dtn_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->seed = 0;
  o->max_steps = 0;
  o->walk_offset = 0;
  o->kappa = std::ldexp(1.0, -20);
  o->delta_rel = std::ldexp(1.0, -21);
  o->form = MSK_FORM_PERSISTENT;
  o->block = 256;
  o->blocks_per_cu = 8;
  o->chunk = 64;
  o->regen_min = 16;
  o->record_log = 0;
  o->se_target = 0;
  o->walks_max = 65536;
  o->collect_stats = 0;
  o->mesh_id = 0;
  o->accum = 0;
}

extern "C" double msk_eps_floor(double radius, const msk_dtn_opts* opts) {
  msk_dtn_opts o;
  msk_dtn_opts_default(&o);
  if (opts) o = *opts;
  if (!(radius > 0.0) || !std::isfinite(radius) || !(o.kappa >= 0.0 && o.kappa < 1.0)) return NAN;
  // a walk at distance d steps by d (1 - kappa) - delta_rel R, which stays
  // positive only for d > delta_rel R / (1 - kappa); below 2^-18 R the FP32
  // distance of the scene frame no longer resolves the shell
  return std::max(o.delta_rel * radius / (1.0 - o.kappa), std::ldexp(radius, -18));
}

namespace {

void dtn_free(msk_dtn* d) {
  dfree(d->d_S);
  dfree(d->d_se);
  dfree(d->d_acc1);
  dfree(d->d_acc2);
  dfree(d->d_q);
  dfree(d->d_esc);
  dfree(d->d_cap);
  dfree(d->d_disc);
  dfree(d->d_walks);
  dfree(d->d_log_status);
  dfree(d->d_log_tri);
  dfree(d->d_log_bary);
  dfree(d->d_log_q);
  dfree(d->d_nonfinite);
}

struct Prepared {
  MeshDev md;
};

msk_status check_problem(msk_ctx* ctx, const msk_mesh* m, const msk_rows* r, const msk_basis* b, int64_t walks,
                         double eps, double h, int32_t side, const msk_dtn_opts* o, bool row_sums = true) {
  if (!m || !r || !b) return fail(ctx, MSK_ERR_INVALID_ARG, "null mesh / rows / basis");
  if (r->mesh != m) return fail(ctx, MSK_ERR_INVALID_ARG, "rows were created for another mesh");
  if (b->nv != m->nv) return fail(ctx, MSK_ERR_INVALID_ARG, "basis vertex count differs from the mesh's");
  if (b->knn_mesh && b->knn_mesh != m) return fail(ctx, MSK_ERR_INVALID_ARG, "point basis built for another mesh");
  if (b->knn_mesh && r->mode != MSK_ROWS_POINT) return fail(ctx, MSK_ERR_INVALID_ARG, "the point basis takes point rows");
  if (row_sums && b->max_row_nnz > kMaxTableNnz)
    return fail(ctx, MSK_ERR_INVALID_ARG, "the walk estimators take at most 32 basis entries per vertex");
  if (walks < 2 || walks > INT32_MAX) return fail(ctx, MSK_ERR_INVALID_ARG, "walks must be in 2..2^31-1");
  if (!(eps > 0) || !(h > eps) || !std::isfinite(h)) return fail(ctx, MSK_ERR_INVALID_ARG, "need 0 < eps < inset_h");
  if (o && !(o->kappa >= 0.0 && o->kappa < 0.5 && o->delta_rel >= 0.0 && o->delta_rel < 0.25))
    return fail(ctx, MSK_ERR_INVALID_ARG, "need 0 <= kappa < 1/2 and 0 <= delta_rel < 1/4");
  const double floor_eps = msk_eps_floor(m->radius, o);
  if (!(eps > floor_eps))
    return fail(ctx, MSK_ERR_INVALID_ARG,
                "eps must exceed " + std::to_string(floor_eps) + " for this mesh (msk_eps_floor: the step guard "
                "delta_rel R / (1 - kappa) and the FP32 distance resolution 2^-18 R)");
  if (side != MSK_INTERIOR && side != MSK_EXTERIOR) return fail(ctx, MSK_ERR_INVALID_ARG, "side must be 0 or 1");
  return MSK_OK;
}

msk_status alloc_dtn(msk_ctx* ctx, const msk_rows* r, const msk_basis* b, int64_t W, bool log, msk_dtn** out) {
  msk_dtn* d = new msk_dtn();
  d->ctx = ctx;
  d->rows = r;
  d->n = r->n;
  d->K = b->K;
  d->W = W;
  d->mode = r->mode;
  const size_t nk = (size_t)d->n * (size_t)d->K;
  hipError_t he;
  if ((he = dalloc(&d->d_S, nk)) != hipSuccess || (he = dalloc(&d->d_se, nk)) != hipSuccess ||
      (he = dalloc(&d->d_acc1, nk)) != hipSuccess || (he = dalloc(&d->d_acc2, nk)) != hipSuccess ||
      (he = dalloc(&d->d_q, d->n)) != hipSuccess || (he = dalloc(&d->d_esc, d->n)) != hipSuccess ||
      (he = dalloc(&d->d_cap, d->n)) != hipSuccess || (he = dalloc(&d->d_disc, d->n)) != hipSuccess ||
      (he = dalloc(&d->d_walks, d->n)) != hipSuccess || (he = dalloc(&d->d_nonfinite, 1)) != hipSuccess) {
    dtn_free(d);
    delete d;
    return fail(ctx, MSK_ERR_OOM, std::string("estimate buffers: ") + hipGetErrorString(he));
  }
  if (log) {
    const size_t nl = (size_t)d->n * (size_t)W;
    if ((he = dalloc(&d->d_log_status, nl)) != hipSuccess || (he = dalloc(&d->d_log_tri, nl)) != hipSuccess ||
        (he = dalloc(&d->d_log_bary, 2 * nl)) != hipSuccess || (he = dalloc(&d->d_log_q, nl)) != hipSuccess) {
      dtn_free(d);
      delete d;
      return fail(ctx, MSK_ERR_OOM, std::string("walk log: ") + hipGetErrorString(he));
    }
  }
  *out = d;
  return MSK_OK;
}

MeshDev make_meshdev(const msk_mesh* m, const msk_rows* r, const msk_basis* b, msk_dtn* d, double eps, double h,
                     int32_t side, const msk_dtn_opts& o, int32_t mesh_id) {
  MeshDev M;
  std::memset(&M, 0, sizeof(M));
  M.nodes = m->d_nodes;
  M.tris = m->d_tris;
  M.slot_of_tri = m->d_slot;
  M.faces = m->d_faces;
  M.n_tris = m->nf;
  M.n_top = m->top_nodes;
  M.mode = r->mode;
  M.radius = (float)m->radius;
  M.radius_d = m->radius;
  M.eps2 = (float)(eps * eps);
  M.inset = (float)h;
  M.inset_d = h;
  M.kappa = (float)o.kappa;
  M.delta = (float)(o.delta_rel * m->radius);
  M.slack = (float)std::ldexp(m->radius, -18);
  M.side = side;
  M.mesh_id = mesh_id;
  M.walks_per_row = (int32_t)d->W;
  M.max_steps = o.max_steps > 0 ? o.max_steps : (side == MSK_EXTERIOR ? 8192 : 1024);
  M.p = r->d_p;
  M.n = r->d_n;
  M.tri = r->d_tri;
  M.bary = r->d_bary;
  M.ring_ptr = r->d_ring_ptr;
  M.ring_tri = r->d_ring_tri;
  M.ring_cum = r->d_ring_cum;
  M.face_normals = r->d_fn;
  M.discarded = d->d_disc;
  M.b_rowptr = b->d_rowptr;
  M.b_col = b->d_col;
  M.b_val = b->d_val;
  M.K = b->K;
  if (b->knn_mesh) M.knn = b->kd;
  M.acc1 = d->d_acc1;
  M.acc2 = d->d_acc2;
  M.row_queries = d->d_q;
  M.row_escaped = d->d_esc;
  M.row_capped = d->d_cap;
  M.log_status = d->d_log_status;
  M.log_tri = d->d_log_tri;
  M.log_bary = d->d_log_bary;
  M.log_queries = d->d_log_q;
  return M;
}

// Queue bounds: 8 contiguous ranges of slots with about equal walk counts.
QueueInit make_queues(int64_t n_slots, int64_t W) {
  QueueInit q;
  for (int i = 0; i < 8; ++i) {
    int64_t s0 = n_slots * i / 8, s1 = n_slots * (i + 1) / 8;
    q.begin[i] = (unsigned long long)(s0 * W);
    q.end[i] = (unsigned long long)(s1 * W);
  }
  return q;
}

}  // namespace

struct LaunchBuffers {
  MeshDev* d_meshes = nullptr;
  RowSlot* d_slots = nullptr;
  unsigned long long* d_qnext = nullptr;
  unsigned long long* d_qend = nullptr;
  unsigned long long* d_stats = nullptr;
  ~LaunchBuffers() {
    dfree(d_stats);
    dfree(d_meshes);
    dfree(d_slots);
    dfree(d_qnext);
    dfree(d_qend);
  }
};

// Runs the walk kernel over `slots` (walks [offset, offset + W) of each
// slot's row) and returns its duration in milliseconds.
static msk_status run_walks(msk_ctx* ctx, const std::vector<MeshDev>& meshes, const std::vector<RowSlot>& slots,
                            int64_t W, int64_t offset, const msk_dtn_opts& o, int use_lds_top, int n_top,
                            double* ms, int64_t stats_out[3]) {
  *ms = 0;
  if (slots.empty()) return MSK_OK;
  LaunchBuffers lb;
  HIP_TRY(ctx, upload(ctx, &lb.d_meshes, meshes.data(), meshes.size()));
  HIP_TRY(ctx, upload(ctx, &lb.d_slots, slots.data(), slots.size()));
  HIP_TRY(ctx, dalloc(&lb.d_qnext, 8));
  HIP_TRY(ctx, dalloc(&lb.d_qend, 8));
  WalkLaunch L;
  std::memset(&L, 0, sizeof(L));
  L.meshes = lb.d_meshes;
  L.slots = lb.d_slots;
  L.n_slots = (int64_t)slots.size();
  L.walks_per_slot = W;
  L.walk_offset = offset;
  L.seed_lo = (uint32_t)o.seed;
  L.seed_hi = (uint32_t)(o.seed >> 32);
  L.queue_next = lb.d_qnext;
  L.queue_end = lb.d_qend;
  L.chunk = std::max(1, o.chunk);
  L.regen_min = std::min(64, std::max(1, o.regen_min));
  L.use_lds_top = use_lds_top;
  L.n_top = n_top;
  L.accum = o.accum;
  for (const MeshDev& md : meshes) L.knn |= md.knn.k > 0 ? 1 : 0;
  if (o.collect_stats) {
    HIP_TRY(ctx, dalloc(&lb.d_stats, 3));
    HIP_TRY(ctx, launch_fill_u64(lb.d_stats, 3, 0, ctx->stream));
    L.stats = lb.d_stats;
  }
  if ((unsigned long long)L.n_slots * (unsigned long long)W >= (1ull << 62))
    return fail(ctx, MSK_ERR_INVALID_ARG, "too many walks");
  QueueInit q = make_queues(L.n_slots, W);
  HIP_TRY(ctx, launch_init_queues(lb.d_qnext, lb.d_qend, q, ctx->stream));
  hipEvent_t e0, e1;
  HIP_TRY(ctx, hipEventCreate(&e0));
  HIP_TRY(ctx, hipEventCreate(&e1));
  HIP_TRY(ctx, hipEventRecord(e0, ctx->stream));
  hipError_t le;
  if (o.form == MSK_FORM_PLAIN) {
    le = launch_walk_plain(L, ctx->stream);
  } else {
    const int grid = std::max(1, ctx->n_cu * std::max(1, o.blocks_per_cu));
    le = launch_walk_persistent(L, grid, ctx->stream);
  }
  HIP_TRY(ctx, le);
  HIP_TRY(ctx, hipEventRecord(e1, ctx->stream));
  HIP_TRY(ctx, hipEventSynchronize(e1));
  float f = 0;
  HIP_TRY(ctx, hipEventElapsedTime(&f, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *ms = f;
  if (o.collect_stats) {
    unsigned long long st[3];
    HIP_TRY(ctx, hipMemcpy(st, lb.d_stats, sizeof(st), hipMemcpyDeviceToHost));
    stats_out[0] += (int64_t)st[0];
    stats_out[1] += (int64_t)st[1];
    stats_out[2] += (int64_t)st[2];
  }
  return MSK_OK;
}

static msk_status collect_info(msk_ctx* ctx, msk_dtn* d) {
  std::vector<unsigned long long> q(d->n), esc(d->n), cap(d->n);
  std::vector<int32_t> disc(d->n);
  std::vector<int64_t> walks(d->n);
  HIP_TRY(ctx, hipMemcpy(q.data(), d->d_q, d->n * 8, hipMemcpyDeviceToHost));
  HIP_TRY(ctx, hipMemcpy(esc.data(), d->d_esc, d->n * 8, hipMemcpyDeviceToHost));
  HIP_TRY(ctx, hipMemcpy(cap.data(), d->d_cap, d->n * 8, hipMemcpyDeviceToHost));
  HIP_TRY(ctx, hipMemcpy(disc.data(), d->d_disc, d->n * 4, hipMemcpyDeviceToHost));
  HIP_TRY(ctx, hipMemcpy(walks.data(), d->d_walks, d->n * 8, hipMemcpyDeviceToHost));
  unsigned long long nonfinite = 0;
  HIP_TRY(ctx, hipMemcpy(&nonfinite, d->d_nonfinite, 8, hipMemcpyDeviceToHost));
  d->info.nonfinite_entries = (int64_t)nonfinite;
  d->info.n_rows = d->n;
  d->info.K = d->K;
  d->info.walks_total = d->info.queries_total = d->info.escaped_total = d->info.capped_total = 0;
  d->info.discarded_rows = 0;
  for (int64_t i = 0; i < d->n; ++i) {
    d->info.queries_total += (int64_t)q[i];
    d->info.escaped_total += (int64_t)esc[i];
    d->info.capped_total += (int64_t)cap[i];
    d->info.discarded_rows += disc[i] ? 1 : 0;
    d->info.walks_total += disc[i] ? 0 : walks[i];
  }
  return MSK_OK;
}

// The same summary from totals summed on the device (launch_row_totals).
static void info_from_totals(msk_dtn* d, const unsigned long long t[6]) {
  d->info.n_rows = d->n;
  d->info.K = d->K;
  d->info.queries_total = (int64_t)t[0];
  d->info.escaped_total = (int64_t)t[1];
  d->info.capped_total = (int64_t)t[2];
  d->info.discarded_rows = (int64_t)t[3];
  d->info.walks_total = (int64_t)t[4];
  d->info.nonfinite_entries = (int64_t)t[5];
}

extern "C" msk_status msk_estimate_dtn(msk_ctx* ctx, const msk_mesh* m, const msk_rows* r, const msk_basis* b,
                                       int64_t walks, double eps, double inset_h, int32_t side,
                                       const msk_dtn_opts* opts, msk_dtn** out) {
  if (!ctx || !out) return MSK_ERR_INVALID_ARG;
  *out = nullptr;
  msk_dtn_opts o;
  msk_dtn_opts_default(&o);
  if (opts) o = *opts;
  msk_status st = check_problem(ctx, m, r, b, walks, eps, inset_h, side, &o);
  if (st != MSK_OK) return st;
  if (o.form != MSK_FORM_PLAIN && o.form != MSK_FORM_PERSISTENT) return fail(ctx, MSK_ERR_INVALID_ARG, "bad form");
  if (o.accum < 0 || o.accum > 2)
    return fail(ctx, MSK_ERR_INVALID_ARG, "accum must be 0 (FP64), 1 (FP32) or 2 (compensated FP32)");
  if (o.jump_only != 0 && (o.jump_only != 1 || side != MSK_EXTERIOR || r->mode != MSK_ROWS_POINT))
    return fail(ctx, MSK_ERR_INVALID_ARG, "jump_only takes exterior estimates with point rows");
  if (o.collect_stats && b && b->knn_mesh)
    return fail(ctx, MSK_ERR_INVALID_ARG, "traversal statistics are not collected with the point basis");
  if (o.walk_offset < 0 || o.walk_offset + walks > ((int64_t)1 << 32) ||
      (o.se_target > 0 && o.walk_offset + o.walks_max > ((int64_t)1 << 32)))
    return fail(ctx, MSK_ERR_INVALID_ARG, "walk indices must fit in 32 bits");
  const bool adaptive = o.se_target > 0;
  if (adaptive && (o.walks_max < walks)) return fail(ctx, MSK_ERR_INVALID_ARG, "walks_max < walks");
  if (adaptive && o.record_log) return fail(ctx, MSK_ERR_INVALID_ARG, "walk log needs a fixed walk count");
  msk_dtn* d = nullptr;
  st = alloc_dtn(ctx, r, b, walks, o.record_log != 0, &d);
  if (st != MSK_OK) return st;
  d->inset = inset_h;
  hipEvent_t t0, t1;
  auto cleanup = [&](msk_status s) {
    dtn_free(d);
    delete d;
    return s;
  };
#define TRY_D(expr)                    \
  do {                                 \
    msk_status s_ = (expr);            \
    if (s_ != MSK_OK) return cleanup(s_); \
  } while (0)
#define HIP_D(expr)                                                                                   \
  do {                                                                                                \
    hipError_t e_ = (expr);                                                                           \
    if (e_ != hipSuccess)                                                                             \
      return cleanup(fail(ctx, MSK_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)));   \
  } while (0)
  HIP_D(hipEventCreate(&t0));
  HIP_D(hipEventCreate(&t1));
  HIP_D(hipEventRecord(t0, ctx->stream));
  const size_t nk = (size_t)d->n * (size_t)d->K;
  HIP_D(launch_fill_u64(d->d_acc1, (int64_t)nk, 0, ctx->stream));
  HIP_D(launch_fill_u64(d->d_acc2, (int64_t)nk, 0, ctx->stream));
  HIP_D(launch_fill_u64(d->d_q, d->n, 0, ctx->stream));
  HIP_D(launch_fill_u64(d->d_esc, d->n, 0, ctx->stream));
  HIP_D(launch_fill_u64(d->d_cap, d->n, 0, ctx->stream));
  HIP_D(launch_fill_u64(d->d_walks, d->n, (unsigned long long)walks, ctx->stream));
  if (d->d_log_status) {  // walks of discarded rows keep status -1
    HIP_D(launch_fill_u32(d->d_log_status, d->n * walks, 0xFFFFFFFFu, ctx->stream));
    HIP_D(launch_fill_u32(d->d_log_tri, d->n * walks, 0xFFFFFFFFu, ctx->stream));
    HIP_D(launch_fill_u32(d->d_log_bary, 2 * d->n * walks, 0u, ctx->stream));
    HIP_D(launch_fill_u32(d->d_log_q, d->n * walks, 0u, ctx->stream));
  }
  // discarded flags: zero, then the inset test for point rows
  HIP_D(launch_fill_u32(d->d_disc, d->n, 0u, ctx->stream));
  if (o.mesh_id < 0 || o.mesh_id > 0xFFFFFF) return cleanup(fail(ctx, MSK_ERR_INVALID_ARG, "mesh_id must be < 2^24"));
  MeshDev M = make_meshdev(m, r, b, d, eps, inset_h, side, o, o.mesh_id);
  if (r->mode == MSK_ROWS_POINT) HIP_D(launch_discard(M, d->n, d->d_disc, ctx->stream));
  HIP_D(hipStreamSynchronize(ctx->stream));
  std::vector<MeshDev> meshes{M};
  std::vector<RowSlot> slots(r->order.size());
  for (size_t i = 0; i < slots.size(); ++i) slots[i] = RowSlot{0, r->order[i], 0u};
  const int use_lds = (o.form == MSK_FORM_PERSISTENT && m->top_nodes > 0) ? 1 : 0;
  double ms = 0;
  d->info.walk_launches = 0;
  d->info.walk_kernel_ms = 0;
  int64_t stats[3] = {0, 0, 0};
  TRY_D(run_walks(ctx, meshes, slots, walks, o.walk_offset, o, use_lds, m->top_nodes, &ms, stats));
  d->info.walk_kernel_ms += ms;
  d->info.walk_launches += 1;
  if (adaptive) {
    // Rounds: every row whose escape-fraction standard error exceeds the
    // target gets a multiple of `walks` more walks, its predicted deficit
    // q(1-q)/target^2 - W_i rounded up, at least one batch and at most
    // doubling its count; a row's slots continue its walk indices, so all its
    // new walks run in the round's single launch.
    std::vector<int64_t> wdone((size_t)d->n, walks);
    std::vector<unsigned long long> esc((size_t)d->n);
    std::vector<int32_t> disc((size_t)d->n);
    HIP_D(hipMemcpy(disc.data(), d->d_disc, d->n * 4, hipMemcpyDeviceToHost));
    const double t2 = o.se_target * o.se_target;
    while (true) {
      HIP_D(hipMemcpy(esc.data(), d->d_esc, d->n * 8, hipMemcpyDeviceToHost));
      std::vector<RowSlot> act;
      std::vector<int64_t> add((size_t)d->n, 0);
      for (int32_t i : r->order) {
        if (disc[i]) continue;
        const double Wi = (double)wdone[i];
        const double q = (double)esc[i] / Wi;
        const double v = std::max(q * (1 - q), 1.0 / Wi);
        if (std::sqrt(v / Wi) <= o.se_target) continue;
        const int64_t room = o.walks_max - wdone[i];
        if (room < walks) continue;
        const double deficit = v / t2 - Wi;
        int64_t batches = (int64_t)std::ceil(std::max(deficit, 1.0) / (double)walks);
        batches = std::max<int64_t>(1, std::min<int64_t>(batches, std::min(wdone[i], room) / walks));
        for (int64_t j = 0; j < batches; ++j) act.push_back(RowSlot{0, i, (uint32_t)(wdone[i] + j * walks)});
        add[i] = batches * walks;
      }
      if (act.empty()) break;
      TRY_D(run_walks(ctx, meshes, act, walks, o.walk_offset, o, use_lds, m->top_nodes, &ms, stats));
      d->info.walk_kernel_ms += ms;
      d->info.walk_launches += 1;
      for (int32_t i : r->order) wdone[i] += add[i];
    }
    HIP_D(hipMemcpy(d->d_walks, wdone.data(), d->n * 8, hipMemcpyHostToDevice));
  }
  HIP_D(launch_finalize(M, d->n, d->d_walks, r->d_w, d->d_S, d->d_se, ctx->stream, o.jump_only));
  HIP_D(launch_fill_u64(d->d_nonfinite, 1, 0, ctx->stream));
  HIP_D(launch_count_nonfinite(d->d_S, (int64_t)nk, d->d_nonfinite, ctx->stream));
  HIP_D(launch_count_nonfinite(d->d_se, (int64_t)nk, d->d_nonfinite, ctx->stream));
  HIP_D(hipEventRecord(t1, ctx->stream));
  HIP_D(hipEventSynchronize(t1));
  float tot = 0;
  HIP_D(hipEventElapsedTime(&tot, t0, t1));
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  d->info.total_ms = tot;
  TRY_D(collect_info(ctx, d));
  d->info.nodes_visited = stats[0];
  d->info.tris_tested = stats[1];
  d->info.valu_flops = stats[2];
#undef TRY_D
#undef HIP_D
  *out = d;
  if (d->info.nonfinite_entries > 0) return fail(ctx, MSK_ERR_NUMERIC, "non-finite entries in S or se");
  return MSK_OK;
}

// ------------------------------------------- estimate without allocation

extern "C" msk_status msk_estimate_dtn_noalloc(msk_ctx* ctx, const msk_mesh* m, const msk_rows* r,
                                               const msk_basis* b, int64_t walks, double eps, double inset_h,
                                               int32_t side, const msk_dtn_opts* opts, double* S, double* se,
                                               msk_dtn_info* info) {
  if (!ctx) return MSK_ERR_INVALID_ARG;
  msk_dtn_opts o;
  msk_dtn_opts_default(&o);
  if (opts) o = *opts;
  msk_status st = check_problem(ctx, m, r, b, walks, eps, inset_h, side, &o);
  if (st != MSK_OK) return st;
  if (!S || !se) return fail(ctx, MSK_ERR_INVALID_ARG, "S and se (device, n_rows x K doubles) must be given");
  if (o.form != MSK_FORM_PLAIN && o.form != MSK_FORM_PERSISTENT) return fail(ctx, MSK_ERR_INVALID_ARG, "bad form");
  if (o.accum < 0 || o.accum > 2)
    return fail(ctx, MSK_ERR_INVALID_ARG, "accum must be 0 (FP64), 1 (FP32) or 2 (compensated FP32)");
  if (o.jump_only != 0 && (o.jump_only != 1 || side != MSK_EXTERIOR || r->mode != MSK_ROWS_POINT))
    return fail(ctx, MSK_ERR_INVALID_ARG, "jump_only takes exterior estimates with point rows");
  if (o.se_target > 0 || o.record_log || o.collect_stats)
    return fail(ctx, MSK_ERR_INVALID_ARG, "the allocation-free estimate takes a fixed walk count, no log and no "
                                          "statistics");
  if (o.walk_offset < 0 || o.walk_offset + walks > ((int64_t)1 << 32))
    return fail(ctx, MSK_ERR_INVALID_ARG, "walk indices must fit in 32 bits");
  if (o.mesh_id < 0 || o.mesh_id > 0xFFFFFF) return fail(ctx, MSK_ERR_INVALID_ARG, "mesh_id must be < 2^24");
  const int64_t n = r->n;
  if ((unsigned long long)n * (unsigned long long)walks >= (1ull << 62))
    return fail(ctx, MSK_ERR_INVALID_ARG, "too many walks");
  // workspace layout, each part 256-byte aligned: the accumulators, the row
  // counters, the walk-launch tables and the queue counters
  const size_t nk = (size_t)n * (size_t)b->K;
  auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t off_acc1 = 0, off_acc2 = off_acc1 + up(nk * 8), off_q = off_acc2 + up(nk * 8);
  const size_t off_esc = off_q + up((size_t)n * 8), off_cap = off_esc + up((size_t)n * 8);
  const size_t off_walks = off_cap + up((size_t)n * 8), off_disc = off_walks + up((size_t)n * 8);
  const size_t off_nonf = off_disc + up((size_t)n * 4), off_qn = off_nonf + 256, off_qe = off_qn + 256;
  const size_t off_mesh = off_qe + 256, off_slots = off_mesh + up(sizeof(MeshDev));
  const size_t need = off_slots + up((size_t)n * sizeof(RowSlot));
  if (need > msk::kNoallocScratchBytes)
    return fail(ctx, MSK_ERR_INVALID_ARG,
                "the allocation-free estimate needs " + std::to_string(need) + " bytes of workspace for " +
                    std::to_string(n) + " rows x " + std::to_string(b->K) + " columns; its fixed workspace holds " +
                    std::to_string(msk::kNoallocScratchBytes) + " (about 16 n K + 64 n bytes are needed)");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  hipError_t serr = hipSuccess;
  char* base = (char*)msk::noalloc_scratch(ctx->device, &serr);
  if (!base) return fail(ctx, MSK_ERR_DEVICE, std::string("workspace address: ") + hipGetErrorString(serr));
  // a stack-held result record pointing into the workspace and the caller's
  // outputs (make_meshdev reads its pointers)
  msk_dtn d;
  d.ctx = ctx;
  d.rows = r;
  d.n = n;
  d.K = b->K;
  d.W = walks;
  d.mode = r->mode;
  d.inset = inset_h;
  d.d_S = S;
  d.d_se = se;
  d.d_acc1 = (double*)(base + off_acc1);
  d.d_acc2 = (double*)(base + off_acc2);
  d.d_q = (unsigned long long*)(base + off_q);
  d.d_esc = (unsigned long long*)(base + off_esc);
  d.d_cap = (unsigned long long*)(base + off_cap);
  d.d_walks = (int64_t*)(base + off_walks);
  d.d_disc = (int32_t*)(base + off_disc);
  d.d_nonfinite = (unsigned long long*)(base + off_nonf);
  unsigned long long* d_qn = (unsigned long long*)(base + off_qn);
  unsigned long long* d_qe = (unsigned long long*)(base + off_qe);
  MeshDev* d_mesh = (MeshDev*)(base + off_mesh);
  RowSlot* d_slots = (RowSlot*)(base + off_slots);
  hipStream_t s = ctx->stream;
  // the workspace keeps the previous call's contents: clear what accumulates
  HIP_TRY(ctx, launch_fill_u64(d.d_acc1, (int64_t)nk, 0, s));
  HIP_TRY(ctx, launch_fill_u64(d.d_acc2, (int64_t)nk, 0, s));
  HIP_TRY(ctx, launch_fill_u64(d.d_q, n, 0, s));
  HIP_TRY(ctx, launch_fill_u64(d.d_esc, n, 0, s));
  HIP_TRY(ctx, launch_fill_u64(d.d_cap, n, 0, s));
  HIP_TRY(ctx, launch_fill_u64(d.d_walks, n, (unsigned long long)walks, s));
  HIP_TRY(ctx, launch_fill_u32(d.d_disc, n, 0u, s));
  HIP_TRY(ctx, launch_fill_u64(d.d_nonfinite, 1, 0, s));
  MeshDev M = make_meshdev(m, r, b, &d, eps, inset_h, side, o, o.mesh_id);
  if (r->mode == MSK_ROWS_POINT) HIP_TRY(ctx, launch_discard(M, n, d.d_disc, s));
  std::vector<RowSlot> slots(r->order.size());
  for (size_t i = 0; i < slots.size(); ++i) slots[i] = RowSlot{0, r->order[i], 0u};
  HIP_TRY(ctx, hipMemcpyAsync(d_mesh, &M, sizeof(MeshDev), hipMemcpyHostToDevice, s));
  HIP_TRY(ctx, hipMemcpyAsync(d_slots, slots.data(), sizeof(RowSlot) * slots.size(), hipMemcpyHostToDevice, s));
  WalkLaunch L;
  std::memset(&L, 0, sizeof(L));
  L.meshes = d_mesh;
  L.slots = d_slots;
  L.n_slots = (int64_t)slots.size();
  L.walks_per_slot = walks;
  L.walk_offset = o.walk_offset;
  L.seed_lo = (uint32_t)o.seed;
  L.seed_hi = (uint32_t)(o.seed >> 32);
  L.queue_next = d_qn;
  L.queue_end = d_qe;
  L.chunk = std::max(1, o.chunk);
  L.regen_min = std::min(64, std::max(1, o.regen_min));
  L.use_lds_top = (o.form == MSK_FORM_PERSISTENT && m->top_nodes > 0) ? 1 : 0;
  L.n_top = m->top_nodes;
  L.accum = o.accum;
  L.knn = b->knn_mesh ? 1 : 0;
  HIP_TRY(ctx, launch_init_queues(d_qn, d_qe, make_queues(L.n_slots, walks), s));
  if (o.form == MSK_FORM_PLAIN)
    HIP_TRY(ctx, launch_walk_plain(L, s));
  else
    HIP_TRY(ctx, launch_walk_persistent(L, std::max(1, ctx->n_cu * std::max(1, o.blocks_per_cu)), s));
  HIP_TRY(ctx, launch_finalize(M, n, d.d_walks, r->d_w, S, se, s, o.jump_only));
  HIP_TRY(ctx, launch_count_nonfinite(S, (int64_t)nk, d.d_nonfinite, s));
  HIP_TRY(ctx, launch_count_nonfinite(se, (int64_t)nk, d.d_nonfinite, s));
  // the host copies above read `slots` and `M`: they are complete once the
  // stream is
  HIP_TRY(ctx, hipStreamSynchronize(s));
  msk_status cs = collect_info(ctx, &d);
  d.d_S = d.d_se = d.d_acc1 = d.d_acc2 = nullptr;  // nothing of the record is freed
  d.d_q = d.d_esc = d.d_cap = d.d_nonfinite = nullptr;
  d.d_walks = nullptr;
  d.d_disc = nullptr;
  if (cs != MSK_OK) return cs;
  if (info) *info = d.info;
  if (d.info.nonfinite_entries > 0) return fail(ctx, MSK_ERR_NUMERIC, "non-finite entries in S or se");
  return MSK_OK;
}

struct msk_batch {
  msk_ctx* ctx = nullptr;
  int32_t n = 0;
  int64_t W = 0;
  msk_dtn_opts o{};
  std::vector<msk_dtn*> dtns;
  std::vector<MeshDev> md;
  std::vector<const msk_rows*> rows;
  LaunchBuffers lb;
  // the discard pass over every mesh's point rows in one launch
  RowRange* d_ranges = nullptr;
  int32_t n_ranges = 0;
  int64_t n_point_rows = 0;
  // per-estimate totals of the row counters, summed on the device
  RowCounters* d_counters = nullptr;
  unsigned long long* d_totals = nullptr;
  // three captured graphs replayed back to back: prepare (zeroing, discard
  // pass, queues), the one persistent walk launch, finalisation
  hipGraph_t graph[3] = {nullptr, nullptr, nullptr};
  hipGraphExec_t exec[3] = {nullptr, nullptr, nullptr};
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  msk_dtn_info total{};
  ~msk_batch() {
    for (int i = 0; i < 3; ++i) {
      if (exec[i]) (void)hipGraphExecDestroy(exec[i]);
      if (graph[i]) (void)hipGraphDestroy(graph[i]);
    }
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
    dfree(d_ranges);
    dfree(d_counters);
    dfree(d_totals);
    for (msk_dtn* d : dtns)
      if (d) {
        dtn_free(d);
        delete d;
      }
  }
};

// Stage `part` of one batch run (0 prepare, 1 walks, 2 finalise), queued on s.
static hipError_t enqueue_batch(msk_batch* B, hipStream_t s, int part) {
  hipError_t e;
  if (part == 0) {
    for (int32_t i = 0; i < B->n; ++i) {
      msk_dtn* d = B->dtns[i];
      const int64_t nk = d->n * d->K;
      if ((e = launch_fill_u64(d->d_acc1, nk, 0, s)) != hipSuccess) return e;
      if ((e = launch_fill_u64(d->d_acc2, nk, 0, s)) != hipSuccess) return e;
      if ((e = launch_fill_u64(d->d_q, d->n, 0, s)) != hipSuccess) return e;
      if ((e = launch_fill_u64(d->d_esc, d->n, 0, s)) != hipSuccess) return e;
      if ((e = launch_fill_u64(d->d_cap, d->n, 0, s)) != hipSuccess) return e;
      if ((e = launch_fill_u64(d->d_walks, d->n, (unsigned long long)B->W, s)) != hipSuccess) return e;
      if ((e = launch_fill_u32(d->d_disc, d->n, 0u, s)) != hipSuccess) return e;
    }
    if ((e = launch_discard_batch(B->lb.d_meshes, B->d_ranges, B->n_ranges, B->n_point_rows, s)) != hipSuccess)
      return e;
    int64_t n_slots = 0;
    for (msk_dtn* d : B->dtns) n_slots += d->n;
    if ((e = launch_init_queues(B->lb.d_qnext, B->lb.d_qend, make_queues(n_slots, B->W), s)) != hipSuccess)
      return e;
    if (B->o.collect_stats && (e = launch_fill_u64(B->lb.d_stats, 3, 0, s)) != hipSuccess) return e;
    return hipSuccess;
  }
  if (part == 1) {
    WalkLaunch L;
    std::memset(&L, 0, sizeof(L));
    L.meshes = B->lb.d_meshes;
    L.slots = B->lb.d_slots;
    L.walks_per_slot = B->W;
    L.walk_offset = B->o.walk_offset;
    L.seed_lo = (uint32_t)B->o.seed;
    L.seed_hi = (uint32_t)(B->o.seed >> 32);
    L.queue_next = B->lb.d_qnext;
    L.queue_end = B->lb.d_qend;
    L.chunk = std::max(1, B->o.chunk);
    L.regen_min = std::min(64, std::max(1, B->o.regen_min));
    L.accum = B->o.accum;
    for (const MeshDev& md : B->md) L.knn |= md.knn.k > 0 ? 1 : 0;
    for (msk_dtn* d : B->dtns) L.n_slots += d->n;
    if (B->o.collect_stats) L.stats = B->lb.d_stats;
    if (B->o.form == MSK_FORM_PLAIN) return launch_walk_plain(L, s);
    return launch_walk_persistent(L, std::max(1, B->ctx->n_cu * std::max(1, B->o.blocks_per_cu)), s);
  }
  for (int32_t i = 0; i < B->n; ++i) {
    msk_dtn* d = B->dtns[i];
    const int64_t nk = d->n * d->K;
    if ((e = launch_finalize(B->md[i], d->n, d->d_walks, B->rows[i]->d_w, d->d_S, d->d_se, s, B->o.jump_only)) !=
            hipSuccess ||
        (e = launch_fill_u64(d->d_nonfinite, 1, 0, s)) != hipSuccess ||
        (e = launch_count_nonfinite(d->d_S, nk, d->d_nonfinite, s)) != hipSuccess ||
        (e = launch_count_nonfinite(d->d_se, nk, d->d_nonfinite, s)) != hipSuccess)
      return e;
  }
  return launch_row_totals(B->d_counters, B->n, B->d_totals, s);
}

extern "C" msk_status msk_batch_create(msk_ctx* ctx, int32_t n_meshes, const msk_mesh* const* meshes,
                                       const msk_rows* const* rows, const msk_basis* const* bases, const double* eps,
                                       const double* inset_h, int64_t walks, int32_t side, const msk_dtn_opts* opts,
                                       msk_batch** out) {
  if (!ctx || !out) return MSK_ERR_INVALID_ARG;
  *out = nullptr;
  if (n_meshes < 1 || n_meshes > 0xFFFFFF || !meshes || !rows || !bases || !eps || !inset_h)
    return fail(ctx, MSK_ERR_INVALID_ARG, "bad batch arrays");
  msk_dtn_opts o;
  msk_dtn_opts_default(&o);
  if (opts) o = *opts;
  if (o.se_target > 0 || o.record_log) return fail(ctx, MSK_ERR_INVALID_ARG, "batches take a fixed walk count, no log");
  if (o.walk_offset < 0 || o.walk_offset + walks > ((int64_t)1 << 32) ||
      (o.se_target > 0 && o.walk_offset + o.walks_max > ((int64_t)1 << 32)))
    return fail(ctx, MSK_ERR_INVALID_ARG, "walk indices must fit in 32 bits");
  if (o.accum < 0 || o.accum > 2)
    return fail(ctx, MSK_ERR_INVALID_ARG, "accum must be 0 (FP64), 1 (FP32) or 2 (compensated FP32)");
  for (int32_t i = 0; i < n_meshes; ++i) {
    if (o.collect_stats && bases[i] && bases[i]->knn_mesh)
      return fail(ctx, MSK_ERR_INVALID_ARG, "traversal statistics are not collected with the point basis");
    if (o.jump_only != 0 && (o.jump_only != 1 || side != MSK_EXTERIOR || !rows[i] || rows[i]->mode != MSK_ROWS_POINT))
      return fail(ctx, MSK_ERR_INVALID_ARG, "jump_only takes exterior estimates with point rows");
    msk_status st = check_problem(ctx, meshes[i], rows[i], bases[i], walks, eps[i], inset_h[i], side, &o);
    if (st != MSK_OK) return fail(ctx, st, "mesh " + std::to_string(i) + ": " + ctx->err);
  }
  msk_batch* B = new msk_batch();
  B->ctx = ctx;
  B->n = n_meshes;
  B->W = walks;
  B->o = o;
  for (int32_t i = 0; i < n_meshes; ++i) {
    msk_dtn* d = nullptr;
    msk_status st = alloc_dtn(ctx, rows[i], bases[i], walks, false, &d);
    if (st != MSK_OK) {
      delete B;
      return st;
    }
    d->inset = inset_h[i];
    B->dtns.push_back(d);
    B->rows.push_back(rows[i]);
    B->md.push_back(make_meshdev(meshes[i], rows[i], bases[i], d, eps[i], inset_h[i], side, o, i));
  }
  // work order: meshes by decreasing cost (rows x log of the triangle count),
  // rows of each mesh in Z-order; the eight queues then hold contiguous runs
  std::vector<int32_t> mo(n_meshes);
  std::iota(mo.begin(), mo.end(), 0);
  auto cost = [&](int32_t i) { return (double)rows[i]->n * std::log2(2.0 + (double)meshes[i]->nf); };
  std::stable_sort(mo.begin(), mo.end(), [&](int32_t a, int32_t b) { return cost(a) > cost(b); });
  std::vector<RowSlot> slots;
  for (int32_t i : mo)
    for (int32_t r : rows[i]->order) slots.push_back(RowSlot{i, r, 0u});
  std::vector<RowRange> ranges;
  std::vector<RowCounters> counters;
  for (int32_t i = 0; i < n_meshes; ++i) {
    msk_dtn* d = B->dtns[i];
    if (B->md[i].mode == kRowsPoint && d->n > 0) {
      ranges.push_back(RowRange{B->n_point_rows, i, d->d_disc});
      B->n_point_rows += d->n;
    }
    counters.push_back(RowCounters{d->d_q, d->d_esc, d->d_cap, d->d_disc, d->d_walks, d->d_nonfinite, d->n});
  }
  B->n_ranges = (int32_t)ranges.size();
  hipError_t he;
  if ((he = upload(ctx, &B->lb.d_meshes, B->md.data(), B->md.size())) != hipSuccess ||
      (he = upload(ctx, &B->lb.d_slots, slots.data(), slots.size())) != hipSuccess ||
      (he = upload(ctx, &B->d_ranges, ranges.data(), ranges.size())) != hipSuccess ||
      (he = upload(ctx, &B->d_counters, counters.data(), counters.size())) != hipSuccess ||
      (he = dalloc(&B->d_totals, 6 * (size_t)n_meshes)) != hipSuccess ||
      (he = dalloc(&B->lb.d_qnext, 8)) != hipSuccess || (he = dalloc(&B->lb.d_qend, 8)) != hipSuccess ||
      (he = dalloc(&B->lb.d_stats, 3)) != hipSuccess) {
    delete B;
    return fail(ctx, MSK_ERR_DEVICE, std::string("batch setup: ") + hipGetErrorString(he));
  }
  for (int i = 0; i < 4; ++i)
    if ((he = hipEventCreate(&B->ev[i])) != hipSuccess) {
      delete B;
      return fail(ctx, MSK_ERR_DEVICE, std::string("batch events: ") + hipGetErrorString(he));
    }
  // capture on a stream of its own (the context's stream may be the legacy
  // null stream, which cannot be captured); replay on the context's stream
  hipStream_t cap = nullptr;
  he = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
  for (int part = 0; part < 3 && he == hipSuccess; ++part) {
    he = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (he != hipSuccess) break;
    hipError_t ee = enqueue_batch(B, cap, part);
    hipGraph_t g = nullptr;
    he = hipStreamEndCapture(cap, &g);
    if (ee != hipSuccess) he = ee;
    if (he == hipSuccess) {
      B->graph[part] = g;
      he = hipGraphInstantiate(&B->exec[part], g, nullptr, nullptr, 0);
    } else if (g) {
      (void)hipGraphDestroy(g);
    }
  }
  if (cap) (void)hipStreamDestroy(cap);
  if (he != hipSuccess) {
    delete B;
    return fail(ctx, MSK_ERR_DEVICE, std::string("batch graph capture: ") + hipGetErrorString(he));
  }
  *out = B;
  return MSK_OK;
}

extern "C" msk_status msk_batch_run(msk_batch* B) {
  if (!B) return MSK_ERR_INVALID_ARG;
  msk_ctx* ctx = B->ctx;
  HIP_TRY(ctx, hipEventRecord(B->ev[0], ctx->stream));
  HIP_TRY(ctx, hipGraphLaunch(B->exec[0], ctx->stream));
  HIP_TRY(ctx, hipEventRecord(B->ev[1], ctx->stream));
  HIP_TRY(ctx, hipGraphLaunch(B->exec[1], ctx->stream));
  HIP_TRY(ctx, hipEventRecord(B->ev[2], ctx->stream));
  HIP_TRY(ctx, hipGraphLaunch(B->exec[2], ctx->stream));
  HIP_TRY(ctx, hipEventRecord(B->ev[3], ctx->stream));
  HIP_TRY(ctx, hipEventSynchronize(B->ev[3]));
  float tot = 0, wk = 0;
  HIP_TRY(ctx, hipEventElapsedTime(&tot, B->ev[0], B->ev[3]));
  HIP_TRY(ctx, hipEventElapsedTime(&wk, B->ev[1], B->ev[2]));
  std::vector<unsigned long long> tot6(6 * (size_t)B->n);
  HIP_TRY(ctx, hipMemcpy(tot6.data(), B->d_totals, tot6.size() * 8, hipMemcpyDeviceToHost));
  msk_dtn_info T{};
  for (int32_t i = 0; i < B->n; ++i) {
    msk_dtn* d = B->dtns[i];
    info_from_totals(d, &tot6[6 * (size_t)i]);
    d->info.walk_kernel_ms = wk;  // one shared launch
    d->info.total_ms = tot;
    d->info.walk_launches = 1;
    T.n_rows += d->info.n_rows;
    T.walks_total += d->info.walks_total;
    T.queries_total += d->info.queries_total;
    T.escaped_total += d->info.escaped_total;
    T.capped_total += d->info.capped_total;
    T.discarded_rows += d->info.discarded_rows;
    T.nonfinite_entries += d->info.nonfinite_entries;
  }
  T.walk_kernel_ms = wk;
  T.total_ms = tot;
  T.walk_launches = 1;
  if (B->o.collect_stats) {
    unsigned long long st[3];
    HIP_TRY(ctx, hipMemcpy(st, B->lb.d_stats, sizeof(st), hipMemcpyDeviceToHost));
    T.nodes_visited = (int64_t)st[0];
    T.tris_tested = (int64_t)st[1];
    T.valu_flops = (int64_t)st[2];
  }
  B->total = T;
  if (T.nonfinite_entries > 0) return fail(ctx, MSK_ERR_NUMERIC, "non-finite entries in S or se");
  return MSK_OK;
}

extern "C" msk_status msk_batch_dtn(const msk_batch* B, int32_t i, const msk_dtn** out) {
  if (!B || !out || i < 0 || i >= B->n) return MSK_ERR_INVALID_ARG;
  *out = B->dtns[i];
  return MSK_OK;
}

extern "C" msk_status msk_batch_get_info(const msk_batch* B, msk_dtn_info* info) {
  if (!B || !info) return MSK_ERR_INVALID_ARG;
  *info = B->total;
  return MSK_OK;
}

extern "C" void msk_batch_destroy(msk_batch* B) { delete B; }

extern "C" msk_status msk_estimate_dtn_batched(msk_ctx* ctx, int32_t n_meshes, const msk_mesh* const* meshes,
                                               const msk_rows* const* rows, const msk_basis* const* bases,
                                               const double* eps, const double* inset_h, int64_t walks, int32_t side,
                                               const msk_dtn_opts* opts, msk_dtn** out) {
  if (!ctx || !out) return MSK_ERR_INVALID_ARG;
  msk_batch* B = nullptr;
  msk_status st = msk_batch_create(ctx, n_meshes, meshes, rows, bases, eps, inset_h, walks, side, opts, &B);
  if (st != MSK_OK) return st;
  st = msk_batch_run(B);
  if (st != MSK_OK && st != MSK_ERR_NUMERIC) {
    msk_batch_destroy(B);
    return st;
  }
  for (int32_t i = 0; i < n_meshes; ++i) {  // hand the results over
    out[i] = B->dtns[i];
    B->dtns[i] = nullptr;
  }
  msk_batch_destroy(B);
  return st;
}

extern "C" msk_status msk_dtn_get_info(const msk_dtn* d, msk_dtn_info* info) {
  if (!d || !info) return MSK_ERR_INVALID_ARG;
  *info = d->info;
  return MSK_OK;
}

extern "C" msk_status msk_dtn_get(const msk_dtn* d, int32_t field, void* dst, int32_t dst_on_device) {
  if (!d || !dst) return MSK_ERR_INVALID_ARG;
  msk_ctx* ctx = d->ctx;
  const void* src = nullptr;
  size_t bytes = 0;
  const size_t nk = (size_t)d->n * (size_t)d->K, nl = (size_t)d->n * (size_t)d->W;
  switch (field) {
    case MSK_FIELD_S: src = d->d_S; bytes = nk * 8; break;
    case MSK_FIELD_SE: src = d->d_se; bytes = nk * 8; break;
    case MSK_FIELD_ROW_WALKS: src = d->d_walks; bytes = d->n * 8; break;
    case MSK_FIELD_ROW_QUERIES: src = d->d_q; bytes = d->n * 8; break;
    case MSK_FIELD_ROW_ESCAPED: src = d->d_esc; bytes = d->n * 8; break;
    case MSK_FIELD_ROW_CAPPED: src = d->d_cap; bytes = d->n * 8; break;
    case MSK_FIELD_ROW_DISCARDED: src = d->d_disc; bytes = d->n * 4; break;
    case MSK_FIELD_LOG_STATUS: src = d->d_log_status; bytes = nl * 4; break;
    case MSK_FIELD_LOG_TRI: src = d->d_log_tri; bytes = nl * 4; break;
    case MSK_FIELD_LOG_BARY: src = d->d_log_bary; bytes = nl * 8; break;
    case MSK_FIELD_LOG_QUERIES: src = d->d_log_q; bytes = nl * 4; break;
    default: return fail(ctx, MSK_ERR_INVALID_ARG, "unknown field");
  }
  if (!src) return fail(ctx, MSK_ERR_INVALID_ARG, "field not recorded (walk log needs opts.record_log)");
  HIP_TRY(ctx, hipMemcpyAsync(dst, src, bytes, dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                              ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  return MSK_OK;
}

extern "C" void msk_dtn_destroy(msk_dtn* d) {
  if (!d) return;
  dtn_free(d);
  delete d;
}

namespace msk {
int steklov_modes_device(hipStream_t s, const double* dS, int64_t n_rows, const std::vector<double>& w,
                         const std::vector<int32_t>& discarded, int k, double* evals, double* evecs, int* iters,
                         int* block_out, double* max_res, double* ms_out, EigGemmTimes* gt, std::string& err);
}

extern "C" msk_status msk_steklov_modes(msk_ctx* ctx, const msk_dtn* d, int32_t k, double* evals, double* evecs,
                                        msk_eig_stats* stats) {
  if (!ctx || !d || !evals) return fail(ctx, MSK_ERR_INVALID_ARG, "null argument");
  if (d->K != d->n) return fail(ctx, MSK_ERR_INVALID_ARG, "the eigen step needs a square estimate (K == n_rows)");
  if (d->info.nonfinite_entries > 0) return fail(ctx, MSK_ERR_NUMERIC, "the estimate holds non-finite entries");
  std::vector<int32_t> disc((size_t)d->n);
  HIP_TRY(ctx, hipMemcpy(disc.data(), d->d_disc, d->n * 4, hipMemcpyDeviceToHost));
  int iters = 0, block = 0;
  double res = 0, ms = 0;
  std::string err;
  EigGemmTimes gt;
  int rc = steklov_modes_device(ctx->stream, d->d_S, d->n, d->rows->w, disc, k, evals, evecs, &iters, &block, &res,
                                &ms, stats ? &gt : nullptr, err);
  if (stats) {
    stats->iterations = iters;
    stats->block = block;
    stats->max_residual = res;
    stats->lanczos_ms = ms;
    stats->fp32_products = gt.fp32_products;
    stats->fp32_product_ms = gt.fp32_ms;
    stats->fp32_product_flops = gt.fp32_flops;
    stats->fp64_products = gt.fp64_products;
    stats->fp64_product_ms = gt.fp64_ms;
    stats->fp64_product_flops = gt.fp64_flops;
  }
  if (rc == 1) return fail(ctx, MSK_ERR_INVALID_ARG, err);
  if (rc == 3) return fail(ctx, MSK_ERR_DEVICE, err);
  if (rc == 4) return fail(ctx, MSK_ERR_NOT_CONVERGED, err.empty() ? "residual target not reached" : err);
  return MSK_OK;
}

// -------------------------------------------------------- PSD estimator

extern "C" void msk_psd_opts_default(msk_psd_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->cap_deg = 2.5;
  o->bisect_iters = 10;
  o->r_max = 0.0;
  o->chunk_pairs = 262144;
}

extern "C" msk_status msk_estimate_psd(msk_ctx* ctx, const msk_mesh* m, const msk_rows* r, const msk_basis* b,
                                       int64_t pairs, double eps, const msk_dtn_opts* walk_opts,
                                       const msk_psd_opts* opts, double* S_out, double* se_out, float* radius_out,
                                       const msk_psd_log* log_out, msk_psd_info* info) {
  if (!ctx) return MSK_ERR_INVALID_ARG;
  if (!S_out) return fail(ctx, MSK_ERR_INVALID_ARG, "S must be given");
  if (!m || !r || !b) return fail(ctx, MSK_ERR_INVALID_ARG, "null mesh, rows or basis");
  if (r->mode != MSK_ROWS_POINT) return fail(ctx, MSK_ERR_INVALID_ARG, "the PSD estimator takes point rows");
  if (pairs < 1 || r->n * pairs < 2) return fail(ctx, MSK_ERR_INVALID_ARG, "need pairs >= 1 and >= 2 pairs in all");
  if (r->n * 2 * pairs >= ((int64_t)1 << 40) || 2 * pairs > ((int64_t)1 << 31))
    return fail(ctx, MSK_ERR_INVALID_ARG, "too many walks");
  if (b->K > 8192) return fail(ctx, MSK_ERR_INVALID_ARG, "the PSD estimator takes K <= 8192 basis functions");
  if (b->knn_mesh) return fail(ctx, MSK_ERR_INVALID_ARG, "the PSD estimator takes a per-vertex table basis");
  msk_psd_opts po;
  msk_psd_opts_default(&po);
  if (opts) po = *opts;
  if (!(po.cap_deg > 0.0 && po.cap_deg < 180.0)) return fail(ctx, MSK_ERR_INVALID_ARG, "cap_deg must be in (0, 180)");
  if (po.bisect_iters < 1 || po.bisect_iters > 40) return fail(ctx, MSK_ERR_INVALID_ARG, "bisect_iters in 1..40");
  if (po.chunk_pairs < 1) return fail(ctx, MSK_ERR_INVALID_ARG, "chunk_pairs must be >= 1");
  msk_dtn_opts o;
  msk_dtn_opts_default(&o);
  if (walk_opts) o = *walk_opts;
  if (o.form != MSK_FORM_PERSISTENT && o.form != MSK_FORM_PLAIN) return fail(ctx, MSK_ERR_INVALID_ARG, "bad form");
  if (o.mesh_id < 0 || o.mesh_id > 0xFFFFFF) return fail(ctx, MSK_ERR_INVALID_ARG, "mesh_id must be < 2^24");
  o.se_target = 0;
  o.walk_offset = 0;
  o.record_log = 1;  // collect_stats is the caller's (the counting kernel; reported in the info)
  const int64_t W = 2 * pairs;
  // the walk problem: interior walks; the inset is not used by ball starts
  if (walk_opts && walk_opts->jump_only) return fail(ctx, MSK_ERR_INVALID_ARG, "jump_only applies to exterior estimates");
  msk_status st = check_problem(ctx, m, r, b, W, eps, 2.0 * eps, MSK_INTERIOR, &o, false);
  if (st != MSK_OK) return st;
  double r_max = po.r_max;
  if (!(r_max > 0.0)) {  // half the shortest side of the bounding box (Appendix A, unbounded tangent balls)
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t v = 0; v < m->nv; ++v)
      for (int k = 0; k < 3; ++k) {
        lo[k] = std::min(lo[k], (double)m->vworld[3 * v + k]);
        hi[k] = std::max(hi[k], (double)m->vworld[3 * v + k]);
      }
    r_max = 0.5 * std::min(hi[0] - lo[0], std::min(hi[1] - lo[1], hi[2] - lo[2]));
  }
  if (!(r_max > 0.0)) return fail(ctx, MSK_ERR_INVALID_ARG, "flat mesh: no tangent balls");
  msk_dtn* d = nullptr;
  st = alloc_dtn(ctx, r, b, W, true, &d);
  if (st != MSK_OK) return st;
  const int64_t K = b->K, n = d->n, Kp = (K + 63) / 64 * 64;
  const int64_t chunk = std::min<int64_t>(po.chunk_pairs, n * pairs);
  // partial-sum slots of the matrix-core products: the fused form (K <= 384)
  // has one per workgroup column; the two-pass form 4 per row slice, at most
  // 1024 slices and about 256 MB per matrix
  const int64_t nblk = psd_blocks(Kp);
  const int64_t fused_slots = psd_fused_slots(Kp, n * pairs);
  const bool fused = fused_slots > 0;
  const int64_t slices = std::max<int64_t>(1, std::min<int64_t>(1024, ((int64_t)1 << 28) / (nblk * 32768 * 4)));
  const int64_t n_slots = fused ? fused_slots : 4 * slices;
  float* d_rad = nullptr;
  float* d_tab = nullptr;
  double *d_S = nullptr, *d_Q = nullptr, *d_se = nullptr, *d_U = nullptr, *d_V = nullptr;
  double *d_PS = nullptr, *d_PQ = nullptr;
  hipEvent_t ev[6] = {};
  auto cleanup = [&](msk_status s) {
    dfree(d_rad);
    dfree(d_tab);
    dfree(d_S);
    dfree(d_Q);
    dfree(d_se);
    dfree(d_U);
    dfree(d_V);
    dfree(d_PS);
    dfree(d_PQ);
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
    dtn_free(d);
    delete d;
    return s;
  };
#define HIP_P(expr)                                                                                   \
  do {                                                                                                \
    hipError_t e_ = (expr);                                                                           \
    if (e_ != hipSuccess)                                                                             \
      return cleanup(fail(ctx, e_ == hipErrorOutOfMemory ? MSK_ERR_OOM : MSK_ERR_DEVICE,             \
                          std::string(#expr) + ": " + hipGetErrorString(e_)));                        \
  } while (0)
  HIP_P(dalloc(&d_rad, n));
  HIP_P(dalloc(&d_tab, b->nv * K));
  HIP_P(dalloc(&d_S, K * K));
  HIP_P(dalloc(&d_Q, K * K));
  HIP_P(dalloc(&d_se, K * K));
  if (!fused) {
    HIP_P(dalloc(&d_U, 2 * chunk * Kp));
    HIP_P(dalloc(&d_V, 3 * chunk * Kp));
  }
  HIP_P(dalloc(&d_PS, n_slots * nblk * 4096));
  HIP_P(dalloc(&d_PQ, n_slots * nblk * 4096));
  for (hipEvent_t& e : ev) HIP_P(hipEventCreate(&e));
  hipStream_t s = ctx->stream;
  HIP_P(hipEventRecord(ev[0], s));
  HIP_P(launch_fill_u32(d_tab, b->nv * K, 0, s));
  HIP_P(launch_dense_table(b->d_rowptr, b->d_col, b->d_val, b->nv, K, d_tab, s));
  if (!fused) {  // the two-pass form adds into its slots call by call
    HIP_P(launch_fill_u64(d_PS, n_slots * nblk * 4096, 0, s));
    HIP_P(launch_fill_u64(d_PQ, n_slots * nblk * 4096, 0, s));
  }
  HIP_P(launch_fill_u64(d->d_q, n, 0, s));
  HIP_P(launch_fill_u64(d->d_esc, n, 0, s));
  HIP_P(launch_fill_u64(d->d_cap, n, 0, s));
  HIP_P(launch_fill_u64(d->d_walks, n, (unsigned long long)W, s));
  HIP_P(launch_fill_u32(d->d_disc, n, 0u, s));
  HIP_P(launch_fill_u32(d->d_log_status, n * W, 0xFFFFFFFFu, s));
  HIP_P(launch_fill_u32(d->d_log_tri, n * W, 0xFFFFFFFFu, s));
  HIP_P(launch_fill_u32(d->d_log_bary, 2 * n * W, 0u, s));
  HIP_P(launch_fill_u32(d->d_log_q, n * W, 0u, s));
  MeshDev M = make_meshdev(m, r, b, d, eps, 2.0 * eps, MSK_INTERIOR, o, o.mesh_id);
  M.ball_r = d_rad;
  M.ball_u0 = std::sin(0.5 * po.cap_deg * M_PI / 180.0);
  // tangent balls (tolerance: half the termination shell)
  HIP_P(launch_tangent_ball(M, n, (float)r_max, po.bisect_iters, (float)(0.5 * eps), d_rad, s));
  HIP_P(hipEventRecord(ev[1], s));
  // walks from the balls
  std::vector<MeshDev> meshes{M};
  std::vector<RowSlot> slots(r->order.size());
  for (size_t i = 0; i < slots.size(); ++i) slots[i] = RowSlot{0, r->order[i], 0u};
  const int use_lds = (o.form == MSK_FORM_PERSISTENT && m->top_nodes > 0) ? 1 : 0;
  double walk_ms = 0;
  int64_t stats[3] = {0, 0, 0};
  {
    msk_status ws = run_walks(ctx, meshes, slots, W, 0, o, use_lds, m->top_nodes, &walk_ms, stats);
    if (ws != MSK_OK) return cleanup(ws);
  }
  HIP_P(hipEventRecord(ev[2], s));
  // rank-one updates: gather a chunk of pairs, then S += U^T U, Q += V^T V
  PsdGather G{};
  G.tab = d_tab;
  G.K = K;
  G.Kp = Kp;
  G.pairs = pairs;
  G.faces = m->d_faces;
  G.tri = r->d_tri;
  G.bary = r->d_bary;
  G.w = r->d_w;
  G.radius = d_rad;
  G.u0 = M.ball_u0;
  G.log_status = d->d_log_status;
  G.log_tri = d->d_log_tri;
  G.log_bary = d->d_log_bary;
  float gather_ms = 0, prod_ms = 0;
  if (fused) {
    HIP_P(hipEventRecord(ev[3], s));
    HIP_P(launch_psd_fused(G, n * pairs, n_slots, d_PS, d_PQ, s));
    HIP_P(hipEventRecord(ev[5], s));
    HIP_P(hipEventSynchronize(ev[5]));
    HIP_P(hipEventElapsedTime(&prod_ms, ev[3], ev[5]));
  }
  for (int64_t q0 = 0; !fused && q0 < n * pairs; q0 += chunk) {
    const int64_t nq = std::min(chunk, n * pairs - q0);
    HIP_P(hipEventRecord(ev[3], s));
    HIP_P(launch_psd_gather(G, q0, nq, d_U, d_V, s));
    HIP_P(hipEventRecord(ev[4], s));
    HIP_P(launch_psd_syrk(d_U, 2 * nq, Kp, slices, d_PS, s));
    HIP_P(launch_psd_syrk(d_V, 3 * nq, Kp, slices, d_PQ, s));
    HIP_P(hipEventRecord(ev[5], s));
    HIP_P(hipEventSynchronize(ev[5]));
    float a = 0, c = 0;
    HIP_P(hipEventElapsedTime(&a, ev[3], ev[4]));
    HIP_P(hipEventElapsedTime(&c, ev[4], ev[5]));
    gather_ms += a;
    prod_ms += c;
  }
  HIP_P(hipEventRecord(ev[3], s));
  HIP_P(launch_psd_reduce(d_PS, n_slots, K, Kp, d_S, s));
  HIP_P(launch_psd_reduce(d_PQ, n_slots, K, Kp, d_Q, s));
  HIP_P(hipEventRecord(ev[4], s));
  HIP_P(launch_psd_se(d_S, d_Q, K * K, (double)(n * pairs), d_se, s));
  HIP_P(launch_fill_u64(d->d_nonfinite, 1, 0, s));
  HIP_P(launch_count_nonfinite(d_S, K * K, d->d_nonfinite, s));
  HIP_P(launch_count_nonfinite(d_se, K * K, d->d_nonfinite, s));
  HIP_P(hipEventRecord(ev[5], s));
  HIP_P(hipEventSynchronize(ev[5]));
  float tot = 0, tb = 0, red = 0;
  HIP_P(hipEventElapsedTime(&red, ev[3], ev[4]));
  prod_ms += red;
  HIP_P(hipEventElapsedTime(&tot, ev[0], ev[5]));
  HIP_P(hipEventElapsedTime(&tb, ev[0], ev[1]));
  // results to the host
  HIP_P(hipMemcpy(S_out, d_S, K * K * 8, hipMemcpyDeviceToHost));
  if (se_out) HIP_P(hipMemcpy(se_out, d_se, K * K * 8, hipMemcpyDeviceToHost));
  std::vector<float> rad((size_t)n);
  HIP_P(hipMemcpy(rad.data(), d_rad, n * 4, hipMemcpyDeviceToHost));
  if (radius_out) std::memcpy(radius_out, rad.data(), n * 4);
  if (log_out) {
    if (log_out->status) HIP_P(hipMemcpy(log_out->status, d->d_log_status, n * W * 4, hipMemcpyDeviceToHost));
    if (log_out->tri) HIP_P(hipMemcpy(log_out->tri, d->d_log_tri, n * W * 4, hipMemcpyDeviceToHost));
    if (log_out->bary) HIP_P(hipMemcpy(log_out->bary, d->d_log_bary, n * W * 8, hipMemcpyDeviceToHost));
    if (log_out->queries) HIP_P(hipMemcpy(log_out->queries, d->d_log_q, n * W * 4, hipMemcpyDeviceToHost));
  }
  {
    msk_status cs = collect_info(ctx, d);
    if (cs != MSK_OK) return cleanup(cs);
  }
  msk_psd_info I;
  std::memset(&I, 0, sizeof(I));
  I.n_rows = n;
  I.K = K;
  I.pairs = pairs;
  I.queries_total = d->info.queries_total;
  I.escaped_total = d->info.escaped_total;
  I.capped_total = d->info.capped_total;
  double rsum = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (rad[i] > 0) {
      rsum += rad[i];
      I.walks_total += W;
    } else {
      ++I.dropped_rows;
    }
  }
  I.mean_radius = (n > I.dropped_rows) ? rsum / (double)(n - I.dropped_rows) : 0.0;
  I.r_max = r_max;
  I.tangent_ms = tb;
  I.walk_kernel_ms = walk_ms;
  I.gather_ms = gather_ms;
  I.product_ms = prod_ms;
  I.total_ms = tot;
  I.nonfinite_entries = d->info.nonfinite_entries;
  I.fused = fused ? 1 : 0;
  I.nodes_visited = stats[0];
  I.tris_tested = stats[1];
  I.valu_flops = stats[2];
  if (info) *info = I;
#undef HIP_P
  const bool bad = I.nonfinite_entries > 0;
  cleanup(MSK_OK);
  if (bad) return fail(ctx, MSK_ERR_NUMERIC, "non-finite entries in S or se");
  return MSK_OK;
}

// ------------------------------------------- Kelvin-inverted exterior

struct msk_kelvin {
  msk_ctx* ctx = nullptr;
  const msk_mesh* mesh = nullptr;
  double centre[3] = {0, 0, 0};
  double radius = 0;                // bound of the inverted domain
  double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};  // box of the inverted vertices
  int32_t depth = 0, leaf_size = 4;
  int64_t n_nodes = 0;
  Node4* d_nodes = nullptr;
  KelvinTri* d_tris = nullptr;
  KelvinPre* d_pre = nullptr;
};

namespace {

double dot3d(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

// Squared distance from the origin to triangle (A, B, C): the nearest point
// of the plane if it lies inside, else of the three edges.
double origin_tri_d2(const double* A, const double* B, const double* C) {
  const double* P[3] = {A, B, C};
  double best = INFINITY;
  for (int e = 0; e < 3; ++e) {
    const double* p0 = P[e];
    const double* p1 = P[(e + 1) % 3];
    double d[3] = {p1[0] - p0[0], p1[1] - p0[1], p1[2] - p0[2]};
    const double dd = dot3d(d, d);
    double t = dd > 0 ? -dot3d(p0, d) / dd : 0.0;
    t = std::min(1.0, std::max(0.0, t));
    const double q[3] = {p0[0] + t * d[0], p0[1] + t * d[1], p0[2] + t * d[2]};
    best = std::min(best, dot3d(q, q));
  }
  const double ab[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]}, ac[3] = {C[0] - A[0], C[1] - A[1], C[2] - A[2]};
  const double n[3] = {ab[1] * ac[2] - ab[2] * ac[1], ab[2] * ac[0] - ab[0] * ac[2], ab[0] * ac[1] - ab[1] * ac[0]};
  const double nn = dot3d(n, n);
  if (nn > 0) {
    const double t = dot3d(n, A) / nn;  // foot of the origin on the plane: t n
    const double f[3] = {t * n[0], t * n[1], t * n[2]};
    // inside test by the signs of the sub-triangle areas
    auto side = [&](const double* u, const double* v) {
      const double a[3] = {u[0] - f[0], u[1] - f[1], u[2] - f[2]}, b[3] = {v[0] - f[0], v[1] - f[1], v[2] - f[2]};
      const double c[3] = {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
      return dot3d(c, n);
    };
    const double s0 = side(A, B), s1 = side(B, C), s2 = side(C, A);
    if ((s0 >= 0 && s1 >= 0 && s2 >= 0) || (s0 <= 0 && s1 <= 0 && s2 <= 0)) best = std::min(best, dot3d(f, f));
  }
  return best;
}

float round_down(double x) {
  float f = (float)x;
  return (double)f > x ? std::nextafter(f, -INFINITY) : f;
}
float round_up(double x) {
  float f = (float)x;
  return (double)f < x ? std::nextafter(f, INFINITY) : f;
}

}  // namespace

extern "C" msk_status msk_kelvin_create(msk_ctx* ctx, const msk_mesh* m, const double* centre, int32_t leaf_size,
                                        msk_kelvin** out) {
  if (!ctx || !out) return MSK_ERR_INVALID_ARG;
  *out = nullptr;
  if (!m || !centre) return fail(ctx, MSK_ERR_INVALID_ARG, "null mesh or centre");
  if (!std::isfinite(centre[0]) || !std::isfinite(centre[1]) || !std::isfinite(centre[2]))
    return fail(ctx, MSK_ERR_INVALID_ARG, "the inversion centre must be finite");
  if (leaf_size == 0) leaf_size = 1;
  if (leaf_size < 1 || leaf_size > 8) return fail(ctx, MSK_ERR_INVALID_ARG, "leaf_size must be in 1..8");
  const int64_t nf = m->nf;
  std::vector<KelvinTri> rec((size_t)nf);
  std::vector<Box3f> boxes((size_t)nf);
  std::vector<float> cen((size_t)nf * 3);
  double dmin = INFINITY, lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  double rmax = 0, far2 = 0;
  for (int64_t v = 0; v < m->nv; ++v) {
    double x[3];
    for (int k = 0; k < 3; ++k) x[k] = (double)m->vworld[3 * v + k] - centre[k];
    const double r2 = dot3d(x, x);
    if (!(r2 > 0)) return fail(ctx, MSK_ERR_INVALID_ARG, "the inversion centre is a mesh vertex");
    far2 = std::max(far2, r2);
    for (int k = 0; k < 3; ++k) {
      lo[k] = std::min(lo[k], x[k] / r2);
      hi[k] = std::max(hi[k], x[k] / r2);
    }
    rmax = std::max(rmax, 1.0 / std::sqrt(r2));
  }
  for (int64_t t = 0; t < nf; ++t) {
    KelvinTri& T = rec[t];
    double* P[3] = {T.a, T.b, T.c};
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k) P[j][k] = (double)m->vworld[3 * (int64_t)m->faces[3 * t + j] + k] - centre[k];
    T.orig = (int32_t)t;
    T.has_plane = kelvin_plane(T.a, T.b, T.c, T.n, T.cpl) ? 1 : 0;
    if (!T.has_plane) T.n[0] = T.n[1] = T.n[2] = T.cpl = 0.0;
    T.M2 = std::max(dot3d(T.a, T.a), std::max(dot3d(T.b, T.b), dot3d(T.c, T.c)));
    // a box containing the image: each coordinate of y / |y|^2 over the
    // triangle is a quotient of a value in the coordinate's range by one in
    // [m2, M2] (squared distances from the centre)
    const double m2 = origin_tri_d2(T.a, T.b, T.c);
    const double M2 = T.M2;
    dmin = std::min(dmin, m2);
    // a centre within 1e-9 of the mesh's extent from a triangle makes the
    // inverted domain ~1e9 times larger than its elements: refused as on it
    if (!(m2 > 1e-18 * far2))
      return fail(ctx, MSK_ERR_INVALID_ARG, "the inversion centre lies on the surface (triangle " + std::to_string(t) +
                                                ", within 1e-9 of the mesh's extent)");
    // a second enclosure, tight for small elements: kappa(y) = kappa(a) +
    // J(a) (y - a) + R with J(a) = (I - 2 a^ a^T) / |a|^2 and the Taylor
    // remainder |R| <= |y - a|^2 / rmin^3 (|D^2 kappa(x)[h, h]| = 2 |h|^2 /
    // |x|^3, and the segment's points are at least rmin = sqrt(m2) from the
    // centre): the affine image of the triangle, padded by twice that bound
    double p3[3][3];
    {
      const double aa = dot3d(T.a, T.a);
      const double e1[3] = {T.b[0] - T.a[0], T.b[1] - T.a[1], T.b[2] - T.a[2]};
      const double e2[3] = {T.c[0] - T.a[0], T.c[1] - T.a[1], T.c[2] - T.a[2]};
      const double ae1 = dot3d(T.a, e1), ae2 = dot3d(T.a, e2);
      for (int k = 0; k < 3; ++k) {
        p3[0][k] = T.a[k] / aa;
        p3[1][k] = p3[0][k] + (e1[k] - 2.0 * T.a[k] * ae1 / aa) / aa;
        p3[2][k] = p3[0][k] + (e2[k] - 2.0 * T.a[k] * ae2 / aa) / aa;
      }
    }
    double h2 = 0.0;
    for (const double* v : {T.b, T.c}) {
      const double e[3] = {v[0] - T.a[0], v[1] - T.a[1], v[2] - T.a[2]};
      h2 = std::max(h2, dot3d(e, e));
    }
    const double rem = 2.0 * h2 / (m2 * std::sqrt(m2));
    for (int k = 0; k < 3; ++k) {
      const double a = std::min(T.a[k], std::min(T.b[k], T.c[k])), b = std::max(T.a[k], std::max(T.b[k], T.c[k]));
      double l, h;
      if (a >= 0) { l = a / M2; h = b / m2; }
      else if (b <= 0) { l = a / m2; h = b / M2; }
      else { l = a / m2; h = b / m2; }
      // the intersection of the two enclosures
      const double l2 = std::min(p3[0][k], std::min(p3[1][k], p3[2][k])) - rem;
      const double u2 = std::max(p3[0][k], std::max(p3[1][k], p3[2][k])) + rem;
      l = std::max(l, l2);
      h = std::min(h, u2);
      const double pad = 1e-12 * (std::fabs(l) + std::fabs(h)) + 1e-15 * std::sqrt(1.0 / m2);
      boxes[t].lo[k] = round_down(l - pad);
      boxes[t].hi[k] = round_up(h + pad);
      cen[3 * t + k] = (float)(0.5 * (l + h));
    }
  }
  std::vector<Node4> nodes;
  std::vector<int32_t> leaf_order;
  int depth = 0;
  std::string err = build_bvh_boxes(boxes, cen, leaf_size, nodes, leaf_order, depth);
  if (!err.empty()) return fail(ctx, MSK_ERR_INVALID_ARG, "inverted BVH: " + err);
  std::vector<KelvinTri> ordered(leaf_order.size());
  for (size_t i = 0; i < leaf_order.size(); ++i) ordered[i] = rec[leaf_order[i]];
  msk_kelvin* K = new msk_kelvin();
  K->ctx = ctx;
  K->mesh = m;
  for (int k = 0; k < 3; ++k) {
    K->centre[k] = centre[k];
    K->lo[k] = lo[k];
    K->hi[k] = hi[k];
  }
  K->radius = std::max(rmax, 1.0 / std::sqrt(dmin));
  K->depth = depth;
  K->leaf_size = leaf_size;
  K->n_nodes = (int64_t)nodes.size();
  hipError_t he;
  if ((he = upload(ctx, &K->d_nodes, nodes.data(), nodes.size())) != hipSuccess ||
      (he = upload(ctx, &K->d_tris, ordered.data(), ordered.size())) != hipSuccess ||
      (he = dalloc(&K->d_pre, ordered.size())) != hipSuccess ||
      (he = launch_kelvin_prepare(K->d_tris, (int64_t)ordered.size(), K->d_pre, ctx->stream)) != hipSuccess ||
      (he = hipStreamSynchronize(ctx->stream)) != hipSuccess) {
    msk_kelvin_destroy(K);
    return fail(ctx, he == hipErrorOutOfMemory ? MSK_ERR_OOM : MSK_ERR_DEVICE,
                std::string("inverted mesh upload: ") + hipGetErrorString(he));
  }
  *out = K;
  return MSK_OK;
}

extern "C" msk_status msk_kelvin_get_info(const msk_kelvin* K, msk_kelvin_info* info) {
  if (!K || !info) return MSK_ERR_INVALID_ARG;
  std::memset(info, 0, sizeof(*info));
  for (int k = 0; k < 3; ++k) {
    info->centre[k] = K->centre[k];
    info->box_lo[k] = K->lo[k];
    info->box_hi[k] = K->hi[k];
  }
  info->radius = K->radius;
  info->r_max = 0.5 * std::min(K->hi[0] - K->lo[0], std::min(K->hi[1] - K->lo[1], K->hi[2] - K->lo[2]));
  info->n_tris = K->mesh->nf;
  info->n_nodes = K->n_nodes;
  info->depth = K->depth;
  info->leaf_size = K->leaf_size;
  return MSK_OK;
}

extern "C" void msk_kelvin_destroy(msk_kelvin* K) {
  if (!K) return;
  dfree(K->d_nodes);
  dfree(K->d_tris);
  dfree(K->d_pre);
  delete K;
}

static KelvinDev kelvin_dev(const msk_kelvin* K, double eps, const msk_dtn_opts& o) {
  KelvinDev D;
  std::memset(&D, 0, sizeof(D));
  D.nodes = K->d_nodes;
  D.tris = K->d_tris;
  D.pre = K->d_pre;
  D.n_tris = K->mesh->nf;
  D.radius = K->radius;
  D.eps2 = eps * eps;
  D.kappa = o.kappa;
  D.delta = o.delta_rel * K->radius;
  D.max_steps = o.max_steps > 0 ? o.max_steps : 1024;
  D.mesh_id = (uint32_t)o.mesh_id;
  D.seed_lo = (uint32_t)o.seed;
  D.seed_hi = (uint32_t)(o.seed >> 32);
  return D;
}

extern "C" msk_status msk_kelvin_closest_points(msk_ctx* ctx, const msk_kelvin* K, const double* Q, int64_t nq,
                                                int32_t* tri, double* d2, double* qpt, double* bary) {
  if (!ctx || !K) return MSK_ERR_INVALID_ARG;
  if (nq < 0 || (nq > 0 && (!Q || !tri || !d2 || !qpt || !bary)))
    return fail(ctx, MSK_ERR_INVALID_ARG, "bad query arrays");
  if (nq == 0) return MSK_OK;
  msk_dtn_opts o;
  msk_dtn_opts_default(&o);
  HIP_TRY(ctx, launch_kelvin_closest(kelvin_dev(K, 0.0, o), Q, nq, tri, d2, qpt, bary, ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  return MSK_OK;
}

extern "C" msk_status msk_estimate_kelvin(msk_ctx* ctx, const msk_kelvin* K, const msk_rows* r, const msk_basis* b,
                                          int64_t pairs, int64_t kill_walks, double eps,
                                          const msk_dtn_opts* walk_opts, const msk_psd_opts* opts, double* S_jump,
                                          double* se_jump, double* S_kill, double* se_kill, double* radius_out,
                                          const msk_kelvin_log* log_out, msk_kelvin_est_info* info) {
  if (!ctx) return MSK_ERR_INVALID_ARG;
  if (!K || !r || !b) return fail(ctx, MSK_ERR_INVALID_ARG, "null inverted mesh, rows or basis");
  if (!S_jump) return fail(ctx, MSK_ERR_INVALID_ARG, "S_jump must be given");
  if (r->mesh != K->mesh) return fail(ctx, MSK_ERR_INVALID_ARG, "rows were created for another mesh");
  if (r->mode != MSK_ROWS_POINT) return fail(ctx, MSK_ERR_INVALID_ARG, "the exterior estimator takes point rows");
  if (b->knn_mesh || !b->d_rowptr) return fail(ctx, MSK_ERR_INVALID_ARG, "a per-vertex table basis is required");
  if (b->nv != K->mesh->nv) return fail(ctx, MSK_ERR_INVALID_ARG, "basis vertex count differs from the mesh's");
  if (b->K > 8192) return fail(ctx, MSK_ERR_INVALID_ARG, "K <= 8192 basis functions");
  if (pairs < 1 || 2 * pairs > ((int64_t)1 << 31) || r->n * 2 * pairs >= ((int64_t)1 << 40))
    return fail(ctx, MSK_ERR_INVALID_ARG, "need 1 <= pairs and fewer than 2^40 walks");
  if (kill_walks < 0 || kill_walks % 2 != 0 || kill_walks > ((int64_t)1 << 31))
    return fail(ctx, MSK_ERR_INVALID_ARG, "kill_walks must be even, in 0..2^31");
  if (kill_walks > 0 && !S_kill) return fail(ctx, MSK_ERR_INVALID_ARG, "S_kill must be given with kill_walks > 0");
  msk_psd_opts po;
  msk_psd_opts_default(&po);
  if (opts) po = *opts;
  if (!(po.cap_deg > 0.0 && po.cap_deg < 180.0)) return fail(ctx, MSK_ERR_INVALID_ARG, "cap_deg must be in (0, 180)");
  if (po.bisect_iters < 1 || po.bisect_iters > 40) return fail(ctx, MSK_ERR_INVALID_ARG, "bisect_iters in 1..40");
  msk_dtn_opts o;
  msk_dtn_opts_default(&o);
  if (walk_opts) o = *walk_opts;
  if (!(o.kappa >= 0.0 && o.kappa < 0.5 && o.delta_rel >= 0.0 && o.delta_rel < 0.25))
    return fail(ctx, MSK_ERR_INVALID_ARG, "need 0 <= kappa < 1/2 and 0 <= delta_rel < 1/4");
  if (o.mesh_id < 0 || o.mesh_id > 0xFFFFFF) return fail(ctx, MSK_ERR_INVALID_ARG, "mesh_id must be < 2^24");
  // the step guard and the FP64 resolution of the inverted scene bound the shell
  const double eps_floor = std::max(o.delta_rel * K->radius / (1.0 - o.kappa), std::ldexp(K->radius, -40));
  if (!(eps > eps_floor) || !std::isfinite(eps))
    return fail(ctx, MSK_ERR_INVALID_ARG, "eps must exceed " + std::to_string(eps_floor) +
                                              " (inverted units: the step guard and the FP64 resolution)");
  const int64_t n = r->n, K_ = b->K, Kp = (K_ + 63) / 64 * 64;
  const int64_t n_jump = n * 2 * pairs, n_walk = n_jump + kill_walks;
  double r_max = po.r_max;
  if (!(r_max > 0.0)) r_max = 0.5 * std::min(K->hi[0] - K->lo[0], std::min(K->hi[1] - K->lo[1], K->hi[2] - K->lo[2]));
  if (!(r_max > 0.0)) return fail(ctx, MSK_ERR_INVALID_ARG, "flat inverted surface: no tangent balls");
  // samples and image normals (host, FP64, relative to the centre)
  std::vector<double> st((size_t)n * 3), nt((size_t)n * 3), s3((size_t)n);
  for (int64_t i = 0; i < n; ++i) {
    double s[3], nn[3];
    for (int k = 0; k < 3; ++k) {
      s[k] = (double)r->p_world[3 * i + k] - K->centre[k];
      nn[k] = r->n_world[3 * i + k];
    }
    const double sl = std::sqrt(dot3d(s, s)), nl = std::sqrt(dot3d(nn, nn));
    if (!(sl > 0) || !(nl > 0)) return fail(ctx, MSK_ERR_INVALID_ARG, "row " + std::to_string(i) + " at the centre");
    const double sh[3] = {s[0] / sl, s[1] / sl, s[2] / sl};
    for (int k = 0; k < 3; ++k) nn[k] /= nl;
    const double sn = dot3d(sh, nn);
    for (int k = 0; k < 3; ++k) {
      st[3 * i + k] = s[k] / (sl * sl);
      nt[3 * i + k] = -(nn[k] - 2.0 * sn * sh[k]);
    }
    s3[i] = 1.0 / (sl * sl * sl);
  }
  const double u0 = std::sin(0.5 * po.cap_deg * M_PI / 180.0);
  double *d_st = nullptr, *d_nt = nullptr, *d_rad = nullptr, *d_g = nullptr, *d_alpha = nullptr, *d_kalpha = nullptr;
  int32_t *d_ls = nullptr, *d_lt = nullptr, *d_lq = nullptr, *d_ktri = nullptr;
  float *d_lb = nullptr, *d_tab = nullptr, *d_kbary = nullptr;
  unsigned long long *d_rq = nullptr, *d_tq = nullptr, *d_kq = nullptr, *d_nonf = nullptr, *d_next = nullptr,
                     *d_wstats = nullptr;
  double *d_S = nullptr, *d_Q = nullptr, *d_se = nullptr, *d_PS = nullptr, *d_PQ = nullptr, *d_U = nullptr,
         *d_V = nullptr;
  hipEvent_t ev[5] = {};
  auto cleanup = [&](msk_status s_) {
    dfree(d_st); dfree(d_nt); dfree(d_rad); dfree(d_g); dfree(d_alpha); dfree(d_kalpha);
    dfree(d_ls); dfree(d_lt); dfree(d_lq); dfree(d_ktri); dfree(d_lb); dfree(d_tab); dfree(d_kbary);
    dfree(d_rq); dfree(d_tq); dfree(d_kq); dfree(d_nonf); dfree(d_next); dfree(d_wstats);
    dfree(d_S); dfree(d_Q); dfree(d_se); dfree(d_PS); dfree(d_PQ); dfree(d_U); dfree(d_V);
    for (hipEvent_t& e : ev) {
      if (e) (void)hipEventDestroy(e);
      e = nullptr;
    }
    return s_;
  };
#define HIP_K(expr)                                                                                   \
  do {                                                                                                \
    hipError_t e_ = (expr);                                                                           \
    if (e_ != hipSuccess)                                                                             \
      return cleanup(fail(ctx, e_ == hipErrorOutOfMemory ? MSK_ERR_OOM : MSK_ERR_DEVICE,             \
                          std::string(#expr) + ": " + hipGetErrorString(e_)));                        \
  } while (0)
  hipStream_t s = ctx->stream;
  for (hipEvent_t& e : ev) HIP_K(hipEventCreate(&e));
  HIP_K(upload(ctx, &d_st, st.data(), st.size()));
  HIP_K(upload(ctx, &d_nt, nt.data(), nt.size()));
  HIP_K(dalloc(&d_rad, n));
  HIP_K(dalloc(&d_tq, n));
  HIP_K(dalloc(&d_rq, n));
  HIP_K(dalloc(&d_kq, 1));
  HIP_K(dalloc(&d_next, 1));
  HIP_K(dalloc(&d_nonf, 1));
  HIP_K(dalloc(&d_g, n_walk));
  HIP_K(dalloc(&d_ls, n_walk));
  HIP_K(dalloc(&d_lt, n_walk));
  HIP_K(dalloc(&d_lq, n_walk));
  HIP_K(dalloc(&d_lb, 2 * n_walk));
  HIP_K(dalloc(&d_tab, b->nv * K_));
  HIP_K(dalloc(&d_S, K_ * K_));
  HIP_K(dalloc(&d_Q, K_ * K_));
  HIP_K(dalloc(&d_se, K_ * K_));
  HIP_K(hipEventRecord(ev[0], s));
  HIP_K(launch_fill_u32(d_tab, b->nv * K_, 0, s));
  HIP_K(launch_dense_table(b->d_rowptr, b->d_col, b->d_val, b->nv, K_, d_tab, s));
  HIP_K(launch_fill_u64(d_rq, n, 0, s));
  HIP_K(launch_fill_u64(d_kq, 1, 0, s));
  const KelvinDev D = kelvin_dev(K, eps, o);
  HIP_K(launch_kelvin_tangent(D, d_st, d_nt, n, r_max, po.bisect_iters, 0.5 * eps, d_rad, d_tq, s));
  HIP_K(hipEventRecord(ev[1], s));
  KelvinDev DW = D;
  if (kill_walks > 0) {  // the origin's nearest element, shared by the first steps of all killing walks
    double* d_o = nullptr;
    int32_t* d_ot = nullptr;
    HIP_K(dalloc(&d_o, 10));
    hipError_t e1 = dalloc(&d_ot, 1);
    double ho[10] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int32_t hot = -1;
    if (e1 == hipSuccess) e1 = hipMemcpyAsync(d_o, ho, sizeof(ho), hipMemcpyHostToDevice, s);
    if (e1 == hipSuccess) e1 = launch_kelvin_closest(D, d_o, 1, d_ot, d_o + 3, d_o + 4, d_o + 7, s);
    if (e1 == hipSuccess) e1 = hipMemcpyAsync(ho, d_o, sizeof(ho), hipMemcpyDeviceToHost, s);
    if (e1 == hipSuccess) e1 = hipMemcpyAsync(&hot, d_ot, sizeof(hot), hipMemcpyDeviceToHost, s);
    if (e1 == hipSuccess) e1 = hipStreamSynchronize(s);
    dfree(d_o);
    dfree(d_ot);
    HIP_K(e1);
    DW.origin_known = 1;
    DW.origin_orig = hot;
    DW.origin_d2 = ho[3];
    for (int c = 0; c < 3; ++c) {
      DW.origin_q[c] = ho[4 + c];
      DW.origin_l[c] = ho[7 + c];
    }
  }
  HIP_K(launch_fill_u64(d_next, 1, 0, s));
  if (o.collect_stats) {  // the counting instantiation: same walks, work tallied
    HIP_K(dalloc(&d_wstats, 3));
    HIP_K(launch_fill_u64(d_wstats, 3, 0, s));
  }
  HIP_K(launch_kelvin_walks(DW, d_st, d_nt, d_rad, n, pairs, u0, kill_walks, d_ls, d_lt, d_lb, d_lq, d_g, d_rq,
                            d_kq, d_next, d_wstats, std::max(1, ctx->n_cu * 4), s));
  HIP_K(hipEventRecord(ev[2], s));
  std::vector<double> rad((size_t)n);
  HIP_K(hipMemcpyAsync(rad.data(), d_rad, n * 8, hipMemcpyDeviceToHost, s));
  HIP_K(hipStreamSynchronize(s));
  // alpha_i = w_i |s~_i|^3 Z_i / (2 pairs), Z_i = (1 / (2 r_i)) (1 / u0 - 1)
  std::vector<double> alpha((size_t)n, 0.0);
  int64_t dropped = 0;
  double rsum = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (rad[i] > 0) {
      alpha[i] = r->w[i] * s3[i] * (1.0 / (2.0 * rad[i])) * (1.0 / u0 - 1.0) / (2.0 * (double)pairs);
      rsum += rad[i];
    } else {
      ++dropped;
    }
  }
  HIP_K(upload(ctx, &d_alpha, alpha.data(), alpha.size()));
  // products of one term: fused (K <= 384) or gathered in chunks, then the
  // partial slots reduced into S and Q, and the standard error
  float prod_ms_total = 0;
  auto products = [&](const PsdGather& G, int64_t n_pairs, double* S_host, double* se_host) -> msk_status {
    const int64_t nblk = psd_blocks(Kp);
    const int64_t fused_slots = psd_fused_slots(Kp, n_pairs);
    const bool fused = fused_slots > 0;
    const int64_t chunk = std::min<int64_t>(std::max<int64_t>(1, po.chunk_pairs), n_pairs);
    const int64_t slices = std::max<int64_t>(1, std::min<int64_t>(1024, ((int64_t)1 << 28) / (nblk * 32768 * 4)));
    const int64_t n_slots = fused ? fused_slots : 4 * slices;
    dfree(d_PS); dfree(d_PQ); dfree(d_U); dfree(d_V);
    HIP_K(dalloc(&d_PS, n_slots * nblk * 4096));
    HIP_K(dalloc(&d_PQ, n_slots * nblk * 4096));
    HIP_K(hipEventRecord(ev[3], s));
    if (fused) {
      HIP_K(launch_psd_fused(G, n_pairs, n_slots, d_PS, d_PQ, s));
    } else {
      HIP_K(dalloc(&d_U, 2 * chunk * Kp));
      HIP_K(dalloc(&d_V, 3 * chunk * Kp));
      HIP_K(launch_fill_u64(d_PS, n_slots * nblk * 4096, 0, s));
      HIP_K(launch_fill_u64(d_PQ, n_slots * nblk * 4096, 0, s));
      for (int64_t q0 = 0; q0 < n_pairs; q0 += chunk) {
        const int64_t nq = std::min(chunk, n_pairs - q0);
        HIP_K(launch_psd_gather(G, q0, nq, d_U, d_V, s));
        HIP_K(launch_psd_syrk(d_U, 2 * nq, Kp, slices, d_PS, s));
        HIP_K(launch_psd_syrk(d_V, 3 * nq, Kp, slices, d_PQ, s));
      }
    }
    HIP_K(launch_psd_reduce(d_PS, n_slots, K_, Kp, d_S, s));
    HIP_K(launch_psd_reduce(d_PQ, n_slots, K_, Kp, d_Q, s));
    HIP_K(launch_psd_se(d_S, d_Q, K_ * K_, (double)n_pairs, d_se, s));
    HIP_K(launch_count_nonfinite(d_S, K_ * K_, d_nonf, s));
    HIP_K(launch_count_nonfinite(d_se, K_ * K_, d_nonf, s));
    HIP_K(hipEventRecord(ev[4], s));
    HIP_K(hipEventSynchronize(ev[4]));
    float ms = 0;
    HIP_K(hipEventElapsedTime(&ms, ev[3], ev[4]));
    prod_ms_total += ms;
    HIP_K(hipMemcpy(S_host, d_S, K_ * K_ * 8, hipMemcpyDeviceToHost));
    if (se_host) HIP_K(hipMemcpy(se_host, d_se, K_ * K_ * 8, hipMemcpyDeviceToHost));
    return MSK_OK;
  };
  HIP_K(launch_fill_u64(d_nonf, 1, 0, s));
  PsdGather G{};
  G.tab = d_tab;
  G.K = K_;
  G.Kp = Kp;
  G.pairs = pairs;
  G.faces = K->mesh->d_faces;
  G.tri = r->d_tri;
  G.bary = r->d_bary;
  G.w = r->d_w;
  G.u0 = u0;
  G.log_status = d_ls;
  G.log_tri = d_lt;
  G.log_bary = d_lb;
  G.alpha_row = d_alpha;
  G.walk_g = d_g;
  {
    msk_status ps = products(G, n * pairs, S_jump, se_jump);
    if (ps != MSK_OK) return cleanup(ps);
  }
  if (kill_walks > 0) {
    // killing walks as pairs of walks from a virtual sample with b(s) = 0:
    // X_p = alpha (g_1 b_1 b_1^T + g_2 b_2 b_2^T) / 2 with alpha = 8 pi / N0
    const int64_t nk = kill_walks / 2;
    std::vector<double> ka((size_t)nk, 8.0 * M_PI / (double)kill_walks);
    HIP_K(upload(ctx, &d_kalpha, ka.data(), ka.size()));
    HIP_K(dalloc(&d_ktri, nk));
    HIP_K(dalloc(&d_kbary, 3 * nk));
    HIP_K(launch_fill_u32(d_ktri, nk, 0u, s));
    HIP_K(launch_fill_u32(d_kbary, 3 * nk, 0u, s));
    PsdGather Gk = G;
    Gk.pairs = 1;
    Gk.tri = d_ktri;
    Gk.bary = d_kbary;
    Gk.w = nullptr;
    Gk.alpha_row = d_kalpha;
    Gk.log_status = d_ls + n_jump;
    Gk.log_tri = d_lt + n_jump;
    Gk.log_bary = d_lb + 2 * n_jump;
    Gk.walk_g = d_g + n_jump;
    msk_status ps = products(Gk, nk, S_kill, se_kill);
    if (ps != MSK_OK) return cleanup(ps);
  }
  // logs, counters and timings
  if (radius_out) std::memcpy(radius_out, rad.data(), n * 8);
  if (log_out) {
    if (log_out->status) HIP_K(hipMemcpy(log_out->status, d_ls, n_walk * 4, hipMemcpyDeviceToHost));
    if (log_out->tri) HIP_K(hipMemcpy(log_out->tri, d_lt, n_walk * 4, hipMemcpyDeviceToHost));
    if (log_out->bary) HIP_K(hipMemcpy(log_out->bary, d_lb, n_walk * 8, hipMemcpyDeviceToHost));
    if (log_out->queries) HIP_K(hipMemcpy(log_out->queries, d_lq, n_walk * 4, hipMemcpyDeviceToHost));
  }
  std::vector<unsigned long long> rq((size_t)n), tq((size_t)n);
  unsigned long long kq = 0, nonf = 0;
  HIP_K(hipMemcpy(rq.data(), d_rq, n * 8, hipMemcpyDeviceToHost));
  HIP_K(hipMemcpy(tq.data(), d_tq, n * 8, hipMemcpyDeviceToHost));
  HIP_K(hipMemcpy(&kq, d_kq, 8, hipMemcpyDeviceToHost));
  HIP_K(hipMemcpy(&nonf, d_nonf, 8, hipMemcpyDeviceToHost));
  std::vector<int32_t> ls((size_t)n_walk);
  HIP_K(hipMemcpy(ls.data(), d_ls, n_walk * 4, hipMemcpyDeviceToHost));
  float t_tan = 0, t_walk = 0;
  HIP_K(hipEventElapsedTime(&t_tan, ev[0], ev[1]));
  HIP_K(hipEventElapsedTime(&t_walk, ev[1], ev[2]));
  msk_kelvin_est_info I;
  std::memset(&I, 0, sizeof(I));
  I.n_rows = n;
  I.K = K_;
  I.pairs = pairs;
  I.kill_walks = kill_walks;
  I.dropped_rows = dropped;
  I.walks_total = (n - dropped) * 2 * pairs + kill_walks;
  for (int64_t i = 0; i < n; ++i) I.queries_total += (int64_t)(rq[i] + tq[i]);
  I.kill_queries = (int64_t)kq;
  I.queries_total += I.kill_queries;
  for (int64_t w = 0; w < n_walk; ++w) I.capped_total += ls[w] == kCapped ? 1 : 0;
  I.mean_radius = n > dropped ? rsum / (double)(n - dropped) : 0.0;
  I.r_max = r_max;
  I.tangent_ms = t_tan;
  I.walk_kernel_ms = t_walk;
  I.product_ms = prod_ms_total;
  I.nonfinite_entries = (int64_t)nonf;
  if (d_wstats) {
    unsigned long long w3[3];
    HIP_K(hipMemcpy(w3, d_wstats, sizeof(w3), hipMemcpyDeviceToHost));
    I.nodes_visited = (int64_t)w3[0];
    I.elements_tested = (int64_t)w3[1];
    I.fp64_ops = (int64_t)w3[2];
  }
  if (info) *info = I;
#undef HIP_K
  cleanup(MSK_OK);
  if (I.nonfinite_entries > 0) return fail(ctx, MSK_ERR_NUMERIC, "non-finite entries in the estimate");
  return MSK_OK;
}

// ------------------------------------------------------------- autotune

extern "C" void msk_tune_space_default(msk_tune_space* sp) {
  if (!sp) return;
  std::memset(sp, 0, sizeof(*sp));
  sp->n_leaf = 3;
  sp->leaf[0] = 2; sp->leaf[1] = 4; sp->leaf[2] = 8;
  sp->n_chunk = 3;
  sp->chunk[0] = 32; sp->chunk[1] = 64; sp->chunk[2] = 128;
  sp->n_regen = 3;
  sp->regen_min[0] = 8; sp->regen_min[1] = 16; sp->regen_min[2] = 24;
  sp->n_bpc = 2;
  sp->blocks_per_cu[0] = 4; sp->blocks_per_cu[1] = 8;
  sp->trial_rows = 65536;
  sp->trial_walks = 256;
  sp->repeats = 2;
  sp->cache_path = nullptr;
}

extern "C" msk_status msk_mesh_rebuild(msk_ctx* ctx, msk_mesh* m, int32_t leaf) {
  if (!ctx || !m) return MSK_ERR_INVALID_ARG;
  if (leaf == m->leaf_size) return MSK_OK;
  HostBvh B;
  std::string e = build_bvh_host(m->vworld.data(), m->nv, m->faces.data(), m->nf, leaf, B);
  if (!e.empty()) return fail(ctx, MSK_ERR_INVALID_ARG, e);
  Node4* dn = nullptr;
  TriRec* dt = nullptr;
  int32_t* ds = nullptr;
  hipError_t he;
  if ((he = upload(ctx, &dn, B.nodes.data(), B.nodes.size())) != hipSuccess ||
      (he = upload(ctx, &dt, B.tris.data(), B.tris.size())) != hipSuccess ||
      (he = upload(ctx, &ds, B.slot_of_tri.data(), B.slot_of_tri.size())) != hipSuccess) {
    dfree(dn);
    dfree(dt);
    dfree(ds);
    return fail(ctx, MSK_ERR_DEVICE, std::string("rebuild upload: ") + hipGetErrorString(he));
  }
  dfree(m->d_nodes);
  dfree(m->d_tris);
  dfree(m->d_slot);
  m->d_nodes = dn;
  m->d_tris = dt;
  m->d_slot = ds;
  m->n_nodes = (int64_t)B.nodes.size();
  m->depth = B.depth;
  m->leaf_size = leaf;
  m->top_nodes = (int)std::min<int64_t>(kMaxTop, m->n_nodes);
  return MSK_OK;
}

// Cached tuning results are keyed by the walk kernels' revision (a hash of
// their sources, set by the build), the device's CU count and the workload's
// shape, so an edit of the kernels forces a new search.
#ifndef MSK_WALK_SRC_SHA
#define MSK_WALK_SRC_SHA "unversioned"
#endif
constexpr const char* kTuneKernel = MSK_WALK_SRC_SHA;

static std::string tune_signature(const msk_ctx* ctx, int32_t n, msk_mesh* const* meshes, const msk_rows* const* rows,
                                  int32_t side) {
  long long tris = 0, nr = 0;
  for (int32_t i = 0; i < n; ++i) {
    tris += meshes[i]->nf;
    nr += rows[i]->n;
  }
  char buf[200];
  std::snprintf(buf, sizeof(buf), "kernel=%s;cu=%d;meshes=%d;tris=%lld;rows=%lld;side=%d", kTuneKernel, ctx->n_cu,
                n, tris, nr, side);
  return buf;
}

extern "C" msk_status msk_autotune(msk_ctx* ctx, int32_t n, msk_mesh* const* meshes, const msk_rows* const* rows,
                                   const msk_basis* const* bases, const double* eps, const double* inset_h,
                                   int32_t side, const msk_tune_space* space, msk_tune_result* out) {
  if (!ctx || !out || n < 1 || !meshes || !rows || !bases || !eps || !inset_h) return MSK_ERR_INVALID_ARG;
  msk_tune_space sp;
  msk_tune_space_default(&sp);
  if (space) sp = *space;
  if (sp.trial_walks < 2 || sp.trial_rows < 1) return fail(ctx, MSK_ERR_INVALID_ARG, "bad trial size");
  for (int32_t i = 0; i < n; ++i) {
    msk_status st = check_problem(ctx, meshes[i], rows[i], bases[i], sp.trial_walks, eps[i], inset_h[i], side,
                                   nullptr);
    if (st != MSK_OK) return st;
  }
  std::memset(out, 0, sizeof(*out));
  out->leaf = meshes[0]->leaf_size;
  out->chunk = 64;
  out->regen_min = 1;
  out->blocks_per_cu = 8;
  const std::string sig = tune_signature(ctx, n, meshes, rows, side);
  if (sp.cache_path) {  // one JSON object per line: {"sig": "...", "leaf": L, ...}
    if (FILE* f = std::fopen(sp.cache_path, "r")) {
      char line[512];
      while (std::fgets(line, sizeof(line), f)) {
        const std::string l(line);
        if (l.find("\"sig\": \"" + sig + "\"") == std::string::npos) continue;
        int lf, ch, rg, bp;
        double wps;
        const char* q = std::strstr(line, "\"leaf\":");
        if (q && std::sscanf(q, "\"leaf\": %d, \"chunk\": %d, \"regen_min\": %d, \"blocks_per_cu\": %d, "
                                "\"walks_per_s\": %lf", &lf, &ch, &rg, &bp, &wps) == 5) {
          out->leaf = lf;
          out->chunk = ch;
          out->regen_min = rg;
          out->blocks_per_cu = bp;
          out->walks_per_s = wps;
          out->from_cache = 1;
        }
      }
      std::fclose(f);
      if (out->from_cache) {
        for (int32_t i = 0; i < n; ++i) {
          msk_status st = msk_mesh_rebuild(ctx, meshes[i], out->leaf);
          if (st != MSK_OK) return st;
        }
        return MSK_OK;
      }
    }
  }
  // trial buffers (kept for the whole search; trial sums are not read)
  std::vector<msk_dtn*> dtns;
  auto free_all = [&]() {
    for (msk_dtn* d : dtns) {
      dtn_free(d);
      delete d;
    }
  };
  msk_dtn_opts o;
  msk_dtn_opts_default(&o);
  for (int32_t i = 0; i < n; ++i) {
    msk_dtn* d = nullptr;
    msk_status st = alloc_dtn(ctx, rows[i], bases[i], sp.trial_walks, false, &d);
    if (st != MSK_OK) {
      free_all();
      return st;
    }
    dtns.push_back(d);
    hipError_t he;
    if ((he = launch_fill_u64(d->d_acc1, d->n * d->K, 0, ctx->stream)) != hipSuccess ||
        (he = launch_fill_u64(d->d_acc2, d->n * d->K, 0, ctx->stream)) != hipSuccess ||
        (he = launch_fill_u64(d->d_q, d->n, 0, ctx->stream)) != hipSuccess ||
        (he = launch_fill_u64(d->d_esc, d->n, 0, ctx->stream)) != hipSuccess ||
        (he = launch_fill_u64(d->d_cap, d->n, 0, ctx->stream)) != hipSuccess ||
        (he = launch_fill_u32(d->d_disc, d->n, 0u, ctx->stream)) != hipSuccess) {
      free_all();
      return fail(ctx, MSK_ERR_DEVICE, std::string("tune buffers: ") + hipGetErrorString(he));
    }
  }
  // sampled rows: evenly spaced in each mesh's Z-order, proportional to its rows
  int64_t total_rows = 0;
  for (int32_t i = 0; i < n; ++i) total_rows += rows[i]->n;
  std::vector<RowSlot> slots;
  for (int32_t i = 0; i < n; ++i) {
    const int64_t ni = rows[i]->n;
    const int64_t k = std::max<int64_t>(1, std::min<int64_t>(ni, (sp.trial_rows * ni + total_rows - 1) / total_rows));
    for (int64_t j = 0; j < k; ++j) slots.push_back(RowSlot{i, rows[i]->order[(size_t)(j * ni / k)], 0u});
  }
  int trials = 0;
  auto evaluate = [&](int leaf, int chunk, int regen, int bpc, double* wps) -> msk_status {
    for (int32_t i = 0; i < n; ++i) {
      msk_status st = msk_mesh_rebuild(ctx, meshes[i], leaf);
      if (st != MSK_OK) return st;
    }
    std::vector<MeshDev> mds;
    for (int32_t i = 0; i < n; ++i) mds.push_back(make_meshdev(meshes[i], rows[i], bases[i], dtns[i], eps[i],
                                                               inset_h[i], side, o, i));
    msk_dtn_opts oc = o;
    oc.chunk = chunk;
    oc.regen_min = regen;
    oc.blocks_per_cu = bpc;
    const int use_lds = (n == 1 && meshes[0]->top_nodes > 0) ? 1 : 0;
    double best = 1e300;
    for (int r = 0; r < std::max(1, sp.repeats); ++r) {
      double ms = 0;
      int64_t st3[3] = {0, 0, 0};
      msk_status st = run_walks(ctx, mds, slots, sp.trial_walks, 0, oc, use_lds, meshes[0]->top_nodes, &ms, st3);
      if (st != MSK_OK) return st;
      best = std::min(best, ms);
      ++trials;
    }
    *wps = (double)slots.size() * (double)sp.trial_walks / (best * 1e-3);
    return MSK_OK;
  };
  double wps = 0, best_wps = 0;
  msk_status st = evaluate(out->leaf, out->chunk, out->regen_min, out->blocks_per_cu, &wps);  // warm-up
  if (st != MSK_OK) {
    free_all();
    return st;
  }
  best_wps = 0;
  auto scan = [&](int dim, int cnt, const int32_t* vals) -> msk_status {
    for (int j = 0; j < cnt; ++j) {
      int lf = out->leaf, ch = out->chunk, rg = out->regen_min, bp = out->blocks_per_cu;
      int* v = dim == 0 ? &lf : dim == 1 ? &ch : dim == 2 ? &rg : &bp;
      *v = vals[j];
      if (lf < 1 || lf > 8 || ch < 1 || rg < 1 || rg > 64 || bp < 1 || bp > 32) continue;
      double w2 = 0;
      msk_status s2 = evaluate(lf, ch, rg, bp, &w2);
      if (s2 != MSK_OK) return s2;
      if (w2 > best_wps) {
        best_wps = w2;
        out->leaf = lf;
        out->chunk = ch;
        out->regen_min = rg;
        out->blocks_per_cu = bp;
      }
    }
    return MSK_OK;
  };
  if ((st = scan(0, std::min(4, sp.n_leaf), sp.leaf)) != MSK_OK ||
      (st = scan(1, std::min(4, sp.n_chunk), sp.chunk)) != MSK_OK ||
      (st = scan(2, std::min(4, sp.n_regen), sp.regen_min)) != MSK_OK ||
      (st = scan(3, std::min(4, sp.n_bpc), sp.blocks_per_cu)) != MSK_OK) {
    free_all();
    return st;
  }
  free_all();
  for (int32_t i = 0; i < n; ++i) {
    msk_status s2 = msk_mesh_rebuild(ctx, meshes[i], out->leaf);
    if (s2 != MSK_OK) return s2;
  }
  out->walks_per_s = best_wps;
  out->trials = trials;
  if (sp.cache_path) {
    if (FILE* f = std::fopen(sp.cache_path, "a")) {
      std::fprintf(f, "{\"sig\": \"%s\", \"leaf\": %d, \"chunk\": %d, \"regen_min\": %d, \"blocks_per_cu\": %d, "
                      "\"walks_per_s\": %.6g}\n", sig.c_str(), out->leaf, out->chunk, out->regen_min,
                   out->blocks_per_cu, best_wps);
      std::fclose(f);
    }
  }
  return MSK_OK;
}

// ------------------------------------------------------- mesh Laplacian basis

extern "C" void msk_laplace_opts_default(msk_laplace_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->degree = 0;
  o->max_iters = 60;
  o->max_degree = 4000;
  o->tol = 1e-12;
}

namespace {

// 30-bit Morton code of a point in the box [lo, lo + ext]
uint32_t morton30(const float* p, const double lo[3], const double ext[3]) {
  uint32_t code = 0;
  uint32_t q[3];
  for (int a = 0; a < 3; ++a) {
    double t = ext[a] > 0 ? (p[a] - lo[a]) / ext[a] : 0.0;
    t = std::min(std::max(t, 0.0), 1.0);
    q[a] = std::min<uint32_t>(1023u, (uint32_t)(t * 1024.0));
  }
  for (int bit = 9; bit >= 0; --bit)
    for (int a = 0; a < 3; ++a) code = (code << 1) | ((q[a] >> bit) & 1u);
  return code;
}

}  // namespace

extern "C" msk_status msk_basis_create_laplacian(msk_ctx* ctx, const float* V, int64_t nv, const int32_t* F,
                                                 int64_t nf, int32_t K, const msk_laplace_opts* opts, double* evals,
                                                 double* phi, msk_laplace_info* info, msk_basis** out) {
  if (!ctx || !out) return MSK_ERR_INVALID_ARG;
  *out = nullptr;
  if (!V || !F || !evals) return fail(ctx, MSK_ERR_INVALID_ARG, "null V, F or evals");
  if (nv < 3 || nv >= INT32_MAX || nf < 1 || nf >= INT32_MAX / 3)
    return fail(ctx, MSK_ERR_INVALID_ARG, "need 3 <= nv < 2^31 and 1 <= nf < 2^31 / 3");
  msk_laplace_opts o;
  msk_laplace_opts_default(&o);
  if (opts) {
    o = *opts;
    if (o.max_iters == 0) o.max_iters = 60;
    if (o.max_degree == 0) o.max_degree = 4000;
    if (o.tol == 0) o.tol = 1e-12;
  }
  if (K < 1 || K + 16 > 512) return fail(ctx, MSK_ERR_INVALID_ARG, "K must be in 1..496");
  if ((int64_t)nv * K >= INT32_MAX) return fail(ctx, MSK_ERR_INVALID_ARG, "nv * K must be below 2^31");
  int64_t m = o.block;
  if (m == 0) m = ((K + std::max(32, K / 4)) + 63) / 64 * 64;
  if (m > 512) m = 512;
  if (m % 64 != 0 || m < 64 || m < K + 16)
    return fail(ctx, MSK_ERR_INVALID_ARG, "block must be a multiple of 64 in [64, 512] and at least K + 16");
  if (o.degree < 0 || o.degree > 100000 || o.max_degree < 8 || o.max_degree > 100000 || o.max_iters < 0 ||
      !(o.tol > 0) || !std::isfinite(o.tol))
    return fail(ctx, MSK_ERR_INVALID_ARG, "need 0 <= degree, 8 <= max_degree <= 1e5, max_iters >= 0, tol > 0");
  for (int64_t i = 0; i < 3 * nv; ++i)
    if (!std::isfinite(V[i])) return fail(ctx, MSK_ERR_INVALID_ARG, "non-finite vertex coordinate");
  for (int64_t i = 0; i < 3 * nf; ++i)
    if (F[i] < 0 || F[i] >= nv) return fail(ctx, MSK_ERR_INVALID_ARG, "face index out of range");

  // ---- host set-up: vertex order (Morton code of the position, then index),
  // faces in internal ids, vertex -> face incidence, sparsity pattern of L
  const auto t0 = std::chrono::steady_clock::now();
  double lo[3], hi[3], ext[3];
  for (int a = 0; a < 3; ++a) lo[a] = hi[a] = V[a];
  for (int64_t i = 0; i < nv; ++i)
    for (int a = 0; a < 3; ++a) {
      lo[a] = std::min(lo[a], (double)V[3 * i + a]);
      hi[a] = std::max(hi[a], (double)V[3 * i + a]);
    }
  for (int a = 0; a < 3; ++a) ext[a] = hi[a] - lo[a];
  std::vector<uint64_t> key(nv);
  for (int64_t i = 0; i < nv; ++i) key[i] = ((uint64_t)morton30(V + 3 * i, lo, ext) << 32) | (uint64_t)i;
  std::sort(key.begin(), key.end());
  std::vector<int32_t> orig(nv), inv(nv);
  for (int64_t i = 0; i < nv; ++i) {
    orig[i] = (int32_t)(key[i] & 0xffffffffu);
    inv[orig[i]] = (int32_t)i;
  }
  std::vector<float> P(3 * nv);
  for (int64_t i = 0; i < nv; ++i)
    for (int a = 0; a < 3; ++a) P[3 * i + a] = V[3 * (int64_t)orig[i] + a];
  std::vector<int32_t> Fi(3 * nf);
  std::vector<char> repeated(nf, 0);
  int64_t n_repeated = 0;
  for (int64_t t = 0; t < nf; ++t) {
    for (int c = 0; c < 3; ++c) Fi[3 * t + c] = inv[F[3 * t + c]];
    if (F[3 * t] == F[3 * t + 1] || F[3 * t + 1] == F[3 * t + 2] || F[3 * t] == F[3 * t + 2]) {
      repeated[t] = 1;
      ++n_repeated;
    }
  }
  std::vector<int32_t> vt_ptr(nv + 1, 0);
  for (int64_t t = 0; t < nf; ++t)
    if (!repeated[t])
      for (int c = 0; c < 3; ++c) ++vt_ptr[Fi[3 * t + c] + 1];
  for (int64_t i = 0; i < nv; ++i) vt_ptr[i + 1] += vt_ptr[i];
  std::vector<int32_t> vt_tri(std::max<int32_t>(1, vt_ptr[nv]));
  {
    std::vector<int32_t> fillp(vt_ptr.begin(), vt_ptr.end() - 1);
    for (int64_t t = 0; t < nf; ++t)
      if (!repeated[t])
        for (int c = 0; c < 3; ++c) vt_tri[fillp[Fi[3 * t + c]]++] = (int32_t)t;
  }
  std::vector<int32_t> rowptr(nv + 1, 0), col;
  col.reserve((size_t)vt_ptr[nv] + nv);
  {
    std::vector<int32_t> nb;
    for (int64_t i = 0; i < nv; ++i) {
      nb.clear();
      nb.push_back((int32_t)i);
      for (int32_t q = vt_ptr[i]; q < vt_ptr[i + 1]; ++q)
        for (int c = 0; c < 3; ++c) nb.push_back(Fi[3 * (int64_t)vt_tri[q] + c]);
      std::sort(nb.begin(), nb.end());
      nb.erase(std::unique(nb.begin(), nb.end()), nb.end());
      if ((int64_t)col.size() + (int64_t)nb.size() >= INT32_MAX)
        return fail(ctx, MSK_ERR_INVALID_ARG, "too many Laplacian entries (2^31)");
      col.insert(col.end(), nb.begin(), nb.end());
      rowptr[i + 1] = (int32_t)col.size();
    }
  }
  const int64_t nnz = (int64_t)col.size();
  const double setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();

  // ---- device buffers
  LaplaceJob J;
  J.stream = ctx->stream;
  J.n = nv;
  J.m = m;
  J.K = K;
  J.nnz = (int64_t)col.size();
  J.lock = o.no_locking ? 0 : 1;
  J.degree = o.degree;
  J.max_degree = o.max_degree;
  J.max_iters = o.max_iters;
  J.tol = o.tol;
  J.seed = o.seed;
  const int64_t slices = std::max<int64_t>(1, std::min<int64_t>(256, (nv + 255) / 256));
  J.n_slots = 4 * slices;
  float* d_P = nullptr;
  int32_t *d_F = nullptr, *d_vtp = nullptr, *d_vtt = nullptr, *d_rp = nullptr, *d_col = nullptr, *d_orig = nullptr;
  double *d_val = nullptr, *d_mass = nullptr, *d_s = nullptr, *d_slots = nullptr, *d_small = nullptr,
         *d_part = nullptr, *d_phi = nullptr;
  double* d_blk[3] = {nullptr, nullptr, nullptr};
  unsigned long long* d_cnt = nullptr;
  msk_basis* b = new msk_basis();
  b->ctx = ctx;
  b->nv = nv;
  b->K = K;
  b->max_row_nnz = K;
  auto free_all = [&]() {
    dfree(d_P);
    dfree(d_F);
    dfree(d_vtp);
    dfree(d_vtt);
    dfree(d_rp);
    dfree(d_col);
    dfree(d_orig);
    dfree(d_val);
    dfree(d_mass);
    dfree(d_s);
    dfree(d_slots);
    dfree(d_small);
    dfree(d_part);
    dfree(d_phi);
    for (double*& p : d_blk) dfree(p);
    dfree(d_cnt);
  };
  hipError_t he = hipSuccess;
  const int64_t nblk = psd_blocks(m);
  if ((he = upload(ctx, &d_P, P.data(), P.size())) != hipSuccess ||
      (he = upload(ctx, &d_F, Fi.data(), Fi.size())) != hipSuccess ||
      (he = upload(ctx, &d_vtp, vt_ptr.data(), vt_ptr.size())) != hipSuccess ||
      (he = upload(ctx, &d_vtt, vt_tri.data(), vt_tri.size())) != hipSuccess ||
      (he = upload(ctx, &d_rp, rowptr.data(), rowptr.size())) != hipSuccess ||
      (he = upload(ctx, &d_col, col.data(), col.size())) != hipSuccess ||
      (he = upload(ctx, &d_orig, orig.data(), orig.size())) != hipSuccess ||
      (he = dalloc(&d_val, (size_t)nnz)) != hipSuccess || (he = dalloc(&d_mass, (size_t)nv)) != hipSuccess ||
      (he = dalloc(&d_s, (size_t)nv)) != hipSuccess ||
      (he = dalloc(&d_slots, (size_t)(J.n_slots * nblk * 4096))) != hipSuccess ||
      (he = dalloc(&d_small, (size_t)std::max<int64_t>(m * m, 4096))) != hipSuccess ||
      (he = dalloc(&d_part, (size_t)1024 * K)) != hipSuccess ||
      (phi && (he = dalloc(&d_phi, (size_t)(nv * K))) != hipSuccess) ||
      (he = dalloc(&d_blk[0], (size_t)(nv * m))) != hipSuccess ||
      (he = dalloc(&d_blk[1], (size_t)(nv * m))) != hipSuccess ||
      (he = dalloc(&d_blk[2], (size_t)(nv * m))) != hipSuccess || (he = dalloc(&d_cnt, 2)) != hipSuccess ||
      (he = dalloc(&b->d_rowptr, (size_t)nv + 1)) != hipSuccess ||
      (he = dalloc(&b->d_col, (size_t)(nv * K))) != hipSuccess ||
      (he = dalloc(&b->d_val, (size_t)(nv * K))) != hipSuccess) {
    free_all();
    msk_basis_destroy(b);
    return fail(ctx, he == hipErrorOutOfMemory ? MSK_ERR_OOM : MSK_ERR_DEVICE,
                std::string("Laplacian basis buffers: ") + hipGetErrorString(he));
  }
  J.P = d_P;
  J.F = d_F;
  J.vt_ptr = d_vtp;
  J.vt_tri = d_vtt;
  J.rowptr = d_rp;
  J.col = d_col;
  J.orig = d_orig;
  J.val = d_val;
  J.mass = d_mass;
  J.s = d_s;
  J.counters = d_cnt;
  for (int i = 0; i < 3; ++i) J.blk[i] = d_blk[i];
  J.slots = d_slots;
  J.small = d_small;
  J.part = d_part;
  J.evals = evals;
  J.phi = d_phi;
  J.out_rowptr = b->d_rowptr;
  J.out_col = b->d_col;
  J.out_val = b->d_val;
  J.info.skipped_faces = n_repeated;
  std::string err;
  const int rc = laplace_basis_device(J, err);
  if (rc == 0 || rc == 4) {
    if (phi && (he = hipMemcpyAsync(phi, d_phi, sizeof(double) * nv * K, hipMemcpyDeviceToHost, ctx->stream)) ==
                   hipSuccess)
      he = hipStreamSynchronize(ctx->stream);
    if (he != hipSuccess) {
      free_all();
      msk_basis_destroy(b);
      return fail(ctx, MSK_ERR_DEVICE, std::string("eigenvector copy: ") + hipGetErrorString(he));
    }
  }
  free_all();
  if (info) {
    std::memset(info, 0, sizeof(*info));
    info->active_vertices = J.info.active_vertices;
    info->skipped_faces = J.info.skipped_faces;
    info->nnz = nnz;
    info->spmm_calls = J.info.spmm_calls;
    info->block = (int32_t)m;
    info->degree = J.info.last_degree;
    info->iters = J.info.iters;
    info->converged = J.info.converged;
    info->grams = J.info.grams;
    info->rotates = J.info.rotates;
    info->rank_drops = J.info.rank_drops;
    info->locked = J.info.locked;
    info->filter_bytes = J.info.filter_bytes;
    info->bound = J.info.bound;
    info->filter_lower = J.info.filter_lower;
    info->max_residual = J.info.max_residual;
    info->setup_ms = setup_ms;
    info->assemble_ms = J.info.assemble_ms;
    info->filter_ms = J.info.filter_ms;
    info->dense_ms = J.info.dense_ms;
    info->total_ms = J.info.total_ms;
  }
  if (rc == 0 || rc == 4) {
    *out = b;
    return rc == 0 ? MSK_OK
                   : fail(ctx, MSK_ERR_NOT_CONVERGED,
                          "Laplacian basis: residual target not met" + (err.empty() ? std::string() : ": " + err));
  }
  msk_basis_destroy(b);
  const msk_status st = rc == 1 ? MSK_ERR_INVALID_ARG : (rc == 5 ? MSK_ERR_NUMERIC : MSK_ERR_DEVICE);
  return fail(ctx, st, "Laplacian basis: " + err);
}

// ------------------------------------------------- Steklov heat and signatures

extern "C" msk_status msk_spectral_heat(msk_ctx* ctx, const msk_basis* b, int32_t n_modes, const double* evals,
                                        const double* coeffs, const double* times, int32_t n_times,
                                        const double* mass, const double* u0, double* hks, double* heat) {
  if (!ctx) return MSK_ERR_INVALID_ARG;
  if (!b || !evals || !coeffs || !times) return fail(ctx, MSK_ERR_INVALID_ARG, "null basis, evals, coeffs or times");
  if (b->knn_mesh || !b->d_rowptr) return fail(ctx, MSK_ERR_INVALID_ARG, "a table basis is required");
  if (!hks && !heat) return fail(ctx, MSK_ERR_INVALID_ARG, "no output requested");
  if (heat && (!mass || !u0)) return fail(ctx, MSK_ERR_INVALID_ARG, "heat needs mass and u0");
  const int64_t K = b->K, nv = b->nv;
  if (n_modes < 1 || n_modes > 512 || n_modes > K) return fail(ctx, MSK_ERR_INVALID_ARG, "n_modes outside 1..min(512, K)");
  if (n_times < 1 || n_times > 4096) return fail(ctx, MSK_ERR_INVALID_ARG, "n_times outside 1..4096");
  for (int32_t k = 0; k < n_modes; ++k)
    if (!std::isfinite(evals[k])) return fail(ctx, MSK_ERR_INVALID_ARG, "non-finite eigenvalue");
  for (int64_t i = 0; i < K * n_modes; ++i)
    if (!std::isfinite(coeffs[i])) return fail(ctx, MSK_ERR_INVALID_ARG, "non-finite coefficient");
  for (int32_t t = 0; t < n_times; ++t)
    if (!std::isfinite(times[t]) || times[t] < 0) return fail(ctx, MSK_ERR_INVALID_ARG, "times must be finite and >= 0");
  std::vector<double> mu0;
  if (heat) {
    mu0.resize(nv);
    for (int64_t v = 0; v < nv; ++v) {
      if (!std::isfinite(mass[v]) || !std::isfinite(u0[v])) return fail(ctx, MSK_ERR_INVALID_ARG, "non-finite mass or u0");
      mu0[v] = mass[v] * u0[v];
    }
  }
  std::vector<double> E((size_t)n_modes * n_times);
  for (int32_t k = 0; k < n_modes; ++k)
    for (int32_t t = 0; t < n_times; ++t) E[(size_t)k * n_times + t] = std::exp(-evals[k] * times[t]);
  const int32_t pgrid = (int32_t)std::max<int64_t>(1, std::min<int64_t>((nv + 3) / 4, 1024));
  double *d_C = nullptr, *d_W = nullptr, *d_out = nullptr, *d_mu0 = nullptr, *d_part = nullptr;
  auto free_all = [&]() {
    dfree(d_C);
    dfree(d_W);
    dfree(d_out);
    dfree(d_mu0);
    dfree(d_part);
  };
  hipError_t he;
  if ((he = upload(ctx, &d_C, coeffs, (size_t)(K * n_modes))) != hipSuccess ||
      (he = dalloc(&d_W, E.size())) != hipSuccess || (he = dalloc(&d_out, (size_t)(nv * n_times))) != hipSuccess ||
      (heat && (he = upload(ctx, &d_mu0, mu0.data(), mu0.size())) != hipSuccess) ||
      (heat && (he = dalloc(&d_part, (size_t)pgrid * n_modes)) != hipSuccess)) {
    free_all();
    return fail(ctx, he == hipErrorOutOfMemory ? MSK_ERR_OOM : MSK_ERR_DEVICE,
                std::string("spectral buffers: ") + hipGetErrorString(he));
  }
  auto run_fields = [&](const std::vector<double>& Wh, int32_t square, double* dst) -> hipError_t {
    hipError_t e = hipMemcpyAsync(d_W, Wh.data(), sizeof(double) * Wh.size(), hipMemcpyHostToDevice, ctx->stream);
    if (e != hipSuccess) return e;
    e = launch_spectral_fields(b->d_rowptr, b->d_col, b->d_val, nv, d_C, n_modes, d_W, n_times, square, d_out,
                               ctx->stream);
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(dst, d_out, sizeof(double) * nv * n_times, hipMemcpyDeviceToHost, ctx->stream);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(ctx->stream);
  };
  if (hks && (he = run_fields(E, 1, hks)) != hipSuccess) {
    free_all();
    return fail(ctx, MSK_ERR_DEVICE, std::string("heat kernel signature: ") + hipGetErrorString(he));
  }
  if (heat) {
    std::vector<double> part((size_t)pgrid * n_modes), a(n_modes, 0.0);
    if ((he = launch_spectral_coeff(b->d_rowptr, b->d_col, b->d_val, nv, d_C, n_modes, d_mu0, pgrid, d_part,
                                    ctx->stream)) != hipSuccess ||
        (he = hipMemcpyAsync(part.data(), d_part, sizeof(double) * part.size(), hipMemcpyDeviceToHost,
                             ctx->stream)) != hipSuccess ||
        (he = hipStreamSynchronize(ctx->stream)) != hipSuccess) {
      free_all();
      return fail(ctx, MSK_ERR_DEVICE, std::string("heat coefficients: ") + hipGetErrorString(he));
    }
    for (int32_t g = 0; g < pgrid; ++g)
      for (int32_t k = 0; k < n_modes; ++k) a[k] += part[(size_t)g * n_modes + k];
    std::vector<double> Wh(E);
    for (int32_t k = 0; k < n_modes; ++k)
      for (int32_t t = 0; t < n_times; ++t) Wh[(size_t)k * n_times + t] *= a[k];
    if ((he = run_fields(Wh, 0, heat)) != hipSuccess) {
      free_all();
      return fail(ctx, MSK_ERR_DEVICE, std::string("Steklov heat: ") + hipGetErrorString(he));
    }
  }
  free_all();
  return MSK_OK;
}
