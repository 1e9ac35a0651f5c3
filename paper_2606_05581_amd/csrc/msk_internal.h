// Internal layouts shared by the host code and the HIP kernels of libmsk.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

namespace msk {

// 4-wide BVH node, one 128-byte line. Child k's box is
// [lo{x,y,z}[k], hi{x,y,z}[k]]; child[k] >= 0 is an inner node index,
// child[k] < 0 a leaf holding triangle slots [-child[k]-1, -child[k]-1+count[k]).
// An unused slot has an empty box (lo = +inf, hi = -inf) and count 0.
struct alignas(128) Node4 {
  float lox[4], loy[4], loz[4];
  float hix[4], hiy[4], hiz[4];
  int32_t child[4];
  int32_t count[4];
};
static_assert(sizeof(Node4) == 128, "node must be one 128-byte line");

// Triangle in BVH leaf order: vertices as float offsets from the scene
// centre; a.w holds the original triangle index (bit pattern of an int32).
struct alignas(16) TriRec {
  float4 a, b, c;
};
static_assert(sizeof(TriRec) == 48, "triangle record must be 48 bytes");

constexpr int kStackDepth = 64;     // traversal stack entries per lane
constexpr int kMaxTableNnz = 32;    // basis entries per vertex
constexpr int kMaxTop = 85;         // BVH nodes a workgroup may keep in LDS (3 levels)

// Host-side BVH build result.
struct HostBvh {
  double centre[3];
  double radius;
  double area;
  std::vector<Node4> nodes;
  std::vector<TriRec> tris;
  std::vector<int32_t> slot_of_tri;  // original triangle -> leaf-order slot
  int depth = 0;                     // levels of 4-wide nodes
  int leaf_size = 4;
};

// Builds the scene frame and a 4-wide BVH over float offsets from the
// centre. Returns an empty string on success, else an error message.
std::string build_bvh_host(const float* V, int64_t nv, const int32_t* F, int64_t nf, int leaf_size, HostBvh& out);

// The same binned-SAH build and 4-wide collapse over any elements given by
// their boxes and centroids (n x 3 floats): the nodes in breadth-first order
// and the element order of the leaf slots.
struct Box3f {
  float lo[3], hi[3];
};
std::string build_bvh_boxes(const std::vector<Box3f>& boxes, const std::vector<float>& cen, int leaf_size,
                            std::vector<Node4>& nodes_out, std::vector<int32_t>& leaf_order, int& depth);

// ------------------------------------------------------------ kernel ABI

enum RowMode : int32_t { kRowsPoint = 0, kRowsHatRing = 1 };
enum WalkStatus : int32_t { kHit = 0, kEscaped = 1, kCapped = 2 };

// Everything a walk needs about one mesh (device pointers).
// Point basis (point-based k-NN interpolator): the k nearest sample points
// of a query, found on a uniform grid, with bilateral weights. k = 0: the
// basis is the per-vertex table instead.
constexpr int kMaxKnn = 16;
struct KnnDev {
  const float4* pts;          // scene-frame positions (w unused)
  const float4* nrm;          // unit normals (w unused)
  const int32_t* cell_start;  // n_cells + 1 offsets into cell_pts
  const int32_t* cell_pts;    // point indices, by cell
  float lo[3];                // grid origin (scene frame)
  float cell;                 // cell edge
  int32_t dim[3];
  int32_t k;
  double inv2s2;              // 1 / (2 sigma^2)
  double inv_tau;             // 1 / tau_n
};

struct MeshDev {
  const Node4* nodes;
  const TriRec* tris;
  const int32_t* slot_of_tri;  // original face -> slot
  const int32_t* faces;        // original faces (n_tris x 3)
  int64_t n_tris;
  int32_t n_top;               // nodes of this mesh that may be read from LDS
  int32_t mode;                // RowMode
  float radius;                // bounding-sphere radius (float)
  double radius_d;
  float eps2;                  // eps^2
  float inset;                 // h (walk geometry)
  double inset_d;              // h (scaling of the estimate)
  float kappa;                 // relative step shrink
  float delta;                 // absolute step shrink (delta_rel * radius)
  float slack;                 // absolute error allowance of the FP32 distance
  int32_t side;                // 0 interior, 1 exterior
  int32_t mesh_id;             // low 24 bits of the fourth Philox counter word
  int32_t walks_per_row;       // W
  int64_t max_steps;
  // rows (original order)
  const float* p;              // point rows: scene-frame float positions (n x 3)
  const float* n;              // point rows: unit normals (n x 3)
  const int32_t* tri;          // point rows: face
  const float* bary;           // point rows: barycentrics (n x 3)
  const int32_t* ring_ptr;     // hat rows
  const int32_t* ring_tri;
  const double* ring_cum;
  const float* face_normals;
  const int32_t* discarded;    // per row (point rows)
  const float* ball_r;         // PSD estimator: per-row tangent-ball radius (0 = dropped); null otherwise
  double ball_u0;              // PSD estimator: sin(theta0 / 2) of the cap left out about s
  // basis table
  const int32_t* b_rowptr;
  const int32_t* b_col;
  const float* b_val;
  int64_t K;
  KnnDev knn;                  // point basis (knn.k > 0) instead of the table
  // accumulators (original row order)
  double* acc1;                // point rows: sum b(t); hat rows: sum c
  double* acc2;                // point rows: sum b(t)^2; hat rows: sum c^2
  unsigned long long* row_queries;
  unsigned long long* row_escaped;
  unsigned long long* row_capped;
  // optional walk log, (row, walk) -> row * W + walk - walk_offset
  int32_t* log_status;
  int32_t* log_tri;
  float* log_bary;
  int32_t* log_queries;
};

// A unit of queued work: one row of one mesh; walk ids are slot * W + w.
struct RowSlot {
  int32_t mesh;
  int32_t row;
  uint32_t walk0;  // the slot's first walk, after the launch's walk_offset
};

struct WalkLaunch {
  const MeshDev* meshes;       // device array
  const RowSlot* slots;        // device array, n_slots
  int64_t n_slots;
  int64_t walks_per_slot;      // W
  int64_t walk_offset;         // first walk index
  uint32_t seed_lo, seed_hi;
  // persistent form: 8 queues over contiguous slot ranges
  unsigned long long* queue_next;  // 8 counters (walk ids)
  const unsigned long long* queue_end;  // 8 bounds
  int32_t chunk;
  int32_t regen_min;
  int32_t use_lds_top;         // single-mesh launch: stage mesh 0's top nodes in LDS
  int32_t n_top;
  unsigned long long* stats;   // optional: [nodes visited, triangles tested, FP32 operations]
  int32_t accum;               // persistent form, wavefront row-table partial sums:
                               // 0 FP64, 1 FP32, 2 compensated FP32 (double-float pairs)
  int32_t knn;                 // some mesh uses the point basis: launch the k-NN instantiations
};

// One mesh's point rows in a discard pass over the rows of several meshes.
struct RowRange {
  int64_t first;         // launch index of the mesh's row 0 (ascending over the ranges)
  int32_t mesh;          // index into the launch's MeshDev array
  int32_t* discarded;    // the mesh's discard flags (written)
};

// The per-row counters of one estimate, summed by launch_row_totals.
struct RowCounters {
  const unsigned long long* queries;
  const unsigned long long* escaped;
  const unsigned long long* capped;
  const int32_t* discarded;
  const int64_t* walks;
  const unsigned long long* nonfinite;  // one count
  int64_t n;
};

}  // namespace msk

namespace msk {
// kernel launch wrappers (walk.hip)
hipError_t launch_walk_plain(const WalkLaunch& L, hipStream_t s);
hipError_t launch_walk_persistent(const WalkLaunch& L, int grid, hipStream_t s);
struct QueueInit {
  unsigned long long begin[8], end[8];
};
hipError_t launch_count_nonfinite(const double* a, int64_t n, unsigned long long* count, hipStream_t s);
hipError_t launch_init_queues(unsigned long long* next, unsigned long long* end, const QueueInit& q, hipStream_t s);
hipError_t launch_fill_u64(void* p, int64_t n, unsigned long long v, hipStream_t s);
hipError_t launch_fill_u32(void* p, int64_t n, uint32_t v, hipStream_t s);
hipError_t launch_tangent_ball(const MeshDev& M, int64_t n_rows, float r_max, int32_t iters, float tol, float* radius,
                               hipStream_t s);
hipError_t launch_discard(const MeshDev& M, int64_t n_rows, int32_t* discarded, hipStream_t s);
hipError_t launch_discard_batch(const MeshDev* meshes, const RowRange* ranges, int32_t n_ranges, int64_t n_total,
                                hipStream_t s);
// out: 6 x n_sets counts (queries, escaped, capped, discarded rows, walks of kept rows, non-finite entries)
hipError_t launch_row_totals(const RowCounters* sets, int32_t n_sets, unsigned long long* out, hipStream_t s);
hipError_t launch_knn_eval(const KnnDev& G, const double* c, const float* Q, const float* Nq, int64_t n, int32_t* idx,
                           float* w, hipStream_t s);
hipError_t launch_closest_points(const Node4* nodes, const TriRec* tris, float radius, const double* c, const float* Q,
                                 int64_t nq, int32_t* tri, float* d2, float* bary, hipStream_t s);
hipError_t launch_finalize(const MeshDev& M, int64_t n_rows, const int64_t* walks, const double* w, double* S,
                           double* se, hipStream_t s, int32_t jump_only = 0);

// Blocked symmetric products shared by the PSD estimator and the mesh basis
// (psd.hip):
int64_t psd_blocks(int64_t Kp);
// Partial 64 x 64 upper blocks of A^T A (A: m x Kp row-major) into P: slices x 4 slots of psd_blocks(Kp) blocks
hipError_t launch_psd_syrk(const double* A, int64_t m, int64_t Kp, int64_t slices, double* P, hipStream_t s);
hipError_t launch_psd_reduce(const double* P, int64_t n_slots, int64_t K, int64_t Kp, double* C, hipStream_t s);

// Fixed workspace of the allocation-free estimate (noalloc.hip): 64 MiB per
// device. noalloc_scratch_init looks its address up on `device` (which must
// be current) once; noalloc_scratch returns it (nullptr if the lookup failed
// or was not made, with the HIP error in *err).
constexpr size_t kNoallocScratchBytes = size_t(64) << 20;
hipError_t noalloc_scratch_init(int device);
void* noalloc_scratch(int device, hipError_t* err);

}  // namespace msk
