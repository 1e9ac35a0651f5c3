/*
 * msk.h -- C ABI of the MI355X Monte Carlo Steklov (DtN) walk library.
 *
 * The library estimates the discrete Dirichlet-to-Neumann (Steklov) operator
 * of a triangle mesh with the naive finite-difference estimator of
 * "Monte Carlo Steklov Operators for Large-Scale Geometry Processing in the
 * Wild" (arXiv 2606.05581), Sec. 3.1, Alg. 1: for every boundary row i, W
 * Walk-on-Spheres walks start at an inset point x = s -/+ h n_s, stop in an
 * eps-shell of the surface (Sec. 2, "Walk-on-Spheres") at t, and add
 * c = b(s) - b(t) to row i (eqs. finite-difference-estimator,
 * naive-stiffness-matrix), b being barycentric interpolation of a per-vertex
 * basis table (Sec. 3.4). Both the interior operator and the exterior one
 * (Sec. 3.3, "Escape to Infinity": a walk hits the surface or escapes) are
 * estimated. The smallest Steklov eigenpairs (Sec. 2, eq.
 * steklov-eigenproblem) are read off the symmetrised estimate (Alg. 1, last
 * step).
 *
 * Conventions common to every entry point:
 *   - Every function returns msk_status; nothing throws across the ABI. On
 *     failure the context keeps a message readable with msk_last_error().
 *   - "host" pointers are ordinary CPU memory; "device" pointers are HIP
 *     device memory of the context's device (e.g. a torch CUDA tensor's
 *     data_ptr()). Host inputs are copied before the call returns; device
 *     pointers are borrowed for the duration of the call only.
 *   - Arrays are dense and row-major; float = IEEE binary32, double = binary64.
 *   - All GPU work runs in order on the context's stream (the stream handed
 *     to msk_create, or the null stream). Calls are synchronous: results are
 *     complete when they return.
 *   - Handles (msk_mesh, msk_rows, msk_basis, msk_dtn) belong to the context
 *     that created them and must be destroyed before it.
 */
#ifndef MSK_H
#define MSK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MSK_OK = 0,
  MSK_ERR_INVALID_ARG = 1, /* bad pointer, size, index, NaN/Inf input ...   */
  MSK_ERR_OOM = 2,         /* device or host allocation failed               */
  MSK_ERR_DEVICE = 3,      /* a HIP call failed; the message carries its text */
  MSK_ERR_NOT_CONVERGED = 4, /* eigen step: partial results are returned     */
  MSK_ERR_NUMERIC = 5      /* a non-finite value was produced                */
} msk_status;

typedef struct msk_ctx msk_ctx;
typedef struct msk_mesh msk_mesh;
typedef struct msk_rows msk_rows;
typedef struct msk_basis msk_basis;
typedef struct msk_dtn msk_dtn;

/* ---------------------------------------------------------------- context */

/* Create a context on HIP device `device`. `hip_stream` is a hipStream_t (or
 * NULL for the null stream) on which all work of this context is queued; the
 * caller keeps ownership of it. */
msk_status msk_create(int device, void* hip_stream, msk_ctx** out);
void msk_destroy(msk_ctx* ctx);
/* Message of the last failed call on this context ("" if none). The string
 * stays valid until the next call on the context. */
const char* msk_last_error(const msk_ctx* ctx);

/* ------------------------------------------------------------------- mesh */

typedef struct {
  int32_t leaf_size; /* triangles per BVH leaf, 1..8 (default 4)            */
  int32_t top_nodes; /* top BVH nodes the persistent kernel may stage in LDS,
                        0..85 (default 85; the kernel stages at most 21)  */
} msk_bvh_opts;

typedef struct {
  double centre[3];  /* scene frame: centre of the FP64 bounding box         */
  double radius;     /* bounding-sphere radius about centre, (1+2^-20) max|v-c| */
  double area;       /* total surface area (FP64)                            */
  int64_t n_verts, n_tris, n_nodes;
  int64_t node_bytes, tri_bytes;
  int32_t depth, leaf_size;
} msk_mesh_info;

/* Build the walk geometry of a triangle mesh (Sec. 4: every triangle is an
 * absorbing boundary element; soups, overlaps and non-manifold parts are
 * accepted as they are, Appendix A).
 *   V: host, n_verts x 3 float, world coordinates.
 *   F: host, n_tris x 3 int32 vertex indices (an unindexed soup is the case
 *      F = [[0,1,2],[3,4,5],...]).
 * Coordinates are re-expressed as float offsets from the bounding-box centre
 * (computed in FP64). A 4-wide BVH (binned surface-area heuristic) is built
 * on the host and uploaded. Errors: INVALID_ARG for NaN/Inf coordinates,
 * out-of-range indices, n_tris < 1 or >= 2^26, or zero total area; zero-area triangles
 * are kept (they still absorb walks). Free with msk_mesh_destroy. */
msk_status msk_build_bvh(msk_ctx* ctx, const float* V, int64_t n_verts, const int32_t* F, int64_t n_tris,
                         const msk_bvh_opts* opts /* NULL = defaults */, msk_mesh** out);
msk_status msk_mesh_get_info(const msk_mesh* mesh, msk_mesh_info* info);
void msk_mesh_destroy(msk_mesh* mesh);

/* Exact nearest triangle of each query point (Sec. 2, "Walk-on-Spheres": the
 * empty-ball radius and the nearest boundary point). The decision is taken in
 * single precision: queries are re-expressed as float offsets from the scene
 * centre, the squared distance to every triangle follows one fixed FP32
 * closest-point evaluation, and the answer is the minimum of (squared
 * distance, original triangle index) in lexicographic order -- the same
 * triangle a brute-force FP32 scan returns.
 *   Q:    device, nq x 3 float, world coordinates.
 *   tri:  device, nq int32, original triangle index (row of F).
 *   d2:   device, nq float, squared distance.
 *   bary: device, nq x 2 float, barycentric weights of the triangle's second
 *         and third vertex at the closest point (first = 1 - sum). */
msk_status msk_closest_points(msk_ctx* ctx, const msk_mesh* mesh, const float* Q, int64_t nq, int32_t* tri,
                              float* d2, float* bary);

/* -------------------------------------------------------- rows and basis */

typedef enum {
  MSK_ROWS_POINT = 0,   /* row i = fixed boundary sample s_i (Alg. 1's s)     */
  MSK_ROWS_HAT_RING = 1 /* row i = vertex i; each walk draws s ~ phi_i / A_i  */
} msk_rows_mode;

/* Boundary rows of an estimate. All pointers are host memory.
 * MSK_ROWS_POINT: p (n_rows x 3 float, world), n (n_rows x 3 float, unit
 *   outward normal), tri (n_rows int32 face index), bary (n_rows x 3 float,
 *   barycentrics of p in that face).
 * MSK_ROWS_HAT_RING (n_rows = number of vertices): ring_ptr (n_rows+1
 *   int32), ring_tri (ring_ptr[n_rows] int32, faces around each vertex),
 *   ring_cum (same length, double, running sum of face areas within each
 *   ring), face_normals (n_tris x 3 float, unit outward).
 * w: n_rows double quadrature weight of each row (|dOmega|/N for point rows,
 *   the one-ring area / 3 for hat rows). */
typedef struct {
  int32_t mode;
  int64_t n_rows;
  const double* w;
  const float* p;
  const float* n;
  const int32_t* tri;
  const float* bary;
  const int32_t* ring_ptr;
  const int32_t* ring_tri;
  const double* ring_cum;
  const float* face_normals;
} msk_rows_desc;

/* Copy rows to the device, expressed in the mesh's scene frame, and order
 * them along a Z-order curve of the sample positions (Sec. 4). Errors:
 * INVALID_ARG for inconsistent sizes, bad face / vertex indices, non-finite
 * values or negative weights. */
msk_status msk_rows_create(msk_ctx* ctx, const msk_mesh* mesh, const msk_rows_desc* desc, msk_rows** out);
void msk_rows_destroy(msk_rows* rows);

/* Per-vertex basis table in CSR form (host): vertex v holds columns
 * col[rowptr[v] .. rowptr[v+1]) with values val[...], columns strictly
 * increasing within a vertex, 0 <= col < K. The walk estimators
 * (msk_estimate_dtn and its batched forms) take at most 32 entries per
 * vertex; the PSD estimator takes any (it uses a dense copy).
 * b(p) for p with barycentrics l on face (a,b,c) is
 * l_a table[a] + l_b table[b] + l_c table[c] (Sec. 3.4). */
msk_status msk_basis_create(msk_ctx* ctx, const int32_t* rowptr, const int32_t* col, const float* val,
                            int64_t n_verts, int64_t K, msk_basis** out);

/* Point basis (Appendix, point-based k-NN interpolator) for point rows of
 * `mesh`: column j is sample point x_j with unit normal n_j (host, n_points
 * x 3 floats each, world coordinates; normals are normalised here). At a
 * query q with normal n_q the basis values are the bilateral weights of its
 * k nearest points (Euclidean distance, ties by index),
 *   w_j = exp(-|q - x_j|^2 / (2 sigma^2)) exp(-(1 - n_q . n_j) / tau_n),
 * normalised over the k (equal shares if all underflow); the other columns
 * are 0. The estimators evaluate it at the sample s (its row's normal) and at
 * each walk's hit point (the hit triangle's face normal), so K = n_points.
 * The points are binned in a uniform grid of the scene frame (cells of about
 * two sample spacings, sqrt(mesh area / n_points)); a query searches rings
 * of cells until the k-th distance is inside the searched block.
 * Errors: INVALID_ARG for k outside 1..16, n_points < k, sigma or tau_n
 * <= 0, non-finite points or zero normals. Used with other meshes, hat rows,
 * the PSD estimator or collect_stats it is rejected (INVALID_ARG). */
msk_status msk_basis_create_knn(msk_ctx* ctx, const msk_mesh* mesh, const float* points, const float* normals,
                                int64_t n_points, int32_t k, double sigma, double tau_n, msk_basis** out);

/* The point basis at n queries (device arrays: Q and Nq n x 3 floats, world
 * positions and normals; out: idx n x k int32 point indices, nearest first,
 * and w n x k float weights). Errors: INVALID_ARG for a table basis. */
msk_status msk_basis_eval_knn(msk_ctx* ctx, const msk_basis* basis, const float* Q, const float* Nq, int64_t n,
                              int32_t* idx, float* w);
void msk_basis_destroy(msk_basis* basis);

/* Mesh-based Galerkin basis (Sec. 5.1, mesh-based Galerkin basis): the K
 * lowest eigenmodes of the mesh's cotangent Laplacian, computed on the GPU.
 * Stiffness L: each triangle adds, for each corner of angle theta opposite
 * the edge (i, j), -cot(theta)/2 to L_ij and L_ji and +cot(theta)/2 to L_ii
 * and L_jj; mass M = diag(m), m_i = a third of the area of the triangles at
 * i. A triangle is left out of both when twice its area is at most 1e-12
 * times its longest squared edge; vertices of zero mass get basis value 0.
 * The basis is the K smallest pairs of L phi = lambda M phi with
 * Phi^T M Phi = I, by Chebyshev-filtered subspace iteration on
 * A = M^-1/2 L M^-1/2 (FP64 throughout). */
typedef struct {
  int32_t block;      /* subspace size, a multiple of 64 in [64, 512]; 0 = K + max(32, K/4)
                         rounded up to 64                                    */
  int32_t degree;     /* Chebyshev filter degree per iteration; 0 = adaptive:
                         the degree that amplifies the K-th Ritz value about
                         1000 times relative to the damped interval          */
  int32_t max_iters;  /* outer iterations (0 = 60)                           */
  int32_t max_degree; /* cap of the adaptive degree (0 = 4000)               */
  double tol;         /* stop when ||A x - lambda x|| <= tol * b for every wanted
                         pair (|x| = 1, b = the Gershgorin bound of A); 0 = 1e-12 */
  uint64_t seed;      /* start block                                        */
  int32_t no_locking; /* 1: filter every column in every iteration (default 0:
                         leading columns whose pairs meet the target, in
                         multiples of 64, are left out of the filter)       */
  int32_t reserved;
} msk_laplace_opts;

typedef struct {
  int64_t active_vertices; /* vertices of positive mass                      */
  int64_t skipped_faces;   /* degenerate faces left out (incl. repeated ids) */
  int64_t nnz;             /* stored entries of L                            */
  int64_t spmm_calls;      /* sparse block products                          */
  int32_t block, degree, iters, converged; /* degree: the last filter's      */
  int32_t grams, rotates, rank_drops, locked; /* locked: columns left out of the
                                                 last filter                */
  double bound;            /* b, the Gershgorin bound of A                   */
  double filter_lower;     /* lower end of the last damped interval          */
  double max_residual;     /* max over the K pairs of ||A x - lambda x|| / b  */
  double setup_ms;         /* host: vertex order, incidence and pattern      */
  double assemble_ms;      /* device: L, M, A and b                          */
  double filter_ms;        /* device: the filter's sparse products           */
  double dense_ms;         /* orthonormalisation and Rayleigh-Ritz           */
  double total_ms;         /* device work from assembly to the basis table   */
  double filter_bytes;     /* algorithmic bytes moved by the filter steps:
                              per step the gathered columns, the previous and
                              the new ones, 8 bytes each per vertex, plus 12
                              bytes per entry of L and 4 per row            */
} msk_laplace_info;

void msk_laplace_opts_default(msk_laplace_opts* opts);

/* V: nv x 3 floats, F: nf x 3 vertex indices (host; copied). Writes the K
 * eigenvalues ascending to evals (host), optionally the eigenvectors to phi
 * (host, nv x K row-major, FP64; NULL to skip) and the run's figures to
 * info (NULL to skip), and returns a dense table basis (K columns per
 * vertex, FP32 values) for msk_estimate_psd in *out, to be freed with
 * msk_basis_destroy. Errors: INVALID_ARG for non-finite positions,
 * out-of-range indices, K < 1, K + 16 > 512, nv * K >= 2^31, a block that
 * is not a multiple of 64 in [64, 512] or smaller than K + 16, or fewer
 * vertices of positive mass than K; NUMERIC when the operator is zero or not
 * finite; NOT_CONVERGED when the residual target was not met within
 * max_iters (*out, evals, phi and info then hold the last iterate and must
 * still be freed). */
msk_status msk_basis_create_laplacian(msk_ctx* ctx, const float* V, int64_t nv, const int32_t* F, int64_t nf,
                                      int32_t K, const msk_laplace_opts* opts, double* evals, double* phi,
                                      msk_laplace_info* info, msk_basis** out);

/* Steklov heat and heat kernel signatures (Sec. 5, eqs. steklovHeat and
 * spectralSteklovHeat) on the vertices, from n_modes Steklov eigenpairs
 * expressed in a table basis (for an M-orthonormal basis, the eigenpairs of
 * the symmetrised K x K estimate of msk_estimate_psd):
 *   psi_k(v) = sum_j Phi_vj coeffs[j][k]   (Phi: the basis table at vertex v),
 *   hks[v][t]  = sum_k exp(-evals[k] times[t]) psi_k(v)^2,
 *   heat[v][t] = sum_k exp(-evals[k] times[t]) a_k psi_k(v),
 *                a_k = sum_v mass[v] u0[v] psi_k(v).
 * Host arrays: evals (n_modes), coeffs (K x n_modes row-major, K = the
 * basis's width), times (n_times, >= 0), mass and u0 (n_verts; needed for
 * heat), outputs hks and heat (n_verts x n_times row-major; either may be
 * NULL, not both). FP64 arithmetic on the FP32 table values. Errors:
 * INVALID_ARG for a point basis, n_modes outside 1..min(512, K), n_times
 * outside 1..4096, or non-finite inputs. */
msk_status msk_spectral_heat(msk_ctx* ctx, const msk_basis* basis, int32_t n_modes, const double* evals,
                             const double* coeffs, const double* times, int32_t n_times, const double* mass,
                             const double* u0, double* hks, double* heat);

/* -------------------------------------------------------------- estimate */

typedef enum { MSK_INTERIOR = 0, MSK_EXTERIOR = 1 } msk_side;
typedef enum { MSK_FORM_PERSISTENT = 0, MSK_FORM_PLAIN = 1 } msk_form;

typedef struct {
  uint64_t seed;       /* Philox key (default 0)                               */
  int64_t max_steps;   /* walk step cap; 0 = 1024 interior / 8192 exterior     */
  int64_t walk_offset; /* index of the first walk (resume / split runs)        */
  double kappa;        /* step radius r = d (1 - kappa) - delta_rel * R       */
  double delta_rel;    /*   (defaults 2^-20 and 2^-21)                         */
  int32_t form;        /* msk_form (default persistent)                        */
  int32_t block;       /* threads per workgroup (default 256)                  */
  int32_t blocks_per_cu; /* persistent grid size / 256 CUs (default 8)         */
  int32_t chunk;       /* walks a wavefront takes from the queue at once (64)  */
  int32_t regen_min;   /* persistent form: a wavefront records ended walks and
                          takes new ones once this many of its 64 lanes are
                          idle (16)                                          */
  int32_t record_log;  /* keep a per-walk log (status, triangle, bary, queries) */
  double se_target;    /* > 0: adaptive walks per row (see msk_estimate_dtn)   */
  int64_t walks_max;   /* adaptive cap (default 65536)                         */
  int32_t collect_stats; /* count BVH nodes visited / triangles tested / FP32
                            operations (a separately compiled, slower kernel) */
  int32_t mesh_id;       /* single-mesh estimates: the mesh index in the Philox
                            counter (a batch uses each mesh's position)       */
  int32_t accum;         /* persistent form, partial row sums of a chunk of
                            walks kept in LDS: 0 = FP64, 1 = FP32 (plain
                            blocked sums), 2 = compensated FP32 (a
                            double-float pair per slot, TwoSum updates);
                            rows are always accumulated in FP64          */
  int32_t jump_only;     /* exterior, point rows: 1 drops the killing term of
                            the exterior form (Sec. 3.3, exterior
                            Beurling-Deny form; the paper's default exterior
                            operator, Sec. 4): an escaped walk contributes 0
                            instead of b(s), so constants are in the kernel */
} msk_dtn_opts;

void msk_dtn_opts_default(msk_dtn_opts* opts);

/* Smallest admissible shell width for a mesh of bounding radius `radius`
 * (msk_mesh_info.radius) under `opts` (NULL = defaults): every estimate
 * (msk_estimate_dtn, its batched forms, msk_estimate_psd) requires
 * eps > max(delta_rel R / (1 - kappa), 2^-18 R). Below the first term a walk
 * at distance d < eps would take the step d (1 - kappa) - delta_rel R <= 0 and
 * could cross the surface (Sec. 2: a WoS step stays inside the empty ball);
 * below the second the FP32 scene-frame distance no longer resolves the
 * shell. Host-only, no device work; NaN for radius <= 0, a non-finite radius
 * or kappa outside [0, 1). */
double msk_eps_floor(double radius, const msk_dtn_opts* opts);

/* Estimate the DtN rows of one mesh (Alg. 1 in row form).
 *   walks:  walks per row W (the first batch when se_target > 0);
 *   eps:    shell width: a walk stops once its squared distance < eps^2;
 *   inset_h: inset distance h of the start point;
 *   side:   MSK_INTERIOR (x = s - h n) or MSK_EXTERIOR (x = s + h n).
 * Row i of the result is S_i = w_i / (h W_i) sum_walks c, c = b(s) - b(t)
 * (t = the hit's closest point; b(t) = 0 for a walk that escaped), with the
 * standard error of every entry. Point rows whose inset point lies closer
 * than h/2 to the surface are discarded (zero row, flagged; Appendix A,
 * self-intersections). With se_target > 0 (exterior), walks are added in
 * rounds to every row whose escape-fraction standard error
 * sqrt(max(q(1-q), 1/W_i)/W_i) exceeds se_target: a multiple of `walks`, the
 * row's predicted deficit q(1-q)/se_target^2 - W_i rounded up (at least
 * `walks`, at most doubling W_i), up to walks_max; walk indices continue
 * the row's Philox walk counter.
 * Errors: INVALID_ARG for walks < 2, eps <= msk_eps_floor(R, opts),
 * inset_h <= eps, kappa outside [0, 1/2), delta_rel outside [0, 1/4), or rows /
 * basis built for a mesh with a different vertex count. Any K is accepted
 * (K == n_rows is needed only by msk_steklov_modes). NUMERIC when an entry
 * of S or se is NaN or infinite (e.g. basis values beyond the FP32 range of
 * the accumulation): *out is still set, holds the estimate as computed and
 * must be destroyed; info.nonfinite_entries counts the entries. Free the
 * result with msk_dtn_destroy. */
msk_status msk_estimate_dtn(msk_ctx* ctx, const msk_mesh* mesh, const msk_rows* rows, const msk_basis* basis,
                            int64_t walks, double eps, double inset_h, int32_t side, const msk_dtn_opts* opts,
                            msk_dtn** out);

/* Many meshes in one persistent launch captured as a HIP graph: the walks of
 * all meshes share one work queue ordered largest-mesh-first. meshes, rows,
 * bases, eps, inset_h and out are arrays of n_meshes entries; each result is
 * the same as msk_estimate_dtn on that mesh with the mesh's index in the
 * Philox counter. se_target must be 0. NUMERIC as for msk_estimate_dtn:
 * every out[i] is then set. */
msk_status msk_estimate_dtn_batched(msk_ctx* ctx, int32_t n_meshes, const msk_mesh* const* meshes,
                                    const msk_rows* const* rows, const msk_basis* const* bases,
                                    const double* eps, const double* inset_h, int64_t walks, int32_t side,
                                    const msk_dtn_opts* opts, msk_dtn** out);

/* A reusable batch: the same meshes, rows and bases estimated again and
 * again (serving). Creation allocates every mesh's outputs, orders the work
 * (meshes largest first, rows in Z-order, split over eight per-XCD queues)
 * and captures HIP graphs of the zeroing and discard pass, of ONE persistent
 * walk launch over all meshes, and of the finalisation; msk_batch_run
 * replays them back to back on the context's stream; it returns NUMERIC
 * (results still readable) when any member holds non-finite entries.
 * Arguments as for msk_estimate_dtn_batched; the handles must outlive the
 * batch. Results of the last run are read with msk_batch_dtn (views owned by
 * the batch, valid until msk_batch_destroy). */
typedef struct msk_batch msk_batch;
msk_status msk_batch_create(msk_ctx* ctx, int32_t n_meshes, const msk_mesh* const* meshes,
                            const msk_rows* const* rows, const msk_basis* const* bases, const double* eps,
                            const double* inset_h, int64_t walks, int32_t side, const msk_dtn_opts* opts,
                            msk_batch** out);
msk_status msk_batch_run(msk_batch* batch);
msk_status msk_batch_dtn(const msk_batch* batch, int32_t i, const msk_dtn** out);
void msk_batch_destroy(msk_batch* batch);

typedef struct {
  int64_t n_rows, K;
  int64_t walks_total, queries_total, escaped_total, capped_total, discarded_rows;
  double walk_kernel_ms; /* summed duration of the walk kernel launches      */
  double total_ms;       /* estimate call, first launch to last completion   */
  int32_t walk_launches;
  int64_t nodes_visited; /* with opts.collect_stats: BVH nodes read by walks */
  int64_t tris_tested;   /* with opts.collect_stats: triangle distance tests */
  int64_t valu_flops;    /* with opts.collect_stats: FP32 operations of those */
  int64_t nonfinite_entries; /* NaN or infinite entries of S and se; when
                                nonzero the call returned MSK_ERR_NUMERIC */
} msk_dtn_info;

msk_status msk_dtn_get_info(const msk_dtn* dtn, msk_dtn_info* info);
/* Totals of a batch's last run over all its meshes (walk_kernel_ms = the one
 * walk launch inside the graph; total_ms = the whole graph). */
msk_status msk_batch_get_info(const msk_batch* batch, msk_dtn_info* info);

/* msk_estimate_dtn for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same walks and the same S and se as msk_estimate_dtn with
 * these arguments, written to caller-provided device arrays, with no device
 * allocation and no allocating library call. The accumulators, row counters
 * and launch tables live in a fixed workspace compiled into the library: 64
 * MiB per device (MSK_NOALLOC_WORKSPACE_BYTES), held by every device the
 * library runs on until the process ends; about 16 n_rows K + 64 n_rows
 * bytes are needed, so e.g. 2,000 rows x 2,000 columns fit. Every call on a
 * device shares that device's workspace and clears what it uses first; calls
 * that overlap on one device (other host threads, other streams) race and
 * must be serialised by the caller.
 *   S, se: device, n_rows x K doubles each (row i = the rows' original i).
 *   info:  optional host copy of the counters (walk_kernel_ms and total_ms
 *          are not measured: 0).
 * Errors: as msk_estimate_dtn; INVALID_ARG also when the workspace is too
 * small for n_rows x K, when S or se is NULL, or for se_target > 0,
 * record_log or collect_stats (not available here); DEVICE when the
 * workspace's address could not be looked up at msk_create. */
#define MSK_NOALLOC_WORKSPACE_BYTES (64ull << 20)
msk_status msk_estimate_dtn_noalloc(msk_ctx* ctx, const msk_mesh* mesh, const msk_rows* rows, const msk_basis* basis,
                                    int64_t walks, double eps, double inset_h, int32_t side,
                                    const msk_dtn_opts* opts, double* S, double* se, msk_dtn_info* info);

typedef enum {
  MSK_FIELD_S = 0,          /* n_rows x K double, the estimate             */
  MSK_FIELD_SE = 1,         /* n_rows x K double, standard errors          */
  MSK_FIELD_ROW_WALKS = 2,  /* n_rows int64                                */
  MSK_FIELD_ROW_QUERIES = 3,/* n_rows int64, closest-point queries         */
  MSK_FIELD_ROW_ESCAPED = 4,/* n_rows int64                                */
  MSK_FIELD_ROW_CAPPED = 5, /* n_rows int64                                */
  MSK_FIELD_ROW_DISCARDED = 6, /* n_rows int32 (1 = discarded)             */
  MSK_FIELD_LOG_STATUS = 7, /* n_rows x W int32: 0 hit, 1 escaped, 2 capped */
  MSK_FIELD_LOG_TRI = 8,    /* n_rows x W int32, terminal triangle (-1)    */
  MSK_FIELD_LOG_BARY = 9,   /* n_rows x W x 2 float                        */
  MSK_FIELD_LOG_QUERIES = 10 /* n_rows x W int32                           */
} msk_field;

/* Copy one result field, rows in the caller's original row order, into dst
 * (host memory, or device memory if dst_on_device != 0). The walk log is
 * available only when opts.record_log was set (and se_target == 0). */
msk_status msk_dtn_get(const msk_dtn* dtn, int32_t field, void* dst, int32_t dst_on_device);
void msk_dtn_destroy(msk_dtn* dtn);

/* ------------------------------------------------------------- autotune */

/* Candidate values (n_x of them in x[]; n_x = 0 keeps the current value). */
typedef struct {
  int32_t n_leaf, leaf[4];            /* BVH leaf width                        */
  int32_t n_chunk, chunk[4];          /* walks a wavefront takes per queue grab */
  int32_t n_regen, regen_min[4];      /* waiting lanes that trigger bookkeeping */
  int32_t n_bpc, blocks_per_cu[4];    /* persistent workgroups per CU          */
  int64_t trial_rows;                 /* rows sampled over all meshes (65536)  */
  int64_t trial_walks;                /* walks per sampled row (256)           */
  int32_t repeats;                    /* timed repeats per candidate, min (2)  */
  const char* cache_path;             /* JSON-lines cache file, or NULL        */
} msk_tune_space;

typedef struct {
  int32_t leaf, chunk, regen_min, blocks_per_cu;
  double walks_per_s;                 /* best trial rate                       */
  int32_t trials;                     /* timed trial launches                  */
  int32_t from_cache;                 /* 1 if read from cache_path             */
} msk_tune_result;

void msk_tune_space_default(msk_tune_space* space);

/* Rebuild a mesh's BVH in place with another leaf width. Rows and bases made
 * for the mesh stay valid; batch plans that include the mesh do not (create
 * them after tuning). The nearest-triangle decision, hence every walk, does
 * not depend on the leaf width. */
msk_status msk_mesh_rebuild(msk_ctx* ctx, msk_mesh* mesh, int32_t leaf_size);

/* Autotune the persistent walk launch for a set of meshes (a batch, or one
 * mesh): coordinate search over leaf width, chunk, refill threshold and
 * workgroups per CU, each candidate timed on short walk launches over an
 * evenly spaced sample of rows of every mesh. The meshes are left rebuilt
 * with the best leaf width; the other values are returned for msk_dtn_opts.
 * With cache_path set, a result stored for the same workload signature
 * (mesh, triangle and row counts, side) is reused without timing. */
msk_status msk_autotune(msk_ctx* ctx, int32_t n_meshes, msk_mesh* const* meshes, const msk_rows* const* rows,
                        const msk_basis* const* bases, const double* eps, const double* inset_h, int32_t side,
                        const msk_tune_space* space, msk_tune_result* out);

/* --------------------------------------------------------- eigen step */

typedef struct {
  int32_t iterations;   /* block-Lanczos steps taken                      */
  int32_t block;        /* block size                                      */
  double max_residual;  /* max_j |C v_j - lambda_j v_j| / |C|_est          */
  double lanczos_ms;    /* the whole call (events)                          */
  /* dense products on the matrix cores: count, summed kernel time (events
   * around each) and algorithmic flops (2 M N K each); FP32 = the products
   * with C, FP64 = the basis products and the final Rayleigh quotients */
  int64_t fp32_products;
  double fp32_product_ms, fp32_product_flops;
  int64_t fp64_products;
  double fp64_product_ms, fp64_product_flops;
} msk_eig_stats;

/* Smallest k eigenpairs of the symmetrised, mass-scaled estimate
 * C = M^-1/2 (S + S^T)/2 M^-1/2, M = diag(w) over the rows that were not
 * discarded (Sec. 2, eq. steklov-eigenproblem; Alg. 1 symmetrisation),
 * by block Lanczos on the GPU: FP32 products with C on the matrix cores, FP64 full
 * re-orthogonalisation and Rayleigh quotients, the projected problem solved
 * in FP64 on the host. Requires K == n_rows.
 *   evals: host, k doubles, ascending.
 *   evecs: host, n_rows x k doubles (psi = M^-1/2 v, zero on discarded rows),
 *          or NULL.
 * Returns NOT_CONVERGED (with the best approximations written) if some
 * residual stays above max(1e-5, 16 sqrt(n) 2^-24) |C|_est (the floor set
 * by FP32 products with C), and NUMERIC without computing anything if the
 * estimate holds non-finite entries. */
msk_status msk_steklov_modes(msk_ctx* ctx, const msk_dtn* dtn, int32_t k, double* evals, double* evecs,
                             msk_eig_stats* stats);

/* ------------------------------------------ PSD estimator (Sec. 3.2, Alg. 2) */

typedef struct {
  double cap_deg;        /* cap about s left out of each tangent ball, as the
                            polar angle at the ball centre in degrees (2.5)    */
  int32_t bisect_iters;  /* tangent-ball bisection steps (10)                  */
  double r_max;          /* largest tangent radius; <= 0: half the shortest
                            side of the mesh's bounding box (Appendix A)       */
  int64_t chunk_pairs;   /* pairs per gathered chunk (262144); device memory of
                            the chunk buffers: 40 x chunk_pairs x K bytes (K
                            rounded up to 64), plus up to 512 MB of partial
                            sums of the products                             */
} msk_psd_opts;

void msk_psd_opts_default(msk_psd_opts* opts);

typedef struct {
  int64_t n_rows, K, pairs;
  int64_t walks_total;     /* walks run (2 x pairs per row with a tangent ball) */
  int64_t queries_total;   /* closest-point queries issued: the bisection's
                              bounded queries (up to 7 per round of three
                              levels) and the walks' queries                 */
  int64_t escaped_total, capped_total;
  int64_t dropped_rows;    /* rows without a tangent ball (radius 0)           */
  double mean_radius;      /* over rows with a tangent ball                    */
  double r_max;            /* the radius bound used                            */
  double tangent_ms;       /* table set-up and tangent-ball kernel             */
  double walk_kernel_ms;   /* the walk launch                                  */
  double gather_ms;        /* two-pass form: gathers of the update rows        */
  double product_ms;       /* the symmetric rank-k products (fused form: with
                              the gathers, in one kernel)                      */
  double total_ms;
  int64_t nonfinite_entries;
  int32_t fused;           /* 1: K <= 384, gathers and products in one kernel  */
  /* the walk launch's traversal work, counted when walk_opts->collect_stats
   * (a separately compiled counting kernel): box-node visits, triangle tests
   * and algorithmic FP32 operations; 0 otherwise                            */
  int64_t nodes_visited, tris_tested, valu_flops;
} msk_psd_info;

typedef struct {  /* optional host walk log, n_rows x 2 pairs entries each    */
  int32_t* status;  /* MSK walk status (0 hit, 1 escaped, 2 capped), -1 = not run */
  int32_t* tri;     /* terminal original triangle                           */
  float* bary;      /* its barycentrics of vertices 1 and 2 (2 per walk)     */
  int32_t* queries;
} msk_psd_log;

/* The paper's PSD estimate of the DtN stiffness matrix (Sec. 3.2, boxed
 * estimator and Alg. 2; eqs. beurling-deny-bilinear, strong-markov-property,
 * ball-jump-kernel, volume-jump-kernel) over point rows:
 *   - row i's sample s_i (its face, barycentrics and outward face normal)
 *     gets the largest inscribed tangent ball B_r(c), c = s - r n, by
 *     bisection (a radius is accepted when c's nearest surface point is at
 *     least r - min(eps/2, r/1024) away and the ball lies in the scene's
 *     bounding sphere; rows with no accepted radius are dropped);
 *   - `pairs` antithetic pairs of points z on the ball are drawn with density
 *     proportional to the ball jump kernel 1/(2 pi |s-z|^3) outside the cap
 *     (Philox counter (row, pair, 0, purpose 4 << 24 | mesh_id)); walk 2j+a
 *     of the row runs Walk-on-Spheres from the pair's point a with the step
 *     streams of that walk index, stopping in the eps-shell (interior);
 *   - each pair adds X = alpha_i (d_1 d_1^T + d_2 d_2^T)/2 with
 *     d = b(s_i) - b(t), alpha_i = w_i Z_i / (2 pairs), Z_i = (1/(2 r_i))
 *     (1/sin(cap/2) - 1) the kernel's mass outside the cap.
 * S = sum of X (K x K, symmetric PSD by construction) and se = its standard
 * error, the n_rows x pairs pair terms taken as independent draws:
 * se^2 = (n Q - S^2)/(n - 1), Q = sum of X*X elementwise. The sums are FP64:
 * the difference rows are gathered from a dense FP32 copy of the basis table
 * (promoted exactly to FP64) and multiplied on the matrix cores (FP64 MFMA,
 * symmetric rank-k blocks);
 * for K <= 384 both happen in one kernel with the rows kept in LDS.
 *   S, se:  host, K x K doubles (se may be NULL);
 *   radius: host, n_rows floats (tangent radii, 0 = dropped) or NULL;
 *   log:    optional host walk log; info: optional.
 * Ball points next to s lie within eps of the surface and their walks end at
 * once, so a coarse shell biases the estimate low (on a unit sphere eps =
 * 1e-3 gives about 1% less than eps <= 1e-4): use eps well below the
 * finite-difference estimator's inset (the paper runs at 1e-6; here eps
 * must exceed msk_eps_floor, 2^-18 R by default).
 * walk_opts: seed, max_steps, kappa, delta_rel, form, launch settings and
 * mesh_id as for msk_estimate_dtn (walk_offset, se_target and record_log
 * are ignored; collect_stats runs the counting kernel and fills the info's
 * traversal counts). Errors: INVALID_ARG for hat rows, pairs < 1,
 * K > 8192, eps <= msk_eps_floor(R, walk_opts), a basis for another vertex count or a flat mesh;
 * NUMERIC (outputs written) when an entry is not finite. */
msk_status msk_estimate_psd(msk_ctx* ctx, const msk_mesh* mesh, const msk_rows* rows, const msk_basis* basis,
                            int64_t pairs, double eps, const msk_dtn_opts* walk_opts, const msk_psd_opts* opts,
                            double* S, double* se, float* radius, const msk_psd_log* log, msk_psd_info* info);

/* ---------------------------------------- Kelvin-inverted exterior (f2) */

/* The exterior DtN form of Sec. 3.3 (eq. exterior-dtn-beurling-deny-form:
 * a jump term and a killing term) estimated in the image of the exterior
 * under the Kelvin transform x -> x / |x|^2 about a centre inside the shape
 * (Sec. 3.3, The Kelvin Transform; Appendix, Kelvin transform): a bounded
 * domain, bounded by the images of the triangles, each a piece of a sphere
 * through the origin cut by three circular arcs (Sec. 4: spherical
 * triangular elements with non-planar distance queries).
 * msk_kelvin_create copies the mesh's triangles relative to `centre` (world,
 * 3 doubles; it must lie inside the shape, off the surface) and builds a
 * 4-wide hierarchy over boxes that contain their images (leaf_size 1..8, 0 =
 * 1: one element per leaf, the fastest on MI355X since an element's exact
 * distance costs far more than a box test). Errors: INVALID_ARG for a centre
 * at a vertex or on the surface (nearer to a triangle than 1e-9 times its
 * largest vertex distance), or a non-finite centre. All geometry of this
 * path is FP64. */
typedef struct msk_kelvin msk_kelvin;
typedef struct {
  double centre[3];     /* inversion centre (world)                         */
  double radius;        /* bound of the inverted domain: max |x~| over its boundary */
  double box_lo[3], box_hi[3]; /* box of the inverted vertices               */
  double r_max;         /* default tangent-ball bound: half its shortest side */
  int64_t n_tris, n_nodes;
  int32_t depth, leaf_size;
} msk_kelvin_info;
msk_status msk_kelvin_create(msk_ctx* ctx, const msk_mesh* mesh, const double* centre, int32_t leaf_size,
                             msk_kelvin** out);
msk_status msk_kelvin_get_info(const msk_kelvin* kelvin, msk_kelvin_info* info);
void msk_kelvin_destroy(msk_kelvin* kelvin);

/* Exact nearest inverted element of each query point: lexicographic minimum
 * of (FP64 squared distance, original index).
 *   Q:    device, nq x 3 doubles, inverted space relative to the centre;
 *   tri:  device, nq int32 original triangle index;
 *   d2:   device, nq doubles, squared distance;
 *   qpt:  device, nq x 3 doubles, the nearest point (inverted space);
 *   bary: device, nq x 3 doubles, barycentrics of the nearest point's image
 *         in the original triangle. */
msk_status msk_kelvin_closest_points(msk_ctx* ctx, const msk_kelvin* kelvin, const double* Q, int64_t nq,
                                     int32_t* tri, double* d2, double* qpt, double* bary);

typedef struct {  /* optional host walk log, n_rows x 2 pairs jump walks then kill_walks */
  int32_t* status;  /* 0 hit, 2 capped, -1 not run (row without a tangent ball) */
  int32_t* tri;     /* terminal original triangle                           */
  float* bary;      /* barycentrics of its vertices 1 and 2 at the terminal point's image (2 per walk) */
  int32_t* queries;
} msk_kelvin_log;

typedef struct {
  int64_t n_rows, K, pairs, kill_walks;
  /* queries_total: nearest-element queries of the tangent-ball bisection
   * (bisect_iters per row), the jump walks and the killing walks;
   * kill_queries: those of the killing walks (part of queries_total) */
  int64_t walks_total, queries_total, kill_queries, dropped_rows, capped_total;
  double mean_radius, r_max;  /* inverted units                              */
  double tangent_ms, walk_kernel_ms, product_ms;
  int64_t nonfinite_entries;
  /* with walk_opts.collect_stats: the walks run in a counting build of the
   * walk kernel (same walks, not the timed one) whose nearest searches tally
   * their box-node visits, element tests and FP64 operations (additions,
   * multiplications, divisions and square roots, one each); else 0 */
  int64_t nodes_visited, elements_tested, fp64_ops;
} msk_kelvin_est_info;

/* The exterior estimate (Sec. 3.3, eq. main-exterior-estimator; Appendix,
 * exterior jump kernel and killing measure) over point rows of the mesh:
 *   - jump term: row i's sample s_i maps to s~_i = kappa(s_i - centre), with
 *     the unit normal n~_i = -(n - 2 (s^ . n) s^) pointing out of the
 *     inverted domain (n the outward normal); its tangent ball in the
 *     inverted domain (bisection as for msk_estimate_psd: bound opts.r_max,
 *     0 = half the shortest side of the inverted vertices' box; tolerance
 *     min(eps/2, r/1024)) gets `pairs` antithetic pairs of ball points drawn
 *     by the ball jump kernel outside the cap (Philox (row, pair, 0, purpose
 *     4 << 24 | mesh_id)); walk 2j + a runs Walk-on-Spheres in the inverted
 *     domain with the step streams of that walk index, ends at t~ in the
 *     eps-shell (inverted units) and adds, per pair,
 *       X_p = alpha_i (d_1 d_1^T / |t~_1| + d_2 d_2^T / |t~_2|) / 2,
 *       alpha_i = w_i |s~_i|^3 Z_i / (2 pairs), d = b(s_i) - b(kappa(t~)),
 *     Z_i = (1/(2 r_i)) (1/sin(cap/2) - 1) (eq. exterior-jump-kernel-final);
 *   - killing term: kill_walks walks (even) start at the origin of the
 *     inverted space (the image of infinity; Philox row 0xFFFFFFFF, walk k)
 *     and add (4 pi / |t~_0|) b(t_0) b(t_0)^T / kill_walks (eq.
 *     killing-measure-poisson-kernel).
 * The full exterior form is S_jump + S_kill; the paper's default drops the
 * killing term (Sec. 4). Standard errors: the pair terms (and the pairs of
 * killing walks) taken as independent draws, se^2 = (n Q - S^2)/(n - 1).
 *   S_jump, se_jump, S_kill, se_kill: host K x K doubles (se may be NULL;
 *     S_kill NULL only with kill_walks = 0);
 *   radius: host n_rows doubles (inverted tangent radii, 0 = dropped) or NULL;
 *   log, info: optional.
 * walk_opts: seed, max_steps (0 = 1024), kappa, delta_rel (the guard is
 * delta_rel times the inverted domain's bound), mesh_id, collect_stats (the
 * counting walk kernel; info's work tallies). Errors: INVALID_ARG
 * for rows of another mesh, hat rows, a point basis, K > 8192, pairs < 1, an
 * odd kill_walks, or eps at or below max(delta_rel R~ / (1 - kappa),
 * 2^-40 R~); NUMERIC when an entry is not finite (outputs written). */
msk_status msk_estimate_kelvin(msk_ctx* ctx, const msk_kelvin* kelvin, const msk_rows* rows, const msk_basis* basis,
                               int64_t pairs, int64_t kill_walks, double eps, const msk_dtn_opts* walk_opts,
                               const msk_psd_opts* opts, double* S_jump, double* se_jump, double* S_kill,
                               double* se_kill, double* radius, const msk_kelvin_log* log, msk_kelvin_est_info* info);

#ifdef __cplusplus
}
#endif
#endif /* MSK_H */
