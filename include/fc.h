/*
 * fc.h -- C ABI of libfactory_sdf.so: vertex-vs-SDF contact queries, contact
 * reduction and the penetration-penalty adjoint on AMD Instinct MI355X (gfx950).
 *
 * The problem (Narang et al., "Factory: Fast Contact for Robotic Assembly",
 * RSS 2022):
 *   - Section III-A: body B is a signed distance field sampled on a voxel
 *     grid and read with trilinear filtering; its value and gradient give a
 *     contact's distance and normal.
 *   - Section III-B: a contact is a point, a normal and a distance (7 floats)
 *     plus the two body indices.
 *   - Section III-C, Algorithm 1: for each shape pair, Generate candidate
 *     contacts for the mesh body queried against the SDF body, then reduce
 *     them: FindDeepest keeps the deepest candidate and BinReduce gathers the
 *     candidates of similar normal.  Here the patches are fixed
 *     normal-direction bins: per (environment, bin) the deepest candidate is
 *     kept, ties going to the lowest vertex index.
 *   - Appendix, Robot Learning Tools, "Using Contact Simulation Methods":
 *     when both bodies carry an SDF, the body with more triangles is the SDF
 *     and the other one's mesh is queried against it.  Here body A is always the queried mesh and
 *     body B the SDF.
 *
 * Conventions for every entry point:
 *   - Pointers named "device" are device memory owned by the caller; the
 *     library never frees them and keeps no reference past the call, except
 *     that a batch keeps the grid and mesh pointers given to fc_batch_create
 *     and reads them on every call (they must outlive the batch).
 *   - Pointers named "host" are read during the call only.
 *   - Every compute call is asynchronous on `stream` (a hipStream_t passed as
 *     void*; NULL = the default stream).  No compute call allocates, frees or
 *     synchronises.  fc_batch_create / fc_batch_set_launch / fc_graph_create
 *     allocate and synchronise (set-up calls).
 *   - Arguments are validated completely before anything is launched; on an
 *     error nothing is written and the status says why.  No call aborts,
 *     throws or prints.  FC_ERR_HIP carries the HIP error in
 *     fc_last_hip_error() (per thread).
 *   - Units are metres.  Poses place A in B's frame.  All outputs are in B's
 *     frame.
 */
#ifndef FACTORY_SDF_FC_H
#define FACTORY_SDF_FC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum fc_status {
  FC_OK = 0,
  FC_ERR_NULL = 1,        /* a required pointer is NULL */
  FC_ERR_SHAPE = 2,       /* a size or count is out of range or inconsistent */
  FC_ERR_DTYPE = 3,       /* unknown dtype or layout, or mixed within a batch */
  FC_ERR_RANGE = 4,       /* a numeric parameter is out of range (h, k, K) */
  FC_ERR_WORKSPACE = 5,   /* workspace NULL or smaller than fc_workspace_bytes */
  FC_ERR_HIP = 6,         /* a HIP runtime call failed; see fc_last_hip_error */
  FC_ERR_UNSUPPORTED = 7, /* valid request the library does not implement */
  FC_ERR_SCRATCH = 8      /* more scratch than fc_sdf_query_noalloc holds */
} fc_status;

typedef enum fc_dtype { FC_F32 = 0, FC_F16 = 1, FC_BF16 = 2 } fc_dtype;

/* FC_LAYOUT_LINEAR: samples [nz][ny][nx], x fastest.
 * FC_LAYOUT_BRICK:  the same samples re-laid out by fc_grid_to_bricks into
 *                   bricks of 4x4x4 nodes covering 3x3x3 cells (neighbouring
 *                   bricks duplicate their shared face nodes), so the 8
 *                   corners of any cell lie in one brick (FP32: 256 bytes,
 *                   FP16/BF16: one 128-byte line).
 * FC_LAYOUT_SLAB:   bricks of 4x4x2 nodes covering 3x3x1 cells (FP32: one
 *                   128-byte line per cell lookup).
 * FC_LAYOUT_SPARSE: the bricks of FC_LAYOUT_BRICK stored only near the
 *                   surface (Section VII: sparse SDFs to cut the memory
 *                   footprint), written by fc_grid_to_sparse.  One buffer:
 *                   a brick map (int32 per brick: slot in the pool, -1 = not
 *                   stored), the coarse grid of the brick-corner nodes
 *                   (node (3i, 3j, 3k) of the linear grid), and the pool of
 *                   stored bricks; sections start at 256-byte offsets.  A
 *                   cell in a stored brick reads its 8 corners as in
 *                   FC_LAYOUT_BRICK (same values, same bits of every
 *                   result); a cell in a brick that is not stored takes the
 *                   trilinear interpolant of the brick's 8 corner nodes
 *                   (spacing 3h) -- value and gradient of that coarse
 *                   interpolant, up to FP32 rounding.
 * Bricks are stored z-major, then y, then x; inside a brick x is fastest.
 * Values are copied, not rounded. */
typedef enum fc_layout {
  FC_LAYOUT_LINEAR = 0,
  FC_LAYOUT_BRICK = 1,
  FC_LAYOUT_SLAB = 2,
  FC_LAYOUT_SPARSE = 3
} fc_layout;

#define FC_MAX_TYPES 8 /* distinct grids and distinct meshes per batch */
#define FC_MAX_BINS 64 /* normal bins K */

/* Body B: a voxel SDF (Section III-A).  Node (i,j,k) sits at
 * origin + h*(i,j,k); values are node samples (node-centred, no half-voxel
 * offset).  A point is inside the grid iff 0 <= (x-origin)/h <= n-1 on every
 * axis; outside points are never candidates. */
typedef struct fc_grid {
  const void* data; /* device; fc_dtype samples; FP16/BF16 are IEEE half / bfloat16 bits */
  int32_t dtype;    /* fc_dtype */
  int32_t layout;   /* fc_layout */
  int32_t nx, ny, nz; /* nodes per axis, each >= 2, nx*ny*nz < 2^31 */
  float origin[3];  /* node (0,0,0), metres */
  float h;          /* node spacing, > 0, metres */
} fc_grid;

/* Body A: the queried mesh's vertices in A's frame, SoA (device), and
 * optionally its triangles for per-face queries (fc_sdf_query_faces):
 * tris = device [3][n_tris] vertex indices (corner a of every face, then b,
 * then c), NULL when n_tris = 0.  A face with an index outside
 * [0, n_verts) is never a candidate. */
typedef struct fc_mesh {
  const float* x;
  const float* y;
  const float* z;
  int32_t n_verts; /* >= 0 (an empty mesh gives empty contact lists) */
  const int32_t* tris;
  int32_t n_tris; /* >= 0 */
} fc_mesh;

/* Static description of a batch of independent environments (shape pairs).
 * Environment e pairs grid env_grid[e] with mesh env_mesh[e]; its query index
 * is q = qoff[e] + v for vertex v, qoff[e] = sum of n_verts over envs < e. */
typedef struct fc_batch_desc {
  int32_t n_env;            /* >= 1 */
  const fc_grid* grids;     /* host [n_grids], 1 <= n_grids <= FC_MAX_TYPES; one dtype and layout */
  int32_t n_grids;
  const fc_mesh* meshes;    /* host [n_meshes], 1 <= n_meshes <= FC_MAX_TYPES */
  int32_t n_meshes;
  const int32_t* env_grid;  /* host [n_env] in [0, n_grids), or NULL = all 0 */
  const int32_t* env_mesh;  /* host [n_env] in [0, n_meshes), or NULL = all 0 */
  int32_t n_bins;           /* K, 1 <= K <= FC_MAX_BINS */
  const float* bin_dirs;    /* host [3][K] unit directions d_k (copied) */
  float margin;             /* a query is a candidate iff phi < margin */
  const int32_t* env_order; /* host [n_env] permutation of 0..n_env-1, or NULL = 0..n_env-1:
                               the order in which environments are scheduled.  Callers pass a
                               spatial sort of their envs (e.g. by position in B's frame) so that
                               work running together reads the same part of the grid.  Contacts
                               do not depend on it; the shared vertex gradient sums envs in
                               this order. */
} fc_batch_desc;

typedef struct fc_batch fc_batch; /* opaque; owns device work tables */

/* Per-query candidates (Algorithm 1, Generate), all device, index q:
 *   phi[q]      trilinear SDF value at x_B, or +inf when x_B is outside the grid;
 *   normal      [3][Q]: grad(phi)/|grad(phi)|, (0,0,0) for a zero gradient or outside;
 *   bin[q]      argmax_k normal.d_k (lowest k on ties) when phi < margin, else -1;
 *   point       [3][Q] the query point in B's frame, per-face queries only
 *               (fc_sdf_query_faces: the descent's final point); ignored by
 *               the vertex calls, which may leave it NULL. */
typedef struct fc_candidates {
  float* phi;
  float* normal;
  int16_t* bin;
  float* point;
} fc_candidates;

/* Reduced contacts, one slot per (environment, bin), slot s = e*K + k (device).
 * Section III-B record: the point, normal and distance of the winner.
 *   vidx[s]   winning vertex index in env e's mesh, -1 if the bin is empty;
 *   depth[s]  -phi of the winner (+0.0 for -0.0), 0 if empty;
 *   point     [3][n_env*K] x_B of the winner, 0 if empty;
 *   normal    [3][n_env*K] unit normal of the winner, 0 if empty;
 *   count[e]  number of non-empty bins of env e. */
typedef struct fc_contacts {
  int32_t* vidx;
  float* depth;
  float* point;
  float* normal;
  int32_t* count;
} fc_contacts;

/* Penetration-penalty outputs (device; each pointer may be NULL = not wanted).
 *   loss[e]    L_e = sum over vertices with phi(x_B) < 0 of 0.5 k phi^2;
 *   d_pose     [6][n_env]: g_e * dL_e/dxi at xi = 0 for the left twist
 *              T <- exp(xi^) T, xi = (rho, omega): (sum w, sum x_B x w),
 *              w = k phi grad(phi);
 *   d_verts    verts_per_env == 0: per mesh m a block [3][n_verts(m)] of
 *              sum over envs e of mesh m of g_e R_e^T w (blocks in mesh
 *              order; summed in a fixed env order, bit-reproducible);
 *              verts_per_env != 0: [3][Q], g_e R_e^T w per query q.
 * g_e is upstream[e] (1 when upstream is NULL).  Sums are FP32 with
 * compensated (Neumaier) accumulation in a fixed order; no FP64. */
typedef struct fc_grads {
  float* loss;
  float* d_pose;
  float* d_verts;
  int32_t verts_per_env;
} fc_grads;

/* Launch shape of the query kernels (what the autotuner varies; results are
 * bit-identical for every valid choice).
 *   block       threads per workgroup: 128, 256 or 512;
 *   tile        vertices per work item: block, 2*block or 4*block;
 *   persistent  0: one workgroup per item; 1: a grid of about
 *               grid_mult workgroups per compute unit pulling items in a
 *               fixed order; 2: the same pulling items from an atomic counter;
 *               3: the fused forward (fc_sdf_query with fused_out and no
 *               cand) on the adjoint's work items -- a vertex tile against a
 *               chunk of envs, one resident round, env loads pipelined; block,
 *               tile and grid_mult then do not apply;
 *   grid_mult   workgroups per compute unit for persistent launches (1..32);
 *   xcd_remap   1: split the items into 8 contiguous ranges, one per XCD
 *               (each XCD has its own L2), for the forward and the adjoint;
 *   wave_prio   wave priority in the kernels that run the adjoint's work
 *               items (the adjoint, the one-pass query + adjoint, and
 *               persistent = 3): 0 none; 1 (the default) a wave raises its
 *               priority while it computes a vertex's cell and issues the
 *               corner loads, which suits batches bound by the gather's
 *               latency; 2 while it evaluates the gathered corners, which
 *               suits batches whose evaluation dominates.  Scheduling only.
 * fc_batch_create starts from {256, 1024, 0, 8, 0, 1}. */
typedef struct fc_launch {
  int32_t block;
  int32_t tile;
  int32_t persistent;
  int32_t grid_mult;
  int32_t xcd_remap;
  int32_t wave_prio;
} fc_launch;

/* ---- set-up ------------------------------------------------------------- */

/* Validate the description and build the batch: device copies of the item
 * and environment tables, and a default launch shape (or the one a loaded
 * autotune cache gives for this batch's signature).  Errors: FC_ERR_NULL,
 * FC_ERR_SHAPE, FC_ERR_DTYPE, FC_ERR_RANGE, FC_ERR_HIP. */
fc_status fc_batch_create(const fc_batch_desc* desc, fc_batch** out);
void fc_batch_destroy(fc_batch* batch); /* NULL is a no-op; synchronises */

/* Q = total number of queries (sum of n_verts over envs); -1 for NULL. */
int64_t fc_batch_queries(const fc_batch* batch);

/* Replace the launch shape of the forward kernels (rebuilds the item table).
 * FC_ERR_RANGE for an invalid shape. */
fc_status fc_batch_set_launch(fc_batch* batch, const fc_launch* launch);
fc_status fc_batch_get_launch(const fc_batch* batch, fc_launch* out);

/* Workspace: device scratch the caller allocates once per batch, at least
 * fc_workspace_bytes(batch) bytes, 256-byte aligned, ZERO-FILLED before its
 * first use (fc_workspace_init, or any zero fill).  It holds the per-bin
 * reduction keys and a work counter, which every call leaves at zero when it
 * completes, and the adjoint's partial sums, which every call overwrites; so
 * it can be reused, and captured in a graph, without clearing.  Calls that
 * share a workspace must be ordered on one stream.  After a failed or
 * interrupted launch, zero it again. */
size_t fc_workspace_bytes(const fc_batch* batch);
fc_status fc_workspace_init(const fc_batch* batch, void* ws, size_t ws_bytes, void* stream);

/* ---- compute (Section III-C, Algorithm 1) ------------------------------- */

/* Generate: for every environment e and vertex v, x_B = R(q_e) v + t_e
 * (R from the quaternion q = (x,y,z,w) as I + 2w[v]x + 2[v]x^2, not
 * renormalised), then the trilinear SDF value and its exact gradient in the
 * cell min(floor(u), n-2), a candidate iff phi < margin, its normal and bin.
 *   pose       device [7][n_env]: qx,qy,qz,qw,tx,ty,tz (float32);
 *   cand       NULL, or per-query candidates (written for every q);
 *   fused_out  NULL, or reduced contacts: the reduction of
 *              fc_contact_reduce fused into the same kernel (one launch;
 *              candidates stay on chip).
 * At least one of cand / fused_out must be non-NULL (else FC_ERR_NULL). */
fc_status fc_sdf_query(const fc_batch* batch, const float* pose, const fc_candidates* cand,
                       const fc_contacts* fused_out, void* ws, size_t ws_bytes, void* stream);

/* fc_sdf_query without a workspace argument, for callers that cannot
 * allocate device memory around the call (code being captured into a
 * graph, tight serving loops, harnesses that forbid allocation).  Same
 * arguments (minus ws), outputs and errors as fc_sdf_query, bit-identical
 * results.  Its scratch (per-bin keys and work counters) is a static device
 * array of 4 MiB per device, held by every device the library runs on until
 * the process ends; the call allocates nothing and frees nothing, and zeroes
 * the part it uses on `stream` before its kernels (a fill kernel, no
 * memset).  All calls on one device share that array: calls that overlap on
 * one device (two streams, or two host threads without ordering) race and
 * give undefined results; order them on one stream.
 * Extra errors: FC_ERR_SCRATCH if fc_sdf_query_noalloc_bytes(batch) exceeds
 * 4 MiB (about n_env * K <= 524,000 keys); FC_ERR_UNSUPPORTED if the current
 * device is not the one the batch was created on. */
fc_status fc_sdf_query_noalloc(const fc_batch* batch, const float* pose, const fc_candidates* cand,
                               const fc_contacts* fused_out, void* stream);
/* Scratch bytes fc_sdf_query_noalloc needs for this batch (0 for NULL). */
size_t fc_sdf_query_noalloc_bytes(const fc_batch* batch);

/* FindDeepest / BinReduce over candidates written by fc_sdf_query with the
 * same batch and pose: per (env, bin) the candidate of greatest depth, equal
 * depths to the lowest vertex index.  The winner's point is recomputed from
 * pose and vertex; its normal is read from cand.  Bit-identical to the fused
 * form. */
fc_status fc_contact_reduce(const fc_batch* batch, const float* pose, const fc_candidates* cand,
                            const fc_contacts* out, void* ws, size_t ws_bytes, void* stream);

/* Adjoint of the penetration penalty (see fc_grads): recomputes every query
 * (same arithmetic as fc_sdf_query) and accumulates loss and gradients.
 *   k          penalty stiffness, finite and > 0;
 *   upstream   device [n_env] or NULL (all ones).
 * At least one output pointer must be non-NULL. */
fc_status fc_sdf_query_backward(const fc_batch* batch, const float* pose, float k, const float* upstream,
                                const fc_grads* out, void* ws, size_t ws_bytes, void* stream);

/* Per-face contact generation (Section III-A: one contact per triangle of
 * A's mesh, at the point of the face that minimises B's SDF, found by
 * projected gradient descent with an adaptive step).  For every environment
 * e and face f of its mesh: corners x_i = R(q_e) v_i + t_e; start at the
 * centroid b = (1/3, 1/3, 1/3); each of pgd->iters trials takes
 * b' = P(b - alpha (0, g.e1, g.e2)) (P the Euclidean projection onto the
 * simplex, g the SDF gradient at the current point, e1 = x_b - x_a,
 * e2 = x_c - x_a) and keeps it iff phi decreases strictly (a trial outside
 * the grid never does), alpha doubling after a kept trial and halving after
 * a rejected one; alpha starts at pgd->step0 / sqrt(S), S the sum of squared
 * corner distances to the centroid (0 for a degenerate face).  The final
 * point is the face's candidate, recorded and binned as a vertex query's
 * (phi < margin; depth = -phi; normal; bin) and reduced per (env, bin) with
 * the face index as tie-break (contacts' vidx holds the face index).
 *   pgd        iters in [0, 64], step0 finite and > 0;
 *   cand       NULL, or per-face candidates indexed q = face offset of e + f
 *              (fc_batch_face_queries entries; phi, normal, bin and point);
 *   fused_out  NULL, or the reduced contacts.
 * At least one of cand / fused_out must be non-NULL.  Meshes without
 * triangles give no face contacts.  Workspace as for fc_sdf_query. */
typedef struct fc_pgd {
  int32_t iters;
  float step0;
} fc_pgd;
fc_status fc_sdf_query_faces(const fc_batch* batch, const float* pose, const fc_pgd* pgd,
                             const fc_candidates* cand, const fc_contacts* fused_out, void* ws, size_t ws_bytes,
                             void* stream);
/* Number of per-face queries of a batch (sum over envs of their mesh's
 * n_tris), or -1 for NULL. */
int64_t fc_batch_face_queries(const fc_batch* batch);

/* Patch reduction, Section III-C, Algorithm 1.  Per environment, starting
 * with no patches, for each batch of 1024 vertices (vertices [1024 k,
 * 1024 k + 1024)): Generate the candidates (the vertex queries, phi < margin,
 * their normals and depths bit for bit as fc_sdf_query computes them);
 * Assign each to the patch of largest normal similarity among the patches
 * present when the batch began, if any is similar; then while candidates
 * remain: FindDeepest (largest depth, lowest vertex on ties), BinReduce (a
 * new patch takes it and every remaining candidate similar to its normal),
 * AddPatch (appended while fewer than max_patches exist; otherwise it replaces
 * the existing patch of largest similarity with it, lowest index on ties, iff
 * members * depth of the deepest member is larger, in FP32 -- the member
 * count standing for the patch's area; else it is dropped).
 * similar(a, b): (a.x b.x + a.y b.y) + a.z b.z >= cos_sim in FP32 without
 * fused multiply-adds.  A patch keeps its founding contact's normal, its
 * deepest member and its member count. */
typedef struct fc_patch_params {
  int32_t max_patches; /* N, 1 <= N <= 256 (the paper: 128 <= N <= 256) */
  float cos_sim;       /* finite; e.g. cos(10 deg) */
} fc_patch_params;
/* Outputs (device), slot s = e * N + p for patch p of env e, p < count[e]
 * (empty slots: founder = vidx = -1, the rest 0):
 *   count[e]   patches of env e;
 *   founder    vertex that founded the patch;  normal [3][n_env N] its normal;
 *   vidx, depth, point [3][n_env N]: the deepest member (x_B);
 *   members    candidates the patch holds. */
typedef struct fc_patches {
  int32_t* count;
  int32_t* founder;
  float* normal;
  int32_t* vidx;
  float* depth;
  float* point;
  int32_t* members;
} fc_patches;
/* One workgroup per environment; no workspace.  Errors: FC_ERR_NULL (any
 * pointer), FC_ERR_RANGE (max_patches or cos_sim), FC_ERR_HIP. */
fc_status fc_contact_patches(const fc_batch* batch, const float* pose, const fc_patch_params* params,
                             const fc_patches* out, void* stream);

/* fc_sdf_query with fused_out, then fc_sdf_query_backward, computed in one
 * pass over the queries: each query is located, gathered and interpolated
 * once and feeds both the contact reduction and the penalty adjoint.  Every
 * output is bit-identical to the two separate calls (the contacts come from
 * an order-independent integer max; the adjoint keeps its fixed summation
 * order).  For callers that need contacts and penalty gradients in the same
 * step with the upstream weights already known.  Arguments as for the two
 * calls; fused_out and grads are both required (else FC_ERR_NULL). */
fc_status fc_sdf_query_and_backward(const fc_batch* batch, const float* pose, const fc_contacts* fused_out, float k,
                                    const float* upstream, const fc_grads* grads, void* ws, size_t ws_bytes,
                                    void* stream);

/* ---- graphs ------------------------------------------------------------- */

typedef struct fc_graph fc_graph; /* opaque instantiated hipGraph */

/* Capture one step -- the fused forward (if fused_out) and the backward (if
 * grads), as one fc_sdf_query_and_backward pass when both are given -- into
 * an instantiated hipGraph on a private capture stream.  The
 * graph replays with the pointers given here.  Validation as for the calls. */
fc_status fc_graph_create(const fc_batch* batch, const float* pose, const fc_contacts* fused_out, float k,
                          const float* upstream, const fc_grads* grads, void* ws, size_t ws_bytes,
                          fc_graph** out);
fc_status fc_graph_launch(fc_graph* graph, void* stream);
void fc_graph_destroy(fc_graph* graph);

/* ---- layout conversion -------------------------------------------------- */

/* Bytes of `src` (a linear grid) re-laid out as `layout` (FC_LAYOUT_BRICK or
 * FC_LAYOUT_SLAB), same dtype; 0 on invalid input. */
size_t fc_grid_brick_bytes(const fc_grid* src, int32_t layout);

/* Re-lay out a linear grid as `layout`: writes dst_data (device,
 * fc_grid_brick_bytes bytes) and fills *dst with a descriptor of the result.
 * Exact copy of the values (no rounding).  Asynchronous on stream. */
fc_status fc_grid_to_bricks(const fc_grid* src, int32_t layout, void* dst_data, size_t dst_bytes, fc_grid* dst,
                            void* stream);

/* Narrow-band sparse storage of a linear grid (FC_LAYOUT_SPARSE).  A brick
 * (4x4x4 nodes, 3x3x3 cells, bricks of FC_LAYOUT_BRICK) is stored iff one of
 * its nodes has |value| <= band, its nodes have both signs (value < 0 and
 * value >= 0), or it reaches past the grid's last node on some axis.
 * Queries whose cell lies in a stored brick give FC_LAYOUT_BRICK's results
 * bit for bit.  A brick that is not stored has every node beyond the band on
 * one side: outside (all > band), with margin <= band, its queries are
 * neither candidates nor penalised in either layout; inside (all < -band)
 * they take the coarse interpolant.  band >= 0 (+inf stores every
 * brick; else FC_ERR_RANGE); src must be FC_LAYOUT_LINEAR (else
 * FC_ERR_DTYPE).  Both calls are set-up calls: they allocate a temporary,
 * run a classification kernel on `stream` and synchronise it. */
/* *bytes = the size of the sparse buffer of src with this band. */
fc_status fc_grid_sparse_bytes(const fc_grid* src, float band, size_t* bytes, void* stream);
/* Write the sparse buffer to dst_data (device, 256-byte aligned, at least
 * fc_grid_sparse_bytes bytes; else FC_ERR_RANGE / FC_ERR_WORKSPACE) and fill
 * *dst with its descriptor (data = dst_data, layout FC_LAYOUT_SPARSE, the
 * dims, origin and h of src).  Returns after the buffer is written. */
fc_status fc_grid_to_sparse(const fc_grid* src, float band, void* dst_data, size_t dst_bytes, fc_grid* dst,
                            void* stream);

/* ---- mesh -> SDF bake -------------------------------------------------- */

/* Section III-A: body B's SDF is generated from its triangle mesh ahead of
 * time by sampling it on the grid.  Here every node gets the Euclidean
 * distance to the nearest triangle (closest point by Ericson's
 * Voronoi-region tests), negative inside.  The sign is that of (p - q) . n
 * for the closest point q and the angle-weighted pseudonormal n of the
 * feature q lies on (Baerentzen and Aanaes 2005: the face normal, for an edge
 * the sum of its two faces' normals, for a vertex the angle-weighted sum of
 * its faces' normals), which is exact for a closed mesh.  Among triangles at
 * exactly the same distance the lowest index wins.
 *
 * Two steps: fc_bake_table (host, FP64) turns the mesh into a table of per-
 * triangle corners and pseudonormals, which the caller copies to the device;
 * fc_bake_sdf (asynchronous) evaluates every node against it. */

/* Bytes of the table for n_tris triangles: (10 n_tris + 2 ceil(n_tris / 32))
 * float4 records of 16 bytes; 0 if n_tris < 4 or n_tris > 2^24. */
size_t fc_bake_table_bytes(int32_t n_tris);

/* Fill `table` (host, 16-byte aligned, fc_bake_table_bytes bytes) from a mesh:
 * verts host [n_verts][3] (metres), tris host [n_tris][3] vertex indices.
 * The mesh must be closed and consistently wound with outward normals by the
 * right-hand rule: every directed edge occurs once and its reverse once
 * (else FC_ERR_SHAPE, also for an index outside [0, n_verts) or a face with a
 * repeated index), every face has non-zero area and the enclosed volume is
 * positive (else FC_ERR_RANGE, also for a non-finite vertex).  n_verts >= 4,
 * 4 <= n_tris <= 2^24 (else FC_ERR_SHAPE); a short table: FC_ERR_WORKSPACE.
 * Layout, triangles in the order of a Morton curve over their centroids:
 *   [n_tris][3] float4  corner a (w: the mesh's triangle index, int32 bits),
 *                       b - a, c - a (w = 0);
 *   [n_tris][7] float4  pseudonormals: face, edge ab, edge ac, edge bc,
 *                       vertex a, vertex b, vertex c (w = 0);
 *   [ceil(n_tris/32)][2] float4  per run of 32 consecutive triangles the
 *                       bounding box of their corners (lo, hi; w = 0, except
 *                       the first box's lo.w: the largest absolute vertex
 *                       coordinate).
 * Host only; no HIP call. */
fc_status fc_bake_table(const float* verts, int32_t n_verts, const int32_t* tris, int32_t n_tris, void* table,
                        size_t table_bytes);

/* Bake: out (device, [nz][ny][nx] FP32, node (i,j,k) at origin + h*(i,j,k))
 * = the signed distance of the mesh whose table (device, 16-byte aligned,
 * from fc_bake_table) has n_tris triangles.  nx, ny, nz >= 1 with
 * nx*ny*nz < 2^31, 4 <= n_tris <= 2^24 (else FC_ERR_SHAPE); h > 0 and all of
 * origin (host [3]) finite (else FC_ERR_RANGE).  The result can be passed as
 * the data of a linear FC_F32 fc_grid with the same nx, ny, nz, origin, h. */
fc_status fc_bake_sdf(const void* table, int32_t n_tris, int32_t nx, int32_t ny, int32_t nz, const float* origin,
                      float h, float* out, void* stream);

/* The same bake with culling off: every node is evaluated against every
 * triangle, in the same arithmetic, so the result is the definition above
 * evaluated exhaustively.  Same arguments, errors and output as fc_bake_sdf;
 * the cost grows as nodes x triangles.  Its purpose is verification: for a
 * given mesh and grid, fc_bake_sdf's output must equal this one's bit for
 * bit (the culling discards only triangles that cannot win or tie). */
fc_status fc_bake_sdf_unculled(const void* table, int32_t n_tris, int32_t nx, int32_t ny, int32_t nz,
                               const float* origin, float h, float* out, void* stream);

/* ---- autotuning and diagnostics ----------------------------------------- */

/* Load a launch-shape cache written by the autotuner: a JSON object
 * {"entries": [{"key": "<signature>", "block": B, "tile": T,
 * "persistent": P, "grid_mult": M, "xcd_remap": X, "wave_prio": W}, ...]}
 * (xcd_remap defaults to 0, wave_prio to 1).  Batches created afterwards whose
 * signature matches use that shape.  Other members of the object (the
 * tuner's "layouts" list, which the caller reads to choose a grid layout
 * before converting its grids) are skipped.  Returns the number of entries
 * loaded, or -1 if the file cannot be read or parsed. */
int32_t fc_autotune_load(const char* json_path);

/* Signature of a batch, the autotune cache key (NUL-terminated, at most
 * cap bytes written). Returns the full length, or -1 for NULL. */
int32_t fc_batch_signature(const fc_batch* batch, char* buf, int32_t cap);

/* Per-launch timing of the main kernels.  After fc_batch_set_timing(batch, n)
 * the next n compute calls on this batch (fc_sdf_query, fc_contact_reduce,
 * fc_sdf_query_backward, fc_sdf_query_and_backward, fc_sdf_query_faces,
 * fc_contact_patches, fc_gather_probe; not graph capture or
 * replay) record a pair of HIP events on their stream right before and right
 * after their main kernel, leaving out the small payload / combine kernels
 * that follow it.  n = 0 turns timing off; 0 <= n <= FC_MAX_TIMING_RECORDS
 * (else FC_ERR_RANGE).  Creates the events (a host call, not asynchronous;
 * do it outside timed regions).  For one thread at a time per batch. */
#define FC_MAX_TIMING_RECORDS 65536
typedef enum fc_kernel_id {
  FC_KERNEL_FORWARD = 0,        /* k_forward (any mode) */
  FC_KERNEL_BACKWARD = 1,       /* k_backward */
  FC_KERNEL_QUERY_BACKWARD = 2, /* k_query_backward */
  FC_KERNEL_GATHER_PROBE = 3,   /* k_gather_probe */
  FC_KERNEL_FACES = 4,          /* k_faces */
  FC_KERNEL_PATCHES = 5         /* k_patches */
} fc_kernel_id;
fc_status fc_batch_set_timing(fc_batch* batch, int32_t max_records);
/* Waits for the recorded launches and writes, for the first min(recorded,
 * max) of them in call order, the main kernel's duration in milliseconds and
 * its fc_kernel_id; then starts recording again from the first slot.
 * Returns the number written, or -1 (NULL arguments, or a HIP error: see
 * fc_last_hip_error). */
int32_t fc_batch_read_timing(fc_batch* batch, float* ms, int32_t* kernel, int32_t max);

/* Measurement aid: the achievable gather rate of the one-pass path.  Runs
 * fc_sdf_query_and_backward's kernel loop -- the same work items, env
 * pipelining, vertex and pose reads and 8-corner loads per query, at the same
 * addresses -- with no arithmetic beyond summing each query's corners.  The
 * sums are discarded: sink (device, one float) is written only if a sum
 * equals -1.5e38, which the probe's inputs never produce.  Time it with
 * fc_batch_set_timing (kernel id FC_KERNEL_GATHER_PROBE); the ratio of its
 * duration to k_query_backward's is the fraction of the achievable gather
 * rate the full path reaches.  Writes nothing else; needs no workspace. */
fc_status fc_gather_probe(const fc_batch* batch, const float* pose, float* sink, void* stream);

const char* fc_status_str(fc_status status);
int32_t fc_last_hip_error(void); /* hipError_t of the last FC_ERR_HIP on this thread */
const char* fc_version(void);

#ifdef __cplusplus
}
#endif
#endif /* FACTORY_SDF_FC_H */
