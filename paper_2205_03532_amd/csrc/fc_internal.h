// Internal declarations shared by the host ABI (fc_api.cpp) and the HIP
// kernels (fc_kernels.hip).  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/fc.h"

namespace fcimpl {

// Backward work decomposition.  Tile and block fix the order of every
// per-env sum of the adjoint, so they are constants, never tuned.  The chunk
// (envs per item, which orders the shared vertex sums) is chosen once per
// batch at creation from the batch's shape and the device's resident
// capacity (choose_bwd_chunk), the same for every grid layout: the gradients
// are bit-identical for every launch shape and call of a batch, and across
// layouts of the same samples.
constexpr int kBwdTile = 512;     // vertices per backward item (pose partial sums)
constexpr int kBwdBlock = 256;    // threads per backward workgroup (2 vertices each)
constexpr int kBwdChunkMin = 4;   // environments per backward item, at least ...
constexpr int kBwdChunkMax = 64;  // ... and at most

// Dispatch places workgroup i on XCD i mod kXcds (MI355X: 8 XCDs, one L2 each).
constexpr int kXcds = 8;

// Brick layouts: nodes per brick along x, y, z (cells per brick = nodes - 1).
template <int LAYOUT>
struct BrickShape;
template <>
struct BrickShape<FC_LAYOUT_BRICK> {
  static constexpr int NX = 4, NY = 4, NZ = 4;
};
template <>
struct BrickShape<FC_LAYOUT_SLAB> {
  static constexpr int NX = 4, NY = 4, NZ = 2;
};
// Sparse: the bricks of FC_LAYOUT_BRICK, stored only near the surface.
template <>
struct BrickShape<FC_LAYOUT_SPARSE> {
  static constexpr int NX = 4, NY = 4, NZ = 4;
};
inline void brick_nodes(int layout, int& nx, int& ny, int& nz) {
  if (layout == FC_LAYOUT_SLAB) {
    nx = BrickShape<FC_LAYOUT_SLAB>::NX, ny = BrickShape<FC_LAYOUT_SLAB>::NY, nz = BrickShape<FC_LAYOUT_SLAB>::NZ;
  } else {
    nx = BrickShape<FC_LAYOUT_BRICK>::NX, ny = BrickShape<FC_LAYOUT_BRICK>::NY, nz = BrickShape<FC_LAYOUT_BRICK>::NZ;
  }
}

// Normal-bin search table: a cube map of 6 x kLutN x kLutN cells over the
// unit sphere; each cell lists (ascending) every bin that can be the argmax
// for a normal in that cell, or is marked for a full search.
constexpr int kLutN = 8;
constexpr int kLutCells = 6 * kLutN * kLutN;
constexpr int kLutMax = 15;
constexpr unsigned char kLutFull = 0xFF;
struct BinCell {
  unsigned char n;  // number of candidate bins, or kLutFull
  unsigned char k[kLutMax];
};

struct GridDev {
  const void* data;     // samples; FC_LAYOUT_SPARSE: the pool of stored bricks
  const int* map;       // FC_LAYOUT_SPARSE: [bz][by][bx] slot in the pool, -1 = not stored
  const void* coarse;   // FC_LAYOUT_SPARSE: [bz+1][by+1][bx+1] the brick-corner nodes
  int nx, ny, nz;
  int bx, by;  // bricks along x and y (brick layouts)
  float ox, oy, oz;
  float inv_h;
};

// Sparse grid buffer: map (int32 per brick), coarse grid, pool; each section
// starts on a 256-byte boundary.
inline size_t sparse_align(size_t x) { return (x + 255) & ~size_t(255); }
inline size_t sparse_coarse_offset(long long bricks) { return sparse_align((size_t)bricks * 4); }
inline size_t sparse_pool_offset(long long bricks, int bx, int by, int bz, int elem) {
  return sparse_coarse_offset(bricks) + sparse_align((size_t)(bx + 1) * (by + 1) * (bz + 1) * elem);
}

struct MeshDev {
  const float* x;
  const float* y;
  const float* z;
  const int* tris;  // [3][nt] corner indices (per-face queries), or null
  int n;
  int nt;
};

struct Item {  // one forward work item: a tile of one environment's vertices
  int env;
  int vstart;
  int vcount;
  int gm;  // grid index | mesh index << 8
};

struct EnvInfo {
  long long qoff;  // first query index of the env
  int n_items;     // forward items of the env (>= 1)
  int gm;
};

struct FwdArgs {
  GridDev grids[FC_MAX_TYPES];
  MeshDev meshes[FC_MAX_TYPES];
  float dirs[3 * FC_MAX_BINS];  // [3][K]
  const BinCell* bin_lut;       // [kLutCells]
  const Item* items;
  const EnvInfo* envs;
  const float* pose;  // [7][n_env]
  int n_items;
  int n_env;
  int K;
  float margin;
  long long Q;
  // candidates (may be null)
  float* c_phi;
  float* c_nrm;
  int16_t* c_bin;
  float* c_point;  // per-face queries only
  // per-face queries: descent trials and first step
  int pgd_iters;
  float pgd_step0;
  // reduced contacts (may be null)
  int* o_vidx;
  float* o_depth;
  float* o_point;
  float* o_nrm;
  int* o_count;
  // workspace (zero between calls)
  unsigned long long* keys;  // [n_env][K] per-bin maxima, taken and reset by the payload kernel
  unsigned* work_ctr;        // [kXcds] persistent work counters, reset by the payload kernel
};

struct BwdItem {
  int vstart;
  int vcount;
  int gm;
  int chunk;  // chunk id: envs env_list[chunk_first[chunk] .. + chunk_len[chunk])
  int tile;   // global tile id
  int tile_in_mesh;
  int pad0, pad1;
};

struct BwdChunk {
  int first;      // into env_list
  int len;        // envs in this chunk (<= kBwdChunkMax)
  int n_tiles;    // tiles of the chunk's mesh
  int mesh;
  long long vpart;  // offset (in float2) of this chunk's vertex partials [3][n_v]
};

struct BwdArgs {
  GridDev grids[FC_MAX_TYPES];
  MeshDev meshes[FC_MAX_TYPES];
  long long mesh_voff[FC_MAX_TYPES];  // shared-mode d_verts offset (floats) of mesh m
  int mesh_tiles[FC_MAX_TYPES];       // backward tiles of mesh m (>= 1)
  int mesh_chunk0[FC_MAX_TYPES];      // first chunk of mesh m (chunks of a mesh are contiguous)
  int mesh_nchunks[FC_MAX_TYPES];     // chunks of mesh m
  long long mesh_vpart0[FC_MAX_TYPES];  // vertex-partial offset (float2) of mesh m's first chunk
  int n_meshes;
  const BwdItem* items;
  const BwdChunk* chunks;
  const int* env_list;
  const int* env_tile_base;  // [n_env] first pose-partial row of the env
  const EnvInfo* envs;
  const float* pose;
  const float* upstream;
  int n_items;
  int n_env;
  float k;
  int per_env;
  int xcd;   // XCD-contiguous item ranges
  int prio;  // wave priority mode (fc_launch::wave_prio)
  long long Q;
  float* loss;
  float* d_pose;
  float* d_verts;
  // workspace: partial sums, fully overwritten by every call
  float2* pose_part;  // [(env, tile) rows][waves][8]: 7 used
  float2* vert_part;  // per chunk [3][n_v]
};

// The forward's binning and reduction inputs, added to BwdArgs by the
// one-pass query + adjoint (contacts and penalty gradients from one gather).
struct QueryExtra {
  float dirs[3 * FC_MAX_BINS];  // [3][K]
  const BinCell* bin_lut;       // [kLutCells]
  int K;
  float margin;
  unsigned long long* keys;  // [n_env][K], as FwdArgs::keys
};

// HIP events (hipEvent_t) recorded on the launch stream right before and right
// after the main kernel of a launch (k_forward, k_backward, k_query_backward),
// not around its small companion kernels; null pointer = no events.
struct KernelMarks {
  void* before;
  void* after;
};

// launch wrappers (fc_kernels.hip)
hipError_t launch_forward(const FwdArgs& a, int dtype, int layout, int block, int vpt, int persistent, int xcd,
                          int grid, bool from_cand, hipStream_t s, const KernelMarks* m);
hipError_t launch_backward(const BwdArgs& a, int dtype, int layout, hipStream_t s, const KernelMarks* m);
// one pass: k_query_backward, then the payload (`payload` holds the contact
// outputs and keys) and the adjoint's combine
hipError_t launch_query_backward(const BwdArgs& a, const QueryExtra& q, const FwdArgs& payload, int dtype, int layout,
                                 hipStream_t s, const KernelMarks* m);

// per-face queries: k_faces over (env, face tile) items, then k_face_payload
hipError_t launch_faces(const FwdArgs& a, int dtype, int layout, hipStream_t s, const KernelMarks* m);
constexpr int kFaceBlock = 256;  // threads per face workgroup
constexpr int kFaceVpt = 2;      // faces per thread (independent descents interleaved)
constexpr int kFaceTile = kFaceBlock * kFaceVpt;

// the fused forward on the adjoint's env-chunked work items (fc_launch
// persistent = 3): k_query_chunked, then the payload
hipError_t launch_query_chunked(const BwdArgs& a, const QueryExtra& q, const FwdArgs& payload, int dtype, int layout,
                                hipStream_t s, const KernelMarks* m);
// measurement aid: k_query_backward's items, loop and corner loads, no arithmetic
hipError_t launch_gather_probe(const BwdArgs& a, int dtype, int layout, hipStream_t s, const KernelMarks* m);
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);
// The no-allocation forward's scratch: a static device array of this many
// bytes per device (fc_kernels.hip), held until the process ends.
constexpr size_t kNoAllocScratchBytes = size_t(4) << 20;
// Device address of the current device's scratch array, looked up once per
// device (hipGetSymbolAddress with that device current) and kept.
hipError_t noalloc_scratch(void** ptr);
// Patch reduction (Algorithm 1): one workgroup per environment, batches of
// kPatchBatch vertices, at most kPatchMax patches.
constexpr int kPatchThreads = 256;                      // threads per workgroup
constexpr int kPatchVpt = 4;                            // vertices per thread and batch
constexpr int kPatchBatch = kPatchThreads * kPatchVpt;  // 1024, the paper's batch
constexpr int kPatchMax = 256;
struct PatchArgs {
  int n_max;       // N, 1 <= N <= kPatchMax
  float cos_sim;   // similar(a, b): dot(a, b) >= cos_sim
  int* count;      // [n_env] patches kept
  int* founder;    // [n_env * N] founding vertex, -1 if the slot is empty
  float* normal;   // [3][n_env * N] the patch normal (the founder's)
  int* vidx;       // [n_env * N] deepest member, -1 if empty
  float* depth;    // [n_env * N] its depth
  float* point;    // [3][n_env * N] its x_B
  int* members;    // [n_env * N]
};
hipError_t launch_patches(const FwdArgs& a, const PatchArgs& p, int dtype, int layout, hipStream_t s,
                          const KernelMarks* m);

// Sparse conversion: flags[b] = 1 if brick b is stored (a node with
// |value| <= band, nodes of both signs, or nodes past the grid's edge).
hipError_t launch_sparse_classify(const void* src, int dtype, int nx, int ny, int nz, int bx, int by, int bz,
                                  float band, unsigned char* flags, hipStream_t s);
// pool[slot] = the 64 nodes of brick list[slot]; coarse = the brick-corner nodes
hipError_t launch_sparse_fill(const void* src, int elem, int nx, int ny, int nz, int bx, int by, int bz,
                              const int* list, int n_stored, void* pool, void* coarse, hipStream_t s);
hipError_t launch_to_bricks(const void* src, void* dst, int elem, int layout, int nx, int ny, int nz, int bx, int by,
                            int bz, hipStream_t s);
bool forward_shape_supported(int block, int vpt);
// workgroups of k_backward and of k_query_backward (the lower) that can be
// resident on one compute unit at once, for a grid of dtype and layout
int backward_blocks_per_cu(int dtype);

}  // namespace fcimpl
