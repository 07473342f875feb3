// Internal declarations of the mesh -> SDF bake (fc_bake.hip), shared with
// the host side (fc_api.cpp).
#pragma once

#include <hip/hip_runtime.h>

namespace fcimpl {

// mesh -> SDF bake.  Table: per triangle (sorted along a Morton curve of the
// centroids) corner a (w = the mesh's triangle index, int bits), edges ab and
// ac (float4), then the 7 pseudonormals in BakeFeature order (float4, w
// unused), then per cluster of kBakeCluster consecutive triangles its
// bounding box (lo, hi float4; w unused except the first cluster's lo.w, the
// mesh's largest absolute coordinate).
constexpr int kBakeBlock = 256;  // 4 waves, one 4x4x4 brick of nodes each
constexpr int kBakeCluster = 32;
constexpr int kBakeFace = 0, kBakeEdgeAB = 1, kBakeEdgeAC = 2, kBakeEdgeBC = 3, kBakeVertA = 4, kBakeVertB = 5,
              kBakeVertC = 6, kBakeFeatures = 7;
struct BakeArgs {
  const float4* pos;  // [n_tris][3]
  const float4* nrm;  // [n_tris][kBakeFeatures]
  const float4* box;  // [n_clusters][2]
  int n_tris, n_clusters;
  int nx, ny, nz;
  int bx, by, bz;  // bricks per axis
  float ox, oy, oz, h;
  float slack;  // metres added to the cull bound (from the grid; the kernel raises it for the mesh)
  float* out;   // [nz][ny][nx]
};
hipError_t launch_bake(const BakeArgs& b, hipStream_t s);

}  // namespace fcimpl
