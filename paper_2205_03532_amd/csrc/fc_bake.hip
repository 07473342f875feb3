// HIP kernel for gfx950 (CDNA4): baking a signed-distance grid from a closed
// triangle mesh.
//
// Section III-A of Narang et al. (Factory, RSS 2022): body B's SDF is
// generated from its mesh ahead of time, by sampling, and stored as a grid.
// Every node gets the Euclidean distance to the nearest triangle (closest
// point by Ericson's Voronoi-region tests, Real-Time Collision Detection
// 5.1.5), signed by the angle-weighted pseudonormal of the closest feature
// (Baerentzen and Aanaes 2005), negative inside.
//
// The work is point-triangle distance evaluation, plain FP32 ALU work with no
// dense contraction, so there is no MFMA: the design work is in not
// evaluating pairs that cannot win.  One wave takes a 4x4x4 brick of nodes;
// triangles come in Morton-sorted clusters of 32 with bounding boxes; a
// cluster, then a triangle, is evaluated only if its box can hold a point
// within some lane's current best distance plus a slack far above FP32
// rounding, so the result equals evaluating every triangle.
//
// Numerics: compiled with -ffp-contract=off; every fused multiply-add is an
// explicit fmaf.
#include <hip/hip_runtime.h>

#include "fc_bake.h"

namespace fcimpl {
namespace {

// Closest point of triangle (a, a + ab, a + ac) to p and its feature, by the
// Voronoi-region tests in the order vertex a, vertex b, edge ab, vertex c,
// edge ac, edge bc, face (codes as BakeFeature).  Returns |p - q|^2.  Lanes
// leave the chain at their region, so a wave whose nodes all see a vertex or
// an edge of a distant triangle skips the rest.
__device__ __forceinline__ float closest_on_triangle(float px, float py, float pz, const float4& A,
                                                     const float4& AB, const float4& AC, float& qx, float& qy,
                                                     float& qz, int& feat) {
  const float apx = px - A.x, apy = py - A.y, apz = pz - A.z;
  const float d1 = fmaf(AB.x, apx, fmaf(AB.y, apy, AB.z * apz));
  const float d2 = fmaf(AC.x, apx, fmaf(AC.y, apy, AC.z * apz));
  const float bpx = apx - AB.x, bpy = apy - AB.y, bpz = apz - AB.z;
  const float d3 = fmaf(AB.x, bpx, fmaf(AB.y, bpy, AB.z * bpz));
  const float d4 = fmaf(AC.x, bpx, fmaf(AC.y, bpy, AC.z * bpz));
  const float cpx = apx - AC.x, cpy = apy - AC.y, cpz = apz - AC.z;
  const float d5 = fmaf(AB.x, cpx, fmaf(AB.y, cpy, AB.z * cpz));
  const float d6 = fmaf(AC.x, cpx, fmaf(AC.y, cpy, AC.z * cpz));
  const float vc = fmaf(d1, d4, -(d3 * d2));
  const float vb = fmaf(d5, d2, -(d1 * d6));
  const float va = fmaf(d3, d6, -(d5 * d4));
  float u = 0.f, v = 0.f;  // q = a + u ab + v ac
  if ((d1 <= 0.f) & (d2 <= 0.f)) {
    feat = kBakeVertA;
  } else if ((d3 >= 0.f) & (d4 <= d3)) {
    u = 1.f;
    feat = kBakeVertB;
  } else if ((vc <= 0.f) & (d1 >= 0.f) & (d3 <= 0.f)) {
    u = d1 * __builtin_amdgcn_rcpf(d1 - d3);
    feat = kBakeEdgeAB;
  } else if ((d6 >= 0.f) & (d5 <= d6)) {
    v = 1.f;
    feat = kBakeVertC;
  } else if ((vb <= 0.f) & (d2 >= 0.f) & (d6 <= 0.f)) {
    v = d2 * __builtin_amdgcn_rcpf(d2 - d6);
    feat = kBakeEdgeAC;
  } else if ((va <= 0.f) & ((d4 - d3) >= 0.f) & ((d5 - d6) >= 0.f)) {
    const float e43 = d4 - d3, e56 = d5 - d6;
    const float r = __builtin_amdgcn_rcpf(e43 + e56);
    u = e56 * r;  // 1 - w
    v = e43 * r;  // w
    feat = kBakeEdgeBC;
  } else {
    const float r = __builtin_amdgcn_rcpf((va + vb) + vc);
    u = vb * r;
    v = vc * r;
    feat = kBakeFace;
  }
  qx = fmaf(v, AC.x, fmaf(u, AB.x, A.x));
  qy = fmaf(v, AC.y, fmaf(u, AB.y, A.y));
  qz = fmaf(v, AC.z, fmaf(u, AB.z, A.z));
  const float dx = px - qx, dy = py - qy, dz = pz - qz;
  return fmaf(dx, dx, fmaf(dy, dy, dz * dz));
}

// Squared distance bounds between a brick of nodes (box bl..bh) and a cluster
// box (cl..ch): no point of one box is nearer than sqrt(lb2) to the other;
// every point of the brick lies within sqrt(ub2) of every point of the cluster.
__device__ __forceinline__ float box_lb2(float blx, float bly, float blz, float bhx, float bhy, float bhz,
                                         const float4& cl, const float4& ch) {
  const float dx = fmaxf(fmaxf(cl.x - bhx, blx - ch.x), 0.f);
  const float dy = fmaxf(fmaxf(cl.y - bhy, bly - ch.y), 0.f);
  const float dz = fmaxf(fmaxf(cl.z - bhz, blz - ch.z), 0.f);
  return fmaf(dx, dx, fmaf(dy, dy, dz * dz));
}
__device__ __forceinline__ float box_ub2(float blx, float bly, float blz, float bhx, float bhy, float bhz,
                                         const float4& cl, const float4& ch) {
  const float dx = fmaxf(fabsf(ch.x - blx), fabsf(bhx - cl.x));
  const float dy = fmaxf(fabsf(ch.y - bly), fabsf(bhy - cl.y));
  const float dz = fmaxf(fabsf(ch.z - blz), fabsf(bhz - cl.z));
  return fmaf(dx, dx, fmaf(dy, dy, dz * dz));
}

struct BakeBest {
  float d2 = __builtin_inff();
  float lim = __builtin_inff();  // (sqrt(d2) + slack)^2: a triangle whose box is farther cannot win or tie
  float qx = 0.f, qy = 0.f, qz = 0.f;
  int t = -1;                   // position in the table
  int orig = 0x7FFFFFFF;        // the mesh's triangle index (ties go to the lowest)
  int feat = 0;
};

__device__ __forceinline__ float lane_f(float x, int j) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), j));
}

// Cluster c against this lane's node.  Lanes 0..31 (and again 32..63) load
// one triangle each and test its bounding box against the brick's box with
// the wave's bound.  Each triangle that passes is broadcast from the lane
// that loaded it; the wave evaluates it only if its box is within some
// lane's own limit.
__device__ __forceinline__ void bake_cluster(const BakeArgs& B, int c, float blx, float bly, float blz, float bhx,
                                             float bhy, float bhz, float bound, float slack, float px, float py,
                                             float pz, BakeBest& b) {
  const int t = c * kBakeCluster + (int)(threadIdx.x & (kBakeCluster - 1));
  float4 A = make_float4(0.f, 0.f, 0.f, 0.f), AB = A, AC = A, lo = A, hi = A;
  float tlb = __builtin_inff();
  if (t < B.n_tris) {
    A = B.pos[3 * t];
    AB = B.pos[3 * t + 1];
    AC = B.pos[3 * t + 2];
    const float bx_ = A.x + AB.x, by_ = A.y + AB.y, bz_ = A.z + AB.z;
    const float cx_ = A.x + AC.x, cy_ = A.y + AC.y, cz_ = A.z + AC.z;
    lo = make_float4(fminf(A.x, fminf(bx_, cx_)), fminf(A.y, fminf(by_, cy_)), fminf(A.z, fminf(bz_, cz_)), 0.f);
    hi = make_float4(fmaxf(A.x, fmaxf(bx_, cx_)), fmaxf(A.y, fmaxf(by_, cy_)), fmaxf(A.z, fmaxf(bz_, cz_)), 0.f);
    tlb = box_lb2(blx, bly, blz, bhx, bhy, bhz, lo, hi);
  }
  unsigned long long m = __ballot(((threadIdx.x & 63) < kBakeCluster) & (t < B.n_tris) & (tlb <= bound));
  while (m) {
    const int j = __ffsll((long long)m) - 1;
    m &= m - 1;
    // this lane's distance to the triangle's box
    const float dx = fmaxf(fmaxf(lane_f(lo.x, j) - px, px - lane_f(hi.x, j)), 0.f);
    const float dy = fmaxf(fmaxf(lane_f(lo.y, j) - py, py - lane_f(hi.y, j)), 0.f);
    const float dz = fmaxf(fmaxf(lane_f(lo.z, j) - pz, pz - lane_f(hi.z, j)), 0.f);
    if (__ballot(fmaf(dx, dx, fmaf(dy, dy, dz * dz)) <= b.lim) == 0) continue;
    const float4 Aj = make_float4(lane_f(A.x, j), lane_f(A.y, j), lane_f(A.z, j), lane_f(A.w, j));
    const float4 ABj = make_float4(lane_f(AB.x, j), lane_f(AB.y, j), lane_f(AB.z, j), 0.f);
    const float4 ACj = make_float4(lane_f(AC.x, j), lane_f(AC.y, j), lane_f(AC.z, j), 0.f);
    float qx, qy, qz;
    int feat;
    const float d2 = closest_on_triangle(px, py, pz, Aj, ABj, ACj, qx, qy, qz, feat);
    const int orig = __float_as_int(Aj.w);
    if (d2 < b.d2 || (d2 == b.d2 && orig < b.orig)) {
      b.d2 = d2;
      const float r = sqrtf(d2) + slack;
      b.lim = r * r;
      b.qx = qx;
      b.qy = qy;
      b.qz = qz;
      b.t = c * kBakeCluster + j;
      b.orig = orig;
      b.feat = feat;
    }
  }
}

// Cull bound of the wave: (sqrt(max over lanes of best d2) + slack)^2.
__device__ __forceinline__ float bake_bound(float d2, float slack) {
  float m = d2;
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  const float r = sqrtf(m) + slack;
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(r * r)));
}

// One wave per brick of 4 x 4 x 4 nodes, one node per lane.  The triangles
// come in spatially sorted clusters with bounding boxes; a wave evaluates a
// cluster only if its box can hold a point nearer than the wave's worst
// current best plus a slack far above FP32 rounding, so the result equals
// evaluating every triangle: the nearest triangle (lowest mesh index among
// exact ties), its distance, and the sign of (p - q) . n for its feature's
// pseudonormal n (negative inside).
__global__ __launch_bounds__(kBakeBlock) void k_bake(BakeArgs B) {
  const int lane = (int)(threadIdx.x & 63);
  const long long brick = (long long)blockIdx.x * (kBakeBlock / 64) + (threadIdx.x >> 6);
  if (brick >= (long long)B.bx * B.by * B.bz) return;  // the whole wave
  const int bxi = (int)(brick % B.bx), byi = (int)((brick / B.bx) % B.by), bzi = (int)(brick / ((long long)B.bx * B.by));
  const int ix0 = 4 * bxi, iy0 = 4 * byi, iz0 = 4 * bzi;
  const int ix = ix0 + (lane & 3), iy = iy0 + ((lane >> 2) & 3), iz = iz0 + (lane >> 4);
  const bool live = (ix < B.nx) & (iy < B.ny) & (iz < B.nz);
  // lanes past the grid's edge repeat an edge node: they stay inside the brick's box
  const float px = fmaf((float)min(ix, B.nx - 1), B.h, B.ox);
  const float py = fmaf((float)min(iy, B.ny - 1), B.h, B.oy);
  const float pz = fmaf((float)min(iz, B.nz - 1), B.h, B.oz);
  const float blx = fmaf((float)ix0, B.h, B.ox), bhx = fmaf((float)min(ix0 + 3, B.nx - 1), B.h, B.ox);
  const float bly = fmaf((float)iy0, B.h, B.oy), bhy = fmaf((float)min(iy0 + 3, B.ny - 1), B.h, B.oy);
  const float blz = fmaf((float)iz0, B.h, B.oz), bhz = fmaf((float)min(iz0 + 3, B.nz - 1), B.h, B.oz);
  const float slack = fmaxf(B.slack, B.box[0].w * 0x1p-12f);  // box[0].w: the mesh's largest coordinate

  // start from the cluster with the least upper bound: after it every lane's
  // best is at most that bound
  float ub = __builtin_inff();
  int uc = 0;  // a valid cluster even if every bound overflows
  for (int c = lane; c < B.n_clusters; c += 64) {
    const float u = box_ub2(blx, bly, blz, bhx, bhy, bhz, B.box[2 * c], B.box[2 * c + 1]);
    if (u < ub) {
      ub = u;
      uc = c;
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    const float u2 = __shfl_xor(ub, o);
    const int c2 = __shfl_xor(uc, o);
    if (u2 < ub || (u2 == ub && c2 < uc)) {
      ub = u2;
      uc = c2;
    }
  }
  const int first = __builtin_amdgcn_readfirstlane(uc);
  BakeBest b;
  // the least upper bound plus the slack: every lane has a triangle that near
  const float r0 = sqrtf(__int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(ub)))) + slack;
  bake_cluster(B, first, blx, bly, blz, bhx, bhy, bhz, r0 * r0, slack, px, py, pz, b);
  float bound = bake_bound(b.d2, slack);

  for (int c0 = 0; c0 < B.n_clusters; c0 += 64) {
    const int c = c0 + lane;
    float lb = __builtin_inff();
    float4 cl = make_float4(0.f, 0.f, 0.f, 0.f), ch = cl;
    if (c < B.n_clusters && c != first) {
      cl = B.box[2 * c];
      ch = B.box[2 * c + 1];
      lb = box_lb2(blx, bly, blz, bhx, bhy, bhz, cl, ch);
    }
    unsigned long long m = __ballot((c < B.n_clusters) & (c != first) & (lb <= bound));
    while (m) {
      const int i = __ffsll((long long)m) - 1;
      m &= m - 1;
      if (lane_f(lb, i) > bound) continue;  // the bound has shrunk since the ballot
      // skip the cluster unless its box is within some lane's own limit
      const float dx = fmaxf(fmaxf(lane_f(cl.x, i) - px, px - lane_f(ch.x, i)), 0.f);
      const float dy = fmaxf(fmaxf(lane_f(cl.y, i) - py, py - lane_f(ch.y, i)), 0.f);
      const float dz = fmaxf(fmaxf(lane_f(cl.z, i) - pz, pz - lane_f(ch.z, i)), 0.f);
      if (__ballot(fmaf(dx, dx, fmaf(dy, dy, dz * dz)) <= b.lim) == 0) continue;
      bake_cluster(B, c0 + i, blx, bly, blz, bhx, bhy, bhz, bound, slack, px, py, pz, b);
      bound = bake_bound(b.d2, slack);
    }
  }
  if (!live) return;
  float val = __builtin_nanf("");  // no triangle gave a number (all degenerate in FP32)
  if (b.t >= 0) {
    const float4 nrm = B.nrm[(long long)b.t * kBakeFeatures + b.feat];
    const float sd = fmaf(px - b.qx, nrm.x, fmaf(py - b.qy, nrm.y, (pz - b.qz) * nrm.z));
    const float d = sqrtf(b.d2);
    val = sd < 0.f ? -d : d;
  }
  B.out[((long long)iz * B.ny + iy) * B.nx + ix] = val;
}

}  // namespace

hipError_t launch_bake(const BakeArgs& b, hipStream_t s) {
  const long long bricks = (long long)b.bx * b.by * b.bz;
  const long long blocks = (bricks + kBakeBlock / 64 - 1) / (kBakeBlock / 64);
  if (blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_bake, dim3((unsigned)blocks), dim3(kBakeBlock), 0, s, b);
  return hipGetLastError();
}

}  // namespace fcimpl
