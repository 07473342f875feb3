// HIP kernels for gfx950 (CDNA4): vertex-vs-SDF queries, contact reduction
// and the penetration-penalty adjoint.
//
// What is computed (Narang et al., Factory, RSS 2022):
//   Section III-A -- the SDF is a grid read with trilinear filtering; value
//   and gradient give a contact's distance and normal.
//   Section III-C, Algorithm 1 -- Generate candidate contacts for a batch of
//   the mesh's features, then FindDeepest / BinReduce: here the deepest
//   candidate per fixed normal-direction bin, lowest vertex index on ties.
//   The reduction runs on chip (LDS) inside the generating kernel, as the
//   paper does in shared memory so that candidates never reach global memory.
//
// Numerics: this file is compiled with -ffp-contract=off; every fused
// multiply-add is an explicit fmaf.  All code paths that evaluate a query
// (candidate pass, fused pass, winner recompute, adjoint) call the same
// inline functions, so they produce the same bits.
//
// The path is a gather-bound stencil (8 corner loads per query and about 100
// flops), so there is no MFMA here: the design work is in the gather
// (coalesced SoA vertex reads, corner pairs loaded as one 8-byte access,
// optional brick layout keeping a cell's corners in one 128-byte line) and in
// keeping the reduction on chip (LDS 64-bit atomic max per bin,
// one global 64-bit atomicMax per bin per work item).
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <mutex>

#include "fc_device.h"

namespace fcimpl {
namespace {


// ---------------------------------------------------------------------------
// DPP lane permutations (register to register) for the adjoint's wavefront
// reduction (wave_sum8): xor-1 and xor-2 quad permutes and the half-row and
// row mirrors; lanes 16 and 32 apart are reached through ds_swizzle and
// ds_bpermute.  All 64 lanes must be active.
// ---------------------------------------------------------------------------
constexpr int kDppXor1 = 0xB1;        // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;        // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141; // lane i <- lane 7-i within each 8 lanes
constexpr int kDppMirror = 0x140;     // lane i <- lane 15-i within each row

template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, false));
}
// Per-bin max over a work item: every candidate lane applies its key to the
// bin's LDS slot with a 64-bit atomic max (ds_max_u64).  Lanes of one
// wavefront that hit the same bin are serialised by the LDS unit, not by
// VALU work; the thread-surface patches of one wavefront span many bins, so
// a per-bin wavefront reduction (one ballot/DPP round per distinct bin) costs
// more than it saves.  The max is order-independent: the result is exact.
__device__ __forceinline__ void bin_max(bool cand, int bin, unsigned long long key, unsigned long long* s_keys) {
  if (cand) atomicMax(&s_keys[bin], key);
}

// ---------------------------------------------------------------------------
// forward: one work item = up to BLOCK*VPT vertices of one environment
// ---------------------------------------------------------------------------
template <int DT, int LAYOUT, int BLOCK, int VPT>
__device__ __forceinline__ void query_item(const FwdArgs& A, const Item& it, unsigned long long* s_keys, bool fused,
                                           const BinCell* s_lut, const float4* s_dir4) {
  const GridDev& g = A.grids[it.gm & 0xff];
  const MeshDev& m = A.meshes[it.gm >> 8];
  const Rigid P = load_pose(A.pose, A.n_env, it.env);
  const int tid = threadIdx.x;
  const int vend = it.vstart + it.vcount;

  float px[VPT], py[VPT], pz[VPT];
  bool ok[VPT];
#pragma unroll
  for (int j = 0; j < VPT; ++j) {
    const int v = it.vstart + j * BLOCK + tid;
    ok[j] = v < vend;
    float x = 0.f, y = 0.f, z = 0.f;
    if (ok[j]) {
      x = m.x[v];
      y = m.y[v];
      z = m.z[v];
    }
    transform(P, x, y, z, px[j], py[j], pz[j]);
  }
  Cell cl[VPT];
  float c[VPT][8];
#pragma unroll
  for (int j = 0; j < VPT; ++j) cl[j] = locate(g, px[j], py[j], pz[j]);
#pragma unroll
  for (int j = 0; j < VPT; ++j) gather<DT, LAYOUT>(g, cl[j], c[j]);

  const bool want_cand = A.c_phi != nullptr;
  const long long qoff = want_cand ? A.envs[it.env].qoff : 0;
#pragma unroll
  for (int j = 0; j < VPT; ++j) {
    float phi, gx, gy, gz;
    trilinear(c[j], cl[j].tx, cl[j].ty, cl[j].tz, phi, gx, gy, gz);
    const bool inside = ok[j] & cl[j].inside;
    const bool cand = inside & (phi < A.margin);
    float nx = 0.f, ny = 0.f, nz = 0.f;
    int bin = -1;
    if (cand | (want_cand & inside)) normalize(gx, gy, gz, nx, ny, nz);
    if (cand) bin = argmax_bin_lut(s_lut, s_dir4, A.dirs, A.K, nx, ny, nz);
    const int v = it.vstart + j * BLOCK + tid;
    if (want_cand & ok[j]) {
      const long long q = qoff + v;
      A.c_phi[q] = inside ? phi : __builtin_inff();
      A.c_nrm[q] = nx;
      A.c_nrm[A.Q + q] = ny;
      A.c_nrm[2 * A.Q + q] = nz;
      A.c_bin[q] = (int16_t)bin;
    }
    if (fused) bin_max(cand, bin, make_key(-phi, (unsigned)v), s_keys);
  }
}

template <int BLOCK, int VPT>
__device__ __forceinline__ void reduce_item(const FwdArgs& A, const Item& it, unsigned long long* s_keys) {
  const long long qoff = A.envs[it.env].qoff;
  const int tid = threadIdx.x;
  const int vend = it.vstart + it.vcount;
  int b[VPT];
  float phi[VPT];
#pragma unroll
  for (int j = 0; j < VPT; ++j) {
    const int v = it.vstart + j * BLOCK + tid;
    b[j] = -1;
    phi[j] = 0.f;
    if (v < vend) {
      b[j] = A.c_bin[qoff + v];
      phi[j] = A.c_phi[qoff + v];
    }
  }
#pragma unroll
  for (int j = 0; j < VPT; ++j) {
    const int v = it.vstart + j * BLOCK + tid;
    const bool cand = (b[j] >= 0) & (b[j] < A.K);  // bins come from caller memory: stay inside s_keys
    bin_max(cand, b[j], make_key(-phi[j], (unsigned)v), s_keys);
  }
}

// Winner slot of (env, bin = lane): point recomputed from pose and vertex;
// normal recomputed (fused) or read from the candidates (unfused).
template <int DT, int LAYOUT>
__device__ __forceinline__ void write_slot(const FwdArgs& A, int gm, int e, int lane, unsigned long long key,
                                           bool from_cand) {
  const long long S = (long long)A.n_env * A.K;
  const long long s = (long long)e * A.K + lane;
  if (key == 0ull) {
    A.o_vidx[s] = -1;
    A.o_depth[s] = 0.f;
    A.o_point[s] = 0.f;
    A.o_point[S + s] = 0.f;
    A.o_point[2 * S + s] = 0.f;
    A.o_nrm[s] = 0.f;
    A.o_nrm[S + s] = 0.f;
    A.o_nrm[2 * S + s] = 0.f;
    return;
  }
  const unsigned v = key_vidx(key);
  const MeshDev& m = A.meshes[gm >> 8];
  if (v >= (unsigned)m.n) {  // only a workspace that was not zeroed can hold such a key
    A.o_vidx[s] = -1;
    return;
  }
  const Rigid P = load_pose(A.pose, A.n_env, e);
  float xb, yb, zb;
  transform(P, m.x[v], m.y[v], m.z[v], xb, yb, zb);
  float nx, ny, nz;
  if (from_cand) {
    const long long q = A.envs[e].qoff + v;
    nx = A.c_nrm[q];
    ny = A.c_nrm[A.Q + q];
    nz = A.c_nrm[2 * A.Q + q];
  } else {
    float phi, gx, gy, gz;
    bool inside;
    sample<DT, LAYOUT>(A.grids[gm & 0xff], xb, yb, zb, phi, gx, gy, gz, inside);
    normalize(gx, gy, gz, nx, ny, nz);
  }
  A.o_vidx[s] = (int)v;
  A.o_depth[s] = key_depth(key);
  A.o_point[s] = xb;
  A.o_point[S + s] = yb;
  A.o_point[2 * S + s] = zb;
  A.o_nrm[s] = nx;
  A.o_nrm[S + s] = ny;
  A.o_nrm[2 * S + s] = nz;
}

// Push a work item's per-bin maxima to its environment's keys.  Relaxed
// device-scope 64-bit atomics and no fence: the keys are consumed by the next
// kernel on the stream, after the kernel boundary.
__device__ __forceinline__ void item_flush(const FwdArgs& A, const Item& it, const unsigned long long* s_keys) {
  if ((int)threadIdx.x < A.K) {
    const unsigned long long k = s_keys[threadIdx.x];
    if (k) atomicMax(&A.keys[(long long)it.env * A.K + threadIdx.x], k);
  }
}

// Work items a workgroup owns.  Plain launch: item = workgroup id.  With
// `xcd` set, the items are split into kXcds contiguous ranges and range x is
// served by the workgroups the dispatcher places on XCD x (ids = x mod kXcds),
// so each XCD's L2 sees a contiguous stretch of the (locality-ordered) item
// list.  Persistent launches stride (1) or pull from a per-range atomic
// counter (2).
struct ItemRange {
  int lo, hi, slot, nslots;
  unsigned* ctr;
};

__device__ __forceinline__ ItemRange item_range(int n_items, int xcd, unsigned* work_ctr) {
  ItemRange r;
  if (xcd) {
    const int x = blockIdx.x % kXcds;
    const int per = (n_items + kXcds - 1) / kXcds;
    r.lo = x * per;
    r.hi = min(n_items, r.lo + per);
    r.slot = blockIdx.x / kXcds;
    r.nslots = gridDim.x / kXcds;
    r.ctr = work_ctr + x;
  } else {
    r.lo = 0;
    r.hi = n_items;
    r.slot = blockIdx.x;
    r.nslots = gridDim.x;
    r.ctr = work_ctr;
  }
  return r;
}

template <int DT, int LAYOUT, int BLOCK, int VPT>
__global__ __launch_bounds__(BLOCK) void k_forward(FwdArgs A, int persistent, int from_cand, int xcd) {
  __shared__ unsigned long long s_keys[FC_MAX_BINS];
  __shared__ int s_item;
  __shared__ BinCell s_lut[kLutCells];
  __shared__ float4 s_dir4[FC_MAX_BINS];
  const bool fused = A.o_vidx != nullptr;
  const ItemRange R = item_range(A.n_items, xcd, A.work_ctr);
  if (!from_cand) {  // bin-search tables into LDS
    static_assert(sizeof(BinCell) == sizeof(uint4), "BinCell is one 16-byte load");
    const uint4* src = reinterpret_cast<const uint4*>(A.bin_lut);
    uint4* dst = reinterpret_cast<uint4*>(s_lut);
    for (int i = threadIdx.x; i < kLutCells; i += BLOCK) dst[i] = src[i];
    if (threadIdx.x < FC_MAX_BINS) {
      const int k = threadIdx.x < A.K ? threadIdx.x : 0;
      s_dir4[threadIdx.x] = make_float4(A.dirs[k], A.dirs[A.K + k], A.dirs[2 * A.K + k], 0.f);
    }
    __syncthreads();
  }
  int idx;
  if (persistent == 2) {
    if (threadIdx.x == 0) s_item = R.lo + (int)atomicAdd(R.ctr, 1u);
    __syncthreads();
    idx = s_item;
    __syncthreads();
  } else {
    idx = R.lo + R.slot;
  }
  while (idx < R.hi) {
    const Item it = A.items[idx];
    if (fused) {
      if (threadIdx.x < FC_MAX_BINS) s_keys[threadIdx.x] = 0ull;
      __syncthreads();
    }
    if (from_cand)
      reduce_item<BLOCK, VPT>(A, it, s_keys);
    else
      query_item<DT, LAYOUT, BLOCK, VPT>(A, it, s_keys, fused, s_lut, s_dir4);
    if (fused) {
      __syncthreads();
      item_flush(A, it, s_keys);
      __syncthreads();
    }
    if (persistent == 0) break;
    if (persistent == 1) {
      idx += R.nslots;
    } else {
      if (threadIdx.x == 0) s_item = R.lo + (int)atomicAdd(R.ctr, 1u);
      __syncthreads();
      idx = s_item;
      __syncthreads();
    }
  }
}

// Winners: one wavefront per environment, lane = bin.  Takes each key
// (resetting it to zero for the next call), writes the slot and the count,
// and resets the persistent work counters.
template <int DT, int LAYOUT>
__device__ __forceinline__ void payload_block(const FwdArgs& A, int from_cand, int block) {
  if (block == 0 && threadIdx.x < kXcds) A.work_ctr[threadIdx.x] = 0u;
  const int e = block * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (e >= A.n_env) return;
  unsigned long long key = 0ull;
  if (lane < A.K) {
    unsigned long long* kp = A.keys + (long long)e * A.K + lane;
    key = *kp;
    *kp = 0ull;
    write_slot<DT, LAYOUT>(A, A.envs[e].gm, e, lane, key, from_cand != 0);
  }
  const unsigned long long nonempty = __ballot((lane < A.K) && (key != 0ull));
  if (lane == 0) A.o_count[e] = __popcll(nonempty);
}

template <int DT, int LAYOUT>
__global__ __launch_bounds__(256) void k_payload(FwdArgs A, int from_cand) {
  payload_block<DT, LAYOUT>(A, from_cand, blockIdx.x);
}

// ---------------------------------------------------------------------------
// per-face queries: projected gradient descent of phi over each face
// ---------------------------------------------------------------------------
// Euclidean projection of (y0, y1, y2) onto the simplex {b >= 0, sum b = 1}:
// with u the values sorted in decreasing order and c_j = u_1 + ... + u_j - 1,
// rho counts the j with u_j > c_j / j (they form a prefix) and the threshold
// is theta = c_rho / rho.
__device__ __forceinline__ void project_simplex3(float y0, float y1, float y2, float& b0, float& b1, float& b2) {
  float u0 = y0, u1 = y1, u2 = y2;
  if (u0 < u1) { const float t = u0; u0 = u1; u1 = t; }
  if (u1 < u2) { const float t = u1; u1 = u2; u2 = t; }
  if (u0 < u1) { const float t = u0; u0 = u1; u1 = t; }
  const float c1 = u0 - 1.f;
  const float c2 = (u0 + u1) - 1.f;
  const float c3 = ((u0 + u1) + u2) - 1.f;
  const int rho = 1 + ((u1 - c2 * 0.5f) > 0.f ? 1 : 0) + ((u2 - c3 * (1.f / 3.f)) > 0.f ? 1 : 0);
  const float theta = rho == 1 ? c1 : (rho == 2 ? c2 * 0.5f : c3 * (1.f / 3.f));
  b0 = fmaxf(y0 - theta, 0.f);
  b1 = fmaxf(y1 - theta, 0.f);
  b2 = fmaxf(y2 - theta, 0.f);
}

// One face's descent state: first corner and edges in B's frame, barycentric
// coordinates, the current point, phi there (+inf outside the grid) and its
// grid-unit gradient, the step.
struct FaceState {
  float ax, ay, az, e1x, e1y, e1z, e2x, e2y, e2z;
  float b1, b2;  // b0 = 1 - b1 - b2 is carried by the projection
  float b0;
  float x, y, z;
  float phi, gx, gy, gz;
  float alpha;
  bool valid;
};

__device__ __forceinline__ void face_point(const FaceState& S, float b1, float b2, float& x, float& y, float& z) {
  x = fmaf(b2, S.e2x, fmaf(b1, S.e1x, S.ax));
  y = fmaf(b2, S.e2y, fmaf(b1, S.e1y, S.ay));
  z = fmaf(b2, S.e2z, fmaf(b1, S.e1z, S.az));
}

// Descent of NV faces at once (their loads interleaved): corners from the
// mesh (a face with an out-of-range index is marked invalid and never
// accepts a trial), start at the centroid, iters projected trials with the
// accept-if-lower rule and a doubling / halving step.
template <int DT, int LAYOUT, int NV>
__device__ __forceinline__ void face_descent(const GridDev& g, const MeshDev& m, const Rigid& P, const int (&f)[NV],
                                             const bool (&ok)[NV], int iters, float step0, FaceState (&S)[NV]) {
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    FaceState& F = S[j];
    unsigned ia = 0, ib = 0, ic = 0;
    if (ok[j]) {
      ia = (unsigned)m.tris[f[j]];
      ib = (unsigned)m.tris[m.nt + f[j]];
      ic = (unsigned)m.tris[2 * m.nt + f[j]];
    }
    F.valid = ok[j] & (ia < (unsigned)m.n) & (ib < (unsigned)m.n) & (ic < (unsigned)m.n);
    if (!F.valid) ia = ib = ic = 0;
    float bx, by, bz, cx, cy, cz;
    const bool any_v = m.n > 0;
    transform(P, any_v ? m.x[ia] : 0.f, any_v ? m.y[ia] : 0.f, any_v ? m.z[ia] : 0.f, F.ax, F.ay, F.az);
    transform(P, any_v ? m.x[ib] : 0.f, any_v ? m.y[ib] : 0.f, any_v ? m.z[ib] : 0.f, bx, by, bz);
    transform(P, any_v ? m.x[ic] : 0.f, any_v ? m.y[ic] : 0.f, any_v ? m.z[ic] : 0.f, cx, cy, cz);
    F.e1x = bx - F.ax; F.e1y = by - F.ay; F.e1z = bz - F.az;
    F.e2x = cx - F.ax; F.e2y = cy - F.ay; F.e2z = cz - F.az;
    const float dx = F.e2x - F.e1x, dy = F.e2y - F.e1y, dz = F.e2z - F.e1z;
    const float S3 = fmaf(F.e1x, F.e1x, fmaf(F.e1y, F.e1y, F.e1z * F.e1z)) +
                     fmaf(F.e2x, F.e2x, fmaf(F.e2y, F.e2y, F.e2z * F.e2z)) + fmaf(dx, dx, fmaf(dy, dy, dz * dz));
    const float SS = S3 * (1.f / 3.f);  // sum of squared corner distances to the centroid
    F.alpha = SS > 0.f ? step0 * rsqrtf(SS) : 0.f;
    F.b0 = F.b1 = F.b2 = 1.f / 3.f;
    face_point(F, F.b1, F.b2, F.x, F.y, F.z);
  }
  Cell cl[NV];
  float cc[NV][8];
#pragma unroll
  for (int j = 0; j < NV; ++j) cl[j] = locate(g, S[j].x, S[j].y, S[j].z);
#pragma unroll
  for (int j = 0; j < NV; ++j) gather<DT, LAYOUT>(g, cl[j], cc[j]);
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    float phi, gx, gy, gz;
    trilinear(cc[j], cl[j].tx, cl[j].ty, cl[j].tz, phi, gx, gy, gz);
    S[j].phi = (S[j].valid & cl[j].inside) ? phi : __builtin_inff();
    S[j].gx = gx;
    S[j].gy = gy;
    S[j].gz = gz;
  }
  for (int it = 0; it < iters; ++it) {
    float tb0[NV], tb1[NV], tb2[NV], tx[NV], ty[NV], tz[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      const FaceState& F = S[j];
      // b-gradient (0, g.e1, g.e2) with g in metres (grid units / h)
      const float d1 = g.inv_h * fmaf(F.gx, F.e1x, fmaf(F.gy, F.e1y, F.gz * F.e1z));
      const float d2 = g.inv_h * fmaf(F.gx, F.e2x, fmaf(F.gy, F.e2y, F.gz * F.e2z));
      project_simplex3(F.b0, fmaf(-F.alpha, d1, F.b1), fmaf(-F.alpha, d2, F.b2), tb0[j], tb1[j], tb2[j]);
      face_point(F, tb1[j], tb2[j], tx[j], ty[j], tz[j]);
      cl[j] = locate(g, tx[j], ty[j], tz[j]);
    }
#pragma unroll
    for (int j = 0; j < NV; ++j) gather<DT, LAYOUT>(g, cl[j], cc[j]);
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      FaceState& F = S[j];
      float phi, gx, gy, gz;
      trilinear(cc[j], cl[j].tx, cl[j].ty, cl[j].tz, phi, gx, gy, gz);
      const bool keep = F.valid & cl[j].inside & (phi < F.phi);
      if (keep) {
        F.b0 = tb0[j];
        F.b1 = tb1[j];
        F.b2 = tb2[j];
        F.x = tx[j];
        F.y = ty[j];
        F.z = tz[j];
        F.phi = phi;
        F.gx = gx;
        F.gy = gy;
        F.gz = gz;
      }
      F.alpha = keep ? 2.f * F.alpha : 0.5f * F.alpha;
    }
  }
}

// One work item: a tile of kFaceTile faces of one environment.  Candidates,
// bins and the per-bin maxima as in query_item, keyed by the face index.
template <int DT, int LAYOUT>
__global__ __launch_bounds__(kFaceBlock) void k_faces(FwdArgs A) {
  __shared__ unsigned long long s_keys[FC_MAX_BINS];
  __shared__ BinCell s_lut[kLutCells];
  __shared__ float4 s_dir4[FC_MAX_BINS];
  static_assert(sizeof(BinCell) == sizeof(uint4), "BinCell is one 16-byte load");
  {
    const uint4* src = reinterpret_cast<const uint4*>(A.bin_lut);
    uint4* dst = reinterpret_cast<uint4*>(s_lut);
    for (int i = threadIdx.x; i < kLutCells; i += kFaceBlock) dst[i] = src[i];
  }
  if (threadIdx.x < FC_MAX_BINS) {
    const int k = threadIdx.x < A.K ? threadIdx.x : 0;
    s_dir4[threadIdx.x] = make_float4(A.dirs[k], A.dirs[A.K + k], A.dirs[2 * A.K + k], 0.f);
    s_keys[threadIdx.x] = 0ull;
  }
  __syncthreads();
  const Item it = A.items[blockIdx.x];
  const GridDev& g = A.grids[it.gm & 0xff];
  const MeshDev& m = A.meshes[it.gm >> 8];
  const Rigid P = load_pose(A.pose, A.n_env, it.env);
  const bool fused = A.o_vidx != nullptr;
  const bool want_cand = A.c_phi != nullptr;
  const long long qoff = A.envs[it.env].qoff;
  int f[kFaceVpt];
  bool ok[kFaceVpt];
#pragma unroll
  for (int j = 0; j < kFaceVpt; ++j) {
    f[j] = it.vstart + j * kFaceBlock + (int)threadIdx.x;
    ok[j] = f[j] < it.vstart + it.vcount;
  }
  FaceState S[kFaceVpt];
  face_descent<DT, LAYOUT, kFaceVpt>(g, m, P, f, ok, A.pgd_iters, A.pgd_step0, S);
#pragma unroll
  for (int j = 0; j < kFaceVpt; ++j) {
    const FaceState& F = S[j];
    const bool inside = F.phi < __builtin_inff();
    const bool cand = inside & (F.phi < A.margin);
    float nx = 0.f, ny = 0.f, nz = 0.f;
    int bin = -1;
    if (cand | (want_cand & inside)) normalize(F.gx, F.gy, F.gz, nx, ny, nz);
    if (cand) bin = argmax_bin_lut(s_lut, s_dir4, A.dirs, A.K, nx, ny, nz);
    if (want_cand & ok[j]) {
      const long long q = qoff + f[j];
      A.c_phi[q] = F.phi;
      A.c_nrm[q] = nx;
      A.c_nrm[A.Q + q] = ny;
      A.c_nrm[2 * A.Q + q] = nz;
      A.c_bin[q] = (int16_t)bin;
      A.c_point[q] = F.x;
      A.c_point[A.Q + q] = F.y;
      A.c_point[2 * A.Q + q] = F.z;
    }
    if (fused) bin_max(cand, bin, make_key(-F.phi, (unsigned)f[j]), s_keys);
  }
  if (fused) {
    __syncthreads();
    if ((int)threadIdx.x < A.K) {
      const unsigned long long k = s_keys[threadIdx.x];
      if (k) atomicMax(&A.keys[(long long)it.env * A.K + threadIdx.x], k);
    }
  }
}

// Winners of the per-face query: one wavefront per environment, lane = bin;
// the winning face's descent is run again (same arithmetic, same bits) for
// its point and normal.  Takes each key, resetting it to zero.
template <int DT, int LAYOUT>
__global__ __launch_bounds__(256) void k_face_payload(FwdArgs A) {
  const int e = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (e >= A.n_env) return;
  unsigned long long key = 0ull;
  if (lane < A.K) {
    unsigned long long* kp = A.keys + (long long)e * A.K + lane;
    key = *kp;
    *kp = 0ull;
  }
  const int gm = A.envs[e].gm;
  const MeshDev& m = A.meshes[gm >> 8];
  const unsigned fv = key_vidx(key);
  const bool have = (lane < A.K) && (key != 0ull) && (fv < (unsigned)m.nt);
  const int f[1] = {have ? (int)fv : 0};
  const bool ok[1] = {have};
  FaceState S[1];
  face_descent<DT, LAYOUT, 1>(A.grids[gm & 0xff], m, load_pose(A.pose, A.n_env, e), f, ok, A.pgd_iters,
                              A.pgd_step0, S);
  if (lane < A.K) {
    const long long NS = (long long)A.n_env * A.K;
    const long long s = (long long)e * A.K + lane;
    float nx = 0.f, ny = 0.f, nz = 0.f;
    if (have) normalize(S[0].gx, S[0].gy, S[0].gz, nx, ny, nz);
    A.o_vidx[s] = have ? (int)fv : -1;
    A.o_depth[s] = have ? key_depth(key) : 0.f;
    A.o_point[s] = have ? S[0].x : 0.f;
    A.o_point[NS + s] = have ? S[0].y : 0.f;
    A.o_point[2 * NS + s] = have ? S[0].z : 0.f;
    A.o_nrm[s] = nx;
    A.o_nrm[NS + s] = ny;
    A.o_nrm[2 * NS + s] = nz;
  }
  const unsigned long long nonempty = __ballot(have);
  if (lane == 0) A.o_count[e] = __popcll(nonempty);
}

// ---------------------------------------------------------------------------
// adjoint of the penetration penalty
// ---------------------------------------------------------------------------
// Neumaier compensated accumulation, (sum, compensation) in a float2.
__device__ __forceinline__ void nadd(float2& a, float x) {
  const float t = a.x + x;
  a.y += (fabsf(a.x) >= fabsf(x)) ? ((a.x - t) + x) : ((x - t) + a.x);
  a.x = t;
}
// Sum of two (sum, compensation) pairs: the sums' exact rounding error (by
// branch-free TwoSum, the same value as the ordered Fast2Sum of Neumaier's
// step) joins the compensations.
__device__ __forceinline__ float2 ncombine(float2 a, float2 b) {
  const float t = a.x + b.x;
  const float bb = t - a.x;
  const float e = (a.x - (t - bb)) + (b.x - bb);
  return make_float2(t, (a.y + b.y) + e);
}

// a + b as an unevaluated (sum, rounding error) pair, exact for finite
// inputs (Knuth's branch-free TwoSum)
__device__ __forceinline__ float2 two_sum(float a, float b) {
  const float s = a + b;
  const float bb = s - a;
  return make_float2(s, (a - (s - bb)) + (b - bb));
}

template <int CTRL>
__device__ __forceinline__ float2 dpp_pair(float2 a) {
  return make_float2(dpp_f<CTRL>(a.x), dpp_f<CTRL>(a.y));
}
template <int PATTERN>
__device__ __forceinline__ float2 swizzle_pair(float2 a) {
  return make_float2(__int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(a.x), PATTERN)),
                     __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(a.y), PATTERN)));
}
__device__ __forceinline__ float2 xor32_pair(float2 a) {
  const int addr = (__lane_id() ^ 32) << 2;
  return make_float2(__int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(a.x))),
                     __int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(a.y))));
}
constexpr int kSwzXor16 = 0x401F;  // ds_swizzle bit mode: lane i <- lane i ^ 16 within 32

__device__ __forceinline__ float2 pick(bool hi, float2 a, float2 b) { return hi ? b : a; }

// Which of the eight pairs lane l holds after wave_sum8:
// (b2^b3) + 2 (b1^b2) + 4 (b0^b2) for the lane's bits b0..b3.
__device__ __forceinline__ int wave_sum8_slot(int lane) {
  const int b0 = lane & 1, b1 = (lane >> 1) & 1, b2 = (lane >> 2) & 1, b3 = (lane >> 3) & 1;
  return (b2 ^ b3) + 2 * (b1 ^ b2) + 4 * (b0 ^ b2);
}

// Compensated sums of eight (sum, compensation) pairs over the 64 lanes of a
// wavefront, in a fixed order, by a transposed butterfly.  In each of the
// first three steps a lane keeps half of its remaining pairs and trades the
// other half with a partner lane (xor 1 and xor 2 within a quad, then the
// mirror within eight lanes), so the pairs per lane halve while the lanes each
// pair covers double; the row mirror, xor 16 and xor 32 then finish the one
// pair left.  The keep/send choices (b0^b2, b1^b2, b2^b3) are invariant under
// every later pairing, so both partners always hold the same pair.  Returns
// the wavefront total of pair wave_sum8_slot(lane); each total sits in eight
// lanes.  About a quarter of the work of one 64-lane tree per pair.
__device__ __forceinline__ float2 wave_sum8(const float2 a[8]) {
  const int lane = __lane_id();
  const int b0 = lane & 1, b1 = (lane >> 1) & 1, b2 = (lane >> 2) & 1, b3 = (lane >> 3) & 1;
  const bool s1 = b0 ^ b2, s2 = b1 ^ b2, s3 = b2 ^ b3;
  float2 x1[4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
    x1[i] = ncombine(pick(s1, a[i], a[i + 4]), dpp_pair<kDppXor1>(pick(s1, a[i + 4], a[i])));
  float2 x2[2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
    x2[i] = ncombine(pick(s2, x1[i], x1[i + 2]), dpp_pair<kDppXor2>(pick(s2, x1[i + 2], x1[i])));
  float2 x = ncombine(pick(s3, x2[0], x2[1]), dpp_pair<kDppHalfMirror>(pick(s3, x2[1], x2[0])));
  x = ncombine(x, dpp_pair<kDppMirror>(x));
  x = ncombine(x, swizzle_pair<kSwzXor16>(x));
  return ncombine(x, xor32_pair(x));
}

// Per-wavefront bin keys in LDS, kKeyCopies copies: lane l updates copy
// l mod kKeyCopies, so lanes that share a bin (a flat face puts a whole
// wavefront in one) spread their atomics over kKeyCopies addresses in
// different banks instead of queueing on one.  The flush takes the largest
// of a bin's copies, clears them and issues one global atomic per non-empty
// bin.
constexpr int kKeyCopies = 4;
constexpr int kKeyStride = FC_MAX_BINS + 1;  // odd stride: the copies of a bin sit in different banks
__device__ __forceinline__ void wave_key_max(unsigned long long* s_wkeys, int bin, unsigned long long key) {
  atomicMax(&s_wkeys[(__lane_id() & (kKeyCopies - 1)) * kKeyStride + bin], key);
}
__device__ __forceinline__ void wave_key_flush(unsigned long long* s_wkeys, unsigned long long* keys, int K) {
  wave_lds_sync();  // the lanes' LDS atomics before the per-bin reads
  const int lane = __lane_id();
  if (lane < K) {
    unsigned long long kk = 0ull;
#pragma unroll
    for (int c = 0; c < kKeyCopies; ++c) {
      const unsigned long long v = s_wkeys[c * kKeyStride + lane];
      kk = v > kk ? v : kk;
    }
    if (kk) {
      atomicMax(&keys[lane], kk);
#pragma unroll
      for (int c = 0; c < kKeyCopies; ++c) s_wkeys[c * kKeyStride + lane] = 0ull;
    }
  }
}

struct NoQuery {};
// Measurement mode: the same items, loop and loads, and no arithmetic beyond
// summing the corners (kept live by a store that a sentinel sum would take).
struct GatherOnly {};
constexpr float kProbeSentinel = -1.5e38f;

// One backward work item: a tile of kBwdTile vertices of one mesh against the
// envs of one chunk.  With QX = QueryExtra the same pass also forms the
// forward's candidates and per-bin maxima (one gather serves both): each
// wavefront keeps its own K keys in LDS, flushed to the env's global keys
// after every env.
// PERV: per-env vertex gradients (A.per_env), stored per query; otherwise the
// shared vertex gradient is summed in LDS.  A compile-time choice keeps the
// stores of the other mode out of the env loop, where any vector-memory
// operation the compiler cannot count ahead makes it wait for the corner
// loads in flight.
template <int DT, int LAYOUT, class QX, bool ADJ = true, bool PERV = false>
__device__ __forceinline__ void backward_item(const BwdArgs& A, const QX& F, unsigned long long* s_wkeys,
                                              const BinCell* s_lut, const float4* s_dir4) {
  constexpr bool PROBE = __is_same(QX, GatherOnly);
  constexpr bool QUERY = !__is_same(QX, NoQuery) && !PROBE;  // ADJ = false: the query half alone
  constexpr int V = kBwdTile / kBwdBlock;
  static_assert(V >= 2, "lane pairs start from two terms");
  constexpr int NW = kBwdBlock / 64;
  int idx = blockIdx.x;
  if (A.xcd) {  // XCD x serves the x-th contiguous range of items (see item_range)
    const int per = (A.n_items + kXcds - 1) / kXcds;
    const int slot = blockIdx.x / kXcds;
    idx = (blockIdx.x % kXcds) * per + slot;
    if (slot >= per || idx >= A.n_items) return;
  }
  const BwdItem it = A.items[idx];
  const BwdChunk ch = A.chunks[it.chunk];
  const GridDev& g = A.grids[it.gm & 0xff];
  const MeshDev& m = A.meshes[it.gm >> 8];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const bool shared_v = !PERV && (A.d_verts != nullptr);

  float vx[V], vy[V], vz[V];
  bool ok[V];
#pragma unroll
  for (int j = 0; j < V; ++j) {
    const int v = it.vstart + j * kBwdBlock + tid;
    ok[j] = v < it.vstart + it.vcount;
    vx[j] = ok[j] ? m.x[v] : 0.f;
    vy[j] = ok[j] ? m.y[v] : 0.f;
    vz[j] = ok[j] ? m.z[v] : 0.f;
  }
  // the vertex-gradient sums of this thread's vertices, (sum, compensation)
  // per component, kept in LDS (they change only for penetrating queries)
  __shared__ float2 s_accv[V][3][kBwdBlock];
  if constexpr (ADJ) {
#pragma unroll
    for (int j = 0; j < V; ++j) s_accv[j][0][tid] = s_accv[j][1][tid] = s_accv[j][2][tid] = make_float2(0.f, 0.f);
  }

  // R, t and the upstream weight of the chunk's envs, computed once per
  // item, with the env ids and the rows they write: read from LDS in the env
  // loop, a global load there would wait for every corner load in flight
  __shared__ float4 s_pose[kBwdChunkMax][4];
  __shared__ int s_env[kBwdChunkMax];
  __shared__ int s_row[kBwdChunkMax];
  __shared__ long long s_qoff[kBwdChunkMax];
  if (tid < ch.len) {
    const int e = A.env_list[ch.first + tid];
    s_env[tid] = e;
    s_row[tid] = A.env_tile_base[e] + it.tile_in_mesh;
    s_qoff[tid] = A.envs[e].qoff;
    const Rigid P = load_pose(A.pose, A.n_env, e);
    s_pose[tid][0] = make_float4(P.r00, P.r01, P.r02, P.tx);
    s_pose[tid][1] = make_float4(P.r10, P.r11, P.r12, P.ty);
    s_pose[tid][2] = make_float4(P.r20, P.r21, P.r22, P.tz);
    s_pose[tid][3] = make_float4(A.upstream ? A.upstream[e] : 1.f, 0.f, 0.f, 0.f);
  }
  __syncthreads();

  // With two vertices per thread the env loop is software-pipelined over two
  // register sets: the corner loads of env c + 1 are in flight while env c is
  // evaluated.
  struct Stage {
    Cell cl[V];
    float cc[V][8];
  };
  const auto pose_of = [&](int c) {
    const float4 p0 = s_pose[c][0], p1 = s_pose[c][1], p2 = s_pose[c][2];
    return Rigid{p0.x, p0.y, p0.z, p1.x, p1.y, p1.z, p2.x, p2.y, p2.z, p0.w, p1.w, p2.w};
  };
  // Wave priority (A.prio): 1 raises it while a wave computes addresses and
  // issues its corner loads, so loads of waves that are ready to issue them
  // go out ahead of other waves' arithmetic; 2 raises it while a wave
  // evaluates.  Scheduling only: the results do not depend on it.
  const auto issue = [&](Stage& S, int c) {  // transform, locate, start the gather
    if (A.prio == 1) __builtin_amdgcn_s_setprio(2);
    const Rigid P = pose_of(c);
#pragma unroll
    for (int j = 0; j < V; ++j) {
      float x, y, z;
      transform(P, vx[j], vy[j], vz[j], x, y, z);
      S.cl[j] = locate(g, x, y, z);
    }
#pragma unroll
    for (int j = 0; j < V; ++j) gather<DT, LAYOUT>(g, S.cl[j], S.cc[j]);
    __builtin_amdgcn_s_setprio(0);
  };
  const auto evaluate = [&](Stage& S, int c) {  // everything after the gather
    if constexpr (PROBE) {
      float sum = 0.f;
#pragma unroll
      for (int j = 0; j < V; ++j)
#pragma unroll
        for (int q = 0; q < 8; ++q) sum += S.cc[j][q];
      if (sum == kProbeSentinel) A.loss[0] = sum;
      return;
    }
    const int e = s_env[c];
    const Cell* cl = S.cl;
    const auto& cc = S.cc;
    if constexpr (!ADJ) {  // the forward's candidates, bins and per-bin maxima only
#pragma unroll
      for (int j = 0; j < V; ++j) {
        float phi, gx, gy, gz;
        trilinear(cc[j], cl[j].tx, cl[j].ty, cl[j].tz, phi, gx, gy, gz);
        if (ok[j] & cl[j].inside & (phi < F.margin)) {
          float nx, ny, nz;
          normalize(gx, gy, gz, nx, ny, nz);
          const int bin = argmax_bin_lut(s_lut, s_dir4, F.dirs, F.K, nx, ny, nz);
          wave_key_max(s_wkeys, bin, make_key(-phi, (unsigned)(it.vstart + j * kBwdBlock + tid)));
        }
      }
      wave_key_flush(s_wkeys, F.keys + (long long)e * F.K, F.K);
      return;
    }
    const Rigid P = pose_of(c);
    const float up = s_pose[c][3].x;
    // x_B again (same arithmetic, same bits) rather than held across the pipeline
    float xb[V], yb[V], zb[V];
#pragma unroll
    for (int j = 0; j < V; ++j) transform(P, vx[j], vy[j], vz[j], xb[j], yb[j], zb[j]);
    float T[V][7];  // this lane's terms of the env's sums (zero where inactive)
    bool any = false;
#pragma unroll
    for (int j = 0; j < V; ++j) {
      float phi, gx, gy, gz;
      trilinear(cc[j], cl[j].tx, cl[j].ty, cl[j].tz, phi, gx, gy, gz);
      if constexpr (QUERY) {  // the forward's candidate, bin and per-bin max, as in query_item
        if (ok[j] & cl[j].inside & (phi < F.margin)) {
          float nx, ny, nz;
          normalize(gx, gy, gz, nx, ny, nz);
          const int bin = argmax_bin_lut(s_lut, s_dir4, F.dirs, F.K, nx, ny, nz);
          wave_key_max(s_wkeys, bin, make_key(-phi, (unsigned)(it.vstart + j * kBwdBlock + tid)));
        }
      }
      const bool act = ok[j] & cl[j].inside & (phi < 0.f);
      float dvx = 0.f, dvy = 0.f, dvz = 0.f;
#pragma unroll
      for (int i = 0; i < 7; ++i) T[j][i] = 0.f;
      if (act) {
        any = true;
        const float kphi = A.k * phi;
        const float s = kphi * g.inv_h;  // k phi / h: grid-unit gradient -> metres
        const float wx = s * gx, wy = s * gy, wz = s * gz;
        const float mx = fmaf(yb[j], wz, -(zb[j] * wy));
        const float my = fmaf(zb[j], wx, -(xb[j] * wz));
        const float mz = fmaf(xb[j], wy, -(yb[j] * wx));
        T[j][0] = 0.5f * kphi * phi;
        T[j][1] = wx;
        T[j][2] = wy;
        T[j][3] = wz;
        T[j][4] = mx;
        T[j][5] = my;
        T[j][6] = mz;
        // R^T w, scaled by the upstream gradient
        dvx = up * fmaf(P.r00, wx, fmaf(P.r10, wy, P.r20 * wz));
        dvy = up * fmaf(P.r01, wx, fmaf(P.r11, wy, P.r21 * wz));
        dvz = up * fmaf(P.r02, wx, fmaf(P.r12, wy, P.r22 * wz));
        if (shared_v) {
          float2 a0 = s_accv[j][0][tid], a1 = s_accv[j][1][tid], a2 = s_accv[j][2][tid];
          nadd(a0, dvx);
          nadd(a1, dvy);
          nadd(a2, dvz);
          s_accv[j][0][tid] = a0;
          s_accv[j][1][tid] = a1;
          s_accv[j][2][tid] = a2;
        }
      }
      if (PERV && ok[j]) {  // launched with PERV only when A.d_verts is set
        const long long q = s_qoff[c] + it.vstart + j * kBwdBlock + tid;
        A.d_verts[q] = dvx;
        A.d_verts[A.Q + q] = dvy;
        A.d_verts[2 * A.Q + q] = dvz;
      }
    }
    if constexpr (QUERY) wave_key_flush(s_wkeys, F.keys + (long long)e * F.K, F.K);
    // fixed-shape reduction within the wavefront; one partial row of eight
    // pairs (the last one zero) per (env, tile, wave), no workgroup barrier
    float2 red = make_float2(0.f, 0.f);
    if (__ballot(any) != 0ull) {
      float2 acc[8];  // the lane's terms, summed exactly as (sum, error) pairs
#pragma unroll
      for (int i = 0; i < 7; ++i) {
        acc[i] = two_sum(T[0][i], T[1][i]);
#pragma unroll
        for (int j = 2; j < V; ++j) nadd(acc[i], T[j][i]);
      }
      acc[7] = make_float2(0.f, 0.f);
      red = wave_sum8(acc);
    }
    if (lane < 8)
      A.pose_part[((long long)s_row[c] * NW + wave) * 8 + wave_sum8_slot(lane)] = red;
  };
  const auto finish = [&](Stage& S, int c) {
    if (A.prio == 2) __builtin_amdgcn_s_setprio(2);
    evaluate(S, c);
    __builtin_amdgcn_s_setprio(0);
  };
  if constexpr (V <= 2) {
    Stage SA, SB;
    if (ch.len > 0) issue(SA, 0);
    for (int c = 0; c < ch.len; c += 2) {
      if (c + 1 < ch.len) issue(SB, c + 1);
      finish(SA, c);
      if (c + 2 < ch.len) issue(SA, c + 2);
      if (c + 1 < ch.len) finish(SB, c + 1);
    }
  } else {  // enough loads per env in flight without a second register set
    Stage S;
    for (int c = 0; c < ch.len; ++c) {
      issue(S, c);
      finish(S, c);
    }
  }

  if (ADJ && !PROBE && shared_v) {
    const long long base = A.chunks[it.chunk].vpart;
    const int n = m.n;
#pragma unroll
    for (int j = 0; j < V; ++j) {
      if (!ok[j]) continue;
      const int v = it.vstart + j * kBwdBlock + tid;
      A.vert_part[base + v] = s_accv[j][0][tid];
      A.vert_part[base + n + v] = s_accv[j][1][tid];
      A.vert_part[base + 2 * (long long)n + v] = s_accv[j][2][tid];
    }
  }
}

template <int DT, int LAYOUT, bool PERV>
__global__ __launch_bounds__(kBwdBlock) void k_backward(BwdArgs A) {
  backward_item<DT, LAYOUT, NoQuery, true, PERV>(A, NoQuery{}, nullptr, nullptr, nullptr);
}

template <int DT, int LAYOUT>
__global__ __launch_bounds__(kBwdBlock) void k_gather_probe(BwdArgs A) {
  backward_item<DT, LAYOUT>(A, GatherOnly{}, nullptr, nullptr, nullptr);
}

// Query and adjoint in one pass (ADJ), or the query alone on the same work
// items (the forward's env-chunked mode): the bin-search tables go to LDS as
// in k_forward, plus K keys per wavefront.
template <int DT, int LAYOUT, bool ADJ, bool PERV = false>
__device__ __forceinline__ void query_chunked_body(const BwdArgs& A, const QueryExtra& F) {
  __shared__ BinCell s_lut[kLutCells];
  __shared__ float4 s_dir4[FC_MAX_BINS];
  __shared__ unsigned long long s_keys[kBwdBlock / 64][kKeyCopies * kKeyStride];
  static_assert(sizeof(BinCell) == sizeof(uint4), "BinCell is one 16-byte load");
  static_assert(FC_MAX_BINS == 64, "one key slot per lane");
  const uint4* src = reinterpret_cast<const uint4*>(F.bin_lut);
  uint4* dst = reinterpret_cast<uint4*>(s_lut);
  for (int i = threadIdx.x; i < kLutCells; i += kBwdBlock) dst[i] = src[i];
  if (threadIdx.x < FC_MAX_BINS) {
    const int k = threadIdx.x < F.K ? threadIdx.x : 0;
    s_dir4[threadIdx.x] = make_float4(F.dirs[k], F.dirs[F.K + k], F.dirs[2 * F.K + k], 0.f);
  }
  for (int i = threadIdx.x & 63; i < kKeyCopies * kKeyStride; i += 64) s_keys[threadIdx.x >> 6][i] = 0ull;
  __syncthreads();
  backward_item<DT, LAYOUT, QueryExtra, ADJ, PERV>(A, F, s_keys[threadIdx.x >> 6], s_lut, s_dir4);
}

template <int DT, int LAYOUT, bool PERV>
__global__ __launch_bounds__(kBwdBlock) void k_query_backward(BwdArgs A, QueryExtra F) {
  query_chunked_body<DT, LAYOUT, true, PERV>(A, F);
}

template <int DT, int LAYOUT>
__global__ __launch_bounds__(kBwdBlock) void k_query_chunked(BwdArgs A, QueryExtra F) {
  query_chunked_body<DT, LAYOUT, false>(A, F);
}

// Fixed-order combine of the adjoint's partial sums.  Workgroups
// [0, pose_blocks) take one environment per wavefront: lane l sums the env's
// partial rows l, l + 64, ... in order, then the lanes are combined by the
// fixed butterfly of wave_sum8.  The remaining workgroups take one (component, vertex) per
// thread and sum the chunks in order, loads issued eight at a time.
constexpr int kCombineBatch = 8;

__device__ __forceinline__ void combine_block(const BwdArgs& A, int shared_v, long long n_vert_total,
                                             int pose_blocks, int block) {
  constexpr int NW = kBwdBlock / 64;
  if (block < pose_blocks) {
    const int e = block * 4 + (threadIdx.x >> 6);
    if (e >= A.n_env) return;  // whole wavefront leaves together
    const int lane = threadIdx.x & 63;
    const int n_rows = A.mesh_tiles[A.envs[e].gm >> 8] * NW;  // (tile, wave) rows in order
    const float2* base = A.pose_part + (long long)A.env_tile_base[e] * NW * 8;
    float2 acc[8];
#pragma unroll
    for (int v = 0; v < 8; ++v) acc[v] = make_float2(0.f, 0.f);
    for (int r = lane; r < n_rows; r += 64) {
      const float2* row = base + (long long)r * 8;
#pragma unroll
      for (int v = 0; v < 7; ++v) acc[v] = ncombine(acc[v], row[v]);
    }
    const float2 tot = wave_sum8(acc);
    const int v = wave_sum8_slot(lane);
    if (lane < 8) {
      if (v == 0) {
        if (A.loss) A.loss[e] = tot.x + tot.y;
      } else if (v < 7 && A.d_pose) {
        const float up = A.upstream ? A.upstream[e] : 1.f;
        A.d_pose[(long long)(v - 1) * A.n_env + e] = up * (tot.x + tot.y);
      }
    }
    return;
  }
  if (!shared_v) return;
  const long long jj = (long long)(block - pose_blocks) * blockDim.x + threadIdx.x;
  if (jj >= 3 * n_vert_total) return;
  const int comp = (int)(jj / n_vert_total);
  long long j = jj - (long long)comp * n_vert_total;
  int m = 0;
  while (m < A.n_meshes - 1 && j >= A.meshes[m].n) {
    j -= A.meshes[m].n;
    ++m;
  }
  const long long n = A.meshes[m].n;
  const int nc = A.mesh_nchunks[m];
  // chunks of mesh m are contiguous and each holds [3][n] partials
  const float2* p = A.vert_part + A.mesh_vpart0[m] + comp * n + j;
  const long long stride = 3 * n;
  float2 r = make_float2(0.f, 0.f);
  for (int c0 = 0; c0 < nc; c0 += kCombineBatch) {
    float2 buf[kCombineBatch];
#pragma unroll
    for (int b = 0; b < kCombineBatch; ++b) buf[b] = (c0 + b < nc) ? p[(c0 + b) * stride] : make_float2(0.f, 0.f);
#pragma unroll
    for (int b = 0; b < kCombineBatch; ++b)
      if (c0 + b < nc) r = (c0 + b == 0) ? buf[b] : ncombine(r, buf[b]);
  }
  A.d_verts[A.mesh_voff[m] + comp * n + j] = r.x + r.y;
}

__global__ __launch_bounds__(256) void k_bwd_combine(BwdArgs A, int shared_v, long long n_vert_total,
                                                     int pose_blocks) {
  combine_block(A, shared_v, n_vert_total, pose_blocks, blockIdx.x);
}

// The one pass's two tails in one launch: workgroups [0, payload_blocks)
// write the contact slots, the rest combine the adjoint's partial sums (the
// two read and write disjoint data).
template <int DT, int LAYOUT>
__global__ __launch_bounds__(256) void k_tail(FwdArgs F, BwdArgs A, int shared_v, long long n_vert_total,
                                              int pose_blocks, int payload_blocks) {
  if ((int)blockIdx.x < payload_blocks)
    payload_block<DT, LAYOUT>(F, 0, blockIdx.x);
  else
    combine_block(A, shared_v, n_vert_total, pose_blocks, blockIdx.x - payload_blocks);
}

// ---------------------------------------------------------------------------
// utilities
// ---------------------------------------------------------------------------
// zero n32 32-bit words (4-byte aligned)
__global__ void k_zero(unsigned* __restrict__ p, size_t n32) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n32; i += stride) p[i] = 0u;
}

template <typename T, int LAYOUT>
__global__ void k_to_bricks(const T* __restrict__ src, T* __restrict__ dst, int nx, int ny, int nz, int bx, int by,
                            int bz) {
  using B = BrickShape<LAYOUT>;
  constexpr int NB = B::NX * B::NY * B::NZ;
  const long long total = (long long)bx * by * bz * NB;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
    const long long brick = i / NB;
    const int local = (int)(i - brick * NB);
    const int lx = local % B::NX, ly = (local / B::NX) % B::NY, lz = local / (B::NX * B::NY);
    const int bxi = (int)(brick % bx), byi = (int)((brick / bx) % by), bzi = (int)(brick / ((long long)bx * by));
    const int x = min(bxi * (B::NX - 1) + lx, nx - 1);
    const int y = min(byi * (B::NY - 1) + ly, ny - 1);
    const int z = min(bzi * (B::NZ - 1) + lz, nz - 1);
    dst[i] = src[((long long)z * ny + y) * nx + x];
  }
}

template <int DT>
__device__ __forceinline__ float load_value(const void* __restrict__ p, long long i) {
  if constexpr (DT == kF32) {
    return static_cast<const float*>(p)[i];
  } else if constexpr (DT == kF16) {
    return __half2float(__ushort_as_half(static_cast<const unsigned short*>(p)[i]));
  } else {
    return __uint_as_float((unsigned)static_cast<const unsigned short*>(p)[i] << 16);
  }
}

// One thread per brick of 4x4x4 nodes (3x3x3 cells): stored iff a node has
// |value| <= band, nodes of both signs occur, or the brick reaches past the
// grid's last node (its corners would not all exist).
template <int DT>
__global__ void k_sparse_classify(const void* __restrict__ src, int nx, int ny, int nz, int bx, int by, int bz,
                                  float band, unsigned char* __restrict__ flags) {
  const long long total = (long long)bx * by * bz;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long b = (long long)blockIdx.x * blockDim.x + threadIdx.x; b < total; b += stride) {
    const int bxi = (int)(b % bx), byi = (int)((b / bx) % by), bzi = (int)(b / ((long long)bx * by));
    const int x0 = 3 * bxi, y0 = 3 * byi, z0 = 3 * bzi;
    unsigned char keep = (x0 + 3 > nx - 1) | (y0 + 3 > ny - 1) | (z0 + 3 > nz - 1);
    if (!keep) {
      float lo = __builtin_inff();
      bool neg = false, nonneg = false;
      for (int z = z0; z <= z0 + 3; ++z)
        for (int y = y0; y <= y0 + 3; ++y)
          for (int x = x0; x <= x0 + 3; ++x) {
            const float v = load_value<DT>(src, ((long long)z * ny + y) * nx + x);
            lo = fminf(lo, fabsf(v));
            neg |= v < 0.f;
            nonneg |= !(v < 0.f);
          }
      keep = (lo <= band) | (neg & nonneg);
    }
    flags[b] = keep;
  }
}

// pool[slot][64] = the nodes of brick list[slot] (past the grid's edge: the
// last node, never read); coarse[K][J][I] = node (3I, 3J, 3K) (clamped).
template <typename T>
__global__ void k_sparse_fill(const T* __restrict__ src, int nx, int ny, int nz, int bx, int by, int bz,
                              const int* __restrict__ list, int n_stored, T* __restrict__ pool,
                              T* __restrict__ coarse) {
  const long long n_pool = (long long)n_stored * 64;
  const long long n_coarse = (long long)(bx + 1) * (by + 1) * (bz + 1);
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n_pool + n_coarse; i += stride) {
    if (i < n_pool) {
      const long long b = list[i >> 6];
      const int local = (int)(i & 63);
      const int bxi = (int)(b % bx), byi = (int)((b / bx) % by), bzi = (int)(b / ((long long)bx * by));
      const int x = min(3 * bxi + (local & 3), nx - 1);
      const int y = min(3 * byi + ((local >> 2) & 3), ny - 1);
      const int z = min(3 * bzi + (local >> 4), nz - 1);
      pool[i] = src[((long long)z * ny + y) * nx + x];
    } else {
      const long long j = i - n_pool;
      const int I = (int)(j % (bx + 1)), J = (int)((j / (bx + 1)) % (by + 1)), K = (int)(j / ((long long)(bx + 1) * (by + 1)));
      const int x = min(3 * I, nx - 1), y = min(3 * J, ny - 1), z = min(3 * K, nz - 1);
      coarse[j] = src[((long long)z * ny + y) * nx + x];
    }
  }
}


template <int DT, int LAYOUT, int BLOCK, int VPT>
hipError_t fwd_launch(const FwdArgs& a, int persistent, int xcd, int grid, bool from_cand, hipStream_t s) {
  hipError_t e = mark(false, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_forward<DT, LAYOUT, BLOCK, VPT>), dim3(grid), dim3(BLOCK), 0, s, a, persistent,
                     from_cand ? 1 : 0, xcd);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = mark(true, s);
  if (e != hipSuccess) return e;
  if (a.o_vidx) {
    hipLaunchKernelGGL((k_payload<DT, LAYOUT>), dim3((a.n_env + 3) / 4), dim3(256), 0, s, a, from_cand ? 1 : 0);
    return hipGetLastError();
  }
  if (persistent == 2) return launch_zero(a.work_ctr, kXcds * sizeof(unsigned), s);
  return hipSuccess;
}

template <int DT, int LAYOUT, int BLOCK>
hipError_t fwd_vpt(const FwdArgs& a, int vpt, int persistent, int xcd, int grid, bool from_cand, hipStream_t s) {
  switch (vpt) {
    case 1: return fwd_launch<DT, LAYOUT, BLOCK, 1>(a, persistent, xcd, grid, from_cand, s);
    case 2: return fwd_launch<DT, LAYOUT, BLOCK, 2>(a, persistent, xcd, grid, from_cand, s);
    case 4: return fwd_launch<DT, LAYOUT, BLOCK, 4>(a, persistent, xcd, grid, from_cand, s);
  }
  return hipErrorInvalidValue;
}

template <int DT, int LAYOUT>
hipError_t fwd_block(const FwdArgs& a, int block, int vpt, int persistent, int xcd, int grid, bool from_cand,
                      hipStream_t s) {
  switch (block) {
    case 128: return fwd_vpt<DT, LAYOUT, 128>(a, vpt, persistent, xcd, grid, from_cand, s);
    case 256: return fwd_vpt<DT, LAYOUT, 256>(a, vpt, persistent, xcd, grid, from_cand, s);
    case 512: return fwd_vpt<DT, LAYOUT, 512>(a, vpt, persistent, xcd, grid, from_cand, s);
  }
  return hipErrorInvalidValue;
}

template <int DT>
hipError_t fwd_layout(const FwdArgs& a, int layout, int block, int vpt, int persistent, int xcd, int grid,
                      bool from_cand, hipStream_t s) {
  if (layout == FC_LAYOUT_BRICK)
    return fwd_block<DT, FC_LAYOUT_BRICK>(a, block, vpt, persistent, xcd, grid, from_cand, s);
  if (layout == FC_LAYOUT_SLAB)
    return fwd_block<DT, FC_LAYOUT_SLAB>(a, block, vpt, persistent, xcd, grid, from_cand, s);
  if (layout == FC_LAYOUT_SPARSE)
    return fwd_block<DT, FC_LAYOUT_SPARSE>(a, block, vpt, persistent, xcd, grid, from_cand, s);
  return fwd_block<DT, FC_LAYOUT_LINEAR>(a, block, vpt, persistent, xcd, grid, from_cand, s);
}

int bwd_grid(const BwdArgs& a) { return a.xcd ? kXcds * ((a.n_items + kXcds - 1) / kXcds) : a.n_items; }

struct CombineShape {
  int shared_v, pose_blocks;
  long long nv, vert_blocks;
};

CombineShape combine_shape(const BwdArgs& a) {
  CombineShape c;
  c.shared_v = (a.d_verts != nullptr) && !a.per_env;
  c.nv = 0;
  for (int m = 0; m < a.n_meshes; ++m) c.nv += a.meshes[m].n;
  c.pose_blocks = (a.n_env + 3) / 4;
  c.vert_blocks = c.shared_v ? (3 * c.nv + 255) / 256 : 0;
  return c;
}

hipError_t combine_launch(const BwdArgs& a, hipStream_t s) {
  const CombineShape c = combine_shape(a);
  hipLaunchKernelGGL(k_bwd_combine, dim3((unsigned)(c.pose_blocks + c.vert_blocks)), dim3(256), 0, s, a, c.shared_v,
                     c.nv, c.pose_blocks);
  return hipGetLastError();
}

template <int DT, int LAYOUT>
hipError_t bwd_launch(const BwdArgs& a, hipStream_t s) {
  hipError_t e = mark(false, s);
  if (e != hipSuccess) return e;
  if (a.per_env && a.d_verts)  // per-env vertex gradients are stored
    hipLaunchKernelGGL((k_backward<DT, LAYOUT, true>), dim3(bwd_grid(a)), dim3(kBwdBlock), 0, s, a);
  else
    hipLaunchKernelGGL((k_backward<DT, LAYOUT, false>), dim3(bwd_grid(a)), dim3(kBwdBlock), 0, s, a);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = mark(true, s);
  if (e != hipSuccess) return e;
  return combine_launch(a, s);
}

template <int DT, int LAYOUT>
hipError_t qbwd_launch(const BwdArgs& a, const QueryExtra& q, const FwdArgs& f, hipStream_t s) {
  hipError_t e = mark(false, s);
  if (e != hipSuccess) return e;
  if (a.per_env && a.d_verts)  // per-env vertex gradients are stored
    hipLaunchKernelGGL((k_query_backward<DT, LAYOUT, true>), dim3(bwd_grid(a)), dim3(kBwdBlock), 0, s, a, q);
  else
    hipLaunchKernelGGL((k_query_backward<DT, LAYOUT, false>), dim3(bwd_grid(a)), dim3(kBwdBlock), 0, s, a, q);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = mark(true, s);
  if (e != hipSuccess) return e;
  const CombineShape c = combine_shape(a);
  const int payload_blocks = (f.n_env + 3) / 4;
  hipLaunchKernelGGL((k_tail<DT, LAYOUT>), dim3((unsigned)(payload_blocks + c.pose_blocks + c.vert_blocks)),
                     dim3(256), 0, s, f, a, c.shared_v, c.nv, c.pose_blocks, payload_blocks);
  return hipGetLastError();
}

template <int DT, int LAYOUT>
hipError_t probe_launch(const BwdArgs& a, hipStream_t s) {
  hipError_t e = mark(false, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_gather_probe<DT, LAYOUT>), dim3(bwd_grid(a)), dim3(kBwdBlock), 0, s, a);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  return mark(true, s);
}

template <int DT>
hipError_t probe_layout(const BwdArgs& a, int layout, hipStream_t s) {
  if (layout == FC_LAYOUT_BRICK) return probe_launch<DT, FC_LAYOUT_BRICK>(a, s);
  if (layout == FC_LAYOUT_SLAB) return probe_launch<DT, FC_LAYOUT_SLAB>(a, s);
  if (layout == FC_LAYOUT_SPARSE) return probe_launch<DT, FC_LAYOUT_SPARSE>(a, s);
  return probe_launch<DT, FC_LAYOUT_LINEAR>(a, s);
}

template <int DT, int LAYOUT>
hipError_t qchunk_launch(const BwdArgs& a, const QueryExtra& q, const FwdArgs& f, hipStream_t s) {
  hipError_t e = mark(false, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_query_chunked<DT, LAYOUT>), dim3(bwd_grid(a)), dim3(kBwdBlock), 0, s, a, q);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = mark(true, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_payload<DT, LAYOUT>), dim3((f.n_env + 3) / 4), dim3(256), 0, s, f, 0);
  return hipGetLastError();
}

template <int DT>
hipError_t qchunk_layout(const BwdArgs& a, const QueryExtra& q, const FwdArgs& f, int layout, hipStream_t s) {
  if (layout == FC_LAYOUT_BRICK) return qchunk_launch<DT, FC_LAYOUT_BRICK>(a, q, f, s);
  if (layout == FC_LAYOUT_SLAB) return qchunk_launch<DT, FC_LAYOUT_SLAB>(a, q, f, s);
  if (layout == FC_LAYOUT_SPARSE) return qchunk_launch<DT, FC_LAYOUT_SPARSE>(a, q, f, s);
  return qchunk_launch<DT, FC_LAYOUT_LINEAR>(a, q, f, s);
}

template <int DT>
hipError_t qbwd_layout(const BwdArgs& a, const QueryExtra& q, const FwdArgs& f, int layout, hipStream_t s) {
  if (layout == FC_LAYOUT_BRICK) return qbwd_launch<DT, FC_LAYOUT_BRICK>(a, q, f, s);
  if (layout == FC_LAYOUT_SLAB) return qbwd_launch<DT, FC_LAYOUT_SLAB>(a, q, f, s);
  if (layout == FC_LAYOUT_SPARSE) return qbwd_launch<DT, FC_LAYOUT_SPARSE>(a, q, f, s);
  return qbwd_launch<DT, FC_LAYOUT_LINEAR>(a, q, f, s);
}

template <int DT>
hipError_t bwd_layout(const BwdArgs& a, int layout, hipStream_t s) {
  if (layout == FC_LAYOUT_BRICK) return bwd_launch<DT, FC_LAYOUT_BRICK>(a, s);
  if (layout == FC_LAYOUT_SLAB) return bwd_launch<DT, FC_LAYOUT_SLAB>(a, s);
  if (layout == FC_LAYOUT_SPARSE) return bwd_launch<DT, FC_LAYOUT_SPARSE>(a, s);
  return bwd_launch<DT, FC_LAYOUT_LINEAR>(a, s);
}

hipError_t bwd_dtype(const BwdArgs& a, int dtype, int layout, hipStream_t s) {
  switch (dtype) {
    case kF32: return bwd_layout<kF32>(a, layout, s);
    case kF16: return bwd_layout<kF16>(a, layout, s);
    case kBF16: return bwd_layout<kBF16>(a, layout, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace

// the lowest over both vertex-gradient modes, so the chunk (which orders the
// shared vertex sums) does not depend on the mode of a call
template <int DT, int LAYOUT>
int bwd_occupancy() {
  int r = 1 << 20;
  const auto take = [&r](const void* k) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, kBwdBlock, 0) != hipSuccess) n = 1;
    r = std::min(r, n);
  };
  take(reinterpret_cast<const void*>(k_backward<DT, LAYOUT, false>));
  take(reinterpret_cast<const void*>(k_backward<DT, LAYOUT, true>));
  take(reinterpret_cast<const void*>(k_query_backward<DT, LAYOUT, false>));
  take(reinterpret_cast<const void*>(k_query_backward<DT, LAYOUT, true>));
  return std::max(1, r);
}

// ... and the lowest over the layouts, so that it does not depend on the
// layout either: every layout of the same samples gives the same bits
template <int DT>
int bwd_occupancy_all_layouts() {
  return std::min(std::min(bwd_occupancy<DT, FC_LAYOUT_LINEAR>(), bwd_occupancy<DT, FC_LAYOUT_BRICK>()),
                  std::min(bwd_occupancy<DT, FC_LAYOUT_SLAB>(), bwd_occupancy<DT, FC_LAYOUT_SPARSE>()));
}

int backward_blocks_per_cu(int dtype) {
  switch (dtype) {
    case kF32: return bwd_occupancy_all_layouts<kF32>();
    case kF16: return bwd_occupancy_all_layouts<kF16>();
    case kBF16: return bwd_occupancy_all_layouts<kBF16>();
  }
  return 1;
}

bool forward_shape_supported(int block, int vpt) {
  return (block == 128 || block == 256 || block == 512) && (vpt == 1 || vpt == 2 || vpt == 4);
}

hipError_t launch_forward(const FwdArgs& a, int dtype, int layout, int block, int vpt, int persistent, int xcd,
                          int grid, bool from_cand, hipStream_t s, const KernelMarks* m) {
  if (persistent < 0 || persistent > 2) return hipErrorInvalidValue;  // k_forward's own modes only
  if (grid <= 0) return hipSuccess;
  const MarksScope scope(m);
  // the reduction-from-candidates pass never reads the grid: one instantiation serves every dtype
  if (from_cand) return fwd_layout<kF32>(a, FC_LAYOUT_LINEAR, block, vpt, persistent, xcd, grid, true, s);
  switch (dtype) {
    case kF32: return fwd_layout<kF32>(a, layout, block, vpt, persistent, xcd, grid, false, s);
    case kF16: return fwd_layout<kF16>(a, layout, block, vpt, persistent, xcd, grid, false, s);
    case kBF16: return fwd_layout<kBF16>(a, layout, block, vpt, persistent, xcd, grid, false, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_backward(const BwdArgs& a, int dtype, int layout, hipStream_t s, const KernelMarks* m) {
  if (a.n_items <= 0) return hipSuccess;
  const MarksScope scope(m);
  return bwd_dtype(a, dtype, layout, s);
}

hipError_t launch_query_backward(const BwdArgs& a, const QueryExtra& q, const FwdArgs& payload, int dtype, int layout,
                                 hipStream_t s, const KernelMarks* m) {
  if (a.n_items <= 0) return hipSuccess;
  const MarksScope scope(m);
  switch (dtype) {
    case kF32: return qbwd_layout<kF32>(a, q, payload, layout, s);
    case kF16: return qbwd_layout<kF16>(a, q, payload, layout, s);
    case kBF16: return qbwd_layout<kBF16>(a, q, payload, layout, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_query_chunked(const BwdArgs& a, const QueryExtra& q, const FwdArgs& payload, int dtype, int layout,
                                hipStream_t s, const KernelMarks* m) {
  if (a.n_items <= 0) return hipSuccess;
  const MarksScope scope(m);
  switch (dtype) {
    case kF32: return qchunk_layout<kF32>(a, q, payload, layout, s);
    case kF16: return qchunk_layout<kF16>(a, q, payload, layout, s);
    case kBF16: return qchunk_layout<kBF16>(a, q, payload, layout, s);
  }
  return hipErrorInvalidValue;
}

template <int DT, int LAYOUT>
hipError_t faces_launch(const FwdArgs& a, hipStream_t s) {
  hipError_t e = mark(false, s);
  if (e != hipSuccess) return e;
  if (a.n_items > 0) {  // none when no env's mesh has faces: the payload still writes empty lists
    hipLaunchKernelGGL((k_faces<DT, LAYOUT>), dim3(a.n_items), dim3(kFaceBlock), 0, s, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  e = mark(true, s);
  if (e != hipSuccess) return e;
  if (a.o_vidx) {
    hipLaunchKernelGGL((k_face_payload<DT, LAYOUT>), dim3((a.n_env + 3) / 4), dim3(256), 0, s, a);
    return hipGetLastError();
  }
  return hipSuccess;
}

template <int DT>
hipError_t faces_layout(const FwdArgs& a, int layout, hipStream_t s) {
  if (layout == FC_LAYOUT_BRICK) return faces_launch<DT, FC_LAYOUT_BRICK>(a, s);
  if (layout == FC_LAYOUT_SLAB) return faces_launch<DT, FC_LAYOUT_SLAB>(a, s);
  if (layout == FC_LAYOUT_SPARSE) return faces_launch<DT, FC_LAYOUT_SPARSE>(a, s);
  return faces_launch<DT, FC_LAYOUT_LINEAR>(a, s);
}

hipError_t launch_faces(const FwdArgs& a, int dtype, int layout, hipStream_t s, const KernelMarks* m) {
  const MarksScope scope(m);
  switch (dtype) {
    case kF32: return faces_layout<kF32>(a, layout, s);
    case kF16: return faces_layout<kF16>(a, layout, s);
    case kBF16: return faces_layout<kBF16>(a, layout, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_gather_probe(const BwdArgs& a, int dtype, int layout, hipStream_t s, const KernelMarks* m) {
  if (a.n_items <= 0) return hipSuccess;
  const MarksScope scope(m);
  switch (dtype) {
    case kF32: return probe_layout<kF32>(a, layout, s);
    case kF16: return probe_layout<kF16>(a, layout, s);
    case kBF16: return probe_layout<kBF16>(a, layout, s);
  }
  return hipErrorInvalidValue;
}

// The no-allocation forward's scratch.  In host code `scratch` names a
// host-side stand-in, not device memory: host code uses only the address
// hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

hipError_t noalloc_scratch(void** ptr) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    addr[dev] = p;
  }
  *ptr = addr[dev];
  return hipSuccess;
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t s) {
  if (bytes == 0) return hipSuccess;
  if ((bytes & 3u) || (((uintptr_t)p) & 3u)) return hipErrorInvalidValue;
  const size_t n32 = bytes / 4;
  size_t blocks = (n32 + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(256), 0, s, static_cast<unsigned*>(p), n32);
  return hipGetLastError();
}

hipError_t launch_sparse_classify(const void* src, int dtype, int nx, int ny, int nz, int bx, int by, int bz,
                                  float band, unsigned char* flags, hipStream_t s) {
  const long long total = (long long)bx * by * bz;
  long long blocks = (total + 255) / 256;
  if (blocks > 65535) blocks = 65535;
  if (blocks < 1) blocks = 1;
  switch (dtype) {
    case kF32: hipLaunchKernelGGL(k_sparse_classify<kF32>, dim3((unsigned)blocks), dim3(256), 0, s, src, nx, ny, nz, bx, by, bz, band, flags); break;
    case kF16: hipLaunchKernelGGL(k_sparse_classify<kF16>, dim3((unsigned)blocks), dim3(256), 0, s, src, nx, ny, nz, bx, by, bz, band, flags); break;
    case kBF16: hipLaunchKernelGGL(k_sparse_classify<kBF16>, dim3((unsigned)blocks), dim3(256), 0, s, src, nx, ny, nz, bx, by, bz, band, flags); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_sparse_fill(const void* src, int elem, int nx, int ny, int nz, int bx, int by, int bz,
                              const int* list, int n_stored, void* pool, void* coarse, hipStream_t s) {
  const long long total = (long long)n_stored * 64 + (long long)(bx + 1) * (by + 1) * (bz + 1);
  long long blocks = (total + 255) / 256;
  if (blocks > 65535) blocks = 65535;
  if (blocks < 1) blocks = 1;
  if (elem == 4)
    hipLaunchKernelGGL(k_sparse_fill<float>, dim3((unsigned)blocks), dim3(256), 0, s, static_cast<const float*>(src),
                       nx, ny, nz, bx, by, bz, list, n_stored, static_cast<float*>(pool), static_cast<float*>(coarse));
  else
    hipLaunchKernelGGL(k_sparse_fill<uint16_t>, dim3((unsigned)blocks), dim3(256), 0, s,
                       static_cast<const uint16_t*>(src), nx, ny, nz, bx, by, bz, list, n_stored,
                       static_cast<uint16_t*>(pool), static_cast<uint16_t*>(coarse));
  return hipGetLastError();
}

hipError_t launch_to_bricks(const void* src, void* dst, int elem, int layout, int nx, int ny, int nz, int bx, int by,
                            int bz, hipStream_t s) {
  int bnx, bny, bnz;
  brick_nodes(layout, bnx, bny, bnz);
  const long long total = (long long)bx * by * bz * bnx * bny * bnz;
  long long blocks = (total + 255) / 256;
  if (blocks > 65535) blocks = 65535;
  if (blocks < 1) blocks = 1;
  const dim3 gd((unsigned)blocks), bd(256);
  if (elem == 4) {
    const float* f = static_cast<const float*>(src);
    float* d = static_cast<float*>(dst);
    if (layout == FC_LAYOUT_SLAB)
      hipLaunchKernelGGL((k_to_bricks<float, FC_LAYOUT_SLAB>), gd, bd, 0, s, f, d, nx, ny, nz, bx, by, bz);
    else
      hipLaunchKernelGGL((k_to_bricks<float, FC_LAYOUT_BRICK>), gd, bd, 0, s, f, d, nx, ny, nz, bx, by, bz);
  } else {
    const uint16_t* f = static_cast<const uint16_t*>(src);
    uint16_t* d = static_cast<uint16_t*>(dst);
    if (layout == FC_LAYOUT_SLAB)
      hipLaunchKernelGGL((k_to_bricks<uint16_t, FC_LAYOUT_SLAB>), gd, bd, 0, s, f, d, nx, ny, nz, bx, by, bz);
    else
      hipLaunchKernelGGL((k_to_bricks<uint16_t, FC_LAYOUT_BRICK>), gd, bd, 0, s, f, d, nx, ny, nz, bx, by, bz);
  }
  return hipGetLastError();
}

}  // namespace fcimpl
