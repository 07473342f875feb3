// Device primitives shared by the HIP translation units of the query path
// (fc_kernels.hip, fc_patches.hip): pose, grid location and gather, trilinear
// value and gradient, normals, bins, reduction keys, and the optional HIP
// events around a launch's main kernel.  Everything here is inline, compiled
// with -ffp-contract=off in every unit, so every unit evaluates a query to
// the same bits.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "fc_internal.h"

namespace fcimpl {
namespace {

constexpr int kF32 = FC_F32, kF16 = FC_F16, kBF16 = FC_BF16;

// Orders a wavefront's own LDS writes (stores and atomics) before its later
// LDS reads of what other lanes wrote: release and acquire fences at
// wavefront scope around a wave barrier, so neither the compiler nor the
// memory model lets the reads move ahead of the writes.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------------------
// rigid transform (quaternion x,y,z,w -> R = I + 2w[v]x + 2[v]x^2, no renormalisation)
// ---------------------------------------------------------------------------
struct Rigid {
  float r00, r01, r02, r10, r11, r12, r20, r21, r22, tx, ty, tz;
};

__device__ __forceinline__ Rigid load_pose(const float* __restrict__ pose, int n_env, int e) {
  const float qx = pose[e], qy = pose[n_env + e], qz = pose[2 * n_env + e], qw = pose[3 * n_env + e];
  const float xx = qx * qx, yy = qy * qy, zz = qz * qz;
  const float xy = qx * qy, xz = qx * qz, yz = qy * qz;
  const float wx = qw * qx, wy = qw * qy, wz = qw * qz;
  Rigid r;
  r.r00 = 1.f - 2.f * (yy + zz);
  r.r01 = 2.f * (xy - wz);
  r.r02 = 2.f * (xz + wy);
  r.r10 = 2.f * (xy + wz);
  r.r11 = 1.f - 2.f * (xx + zz);
  r.r12 = 2.f * (yz - wx);
  r.r20 = 2.f * (xz - wy);
  r.r21 = 2.f * (yz + wx);
  r.r22 = 1.f - 2.f * (xx + yy);
  r.tx = pose[4 * n_env + e];
  r.ty = pose[5 * n_env + e];
  r.tz = pose[6 * n_env + e];
  return r;
}

__device__ __forceinline__ void transform(const Rigid& P, float x, float y, float z, float& ox, float& oy,
                                          float& oz) {
  ox = fmaf(P.r00, x, fmaf(P.r01, y, fmaf(P.r02, z, P.tx)));
  oy = fmaf(P.r10, x, fmaf(P.r11, y, fmaf(P.r12, z, P.ty)));
  oz = fmaf(P.r20, x, fmaf(P.r21, y, fmaf(P.r22, z, P.tz)));
}

// ---------------------------------------------------------------------------
// grid access
// ---------------------------------------------------------------------------
struct Cell {
  int ix, iy, iz;
  float tx, ty, tz;
  bool inside;
};

// Grid coordinate u = (x - origin)/h; inside iff 0 <= u <= n-1 on every axis;
// cell = min(floor(u), n-2); t = u - cell.
__device__ __forceinline__ Cell locate(const GridDev& g, float x, float y, float z) {
  float ux = (x - g.ox) * g.inv_h;
  float uy = (y - g.oy) * g.inv_h;
  float uz = (z - g.oz) * g.inv_h;
  Cell c;
  c.inside = (ux >= 0.f) & (ux <= (float)(g.nx - 1)) & (uy >= 0.f) & (uy <= (float)(g.ny - 1)) & (uz >= 0.f) &
             (uz <= (float)(g.nz - 1));
  if (!c.inside) ux = uy = uz = 0.f;  // also clears NaN: the gather stays in bounds
  c.ix = min((int)floorf(ux), g.nx - 2);
  c.iy = min((int)floorf(uy), g.ny - 2);
  c.iz = min((int)floorf(uz), g.nz - 2);
  c.tx = ux - (float)c.ix;
  c.ty = uy - (float)c.iy;
  c.tz = uz - (float)c.iz;
  return c;
}

// (v[0], v[1]) at p as one unaligned 8-byte (FP32) or 4-byte (FP16/BF16) load
template <int DT>
__device__ __forceinline__ float2 ld_pair(const void* __restrict__ p);

template <>
__device__ __forceinline__ float2 ld_pair<kF32>(const void* __restrict__ p) {
  float2 r;
  __builtin_memcpy(&r, p, 8);
  return r;
}
template <>
__device__ __forceinline__ float2 ld_pair<kF16>(const void* __restrict__ p) {
  unsigned u;
  __builtin_memcpy(&u, p, 4);
  return make_float2(__half2float(__ushort_as_half((unsigned short)(u & 0xffffu))),
                     __half2float(__ushort_as_half((unsigned short)(u >> 16))));
}
template <>
__device__ __forceinline__ float2 ld_pair<kBF16>(const void* __restrict__ p) {
  unsigned u;
  __builtin_memcpy(&u, p, 4);
  return make_float2(__uint_as_float(u << 16), __uint_as_float(u & 0xffff0000u));
}

// Sparse grid, brick not stored: the fine cell (lx, ly, lz) of the brick's
// 3x3x3 cells takes the values at its corners of the trilinear interpolant of
// the brick's 8 corner nodes (the coarse grid).  Trilinear interpolation
// reproduces a trilinear function exactly, so the cell's interpolant is the
// coarse one (up to FP32 rounding), value and gradient.
template <int DT>
__device__ __forceinline__ void coarse_corners(const GridDev& g, unsigned bxi, unsigned byi, unsigned bzi,
                                               unsigned lx, unsigned ly, unsigned lz, float c[8]) {
  constexpr size_t E = DT == kF32 ? 4 : 2;
  const unsigned cx = (unsigned)g.bx + 1, cxy = cx * ((unsigned)g.by + 1);
  const char* b = static_cast<const char*>(g.coarse) + (size_t)((bzi * ((unsigned)g.by + 1) + byi) * cx + bxi) * E;
  const float2 e00 = ld_pair<DT>(b);                        // y0 z0
  const float2 e10 = ld_pair<DT>(b + (size_t)cx * E);        // y1 z0
  const float2 e01 = ld_pair<DT>(b + (size_t)cxy * E);       // y0 z1
  const float2 e11 = ld_pair<DT>(b + (size_t)(cxy + cx) * E);  // y1 z1
  const auto third = [](unsigned k) { return k == 3u ? 1.f : (float)k * (1.f / 3.f); };  // k / 3
  const float fx0 = third(lx), fx1 = third(lx + 1);
  const float fy0 = third(ly), fy1 = third(ly + 1);
  const float fz0 = third(lz), fz1 = third(lz + 1);
  // along x: a[sx][y + 2z]
  const float d00 = e00.y - e00.x, d10 = e10.y - e10.x, d01 = e01.y - e01.x, d11 = e11.y - e11.x;
  const float a0[4] = {fmaf(fx0, d00, e00.x), fmaf(fx0, d10, e10.x), fmaf(fx0, d01, e01.x), fmaf(fx0, d11, e11.x)};
  const float a1[4] = {fmaf(fx1, d00, e00.x), fmaf(fx1, d10, e10.x), fmaf(fx1, d01, e01.x), fmaf(fx1, d11, e11.x)};
  // along y, then z
#pragma unroll
  for (int sx = 0; sx < 2; ++sx) {
    const float* a = sx ? a1 : a0;
    const float dy_z0 = a[1] - a[0], dy_z1 = a[3] - a[2];
    const float b00 = fmaf(fy0, dy_z0, a[0]), b10 = fmaf(fy1, dy_z0, a[0]);  // z0: y0, y1
    const float b01 = fmaf(fy0, dy_z1, a[2]), b11 = fmaf(fy1, dy_z1, a[2]);  // z1: y0, y1
    const float u0 = b01 - b00, u1 = b11 - b10;                              // along z at y0, y1
    c[sx + 0] = fmaf(fz0, u0, b00);
    c[sx + 2] = fmaf(fz0, u1, b10);
    c[sx + 4] = fmaf(fz1, u0, b00);
    c[sx + 6] = fmaf(fz1, u1, b10);
  }
}

// Corner order: c[a + 2b + 4c] = value at node (ix+a, iy+b, iz+c).
template <int DT, int LAYOUT>
__device__ __forceinline__ void gather(const GridDev& g, const Cell& cl, float c[8]) {
  // cell indexes are >= 0 and element indexes < 2^31 (checked at batch
  // creation): unsigned arithmetic, so the divisions need no sign fix-up
  unsigned i0, sy, sz;
  const unsigned ix = (unsigned)cl.ix, iy = (unsigned)cl.iy, iz = (unsigned)cl.iz;
  if constexpr (LAYOUT == FC_LAYOUT_LINEAR) {
    sy = (unsigned)g.nx;
    sz = (unsigned)g.nx * (unsigned)g.ny;
    i0 = (iz * (unsigned)g.ny + iy) * (unsigned)g.nx + ix;
  } else if constexpr (LAYOUT == FC_LAYOUT_SPARSE) {
    const unsigned bxi = ix / 3u, byi = iy / 3u, bzi = iz / 3u;
    const unsigned lx = ix - 3u * bxi, ly = iy - 3u * byi, lz = iz - 3u * bzi;
    const int slot = g.map[(bzi * (unsigned)g.by + byi) * (unsigned)g.bx + bxi];
    if (slot < 0) {
      coarse_corners<DT>(g, bxi, byi, bzi, lx, ly, lz, c);
      return;
    }
    sy = 4;
    sz = 16;
    i0 = (unsigned)slot * 64u + (lz * 16u + ly * 4u + lx);
  } else {
    using B = BrickShape<LAYOUT>;
    constexpr unsigned CX = B::NX - 1, CY = B::NY - 1, CZ = B::NZ - 1;
    const unsigned bxi = ix / CX, byi = iy / CY, bzi = iz / CZ;
    const unsigned lx = ix - CX * bxi, ly = iy - CY * byi, lz = iz - CZ * bzi;
    sy = B::NX;
    sz = B::NX * B::NY;
    i0 = ((bzi * (unsigned)g.by + byi) * (unsigned)g.bx + bxi) * (B::NX * B::NY * B::NZ) + (lz * sz + ly * sy + lx);
  }
  // one 64-bit base per query; the other rows at constant offsets (bricks)
  constexpr size_t E = DT == kF32 ? 4 : 2;
  const char* b = static_cast<const char*>(g.data) + (size_t)i0 * E;
  const float2 p00 = ld_pair<DT>(b);
  const float2 p10 = ld_pair<DT>(b + (size_t)sy * E);
  const float2 p01 = ld_pair<DT>(b + (size_t)sz * E);
  const float2 p11 = ld_pair<DT>(b + (size_t)(sz + sy) * E);
  c[0] = p00.x; c[1] = p00.y;
  c[2] = p10.x; c[3] = p10.y;
  c[4] = p01.x; c[5] = p01.y;
  c[6] = p11.x; c[7] = p11.y;
}

// Trilinear value and its exact gradient in grid units (multiply by 1/h for
// metres): phi = sum W_a(tx) W_b(ty) W_c(tz) C_abc, evaluated as nested lerps.
__device__ __forceinline__ void trilinear(const float c[8], float tx, float ty, float tz, float& phi, float& gx,
                                          float& gy, float& gz) {
  const float dx00 = c[1] - c[0], dx10 = c[3] - c[2], dx01 = c[5] - c[4], dx11 = c[7] - c[6];
  const float a00 = fmaf(tx, dx00, c[0]);
  const float a10 = fmaf(tx, dx10, c[2]);
  const float a01 = fmaf(tx, dx01, c[4]);
  const float a11 = fmaf(tx, dx11, c[6]);
  const float dy0 = a10 - a00, dy1 = a11 - a01;
  const float b0 = fmaf(ty, dy0, a00);
  const float b1 = fmaf(ty, dy1, a01);
  const float dz = b1 - b0;
  phi = fmaf(tz, dz, b0);
  gz = dz;
  gy = fmaf(tz, dy1 - dy0, dy0);
  const float e0 = fmaf(ty, dx10 - dx00, dx00);
  const float e1 = fmaf(ty, dx11 - dx01, dx01);
  gx = fmaf(tz, e1 - e0, e0);
}

template <int DT, int LAYOUT>
__device__ __forceinline__ void sample(const GridDev& g, float x, float y, float z, float& phi, float& gx, float& gy,
                                       float& gz, bool& inside) {
  const Cell cl = locate(g, x, y, z);
  float c[8];
  gather<DT, LAYOUT>(g, cl, c);
  trilinear(c, cl.tx, cl.ty, cl.tz, phi, gx, gy, gz);
  inside = cl.inside;
}

__device__ __forceinline__ void normalize(float gx, float gy, float gz, float& nx, float& ny, float& nz) {
  const float l2 = fmaf(gx, gx, fmaf(gy, gy, gz * gz));
  if (l2 > 0.f) {
    const float r = rsqrtf(l2);
    nx = gx * r;
    ny = gy * r;
    nz = gz * r;
  } else {
    nx = ny = nz = 0.f;
  }
}

// lowest k maximising n . d_k
__device__ __forceinline__ int argmax_bin(const float* __restrict__ dirs, int K, float nx, float ny, float nz) {
  float best = fmaf(nz, dirs[2 * K], fmaf(ny, dirs[K], nx * dirs[0]));
  int bin = 0;
  for (int k = 1; k < K; ++k) {
    const float d = fmaf(nz, dirs[2 * K + k], fmaf(ny, dirs[K + k], nx * dirs[k]));
    if (d > best) {
      best = d;
      bin = k;
    }
  }
  return bin;
}

// Cube-map cell of a nonzero normal (see BinCell): the dominant axis picks the
// face, the other two components divided by it give (u, v) in [-1, 1].
__device__ __forceinline__ int cube_cell(float nx, float ny, float nz) {
  const float ax = fabsf(nx), ay = fabsf(ny), az = fabsf(nz);
  // x face if x dominates, else y if y dominates z, else z (selects, no branches)
  const bool fx = (ax >= ay) & (ax >= az);
  const bool fy = !fx & (ay >= az);
  const int axis = fx ? 0 : (fy ? 1 : 2);
  const float comp = fx ? nx : (fy ? ny : nz);
  const int face = 2 * axis + (comp >= 0.f ? 0 : 1);
  const float u = fx ? ny : nx;
  const float v = (fx | fy) ? nz : ny;
  const float m = fx ? ax : (fy ? ay : az);
  // hardware reciprocal (1 ulp): the table's cones carry a 1e-4 rad margin
  // for the cell choice, far above this rounding
  const float s = (0.5f * kLutN) * __builtin_amdgcn_rcpf(m);
  const int iu = min(max((int)floorf(fmaf(u, s, 0.5f * kLutN)), 0), kLutN - 1);
  const int iv = min(max((int)floorf(fmaf(v, s, 0.5f * kLutN)), 0), kLutN - 1);
  return (face * kLutN + iv) * kLutN + iu;
}

// The same argmax as argmax_bin (same dot products, same lowest-k tie rule),
// evaluated only over the bins the normal's cube-map cell lists.  The table
// is built so that every bin that can reach the maximum for a normal in the
// cell is listed, so the result is identical.
__device__ __forceinline__ int argmax_bin_lut(const BinCell* __restrict__ lut, const float4* __restrict__ dir4,
                                              const float* __restrict__ dirs, int K, float nx, float ny,
                                              float nz) {
  if ((nx == 0.f) & (ny == 0.f) & (nz == 0.f)) return 0;
  // the cell's 16 bytes (n, k[0..14]) in four registers; the loop is unrolled
  // so every byte index is a constant (no private-array indexing)
  const uint4 cw = *reinterpret_cast<const uint4*>(&lut[cube_cell(nx, ny, nz)]);
  const unsigned w[4] = {cw.x, cw.y, cw.z, cw.w};
  const int n = (int)(w[0] & 0xffu);
  if (n == kLutFull) return argmax_bin(dirs, K, nx, ny, nz);
  int bin = (int)((w[0] >> 8) & 0xffu);
  float4 d = dir4[bin];
  float best = fmaf(nz, d.z, fmaf(ny, d.y, nx * d.x));
  // entries 1..kLutEager - 1 for every lane, kept only where the list has
  // them (an absent entry reads byte 0, bin 0, and is never taken); the
  // rest, which few cells have, behind a branch the wavefront takes together
  constexpr int kLutEager = 4;
#pragma unroll
  for (int i = 1; i < kLutEager; ++i) {
    const int b = i + 1;  // byte of k[i]
    const int k = (int)((w[b >> 2] >> ((b & 3) * 8)) & 0xffu);
    d = dir4[k];
    const float v = fmaf(nz, d.z, fmaf(ny, d.y, nx * d.x));
    const bool take = (i < n) & (v > best);
    best = take ? v : best;
    bin = take ? k : bin;
  }
  if (__ballot(n > kLutEager) != 0ull) {
#pragma unroll
    for (int i = kLutEager; i < kLutMax; ++i) {
      if (i < n) {
        const int b = i + 1;
        const int k = (int)((w[b >> 2] >> ((b & 3) * 8)) & 0xffu);
        d = dir4[k];
        const float v = fmaf(nz, d.z, fmaf(ny, d.y, nx * d.x));
        if (v > best) {
          best = v;
          bin = k;
        }
      }
    }
  }
  return bin;
}

// ---------------------------------------------------------------------------
// reduction keys: (sortable depth << 32) | (0xFFFFFFFF - vidx); max = deepest,
// then lowest index.  -0.0 is folded to +0.0; key 0 means "empty".
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned long long make_key(float depth, unsigned vidx) {
  if (depth == 0.f) depth = 0.f;
  unsigned u = __float_as_uint(depth);
  u = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
  return ((unsigned long long)u << 32) | (unsigned long long)(0xFFFFFFFFu - vidx);
}

__device__ __forceinline__ float key_depth(unsigned long long key) {
  unsigned u = (unsigned)(key >> 32);
  u = (u & 0x80000000u) ? (u & 0x7FFFFFFFu) : ~u;
  return __uint_as_float(u);
}

__device__ __forceinline__ unsigned key_vidx(unsigned long long key) { return 0xFFFFFFFFu - (unsigned)key; }

// Optional HIP events around the main kernel of the launch in progress (set
// by the launch_* entry points for the calling thread; see KernelMarks).
thread_local const KernelMarks* t_marks = nullptr;

struct MarksScope {
  explicit MarksScope(const KernelMarks* m) { t_marks = m; }
  ~MarksScope() { t_marks = nullptr; }
};

hipError_t mark(bool after, hipStream_t s) {
  if (!t_marks) return hipSuccess;
  return hipEventRecord(after ? static_cast<hipEvent_t>(t_marks->after) : static_cast<hipEvent_t>(t_marks->before),
                        s);
}

}  // namespace
}  // namespace fcimpl
