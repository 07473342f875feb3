// HIP kernel for gfx950 (CDNA4): the patch-based contact reduction of
// Narang et al. (Factory, RSS 2022), Section III-C, Algorithm 1: per shape
// pair, for each batch of 1024 features, Generate candidates, Assign them to
// existing patches by normal similarity, then FindDeepest / BinReduce /
// AddPatch until none remain -- in LDS, as the paper does in shared memory.
//
// Numerics: compiled with -ffp-contract=off; the candidates are the vertex
// queries of fc_device.h, bit for bit; the similarity dot has no fused
// multiply-add, so a CPU evaluation in FP32 takes the same decisions.
#include "fc_device.h"

namespace fcimpl {
namespace {

// ---------------------------------------------------------------------------
// patch reduction (Algorithm 1)
// ---------------------------------------------------------------------------
// FP32 dot without fused multiply-adds: (a.x b.x + a.y b.y) + a.z b.z (the
// file is compiled with -ffp-contract=off).
__device__ __forceinline__ float dot3_nofma(float ax, float ay, float az, float bx, float by, float bz) {
  return (ax * bx + ay * by) + az * bz;
}

// Wave-wide reductions on the data-parallel primitives instead of LDS
// permutes: DPP quad xor 1 and xor 2, the 8-lane and 16-lane mirrors (with
// every lane of a group holding the group's result, a mirror pairs the two
// halves), a ds_swizzle xor 16, then lanes 0 and 32 read as scalars.  The
// result is the same in every lane.
template <int CTRL>
__device__ __forceinline__ unsigned dpp_u32(unsigned v) {
  return (unsigned)__builtin_amdgcn_mov_dpp((int)v, CTRL, 0xF, 0xF, false);
}
__device__ __forceinline__ unsigned swz16_u32(unsigned v) {
  return (unsigned)__builtin_amdgcn_ds_swizzle((int)v, 0x401F);  // bit mode: lane i <- lane i ^ 16
}
__device__ __forceinline__ unsigned long long join64(unsigned lo, unsigned hi) {
  return ((unsigned long long)hi << 32) | lo;
}
__device__ __forceinline__ unsigned long long max64_with(unsigned long long v, unsigned lo, unsigned hi) {
  const unsigned long long w = join64(lo, hi);
  return w > v ? w : v;
}
template <int CTRL>
__device__ __forceinline__ unsigned long long max64_dpp(unsigned long long v) {
  return max64_with(v, dpp_u32<CTRL>((unsigned)v), dpp_u32<CTRL>((unsigned)(v >> 32)));
}
__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
  v = max64_dpp<0xB1>(v);   // quad_perm [1,0,3,2]
  v = max64_dpp<0x4E>(v);   // quad_perm [2,3,0,1]
  v = max64_dpp<0x141>(v);  // lane i <- lane 7-i within each 8 lanes
  v = max64_dpp<0x140>(v);  // lane i <- lane 15-i within each row
  v = max64_with(v, swz16_u32((unsigned)v), swz16_u32((unsigned)(v >> 32)));
  const unsigned long long a = join64((unsigned)__builtin_amdgcn_readlane((int)(unsigned)v, 0),
                                      (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(v >> 32), 0));
  const unsigned long long b = join64((unsigned)__builtin_amdgcn_readlane((int)(unsigned)v, 32),
                                      (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(v >> 32), 32));
  return a > b ? a : b;
}

__device__ __forceinline__ int wave_sum_i32(int v) {
  v += (int)dpp_u32<0xB1>((unsigned)v);
  v += (int)dpp_u32<0x4E>((unsigned)v);
  v += (int)dpp_u32<0x141>((unsigned)v);
  v += (int)dpp_u32<0x140>((unsigned)v);
  v += (int)swz16_u32((unsigned)v);
  return __builtin_amdgcn_readlane(v, 0) + __builtin_amdgcn_readlane(v, 32);
}

// (d, p) with the largest d, the lowest p on ties
__device__ __forceinline__ void wave_argmax(float& d, int& p) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const float d2 = __shfl_xor(d, o);
    const int p2 = __shfl_xor(p, o);
    if (d2 > d || (d2 == d && p2 < p)) {
      d = d2;
      p = p2;
    }
  }
}

// One workgroup per environment.  For each batch of 1024 vertices: Generate
// the candidates (the vertex query's values, bit for bit) and compact them in
// LDS; Assign each to the most similar patch that existed when the batch
// began (all waves; member counts and deepest keys are order-independent LDS
// atomics); then one wave repeats FindDeepest / BinReduce / AddPatch until no
// candidate remains.  Patches live in LDS.
template <int DT, int LAYOUT>
__global__ __launch_bounds__(kPatchBlock) void k_patches(FwdArgs A, PatchArgs P) {
  __shared__ float s_pn[kPatchMax][3];
  __shared__ unsigned long long s_pkey[kPatchMax];
  __shared__ int s_pmem[kPatchMax];
  __shared__ int s_pfound[kPatchMax];
  __shared__ int s_np;
  __shared__ unsigned long long s_ck[kPatchBatch];  // the batch's candidates, compacted
  __shared__ float s_cn[kPatchBatch][3];
  __shared__ int s_nc;

  const int e = blockIdx.x;
  const int gm = A.envs[e].gm;
  const GridDev& g = A.grids[gm & 0xff];
  const MeshDev& m = A.meshes[gm >> 8];
  const Rigid R = load_pose(A.pose, A.n_env, e);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const float cs = P.cos_sim;
  if (tid == 0) s_np = 0;
  __syncthreads();

  for (int b0 = 0; b0 < m.n; b0 += kPatchBatch) {
    if (tid == 0) s_nc = 0;
    __syncthreads();
    // Generate, then compact the candidates into LDS: every later step is
    // independent of their order, and each thread then holds ceil(nc / 256)
    // of them instead of 4 vertices mostly without a candidate
    unsigned long long key[kPatchVpt];
    float nx[kPatchVpt], ny[kPatchVpt], nz[kPatchVpt];
    bool live[kPatchVpt];
    {
      float px[kPatchVpt], py[kPatchVpt], pz[kPatchVpt];
      bool ok[kPatchVpt];
#pragma unroll
      for (int j = 0; j < kPatchVpt; ++j) {
        const int v = b0 + j * kPatchBlock + tid;
        ok[j] = v < m.n;
        float x = 0.f, y = 0.f, z = 0.f;
        if (ok[j]) {
          x = m.x[v];
          y = m.y[v];
          z = m.z[v];
        }
        transform(R, x, y, z, px[j], py[j], pz[j]);
      }
      Cell cl[kPatchVpt];
      float c[kPatchVpt][8];
#pragma unroll
      for (int j = 0; j < kPatchVpt; ++j) cl[j] = locate(g, px[j], py[j], pz[j]);
#pragma unroll
      for (int j = 0; j < kPatchVpt; ++j) gather<DT, LAYOUT>(g, cl[j], c[j]);
#pragma unroll
      for (int j = 0; j < kPatchVpt; ++j) {
        float phi, gx, gy, gz;
        trilinear(c[j], cl[j].tx, cl[j].ty, cl[j].tz, phi, gx, gy, gz);
        if (ok[j] & cl[j].inside & (phi < A.margin)) {
          float ux, uy, uz;
          normalize(gx, gy, gz, ux, uy, uz);
          const int pos = atomicAdd(&s_nc, 1);
          s_ck[pos] = make_key(-phi, (unsigned)(b0 + j * kPatchBlock + tid));
          s_cn[pos][0] = ux;
          s_cn[pos][1] = uy;
          s_cn[pos][2] = uz;
        }
      }
    }
    __syncthreads();
    {
      const int nc = s_nc;
#pragma unroll
      for (int j = 0; j < kPatchVpt; ++j) {
        const int i = j * kPatchBlock + tid;
        live[j] = i < nc;
        key[j] = 0ull;
        nx[j] = ny[j] = nz[j] = 0.f;
        if (live[j]) {
          key[j] = s_ck[i];
          nx[j] = s_cn[i][0];
          ny[j] = s_cn[i][1];
          nz[j] = s_cn[i][2];
        }
      }
    }
    // Assign, against the patches present as the batch begins.  The first
    // patch of largest dot over all patches is the patch of largest dot
    // among the similar ones (lowest index on ties) whenever it is similar
    // itself, and no patch is similar otherwise.
    const int np0 = s_np;
#pragma unroll
    for (int j = 0; j < kPatchVpt; ++j) {
      if (!live[j]) continue;
      int best = -1;
      float bd = -INFINITY;
      for (int p = 0; p < np0; ++p) {
        const float d = dot3_nofma(nx[j], ny[j], nz[j], s_pn[p][0], s_pn[p][1], s_pn[p][2]);
        if (d > bd) {
          best = p;
          bd = d;
        }
      }
      if ((best >= 0) & (bd >= cs)) {
        atomicAdd(&s_pmem[best], 1);
        atomicMax(&s_pkey[best], key[j]);
        s_ck[j * kPatchBlock + tid] = 0ull;  // assigned: out of the loop below
      }
    }
    __syncthreads();
    // FindDeepest / BinReduce / AddPatch while candidates remain: one wave,
    // no workgroup barrier per patch.  Each lane owns the compacted entries
    // i = lane (mod 64) and is the only one to clear them; lane 0 writes the
    // patch list, which the wave reads back after a wave barrier.
    // The BinReduce pass visits every entry that is left after it, so it
    // also finds the next FindDeepest's lane maxima: one pass per patch.
    if (wave == 0) {
      const int nc = s_nc;
      int np = s_np;
      unsigned long long mk = 0ull;
      int mi = -1;
      for (int i = lane; i < nc; i += 64) {
        const unsigned long long k = s_ck[i];
        if (k > mk) {
          mk = k;
          mi = i;
        }
      }
      for (;;) {
        const unsigned long long best = wave_max_u64(mk);
        if (best == 0ull) break;  // the same value in every lane
        // the owner's normal, broadcast (keys are unique: one owner lane)
        const unsigned long long own = __ballot(mk == best);
        const int ol = __ffsll((long long)own) - 1;
        float ox = 0.f, oy = 0.f, oz = 0.f;
        if (mk == best) {
          ox = s_cn[mi][0];
          oy = s_cn[mi][1];
          oz = s_cn[mi][2];
        }
        const float bx = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(ox), ol));
        const float by = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(oy), ol));
        const float bz = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(oz), ol));
        int cnt = 0;
        mk = 0ull;
        mi = -1;
        for (int i = lane; i < nc; i += 64) {
          const unsigned long long k = s_ck[i];
          if (k == 0ull) continue;
          if (k == best || dot3_nofma(bx, by, bz, s_cn[i][0], s_cn[i][1], s_cn[i][2]) >= cs) {
            ++cnt;
            s_ck[i] = 0ull;
          } else if (k > mk) {  // remains: a candidate for the next FindDeepest
            mk = k;
            mi = i;
          }
        }
        const int members = wave_sum_i32(cnt);
        int slot = -1;
        if (np < P.n_max) {
          slot = np++;
        } else {  // the most similar existing patch, lowest index on ties
          float d = -__builtin_inff();
          int pj = 0x7fffffff;
          for (int q = lane; q < np; q += 64) {
            const float dq = dot3_nofma(bx, by, bz, s_pn[q][0], s_pn[q][1], s_pn[q][2]);
            if (dq > d) {  // ascending q: the first maximum stays
              d = dq;
              pj = q;
            }
          }
          wave_argmax(d, pj);
          if ((float)members * key_depth(best) > (float)s_pmem[pj] * key_depth(s_pkey[pj])) slot = pj;
        }
        if (slot >= 0 && lane == 0) {
          s_pn[slot][0] = bx;
          s_pn[slot][1] = by;
          s_pn[slot][2] = bz;
          s_pkey[slot] = best;
          s_pmem[slot] = members;
          s_pfound[slot] = (int)key_vidx(best);
        }
        wave_lds_sync();
      }
      if (lane == 0) s_np = np;
    }
    __syncthreads();
  }
  // the patch list, each with its deepest member's record
  const int np = s_np;
  if (tid == 0) P.count[e] = np;
  const long long S = (long long)A.n_env * P.n_max;
  for (int p = tid; p < P.n_max; p += kPatchBlock) {
    const long long s = (long long)e * P.n_max + p;
    if (p < np) {
      const unsigned v = key_vidx(s_pkey[p]);
      float xb, yb, zb;
      transform(R, m.x[v], m.y[v], m.z[v], xb, yb, zb);
      P.founder[s] = s_pfound[p];
      P.vidx[s] = (int)v;
      P.depth[s] = key_depth(s_pkey[p]);
      P.members[s] = s_pmem[p];
      P.normal[s] = s_pn[p][0];
      P.normal[S + s] = s_pn[p][1];
      P.normal[2 * S + s] = s_pn[p][2];
      P.point[s] = xb;
      P.point[S + s] = yb;
      P.point[2 * S + s] = zb;
    } else {
      P.founder[s] = -1;
      P.vidx[s] = -1;
      P.depth[s] = 0.f;
      P.members[s] = 0;
      P.normal[s] = P.normal[S + s] = P.normal[2 * S + s] = 0.f;
      P.point[s] = P.point[S + s] = P.point[2 * S + s] = 0.f;
    }
  }
}

}  // namespace

template <int DT, int LAYOUT>
hipError_t patches_launch(const FwdArgs& a, const PatchArgs& p, hipStream_t s) {
  hipError_t e = mark(false, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_patches<DT, LAYOUT>), dim3(a.n_env), dim3(kPatchBlock), 0, s, a, p);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  return mark(true, s);
}

template <int DT>
hipError_t patches_layout(const FwdArgs& a, const PatchArgs& p, int layout, hipStream_t s) {
  if (layout == FC_LAYOUT_BRICK) return patches_launch<DT, FC_LAYOUT_BRICK>(a, p, s);
  if (layout == FC_LAYOUT_SLAB) return patches_launch<DT, FC_LAYOUT_SLAB>(a, p, s);
  if (layout == FC_LAYOUT_SPARSE) return patches_launch<DT, FC_LAYOUT_SPARSE>(a, p, s);
  return patches_launch<DT, FC_LAYOUT_LINEAR>(a, p, s);
}

hipError_t launch_patches(const FwdArgs& a, const PatchArgs& p, int dtype, int layout, hipStream_t s,
                          const KernelMarks* m) {
  if (a.n_env <= 0) return hipSuccess;
  const MarksScope scope(m);
  switch (dtype) {
    case kF32: return patches_layout<kF32>(a, p, layout, s);
    case kF16: return patches_layout<kF16>(a, p, layout, s);
    case kBF16: return patches_layout<kBF16>(a, p, layout, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace fcimpl
