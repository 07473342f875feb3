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

// Wave-wide reductions on the data-parallel primitives: DPP quad xor 1 and
// xor 2, then the 8-lane and 16-lane mirrors (with every lane of a group
// holding the group's result, a mirror pairs the two halves), which leaves
// each 16-lane row's result in all its lanes; the four rows are then read as
// scalars.  A 64-bit maximum takes the high words' maximum first, then, if
// several lanes hold it, the low words of those lanes.  The result is the
// same in every lane.
template <int CTRL>
__device__ __forceinline__ unsigned dpp_u32(unsigned v) {
  return (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, true);
}
__device__ __forceinline__ unsigned long long join64(unsigned lo, unsigned hi) {
  return ((unsigned long long)hi << 32) | lo;
}
__device__ __forceinline__ unsigned umax(unsigned a, unsigned b) { return a > b ? a : b; }
__device__ __forceinline__ unsigned row_max_u32(unsigned v) {
  v = umax(v, dpp_u32<0xB1>(v));   // quad_perm [1,0,3,2]
  v = umax(v, dpp_u32<0x4E>(v));   // quad_perm [2,3,0,1]
  v = umax(v, dpp_u32<0x141>(v));  // lane i <- lane 7-i within each 8 lanes
  return umax(v, dpp_u32<0x140>(v));  // lane i <- lane 15-i within each row
}
__device__ __forceinline__ unsigned wave_max_u32(unsigned v) {
  v = row_max_u32(v);
  const unsigned a = (unsigned)__builtin_amdgcn_readlane((int)v, 0), b = (unsigned)__builtin_amdgcn_readlane((int)v, 16);
  const unsigned c = (unsigned)__builtin_amdgcn_readlane((int)v, 32), d = (unsigned)__builtin_amdgcn_readlane((int)v, 48);
  return umax(umax(a, b), umax(c, d));
}

__device__ __forceinline__ int wave_sum_i32(int v) {
  v += (int)dpp_u32<0xB1>((unsigned)v);
  v += (int)dpp_u32<0x4E>((unsigned)v);
  v += (int)dpp_u32<0x141>((unsigned)v);
  v += (int)dpp_u32<0x140>((unsigned)v);
  return (__builtin_amdgcn_readlane(v, 0) + __builtin_amdgcn_readlane(v, 16)) +
         (__builtin_amdgcn_readlane(v, 32) + __builtin_amdgcn_readlane(v, 48));
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

// One workgroup per environment.  Per batch of kPatchBatch vertices:
//   Generate  every wave evaluates kPatchVpt vertex queries per thread (the
//             vertex query's values, bit for bit) and compacts the batch's
//             candidates into LDS;
//   Assign    each candidate joins the most similar patch of the list as it
//             stands after every earlier batch (member counts and deepest
//             keys by order-independent LDS atomics); the unassigned ones
//             are packed to the front of the buffer (rank by ballot within
//             a wave, by the waves' counts across them);
//   loop      the unassigned entries are dealt to the waves' registers (row
//             r of 64 to wave r mod 4); per patch each wave finds its
//             deepest entry, one barrier exchanges the four, every wave
//             takes the deepest of them (FindDeepest), removes its entries
//             similar to it (BinReduce) while finding its next deepest, and
//             the patch is added with its member count summed by LDS
//             atomics (AddPatch).  The per-wave records alternate between
//             two LDS slots, so one barrier per patch suffices.  A batch
//             with at most 64 unassigned entries and room for a patch per
//             entry (most batches after the first) runs the loop on wave 0
//             alone, with no barrier.
// The waves of the workgroups sharing a compute unit take the SIMDs by
// phase: the loop (a chain of short dependent steps) at the highest wave
// priority, Assign next, Generate (the gather and evaluation, which the
// others' gaps absorb) last.  Scheduling only; the results do not depend
// on it.
template <int DT, int LAYOUT>
__global__ __launch_bounds__(kPatchThreads) void k_patches(FwdArgs A, PatchArgs P) {
  constexpr int kWaves = kPatchThreads / 64;
  constexpr int kRows = kPatchBatch / 64;
  constexpr int kSlots = kRows / kWaves;  // register rows per wave
  static_assert(kRows % kWaves == 0, "rows deal evenly to the waves");
  constexpr int kAsg = kPatchBatch / kPatchThreads;  // Assign entries per thread
  static_assert(kPatchBatch % kPatchThreads == 0, "Assign covers the buffer");
  __shared__ float s_pn[kPatchMax][3];
  __shared__ unsigned long long s_pkey[kPatchMax];
  __shared__ int s_pmem[kPatchMax];
  __shared__ int s_pfound[kPatchMax];
  __shared__ unsigned long long s_ck[kPatchBatch];  // the batch's candidates, compacted
  __shared__ float s_cn[kPatchBatch][3];
  __shared__ int s_nc;
  __shared__ int s_wcnt[kAsg][kWaves];  // unassigned entries per (Assign slot, wave)
  __shared__ uint4 s_red[2][kWaves];    // each wave's deepest entry: key (x, y), normal x, y (z: s_redz)
  __shared__ float s_redz[2][kWaves];
  __shared__ int s_members[2];          // a replaced patch's member count
  __shared__ int s_np;                  // the patch count, for the waves that sat out a batch's loop

  const int e = blockIdx.x;
  const int gm = A.envs[e].gm;
  const GridDev& g = A.grids[gm & 0xff];
  const MeshDev& m = A.meshes[gm >> 8];
  const Rigid R = load_pose(A.pose, A.n_env, e);
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const float cs = P.cos_sim;
  for (int p = tid; p < kPatchMax; p += kPatchThreads) s_pmem[p] = 0;  // new patches' counts are summed in
  if (tid < 2) s_members[tid] = 0;
  int np = 0;   // patches (the same in every thread)
  int par = 0;  // LDS record slot of the current patch step

  for (int b0 = 0; b0 < m.n; b0 += kPatchBatch) {
    __builtin_amdgcn_s_setprio(0);  // Generate
    if (tid == 0) s_nc = 0;
    __syncthreads();
    if (b0 > 0) np = s_np;  // written by thread 0 at the end of the previous batch
    // Generate
    {
      float px[kPatchVpt], py[kPatchVpt], pz[kPatchVpt];
      bool ok[kPatchVpt];
#pragma unroll
      for (int j = 0; j < kPatchVpt; ++j) {
        const int v = b0 + j * kPatchThreads + tid;
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
          s_ck[pos] = make_key(-phi, (unsigned)(b0 + j * kPatchThreads + tid));
          s_cn[pos][0] = ux;
          s_cn[pos][1] = uy;
          s_cn[pos][2] = uz;
        }
      }
    }
    __syncthreads();
    __builtin_amdgcn_s_setprio(1);  // Assign
    const int nc = s_nc;
    // Assign, against the patch list as it stands.  The first patch of
    // largest dot over all patches is the patch of largest dot among the
    // similar ones (lowest index on ties) whenever it is similar itself, and
    // no patch is similar otherwise.
    unsigned long long ak[kAsg];
    float ax[kAsg], ay[kAsg], az[kAsg];
    bool un[kAsg];  // unassigned: goes on to the loop
    const int np0 = __builtin_amdgcn_readfirstlane(np);
#pragma unroll
    for (int j = 0; j < kAsg; ++j) {
      const int i = j * kPatchThreads + tid;
      ak[j] = 0ull;
      ax[j] = ay[j] = az[j] = 0.f;
      un[j] = false;
      if (i < nc) {
        ak[j] = s_ck[i];
        ax[j] = s_cn[i][0];
        ay[j] = s_cn[i][1];
        az[j] = s_cn[i][2];
        int best = -1;
        float bd = -INFINITY;
        for (int p = 0; p < np0; ++p) {
          const float d = dot3_nofma(ax[j], ay[j], az[j], s_pn[p][0], s_pn[p][1], s_pn[p][2]);
          if (d > bd) {
            best = p;
            bd = d;
          }
        }
        if ((best >= 0) & (bd >= cs)) {
          atomicAdd(&s_pmem[best], 1);
          atomicMax(&s_pkey[best], ak[j]);
        } else {
          un[j] = true;
        }
      }
      const unsigned long long bal = __ballot(un[j]);
      if (lane == 0) s_wcnt[j][wave] = __popcll(bal);
    }
    __syncthreads();  // every entry read; the counts known
    // pack the unassigned entries to the front, in (slot, wave, lane) order
    int u = 0;
    {
      int base = 0;
#pragma unroll
      for (int j = 0; j < kAsg; ++j) {
        const unsigned long long bal = __ballot(un[j]);
        int before = base;
        for (int w = 0; w < wave; ++w) before += s_wcnt[j][w];
        for (int w = 0; w < kWaves; ++w) base += s_wcnt[j][w];
        if (un[j]) {
          const int pos = before + (int)__builtin_amdgcn_mbcnt_hi((unsigned)(bal >> 32),
                                                                  __builtin_amdgcn_mbcnt_lo((unsigned)bal, 0u));
          s_ck[pos] = ak[j];
          s_cn[pos][0] = ax[j];
          s_cn[pos][1] = ay[j];
          s_cn[pos][2] = az[j];
        }
      }
      u = base;
    }
    if (u == 0) {  // the same in every thread: nothing left for the loop
      if (tid == 0) s_np = np;
      continue;
    }
    __syncthreads();
    __builtin_amdgcn_s_setprio(2);  // the loop
    if ((u <= 64) & (np + u <= P.n_max)) {
      // Few entries and no replacement possible (each pass adds one patch):
      // wave 0 holds them all in one row and runs the loop alone, with no
      // exchange or barrier per patch; the other waves go on to the next
      // batch's barrier.  The same decisions as the four-wave loop.
      if (wave == 0) {
        unsigned long long k = lane < u ? s_ck[lane] : 0ull;
        const float x = lane < u ? s_cn[lane][0] : 0.f, y = lane < u ? s_cn[lane][1] : 0.f,
                    z = lane < u ? s_cn[lane][2] : 0.f;
        for (;;) {
          const unsigned hi = wave_max_u32((unsigned)(k >> 32));
          unsigned long long own = __ballot((unsigned)(k >> 32) == hi);
          if (__popcll(own) != 1) {
            const unsigned lo = wave_max_u32((unsigned)(k >> 32) == hi ? (unsigned)k : 0u);
            own = __ballot(k == join64(lo, hi));
          }
          const int ol = __ffsll((long long)own) - 1;  // the owner lane (keys are unique)
          const unsigned long long best = join64((unsigned)__builtin_amdgcn_readlane((int)(unsigned)k, ol), hi);
          if (best == 0ull) break;  // the same in every lane: the batch is done
          const float bx = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), ol));
          const float by = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(y), ol));
          const float bz = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(z), ol));
          // BinReduce and AddPatch (a free slot exists: np + u <= n_max)
          const bool in = (k != 0ull) & ((k == best) | (dot3_nofma(bx, by, bz, x, y, z) >= cs));
          k = in ? 0ull : k;
          const int slot = np++;
          if (in) atomicAdd(&s_pmem[slot], 1);
          if (lane == 0) {
            s_pn[slot][0] = bx;
            s_pn[slot][1] = by;
            s_pn[slot][2] = bz;
            s_pkey[slot] = best;
            s_pfound[slot] = (int)key_vidx(best);
          }
        }
        if (tid == 0) s_np = np;
      }
      continue;
    }
    // the loop: rows r = s * kWaves + wave of the packed entries in registers
    unsigned long long ek[kSlots];
    float ex[kSlots], ey[kSlots], ez[kSlots];
    unsigned long long mk = 0ull;
    float mx = 0.f, my = 0.f, mz = 0.f;
    const auto keep_max = [&](unsigned long long k, float x, float y, float z) {  // selects, no branch
      const bool gt = k > mk;
      mk = gt ? k : mk;
      mx = gt ? x : mx;
      my = gt ? y : my;
      mz = gt ? z : mz;
    };
#pragma unroll
    for (int sl = 0; sl < kSlots; ++sl) {
      const int i = (sl * kWaves + wave) * 64 + lane;
      ek[sl] = 0ull;
      ex[sl] = ey[sl] = ez[sl] = 0.f;
      if (i < u) {
        ek[sl] = s_ck[i];
        ex[sl] = s_cn[i][0];
        ey[sl] = s_cn[i][1];
        ez[sl] = s_cn[i][2];
      }
      keep_max(ek[sl], ex[sl], ey[sl], ez[sl]);
    }
    for (;;) {
      {  // this wave's deepest remaining entry, to the exchange slot
        // the high words' maximum; when one lane holds it (the usual case)
        // that lane's key is the maximum, else the low words decide
        const unsigned hi = wave_max_u32((unsigned)(mk >> 32));
        unsigned long long own = __ballot((unsigned)(mk >> 32) == hi);
        if (__popcll(own) != 1) {
          const unsigned lo = wave_max_u32((unsigned)(mk >> 32) == hi ? (unsigned)mk : 0u);
          own = __ballot(mk == join64(lo, hi));
        }
        const int ol = __ffsll((long long)own) - 1;  // the owner lane (keys are unique)
        const unsigned long long wbest = join64((unsigned)__builtin_amdgcn_readlane((int)(unsigned)mk, ol), hi);
        const float wx = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(mx), ol));
        const float wy = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(my), ol));
        const float wz = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(mz), ol));
        if (lane == 0) {
          s_red[par][wave] = make_uint4((unsigned)wbest, (unsigned)(wbest >> 32), __float_as_uint(wx),
                                        __float_as_uint(wy));
          s_redz[par][wave] = wz;
        }
      }
      __syncthreads();
      // FindDeepest: the deepest of the waves' (keys are unique)
      unsigned long long best = 0ull;
      float bx = 0.f, by = 0.f, bz = 0.f;
#pragma unroll
      for (int w = 0; w < kWaves; ++w) {
        const uint4 r = s_red[par][w];
        const unsigned long long k = join64(r.x, r.y);
        const bool gt = k > best;
        best = gt ? k : best;
        bx = gt ? __uint_as_float(r.z) : bx;
        by = gt ? __uint_as_float(r.w) : by;
        bz = gt ? s_redz[par][w] : bz;
      }
      if (best == 0ull) break;  // the same in every thread: the batch is done
      // BinReduce: the deepest and every entry similar to it leave
      int cnt = 0;
      mk = 0ull;
#pragma unroll
      for (int sl = 0; sl < kSlots; ++sl) {
        if ((sl * kWaves + wave) * 64 < u) {  // the same in every lane of the wave
          const bool in = (ek[sl] != 0ull) & ((ek[sl] == best) | (dot3_nofma(bx, by, bz, ex[sl], ey[sl], ez[sl]) >= cs));
          cnt += in ? 1 : 0;
          ek[sl] = in ? 0ull : ek[sl];
          keep_max(ek[sl], ex[sl], ey[sl], ez[sl]);
        }
      }
      if (np < P.n_max) {  // AddPatch into a free slot: the members' count by LDS atomics
        const int slot = np++;
        if (cnt) atomicAdd(&s_pmem[slot], cnt);
        if (tid == 0) {
          s_pn[slot][0] = bx;
          s_pn[slot][1] = by;
          s_pn[slot][2] = bz;
          s_pkey[slot] = best;
          s_pfound[slot] = (int)key_vidx(best);
        }
      } else {  // replace the most similar existing patch (lowest index on ties) or drop
        if (cnt) atomicAdd(&s_members[par], cnt);
        __syncthreads();  // the member count summed; the patch list as written so far
        const int members = s_members[par];
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
        const bool take = (float)members * key_depth(best) > (float)s_pmem[pj] * key_depth(s_pkey[pj]);
        __syncthreads();  // every thread has read the list before it changes
        if (tid == 0) {
          s_members[par] = 0;
          if (take) {
            s_pn[pj][0] = bx;
            s_pn[pj][1] = by;
            s_pn[pj][2] = bz;
            s_pkey[pj] = best;
            s_pmem[pj] = members;
            s_pfound[pj] = (int)key_vidx(best);
          }
        }
      }
      par ^= 1;
    }
    par ^= 1;
    if (tid == 0) s_np = np;
  }
  __builtin_amdgcn_s_setprio(0);
  __syncthreads();
  np = m.n > 0 ? s_np : 0;
  // the patch list, each with its deepest member's record
  if (tid == 0) P.count[e] = np;
  const long long S = (long long)A.n_env * P.n_max;
  for (int p = tid; p < P.n_max; p += kPatchThreads) {
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
  hipLaunchKernelGGL((k_patches<DT, LAYOUT>), dim3(a.n_env), dim3(kPatchThreads), 0, s, a, p);
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
