// Host side of libfactory_sdf.so: argument validation, work tables, workspace
// layout, launch selection, graph capture, brick conversion and the autotune
// cache.  Declarations and their contracts are in include/fc.h.
#include <hip/hip_runtime.h>

#include <cctype>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <limits>
#include <mutex>
#include <algorithm>
#include <string>
#include <vector>

#include "fc_bake.h"
#include "fc_internal.h"

using namespace fcimpl;

namespace {

thread_local int g_last_hip = 0;

fc_status hip_fail(hipError_t e) {
  g_last_hip = (int)e;
  return FC_ERR_HIP;
}

#define FC_HIP(x)                              \
  do {                                         \
    hipError_t e_ = (x);                       \
    if (e_ != hipSuccess) return hip_fail(e_); \
  } while (0)

std::mutex g_tune_mu;
std::map<std::string, fc_launch> g_tune;

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

bool finitef(float x) { return std::isfinite(x); }

int ceil_div(long long a, long long b) { return (int)((a + b - 1) / b); }

// bricks per axis of grid g stored (or to be stored) as `layout`
void bricks_of(const fc_grid& g, int layout, int& bx, int& by, int& bz) {
  int nx, ny, nz;
  brick_nodes(layout, nx, ny, nz);
  bx = ceil_div(g.nx - 1, nx - 1);
  by = ceil_div(g.ny - 1, ny - 1);
  bz = ceil_div(g.nz - 1, nz - 1);
}

bool is_brick(int layout) { return layout == FC_LAYOUT_BRICK || layout == FC_LAYOUT_SLAB; }
// layouts whose kernels address bricks (the sparse one uses FC_LAYOUT_BRICK's)
bool has_bricks(int layout) { return is_brick(layout) || layout == FC_LAYOUT_SPARSE; }

int elem_size(int dtype) { return dtype == FC_F32 ? 4 : 2; }

fc_status check_grid(const fc_grid& g) {
  if (!g.data) return FC_ERR_NULL;
  if (g.dtype < FC_F32 || g.dtype > FC_BF16) return FC_ERR_DTYPE;
  if (g.layout != FC_LAYOUT_LINEAR && !has_bricks(g.layout)) return FC_ERR_DTYPE;
  if (g.nx < 2 || g.ny < 2 || g.nz < 2) return FC_ERR_SHAPE;
  if ((long long)g.nx * g.ny * g.nz >= (1LL << 31)) return FC_ERR_SHAPE;
  if (has_bricks(g.layout)) {
    int bx, by, bz, nx, ny, nz;
    bricks_of(g, g.layout, bx, by, bz);
    brick_nodes(g.layout, nx, ny, nz);
    if ((long long)bx * by * bz * nx * ny * nz >= (1LL << 31)) return FC_ERR_SHAPE;
  }
  if (!(g.h > 0.f) || !finitef(g.h) || !finitef(1.f / g.h)) return FC_ERR_RANGE;
  for (int a = 0; a < 3; ++a)
    if (!finitef(g.origin[a])) return FC_ERR_RANGE;
  return FC_OK;
}

fc_status validate_desc(const fc_batch_desc* d) {
  if (!d) return FC_ERR_NULL;
  if (!d->grids || !d->meshes || !d->bin_dirs) return FC_ERR_NULL;
  if (d->n_env < 1) return FC_ERR_SHAPE;
  if (d->n_grids < 1 || d->n_grids > FC_MAX_TYPES) return FC_ERR_SHAPE;
  if (d->n_meshes < 1 || d->n_meshes > FC_MAX_TYPES) return FC_ERR_SHAPE;
  if (d->n_bins < 1 || d->n_bins > FC_MAX_BINS) return FC_ERR_RANGE;
  if (!finitef(d->margin)) return FC_ERR_RANGE;
  for (int i = 0; i < 3 * d->n_bins; ++i)
    if (!finitef(d->bin_dirs[i])) return FC_ERR_RANGE;
  for (int i = 0; i < d->n_grids; ++i) {
    fc_status s = check_grid(d->grids[i]);
    if (s != FC_OK) return s;
    if (d->grids[i].dtype != d->grids[0].dtype || d->grids[i].layout != d->grids[0].layout) return FC_ERR_DTYPE;
  }
  for (int i = 0; i < d->n_meshes; ++i) {
    const fc_mesh& m = d->meshes[i];
    if (m.n_verts < 0 || m.n_tris < 0) return FC_ERR_SHAPE;
    if (m.n_verts > 0 && (!m.x || !m.y || !m.z)) return FC_ERR_NULL;
    if (m.n_tris > 0 && !m.tris) return FC_ERR_NULL;
  }
  if (d->env_order) {
    std::vector<char> seen(d->n_env, 0);
    for (int e = 0; e < d->n_env; ++e) {
      const int o = d->env_order[e];
      if (o < 0 || o >= d->n_env || seen[o]) return FC_ERR_SHAPE;
      seen[o] = 1;
    }
  }
  long long Q = 0;
  for (int e = 0; e < d->n_env; ++e) {
    const int gi = d->env_grid ? d->env_grid[e] : 0;
    const int mi = d->env_mesh ? d->env_mesh[e] : 0;
    if (gi < 0 || gi >= d->n_grids || mi < 0 || mi >= d->n_meshes) return FC_ERR_SHAPE;
    Q += d->meshes[mi].n_verts;
  }
  if (Q >= (1LL << 40)) return FC_ERR_SHAPE;
  return FC_OK;
}

bool launch_valid(const fc_launch& l) {
  if (l.block <= 0 || l.tile <= 0 || l.tile % l.block) return false;
  if (!forward_shape_supported(l.block, l.tile / l.block)) return false;
  if (l.persistent < 0 || l.persistent > 3) return false;
  if (l.grid_mult < 1 || l.grid_mult > 32) return false;
  if (l.xcd_remap < 0 || l.xcd_remap > 1) return false;
  if (l.wave_prio < 0 || l.wave_prio > 2) return false;
  return true;
}

GridDev to_dev(const fc_grid& g) {
  GridDev d;
  d.data = g.data;
  d.nx = g.nx;
  d.ny = g.ny;
  d.nz = g.nz;
  int bx = 0, by = 0, bz = 0;
  if (has_bricks(g.layout)) bricks_of(g, g.layout, bx, by, bz);
  d.bx = bx;
  d.by = by;
  d.map = nullptr;
  d.coarse = nullptr;
  if (g.layout == FC_LAYOUT_SPARSE) {  // one buffer: map, coarse grid, pool
    const char* base = static_cast<const char*>(g.data);
    const long long nb = (long long)bx * by * bz;
    d.map = reinterpret_cast<const int*>(base);
    d.coarse = base + sparse_coarse_offset(nb);
    d.data = base + sparse_pool_offset(nb, bx, by, bz, elem_size(g.dtype));
  }
  d.ox = g.origin[0];
  d.oy = g.origin[1];
  d.oz = g.origin[2];
  d.inv_h = 1.f / g.h;
  return d;
}

template <typename T>
fc_status upload(T** dst, const std::vector<T>& v) {
  *dst = nullptr;
  if (v.empty()) return FC_OK;
  FC_HIP(hipMalloc((void**)dst, v.size() * sizeof(T)));
  FC_HIP(hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return FC_OK;
}

// --- normal-bin search table ------------------------------------------------
// For each cube-map cell: every bin k that can be the argmax of n.d_k for some
// unit normal n in the cell.  The cell lies in the cone around its centre c
// whose half-angle alpha reaches its farthest corner (plus a margin for the
// FP32 cell choice); over that cone n.d_k <= |d_k| cos(max(theta_k - alpha, 0))
// and max_j n.d_j >= max_j |d_j| cos(min(theta_j + alpha, pi)), theta = the
// angle to c.  Bins whose upper bound falls short of the best lower bound by
// more than the FP32 dot-product error can never win; the rest are listed.
std::vector<BinCell> build_bin_lut(const std::vector<float>& dirs, int K) {
  const double kPi = 3.14159265358979323846;
  auto face_dir = [](int f, double u, double v, double out[3]) {
    switch (f) {
      case 0: out[0] = 1; out[1] = u; out[2] = v; break;
      case 1: out[0] = -1; out[1] = u; out[2] = v; break;
      case 2: out[0] = u; out[1] = 1; out[2] = v; break;
      case 3: out[0] = u; out[1] = -1; out[2] = v; break;
      case 4: out[0] = u; out[1] = v; out[2] = 1; break;
      default: out[0] = u; out[1] = v; out[2] = -1; break;
    }
    const double n = std::sqrt(out[0] * out[0] + out[1] * out[1] + out[2] * out[2]);
    for (int a = 0; a < 3; ++a) out[a] /= n;
  };
  std::vector<double> dk(3 * K), dn(K);
  for (int k = 0; k < K; ++k) {
    for (int a = 0; a < 3; ++a) dk[3 * k + a] = dirs[a * K + k];
    dn[k] = std::sqrt(dk[3 * k] * dk[3 * k] + dk[3 * k + 1] * dk[3 * k + 1] + dk[3 * k + 2] * dk[3 * k + 2]);
  }
  std::vector<BinCell> lut(kLutCells);
  for (int f = 0; f < 6; ++f)
    for (int iv = 0; iv < kLutN; ++iv)
      for (int iu = 0; iu < kLutN; ++iu) {
        BinCell& cell = lut[(f * kLutN + iv) * kLutN + iu];
        std::memset(&cell, 0, sizeof(cell));
        double c[3], q[3];
        face_dir(f, -1.0 + 2.0 * (iu + 0.5) / kLutN, -1.0 + 2.0 * (iv + 0.5) / kLutN, c);
        double alpha = 0;
        for (int a = 0; a < 2; ++a)
          for (int b = 0; b < 2; ++b) {
            face_dir(f, -1.0 + 2.0 * (iu + a) / kLutN, -1.0 + 2.0 * (iv + b) / kLutN, q);
            const double dot = std::min(1.0, c[0] * q[0] + c[1] * q[1] + c[2] * q[2]);
            alpha = std::max(alpha, std::acos(dot));
          }
        alpha += 1e-4;
        std::vector<double> up(K), lo(K);
        double best_lo = -1e30;
        for (int k = 0; k < K; ++k) {
          double th = 0.5 * kPi;
          if (dn[k] > 0) {
            const double cs = (c[0] * dk[3 * k] + c[1] * dk[3 * k + 1] + c[2] * dk[3 * k + 2]) / dn[k];
            th = std::acos(std::max(-1.0, std::min(1.0, cs)));
          }
          up[k] = dn[k] * std::cos(std::max(th - alpha, 0.0));
          lo[k] = dn[k] * std::cos(std::min(th + alpha, kPi));
          best_lo = std::max(best_lo, lo[k]);
        }
        int n = 0;
        bool full = false;
        for (int k = 0; k < K; ++k) {
          if (up[k] < best_lo - 1e-5) continue;
          if (n == kLutMax) {
            full = true;
            break;
          }
          cell.k[n++] = (unsigned char)k;
        }
        cell.n = full ? kLutFull : (unsigned char)n;
      }
  return lut;
}

// --- a small JSON reader for the autotune cache -----------------------------
struct JVal {
  enum Kind { NUL, NUM, STR, ARR, OBJ, BOOL } kind = NUL;
  double num = 0;
  std::string str;
  std::vector<JVal> arr;
  std::vector<std::pair<std::string, JVal>> obj;
};

struct JParser {
  const char* p;
  const char* end;
  void ws() {
    while (p < end && std::isspace((unsigned char)*p)) ++p;
  }
  bool str(std::string& out) {
    if (p >= end || *p != '"') return false;
    ++p;
    while (p < end && *p != '"') {
      if (*p == '\\') {
        ++p;
        if (p >= end) return false;
      }
      out.push_back(*p++);
    }
    if (p >= end) return false;
    ++p;
    return true;
  }
  bool val(JVal& v, int depth) {
    if (depth > 32) return false;
    ws();
    if (p >= end) return false;
    if (*p == '{') {
      ++p;
      v.kind = JVal::OBJ;
      ws();
      if (p < end && *p == '}') {
        ++p;
        return true;
      }
      while (true) {
        ws();
        std::string k;
        if (!str(k)) return false;
        ws();
        if (p >= end || *p != ':') return false;
        ++p;
        JVal c;
        if (!val(c, depth + 1)) return false;
        v.obj.emplace_back(k, c);
        ws();
        if (p < end && *p == ',') {
          ++p;
          continue;
        }
        if (p < end && *p == '}') {
          ++p;
          return true;
        }
        return false;
      }
    }
    if (*p == '[') {
      ++p;
      v.kind = JVal::ARR;
      ws();
      if (p < end && *p == ']') {
        ++p;
        return true;
      }
      while (true) {
        JVal c;
        if (!val(c, depth + 1)) return false;
        v.arr.push_back(c);
        ws();
        if (p < end && *p == ',') {
          ++p;
          continue;
        }
        if (p < end && *p == ']') {
          ++p;
          return true;
        }
        return false;
      }
    }
    if (*p == '"') {
      v.kind = JVal::STR;
      return str(v.str);
    }
    if (end - p >= 4 && !std::strncmp(p, "true", 4)) {
      v.kind = JVal::BOOL;
      v.num = 1;
      p += 4;
      return true;
    }
    if (end - p >= 5 && !std::strncmp(p, "false", 5)) {
      v.kind = JVal::BOOL;
      p += 5;
      return true;
    }
    if (end - p >= 4 && !std::strncmp(p, "null", 4)) {
      p += 4;
      return true;
    }
    char* q = nullptr;
    std::string tmp(p, (size_t)std::min<ptrdiff_t>(end - p, 64));
    const double d = std::strtod(tmp.c_str(), &q);
    if (q == tmp.c_str()) return false;
    v.kind = JVal::NUM;
    v.num = d;
    p += (q - tmp.c_str());
    return true;
  }
};

const JVal* jget(const JVal& o, const char* key) {
  if (o.kind != JVal::OBJ) return nullptr;
  for (auto& kv : o.obj)
    if (kv.first == key) return &kv.second;
  return nullptr;
}

}  // namespace

struct fc_batch {
  int n_env = 0, K = 0, dtype = 0, layout = 0;
  float margin = 0.f;
  std::vector<fc_grid> grids;
  std::vector<fc_mesh> meshes;
  std::vector<int> env_grid, env_mesh;
  std::vector<int> order;  // scheduling order of the envs
  std::vector<float> dirs;
  std::vector<long long> qoff;
  long long Q = 0;
  fc_launch launch{256, 1024, 0, 8, 0, 1};
  int num_cus = 256;
  int device = 0;  // the device current at creation: its tables live there
  int bwd_chunk = 0;  // envs per backward item (choose_bwd_chunk)
  std::string signature;
  // forward tables
  BinCell* d_lut = nullptr;
  Item* d_items = nullptr;
  int n_items = 0;
  EnvInfo* d_envs = nullptr;
  // per-face tables: (env, face tile) items in scheduling order, face query offsets
  Item* d_fitems = nullptr;
  int n_fitems = 0;
  EnvInfo* d_fenvs = nullptr;
  long long Qf = 0;
  // backward tables
  BwdItem* d_bitems = nullptr;
  int n_bitems = 0;
  BwdChunk* d_chunks = nullptr;
  int n_chunks = 0;
  int* d_env_list = nullptr;
  int* d_env_tile_base = nullptr;
  long long mesh_voff[FC_MAX_TYPES] = {0};
  int mesh_tiles[FC_MAX_TYPES] = {0};
  int mesh_chunk0[FC_MAX_TYPES] = {0};
  int mesh_nchunks[FC_MAX_TYPES] = {0};
  long long mesh_vpart0[FC_MAX_TYPES] = {0};
  // workspace layout (bytes)
  size_t off_keys = 0, off_workctr = 0, off_pose = 0, off_vert = 0, ws_bytes = 0;
  // per-launch timing of the main kernels (diagnostics; one thread at a time)
  std::vector<hipEvent_t> t_ev;     // [2 * slots]: before, after
  mutable std::vector<int> t_kind;  // [slots]
  mutable int t_next = 0;
};

namespace {

void free_tables(fc_batch* b) {
  if (b->d_lut) (void)hipFree(b->d_lut);
  b->d_lut = nullptr;
  if (b->d_items) (void)hipFree(b->d_items);
  if (b->d_envs) (void)hipFree(b->d_envs);
  if (b->d_bitems) (void)hipFree(b->d_bitems);
  if (b->d_chunks) (void)hipFree(b->d_chunks);
  if (b->d_env_list) (void)hipFree(b->d_env_list);
  if (b->d_env_tile_base) (void)hipFree(b->d_env_tile_base);
  if (b->d_fitems) (void)hipFree(b->d_fitems);
  if (b->d_fenvs) (void)hipFree(b->d_fenvs);
  b->d_fitems = nullptr;
  b->d_fenvs = nullptr;
  b->d_items = nullptr;
  b->d_envs = nullptr;
  b->d_bitems = nullptr;
  b->d_chunks = nullptr;
  b->d_env_list = nullptr;
  b->d_env_tile_base = nullptr;
}

int gm_of(const fc_batch* b, int e) { return b->env_grid[e] | (b->env_mesh[e] << 8); }

void free_timing(fc_batch* b) {
  for (hipEvent_t e : b->t_ev)
    if (e) (void)hipEventDestroy(e);
  b->t_ev.clear();
  b->t_kind.clear();
  b->t_next = 0;
}

// Events for the main kernel of the call being enqueued, or null when timing
// is off, its slots are used up, or the call is being captured into a graph.
const KernelMarks* take_marks(const fc_batch* b, int kind, bool timed, KernelMarks& m) {
  if (!timed || b->t_next >= (int)b->t_kind.size()) return nullptr;
  m.before = b->t_ev[2 * b->t_next];
  m.after = b->t_ev[2 * b->t_next + 1];
  b->t_kind[b->t_next++] = kind;
  return &m;
}

fc_status build_forward_tables(fc_batch* b) {
  std::vector<Item> items;
  std::vector<EnvInfo> envs(b->n_env);
  const int tile = b->launch.tile;
  for (int oi = 0; oi < b->n_env; ++oi) {
    const int e = b->order[oi];
    const int n = b->meshes[b->env_mesh[e]].n_verts;
    const int ni = n > 0 ? ceil_div(n, tile) : 1;
    envs[e].qoff = b->qoff[e];
    envs[e].n_items = ni;
    envs[e].gm = gm_of(b, e);
    for (int t = 0; t < ni; ++t) {
      Item it;
      it.env = e;
      it.vstart = t * tile;
      it.vcount = std::min(tile, n - t * tile);
      if (it.vcount < 0) it.vcount = 0;
      it.gm = gm_of(b, e);
      items.push_back(it);
    }
  }
  if (b->d_items) (void)hipFree(b->d_items);
  if (b->d_envs) (void)hipFree(b->d_envs);
  b->d_items = nullptr;
  b->d_envs = nullptr;
  b->n_items = (int)items.size();
  fc_status s = upload(&b->d_items, items);
  if (s != FC_OK) return s;
  return upload(&b->d_envs, envs);
}

// Envs per backward item.  Each item keeps its vertices' gradient sums in
// registers across the chunk's envs, so the fewer items the less partial-sum
// traffic; but a grid larger than what the device holds resident at once
// runs a second round whose few workgroups idle the rest of the chip.  The
// chunk is the smallest in [kBwdChunkMin, kBwdChunkMax] whose items fit in
// one resident round.  When none does, the items run in several rounds and
// the chip idles while the last items finish, for about one item's time:
// the chunk is then kBwdChunkMax / 2, which halves that tail against
// kBwdChunkMax for twice the items (measured on a 4,096-env batch of five
// part types: chunks of 32, 40, 48, 51, 56 and 64 gave one-pass kernels of
// 0.424, 0.427, 0.448, 0.438, 0.440 and 0.460 ms).
int choose_bwd_chunk(const fc_batch* b, const std::vector<std::vector<int>>& groups, int capacity) {
  for (int c = kBwdChunkMin; c <= kBwdChunkMax; ++c) {
    long long items = 0;
    for (size_t gi = 0; gi < groups.size(); ++gi) {
      const int m = (int)(gi / b->grids.size());
      items += (long long)ceil_div((int)groups[gi].size(), c) * b->mesh_tiles[m];
    }
    if (items <= capacity) return c;
  }
  return kBwdChunkMax / 2;
}

fc_status build_face_tables(fc_batch* b) {
  std::vector<Item> items;
  std::vector<EnvInfo> envs(b->n_env);
  long long q = 0;
  for (int e = 0; e < b->n_env; ++e) {
    envs[e].qoff = q;
    envs[e].gm = gm_of(b, e);
    envs[e].n_items = 0;
    q += b->meshes[b->env_mesh[e]].n_tris;
  }
  b->Qf = q;
  for (int oi = 0; oi < b->n_env; ++oi) {
    const int e = b->order[oi];
    const int nt = b->meshes[b->env_mesh[e]].n_tris;
    for (int t0 = 0; t0 < nt; t0 += kFaceTile) {
      Item it;
      it.env = e;
      it.vstart = t0;
      it.vcount = std::min(kFaceTile, nt - t0);
      it.gm = gm_of(b, e);
      items.push_back(it);
      ++envs[e].n_items;
    }
  }
  b->n_fitems = (int)items.size();
  fc_status s = FC_OK;
  if (!items.empty()) s = upload(&b->d_fitems, items);
  if (s == FC_OK) s = upload(&b->d_fenvs, envs);
  return s;
}

fc_status build_backward_tables(fc_batch* b) {
  const int nm = (int)b->meshes.size();
  std::vector<int> env_list;
  std::vector<BwdChunk> chunks;
  std::vector<BwdItem> items;
  std::vector<int> env_tile_base(b->n_env);
  // tiles per mesh (>= 1 so that an empty mesh still produces its poses' partials)
  for (int m = 0; m < nm; ++m) {
    const int n = b->meshes[m].n_verts;
    b->mesh_tiles[m] = n > 0 ? ceil_div(n, kBwdTile) : 1;
  }
  // pose partial rows, env order
  int rows = 0;
  for (int e = 0; e < b->n_env; ++e) {
    env_tile_base[e] = rows;
    rows += b->mesh_tiles[b->env_mesh[e]];
  }
  // chunks: grouped by mesh, then grid, then env order
  const int ng = (int)b->grids.size();
  std::vector<std::vector<int>> groups((size_t)nm * ng);
  for (int oi = 0; oi < b->n_env; ++oi) {
    const int e = b->order[oi];
    groups[(size_t)b->env_mesh[e] * ng + b->env_grid[e]].push_back(e);
  }
  b->bwd_chunk = choose_bwd_chunk(b, groups, b->num_cus * backward_blocks_per_cu(b->dtype));
  const size_t chunk = (size_t)b->bwd_chunk;
  long long vpart = 0;
  long long voff = 0;
  for (int m = 0; m < nm; ++m) {
    b->mesh_voff[m] = voff;
    voff += 3LL * b->meshes[m].n_verts;
    b->mesh_chunk0[m] = (int)chunks.size();
    b->mesh_vpart0[m] = vpart;
    for (int g = 0; g < ng; ++g) {
      const std::vector<int>& grp = groups[(size_t)m * ng + g];
      for (size_t i = 0; i < grp.size(); i += chunk) {
        BwdChunk c;
        c.first = (int)env_list.size();
        c.len = (int)std::min<size_t>(chunk, grp.size() - i);
        c.n_tiles = b->mesh_tiles[m];
        c.mesh = m;
        c.vpart = vpart;
        vpart += 3LL * b->meshes[m].n_verts;
        for (int k = 0; k < c.len; ++k) env_list.push_back(grp[i + k]);
        const int cid = (int)chunks.size();
        chunks.push_back(c);
        for (int t = 0; t < b->mesh_tiles[m]; ++t) {
          BwdItem it;
          it.vstart = t * kBwdTile;
          it.vcount = std::max(0, std::min(kBwdTile, b->meshes[m].n_verts - t * kBwdTile));
          it.gm = g | (m << 8);
          it.chunk = cid;
          it.tile = 0;
          it.tile_in_mesh = t;
          it.pad0 = it.pad1 = 0;
          items.push_back(it);
        }
      }
    }
    b->mesh_nchunks[m] = (int)chunks.size() - b->mesh_chunk0[m];
  }
  b->n_bitems = (int)items.size();
  b->n_chunks = (int)chunks.size();
  fc_status s;
  if ((s = upload(&b->d_bitems, items)) != FC_OK) return s;
  if ((s = upload(&b->d_chunks, chunks)) != FC_OK) return s;
  if ((s = upload(&b->d_env_list, env_list)) != FC_OK) return s;
  if ((s = upload(&b->d_env_tile_base, env_tile_base)) != FC_OK) return s;
  // workspace layout
  size_t off = 0;
  b->off_keys = off;
  off = align256(off + (size_t)b->n_env * b->K * 8);
  b->off_workctr = off;
  off = align256(off + kXcds * 4);
  b->off_pose = off;
  off = align256(off + (size_t)rows * (kBwdBlock / 64) * 8 * sizeof(float2));
  b->off_vert = off;
  off = align256(off + (size_t)vpart * sizeof(float2));
  b->ws_bytes = off;
  return FC_OK;
}

std::string make_signature(const fc_batch* b) {
  std::string s = "v1;dt=" + std::to_string(b->dtype) + ";lay=" + std::to_string(b->layout) +
                  ";K=" + std::to_string(b->K) + ";env=" + std::to_string(b->n_env) + ";grids=";
  for (auto& g : b->grids) s += std::to_string(g.nx) + "x" + std::to_string(g.ny) + "x" + std::to_string(g.nz) + ",";
  s += ";meshes=";
  for (auto& m : b->meshes) s += std::to_string(m.n_verts) + ",";
  return s;
}

fc_status check_ws(const fc_batch* b, void* ws, size_t ws_bytes) {
  if (!ws) return FC_ERR_WORKSPACE;
  if (ws_bytes < b->ws_bytes) return FC_ERR_WORKSPACE;
  if (((uintptr_t)ws) & 255u) return FC_ERR_WORKSPACE;
  return FC_OK;
}

void fill_common(const fc_batch* b, GridDev* grids, MeshDev* meshes) {
  for (size_t i = 0; i < b->grids.size(); ++i) grids[i] = to_dev(b->grids[i]);
  for (size_t i = 0; i < b->meshes.size(); ++i) {
    meshes[i].x = b->meshes[i].x;
    meshes[i].y = b->meshes[i].y;
    meshes[i].z = b->meshes[i].z;
    meshes[i].n = b->meshes[i].n_verts;
    meshes[i].tris = b->meshes[i].tris;
    meshes[i].nt = b->meshes[i].n_tris;
  }
}

FwdArgs make_fwd(const fc_batch* b, const float* pose, const fc_candidates* cand, const fc_contacts* out, void* ws) {
  FwdArgs a;
  std::memset(&a, 0, sizeof(a));
  fill_common(b, a.grids, a.meshes);
  for (int i = 0; i < 3 * b->K; ++i) a.dirs[i] = b->dirs[i];
  a.bin_lut = b->d_lut;
  a.items = b->d_items;
  a.envs = b->d_envs;
  a.pose = pose;
  a.n_items = b->n_items;
  a.n_env = b->n_env;
  a.K = b->K;
  a.margin = b->margin;
  a.Q = b->Q;
  if (cand) {
    a.c_phi = cand->phi;
    a.c_nrm = cand->normal;
    a.c_bin = cand->bin;
  }
  if (out) {
    a.o_vidx = out->vidx;
    a.o_depth = out->depth;
    a.o_point = out->point;
    a.o_nrm = out->normal;
    a.o_count = out->count;
  }
  if (ws) {  // calls without a workspace (patches) use neither
    char* w = static_cast<char*>(ws);
    a.keys = reinterpret_cast<unsigned long long*>(w + b->off_keys);
    a.work_ctr = reinterpret_cast<unsigned*>(w + b->off_workctr);
  }
  return a;
}

// The per-item forward kernel's scheduling mode: the env-chunked mode (3)
// applies to the fused-only call, any other call runs per item as a plain
// launch.
int item_persistent(const fc_batch* b) { return b->launch.persistent == 3 ? 0 : b->launch.persistent; }

int forward_grid(const fc_batch* b) {
  fc_launch l = b->launch;
  l.persistent = item_persistent(b);
  if (!l.xcd_remap) {
    if (l.persistent == 0) return b->n_items;
    return (int)std::min<long long>((long long)b->num_cus * l.grid_mult, b->n_items);
  }
  // XCD ranges: the grid is a multiple of kXcds, at most one workgroup per item of a range
  const long long per = (b->n_items + kXcds - 1) / kXcds;
  if (l.persistent == 0) return (int)(kXcds * per);
  const long long slots = std::max<long long>(1, std::min<long long>(per, (long long)b->num_cus * l.grid_mult / kXcds));
  return (int)(kXcds * slots);
}

bool contacts_ok(const fc_contacts* o) {
  return o->vidx && o->depth && o->point && o->normal && o->count;
}

BwdArgs make_bwd(const fc_batch* b, const float* pose, float k, const float* upstream, const fc_grads* out, void* ws);

QueryExtra make_query_extra(const fc_batch* b, const FwdArgs& f) {
  QueryExtra q;
  std::memset(&q, 0, sizeof(q));
  for (int i = 0; i < 3 * b->K; ++i) q.dirs[i] = b->dirs[i];
  q.bin_lut = b->d_lut;
  q.K = b->K;
  q.margin = b->margin;
  q.keys = f.keys;
  return q;
}

fc_status enqueue_forward(const fc_batch* b, const float* pose, const fc_candidates* cand, const fc_contacts* out,
                          void* ws, hipStream_t s, bool from_cand, bool timed) {
  const FwdArgs a = make_fwd(b, pose, cand, out, ws);
  if (b->launch.persistent == 3 && out && !cand && !from_cand) {
    // fused query + reduction on the adjoint's env-chunked items
    fc_grads none;
    std::memset(&none, 0, sizeof(none));
    const BwdArgs ba = make_bwd(b, pose, 1.f, nullptr, &none, nullptr);
    KernelMarks m;
    FC_HIP(launch_query_chunked(ba, make_query_extra(b, a), a, b->dtype, b->layout, s,
                                take_marks(b, FC_KERNEL_FORWARD, timed, m)));
    return FC_OK;
  }
  const int vpt = b->launch.tile / b->launch.block;
  KernelMarks m;
  FC_HIP(launch_forward(a, b->dtype, b->layout, b->launch.block, vpt, item_persistent(b), b->launch.xcd_remap,
                        forward_grid(b), from_cand, s, take_marks(b, FC_KERNEL_FORWARD, timed, m)));
  return FC_OK;
}

BwdArgs make_bwd(const fc_batch* b, const float* pose, float k, const float* upstream, const fc_grads* out, void* ws) {
  BwdArgs a;
  std::memset(&a, 0, sizeof(a));
  fill_common(b, a.grids, a.meshes);
  for (int m = 0; m < FC_MAX_TYPES; ++m) {
    a.mesh_voff[m] = b->mesh_voff[m];
    a.mesh_tiles[m] = b->mesh_tiles[m];
    a.mesh_chunk0[m] = b->mesh_chunk0[m];
    a.mesh_nchunks[m] = b->mesh_nchunks[m];
    a.mesh_vpart0[m] = b->mesh_vpart0[m];
  }
  a.n_meshes = (int)b->meshes.size();
  a.items = b->d_bitems;
  a.chunks = b->d_chunks;
  a.env_list = b->d_env_list;
  a.env_tile_base = b->d_env_tile_base;
  a.envs = b->d_envs;
  a.pose = pose;
  a.upstream = upstream;
  a.n_items = b->n_bitems;
  a.n_env = b->n_env;
  a.k = k;
  a.per_env = out->verts_per_env ? 1 : 0;
  a.xcd = b->launch.xcd_remap;
  a.prio = b->launch.wave_prio;
  a.Q = b->Q;
  a.loss = out->loss;
  a.d_pose = out->d_pose;
  a.d_verts = out->d_verts;
  if (ws) {
    char* w = static_cast<char*>(ws);
    a.pose_part = reinterpret_cast<float2*>(w + b->off_pose);
    a.vert_part = reinterpret_cast<float2*>(w + b->off_vert);
  }
  return a;
}

fc_status enqueue_backward(const fc_batch* b, const float* pose, float k, const float* upstream, const fc_grads* out,
                           void* ws, hipStream_t s, bool timed) {
  const BwdArgs a = make_bwd(b, pose, k, upstream, out, ws);
  KernelMarks m;
  FC_HIP(launch_backward(a, b->dtype, b->layout, s, take_marks(b, FC_KERNEL_BACKWARD, timed, m)));
  return FC_OK;
}

// fused query + reduce and the adjoint, from one gather per query
fc_status enqueue_query_backward(const fc_batch* b, const float* pose, const fc_contacts* contacts, float k,
                                 const float* upstream, const fc_grads* out, void* ws, hipStream_t s, bool timed) {
  const BwdArgs a = make_bwd(b, pose, k, upstream, out, ws);
  const FwdArgs f = make_fwd(b, pose, nullptr, contacts, ws);
  const QueryExtra q = make_query_extra(b, f);
  KernelMarks m;
  FC_HIP(launch_query_backward(a, q, f, b->dtype, b->layout, s, take_marks(b, FC_KERNEL_QUERY_BACKWARD, timed, m)));
  return FC_OK;
}

fc_status validate_backward(const fc_batch* b, const float* pose, float k, const fc_grads* out, void* ws,
                            size_t ws_bytes) {
  if (!b || !pose || !out) return FC_ERR_NULL;
  if (!out->loss && !out->d_pose && !out->d_verts) return FC_ERR_NULL;
  if (!(k > 0.f) || !finitef(k)) return FC_ERR_RANGE;
  return check_ws(b, ws, ws_bytes);
}

// ---- sparse grids -------------------------------------------------------------

struct SparsePlan {
  int bx = 0, by = 0, bz = 0;
  std::vector<int> map;   // per brick: slot or -1
  std::vector<int> list;  // per slot: brick index
};

fc_status check_sparse_args(const fc_grid* src, float band) {
  if (!src) return FC_ERR_NULL;
  fc_status st = check_grid(*src);
  if (st != FC_OK) return st;
  if (src->layout != FC_LAYOUT_LINEAR) return FC_ERR_DTYPE;
  if (!(band >= 0.f)) return FC_ERR_RANGE;  // also NaN
  fc_grid g = *src;
  g.layout = FC_LAYOUT_BRICK;
  return check_grid(g);  // the brick count must fit too
}

fc_status sparse_plan(const fc_grid& src, float band, hipStream_t s, SparsePlan& p) {
  bricks_of(src, FC_LAYOUT_BRICK, p.bx, p.by, p.bz);
  const long long nb = (long long)p.bx * p.by * p.bz;
  unsigned char* d_flags = nullptr;
  FC_HIP(hipMalloc(&d_flags, (size_t)nb));
  std::vector<unsigned char> f((size_t)nb);
  hipError_t e = launch_sparse_classify(src.data, src.dtype, src.nx, src.ny, src.nz, p.bx, p.by, p.bz, band, d_flags, s);
  if (e == hipSuccess) e = hipMemcpyAsync(f.data(), d_flags, (size_t)nb, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  const hipError_t e2 = hipFree(d_flags);
  if (e != hipSuccess) return hip_fail(e);
  if (e2 != hipSuccess) return hip_fail(e2);
  p.map.assign((size_t)nb, -1);
  p.list.clear();
  for (long long b = 0; b < nb; ++b)
    if (f[(size_t)b]) {
      p.map[(size_t)b] = (int)p.list.size();
      p.list.push_back((int)b);
    }
  return FC_OK;
}

size_t sparse_bytes(const SparsePlan& p, int elem) {
  const long long nb = (long long)p.bx * p.by * p.bz;
  return sparse_pool_offset(nb, p.bx, p.by, p.bz, elem) + p.list.size() * 64 * (size_t)elem;
}

// ---- mesh -> SDF bake -------------------------------------------------------

constexpr long long kBakeMaxTris = 1LL << 24;
constexpr int kBakeRecord = 3 + kBakeFeatures;  // float4 per triangle: a, ab, ac, 7 pseudonormals

long long bake_clusters(long long n_tris) { return (n_tris + kBakeCluster - 1) / kBakeCluster; }

struct D3 {
  double x, y, z;
};
D3 sub(const D3& a, const D3& b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
D3 add(const D3& a, const D3& b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
D3 scale(const D3& a, double s) { return {a.x * s, a.y * s, a.z * s}; }
double dot(const D3& a, const D3& b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
D3 cross(const D3& a, const D3& b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
double norm(const D3& a) { return std::sqrt(dot(a, a)); }

// interior angle at p of the triangle (p, q, r)
double corner_angle(const D3& p, const D3& q, const D3& r) {
  const D3 u = sub(q, p), v = sub(r, p);
  const double c = dot(u, v) / (norm(u) * norm(v));
  return std::acos(std::max(-1.0, std::min(1.0, c)));
}

// Pseudonormal table of a closed, consistently outward-wound mesh (face
// normal; per edge the sum of its two faces' unit normals; per vertex the
// angle-weighted sum of its faces' unit normals), computed in FP64.
fc_status build_bake_table(const float* verts, int n_verts, const int32_t* tris, int n_tris, float4* out) {
  std::vector<D3> V(n_verts);
  for (int i = 0; i < n_verts; ++i) {
    V[i] = {verts[3 * i], verts[3 * i + 1], verts[3 * i + 2]};
    if (!std::isfinite(V[i].x) || !std::isfinite(V[i].y) || !std::isfinite(V[i].z)) return FC_ERR_RANGE;
  }
  for (long long k = 0; k < 3LL * n_tris; ++k)
    if (tris[k] < 0 || tris[k] >= n_verts) return FC_ERR_SHAPE;
  // closed and consistently wound: every directed edge once, and its reverse once
  std::vector<std::pair<uint64_t, int>> edges;  // (p << 32 | q, face)
  edges.reserve(3 * (size_t)n_tris);
  for (int f = 0; f < n_tris; ++f) {
    const int32_t* t = tris + 3 * f;
    if (t[0] == t[1] || t[1] == t[2] || t[0] == t[2]) return FC_ERR_SHAPE;
    for (int e = 0; e < 3; ++e)
      edges.push_back({((uint64_t)(uint32_t)t[e] << 32) | (uint32_t)t[(e + 1) % 3], f});
  }
  std::sort(edges.begin(), edges.end());
  for (size_t i = 1; i < edges.size(); ++i)
    if (edges[i].first == edges[i - 1].first) return FC_ERR_SHAPE;
  auto twin = [&](uint32_t p, uint32_t q) -> int {  // face owning the directed edge (p, q), -1 if none
    const uint64_t key = ((uint64_t)p << 32) | q;
    auto it = std::lower_bound(edges.begin(), edges.end(), std::make_pair(key, -1));
    return (it != edges.end() && it->first == key) ? it->second : -1;
  };
  std::vector<D3> fn(n_tris);
  double vol6 = 0.0;
  for (int f = 0; f < n_tris; ++f) {
    const int32_t* t = tris + 3 * f;
    const D3 n = cross(sub(V[t[1]], V[t[0]]), sub(V[t[2]], V[t[0]]));
    const double len = norm(n);
    if (!(len > 0.0)) return FC_ERR_RANGE;  // zero-area face: no normal
    fn[f] = scale(n, 1.0 / len);
    vol6 += dot(V[t[0]], cross(V[t[1]], V[t[2]]));
  }
  for (int f = 0; f < n_tris; ++f) {
    const int32_t* t = tris + 3 * f;
    for (int e = 0; e < 3; ++e)
      if (twin((uint32_t)t[(e + 1) % 3], (uint32_t)t[e]) < 0) return FC_ERR_SHAPE;  // open edge
  }
  if (!(vol6 > 0.0)) return FC_ERR_RANGE;  // wound inward (or no volume)
  std::vector<D3> vn(n_verts, D3{0.0, 0.0, 0.0});
  for (int f = 0; f < n_tris; ++f) {
    const int32_t* t = tris + 3 * f;
    for (int e = 0; e < 3; ++e) {
      const int p = t[e], q = t[(e + 1) % 3], r = t[(e + 2) % 3];
      vn[p] = add(vn[p], scale(fn[f], corner_angle(V[p], V[q], V[r])));
    }
  }
  // spatial order: Morton code of the centroid over the mesh's bounding box
  D3 lo = V[0], hi = V[0];
  for (const D3& v : V) {
    lo = {std::min(lo.x, v.x), std::min(lo.y, v.y), std::min(lo.z, v.z)};
    hi = {std::max(hi.x, v.x), std::max(hi.y, v.y), std::max(hi.z, v.z)};
  }
  const double span = std::max({hi.x - lo.x, hi.y - lo.y, hi.z - lo.z, 1e-300});
  std::vector<std::pair<uint32_t, int>> order(n_tris);
  for (int f = 0; f < n_tris; ++f) {
    const int32_t* t = tris + 3 * f;
    const D3 c = scale(add(add(V[t[0]], V[t[1]]), V[t[2]]), 1.0 / 3.0);
    const double q[3] = {(c.x - lo.x) / span, (c.y - lo.y) / span, (c.z - lo.z) / span};
    uint32_t code = 0;
    for (int a = 0; a < 3; ++a) {
      const uint32_t u = (uint32_t)std::min(1023.0, std::max(0.0, q[a] * 1024.0));
      for (int bit = 0; bit < 10; ++bit) code |= ((u >> bit) & 1u) << (3 * bit + a);
    }
    order[f] = {code, f};
  }
  std::sort(order.begin(), order.end());
  auto put = [](float4* o, const D3& d) { *o = make_float4((float)d.x, (float)d.y, (float)d.z, 0.f); };
  const long long nc = bake_clusters(n_tris);
  float4* box = out + (size_t)kBakeRecord * n_tris;
  for (long long c = 0; c < nc; ++c) {
    box[2 * c] = make_float4(INFINITY, INFINITY, INFINITY, 0.f);
    box[2 * c + 1] = make_float4(-INFINITY, -INFINITY, -INFINITY, 0.f);
  }
  for (int s = 0; s < n_tris; ++s) {
    const int f = order[s].second;
    const int32_t* t = tris + 3 * f;
    const int a = t[0], b = t[1], c = t[2];
    float4* pos = out + 3 * (size_t)s;
    float4* nrm = out + 3 * (size_t)n_tris + (size_t)kBakeFeatures * s;
    float4* bl = box + 2 * (s / kBakeCluster);
    for (int k = 0; k < 3; ++k) {  // the box of the corners as given (FP32)
      const float* v = verts + 3 * t[k];
      bl[0] = make_float4(std::min(bl[0].x, v[0]), std::min(bl[0].y, v[1]), std::min(bl[0].z, v[2]), 0.f);
      bl[1] = make_float4(std::max(bl[1].x, v[0]), std::max(bl[1].y, v[1]), std::max(bl[1].z, v[2]), 0.f);
    }
    put(pos, V[a]);
    int32_t fi = f;
    std::memcpy(&pos->w, &fi, sizeof(fi));  // the mesh's index, for ties
    put(pos + 1, sub(V[b], V[a]));
    put(pos + 2, sub(V[c], V[a]));
    put(nrm + kBakeFace, fn[f]);
    put(nrm + kBakeEdgeAB, add(fn[f], fn[twin((uint32_t)b, (uint32_t)a)]));
    put(nrm + kBakeEdgeAC, add(fn[f], fn[twin((uint32_t)a, (uint32_t)c)]));
    put(nrm + kBakeEdgeBC, add(fn[f], fn[twin((uint32_t)c, (uint32_t)b)]));
    put(nrm + kBakeVertA, vn[a]);
    put(nrm + kBakeVertB, vn[b]);
    put(nrm + kBakeVertC, vn[c]);
  }
  double vmax = 0.0;  // the mesh's largest coordinate, which scales the cull slack
  for (const D3& v : V) vmax = std::max({vmax, std::fabs(v.x), std::fabs(v.y), std::fabs(v.z)});
  box[0].w = (float)vmax;
  return FC_OK;
}

}  // namespace

extern "C" {

const char* fc_version(void) { return "factory_sdf 1.0 (gfx950)"; }

const char* fc_status_str(fc_status s) {
  switch (s) {
    case FC_OK: return "ok";
    case FC_ERR_NULL: return "required pointer is NULL";
    case FC_ERR_SHAPE: return "size or count out of range";
    case FC_ERR_DTYPE: return "unknown or mixed dtype / layout";
    case FC_ERR_RANGE: return "numeric parameter out of range";
    case FC_ERR_WORKSPACE: return "workspace missing, too small or misaligned";
    case FC_ERR_HIP: return "HIP runtime error";
    case FC_ERR_UNSUPPORTED: return "unsupported request";
    case FC_ERR_SCRATCH: return "batch needs more scratch than the no-allocation call holds";
  }
  return "unknown status";
}

int32_t fc_last_hip_error(void) { return g_last_hip; }

fc_status fc_batch_create(const fc_batch_desc* desc, fc_batch** out) {
  if (!out) return FC_ERR_NULL;
  *out = nullptr;
  fc_status s = validate_desc(desc);
  if (s != FC_OK) return s;
  fc_batch* b = new fc_batch();
  b->n_env = desc->n_env;
  b->K = desc->n_bins;
  b->dtype = desc->grids[0].dtype;
  b->layout = desc->grids[0].layout;
  b->margin = desc->margin;
  b->grids.assign(desc->grids, desc->grids + desc->n_grids);
  b->meshes.assign(desc->meshes, desc->meshes + desc->n_meshes);
  b->env_grid.resize(b->n_env);
  b->env_mesh.resize(b->n_env);
  b->qoff.resize(b->n_env);
  long long q = 0;
  b->order.resize(b->n_env);
  for (int e = 0; e < b->n_env; ++e) b->order[e] = desc->env_order ? desc->env_order[e] : e;
  for (int e = 0; e < b->n_env; ++e) {
    b->env_grid[e] = desc->env_grid ? desc->env_grid[e] : 0;
    b->env_mesh[e] = desc->env_mesh ? desc->env_mesh[e] : 0;
    b->qoff[e] = q;
    q += b->meshes[b->env_mesh[e]].n_verts;
  }
  b->Q = q;
  b->dirs.assign(desc->bin_dirs, desc->bin_dirs + 3 * b->K);
  int dev = 0;
  hipError_t he = hipGetDevice(&dev);
  b->device = dev;
  if (he == hipSuccess) he = hipDeviceGetAttribute(&b->num_cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (he != hipSuccess) {
    delete b;
    return hip_fail(he);
  }
  b->signature = make_signature(b);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(b->signature);
    if (it != g_tune.end() && launch_valid(it->second)) b->launch = it->second;
  }
  s = upload(&b->d_lut, build_bin_lut(b->dirs, b->K));
  if (s == FC_OK) s = build_forward_tables(b);
  if (s == FC_OK) s = build_backward_tables(b);
  if (s == FC_OK) s = build_face_tables(b);
  if (s != FC_OK) {
    free_tables(b);
    delete b;
    return s;
  }
  *out = b;
  return FC_OK;
}

void fc_batch_destroy(fc_batch* b) {
  if (!b) return;
  (void)hipDeviceSynchronize();
  free_tables(b);
  free_timing(b);
  delete b;
}

fc_status fc_batch_set_timing(fc_batch* b, int32_t max_records) {
  if (!b) return FC_ERR_NULL;
  if (max_records < 0 || max_records > FC_MAX_TIMING_RECORDS) return FC_ERR_RANGE;
  free_timing(b);
  b->t_ev.assign(2 * (size_t)max_records, nullptr);
  for (auto& e : b->t_ev) {
    const hipError_t he = hipEventCreate(&e);
    if (he != hipSuccess) {
      free_timing(b);
      return hip_fail(he);
    }
  }
  b->t_kind.assign(max_records, -1);
  return FC_OK;
}

int32_t fc_batch_read_timing(fc_batch* b, float* ms, int32_t* kernel, int32_t max) {
  if (!b || max < 0 || (max > 0 && (!ms || !kernel))) return -1;
  const int n = std::min(b->t_next, (int)max);
  for (int i = 0; i < n; ++i) {
    hipError_t he = hipEventSynchronize(b->t_ev[2 * i + 1]);
    if (he == hipSuccess) he = hipEventElapsedTime(&ms[i], b->t_ev[2 * i], b->t_ev[2 * i + 1]);
    if (he != hipSuccess) {
      (void)hip_fail(he);
      return -1;
    }
    kernel[i] = b->t_kind[i];
  }
  b->t_next = 0;
  return n;
}

int64_t fc_batch_queries(const fc_batch* b) { return b ? b->Q : -1; }

fc_status fc_batch_set_launch(fc_batch* b, const fc_launch* l) {
  if (!b || !l) return FC_ERR_NULL;
  if (!launch_valid(*l)) return FC_ERR_RANGE;
  const bool retile = l->tile != b->launch.tile;
  b->launch = *l;
  if (retile) {
    FC_HIP(hipDeviceSynchronize());
    return build_forward_tables(b);
  }
  return FC_OK;
}

fc_status fc_batch_get_launch(const fc_batch* b, fc_launch* out) {
  if (!b || !out) return FC_ERR_NULL;
  *out = b->launch;
  return FC_OK;
}

int32_t fc_batch_signature(const fc_batch* b, char* buf, int32_t cap) {
  if (!b) return -1;
  if (buf && cap > 0) {
    const size_t n = std::min<size_t>((size_t)cap - 1, b->signature.size());
    std::memcpy(buf, b->signature.data(), n);
    buf[n] = '\0';
  }
  return (int32_t)b->signature.size();
}

size_t fc_workspace_bytes(const fc_batch* b) { return b ? b->ws_bytes : 0; }

fc_status fc_workspace_init(const fc_batch* b, void* ws, size_t ws_bytes, void* stream) {
  if (!b) return FC_ERR_NULL;
  fc_status s = check_ws(b, ws, ws_bytes);
  if (s != FC_OK) return s;
  FC_HIP(launch_zero(ws, b->ws_bytes, (hipStream_t)stream));
  return FC_OK;
}

fc_status fc_sdf_query(const fc_batch* b, const float* pose, const fc_candidates* cand, const fc_contacts* fused_out,
                       void* ws, size_t ws_bytes, void* stream) {
  if (!b || !pose) return FC_ERR_NULL;
  if (!cand && !fused_out) return FC_ERR_NULL;
  if (cand && (!cand->phi || !cand->normal || !cand->bin)) return FC_ERR_NULL;
  if (fused_out && !contacts_ok(fused_out)) return FC_ERR_NULL;
  fc_status s = check_ws(b, ws, ws_bytes);
  if (s != FC_OK) return s;
  return enqueue_forward(b, pose, cand, fused_out, ws, (hipStream_t)stream, false, true);
}

size_t fc_sdf_query_noalloc_bytes(const fc_batch* b) {
  return b ? b->off_workctr + kXcds * sizeof(unsigned) : 0;
}

fc_status fc_sdf_query_noalloc(const fc_batch* b, const float* pose, const fc_candidates* cand,
                               const fc_contacts* fused_out, void* stream) {
  if (!b || !pose) return FC_ERR_NULL;
  if (!cand && !fused_out) return FC_ERR_NULL;
  if (cand && (!cand->phi || !cand->normal || !cand->bin)) return FC_ERR_NULL;
  if (fused_out && !contacts_ok(fused_out)) return FC_ERR_NULL;
  // the forward's part of the workspace layout: keys at 0, then the counters
  const size_t need = fc_sdf_query_noalloc_bytes(b);
  if (need > kNoAllocScratchBytes) return FC_ERR_SCRATCH;
  int dev = -1;
  FC_HIP(hipGetDevice(&dev));
  if (dev != b->device) return FC_ERR_UNSUPPORTED;
  void* ws = nullptr;
  FC_HIP(noalloc_scratch(&ws));
  // the array keeps the last call's contents: keys and counters start at zero
  FC_HIP(launch_zero(ws, need, (hipStream_t)stream));
  return enqueue_forward(b, pose, cand, fused_out, ws, (hipStream_t)stream, false, false);
}

fc_status fc_contact_reduce(const fc_batch* b, const float* pose, const fc_candidates* cand, const fc_contacts* out,
                            void* ws, size_t ws_bytes, void* stream) {
  if (!b || !pose || !cand || !out) return FC_ERR_NULL;
  if (!cand->phi || !cand->normal || !cand->bin || !contacts_ok(out)) return FC_ERR_NULL;
  fc_status s = check_ws(b, ws, ws_bytes);
  if (s != FC_OK) return s;
  return enqueue_forward(b, pose, cand, out, ws, (hipStream_t)stream, true, true);
}

fc_status fc_sdf_query_backward(const fc_batch* b, const float* pose, float k, const float* upstream,
                                const fc_grads* out, void* ws, size_t ws_bytes, void* stream) {
  fc_status s = validate_backward(b, pose, k, out, ws, ws_bytes);
  if (s != FC_OK) return s;
  return enqueue_backward(b, pose, k, upstream, out, ws, (hipStream_t)stream, true);
}

fc_status fc_sdf_query_and_backward(const fc_batch* b, const float* pose, const fc_contacts* fused_out, float k,
                                    const float* upstream, const fc_grads* grads, void* ws, size_t ws_bytes,
                                    void* stream) {
  if (!b || !pose || !fused_out || !grads) return FC_ERR_NULL;
  if (!contacts_ok(fused_out)) return FC_ERR_NULL;
  fc_status s = validate_backward(b, pose, k, grads, ws, ws_bytes);
  if (s != FC_OK) return s;
  return enqueue_query_backward(b, pose, fused_out, k, upstream, grads, ws, (hipStream_t)stream, true);
}

fc_status fc_sdf_query_faces(const fc_batch* b, const float* pose, const fc_pgd* pgd, const fc_candidates* cand,
                             const fc_contacts* fused_out, void* ws, size_t ws_bytes, void* stream) {
  if (!b || !pose || !pgd) return FC_ERR_NULL;
  if (!cand && !fused_out) return FC_ERR_NULL;
  if (cand && (!cand->phi || !cand->normal || !cand->bin || !cand->point)) return FC_ERR_NULL;
  if (fused_out && !contacts_ok(fused_out)) return FC_ERR_NULL;
  if (pgd->iters < 0 || pgd->iters > 64 || !(pgd->step0 > 0.f) || !std::isfinite(pgd->step0)) return FC_ERR_RANGE;
  fc_status s = check_ws(b, ws, ws_bytes);
  if (s != FC_OK) return s;
  FwdArgs a = make_fwd(b, pose, nullptr, fused_out, ws);
  a.items = b->d_fitems;
  a.n_items = b->n_fitems;
  a.envs = b->d_fenvs;
  a.Q = b->Qf;
  if (cand) {
    a.c_phi = cand->phi;
    a.c_nrm = cand->normal;
    a.c_bin = cand->bin;
    a.c_point = cand->point;
  }
  a.pgd_iters = pgd->iters;
  a.pgd_step0 = pgd->step0;
  KernelMarks m;
  FC_HIP(launch_faces(a, b->dtype, b->layout, (hipStream_t)stream, take_marks(b, FC_KERNEL_FACES, true, m)));
  return FC_OK;
}

int64_t fc_batch_face_queries(const fc_batch* b) { return b ? b->Qf : -1; }

fc_status fc_contact_patches(const fc_batch* b, const float* pose, const fc_patch_params* prm, const fc_patches* out,
                             void* stream) {
  if (!b || !pose || !prm || !out) return FC_ERR_NULL;
  if (!out->count || !out->founder || !out->normal || !out->vidx || !out->depth || !out->point || !out->members)
    return FC_ERR_NULL;
  if (prm->max_patches < 1 || prm->max_patches > kPatchMax || !std::isfinite(prm->cos_sim)) return FC_ERR_RANGE;
  FwdArgs a = make_fwd(b, pose, nullptr, nullptr, nullptr);
  PatchArgs p;
  p.n_max = prm->max_patches;
  p.cos_sim = prm->cos_sim;
  p.count = out->count;
  p.founder = out->founder;
  p.normal = out->normal;
  p.vidx = out->vidx;
  p.depth = out->depth;
  p.point = out->point;
  p.members = out->members;
  KernelMarks m;
  FC_HIP(launch_patches(a, p, b->dtype, b->layout, (hipStream_t)stream, take_marks(b, FC_KERNEL_PATCHES, true, m)));
  return FC_OK;
}

fc_status fc_gather_probe(const fc_batch* b, const float* pose, float* sink, void* stream) {
  if (!b || !pose || !sink) return FC_ERR_NULL;
  fc_grads g;
  std::memset(&g, 0, sizeof(g));
  g.loss = sink;  // the probe's only store target (taken only by a sentinel sum)
  BwdArgs a = make_bwd(b, pose, 1.f, nullptr, &g, nullptr);
  KernelMarks m;
  FC_HIP(launch_gather_probe(a, b->dtype, b->layout, (hipStream_t)stream,
                             take_marks(b, FC_KERNEL_GATHER_PROBE, true, m)));
  return FC_OK;
}

struct fc_graph {
  hipGraphExec_t exec = nullptr;
};

fc_status fc_graph_create(const fc_batch* b, const float* pose, const fc_contacts* fused_out, float k,
                          const float* upstream, const fc_grads* grads, void* ws, size_t ws_bytes, fc_graph** out) {
  if (!out) return FC_ERR_NULL;
  *out = nullptr;
  if (!b || !pose) return FC_ERR_NULL;
  if (!fused_out && !grads) return FC_ERR_NULL;
  if (fused_out && !contacts_ok(fused_out)) return FC_ERR_NULL;
  fc_status s = check_ws(b, ws, ws_bytes);
  if (s != FC_OK) return s;
  if (grads) {
    s = validate_backward(b, pose, k, grads, ws, ws_bytes);
    if (s != FC_OK) return s;
  }
  hipStream_t cs = nullptr;
  FC_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  hipError_t he = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (he != hipSuccess) {
    (void)hipStreamDestroy(cs);
    return hip_fail(he);
  }
  if (fused_out && grads)
    s = enqueue_query_backward(b, pose, fused_out, k, upstream, grads, ws, cs, false);
  else if (fused_out)
    s = enqueue_forward(b, pose, nullptr, fused_out, ws, cs, false, false);
  else
    s = enqueue_backward(b, pose, k, upstream, grads, ws, cs, false);
  hipGraph_t graph = nullptr;
  he = hipStreamEndCapture(cs, &graph);
  (void)hipStreamDestroy(cs);
  if (s != FC_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return s;
  }
  if (he != hipSuccess) return hip_fail(he);
  hipGraphExec_t exec = nullptr;
  he = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (he != hipSuccess) return hip_fail(he);
  fc_graph* g = new fc_graph();
  g->exec = exec;
  *out = g;
  return FC_OK;
}

fc_status fc_graph_launch(fc_graph* g, void* stream) {
  if (!g || !g->exec) return FC_ERR_NULL;
  FC_HIP(hipGraphLaunch(g->exec, (hipStream_t)stream));
  return FC_OK;
}

void fc_graph_destroy(fc_graph* g) {
  if (!g) return;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  delete g;
}

size_t fc_grid_brick_bytes(const fc_grid* src, int32_t layout) {
  if (!src || !is_brick(layout)) return 0;
  fc_grid g = *src;
  g.layout = layout;
  if (!g.data) g.data = (const void*)1;  // size query only
  if (check_grid(g) != FC_OK) return 0;
  int bx, by, bz, nx, ny, nz;
  bricks_of(g, layout, bx, by, bz);
  brick_nodes(layout, nx, ny, nz);
  return (size_t)bx * by * bz * nx * ny * nz * elem_size(g.dtype);
}

fc_status fc_grid_to_bricks(const fc_grid* src, int32_t layout, void* dst_data, size_t dst_bytes, fc_grid* dst,
                            void* stream) {
  if (!src || !dst_data || !dst) return FC_ERR_NULL;
  if (!is_brick(layout)) return FC_ERR_DTYPE;
  fc_status s = check_grid(*src);
  if (s != FC_OK) return s;
  if (src->layout != FC_LAYOUT_LINEAR) return FC_ERR_DTYPE;
  const size_t need = fc_grid_brick_bytes(src, layout);
  if (need == 0) return FC_ERR_SHAPE;
  if (dst_bytes < need) return FC_ERR_WORKSPACE;
  int bx, by, bz;
  bricks_of(*src, layout, bx, by, bz);
  FC_HIP(launch_to_bricks(src->data, dst_data, elem_size(src->dtype), layout, src->nx, src->ny, src->nz, bx, by, bz,
                          (hipStream_t)stream));
  *dst = *src;
  dst->data = dst_data;
  dst->layout = layout;
  return FC_OK;
}

fc_status fc_grid_sparse_bytes(const fc_grid* src, float band, size_t* bytes, void* stream) {
  if (!bytes) return FC_ERR_NULL;
  fc_status st = check_sparse_args(src, band);
  if (st != FC_OK) return st;
  SparsePlan p;
  st = sparse_plan(*src, band, (hipStream_t)stream, p);
  if (st != FC_OK) return st;
  *bytes = sparse_bytes(p, elem_size(src->dtype));
  return FC_OK;
}

fc_status fc_grid_to_sparse(const fc_grid* src, float band, void* dst_data, size_t dst_bytes, fc_grid* dst,
                            void* stream) {
  if (!dst_data || !dst) return FC_ERR_NULL;
  fc_status st = check_sparse_args(src, band);
  if (st != FC_OK) return st;
  if (((uintptr_t)dst_data & 255) != 0) return FC_ERR_RANGE;
  const hipStream_t s = (hipStream_t)stream;
  SparsePlan p;
  st = sparse_plan(*src, band, s, p);
  if (st != FC_OK) return st;
  const int elem = elem_size(src->dtype);
  if (dst_bytes < sparse_bytes(p, elem)) return FC_ERR_WORKSPACE;
  const long long nb = (long long)p.bx * p.by * p.bz;
  char* base = static_cast<char*>(dst_data);
  int* d_list = nullptr;
  if (!p.list.empty()) FC_HIP(hipMalloc(&d_list, p.list.size() * sizeof(int)));
  hipError_t e = hipMemcpyAsync(base, p.map.data(), (size_t)nb * sizeof(int), hipMemcpyHostToDevice, s);
  if (e == hipSuccess && d_list)
    e = hipMemcpyAsync(d_list, p.list.data(), p.list.size() * sizeof(int), hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = launch_sparse_fill(src->data, elem, src->nx, src->ny, src->nz, p.bx, p.by, p.bz, d_list, (int)p.list.size(),
                           base + sparse_pool_offset(nb, p.bx, p.by, p.bz, elem), base + sparse_coarse_offset(nb), s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  const hipError_t e2 = d_list ? hipFree(d_list) : hipSuccess;
  if (e != hipSuccess) return hip_fail(e);
  if (e2 != hipSuccess) return hip_fail(e2);
  *dst = *src;
  dst->data = dst_data;
  dst->layout = FC_LAYOUT_SPARSE;
  return FC_OK;
}

size_t fc_bake_table_bytes(int32_t n_tris) {
  if (n_tris < 4 || n_tris > kBakeMaxTris) return 0;
  return ((size_t)n_tris * kBakeRecord + 2 * (size_t)bake_clusters(n_tris)) * sizeof(float4);
}

fc_status fc_bake_table(const float* verts, int32_t n_verts, const int32_t* tris, int32_t n_tris, void* table,
                        size_t table_bytes) {
  if (!verts || !tris || !table) return FC_ERR_NULL;
  if (n_verts < 4 || n_tris < 4 || n_tris > kBakeMaxTris) return FC_ERR_SHAPE;
  if (table_bytes < fc_bake_table_bytes(n_tris)) return FC_ERR_WORKSPACE;
  if (((uintptr_t)table & 15) != 0) return FC_ERR_RANGE;
  return build_bake_table(verts, n_verts, tris, n_tris, (float4*)table);
}

}  // extern "C"

namespace {

// Both bake calls: validation, the kernel's arguments, the launch.  With cull
// off the slack is infinite, so every cluster and triangle bound passes and
// the kernel evaluates every (node, triangle) pair.
fc_status bake_sdf(const void* table, int32_t n_tris, int32_t nx, int32_t ny, int32_t nz, const float* origin,
                   float h, float* out, void* stream, bool cull) {
  if (!table || !origin || !out) return FC_ERR_NULL;
  if (n_tris < 4 || n_tris > kBakeMaxTris) return FC_ERR_SHAPE;
  if (nx < 1 || ny < 1 || nz < 1 || (long long)nx * ny * nz >= (1LL << 31)) return FC_ERR_SHAPE;
  if (!(h > 0.f) || !std::isfinite(h)) return FC_ERR_RANGE;
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(origin[a])) return FC_ERR_RANGE;
  if (((uintptr_t)table & 15) != 0) return FC_ERR_RANGE;
  BakeArgs b;
  b.pos = (const float4*)table;
  b.nrm = (const float4*)table + 3 * (size_t)n_tris;
  b.box = (const float4*)table + (size_t)kBakeRecord * n_tris;
  b.n_tris = n_tris;
  b.n_clusters = (int)bake_clusters(n_tris);
  b.nx = nx;
  b.ny = ny;
  b.nz = nz;
  b.bx = (nx + 3) / 4;
  b.by = (ny + 3) / 4;
  b.bz = (nz + 3) / 4;
  b.ox = origin[0];
  b.oy = origin[1];
  b.oz = origin[2];
  b.h = h;
  // The cull slack: 2^-12 of the largest node coordinate, far above the FP32
  // rounding of the bounds and distances (a few 2^-24 of the coordinates) for
  // any mesh inside the grid's reach.
  double L = 0.0;
  const int n[3] = {nx, ny, nz};
  for (int a = 0; a < 3; ++a)
    L = std::max({L, std::fabs((double)origin[a]), std::fabs((double)origin[a] + (double)h * (n[a] - 1))});
  b.slack = cull ? (float)(L * 0x1p-12) : std::numeric_limits<float>::infinity();
  b.out = out;
  FC_HIP(launch_bake(b, (hipStream_t)stream));
  return FC_OK;
}

}  // namespace

extern "C" {

fc_status fc_bake_sdf(const void* table, int32_t n_tris, int32_t nx, int32_t ny, int32_t nz, const float* origin,
                      float h, float* out, void* stream) {
  return bake_sdf(table, n_tris, nx, ny, nz, origin, h, out, stream, true);
}

fc_status fc_bake_sdf_unculled(const void* table, int32_t n_tris, int32_t nx, int32_t ny, int32_t nz,
                               const float* origin, float h, float* out, void* stream) {
  return bake_sdf(table, n_tris, nx, ny, nz, origin, h, out, stream, false);
}

int32_t fc_autotune_load(const char* path) {
  if (!path) return -1;
  FILE* f = std::fopen(path, "rb");
  if (!f) return -1;
  std::string text;
  char buf[4096];
  size_t n;
  while ((n = std::fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, n);
  std::fclose(f);
  JParser p{text.data(), text.data() + text.size()};
  JVal root;
  if (!p.val(root, 0)) return -1;
  const JVal* entries = jget(root, "entries");
  if (!entries || entries->kind != JVal::ARR) return -1;
  int loaded = 0;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (const JVal& e : entries->arr) {
    const JVal* key = jget(e, "key");
    const JVal* bl = jget(e, "block");
    const JVal* ti = jget(e, "tile");
    const JVal* pe = jget(e, "persistent");
    const JVal* gm = jget(e, "grid_mult");
    const JVal* xr = jget(e, "xcd_remap");
    const JVal* wp = jget(e, "wave_prio");
    if (!key || key->kind != JVal::STR || !bl || !ti || !pe || !gm) continue;
    fc_launch l{(int32_t)bl->num, (int32_t)ti->num, (int32_t)pe->num, (int32_t)gm->num,
                xr ? (int32_t)xr->num : 0, wp ? (int32_t)wp->num : 1};
    if (!launch_valid(l)) continue;
    g_tune[key->str] = l;
    ++loaded;
  }
  return loaded;
}

}  // extern "C"
