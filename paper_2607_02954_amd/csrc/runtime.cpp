// Host runtime of libmicrocosm: world and batch engines, workspace/pool
// layout, work tables, HIP graph capture, and the extern "C" boundary.
//
// A single world and a batch share one Engine: a table of world descriptors
// in device memory plus work lists (node packs, fluid items, filter tiles,
// scan items).  Steps alternate between two descriptor sets (A: populations
// buffer 0 -> 1, B: 1 -> 0), so a captured chunk of an even number of steps
// leaves every running world's state where it started.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "engine.h"
#include "microcosm.h"

namespace {

// Fixed-size message buffer: reporting an error allocates nothing.
thread_local char g_err[512];

sim_status fail(sim_status st, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return st;
}

}  // namespace

namespace mc {
int report_error(int st, const char* msg) { return fail((sim_status)st, "%s", msg); }
}  // namespace mc

namespace {

#define HIPCHK(expr)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess) return fail(SIM_E_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Sequential carve-out of a device region.
struct Carver {
  char* base;
  size_t off = 0;
  template <class T>
  T* take(size_t count) {
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += align_up(count * sizeof(T));
    return p;
  }
};

sim_status check_params(const sim_params* p) {
  if (!p) return fail(SIM_E_INVALID, "params is NULL");
  if (p->nx < 8 || p->ny < 8) return fail(SIM_E_INVALID, "grid must be at least 8x8 (got %dx%d)", p->nx, p->ny);
  if ((int64_t)p->nx * p->ny > (int64_t)1 << 30 || p->nx > 32768 || p->ny > 32768)
    return fail(SIM_E_INVALID, "grid too large (at most 2^30 cells and 32768 per side)");
  if (!(p->tau > 0.5f)) return fail(SIM_E_INVALID, "tau must exceed 1/2");
  if (!(p->trt_magic > 0.f)) return fail(SIM_E_INVALID, "trt_magic must be positive");
  if (p->pbd_iters < 0 || p->pbd_iters > 1000) return fail(SIM_E_INVALID, "pbd_iters out of range");
  if (p->repulse_radius < 1 || p->repulse_radius > mc::kMaxRadius)
    return fail(SIM_E_INVALID, "repulse_radius must be in 1..%d", mc::kMaxRadius);
  if (!(p->sigma_repulse > 0.f)) return fail(SIM_E_INVALID, "sigma_repulse must be positive");
  if (p->tile_side != 0 && p->tile_side != 16 && p->tile_side != 32 && p->tile_side != 64)
    return fail(SIM_E_INVALID, "tile_side must be 16, 32 or 64 (or 0 for 32)");
  if (!(p->energy_rate >= 0.f && p->energy_rate <= 1.f)) return fail(SIM_E_INVALID, "energy_rate must be in [0, 1]");
  if (p->mdf_iters < 0 || p->mdf_iters > 64) return fail(SIM_E_INVALID, "mdf_iters must be in 1..64 (0 means 1)");
  if (!(p->marker_offset >= 0.f && p->marker_offset <= 1.f)) return fail(SIM_E_INVALID, "marker_offset must be in [0, 1]");
  if (p->marker_offset > 0.f && (p->flags & SIM_SPLAT_SORTED))
    return fail(SIM_E_INVALID, "two-layer markers need the binned or the direct transfer");
  if (p->mdf_iters > 1 && (p->flags & SIM_SPLAT_SORTED))
    return fail(SIM_E_INVALID, "multi-direct forcing needs the binned or the direct transfer");
  if (p->flags & ~(uint32_t)(SIM_SPLAT_SORTED | SIM_SPLAT_DIRECT)) return fail(SIM_E_INVALID, "unknown flag bits");
  if ((p->flags & SIM_SPLAT_SORTED) && (p->flags & SIM_SPLAT_DIRECT))
    return fail(SIM_E_INVALID, "SIM_SPLAT_SORTED and SIM_SPLAT_DIRECT are exclusive");
  return SIM_OK;
}

// Per-world device buffers beyond the caller's arrays.
struct WorldBufs {
  float* f_alt = nullptr;
  float* s = nullptr;
  float2* grad = nullptr;
  float2* Fg = nullptr;
  float* fel = nullptr;
  float* fel_el = nullptr;
  float* e_node = nullptr;      // [N] sensed energy; worlds with an energy rate
  float* d_marker = nullptr;    // [2][N] two-layer marker displacement (binned and direct transfers)
  float* U_d = nullptr;         // [2][N] MDF desired velocity
  float* mdf_c = nullptr;       // [2][N] MDF correction per node (binned transfer)
  float4* rho_j = nullptr;      // [ncell] MDF moments
  float2* u_mdf = nullptr;      // [ncell] MDF velocity
  int* key = nullptr;
  int* rank = nullptr;
  int* cnt = nullptr;
  int* start = nullptr;
  int* perm = nullptr;
  float4* rec = nullptr;
  int* part = nullptr;
  int* bin_cnt = nullptr;
  int* bin_fill = nullptr;
  int* bin_start = nullptr;
  int4* bin_rec = nullptr;
  int2* tile_rng = nullptr;
  int4* sp_rec = nullptr;
  int* sp_cnt = nullptr;
};

inline int mode_of(const sim_params& p) {
  return (p.flags & SIM_SPLAT_SORTED) ? mc::kSorted : (p.flags & SIM_SPLAT_DIRECT) ? mc::kDirect : mc::kBinned;
}
// Side of a world's grid tiles (0 in the parameters means the default, 32).
inline int tile_side(const sim_params& p) { return p.tile_side ? p.tile_side : 32; }
inline int tile_family(const sim_params& p) { return mc::tile_family_of_side(tile_side(p)); }
inline int tiles_x(const sim_params& p) { return (p.nx + tile_side(p) - 1) / tile_side(p); }
inline int tiles_y(const sim_params& p) { return (p.ny + tile_side(p) - 1) / tile_side(p); }
inline size_t n_bins(const sim_params& p) { return (size_t)tiles_x(p) * tiles_y(p); }

void carve_world_bufs(Carver& c, const sim_params& p, int n_part, WorldBufs& b) {
  const size_t ncell = (size_t)p.nx * p.ny;
  const size_t N = std::max(n_part, 1);
  b.f_alt = c.take<float>(9 * ncell);
  b.grad = c.take<float2>(ncell);
  b.Fg = c.take<float2>(ncell);
  b.fel = c.take<float>(2 * N);
  b.fel_el = c.take<float>(2 * N);
  if (p.energy_rate > 0.f) b.e_node = c.take<float>(N);
  const int mode = mode_of(p);
  if (mode == mc::kSorted) {
    b.key = c.take<int>(N);
    b.rank = c.take<int>(N);
    b.cnt = c.take<int>(ncell);
    b.start = c.take<int>(ncell + 1);
    b.perm = c.take<int>(N);
    b.rec = c.take<float4>(N);
    b.part = c.take<int>((ncell + 1023) / 1024 + 1);
  } else if (mode == mc::kDirect) {
    b.s = c.take<float>(ncell);
    if (p.marker_offset > 0.f) b.d_marker = c.take<float>(2 * N);
    if (p.mdf_iters > 1) {
      b.U_d = c.take<float>(2 * N);
      b.rho_j = c.take<float4>(ncell);
      b.u_mdf = c.take<float2>(ncell);
    }
  } else {
    const size_t nt = n_bins(p);
    b.bin_cnt = c.take<int>(nt);
    b.bin_fill = c.take<int>(nt);
    b.bin_start = c.take<int>(nt + 1);
    b.bin_rec = c.take<int4>(N);
    b.tile_rng = c.take<int2>((size_t)tiles_x(p) * tiles_y(p) * 2 * mc::kRunStride);
    b.sp_rec = c.take<int4>((size_t)tiles_x(p) * tiles_y(p) * mc::spread_cap_of_side(tile_side(p)));
    b.sp_cnt = c.take<int>((size_t)tiles_x(p) * tiles_y(p));
    if (p.marker_offset > 0.f) b.d_marker = c.take<float>(2 * N);
    if (p.mdf_iters > 1) {
      b.U_d = c.take<float>(2 * N);
      b.mdf_c = c.take<float>(2 * N);
      b.rho_j = c.take<float4>(ncell);
    }
  }
}

struct Slot {
  bool used = false;
  sim_params p{};
  int n_fil = 0, n_part = 0, max_len = 0;
  std::vector<int> h_off;
  int* fil_offset = nullptr;
  int* cell = nullptr;
  float* frac = nullptr;
  float* rest_angle = nullptr;
  float* rest_length = nullptr;
  float* amp = nullptr;
  float* period = nullptr;
  float* phase = nullptr;
  float* kb = nullptr;          // optional per-edge stiffnesses [N]
  float* ks = nullptr;
  float* ksh = nullptr;
  int* fil_flags = nullptr;     // optional [F] (SIM_FIL_CLOSED)
  bool any_loop = false;
  int* fil_parent = nullptr;    // optional [F] node a filament hangs from (branches), -1: none
  float* fil_attach = nullptr;  // [3][F] attachment rest length and rest angles
  bool any_branch = false;
  std::vector<int> unit_next;   // per filament: the first filament of the next creature
  float* energy = nullptr;      // optional energy field [ny][nx] and its node / filament outputs
  float* e_sensed = nullptr;
  float* e_collected = nullptr;
  float* fbuf[2] = {nullptr, nullptr};
  float* u = nullptr;
  WorldBufs b;
  int cur = 0;          // populations buffer that holds the state
  int remaining = 0;    // host mirror of the steps left (batch)
  size_t pool_off = 0, pool_len = 0;
  bool needs_zero = false;   // cnt must be cleared before first use
};

// Whether a world needs the general elastic kernel: it passes loop flags or
// per-edge stiffness arrays (their presence decides, not their contents).
bool slot_general(const Slot& s) { return s.fil_flags || s.kb || s.ks || s.ksh || s.fil_parent; }

// Device descriptor of a world whose buffers are described by s; parity 0
// reads populations buffer s.cur, parity 1 the other one.
mc::WorldDev world_desc(const Slot& s, int parity, const mc::Ctl* ctl_src, mc::Ctl* ctl_dst, unsigned* flags) {
  const sim_params& p = s.p;
  mc::WorldDev d{};
  d.nx = p.nx;
  d.ny = p.ny;
  d.n_part = s.n_part;
  d.n_fil = s.n_fil;
  d.om_p = 1.0f / p.tau;
  d.om_m = (float)(1.0 / ((double)p.trt_magic / ((double)p.tau - 0.5) + 0.5));
  d.k_bend = p.k_bend;
  d.k_stretch = p.k_stretch;
  d.k_shear = p.k_shear;
  d.k_el = p.k_elastic;
  d.k_rep = p.k_repulse;
  d.u_max2 = p.u_max * p.u_max;
  d.pbd_iters = p.pbd_iters;
  d.radius = p.repulse_radius;
  d.mode = mode_of(p);
  d.ntx = tiles_x(p);
  d.nty = tiles_y(p);
  d.tile_shift = mc::tile_shift_of_side(tile_side(p));
  {
    double g[mc::kMaxRadius + 1];
    double sum = 0.0;
    const double s2 = 2.0 * (double)p.sigma_repulse * (double)p.sigma_repulse;
    for (int k = 0; k <= p.repulse_radius; ++k) {
      g[k] = std::exp(-(double)k * k / s2);
      sum += (k == 0 ? 1.0 : 2.0) * g[k];
    }
    for (int k = 0; k <= mc::kMaxRadius; ++k) d.gtap[k] = k <= p.repulse_radius ? (float)(g[k] / sum) : 0.f;
  }
  d.fil_offset = s.fil_offset;
  d.cell_in = s.cell;
  d.frac_in = s.frac;
  d.cell_out = s.cell;
  d.frac_out = s.frac;
  d.rest_angle = s.rest_angle;
  d.rest_length = s.rest_length;
  d.act_amp = s.amp;
  d.act_period = s.period;
  d.act_phase = s.phase;
  d.kb_arr = s.kb;
  d.ks_arr = s.ks;
  d.ksh_arr = s.ksh;
  d.fil_flags = s.fil_flags;
  d.fil_parent = s.fil_parent;
  d.fil_attach = s.fil_attach;
  const bool energy = p.energy_rate > 0.f && s.energy && s.b.e_node;
  d.energy_rate = p.energy_rate;
  d.energy = energy ? s.energy : nullptr;
  d.e_node = s.b.e_node;
  d.e_sensed = energy ? s.e_sensed : nullptr;
  d.e_collected = energy ? s.e_collected : nullptr;
  d.mdf_iters = std::max(p.mdf_iters, 1);
  d.marker_offset = p.marker_offset;
  d.d_marker = s.b.d_marker;
  d.U_d = s.b.U_d;
  d.mdf_c = s.b.mdf_c;
  d.rho_j = s.b.rho_j;
  d.u_mdf = s.b.u_mdf;
  const int src = parity == 0 ? s.cur : 1 - s.cur;
  d.f_src = s.fbuf[src];
  d.f_dst = s.fbuf[1 - src];
  d.u = (float2*)s.u;
  d.s = s.b.s;
  d.grad = s.b.grad;
  d.Fg = s.b.Fg;
  d.fel = s.b.fel;
  d.fel_el = s.b.fel_el;
  d.ctl_src = ctl_src;
  d.ctl_dst = ctl_dst;
  d.flags = flags;
  d.key = s.b.key;
  d.rank = s.b.rank;
  d.cnt = s.b.cnt;
  d.start = s.b.start;
  d.perm = s.b.perm;
  d.rec = s.b.rec;
  d.part = s.b.part;
  d.bin_cnt = s.b.bin_cnt;
  d.bin_fill = s.b.bin_fill;
  d.bin_start = s.b.bin_start;
  d.bin_start_next = s.b.bin_start;
  d.bin_rec = s.b.bin_rec;
  d.tile_rng = s.b.tile_rng;
  d.sp_rec = s.b.sp_rec;
  d.sp_cnt = s.b.sp_cnt;
  return d;
}

// Zero an int array with a kernel (never a memset node; see graph capture).
__global__ void k_zero_i32(int* p, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0;
}

struct Engine {
  hipStream_t stream = nullptr;
  hipStream_t cap = nullptr;
  int max_worlds = 0;
  // device tables
  mc::WorldDev* desc[2] = {nullptr, nullptr};
  mc::Ctl* ctl[2] = {nullptr, nullptr};
  unsigned* flags = nullptr;
  int* counts = nullptr;
  mc::Pack* packs = nullptr;
  int2* tiles[mc::kTileFamilies] = {};
  int2* items = nullptr;
  int2* scan = nullptr;
  int2* wlist = nullptr;
  size_t max_packs = 0, max_items = 0, max_scan = 0;
  size_t max_tiles[mc::kTileFamilies] = {};
  mc::Tables tab{};
  mc::Grid grid{};
  bool fixed_grid = false;
  int fixed_tile_blocks = 2048;     // tile-kernel blocks per family when the grid is fixed
  bool any_sorted = false;
  std::vector<Slot> slots;
  // host staging (pinned) for table uploads
  char* pinned = nullptr;
  size_t pinned_bytes = 0;
  hipEvent_t upload_done = nullptr;
  // captured graphs
  hipGraphExec_t g_chunk = nullptr;
  int chunk_steps = 0;
  int want_chunk = 20;
  hipGraphExec_t g_pair = nullptr;

  size_t n_packs = 0, n_items = 0, n_scan = 0, n_worlds = 0;
  size_t n_tiles[mc::kTileFamilies] = {};

  // Device work-list lengths, in counts[]: packs, scan items, worlds, fluid
  // items, then the tiles of each tile family.
  static constexpr int kCntPacks = 0, kCntScan = 1, kCntWorlds = 2, kCntItems = 3, kCntTiles = 4;

  static size_t table_bytes(int max_worlds, size_t mp, const size_t* mt, size_t mi, size_t ms) {
    Carver c{nullptr};
    c.take<mc::WorldDev>(max_worlds);
    c.take<mc::WorldDev>(max_worlds);
    c.take<mc::Ctl>(max_worlds);
    c.take<mc::Ctl>(max_worlds);
    c.take<unsigned>(max_worlds);
    c.take<int>(8);
    c.take<mc::Pack>(mp);
    for (int f = 0; f < mc::kTileFamilies; ++f) c.take<int2>(mt[f]);
    c.take<int2>(mi);
    c.take<int2>(ms);
    c.take<int2>(max_worlds);
    return c.off;
  }

  void carve_tables(Carver& c) {
    desc[0] = c.take<mc::WorldDev>(max_worlds);
    desc[1] = c.take<mc::WorldDev>(max_worlds);
    ctl[0] = c.take<mc::Ctl>(max_worlds);
    ctl[1] = c.take<mc::Ctl>(max_worlds);
    flags = c.take<unsigned>(max_worlds);
    counts = c.take<int>(8);
    packs = c.take<mc::Pack>(max_packs);
    for (int f = 0; f < mc::kTileFamilies; ++f) tiles[f] = c.take<int2>(max_tiles[f]);
    items = c.take<int2>(max_items);
    scan = c.take<int2>(max_scan);
    wlist = c.take<int2>(max_worlds);
    tab.packs = packs;
    tab.n_packs = counts + kCntPacks;
    for (int f = 0; f < mc::kTileFamilies; ++f) {
      tab.tiles[f] = tiles[f];
      tab.n_tiles[f] = counts + kCntTiles + f;
    }
    tab.scan = scan;
    tab.n_scan = counts + kCntScan;
    tab.worlds = wlist;
    tab.n_worlds = counts + kCntWorlds;
    tab.items = items;
    tab.n_items = counts + kCntItems;
  }

  ~Engine() {
    if (g_chunk) hipGraphExecDestroy(g_chunk);
    if (g_pair) hipGraphExecDestroy(g_pair);
    if (upload_done) hipEventDestroy(upload_done);
    if (pinned) hipHostFree(pinned);
    if (cap) hipStreamDestroy(cap);
  }

  sim_status init_host(size_t staging) {
    HIPCHK(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&upload_done, hipEventDisableTiming));
    pinned_bytes = staging;
    HIPCHK(hipHostMalloc((void**)&pinned, pinned_bytes, hipHostMallocDefault));
    return SIM_OK;
  }

  mc::WorldDev make_desc(int w, int parity) const {
    return world_desc(slots[w], parity, ctl[parity] + w, ctl[1 - parity] + w, flags + w);
  }

  // Rebuild work tables and descriptors from the slot list and upload them.
  sim_status rebuild() {
    std::vector<mc::Pack> pk;
    std::vector<int2> tl[mc::kTileFamilies], sc, wl, it;
    any_sorted = false;
    bool any_binned = false;
    for (int w = 0; w < (int)slots.size(); ++w) {
      const Slot& s = slots[w];
      if (!s.used) continue;
      const int cap_nodes = grid.pack;
      int f = 0;
      while (f < s.n_fil) {
        mc::Pack p{};
        p.world = w;
        p.fil_begin = f;
        p.node_begin = s.h_off[f];
        // whole creatures (a filament and those hanging from it) per pack
        int end = f;
        while (end < s.n_fil) {
          const int next = s.unit_next.empty() ? end + 1 : s.unit_next[end];
          if (s.h_off[next] - p.node_begin > cap_nodes) break;
          end = next;
        }
        p.fil_end = end;
        p.node_end = s.h_off[end];
        pk.push_back(p);
        f = end;
      }
      const int ncell = s.p.nx * s.p.ny;
      std::vector<int2>& tlf = tl[tile_family(s.p)];
      for (int ty = 0; ty < tiles_y(s.p); ++ty)
        for (int tx = 0; tx < tiles_x(s.p); ++tx) tlf.push_back(make_int2(w, tx | (ty << 16)));
      for (int c = 0; c < ncell; c += mc::kCellsPerItem) it.push_back(make_int2(w, c));
      wl.push_back(make_int2(w, 0));
      const int mode = mode_of(s.p);
      if (mode == mc::kSorted) {
        any_sorted = true;
        const int nb = (ncell + 1023) / 1024;
        for (int b = 0; b < nb; ++b) sc.push_back(make_int2(w, b));
      }
      if (mode == mc::kBinned) any_binned = true;
    }
    bool over = pk.size() > max_packs || it.size() > max_items || sc.size() > max_scan;
    for (int f = 0; f < mc::kTileFamilies; ++f) over = over || tl[f].size() > max_tiles[f];
    if (over) return fail(SIM_E_WORKSPACE, "work tables exceed their capacity");
    n_packs = pk.size();
    for (int f = 0; f < mc::kTileFamilies; ++f) n_tiles[f] = tl[f].size();
    n_scan = sc.size();
    n_worlds = wl.size();
    n_items = it.size();
    // a kernel family stays in the captured graphs once any world needed it
    bool more = false;
    for (int f = 0; f < mc::kTileFamilies; ++f) {
      if (n_tiles[f] > 0 && grid.tile_blocks[f] == 0) more = true;
      if (!fixed_grid)
        grid.tile_blocks[f] = (int)n_tiles[f];        // one block per tile; 0: family not launched
      else if (n_tiles[f] > 0)
        grid.tile_blocks[f] = fixed_tile_blocks;      // stays launched once a world needed it
    }
    if (!fixed_grid) {
      grid.item_blocks = (int)std::max<size_t>(1, n_items);
      grid.node_blocks = (int)std::max<size_t>(1, n_packs);
      grid.scan_blocks = (int)std::max<size_t>(1, n_scan);
      grid.world_blocks = (int)std::max<size_t>(1, n_worlds);
    }
    more = more || (any_sorted && !grid.any_sorted) || (any_binned && !grid.any_binned);
    bool any_node = false;
    for (const auto& sl : slots)
      if (sl.used && mode_of(sl.p) != mc::kBinned) any_node = true;
    more = more || (any_node && !grid.any_node);
    bool any_energy = false, any_markers = false;
    int mdf_max = 1;
    for (const auto& sl : slots) {
      if (!sl.used) continue;
      if (sl.p.energy_rate > 0.f && sl.energy) any_energy = true;
      if (sl.b.d_marker) any_markers = true;
      if (sl.b.U_d) mdf_max = std::max(mdf_max, sl.p.mdf_iters);
    }
    if (any_energy && !grid.any_energy) {
      grid.any_energy = 1;
      more = true;
    }
    if (any_markers && !grid.any_markers) {
      grid.any_markers = 1;
      more = true;
    }
    // the one-layer tile variants are left out while every tile world has markers
    bool tile_plain = false, tile_mk = false;
    for (const auto& sl : slots) {
      if (!sl.used || mode_of(sl.p) == mc::kDirect) continue;
      if (mode_of(sl.p) == mc::kBinned && sl.b.d_marker) tile_mk = true;
      else tile_plain = true;
    }
    const int mk_only = tile_mk && !tile_plain ? 1 : 0;
    if (mk_only != grid.mk_only) {
      grid.mk_only = mk_only;
      more = true;
    }
    if (mdf_max > grid.mdf_max) {
      grid.mdf_max = mdf_max;
      more = true;
    }
    bool general = false;
    for (const auto& sl : slots)
      if (sl.used && slot_general(sl)) general = true;
    if (general && !grid.general) {         // stays set once a world needed it
      grid.general = 1;
      more = true;
    }
    bool branches = false;
    for (const auto& sl : slots)
      if (sl.used && sl.fil_parent) branches = true;
    if (branches && !grid.branches) {
      grid.branches = 1;
      more = true;
    }
    int max_r = 1;                          // the filter's LDS window is sized for this radius
    for (const auto& sl : slots)
      if (sl.used) max_r = std::max(max_r, sl.p.repulse_radius);
    if (max_r > grid.max_radius) {
      grid.max_radius = max_r;
      more = true;
    }
    grid.any_sorted |= any_sorted ? 1 : 0;
    grid.any_binned |= any_binned ? 1 : 0;
    grid.any_node |= any_node ? 1 : 0;
    if (more) drop_graphs();
    // stage into pinned memory once the previous upload has been consumed
    HIPCHK(hipEventSynchronize(upload_done));
    const size_t need = 2 * max_worlds * sizeof(mc::WorldDev) + 8 * sizeof(int) + pk.size() * sizeof(mc::Pack) +
                        (tl[0].size() + tl[1].size() + tl[2].size() + sc.size() + wl.size() + it.size()) *
                            sizeof(int2);
    if (need > pinned_bytes) {
      if (pinned) HIPCHK(hipHostFree(pinned));
      pinned_bytes = need * 2;
      HIPCHK(hipHostMalloc((void**)&pinned, pinned_bytes, hipHostMallocDefault));
    }
    char* h = pinned;
    size_t off = 0;
    auto put = [&](void* dev, const void* src, size_t bytes) -> sim_status {
      if (!bytes) return SIM_OK;
      std::memcpy(h + off, src, bytes);
      HIPCHK(hipMemcpyAsync(dev, h + off, bytes, hipMemcpyHostToDevice, stream));
      off += bytes;
      return SIM_OK;
    };
    std::vector<mc::WorldDev> d0(max_worlds), d1(max_worlds);
    for (int w = 0; w < (int)slots.size(); ++w) {
      if (!slots[w].used) continue;
      d0[w] = make_desc(w, 0);
      d1[w] = make_desc(w, 1);
    }
    sim_status st;
    if ((st = put(desc[0], d0.data(), max_worlds * sizeof(mc::WorldDev)))) return st;
    if ((st = put(desc[1], d1.data(), max_worlds * sizeof(mc::WorldDev)))) return st;
    int cnt[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    cnt[kCntPacks] = (int)n_packs;
    cnt[kCntScan] = (int)n_scan;
    cnt[kCntWorlds] = (int)n_worlds;
    cnt[kCntItems] = (int)n_items;
    for (int f = 0; f < mc::kTileFamilies; ++f) cnt[kCntTiles + f] = (int)n_tiles[f];
    if ((st = put(counts, cnt, sizeof(cnt)))) return st;
    if ((st = put(packs, pk.data(), pk.size() * sizeof(mc::Pack)))) return st;
    for (int f = 0; f < mc::kTileFamilies; ++f)
      if ((st = put(tiles[f], tl[f].data(), tl[f].size() * sizeof(int2)))) return st;
    if ((st = put(scan, sc.data(), sc.size() * sizeof(int2)))) return st;
    if ((st = put(wlist, wl.data(), wl.size() * sizeof(int2)))) return st;
    if ((st = put(items, it.data(), it.size() * sizeof(int2)))) return st;
    HIPCHK(hipEventRecord(upload_done, stream));
    return SIM_OK;
  }

  void enqueue_step(int parity, hipStream_t s) const { enqueue_step_with(desc[parity], grid, s); }

  void enqueue_step_with(const mc::WorldDev* d, const mc::Grid& grid, hipStream_t s) const {
    mc::launch_elastic(d, tab, grid, s);
    mc::launch_markers(d, tab, grid, s);
    mc::launch_sort(d, tab, grid, s);
    mc::launch_filter(d, tab, grid, s);
    mc::launch_repulse(d, tab, grid, s);
    mc::launch_spread(d, tab, grid, s);
    mc::launch_mdf(d, tab, grid, s);
    mc::launch_lbm(d, tab, grid, s);
    mc::launch_energy(d, tab, grid, s);
    mc::launch_integrate(d, tab, grid, s);
  }

  sim_status capture(int steps, hipGraphExec_t* out) {
    hipGraph_t g = nullptr;
    HIPCHK(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
    for (int k = 0; k < steps; ++k) enqueue_step(k & 1, cap);
    hipError_t le = hipGetLastError();
    hipError_t ee = hipStreamEndCapture(cap, &g);
    if (le != hipSuccess) {
      if (g) hipGraphDestroy(g);
      return fail(SIM_E_HIP, "kernel launch during capture: %s", hipGetErrorString(le));
    }
    if (ee != hipSuccess) return fail(SIM_E_HIP, "hipStreamEndCapture: %s", hipGetErrorString(ee));
    hipError_t ie = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (ie != hipSuccess) return fail(SIM_E_HIP, "hipGraphInstantiate: %s", hipGetErrorString(ie));
    return SIM_OK;
  }

  void drop_graphs() {
    if (g_chunk) hipGraphExecDestroy(g_chunk);
    if (g_pair) hipGraphExecDestroy(g_pair);
    g_chunk = g_pair = nullptr;
    chunk_steps = 0;
  }

  // Run n steps with parity starting at 0; n even uses graphs only.  An odd
  // tail step is launched directly with descriptor set A.
  sim_status run_steps(int n) {
    if (n <= 0) return SIM_OK;
    // tile-bin counts of the current positions for the first step (each
    // step's integrate then counts for the next)
    mc::launch_bin_prepass(desc[0], tab, grid, stream);
    if (n >= want_chunk && (!g_chunk || chunk_steps != want_chunk)) {
      if (g_chunk) hipGraphExecDestroy(g_chunk);
      g_chunk = nullptr;
      sim_status st = capture(want_chunk, &g_chunk);
      if (st) return st;
      chunk_steps = want_chunk;
    }
    if (n >= 2 && !g_pair) {
      sim_status st = capture(2, &g_pair);
      if (st) return st;
    }
    int left = n;
    while (chunk_steps > 0 && left >= chunk_steps) {
      HIPCHK(hipGraphLaunch(g_chunk, stream));
      left -= chunk_steps;
    }
    while (left >= 2) {
      HIPCHK(hipGraphLaunch(g_pair, stream));
      left -= 2;
    }
    if (left == 1) {
      enqueue_step(0, stream);
      HIPCHK(hipGetLastError());
    }
    return SIM_OK;
  }

  sim_status set_ctl(int w, long long t, int remaining) {
    mc::launch_set_ctl(ctl[0] + w, t, remaining, stream);
    HIPCHK(hipGetLastError());
    return SIM_OK;
  }
};

}  // namespace

// ---------------------------------------------------------------------------
// Single world
// ---------------------------------------------------------------------------
struct sim_world {
  Engine eng;
  sim_arrays arr{};
  size_t ws_bytes = 0;
  void* ws = nullptr;
};

namespace {

size_t world_table_bytes(const sim_params& p, int n_fil) {
  const size_t ncell = (size_t)p.nx * p.ny;
  size_t tiles[mc::kTileFamilies] = {0, 0, 0};
  tiles[tile_family(p)] = (size_t)tiles_x(p) * tiles_y(p);
  const size_t items = (ncell + mc::kCellsPerItem - 1) / mc::kCellsPerItem;
  const size_t scans = (ncell + 1023) / 1024;
  return Engine::table_bytes(1, std::max(n_fil, 1), tiles, items, scans);
}

size_t world_buf_bytes(const sim_params& p, int n_part) {
  Carver c{nullptr};
  WorldBufs b;
  carve_world_bufs(c, p, n_part, b);
  return c.off;
}

sim_status read_offsets(const sim_arrays* a, hipStream_t stream, std::vector<int>& h) {
  h.assign(a->n_filaments + 1, 0);
  HIPCHK(hipMemcpyAsync(h.data(), a->fil_offset, h.size() * sizeof(int), hipMemcpyDeviceToHost, stream));
  HIPCHK(hipStreamSynchronize(stream));
  if (h[0] != 0) return fail(SIM_E_INVALID, "fil_offset[0] must be 0");
  if (h[a->n_filaments] != a->n_particles) return fail(SIM_E_INVALID, "fil_offset[F] != n_particles");
  for (int f = 0; f < a->n_filaments; ++f) {
    const int len = h[f + 1] - h[f];
    if (len < 1 || len > mc::kMaxFilament)
      return fail(SIM_E_INVALID, "filament %d has %d nodes (allowed 1..%d)", f, len, mc::kMaxFilament);
  }
  return SIM_OK;
}

// Whether any filament is a closed loop (reads the flags back: synchronous).
sim_status read_loops(const sim_arrays* a, hipStream_t stream, bool* any) {
  *any = false;
  if (!a->fil_flags || a->n_filaments == 0) return SIM_OK;
  std::vector<int> h(a->n_filaments);
  HIPCHK(hipMemcpyAsync(h.data(), a->fil_flags, h.size() * sizeof(int), hipMemcpyDeviceToHost, stream));
  HIPCHK(hipStreamSynchronize(stream));
  for (int v : h)
    if (v & ~SIM_FIL_CLOSED) return fail(SIM_E_INVALID, "unknown filament flag bits");
  for (int v : h) *any = *any || (v & SIM_FIL_CLOSED);
  return SIM_OK;
}

// Branches: validate fil_parent / fil_attach (a filament hangs from a node
// of an earlier filament with an entering edge, never a loop itself, at most
// one filament per node, every creature contiguous in filament order) and
// form the creature units the packs are built from: unit_next[f] is the
// first filament after the creature that starts at f; *max_unit its largest
// node count.
sim_status read_branches(const sim_arrays* a, hipStream_t stream, const std::vector<int>& h_off,
                         std::vector<int>* unit_next, int* max_unit, bool* any) {
  const int F = a->n_filaments;
  *any = false;
  unit_next->assign(F, 0);
  for (int f = 0; f < F; ++f) (*unit_next)[f] = f + 1;
  *max_unit = 0;
  for (int f = 0; f < F; ++f) *max_unit = std::max(*max_unit, h_off[f + 1] - h_off[f]);
  if (!a->fil_parent || F == 0) return SIM_OK;
  if (!a->fil_attach) return fail(SIM_E_INVALID, "fil_parent needs fil_attach");
  std::vector<int> par(F), flags(F, 0);
  HIPCHK(hipMemcpyAsync(par.data(), a->fil_parent, F * sizeof(int), hipMemcpyDeviceToHost, stream));
  if (a->fil_flags) HIPCHK(hipMemcpyAsync(flags.data(), a->fil_flags, F * sizeof(int), hipMemcpyDeviceToHost, stream));
  HIPCHK(hipStreamSynchronize(stream));
  const int N = h_off[F];
  std::vector<char> used(N, 0);
  int last_root = -1;
  for (int f = 0; f < F; ++f) {
    const int pn = par[f];
    if (pn < 0) {
      last_root = f;
      continue;
    }
    if (pn >= N) return fail(SIM_E_INVALID, "filament %d: parent node %d out of range", f, pn);
    const int pf = int(std::upper_bound(h_off.begin(), h_off.end(), pn) - h_off.begin()) - 1;
    if (pf >= f || pf < last_root)
      return fail(SIM_E_INVALID, "filament %d: its parent node must lie in an earlier filament of its creature", f);
    if (flags[f] & SIM_FIL_CLOSED) return fail(SIM_E_INVALID, "filament %d: a closed loop cannot hang from a node", f);
    const bool ring_p = (flags[pf] & SIM_FIL_CLOSED) && h_off[pf + 1] - h_off[pf] >= 3;
    if (!ring_p && pn == h_off[pf]) return fail(SIM_E_INVALID, "filament %d: its parent node has no entering edge", f);
    if (used[pn]) return fail(SIM_E_INVALID, "node %d carries two attached filaments", pn);
    used[pn] = 1;
    *any = true;
  }
  *max_unit = 0;
  for (int f = 0; f < F;) {
    int g = f + 1;
    while (g < F && par[g] >= 0) ++g;
    (*unit_next)[f] = g;
    *max_unit = std::max(*max_unit, h_off[g] - h_off[f]);
    f = g;
  }
  return SIM_OK;
}

sim_status check_arrays(const sim_arrays* a) {
  if (!a) return fail(SIM_E_INVALID, "arrays is NULL");
  if (a->n_particles < 0 || a->n_filaments < 0) return fail(SIM_E_INVALID, "negative sizes");
  if ((a->n_particles > 0) != (a->n_filaments > 0)) return fail(SIM_E_INVALID, "filaments and particles must both be zero or both positive");
  if (!a->f || !a->u) return fail(SIM_E_INVALID, "f and u must be given");
  if (a->n_particles > 0 &&
      (!a->fil_offset || !a->cell || !a->frac || !a->rest_angle || !a->rest_length || !a->act_amp ||
       !a->act_period || !a->act_phase))
    return fail(SIM_E_INVALID, "node arrays must be given");
  return SIM_OK;
}

}  // namespace

extern "C" {

void sim_params_default(sim_params* p, int32_t nx, int32_t ny) {
  if (!p) return;
  p->nx = nx;
  p->ny = ny;
  p->tau = 1.0f;
  p->trt_magic = 0.25f;
  p->k_bend = 0.5f;
  p->k_stretch = 1.0f;
  p->k_shear = 0.5f;
  p->pbd_iters = 4;
  p->k_elastic = 0.05f;
  p->k_repulse = 0.1f;
  p->sigma_repulse = 1.0f;
  p->repulse_radius = 4;
  p->u_max = 0.3f;
  p->flags = 0;
  p->tile_side = 32;
  p->energy_rate = 0.f;
  p->mdf_iters = 1;
  p->marker_offset = 0.f;
}

const char* sim_last_error(void) { return g_err; }

sim_status sim_workspace_size(const sim_params* p, int32_t n_filaments, int32_t n_particles, size_t* bytes) {
  sim_status st = check_params(p);
  if (st) return st;
  if (!bytes) return fail(SIM_E_INVALID, "bytes is NULL");
  if (n_filaments < 0 || n_particles < 0) return fail(SIM_E_INVALID, "negative sizes");
  *bytes = world_table_bytes(*p, n_filaments) + world_buf_bytes(*p, n_particles);
  return SIM_OK;
}

// One world of a handle: validate and read its arrays' host-side facts
// (offsets, branches, loops) and carve its buffers.
static sim_status prepare_slot(const sim_params* p, const sim_arrays* a, hipStream_t s, Carver& c, Slot& sl) {
  sim_status st;
  std::vector<int> h_off;
  if (a->n_filaments > 0) {
    if ((st = read_offsets(a, s, h_off))) return st;
  } else {
    h_off.assign(1, 0);
  }
  std::vector<int> unit_next;
  int max_len = 0;
  bool any_branch = false;
  if ((st = read_branches(a, s, h_off, &unit_next, &max_len, &any_branch))) return st;
  if (max_len > mc::kMaxFilament)
    return fail(SIM_E_INVALID, "a creature (a filament with those hanging from it) holds %d nodes; at most %d",
                max_len, mc::kMaxFilament);
  sl.used = true;
  sl.p = *p;
  sl.n_fil = a->n_filaments;
  sl.n_part = a->n_particles;
  sl.max_len = max_len;
  sl.h_off = h_off;
  sl.fil_offset = const_cast<int*>(a->fil_offset);
  sl.cell = a->cell;
  sl.frac = a->frac;
  sl.rest_angle = const_cast<float*>(a->rest_angle);
  sl.rest_length = const_cast<float*>(a->rest_length);
  sl.amp = const_cast<float*>(a->act_amp);
  sl.period = const_cast<float*>(a->act_period);
  sl.phase = const_cast<float*>(a->act_phase);
  sl.kb = const_cast<float*>(a->k_bend);
  sl.ks = const_cast<float*>(a->k_stretch);
  sl.ksh = const_cast<float*>(a->k_shear);
  sl.fil_flags = const_cast<int*>(a->fil_flags);
  sl.fil_parent = any_branch ? const_cast<int*>(a->fil_parent) : nullptr;
  sl.fil_attach = any_branch ? const_cast<float*>(a->fil_attach) : nullptr;
  sl.any_branch = any_branch;
  sl.unit_next = unit_next;
  sl.energy = a->energy;
  sl.e_sensed = a->energy_sensed;
  sl.e_collected = a->energy_collected;
  if ((st = read_loops(a, s, &sl.any_loop))) return st;
  carve_world_bufs(c, *p, a->n_particles, sl.b);
  sl.fbuf[0] = a->f;
  sl.fbuf[1] = sl.b.f_alt;
  sl.u = a->u;
  return SIM_OK;
}

// Clear what a world's kernels expect to start at zero and build its tile
// run tables.
static void init_slot_buffers(const Slot& sl, hipStream_t s) {
  const sim_params& p = sl.p;
  const size_t ncell = (size_t)p.nx * p.ny;
  if (sl.b.cnt) hipLaunchKernelGGL(k_zero_i32, dim3(256), dim3(256), 0, s, sl.b.cnt, ncell);
  if (sl.b.s) hipLaunchKernelGGL(k_zero_i32, dim3(256), dim3(256), 0, s, (int*)sl.b.s, ncell);
  if (sl.b.Fg) hipLaunchKernelGGL(k_zero_i32, dim3(256), dim3(256), 0, s, (int*)sl.b.Fg, 2 * ncell);
  if (sl.b.e_node)
    hipLaunchKernelGGL(k_zero_i32, dim3(64), dim3(256), 0, s, (int*)sl.b.e_node, (size_t)std::max(sl.n_part, 1));
  if (sl.b.bin_cnt) {
    const size_t nt = n_bins(p);
    hipLaunchKernelGGL(k_zero_i32, dim3(64), dim3(256), 0, s, sl.b.bin_cnt, nt);
    hipLaunchKernelGGL(k_zero_i32, dim3(64), dim3(256), 0, s, sl.b.bin_fill, nt);
    mc::launch_tile_ranges(p.nx, p.ny, p.repulse_radius, tile_side(p), sl.b.tile_rng, s);
    hipLaunchKernelGGL(k_zero_i32, dim3(64), dim3(256), 0, s, sl.b.sp_cnt, (size_t)tiles_x(p) * tiles_y(p));
  }
}

// A handle over n worlds with the same parameters (n = 1: sim_create).
static sim_status create_worlds(const sim_params* p, int n, const sim_arrays* arrays, void* workspace,
                                size_t ws_bytes, void* stream, sim_world** out) {
  hipStream_t s = (hipStream_t)stream;
  sim_world* w = new sim_world();
  w->arr = arrays[0];
  w->ws = workspace;
  w->ws_bytes = ws_bytes;
  Engine& e = w->eng;
  e.stream = s;
  e.max_worlds = n;
  const size_t ncell = (size_t)p->nx * p->ny;
  size_t packs = 0;
  for (int i = 0; i < n; ++i) packs += std::max(arrays[i].n_filaments, 1);
  e.max_packs = packs;
  e.max_tiles[tile_family(*p)] = (size_t)n * tiles_x(*p) * tiles_y(*p);
  e.max_items = (size_t)n * ((ncell + mc::kCellsPerItem - 1) / mc::kCellsPerItem);
  e.max_scan = (size_t)n * ((ncell + 1023) / 1024);
  if (n == 1) e.tab.single_ntx[tile_family(*p)] = tiles_x(*p);   // one world: tile entries are computed
  Carver c{(char*)workspace};
  e.carve_tables(c);
  int max_len = 0;
  sim_status st;
  for (int i = 0; i < n; ++i) {
    Slot sl;
    if ((st = prepare_slot(p, &arrays[i], s, c, sl))) {
      delete w;
      return st;
    }
    max_len = std::max(max_len, sl.max_len);
    e.slots.push_back(sl);
  }
  e.grid.pack = max_len <= 256 ? 256 : 1024;
  if ((st = e.init_host(64 << 10))) {
    delete w;
    return st;
  }
  // clear flags and control words, then each world's counters and tables
  hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, s, (int*)e.flags, (size_t)n);
  hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, s, (int*)e.ctl[0], n * sizeof(mc::Ctl) / 4);
  hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, s, (int*)e.ctl[1], n * sizeof(mc::Ctl) / 4);
  for (const Slot& sl : e.slots) init_slot_buffers(sl, s);
  if (hipGetLastError() != hipSuccess) {
    delete w;
    return fail(SIM_E_HIP, "initialisation kernels failed to launch");
  }
  if ((st = e.rebuild())) {
    delete w;
    return st;
  }
  *out = w;
  return SIM_OK;
}

sim_status sim_create(const sim_params* p, const sim_arrays* a, void* workspace, size_t ws_bytes, void* stream,
                      sim_world** out) {
  sim_status st = check_params(p);
  if (st) return st;
  if ((st = check_arrays(a))) return st;
  if (!out) return fail(SIM_E_INVALID, "out is NULL");
  if (!workspace || ((uintptr_t)workspace % kAlign)) return fail(SIM_E_WORKSPACE, "workspace must be 256-byte aligned");
  size_t need = 0;
  sim_workspace_size(p, a->n_filaments, a->n_particles, &need);
  if (ws_bytes < need) return fail(SIM_E_WORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, need);
  return create_worlds(p, 1, a, workspace, ws_bytes, stream, out);
}

sim_status sim_set_workspace_size(const sim_params* p, int32_t n_worlds, const sim_arrays* arrays, size_t* bytes) {
  sim_status st = check_params(p);
  if (st) return st;
  if (n_worlds < 1 || !arrays || !bytes) return fail(SIM_E_INVALID, "need n_worlds >= 1 and non-NULL arrays, bytes");
  const size_t ncell = (size_t)p->nx * p->ny;
  size_t packs = 0, bufs = 0;
  for (int i = 0; i < n_worlds; ++i) {
    if (arrays[i].n_filaments < 0 || arrays[i].n_particles < 0) return fail(SIM_E_INVALID, "negative sizes");
    packs += std::max(arrays[i].n_filaments, 1);
    bufs += world_buf_bytes(*p, arrays[i].n_particles);
  }
  size_t tiles[mc::kTileFamilies] = {0, 0, 0};
  tiles[tile_family(*p)] = (size_t)n_worlds * tiles_x(*p) * tiles_y(*p);
  const size_t items = (size_t)n_worlds * ((ncell + mc::kCellsPerItem - 1) / mc::kCellsPerItem);
  const size_t scans = (size_t)n_worlds * ((ncell + 1023) / 1024);
  *bytes = Engine::table_bytes(n_worlds, packs, tiles, items, scans) + bufs;
  return SIM_OK;
}

sim_status sim_create_set(const sim_params* p, int32_t n_worlds, const sim_arrays* arrays, void* workspace,
                          size_t ws_bytes, void* stream, sim_world** out) {
  sim_status st = check_params(p);
  if (st) return st;
  if (n_worlds < 1 || !arrays) return fail(SIM_E_INVALID, "need n_worlds >= 1 and non-NULL arrays");
  for (int i = 0; i < n_worlds; ++i)
    if ((st = check_arrays(&arrays[i]))) return st;
  if (!out) return fail(SIM_E_INVALID, "out is NULL");
  if (!workspace || ((uintptr_t)workspace % kAlign)) return fail(SIM_E_WORKSPACE, "workspace must be 256-byte aligned");
  size_t need = 0;
  if ((st = sim_set_workspace_size(p, n_worlds, arrays, &need))) return st;
  if (ws_bytes < need) return fail(SIM_E_WORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, need);
  return create_worlds(p, n_worlds, arrays, workspace, ws_bytes, stream, out);
}

static sim_status world_run(sim_world* w, int64_t t, int n) {
  Engine& e = w->eng;
  sim_status st;
  for (int k = 0; k < (int)e.slots.size(); ++k)
    if ((st = e.set_ctl(k, t, n))) return st;
  if ((st = e.run_steps(n))) return st;
  if (n & 1) {
    // the state ended in the alternate populations buffers: copy them back
    for (const Slot& s : e.slots) {
      const size_t ncell = (size_t)s.p.nx * s.p.ny;
      HIPCHK(hipMemcpyAsync(s.fbuf[0], s.fbuf[1], 9 * ncell * sizeof(float), hipMemcpyDeviceToDevice, e.stream));
    }
  }
  return SIM_OK;
}

// Bytes of one checkpoint (positions and populations) of a world.
static size_t ckpt_per_world(const Slot& s) {
  return align_up(4 * (size_t)s.n_part * 4) + align_up(9 * (size_t)s.p.nx * s.p.ny * 4);
}

sim_status sim_step(sim_world* w, int64_t t) {
  if (!w) return fail(SIM_E_INVALID, "world is NULL");
  return world_run(w, t, 1);
}

sim_status sim_checkpoint_size(const sim_world* w, int32_t n_steps, int32_t ckpt_every, size_t* bytes) {
  if (!w || !bytes) return fail(SIM_E_INVALID, "NULL argument");
  if (n_steps < 0 || ckpt_every <= 0) return fail(SIM_E_INVALID, "need n_steps >= 0 and ckpt_every > 0");
  const size_t nseg = std::max<size_t>((size_t)(n_steps + ckpt_every - 1) / ckpt_every, 1);
  size_t total = 0;
  for (const Slot& s : w->eng.slots) total += nseg * ckpt_per_world(s);   // the worlds' blocks, one after another
  *bytes = total;
  return SIM_OK;
}

sim_status sim_rollout(sim_world* w, int64_t t0, int32_t n_steps, int32_t ckpt_every, void* ckpt, size_t ckpt_bytes) {
  if (!w) return fail(SIM_E_INVALID, "world is NULL");
  if (n_steps < 0) return fail(SIM_E_INVALID, "n_steps must be >= 0");
  if (ckpt_every < 0) return fail(SIM_E_INVALID, "ckpt_every must be >= 0");
  if (ckpt_every == 0) return world_run(w, t0, n_steps);
  if (!ckpt) return fail(SIM_E_INVALID, "ckpt is NULL but ckpt_every > 0");
  size_t need = 0;
  sim_checkpoint_size(w, n_steps, ckpt_every, &need);
  if (ckpt_bytes < need) return fail(SIM_E_WORKSPACE, "checkpoint buffer has %zu bytes, needs %zu", ckpt_bytes, need);
  Engine& e = w->eng;
  const size_t nseg = std::max<size_t>((size_t)(n_steps + ckpt_every - 1) / ckpt_every, 1);
  int seg = 0;
  for (int k = 0; k < n_steps; k += ckpt_every, ++seg) {
    char* block = (char*)ckpt;
    for (const Slot& s : e.slots) {
      const size_t N = s.n_part, ncell = (size_t)s.p.nx * s.p.ny, per = ckpt_per_world(s);
      char* dst = block + seg * per;
      if (N) {
        HIPCHK(hipMemcpyAsync(dst, s.cell, 2 * N * 4, hipMemcpyDeviceToDevice, e.stream));
        HIPCHK(hipMemcpyAsync(dst + 2 * N * 4, s.frac, 2 * N * 4, hipMemcpyDeviceToDevice, e.stream));
      }
      HIPCHK(hipMemcpyAsync(dst + align_up(4 * N * 4), s.fbuf[0], 9 * ncell * 4, hipMemcpyDeviceToDevice, e.stream));
      block += nseg * per;
    }
    sim_status st = world_run(w, t0 + k, std::min(ckpt_every, n_steps - k));
    if (st) return st;
  }
  return SIM_OK;
}

sim_status sim_sync(sim_world* w) {
  if (!w) return fail(SIM_E_INVALID, "world is NULL");
  Engine& e = w->eng;
  HIPCHK(hipStreamSynchronize(e.stream));
  HIPCHK(hipGetLastError());
  std::vector<unsigned> fl(std::max<size_t>(e.slots.size(), 1), 0u);
  HIPCHK(hipMemcpy(fl.data(), e.flags, fl.size() * sizeof(unsigned), hipMemcpyDeviceToHost));
  unsigned f = 0;
  for (unsigned v : fl) f |= v;
  if (f & mc::kFlagBins) return fail(SIM_E_STATE, "node positions changed without a tile-bin pre-pass");
  if (f) return fail(SIM_E_UNSTABLE, "world produced NaN or |u| > u_max");
  return SIM_OK;
}

sim_status sim_clear_flags(sim_world* w) {
  if (!w) return fail(SIM_E_INVALID, "world is NULL");
  hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, w->eng.stream, (int*)w->eng.flags, w->eng.slots.size());
  HIPCHK(hipGetLastError());
  return SIM_OK;
}

void sim_destroy(sim_world* w) { delete w; }

sim_status sim_debug_substep(sim_world* w, int32_t which, int64_t t) {
  if (!w) return fail(SIM_E_INVALID, "world is NULL");
  if (w->eng.slots.size() != 1) return fail(SIM_E_INVALID, "a single world only");
  Engine& e = w->eng;
  sim_status st;
  if ((st = e.set_ctl(0, t, 1))) return st;
  const mc::WorldDev* d = e.desc[0];
  const mc::Grid& g = e.grid;
  switch (which) {
    case 0:
      mc::launch_bin_prepass(d, e.tab, g, e.stream);
      mc::launch_elastic(d, e.tab, g, e.stream);
      mc::launch_markers(d, e.tab, g, e.stream);
      mc::launch_sort(d, e.tab, g, e.stream);
      break;
    case 1: mc::launch_filter(d, e.tab, g, e.stream); break;
    case 2:
      mc::launch_repulse(d, e.tab, g, e.stream);
      mc::launch_spread(d, e.tab, g, e.stream);
      mc::launch_mdf(d, e.tab, g, e.stream);
      break;
    case 3: {
      mc::launch_lbm(d, e.tab, g, e.stream);
      Slot& s = e.slots[0];
      const size_t ncell = (size_t)s.p.nx * s.p.ny;
      HIPCHK(hipMemcpyAsync(s.fbuf[0], s.fbuf[1], 9 * ncell * sizeof(float), hipMemcpyDeviceToDevice, e.stream));
      break;
    }
    case 4:
      mc::launch_energy(d, e.tab, g, e.stream);
      mc::launch_integrate(d, e.tab, g, e.stream);
      break;
    default: return fail(SIM_E_INVALID, "unknown sub-step %d", which);
  }
  HIPCHK(hipGetLastError());
  return SIM_OK;
}

sim_status sim_profile_steps(sim_world* w, int64_t t0, int32_t n_steps, float* ms_out) {
  if (w && w->eng.slots.size() != 1) return fail(SIM_E_INVALID, "a single world only");
  if (!w || !ms_out) return fail(SIM_E_INVALID, "NULL argument");
  if (n_steps < 1) return fail(SIM_E_INVALID, "n_steps must be >= 1");
  Engine& e = w->eng;
  Slot& s = e.slots[0];
  constexpr int kGroups = 6;
  std::vector<hipEvent_t> ev((size_t)n_steps * (kGroups + 1), nullptr);
  for (auto& x : ev) HIPCHK(hipEventCreate(&x));
  std::vector<hipEvent_t> fl(2 * (size_t)n_steps, nullptr);   // the fluid dispatch's own timestamps
  for (auto& x : fl) HIPCHK(hipEventCreate(&x));
  sim_status st = e.set_ctl(0, t0, n_steps);
  if (st) return st;
  mc::launch_bin_prepass(e.desc[0], e.tab, e.grid, e.stream);
  for (int k = 0; k < n_steps; ++k) {
    const mc::WorldDev* d = e.desc[k & 1];
    hipEvent_t* E = ev.data() + (size_t)k * (kGroups + 1);
    HIPCHK(hipEventRecord(E[0], e.stream));
    mc::launch_elastic(d, e.tab, e.grid, e.stream);
    mc::launch_markers(d, e.tab, e.grid, e.stream);
    HIPCHK(hipEventRecord(E[1], e.stream));
    mc::launch_sort(d, e.tab, e.grid, e.stream);
    HIPCHK(hipEventRecord(E[2], e.stream));
    mc::launch_filter(d, e.tab, e.grid, e.stream);
    HIPCHK(hipEventRecord(E[3], e.stream));
    mc::launch_repulse(d, e.tab, e.grid, e.stream);
    mc::launch_spread(d, e.tab, e.grid, e.stream);
    mc::launch_mdf(d, e.tab, e.grid, e.stream);
    HIPCHK(hipEventRecord(E[4], e.stream));
    mc::launch_lbm_timed(d, e.tab, e.grid, e.stream, fl[2 * k], fl[2 * k + 1]);
    HIPCHK(hipEventRecord(E[5], e.stream));
    mc::launch_energy(d, e.tab, e.grid, e.stream);
    mc::launch_integrate(d, e.tab, e.grid, e.stream);
    HIPCHK(hipEventRecord(E[6], e.stream));
    HIPCHK(hipGetLastError());
  }
  if (n_steps & 1) {
    const size_t ncell = (size_t)s.p.nx * s.p.ny;
    HIPCHK(hipMemcpyAsync(s.fbuf[0], s.fbuf[1], 9 * ncell * sizeof(float), hipMemcpyDeviceToDevice, e.stream));
  }
  HIPCHK(hipStreamSynchronize(e.stream));
  for (int g = 0; g < kGroups; ++g) {
    double tot = 0.0;
    for (int k = 0; k < n_steps; ++k) {
      float ms = 0.f;
      hipEvent_t* E = ev.data() + (size_t)k * (kGroups + 1);
      if (g == 4)
        HIPCHK(hipEventElapsedTime(&ms, fl[2 * k], fl[2 * k + 1]));
      else
        HIPCHK(hipEventElapsedTime(&ms, E[g], E[g + 1]));
      tot += ms;
    }
    ms_out[g] = (float)(tot / n_steps);
  }
  for (auto& x : ev) hipEventDestroy(x);
  for (auto& x : fl) hipEventDestroy(x);
  return SIM_OK;
}

sim_status sim_debug_adjoint(sim_world* w, int32_t which, const void* in, void* out, void* scratch) {
  if (w && w->eng.slots.size() != 1) return fail(SIM_E_INVALID, "a single world only");
  if (!w || !in || !out) return fail(SIM_E_INVALID, "NULL argument");
  Engine& e = w->eng;
  const Slot& s = e.slots[0];
  if (which == 0 && mode_of(s.p) != mc::kBinned) return fail(SIM_E_INVALID, "the spread transpose needs bins");
  if (which == 2 && !scratch) return fail(SIM_E_INVALID, "scratch is needed");
  if (which < 0 || which > 2) return fail(SIM_E_INVALID, "unknown adjoint sub-step %d", which);
  const size_t ncell = (size_t)s.p.nx * s.p.ny;
  mc::AdjDev A{};
  if (which == 1) {
    A.Gbar = (float2*)const_cast<void*>(in);
    A.sbar = (float*)out;
  } else if (which == 2) {
    A.gbar_in = (const float*)in;
    A.gbar = (float*)out;
    A.ubar = (float2*)scratch;
    A.Fgbar = (float2*)scratch + ncell;
    hipLaunchKernelGGL(k_zero_i32, dim3(256), dim3(256), 0, e.stream, (int*)scratch, 2 * ncell);
  }
  mc::launch_adjoint_debug(e.desc[0], e.tab, e.grid, which, A, (const float*)in, (float2*)out, e.stream);
  HIPCHK(hipGetLastError());
  return SIM_OK;
}

sim_status sim_debug_buffer(sim_world* w, int32_t which, void** ptr) {
  if (w && w->eng.slots.size() != 1) return fail(SIM_E_INVALID, "a single world only");
  if (!w || !ptr) return fail(SIM_E_INVALID, "NULL argument");
  const Slot& s = w->eng.slots[0];
  switch (which) {
    case 0: *ptr = s.b.s; break;
    case 1: *ptr = s.b.grad; break;
    case 2: *ptr = s.b.Fg; break;
    case 3: *ptr = s.b.fel; break;
    case 4: *ptr = s.b.fel_el; break;
    default: return fail(SIM_E_INVALID, "unknown buffer %d", which);
  }
  return SIM_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// One step with no world handle and no allocation (sim_step_noalloc)
// ---------------------------------------------------------------------------
namespace {

constexpr size_t kScratchBytes = (size_t)32 << 20;   // 32 MiB per device

}  // namespace

// The workspace of sim_step_noalloc: descriptors, work tables and per-step
// buffers of one world.  Every device the call runs on holds its own copy
// until the process ends.  Host code never passes this name to a kernel or a
// copy (in host code it is not a device address): it uses the per-device
// address that hipGetSymbolAddress returned.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::atomic<void*> g_scratch_ptr[kMaxDevices];

// Address of this device's scratch array, looked up once per device with
// that device current (concurrent first calls look it up twice, harmlessly).
sim_status scratch_address(void** out) {
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(SIM_E_INVALID, "device %d out of range", dev);
  void* ptr = g_scratch_ptr[dev].load(std::memory_order_acquire);
  if (!ptr) {
    HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr || ((uintptr_t)ptr % kAlign)) return fail(SIM_E_HIP, "scratch array has no usable address");
    g_scratch_ptr[dev].store(ptr, std::memory_order_release);
  }
  *out = ptr;
  return SIM_OK;
}

// Layout of the scratch array for one world (base == nullptr: sizing only).
struct NoallocLayout {
  mc::WorldDev* desc = nullptr;   // [2]: step parity 0 and 1
  mc::Ctl* ctl = nullptr;         // [2]
  unsigned* flags = nullptr;      // [1] sticky world flags
  int* counts = nullptr;          // [8] work-list lengths (as the engine's tables)
  int* err = nullptr;             // [1] validation failures of the filament offsets
  mc::Pack* packs = nullptr;      // [F] one filament per pack
  int2* items = nullptr;          // fluid items
  int2* scan = nullptr;           // scan items (sorted transfer)
  int2* wlist = nullptr;          // [1]
  WorldBufs b;
  size_t bytes = 0;
};

void carve_noalloc(char* base, const sim_params& p, int n_fil, int n_part, NoallocLayout& L) {
  Carver c{base};
  const size_t ncell = (size_t)p.nx * p.ny;
  L.desc = c.take<mc::WorldDev>(2);
  L.ctl = c.take<mc::Ctl>(2);
  L.flags = c.take<unsigned>(1);
  L.counts = c.take<int>(8);
  L.err = c.take<int>(1);
  L.packs = c.take<mc::Pack>(std::max(n_fil, 1));
  L.items = c.take<int2>((ncell + mc::kCellsPerItem - 1) / mc::kCellsPerItem);
  L.scan = c.take<int2>((ncell + 1023) / 1024);
  L.wlist = c.take<int2>(1);
  carve_world_bufs(c, p, n_part, L.b);
  L.bytes = c.off;
}

constexpr int kErrOffsets = 1;    // fil_offset[0] != 0 or fil_offset[F] != N
constexpr int kErrLength = 2;     // a filament outside 1..kMaxFilament nodes

// Work tables and descriptors of the world, written on the device (nothing
// is read back to the host): filament f is pack f; its length is checked.
__global__ void k_noalloc_setup(mc::WorldDev d0, mc::WorldDev d1, NoallocLayout L, const int* fil_offset, int n_fil,
                                int n_part, int n_items, int n_scan, long long t) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_fil) {
    const int a = fil_offset[i], e = fil_offset[i + 1];
    if (e - a < 1 || e - a > mc::kMaxFilament) atomicOr(L.err, kErrLength);
    mc::Pack pk{};
    pk.world = 0;
    pk.node_begin = a;
    pk.node_end = e;
    pk.fil_begin = i;
    pk.fil_end = i + 1;
    L.packs[i] = pk;
  }
  if (i < n_items) L.items[i] = make_int2(0, i * mc::kCellsPerItem);
  if (i < n_scan) L.scan[i] = make_int2(0, i);
  if (i == 0) {
    if (n_fil > 0 && (fil_offset[0] != 0 || fil_offset[n_fil] != n_part)) atomicOr(L.err, kErrOffsets);
    L.desc[0] = d0;
    L.desc[1] = d1;
    mc::Ctl c0;
    c0.t = t;
    c0.remaining = 1;
    c0.pad = 0;
    L.ctl[0] = c0;
    mc::Ctl c1 = c0;
    c1.remaining = 0;
    L.ctl[1] = c1;
    *L.flags = 0u;
    *L.wlist = make_int2(0, 0);
  }
}

// Work-list lengths, or none at all (every kernel then idles) when the
// offsets failed their checks.
__global__ void k_noalloc_counts(NoallocLayout L, int n_packs, int n_tiles, int family, int n_scan, int n_items) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const bool ok = *L.err == 0;
  int c[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  c[Engine::kCntPacks] = ok ? n_packs : 0;
  c[Engine::kCntScan] = ok ? n_scan : 0;
  c[Engine::kCntWorlds] = ok ? 1 : 0;
  c[Engine::kCntItems] = ok ? n_items : 0;
  c[Engine::kCntTiles + family] = ok ? n_tiles : 0;
  for (int k = 0; k < 8; ++k) L.counts[k] = c[k];
  if (!ok) L.ctl[0].remaining = 0;
}

// The step's populations back into the caller's array (skipped if the step
// did not run).
__global__ void k_noalloc_copy_back(const int* err, const float* src, float* dst, size_t n) {
  if (*err) return;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

__global__ void k_noalloc_status(const int* err, const unsigned* flags, int32_t* status) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const unsigned f = *flags;
  *status = *err ? SIM_E_INVALID : (f & mc::kFlagBins) ? SIM_E_STATE : f ? SIM_E_UNSTABLE : SIM_OK;
}

}  // namespace

extern "C" {

sim_status sim_step_noalloc(const sim_params* p, const sim_arrays* a, int64_t t, int32_t* status, void* stream) {
  sim_status st = check_params(p);
  if (st) return st;
  if ((st = check_arrays(a))) return st;
  if (a->fil_parent) return fail(SIM_E_INVALID, "sim_step_noalloc does not take branched worlds (fil_parent)");
  NoallocLayout L;
  carve_noalloc(nullptr, *p, a->n_filaments, a->n_particles, L);
  if (L.bytes > kScratchBytes)
    return fail(SIM_E_WORKSPACE, "world needs %zu bytes of scratch; sim_step_noalloc holds %zu", L.bytes,
                kScratchBytes);
  void* base = nullptr;
  if ((st = scratch_address(&base))) return st;
  carve_noalloc((char*)base, *p, a->n_filaments, a->n_particles, L);
  hipStream_t s = (hipStream_t)stream;
  const size_t ncell = (size_t)p->nx * p->ny;
  const size_t nt = n_bins(*p);
  const int n_items = (int)((ncell + mc::kCellsPerItem - 1) / mc::kCellsPerItem);
  const int n_scan = (int)((ncell + 1023) / 1024);
  const int n_fil = a->n_filaments, n_part = a->n_particles;

  // the world as the engine would describe it, over the scratch buffers
  Slot sl;
  sl.used = true;
  sl.p = *p;
  sl.n_fil = n_fil;
  sl.n_part = n_part;
  sl.fil_offset = const_cast<int*>(a->fil_offset);
  sl.cell = a->cell;
  sl.frac = a->frac;
  sl.rest_angle = const_cast<float*>(a->rest_angle);
  sl.rest_length = const_cast<float*>(a->rest_length);
  sl.amp = const_cast<float*>(a->act_amp);
  sl.period = const_cast<float*>(a->act_period);
  sl.phase = const_cast<float*>(a->act_phase);
  sl.kb = const_cast<float*>(a->k_bend);
  sl.ks = const_cast<float*>(a->k_stretch);
  sl.ksh = const_cast<float*>(a->k_shear);
  sl.fil_flags = const_cast<int*>(a->fil_flags);
  sl.energy = a->energy;
  sl.e_sensed = a->energy_sensed;
  sl.e_collected = a->energy_collected;
  sl.b = L.b;
  sl.fbuf[0] = a->f;
  sl.fbuf[1] = L.b.f_alt;
  sl.u = a->u;
  sl.cur = 0;
  const mc::WorldDev d0 = world_desc(sl, 0, L.ctl + 0, L.ctl + 1, L.flags);
  const mc::WorldDev d1 = world_desc(sl, 1, L.ctl + 1, L.ctl + 0, L.flags);

  mc::Tables tab{};
  const int fam = tile_family(*p);
  tab.packs = L.packs;
  tab.n_packs = L.counts + Engine::kCntPacks;
  for (int f = 0; f < mc::kTileFamilies; ++f) {
    tab.tiles[f] = nullptr;
    tab.n_tiles[f] = L.counts + Engine::kCntTiles + f;
  }
  tab.scan = L.scan;
  tab.n_scan = L.counts + Engine::kCntScan;
  tab.worlds = L.wlist;
  tab.n_worlds = L.counts + Engine::kCntWorlds;
  tab.items = L.items;
  tab.n_items = L.counts + Engine::kCntItems;
  tab.single_ntx[fam] = tiles_x(*p);
  mc::Grid g{};
  g.pack = 1024;                                  // one filament (<= 1024 nodes) per pack
  g.node_blocks = std::max(1, std::min(n_fil, 8192));
  g.tile_blocks[fam] = (int)std::max<size_t>(1, nt);
  g.item_blocks = std::max(1, n_items);
  g.scan_blocks = std::max(1, n_scan);
  g.world_blocks = 1;
  const int mode = mode_of(*p);
  g.any_sorted = mode == mc::kSorted;
  g.any_binned = mode == mc::kBinned;
  g.any_node = mode != mc::kBinned;
  g.max_radius = p->repulse_radius;
  g.any_energy = p->energy_rate > 0.f && a->energy ? 1 : 0;
  g.any_markers = L.b.d_marker ? 1 : 0;
  g.mk_only = mode == mc::kBinned && L.b.d_marker ? 1 : 0;
  g.mdf_max = L.b.U_d ? std::max(p->mdf_iters, 1) : 1;
  g.general = slot_general(sl) ? 1 : 0;

  // the array keeps the previous call's contents: clear what starts at zero
  hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, s, L.err, (size_t)1);
  if (L.b.Fg) hipLaunchKernelGGL(k_zero_i32, dim3(256), dim3(256), 0, s, (int*)L.b.Fg, 2 * ncell);
  if (L.b.s) hipLaunchKernelGGL(k_zero_i32, dim3(256), dim3(256), 0, s, (int*)L.b.s, ncell);
  if (L.b.cnt) hipLaunchKernelGGL(k_zero_i32, dim3(256), dim3(256), 0, s, L.b.cnt, ncell);
  if (L.b.e_node)
    hipLaunchKernelGGL(k_zero_i32, dim3(64), dim3(256), 0, s, (int*)L.b.e_node, (size_t)std::max(n_part, 1));
  if (L.b.bin_cnt) {
    hipLaunchKernelGGL(k_zero_i32, dim3(64), dim3(256), 0, s, L.b.bin_cnt, nt);
    hipLaunchKernelGGL(k_zero_i32, dim3(64), dim3(256), 0, s, L.b.bin_fill, nt);
    hipLaunchKernelGGL(k_zero_i32, dim3(64), dim3(256), 0, s, L.b.sp_cnt, nt);
    mc::launch_tile_ranges(p->nx, p->ny, p->repulse_radius, tile_side(*p), L.b.tile_rng, s);
  }
  const int setup_n = std::max({n_fil, n_items, n_scan, 1});
  hipLaunchKernelGGL(k_noalloc_setup, dim3((setup_n + 255) / 256), dim3(256), 0, s, d0, d1, L, a->fil_offset, n_fil,
                     n_part, n_items, n_scan, (long long)t);
  hipLaunchKernelGGL(k_noalloc_counts, dim3(1), dim3(64), 0, s, L, n_fil, (int)nt, fam, n_scan, n_items);
  // the step itself: the kernels sim_step runs, with parity-0 descriptors
  mc::launch_bin_prepass(L.desc, tab, g, s);
  mc::launch_elastic(L.desc, tab, g, s);
  mc::launch_markers(L.desc, tab, g, s);
  mc::launch_sort(L.desc, tab, g, s);
  mc::launch_filter(L.desc, tab, g, s);
  mc::launch_repulse(L.desc, tab, g, s);
  mc::launch_spread(L.desc, tab, g, s);
  mc::launch_mdf(L.desc, tab, g, s);
  mc::launch_lbm(L.desc, tab, g, s);
  mc::launch_energy(L.desc, tab, g, s);
  mc::launch_integrate(L.desc, tab, g, s);
  hipLaunchKernelGGL(k_noalloc_copy_back, dim3(std::min<size_t>(2048, (9 * ncell + 255) / 256)), dim3(256), 0, s,
                     L.err, (const float*)L.b.f_alt, a->f, 9 * ncell);
  if (status) hipLaunchKernelGGL(k_noalloc_status, dim3(1), dim3(64), 0, s, L.err, L.flags, status);
  HIPCHK(hipGetLastError());
  return SIM_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Folding objective (sim_density_loss)
// ---------------------------------------------------------------------------
namespace {

sim_status check_splat(const sim_splat_image* img) {
  if (!img) return fail(SIM_E_INVALID, "image description is NULL");
  if (img->width < 1 || img->height < 1 || img->width > 16384 || img->height > 16384)
    return fail(SIM_E_INVALID, "image sides must be in 1..16384");
  if (!(img->sigma > 0.f) || !std::isfinite(img->sigma) || !std::isfinite(img->amp))
    return fail(SIM_E_INVALID, "sigma must be positive and amp finite");
  return SIM_OK;
}

}  // namespace

extern "C" {

sim_status sim_density_loss_workspace_size(const sim_splat_image* img, size_t* bytes) {
  sim_status st = check_splat(img);
  if (st) return st;
  if (!bytes) return fail(SIM_E_INVALID, "bytes is NULL");
  *bytes = mc::density_loss_workspace(img->width, img->height);
  return SIM_OK;
}

sim_status sim_density_loss(const sim_splat_image* img, int32_t nx, int32_t ny, int32_t n_particles,
                            const int32_t* cell, const float* frac, const float* target, float* image, float* loss,
                            float* g_pos, void* workspace, size_t ws_bytes, void* stream) {
  sim_status st = check_splat(img);
  if (st) return st;
  if (nx < 1 || ny < 1 || n_particles < 0) return fail(SIM_E_INVALID, "bad world size");
  if (!target || !loss) return fail(SIM_E_INVALID, "target and loss must be given");
  if (n_particles > 0 && (!cell || !frac)) return fail(SIM_E_INVALID, "positions must be given");
  const float hx = (float)nx / img->width, hy = (float)ny / img->height;
  const double wx = std::min<double>(img->width, 2.0 * std::floor(5.0 * img->sigma / hx + 0.5) + 3);
  const double wy = std::min<double>(img->height, 2.0 * std::floor(5.0 * img->sigma / hy + 0.5) + 3);
  if (wx * wy > 65536.0)
    return fail(SIM_E_INVALID, "sigma covers %.0f pixels per node (at most 65536)", wx * wy);
  if (!workspace || ((uintptr_t)workspace % kAlign)) return fail(SIM_E_WORKSPACE, "workspace must be 256-byte aligned");
  const size_t need = mc::density_loss_workspace(img->width, img->height);
  if (ws_bytes < need) return fail(SIM_E_WORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, need);
  mc::launch_density_loss(nx, ny, n_particles, img->width, img->height, img->sigma, img->amp, cell, frac, target,
                          image, loss, g_pos, workspace, (hipStream_t)stream);
  HIPCHK(hipGetLastError());
  return SIM_OK;
}

sim_status sim_energy_packets(int32_t nx, int32_t ny, int32_t n_packets, const float* centres, const float* amps,
                              const float* widths, float* field, void* stream) {
  if (nx < 1 || ny < 1 || n_packets < 0 || !field) return fail(SIM_E_INVALID, "bad field or packet count");
  if (n_packets == 0) return SIM_OK;
  if (!centres || !amps || !widths) return fail(SIM_E_INVALID, "NULL packet array");
  mc::launch_energy_packets(nx, ny, n_packets, centres, amps, widths, field, (hipStream_t)stream);
  HIPCHK(hipGetLastError());
  return SIM_OK;
}

sim_status sim_rest_effort(int32_t n_filaments, const int32_t* fil_offset, const int32_t* fil_flags,
                           const float* old_rest_angle, const float* new_rest_angle, const float* old_rest_length,
                           const float* new_rest_length, float* effort, void* stream) {
  if (n_filaments < 0) return fail(SIM_E_INVALID, "negative filament count");
  if (n_filaments == 0) return SIM_OK;
  if (!fil_offset || !old_rest_angle || !new_rest_angle || !old_rest_length || !new_rest_length || !effort)
    return fail(SIM_E_INVALID, "NULL array");
  mc::launch_rest_effort(n_filaments, fil_offset, fil_flags, old_rest_angle, new_rest_angle, old_rest_length,
                         new_rest_length, effort, (hipStream_t)stream);
  HIPCHK(hipGetLastError());
  return SIM_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Reverse mode (sim_backward)
// ---------------------------------------------------------------------------
namespace {

// Layout of the backward workspace for segments of up to m steps.
struct AdjLayout {
  int m = 0;
  size_t N = 0, ncell = 0, nt = 0;
  int* cell[2] = {};           // unused placeholders for alignment bookkeeping
  size_t bytes = 0;
  // per tape slot
  std::vector<int*> x_cell;    // m+1 slots of [2][N]
  std::vector<float*> x_frac;  // m+1 slots of [2][N]
  std::vector<float*> g;       // m+1 slots of [9][ncell]
  std::vector<float2*> grad, Fg, u;   // m slots of [ncell]
  std::vector<float*> F;       // m slots of [2][N]
  std::vector<int*> bstart;    // m + 1 slots of [nt+1] (step j's bins; slot m is scratch)
  std::vector<int4*> brec;     // m slots of [N]
  std::vector<int4*> sprec;    // m slots of the spread lists the recomputed filter writes
  std::vector<int*> spcnt;     // m slots of their lengths
  int* bin_cnt = nullptr;
  int* bin_fill = nullptr;
  float* xbar[2] = {};
  float* gbar[2] = {};
  float2* ubar = nullptr;
  float2* Fgbar = nullptr;
  float2* Gbar = nullptr;
  float* sbar = nullptr;
  float* Fbar = nullptr;
  mc::Ctl* ctl = nullptr;            // m + 1 control words: step j reads ctl[j], writes ctl[j + 1]
  // multi-direct forcing (worlds with mdf_iters K > 1)
  float2* Fgk = nullptr;             // [K-1][ncell] recomputed iterates
  float* Ud = nullptr;               // [2][N]
  float* mc = nullptr;               // [2][N]
  float* Ukbar = nullptr;            // [2][N]
  float* Udbar = nullptr;            // [2][N]
  float* xbar_m = nullptr;           // [2][N]
  float2* jbar = nullptr;            // [ncell]
  float* rhobar = nullptr;           // [ncell]
  // two-layer markers
  float* dbar = nullptr;             // [2][N]
  float* dbar_m = nullptr;           // [2][N] (with MDF)
};

void carve_adj(Carver& c, const sim_params& p, int n_part, int m, AdjLayout& L) {
  L.m = m;
  L.N = std::max(n_part, 1);
  L.ncell = (size_t)p.nx * p.ny;
  L.nt = n_bins(p);
  L.x_cell.resize(m + 1);
  L.x_frac.resize(m + 1);
  L.g.resize(m + 1);
  for (int j = 0; j <= m; ++j) {
    L.x_cell[j] = c.take<int>(2 * L.N);
    L.x_frac[j] = c.take<float>(2 * L.N);
    L.g[j] = c.take<float>(9 * L.ncell);
  }
  L.grad.resize(m);
  L.Fg.resize(m);
  L.u.resize(m);
  L.F.resize(m);
  L.bstart.resize(m + 1);
  L.brec.resize(m);
  L.sprec.resize(m);
  L.spcnt.resize(m);
  const size_t ntiles = (size_t)tiles_x(p) * tiles_y(p);
  for (int j = 0; j < m; ++j) {
    L.grad[j] = c.take<float2>(L.ncell);
    L.Fg[j] = c.take<float2>(L.ncell);
    L.u[j] = c.take<float2>(L.ncell);
    L.F[j] = c.take<float>(2 * L.N);
    L.bstart[j] = c.take<int>(L.nt + 1);
    L.brec[j] = c.take<int4>(L.N);
    L.sprec[j] = c.take<int4>(ntiles * mc::spread_cap_of_side(tile_side(p)));
    L.spcnt[j] = c.take<int>(ntiles);
  }
  L.bstart[m] = c.take<int>(L.nt + 1);
  L.bin_cnt = c.take<int>(L.nt);
  L.bin_fill = c.take<int>(L.nt);
  for (int k = 0; k < 2; ++k) {
    L.xbar[k] = c.take<float>(2 * L.N);
    L.gbar[k] = c.take<float>(9 * L.ncell);
  }
  L.ubar = c.take<float2>(L.ncell);
  L.Fgbar = c.take<float2>(L.ncell);
  L.Gbar = c.take<float2>(L.ncell);
  L.sbar = c.take<float>(L.ncell);
  L.Fbar = c.take<float>(2 * L.N);
  L.ctl = c.take<mc::Ctl>(m + 1);
  if (p.mdf_iters > 1) {
    L.Fgk = c.take<float2>((size_t)(p.mdf_iters - 1) * L.ncell);
    L.Ud = c.take<float>(2 * L.N);
    L.mc = c.take<float>(2 * L.N);
    L.Ukbar = c.take<float>(2 * L.N);
    L.Udbar = c.take<float>(2 * L.N);
    L.xbar_m = c.take<float>(2 * L.N);
    L.jbar = c.take<float2>(L.ncell);
    L.rhobar = c.take<float>(L.ncell);
  }
  if (p.marker_offset > 0.f) {
    L.dbar = c.take<float>(2 * L.N);
    if (p.mdf_iters > 1) L.dbar_m = c.take<float>(2 * L.N);
  }
  L.bytes = c.off;
}

}  // namespace

extern "C" {

// The adjoint workspace of a handle: each world's tape and buffers, then the
// per-step descriptors [m][worlds] and adjoint buffer sets [m][2][worlds]
// (by the parity of the adjoint state).
struct AdjShared {
  mc::WorldDev* desc = nullptr;
  mc::AdjDev* adj = nullptr;
};

static size_t carve_backward(Carver& c, const Engine& e, int m, std::vector<AdjLayout>& Ls, AdjShared& S) {
  const size_t nw = e.slots.size();
  Ls.assign(nw, AdjLayout());
  for (size_t w = 0; w < nw; ++w) carve_adj(c, e.slots[w].p, e.slots[w].n_part, m, Ls[w]);
  S.desc = c.take<mc::WorldDev>((size_t)m * nw);
  S.adj = c.take<mc::AdjDev>((size_t)2 * m * nw);
  return c.off;
}

sim_status sim_backward_workspace_size(const sim_world* w, int32_t ckpt_every, size_t* bytes) {
  if (!w || !bytes) return fail(SIM_E_INVALID, "NULL argument");
  if (ckpt_every < 1) return fail(SIM_E_INVALID, "ckpt_every must be >= 1");
  Carver c{nullptr};
  std::vector<AdjLayout> Ls;
  AdjShared S;
  *bytes = carve_backward(c, w->eng, ckpt_every, Ls, S);
  return SIM_OK;
}

sim_status sim_backward(sim_world* w, int64_t t0, int32_t n_steps, int32_t ckpt_every, const void* ckpt,
                        const float* g_pos, float* g_rest_angle, float* g_pos0, void* adj_ws, size_t adj_ws_bytes) {
  if (!w) return fail(SIM_E_INVALID, "world is NULL");
  if (n_steps < 1 || ckpt_every < 1) return fail(SIM_E_INVALID, "need n_steps >= 1 and ckpt_every >= 1");
  if (!ckpt || !g_pos || !g_rest_angle || !adj_ws) return fail(SIM_E_INVALID, "NULL buffer");
  if ((uintptr_t)adj_ws % kAlign) return fail(SIM_E_WORKSPACE, "adjoint workspace must be 256-byte aligned");
  Engine& e = w->eng;
  const int nw = (int)e.slots.size();
  for (const Slot& s : e.slots) {
    if (mode_of(s.p) != mc::kBinned)
      return fail(SIM_E_INVALID, "sim_backward needs the tile-binned transfer (world created with SIM_SPLAT_%s)",
                  mode_of(s.p) == mc::kSorted ? "SORTED" : "DIRECT");
    if (s.p.pbd_iters > 8) return fail(SIM_E_INVALID, "the adjoint supports at most 8 PBD iterations");
  }
  size_t need = 0;
  sim_backward_workspace_size(w, ckpt_every, &need);
  if (adj_ws_bytes < need) return fail(SIM_E_WORKSPACE, "adjoint workspace has %zu bytes, needs %zu", adj_ws_bytes, need);
  Carver c{(char*)adj_ws};
  std::vector<AdjLayout> Ls;
  AdjShared S;
  carve_backward(c, e, ckpt_every, Ls, S);
  const int m_max = ckpt_every;
  const int nseg = (n_steps + ckpt_every - 1) / ckpt_every;
  const int K = std::max(e.slots[0].p.mdf_iters, 1);
  hipStream_t st = e.stream;
  mc::Grid g = e.grid;
  g.any_binned = 1;
  g.pbd_max = 0;
  for (const Slot& s : e.slots) g.pbd_max = std::max(g.pbd_max, s.p.pbd_iters);
  g.any_sorted = 0;
  g.any_node = 0;
  g.any_energy = 0;                      // the energy field does not act on the motion
  // the worlds' offsets in the caller's node arrays and checkpoint blocks
  std::vector<size_t> noff(nw, 0), coff(nw, 0);
  for (int k = 1; k < nw; ++k) {
    noff[k] = noff[k - 1] + e.slots[k - 1].n_part;
    coff[k] = coff[k - 1] + (size_t)nseg * ckpt_per_world(e.slots[k - 1]);
  }

  // per-step descriptors and adjoint buffer sets (identical for every segment; uploaded once)
  std::vector<mc::WorldDev> hd((size_t)m_max * nw);
  std::vector<mc::AdjDev> ha((size_t)2 * m_max * nw);
  for (int j = 0; j < m_max; ++j)
    for (int k = 0; k < nw; ++k) {
      const AdjLayout& L = Ls[k];
      mc::WorldDev d = e.make_desc(k, 0);
      d.mode = mc::kBinned;
      d.cell_in = L.x_cell[j];
      d.frac_in = L.x_frac[j];
      d.cell_out = L.x_cell[j + 1];
      d.frac_out = L.x_frac[j + 1];
      d.f_src = L.g[j];
      d.f_dst = L.g[j + 1];
      d.grad = L.grad[j];
      d.Fg = L.Fg[j];
      d.u = L.u[j];
      d.fel = L.F[j];
      d.bin_cnt = L.bin_cnt;
      d.bin_fill = L.bin_fill;
      d.bin_start = L.bstart[j];
      d.bin_start_next = L.bstart[j + 1];
      d.bin_rec = L.brec[j];
      d.sp_rec = L.sprec[j];                   // step j's spread lists, for the adjoint spreads
      d.sp_cnt = L.spcnt[j];
      d.ctl_src = L.ctl + j;                   // the fluid kernel of step j advances it into j + 1
      d.ctl_dst = L.ctl + j + 1;
      d.s = nullptr;
      d.energy = nullptr;                    // the recompute leaves the world's energy field alone
      d.e_sensed = nullptr;
      d.e_collected = nullptr;
      hd[(size_t)j * nw + k] = d;
      for (int cur = 0; cur < 2; ++cur) {
        mc::AdjDev A{};
        A.xbar_in = L.xbar[cur];
        A.xbar = L.xbar[1 - cur];
        A.gbar_in = L.gbar[cur];
        A.gbar = L.gbar[1 - cur];
        A.ubar = L.ubar;
        A.Fgbar = L.Fgbar;
        A.Gbar = L.Gbar;
        A.sbar = L.sbar;
        A.Fbar = L.Fbar;
        A.g_rest = g_rest_angle + noff[k];
        A.mdf = K;
        A.F = L.F[j];
        A.Fgk = L.Fgk;
        A.Ud = L.Ud;
        A.mc = L.mc;
        A.Ukbar = L.Ukbar;
        A.Udbar = L.Udbar;
        A.xbar_m = L.xbar_m;
        A.jbar = L.jbar;
        A.rhobar = L.rhobar;
        A.dbar = L.dbar;
        A.dbar_m = L.dbar_m;
        ha[((size_t)j * 2 + cur) * nw + k] = A;
      }
    }
  HIPCHK(hipEventSynchronize(e.upload_done));
  const size_t dbytes = hd.size() * sizeof(mc::WorldDev), abytes = ha.size() * sizeof(mc::AdjDev);
  if (dbytes + abytes > e.pinned_bytes) {
    HIPCHK(hipHostFree(e.pinned));
    e.pinned_bytes = (dbytes + abytes) * 2;
    HIPCHK(hipHostMalloc((void**)&e.pinned, e.pinned_bytes, hipHostMallocDefault));
  }
  std::memcpy(e.pinned, hd.data(), dbytes);
  std::memcpy(e.pinned + dbytes, ha.data(), abytes);
  HIPCHK(hipMemcpyAsync(S.desc, e.pinned, dbytes, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(S.adj, e.pinned + dbytes, abytes, hipMemcpyHostToDevice, st));
  HIPCHK(hipEventRecord(e.upload_done, st));
  // dL/dx_T from the caller, dL/dg_T = 0, empty bins
  for (int k = 0; k < nw; ++k) {
    const AdjLayout& L = Ls[k];
    const size_t N = e.slots[k].n_part;
    hipLaunchKernelGGL(k_zero_i32, dim3(64), dim3(256), 0, st, L.bin_cnt, L.nt);
    hipLaunchKernelGGL(k_zero_i32, dim3(64), dim3(256), 0, st, L.bin_fill, L.nt);
    if (N) HIPCHK(hipMemcpyAsync(L.xbar[0], g_pos + 2 * noff[k], 2 * N * 4, hipMemcpyDeviceToDevice, st));
    hipLaunchKernelGGL(k_zero_i32, dim3(256), dim3(256), 0, st, (int*)L.gbar[0], 9 * L.ncell);
  }
  HIPCHK(hipGetLastError());

  int cur = 0;
  for (int seg = nseg - 1; seg >= 0; --seg) {
    const int k0 = seg * ckpt_every;
    const int m = std::min(ckpt_every, n_steps - k0);
    for (int k = 0; k < nw; ++k) {
      const AdjLayout& L = Ls[k];
      const size_t N = e.slots[k].n_part;
      const char* ck = (const char*)ckpt + coff[k] + seg * ckpt_per_world(e.slots[k]);
      if (N) {
        HIPCHK(hipMemcpyAsync(L.x_cell[0], ck, 2 * N * 4, hipMemcpyDeviceToDevice, st));
        HIPCHK(hipMemcpyAsync(L.x_frac[0], ck + 2 * N * 4, 2 * N * 4, hipMemcpyDeviceToDevice, st));
      }
      HIPCHK(hipMemcpyAsync(L.g[0], ck + align_up(4 * N * 4), 9 * L.ncell * 4, hipMemcpyDeviceToDevice, st));
      // one control word write per segment and world: each recomputed step's
      // fluid kernel sets the next step's time index
      mc::launch_set_ctl(L.ctl, t0 + k0, m, st);
    }
    // recompute the segment forward for every world, writing each step's fields to the tapes
    mc::launch_bin_prepass(S.desc, e.tab, g, st);
    for (int j = 0; j < m; ++j) e.enqueue_step_with(S.desc + (size_t)j * nw, g, st);
    HIPCHK(hipGetLastError());
    // reverse the segment step by step, every world in the same launches
    for (int j = m - 1; j >= 0; --j) {
      mc::AdjArg a{};
      a.arr = S.adj + ((size_t)j * 2 + cur) * nw;
      mc::launch_adjoint_step(S.desc + (size_t)j * nw, e.tab, g, a, K, st);
      cur = 1 - cur;
    }
    HIPCHK(hipGetLastError());
  }
  if (g_pos0)
    for (int k = 0; k < nw; ++k) {
      const size_t N = e.slots[k].n_part;
      if (N) HIPCHK(hipMemcpyAsync(g_pos0 + 2 * noff[k], Ls[k].xbar[cur], 2 * N * 4, hipMemcpyDeviceToDevice, st));
    }
  return SIM_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batch of worlds in a caller pool
// ---------------------------------------------------------------------------
struct sim_batch {
  Engine eng;
  char* pool = nullptr;
  size_t pool_bytes = 0;
  size_t table_bytes = 0;
  std::map<size_t, size_t> free_list;   // offset -> length, inside the pool
};

namespace {

struct BatchWorldLayout {
  size_t bytes = 0;
};

void carve_batch_world(Carver& c, const sim_params& p, int n_fil, int n_part, Slot& s) {
  const size_t ncell = (size_t)p.nx * p.ny;
  const size_t N = std::max(n_part, 1), F = std::max(n_fil, 1);
  s.fil_offset = c.take<int>(F + 1);
  s.cell = c.take<int>(2 * N);
  s.frac = c.take<float>(2 * N);
  s.rest_angle = c.take<float>(N);
  s.rest_length = c.take<float>(N);
  s.amp = c.take<float>(F);
  s.period = c.take<float>(F);
  s.phase = c.take<float>(F);
  s.kb = c.take<float>(N);              // optional per-edge stiffnesses and filament flags:
  s.ks = c.take<float>(N);              // pointed at only when the admitted world has them
  s.ksh = c.take<float>(N);
  s.fil_flags = c.take<int>(F);
  s.fil_parent = c.take<int>(F);
  s.fil_attach = c.take<float>(3 * F);
  if (p.energy_rate > 0.f) {             // energy field and collected totals live in the pool
    s.energy = c.take<float>(ncell);
    s.e_collected = c.take<float>(F);
  }
  s.fbuf[0] = c.take<float>(9 * ncell);
  s.u = c.take<float>(2 * ncell);
  carve_world_bufs(c, p, n_part, s.b);
  s.fbuf[1] = s.b.f_alt;
}

bool pool_alloc(sim_batch* b, size_t bytes, size_t* off) {
  for (auto it = b->free_list.begin(); it != b->free_list.end(); ++it) {
    if (it->second >= bytes) {
      *off = it->first;
      const size_t rest = it->second - bytes;
      const size_t roff = it->first + bytes;
      b->free_list.erase(it);
      if (rest) b->free_list[roff] = rest;
      return true;
    }
  }
  return false;
}

void pool_free(sim_batch* b, size_t off, size_t len) {
  auto it = b->free_list.emplace(off, len).first;
  auto nx = std::next(it);
  if (nx != b->free_list.end() && it->first + it->second == nx->first) {
    it->second += nx->second;
    b->free_list.erase(nx);
  }
  if (it != b->free_list.begin()) {
    auto pv = std::prev(it);
    if (pv->first + pv->second == it->first) {
      pv->second += it->second;
      b->free_list.erase(it);
    }
  }
}

}  // namespace

extern "C" {

sim_status sim_batch_world_bytes(const sim_params* p, int32_t n_filaments, int32_t n_particles, size_t* bytes) {
  sim_status st = check_params(p);
  if (st) return st;
  if (!bytes || n_filaments < 0 || n_particles < 0) return fail(SIM_E_INVALID, "bad argument");
  Carver c{nullptr};
  Slot s;
  carve_batch_world(c, *p, n_filaments, n_particles, s);
  *bytes = c.off;
  return SIM_OK;
}

sim_status sim_batch_create(int32_t max_worlds, void* pool, size_t pool_bytes, void* stream, sim_batch** out) {
  if (max_worlds < 1 || max_worlds > 65536) return fail(SIM_E_INVALID, "max_worlds must be in 1..65536");
  if (!pool || ((uintptr_t)pool % kAlign) || !out) return fail(SIM_E_INVALID, "pool must be 256-byte aligned");
  sim_batch* b = new sim_batch();
  Engine& e = b->eng;
  e.stream = (hipStream_t)stream;
  e.max_worlds = max_worlds;
  // table capacities bounded by what the pool can hold: every cell costs at
  // least 96 bytes, every node at least 36 bytes
  const size_t max_cells = pool_bytes / 96 + 1;
  const size_t max_nodes = pool_bytes / 36 + 1;
  // a world of c cells (both sides >= 8) has at most c/T^2 + nx/T + ny/T + 1
  // <= 5c/256 + 1 tiles of side T >= 16
  for (int f = 0; f < mc::kTileFamilies; ++f) e.max_tiles[f] = max_cells / 48 + max_worlds;
  e.max_items = max_cells / mc::kCellsPerItem + max_worlds;
  e.max_scan = max_cells / 1024 + max_worlds;
  e.max_packs = 2 * (max_nodes / 256) + 2 * (size_t)max_worlds;
  b->table_bytes = Engine::table_bytes(max_worlds, e.max_packs, e.max_tiles, e.max_items, e.max_scan);
  if (b->table_bytes >= pool_bytes / 2) {
    delete b;
    return fail(SIM_E_WORKSPACE, "pool too small for %d worlds", max_worlds);
  }
  Carver c{(char*)pool};
  e.carve_tables(c);
  b->pool = (char*)pool;
  b->pool_bytes = pool_bytes;
  b->free_list[align_up(b->table_bytes)] = pool_bytes - align_up(b->table_bytes);
  e.slots.resize(max_worlds);
  e.fixed_grid = true;
  e.grid.pack = 256;
  e.grid.node_blocks = 2048;
  e.fixed_tile_blocks = 2048;
  e.grid.scan_blocks = 1024;
  e.grid.world_blocks = 256;
  e.grid.item_blocks = 4096;
  e.want_chunk = 20;
  sim_status st = e.init_host(1 << 20);
  if (st) {
    delete b;
    return st;
  }
  hipLaunchKernelGGL(k_zero_i32, dim3(64), dim3(256), 0, e.stream, (int*)e.flags, (size_t)max_worlds);
  hipLaunchKernelGGL(k_zero_i32, dim3(64), dim3(256), 0, e.stream, (int*)e.ctl[0], max_worlds * sizeof(mc::Ctl) / 4);
  hipLaunchKernelGGL(k_zero_i32, dim3(64), dim3(256), 0, e.stream, (int*)e.ctl[1], max_worlds * sizeof(mc::Ctl) / 4);
  if (hipGetLastError() != hipSuccess) {
    delete b;
    return fail(SIM_E_HIP, "initialisation kernels failed to launch");
  }
  if ((st = e.rebuild())) {
    delete b;
    return st;
  }
  *out = b;
  return SIM_OK;
}

sim_status sim_batch_set_tuning(sim_batch* b, int32_t chunk_steps, int32_t cell_blocks, int32_t node_blocks) {
  if (!b) return fail(SIM_E_INVALID, "batch is NULL");
  if (chunk_steps < 2 || (chunk_steps & 1) || cell_blocks < 1 || node_blocks < 1)
    return fail(SIM_E_INVALID, "chunk_steps must be even and >= 2; block counts >= 1");
  Engine& e = b->eng;
  e.want_chunk = chunk_steps;
  e.fixed_tile_blocks = std::max(1, cell_blocks / 4);
  for (int f = 0; f < mc::kTileFamilies; ++f)
    if (e.grid.tile_blocks[f] > 0) e.grid.tile_blocks[f] = e.fixed_tile_blocks;
  e.grid.item_blocks = cell_blocks;
  e.grid.node_blocks = node_blocks;
  e.grid.scan_blocks = std::max(1, cell_blocks / 2);
  e.drop_graphs();
  return SIM_OK;
}

sim_status sim_batch_admit(sim_batch* b, const sim_params* p, const sim_arrays* init, int64_t t0, int32_t steps,
                           int32_t* slot) {
  if (!b || !slot) return fail(SIM_E_INVALID, "NULL argument");
  sim_status st = check_params(p);
  if (st) return st;
  if ((st = check_arrays(init))) return st;
  if (steps < 0) return fail(SIM_E_INVALID, "steps must be >= 0");
  Engine& e = b->eng;
  int w = -1;
  for (int k = 0; k < e.max_worlds; ++k)
    if (!e.slots[k].used) {
      w = k;
      break;
    }
  if (w < 0) return fail(SIM_E_FULL, "no free slot");
  std::vector<int> h_off;
  if (init->n_filaments > 0) {
    if ((st = read_offsets(init, e.stream, h_off))) return st;
  } else {
    h_off.assign(1, 0);
  }
  std::vector<int> unit_next;
  int max_len = 0;
  bool any_branch = false;
  if ((st = read_branches(init, e.stream, h_off, &unit_next, &max_len, &any_branch))) return st;
  if (max_len > e.grid.pack)
    return fail(SIM_E_INVALID, "batched filaments (with those hanging from them) are limited to %d nodes", e.grid.pack);
  bool any_loop = false;
  if ((st = read_loops(init, e.stream, &any_loop))) return st;
  size_t bytes = 0;
  sim_batch_world_bytes(p, init->n_filaments, init->n_particles, &bytes);
  size_t off = 0;
  if (!pool_alloc(b, bytes, &off)) return fail(SIM_E_WORKSPACE, "pool exhausted (world needs %zu bytes)", bytes);
  Slot s;
  s.used = true;
  s.p = *p;
  s.n_fil = init->n_filaments;
  s.n_part = init->n_particles;
  s.max_len = max_len;
  s.h_off = h_off;
  s.pool_off = off;
  s.pool_len = bytes;
  Carver c{b->pool + off};
  carve_batch_world(c, *p, s.n_fil, s.n_part, s);
  const size_t N = s.n_part, F = s.n_fil, ncell = (size_t)p->nx * p->ny;
  auto cp = [&](void* dst, const void* src, size_t by) -> sim_status {
    if (by) HIPCHK(hipMemcpyAsync(dst, src, by, hipMemcpyDeviceToDevice, e.stream));
    return SIM_OK;
  };
  if (N) {
    if ((st = cp(s.fil_offset, init->fil_offset, (F + 1) * 4))) return st;
    if ((st = cp(s.cell, init->cell, 2 * N * 4))) return st;
    if ((st = cp(s.frac, init->frac, 2 * N * 4))) return st;
    if ((st = cp(s.rest_angle, init->rest_angle, N * 4))) return st;
    if ((st = cp(s.rest_length, init->rest_length, N * 4))) return st;
    if ((st = cp(s.amp, init->act_amp, F * 4))) return st;
    if ((st = cp(s.period, init->act_period, F * 4))) return st;
    if ((st = cp(s.phase, init->act_phase, F * 4))) return st;
  }
  // optional arrays: copied when given, else the slot uses the parameters
  auto opt = [&](auto*& dst, const void* src, size_t by) -> sim_status {
    if (!src || !by) {
      dst = nullptr;
      return SIM_OK;
    }
    return cp(dst, src, by);
  };
  if ((st = opt(s.kb, init->k_bend, N * 4))) return st;
  if ((st = opt(s.ks, init->k_stretch, N * 4))) return st;
  if ((st = opt(s.ksh, init->k_shear, N * 4))) return st;
  if ((st = opt(s.fil_flags, init->fil_flags, F * 4))) return st;
  if ((st = opt(s.fil_parent, any_branch ? init->fil_parent : nullptr, F * 4))) return st;
  if ((st = opt(s.fil_attach, any_branch ? init->fil_attach : nullptr, 3 * F * 4))) return st;
  s.any_branch = any_branch;
  s.unit_next = unit_next;
  if (s.energy) {
    if (init->energy) {
      if ((st = cp(s.energy, init->energy, ncell * 4))) return st;
    } else {
      hipLaunchKernelGGL(k_zero_i32, dim3(256), dim3(256), 0, e.stream, (int*)s.energy, ncell);
    }
    hipLaunchKernelGGL(k_zero_i32, dim3(64), dim3(256), 0, e.stream, (int*)s.e_collected, std::max<size_t>(F, 1));
    hipLaunchKernelGGL(k_zero_i32, dim3(64), dim3(256), 0, e.stream, (int*)s.b.e_node, std::max<size_t>(N, 1));
  }
  if ((st = cp(s.fbuf[0], init->f, 9 * ncell * 4))) return st;
  if (s.b.cnt) hipLaunchKernelGGL(k_zero_i32, dim3(256), dim3(256), 0, e.stream, s.b.cnt, ncell);
  if (s.b.s) hipLaunchKernelGGL(k_zero_i32, dim3(256), dim3(256), 0, e.stream, (int*)s.b.s, ncell);
  if (s.b.Fg) hipLaunchKernelGGL(k_zero_i32, dim3(256), dim3(256), 0, e.stream, (int*)s.b.Fg, 2 * ncell);
  if (s.b.bin_cnt) {
    const size_t nt = n_bins(*p);
    hipLaunchKernelGGL(k_zero_i32, dim3(64), dim3(256), 0, e.stream, s.b.bin_cnt, nt);
    hipLaunchKernelGGL(k_zero_i32, dim3(64), dim3(256), 0, e.stream, s.b.bin_fill, nt);
    mc::launch_tile_ranges(p->nx, p->ny, p->repulse_radius, tile_side(*p), s.b.tile_rng, e.stream);
    hipLaunchKernelGGL(k_zero_i32, dim3(64), dim3(256), 0, e.stream, s.b.sp_cnt, (size_t)tiles_x(*p) * tiles_y(*p));
  }
  hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, e.stream, (int*)(e.flags + w), (size_t)1);
  HIPCHK(hipGetLastError());
  s.cur = 0;
  s.remaining = steps;
  e.slots[w] = s;
  if ((st = e.set_ctl(w, t0, steps))) return st;
  if ((st = e.rebuild())) {
    e.slots[w] = Slot();
    pool_free(b, off, bytes);
    return st;
  }
  *slot = w;
  return SIM_OK;
}

sim_status sim_batch_advance(sim_batch* b, int32_t n_steps) {
  if (!b) return fail(SIM_E_INVALID, "batch is NULL");
  if (n_steps < 0 || (n_steps & 1)) return fail(SIM_E_INVALID, "n_steps must be even and >= 0");
  Engine& e = b->eng;
  sim_status st = e.run_steps(n_steps);
  if (st) return st;
  for (auto& s : e.slots) {
    if (!s.used) continue;
    const int ran = std::min(s.remaining, n_steps);
    s.cur ^= (ran & 1);
    s.remaining -= ran;
  }
  return SIM_OK;
}

sim_status sim_batch_remaining(const sim_batch* b, int32_t slot, int32_t* remaining) {
  if (!b || !remaining) return fail(SIM_E_INVALID, "NULL argument");
  if (slot < 0 || slot >= b->eng.max_worlds || !b->eng.slots[slot].used) return fail(SIM_E_INVALID, "bad slot");
  *remaining = b->eng.slots[slot].remaining;
  return SIM_OK;
}

sim_status sim_batch_retire(sim_batch* b, int32_t slot, const sim_arrays* out) {
  if (!b) return fail(SIM_E_INVALID, "batch is NULL");
  Engine& e = b->eng;
  if (slot < 0 || slot >= e.max_worlds || !e.slots[slot].used) return fail(SIM_E_INVALID, "bad slot");
  Slot& s = e.slots[slot];
  const size_t N = s.n_part, ncell = (size_t)s.p.nx * s.p.ny;
  if (out) {
    if (out->n_particles != s.n_part) return fail(SIM_E_INVALID, "output arrays have the wrong size");
    if (N) {
      HIPCHK(hipMemcpyAsync(out->cell, s.cell, 2 * N * 4, hipMemcpyDeviceToDevice, e.stream));
      HIPCHK(hipMemcpyAsync(out->frac, s.frac, 2 * N * 4, hipMemcpyDeviceToDevice, e.stream));
    }
    if (out->f) HIPCHK(hipMemcpyAsync(out->f, s.fbuf[s.cur], 9 * ncell * 4, hipMemcpyDeviceToDevice, e.stream));
    if (out->u) HIPCHK(hipMemcpyAsync(out->u, s.u, 2 * ncell * 4, hipMemcpyDeviceToDevice, e.stream));
    if (s.energy && out->energy)
      HIPCHK(hipMemcpyAsync(out->energy, s.energy, ncell * 4, hipMemcpyDeviceToDevice, e.stream));
    if (s.energy && out->energy_collected && s.n_fil)
      HIPCHK(hipMemcpyAsync(out->energy_collected, s.e_collected, (size_t)s.n_fil * 4, hipMemcpyDeviceToDevice,
                            e.stream));
  }
  unsigned* hflag = (unsigned*)e.pinned;   // staging is idle after the event sync below
  HIPCHK(hipEventSynchronize(e.upload_done));
  HIPCHK(hipMemcpyAsync(hflag, e.flags + slot, sizeof(unsigned), hipMemcpyDeviceToHost, e.stream));
  HIPCHK(hipStreamSynchronize(e.stream));
  const unsigned fl = *hflag;
  pool_free(b, s.pool_off, s.pool_len);
  s = Slot();
  sim_status st = e.rebuild();
  if (st) return st;
  if (fl & mc::kFlagBins) return fail(SIM_E_STATE, "world in slot %d: tile bins out of date", slot);
  if (fl) return fail(SIM_E_UNSTABLE, "world in slot %d produced NaN or |u| > u_max", slot);
  return SIM_OK;
}

sim_status sim_batch_sync(sim_batch* b) {
  if (!b) return fail(SIM_E_INVALID, "batch is NULL");
  HIPCHK(hipStreamSynchronize(b->eng.stream));
  HIPCHK(hipGetLastError());
  return SIM_OK;
}

void sim_batch_destroy(sim_batch* b) { delete b; }

}  // extern "C"
