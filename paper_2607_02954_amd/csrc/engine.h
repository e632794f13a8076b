// Internal device-side data structures of libmicrocosm (not part of the ABI).
//
// Every kernel runs over a table of world descriptors plus work lists, so one
// launch advances any number of independent worlds of uneven size; a single
// world is simply a table of one.  Kernels grid-stride over their work list
// and read the list length from device memory, so a captured graph stays
// valid while the host rewrites the tables between launches.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mc {

// Pointers read from the world table carry no address space, so the compiler
// would access them with flat instructions, whose completion counter is
// shared with LDS operations.  Kernels cast them to the global address space
// once per work item.
#define MC_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ MC_GLOBAL T* glb(T* p) {
  return (MC_GLOBAL T*)p;
}
// Vector element types for global-address-space access (HIP's float2/int4
// classes cannot be copied through address-space-qualified references).
typedef float vf2 __attribute__((ext_vector_type(2)));
typedef float vf4 __attribute__((ext_vector_type(4)));
typedef int vi2 __attribute__((ext_vector_type(2)));
typedef int vi4 __attribute__((ext_vector_type(4)));
template <class V, class T>
__device__ __forceinline__ MC_GLOBAL V* glbv(T* p) {
  return (MC_GLOBAL V*)p;
}

// Square grid tiles of the tile kernels (filter, spread, integrate; node bins
// of the binned transfer): side 16, 32 or 64 cells, chosen per world.  Each
// side is a family of kernel instances; a table of worlds launches the
// families it holds.
constexpr int kTileFamilies = 3;
__host__ __device__ constexpr int tile_side_of_family(int f) { return 16 << f; }
__host__ __device__ constexpr int tile_family_of_side(int side) { return side == 16 ? 0 : side == 64 ? 2 : 1; }
__host__ __device__ constexpr int tile_shift_of_side(int side) { return side == 16 ? 4 : side == 64 ? 6 : 5; }
// records a tile's spread list holds (else it reads the bins): one per cell
__host__ __device__ constexpr int spread_cap_of_side(int side) { return side * side; }
constexpr int kRunStride = 8;        // bin runs stored per tile and reader
constexpr int kCellsPerItem = 256;   // contiguous cells per fluid work item
constexpr int kMaxRadius = 8;        // largest Gaussian truncation radius

// Particle -> grid transfer modes (per world).
enum TransferMode : int {
  kBinned = 0,   // nodes binned by home tile; sums formed in LDS, tiles written whole
  kSorted = 1,   // counting sort by home cell; fixed-order segmented sums
  kDirect = 2    // global float atomics into HBM accumulators
};
constexpr int kMaxFilament = 1024;   // longest filament a node pack can hold

// Sticky per-world flag bits.
constexpr unsigned kFlagUnstable = 1u;   // NaN or |u| > u_max
constexpr unsigned kFlagBins = 2u;       // a node found its tile bin full (positions changed
                                         // without a bin pre-pass); the record was dropped

// Per-world control word, double-buffered by step parity: kernels of a step
// read ctl_src; the fluid kernel writes the next step's values to ctl_dst.
struct Ctl {
  long long t;       // time index of the step about to run
  int remaining;     // steps left; a world with remaining <= 0 idles
  int pad;
};

// Everything a kernel needs to know about one world.
struct WorldDev {
  int nx, ny, n_part, n_fil;
  float om_p, om_m;                     // TRT rates: 1/tau and 1/(Lambda/(tau-1/2) + 1/2)
  float k_bend, k_stretch, k_shear, k_el, k_rep, u_max2;
  int pbd_iters, radius, mode, ntx;     // ntx, nty: tiles per row / column
  int nty, tile_shift, pad1, pad2;      // tile side = 1 << tile_shift
  float gtap[kMaxRadius + 1];           // normalised Gaussian taps g[0..R]
  const int* fil_offset;                // [F+1]
  const int* cell_in;  const float* frac_in;     // positions at the start of the step
  int* cell_out;       float* frac_out;          // positions after the step (may alias)
  const float* rest_angle; const float* rest_length;
  const float* act_amp; const float* act_period; const float* act_phase;
  const float* kb_arr; const float* ks_arr; const float* ksh_arr;   // [N] per-edge stiffnesses, or null
  const int* fil_flags;                 // [F] bit 0: closed loop, or null (all chains)
  const int* fil_parent;                // [F] node filament f hangs from (-1: none), or null
  const float* fil_attach;              // [3][F] attachment rest length, rest angle at the
                                        // parent node, rest angle at the first node
  // energy field (null energy: none): sensed at the nodes, collected at
  // `energy_rate` per step and taken out of the field
  float energy_rate; int pad3;
  float* energy;                        // [ny][nx] persistent field
  float* e_node;                        // [N] sensed value
  float* e_sensed;                      // [N] caller copy of the sensed values, or null
  float* e_collected;                   // [F] accumulated collected energy, or null
  // coupling leakage fixes (direct transfer): two-layer markers and MDF
  int mdf_iters;                        // 1: explicit coupling
  float marker_offset;                  // 0: one layer
  float* d_marker;                      // [2][N] marker displacement offset * normal, or null
  float* U_d;                           // [2][N] MDF desired node velocity
  float* mdf_c;                         // [2][N] MDF correction per node (binned transfer)
  float4* rho_j;                        // [ny][nx] (rho, jx, jy, 0) of the step's populations
  float2* u_mdf;                        // [ny][nx] fluid velocity of the current MDF force
  const float* f_src;  float* f_dst;    // shifted populations f - w, [9][ny][nx]
  float2* u;                            // [ny][nx] fluid velocity (x, y interleaved)
  float* s;                             // deposit accumulator [ny][nx] (direct mode)
  float2* grad;                         // [ny][nx] central difference of the filtered density
  float2* Fg;                           // [ny][nx] grid force
  float* fel;                           // node force [2][N]: total (elastic + repulsion)
  float* fel_el;                        // node elastic force [2][N]
  const Ctl* ctl_src; Ctl* ctl_dst;
  unsigned* flags;                      // sticky: kFlagUnstable, kFlagBins
  // deterministic sorted-segment transfer (SIM_SPLAT_SORTED)
  int* key;                             // [N] home cell of each node
  int* rank;                            // [N] arrival rank within its home cell
  int* cnt;                             // [ny*nx] nodes per home cell (zeroed after use)
  int* start;                           // [ny*nx + 1] exclusive prefix of cnt
  int* perm;                            // [N] node index of each sorted slot
  float4* rec;                          // [N] sorted records (frac x, frac y, Fx, Fy)
  int* part;                            // scan partials
  // tile bins (binned mode): one record per node, grouped by home tile
  int* bin_cnt;                         // [ntx*nty] nodes per tile (zeroed after use)
  int* bin_fill;                        // [ntx*nty] fill cursors (zeroed after use)
  int* bin_start;                       // [ntx*nty + 1] exclusive prefix of bin_cnt
  int* bin_start_next;                  // where the scan after integrate puts the next step's
                                        // starts (bin_start itself, except on the adjoint tape)
  int4* bin_rec;                        // [N] record: (x | y << 16 home cell, frac x, frac y, node)
  int4* sp_rec;                         // [ntx*nty][side^2] the records each tile's spread reads,
  int* sp_cnt;                          // [ntx*nty] and their number: both written by the filter
  const int2* tile_rng;                 // [ntx*nty][2][kRunStride] bin runs (first, end) that the
                                        // filter (0) and the spread (1) of each tile read; unused
                                        // runs (0, 0)
};

// A node pack: whole filaments with at most `pack` nodes, run by one block.
struct Pack {
  int world, node_begin, node_end, fil_begin;
  int fil_end, pad0, pad1, pad2;
};

struct Tables {
  const Pack* packs;  const int* n_packs;
  // per tile family: (world, tx | ty << 16) of every tile of the worlds with that tile side
  const int2* tiles[kTileFamilies];  const int* n_tiles[kTileFamilies];
  const int2* items;  const int* n_items;    // (world, first cell) of 256 contiguous cells
  const int2* scan;   const int* n_scan;     // (world, block) for the cell scan (sorted mode)
  const int2* worlds; const int* n_worlds;   // (world, 0) for per-world kernels
  int single_ntx[kTileFamilies];             // > 0: the family holds one world whose tiles are
                                             // its row-major tiles, ntx per row (no table read)
};

struct Grid {
  int node_blocks, scan_blocks, world_blocks, item_blocks;
  int tile_blocks[kTileFamilies];            // 0: no world of that tile side (family not launched)
  int pack;                                  // node pack capacity: 256 or 1024
  int any_sorted, any_binned, any_node;      // which transfer families the table holds
                                             // (any_node: a world not in binned mode)
  int max_radius;                            // largest Gaussian radius of any world (LDS sizing)
  int any_energy;                            // a world has an energy field
  int any_markers;                           // a world broadcasts two-layer markers
  int mk_only;                               // every world of the tile kernels has markers (the
                                             // one-layer tile variants are not launched)
  int mdf_max;                               // most MDF iterations of any world (1: none)
  int general;                               // a world passes loop flags or per-edge stiffnesses
  int branches;                              // a world has branches (filaments hanging from nodes)
  int pbd_max;                               // most PBD iterations of any world (set by the
                                             // reverse mode: sizes its register states)
};

// Reverse-mode buffers of one step (adjoint.hip).  "_in" holds dL/d(state at
// t+1); the kernels produce dL/d(state at t).  The step's time index is the
// one its descriptor's control word holds after the recomputed forward.
struct AdjDev {
  const float* xbar_in;   // [2][N]
  float* xbar;            // [2][N]
  const float* gbar_in;   // [9][ny][nx]
  float* gbar;            // [9][ny][nx]
  float2* ubar;           // [ny][nx]
  float2* Fgbar;          // [ny][nx]
  float2* Gbar;           // [ny][nx]
  float* sbar;            // [ny][nx]
  float* Fbar;            // [2][N]
  float* g_rest;          // [N] accumulated dL/d(rest angle)
  // multi-direct forcing (binned worlds with mdf_iters > 1)
  int mdf;                // the world's MDF iterations K (1: none; the rest unused)
  const float* F;         // [2][N] the step's total node forces (tape)
  float2* Fgk;            // [K-1][ny][nx] the iterates F_grid_1 .. F_grid_{K-1}, recomputed
  float* Ud;              // [2][N] desired node velocity, recomputed
  float* mc;              // [2][N] the correction of an iterate, recomputed
  float* Ukbar;           // [2][N] dL/d(velocity sampled at the nodes) of one iteration
  float* Udbar;           // [2][N] dL/dU_d
  float* xbar_m;          // [2][N] the MDF transfers' terms of dL/dx_t
  float2* jbar;           // [ny][nx] dL/dj through MDF
  float* rhobar;          // [ny][nx] dL/drho through MDF
  // two-layer markers (worlds with marker displacements d; X = x +- d)
  float* dbar;            // [2][N] dL/dd of the step, from the node kernels
  float* dbar_m;          // [2][N] dL/dd through the MDF transfers (MDF worlds)
  const float* dbg_v;     // test hook: the node vector a single spread reads
  float2* dbg_out;        // and the grid it writes
};
// The adjoint buffers of the worlds of a launch: one set (arr null: a single
// world) or an array indexed by the world of each work item (a set of worlds).
struct AdjArg {
  const AdjDev* arr;
  AdjDev one;
};
void launch_mdf_moments(const WorldDev* W, const Tables& T, const Grid& G, hipStream_t s);

void launch_adjoint_step(const WorldDev* W, const Tables& T, const Grid& G, const AdjArg& A, int mdf, hipStream_t s);
void launch_adjoint_debug(const WorldDev* W, const Tables& T, const Grid& G, int which, const AdjDev& A,
                          const float* v, float2* out, hipStream_t s);

// Forward step launchers (kernels.hip).  `W` points at a device array of
// world descriptors.
void launch_elastic(const WorldDev* W, const Tables& T, const Grid& G, hipStream_t s);
void launch_bin_prepass(const WorldDev* W, const Tables& T, const Grid& G, hipStream_t s);
void launch_sort(const WorldDev* W, const Tables& T, const Grid& G, hipStream_t s);
void launch_filter(const WorldDev* W, const Tables& T, const Grid& G, hipStream_t s);
void launch_repulse(const WorldDev* W, const Tables& T, const Grid& G, hipStream_t s);
void launch_spread(const WorldDev* W, const Tables& T, const Grid& G, hipStream_t s);
void launch_lbm(const WorldDev* W, const Tables& T, const Grid& G, hipStream_t s);
// the same launch with the dispatch's own start and end timestamps in two events
void launch_lbm_timed(const WorldDev* W, const Tables& T, const Grid& G, hipStream_t s, hipEvent_t start,
                      hipEvent_t stop);
void launch_integrate(const WorldDev* W, const Tables& T, const Grid& G, hipStream_t s);
// two-layer markers (before the force spread) and MDF corrections of the grid
// force (after it, before the fluid update); direct-transfer worlds
void launch_markers(const WorldDev* W, const Tables& T, const Grid& G, hipStream_t s);
void launch_mdf(const WorldDev* W, const Tables& T, const Grid& G, hipStream_t s);
// energy field: sensing and collection at the step's starting positions
// (between the fluid update and the integration)
void launch_energy(const WorldDev* W, const Tables& T, const Grid& G, hipStream_t s);
// add Gaussian packets to a field
void launch_energy_packets(int nx, int ny, int n_packets, const float* centres, const float* amps,
                           const float* widths, float* field, hipStream_t s);
// set-up: the bin runs of every tile (side `tile`) of an nx x ny world of Gaussian radius R
void launch_tile_ranges(int nx, int ny, int R, int tile, int2* out, hipStream_t s);
void launch_set_ctl(Ctl* c, long long t, int remaining, hipStream_t s);

// Folding objective (loss.hip): Gaussian-splatted node density on a W x H
// image over the nx x ny world, its mean squared error to `target` (written
// to *loss), the image (if `image`) and dL/dx of every node (if `g_pos`).
size_t density_loss_workspace(int W, int H);
void launch_density_loss(int nx, int ny, int n, int W, int H, float sigma, float amp, const int* cell,
                         const float* frac, const float* target, float* image, float* loss, float* g_pos,
                         void* ws, hipStream_t s);

// Bending and stretching effort of a change of the rest values, per filament
// (accumulated into effort[2][F]).
void launch_rest_effort(int n_fil, const int* fil_offset, const int* fil_flags, const float* old_a,
                        const float* new_a, const float* old_l, const float* new_l, float* effort, hipStream_t s);

// Record msg as the thread's last error message (sim_last_error) and return st.
int report_error(int st, const char* msg);

}  // namespace mc
