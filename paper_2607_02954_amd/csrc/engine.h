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

constexpr int kCellsPerItem = 256;   // cells per fluid work item (one block)
constexpr int kTileX = 64;           // filter output tile (x)
constexpr int kTileY = 16;           // filter output tile (y)
constexpr int kMaxRadius = 8;        // largest Gaussian truncation radius
constexpr int kMaxFilament = 1024;   // longest filament a node pack can hold

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
  int pbd_iters, radius, sorted, pad0;
  float gtap[kMaxRadius + 1];           // normalised Gaussian taps g[0..R]
  const int* fil_offset;                // [F+1]
  const int* cell_in;  const float* frac_in;     // positions at the start of the step
  int* cell_out;       float* frac_out;          // positions after the step (may alias)
  const float* rest_angle; const float* rest_length;
  const float* act_amp; const float* act_period; const float* act_phase;
  const float* f_src;  float* f_dst;    // shifted populations f - w, [9][ny][nx]
  float* u;                             // [2][ny][nx]
  float* s;                             // deposit accumulator [ny][nx]
  float* st;                            // filtered density [ny][nx]
  float* Fg;                            // grid force accumulator [2][ny][nx]
  float* fel;                           // node force [2][N] (elastic, then total)
  const Ctl* ctl_src; Ctl* ctl_dst;
  unsigned* flags;                      // sticky: bit 0 = NaN or |u| > u_max
  // deterministic sorted-segment transfer (SIM_SPLAT_SORTED)
  int* key;                             // [N] home cell of each node
  int* rank;                            // [N] arrival rank within its home cell
  int* cnt;                             // [ny*nx] nodes per home cell (zeroed after use)
  int* start;                           // [ny*nx + 1] exclusive prefix of cnt
  int* perm;                            // [N] node index of each sorted slot
  float4* rec;                          // [N] sorted records (frac x, frac y, Fx, Fy)
  int* part;                            // scan partials
};

// A node pack: whole filaments with at most `pack` nodes, run by one block.
struct Pack {
  int world, node_begin, node_end, fil_begin;
  int fil_end, pad0, pad1, pad2;
};

struct Tables {
  const Pack* packs;  const int* n_packs;
  const int2* items;  const int* n_items;    // (world, first cell) of 256 cells
  const int2* tiles;  const int* n_tiles;    // (world, tile index) for the filter
  const int2* scan;   const int* n_scan;     // (world, block) for the cell scan
};

struct Grid {
  int node_blocks, cell_blocks, tile_blocks, scan_blocks;
  int pack;                                  // node pack capacity: 256 or 1024
};

// Forward step launchers (kernels.hip).  `W` points at a device array of
// world descriptors.
void launch_elastic(const WorldDev* W, const Tables& T, const Grid& G, hipStream_t s);
void launch_sort(const WorldDev* W, const Tables& T, const Grid& G, hipStream_t s, bool any_sorted);
void launch_filter(const WorldDev* W, const Tables& T, const Grid& G, hipStream_t s);
void launch_repulse(const WorldDev* W, const Tables& T, const Grid& G, hipStream_t s);
void launch_lbm(const WorldDev* W, const Tables& T, const Grid& G, hipStream_t s);
void launch_integrate(const WorldDev* W, const Tables& T, const Grid& G, hipStream_t s);
void launch_set_ctl(Ctl* c, long long t, int remaining, hipStream_t s);

}  // namespace mc
