// Device helpers shared by the forward and adjoint kernels.
#pragma once

#include <math.h>

#include <type_traits>

#include "engine.h"

namespace mc {

constexpr float kPi = 3.14159265358979323846f;
constexpr float kTwoPi = 6.28318530717958647692f;

// i mod n in [0, n) for any i; integer division only outside [-n, 2n).
static __device__ __forceinline__ int wrap_index(int i, int n) {
  if (i >= 0 && i < n) return i;
  if (i >= n && i < 2 * n) return i - n;
  if (i < 0 && i >= -n) return i + n;
  const int r = i % n;
  return r < 0 ? r + n : r;
}

// Compile-time shape of the tile kernels for tiles of side TILE.
constexpr int kWaveList = 64;              // records per wavefront list (for_bin_records)
template <int TILE>
struct TileCfg {
  static constexpr int kTile = TILE;
  static constexpr int kShift = tile_shift_of_side(TILE);
  static constexpr int kFamily = tile_family_of_side(TILE);
  static constexpr int kThreads = TILE == 64 ? 1024 : 256;   // threads per tile block
  // bin columns (and rows) a reader's home range can touch, and bin runs
  // it reads: the filter's range is the tile plus R + 3 <= 11 < TILE cells
  // on each side, so it touches the tile and one neighbour per side, and
  // one tile more where that neighbour is the partial last tile of an axis
  // (shorter than the margin) on one side: at most 4; a row of bins needs at
  // most two runs (its cyclic column list is broken once at most)
  static constexpr int kMaxCols = 4;
  static constexpr int kRanges = 2 * kMaxCols;
  static constexpr int kSpreadSide = TILE + 6;              // spread window side
  static constexpr int kSpreadCells = kSpreadSide * kSpreadSide;
  static constexpr int kSpreadCap = spread_cap_of_side(TILE);
  static constexpr int kListBytes = (kThreads / 64) * kWaveList * 16;
  static_assert(kRanges <= kRunStride, "run table too narrow");
};

// Tile table entry it of a tile family: (world, tx | ty << 16); computed
// rather than read when the family holds a single world.
template <int TILE>
static __device__ __forceinline__ int2 tile_entry(const Tables& T, int it) {
  constexpr int f = TileCfg<TILE>::kFamily;
  if (T.single_ntx[f] > 0) {
    const int ty = it / T.single_ntx[f];
    return make_int2(0, (it - ty * T.single_ntx[f]) | (ty << 16));
  }
  return T.tiles[f][it];
}
template <int TILE>
static __device__ __forceinline__ int n_tiles(const Tables& T) {
  return *T.n_tiles[TileCfg<TILE>::kFamily];
}

// Tile table entries hold (world, tx | ty << 16).
static __device__ __forceinline__ int tile_x(int packed) { return packed & 0xffff; }
static __device__ __forceinline__ int tile_y(int packed) { return packed >> 16; }

static __device__ __forceinline__ int wrap_near(int v, int n) {   // v in [-n, 2n)
  return v < 0 ? v + n : (v >= n ? v - n : v);
}

// Map an angle difference into (-pi, pi] (the quotient by 2 pi is formed
// with its reciprocal; that can only matter at the boundary itself).
static __device__ __forceinline__ float wrap_angle(float d) {
  return d - kTwoPi * ceilf((d - kPi) * (1.0f / kTwoPi));
}

// Hardware square root and reciprocal (within 1 ulp; the edge lengths they
// see are near 1, far from denormals).
static __device__ __forceinline__ float hw_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
static __device__ __forceinline__ float hw_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// The four 1D weights of Peskin's 4-point function for offsets
// (-1 - f, -f, 1 - f, 2 - f), f in [0, 1): with q = sqrt(1 + 4f - 4f^2) they
// are (3 - 2f - q)/8, (3 - 2f + q)/8, (1 + 2f + q)/8, (1 + 2f - q)/8.
// The square root's argument lies in [1, 2], where the hardware square root
// (within 1 ulp) needs none of the scaling of the library's sqrtf.
static __device__ __forceinline__ float peskin_q(float f) {
  return __builtin_amdgcn_sqrtf(fmaf(4.0f * f, 1.0f - f, 1.0f));
}
static __device__ __forceinline__ void peskin4(float f, float w[4]) {
  const float q = peskin_q(f);
  const float a = 3.0f - 2.0f * f;
  const float b = 1.0f + 2.0f * f;
  w[0] = 0.125f * (a - q);
  w[1] = 0.125f * (a + q);
  w[2] = 0.125f * (b + q);
  w[3] = 0.125f * (b - q);
}

// Derivatives of the four weights above with respect to f:
// with q' = (2 - 4f)/q they are (-2 - q')/8, (-2 + q')/8, (2 + q')/8, (2 - q')/8.
static __device__ __forceinline__ void peskin4_d(float f, float w[4], float dw[4]) {
  const float q = peskin_q(f);
  const float a = 3.0f - 2.0f * f;
  const float b = 1.0f + 2.0f * f;
  w[0] = 0.125f * (a - q);
  w[1] = 0.125f * (a + q);
  w[2] = 0.125f * (b + q);
  w[3] = 0.125f * (b - q);
  const float qd = (2.0f - 4.0f * f) / q;
  dw[0] = 0.125f * (-2.0f - qd);
  dw[1] = 0.125f * (-2.0f + qd);
  dw[2] = 0.125f * (2.0f + qd);
  dw[3] = 0.125f * (2.0f - qd);
}

// Actuated rest angle of joint j (of m: n - 2 on a chain, n on a loop) of a
// filament at time step t: ra + amp sin(2 pi t / period + phase - 2 pi j / m).
// The phase is formed in revolutions and reduced to [-1/2, 1/2] (the integer
// part of t / period is removed in FP64), so FP32 sinf sees a small argument.
static __device__ __forceinline__ float actuated_angle(float ra, float amp, float period, float phase, long long t,
                                                       int j, int m) {
  if (amp == 0.0f) return ra;
  float frac_t;                                 // (t / period) mod 1
  if (t < (1ll << 24)) {
    // t is exact in FP32; t - k period is formed with one rounding (fma), so
    // the remainder keeps FP32 accuracy whatever the size of t / period
    const float tf = (float)t;
    const float k = floorf(tf * hw_rcp(period));
    float rem = fmaf(-k, period, tf);
    if (rem < 0.0f) rem += period;
    if (rem >= period) rem -= period;
    frac_t = rem * hw_rcp(period);
  } else {
    const double q = (double)t / (double)period;
    frac_t = (float)(q - floor(q));
  }
  float r = frac_t + phase * (1.0f / kTwoPi) - (float)j / (float)m;
  r -= rintf(r);
  return ra + amp * sinf(kTwoPi * r);
}

// (cos t, sin t) of an edge angle t that started the step at t0, whose unit
// vector (c0, s0) is known: the rotation of (c0, s0) by d = t - t0, with
// cos d and sin d from their Taylor series (to d^8 and d^9; truncation below
// 3e-8 for |d| <= pi/4).  Larger turns take sincosf.
static __device__ __forceinline__ void edge_direction(float t, float t0, float c0, float s0, float* c, float* s) {
  const float d = t - t0;
  if (fabsf(d) <= 0.25f * kPi) {
    const float d2 = d * d;
    const float cd = fmaf(d2, fmaf(d2, fmaf(d2, fmaf(d2, 1.0f / 40320.0f, -1.0f / 720.0f), 1.0f / 24.0f), -0.5f), 1.0f);
    const float sd = d * fmaf(d2, fmaf(d2, fmaf(d2, fmaf(d2, 1.0f / 362880.0f, -1.0f / 5040.0f), 1.0f / 120.0f),
                                       -1.0f / 6.0f), 1.0f);
    *c = c0 * cd - s0 * sd;
    *s = s0 * cd + c0 * sd;
  } else {
    sincosf(t, s, c);
  }
}

// A marker displaced by d (|d| <= 1 cell) along one axis from a node with
// fraction f: the shift of its home cell from the node's (-1, 0 or 1) and
// its own fraction.  The shift stays in [-1, 1] also where |d| exceeds one
// cell by a rounding step: f + d rounded up to 2 is the same point as shift
// 1 with fraction 1 (the 4-point weights of fraction 1 put nothing on the
// first cell); f + d below -1 (by rounding only) moves to shift -1,
// fraction 0, at most one rounding step away.
static __device__ __forceinline__ void marker_shift(float f, float d, int* shift, float* fr) {
  const float m = f + d;
  const float fl = floorf(m);
  int h = (int)fl;
  float r = m - fl;
  if (r >= 1.0f) {
    r = 0.0f;
    h += 1;
  }
  if (h > 1) {
    h = 1;
    r = 1.0f;
  } else if (h < -1) {
    h = -1;
    r = 0.0f;
  }
  *shift = h;
  *fr = r;
}

// The same marker's wrapped home cell on an axis of n cells, for a node at cell c.
static __device__ __forceinline__ void marker_home(int c, float f, float d, int n, int* home, float* fr) {
  int sh;
  marker_shift(f, d, &sh, fr);
  *home = wrap_index(c + sh, n);
}

// Global float atomics of s * W(c - X) * (vx, vy) into an interleaved
// float2 field, for a point X with wrapped home cell (bx, by) and fraction (fx, fy).
static __device__ __forceinline__ void atomic_spread_vec(MC_GLOBAL float* field, int nx, int ny, int bx, int by,
                                                         float fx, float fy, float vx, float vy) {
  float wx[4], wy[4];
  peskin4(fx, wx);
  peskin4(fy, wy);
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    MC_GLOBAL float* row = field + 2 * (size_t)wrap_near(by - 1 + b, ny) * nx;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int x = wrap_near(bx - 1 + a, nx);
      const float ww = wx[a] * wy[b];
      unsafeAtomicAdd((float*)(row + 2 * x), ww * vx);
      unsafeAtomicAdd((float*)(row + 2 * x + 1), ww * vy);
    }
  }
}

// sum_c W(c - X) v_c of an interleaved float2 field at a point X.
static __device__ __forceinline__ vf2 gather_vec(const MC_GLOBAL vf2* field, int nx, int ny, int bx, int by, float fx,
                                                 float fy) {
  float wx[4], wy[4];
  peskin4(fx, wx);
  peskin4(fy, wy);
  float gx = 0.f, gy = 0.f;
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const MC_GLOBAL vf2* row = field + (size_t)wrap_near(by - 1 + b, ny) * nx;
    float ax = 0.f, ay = 0.f;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const vf2 v = row[wrap_near(bx - 1 + a, nx)];
      ax += wx[a] * v.x;
      ay += wx[a] * v.y;
    }
    gx += wy[b] * ax;
    gy += wy[b] * ay;
  }
  const vf2 out = {gx, gy};
  return out;
}

// D2Q9 lattice: velocity q has components (CX[q], CY[q]); q and q+2 are
// opposite for q = 1, 2, 5, 6.
static __constant__ int kCX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static __constant__ int kCY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

// Bin (home tile) of a wrapped home cell (bx, by) of a world with ntx tiles
// per row of side 1 << shift, and the bin at tile column sx, row sy.
static __device__ __forceinline__ int bin_of(int bx, int by, int ntx, int shift) {
  return (by >> shift) * ntx + (bx >> shift);
}
static __device__ __forceinline__ int bin_at(int sx, int sy, int ntx) { return sy * ntx + sx; }

// Distinct tile columns holding the cells lo..hi of a periodic axis of n
// cells (at most TileCfg<TILE>::kMaxCols for the ranges the readers use).
template <int TILE>
static __device__ __forceinline__ int bins_covering(int lo, int hi, int n, int* t) {
  constexpr int kMax = TileCfg<TILE>::kMaxCols;
  int cnt = 0;
  if (hi - lo + 1 >= n) {                       // whole axis (a short one)
    for (int k = 0; k * TILE < n && cnt < kMax; ++k) t[cnt++] = k;
    return cnt;
  }
  int c = lo;
  while (c <= hi && cnt < kMax) {
    const int cc = wrap_index(c, n);
    const int tt = cc / TILE;
    bool seen = false;
    for (int k = 0; k < cnt; ++k) seen |= (t[k] == tt);
    if (!seen) t[cnt++] = tt;
    c += min((tt + 1) * TILE, n) - cc;          // jump to the next tile boundary
  }
  return cnt;
}

// 64-bit fixed-point accumulation in LDS (2^-36 resolution, range +-2^27).
constexpr float kFixScale = 68719476736.0f;           // 2^36
constexpr float kFixInv = 1.4551915228366852e-11f;    // 2^-36
// Nearest 64-bit integer to a float x with |x| < 2^62, from 32-bit
// conversions: |x| = hi 2^32 + lo, where hi = floor(|x| / 2^32) and
// lo = |x| - hi 2^32 in [0, 2^32) are both exact in FP32 (|x| has 24
// significant bits, and so do its bits below 2^32), and lo only has a
// fraction when it is below 2^24.
static __device__ __forceinline__ long long f32_to_fix(float x) {
  const float ax = fabsf(x);
  const float hf = floorf(ax * 2.3283064365386963e-10f);
  const float lof = fmaf(hf, -4294967296.0f, ax);
  const long long m = (long long)(((unsigned long long)(unsigned)hf << 32) + (unsigned long long)__float2uint_rn(lof));
  return x < 0.0f ? -m : m;
}
static __device__ __forceinline__ float fix_to_float(long long v) {
  const int hi = (int)(v >> 32);
  const unsigned lo = (unsigned)v;
  return (float)((double)hi * 4294967296.0 + (double)lo) * kFixInv;
}

// Density deposits use the 1D weights rounded to multiples of 2^-23 (each
// weight is at most 1/2, so it is an integer below 2^23): a 2D weight is then
// the exact product of two such integers, a multiple of 2^-46 formed by two
// 24-bit multiplies, and sums of them are exact in 64 bits.
constexpr float kWeightQ = 8388608.0f;                   // 2^23
static __device__ __forceinline__ void peskin4_quant(float f, unsigned q[4]) {
  float w[4];
  peskin4(f, w);
#pragma unroll
  for (int a = 0; a < 4; ++a) q[a] = __float2uint_rn(w[a] * kWeightQ) & 0xffffffu;
}
static __device__ __forceinline__ unsigned long long weight_product(unsigned a, unsigned b) {
  return (unsigned long long)(a & 0xffffffu) * (b & 0xffffffu);   // v_mul_u32_u24 + v_mul_hi_u32_u24
}
// The high word converts exactly (densities stay far below 2^14), the low
// word with one FP32 rounding (an absolute error below 2^-38), then one fma.
static __device__ __forceinline__ float density_to_float(unsigned long long v) {
  return fmaf((float)(unsigned)(v >> 32), 6.103515625e-05f, (float)(unsigned)v * 1.4210854715202004e-14f);
}

// Work-item order of the tile kernels.  The hardware hands workgroups to the
// eight XCDs in turn (block b to XCD b mod 8) and each XCD has its own L2, so
// a plain grid-stride loop puts neighbouring tiles, which read each other's
// halos and bins, on different XCDs.  Here the blocks of each XCD take one
// contiguous share of the item list instead.
struct XcdLoop {
  int first, end, step;
  __device__ __forceinline__ explicit XcdLoop(int n) {
    const int G = gridDim.x, b = blockIdx.x;
    if (G < 8) {
      first = b;
      end = n;
      step = G;
      return;
    }
    const int x = b & 7, per = (n + 7) >> 3;
    first = x * per + (b >> 3);
    end = min(n, x * per + per);
    step = (G - x + 7) >> 3;                   // blocks on this XCD
  }
};

// Clear n 64-bit words of LDS at a 16-byte aligned address, 16 bytes per
// store (block-wide; the caller synchronises before use).
static __device__ __forceinline__ void zero_lds_u64(void* p, int n) {
  vi4* q = (vi4*)p;
  const vi4 z = {0, 0, 0, 0};
  for (int k = threadIdx.x; k < (n >> 1); k += blockDim.x) q[k] = z;
  if ((n & 1) && threadIdx.x == 0) ((long long*)p)[n - 1] = 0;
}

// Wavefront-aggregated atomic increment: lanes that target the same counter
// are served by one atomic from a leader lane.  Returns, for lanes with `has`,
// a distinct slot (the counter's old value plus the lane's rank among the
// matching lanes).  Must be called by every lane of the wavefront.
static __device__ __forceinline__ int agg_atomic_inc(MC_GLOBAL int* counters, int key, bool has) {
  const int lane = __lane_id();
  unsigned long long pending = __ballot(has);
  int slot = 0;
  while (pending) {
    const int leader = __ffsll((unsigned long long)pending) - 1;
    const int lkey = __shfl(key, leader);
    const unsigned long long match = __ballot(has && key == lkey) & pending;
    int base = 0;
    if (lane == leader) base = atomicAdd((int*)(counters + lkey), __popcll(match));
    base = __shfl(base, leader);
    if ((match >> lane) & 1ull) slot = base + __popcll(match & ((1ull << lane) - 1ull));
    pending &= ~match;
  }
  return slot;
}

// Block-wide exclusive scan of one int per thread (NT threads), wave
// shuffles plus one LDS exchange (s_wave holds NT/64 ints).  Returns the
// exclusive prefix; *total gets the block sum.  All threads must call it.
template <int NT>
static __device__ __forceinline__ int block_scan(int v, int* s_wave, int* total) {
  const int lane = __lane_id();
  const int wid = threadIdx.x >> 6;
  int x = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int n = __shfl_up(x, off);
    if (lane >= off) x += n;
  }
  if (lane == 63) s_wave[wid] = x;
  __syncthreads();
  int before = 0, all = 0;
#pragma unroll
  for (int k = 0; k < NT / 64; ++k) {
    const int sw = s_wave[k];
    before += (k < wid) ? sw : 0;
    all += sw;
  }
  __syncthreads();
  *total = all;
  return before + x - v;
}
static __device__ __forceinline__ int block_scan256(int v, int* s_wave, int* total) {
  return block_scan<256>(v, s_wave, total);
}


// Records of a set of home-tile bins.  Every wavefront streams its share of
// the records (PER loads in flight per lane) and appends those for which
// keep(r) holds to its own LDS list (one ballot per record batch); whenever
// the list reaches a full wavefront of records the wavefront runs body(r) on
// them and starts the list again with the batch's overflow.  No block barrier
// is needed until all records are done, body always runs on full wavefronts
// (except for the last partial one), and lanes holding irrelevant records
// never idle through it.  body(r) may only use per-lane work and LDS atomics.
// A bin set as every wavefront holds it, in scalar registers: range j (of
// NR) covers flat record numbers [pre[j], pre[j + 1]) (pre = 2^31 - 1 past
// the last range), and flat number f of range j is record f + delta[j].
template <int NR>
struct BinSet {
  int total;
  int pre[NR];
  int delta[NR];
};

static __device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// A bin set in flight: lane i < n of every wavefront holds the first record
// and the length of range i.  Fetching it only issues loads; committing forms
// the prefix and moves the set into scalar registers, then synchronises the
// block.
struct BinFetch {
  int n;
  int b0, len;
};

// The bins holding homes in [lox, hix] x [loy, hiy] (periodic), as runs of
// consecutive bins (first, end), written to out[kRunStride] and padded with
// (0, 0).  Bins of one tile row are stored by increasing column, so a run of
// consecutive columns is one contiguous record range; the column list is a
// cyclic run, broken at most once where it wraps: at most two runs per row.
template <int TILE>
static __device__ void tile_runs(int lox, int hix, int loy, int hiy, int nx, int ny, int ntx, int2* out) {
  int tx[TileCfg<TILE>::kMaxCols], ty[TileCfg<TILE>::kMaxCols];
  const int ncx = bins_covering<TILE>(lox, hix, nx, tx);
  const int ncy = bins_covering<TILE>(loy, hiy, ny, ty);
  int n = 0;
  for (int r = 0; r < ncy; ++r) {
    int c = 0;
    while (c < ncx) {
      int m = 1;
      while (c + m < ncx && tx[c + m] == tx[c + m - 1] + 1) ++m;
      const int first = bin_at(tx[c], ty[r], ntx);
      out[n++] = make_int2(first, first + m);
      c += m;
    }
  }
  for (; n < kRunStride; ++n) out[n] = make_int2(0, 0);
}

// Fetch of the bin set of tile `tile` (row-major index) for reader `kind`
// (0 filter, 1 spread) from the world's run table (NR runs).
template <int NR>
static __device__ __forceinline__ BinFetch binset_fetch(const WorldDev& w, int tile, int kind) {
  const int lane = __lane_id();
  BinFetch f;
  f.n = NR;
  f.b0 = 0;
  f.len = 0;
  if (lane < NR) {
    const vi2 run = glbv<const vi2>(w.tile_rng)[((size_t)tile * 2 + kind) * kRunStride + lane];
    const MC_GLOBAL int* bstart = glb(w.bin_start);
    f.b0 = bstart[run.x];
    f.len = bstart[run.y] - f.b0;
  }
  return f;
}

template <int NR>
static __device__ __forceinline__ BinSet<NR> binset_commit(const BinFetch& f) {
  const int lane = __lane_id();
  const int len = lane < f.n ? f.len : 0;
  int x = len;                                 // inclusive prefix over lanes 0..NR-1
#pragma unroll
  for (int off = 1; off < NR; off <<= 1) {
    const int y = __shfl_up(x, off);
    if (lane >= off) x += y;
  }
  const int excl = x - len;
  const int pre = lane < f.n ? excl : 0x7fffffff;
  const int del = f.b0 - excl;
  BinSet<NR> bs;
  bs.total = __builtin_amdgcn_readlane(x, NR - 1);
#pragma unroll
  for (int j = 0; j < NR; ++j) {
    bs.pre[j] = __builtin_amdgcn_readlane(pre, j);
    bs.delta[j] = __builtin_amdgcn_readlane(del, j);
  }
  __syncthreads();
  return bs;
}

// A list whose every record is needed (the spread lists the filter writes):
// the NT threads take the records in turn, with no keep test and no compaction.
template <int NT, int NR, class Body>
static __device__ __forceinline__ void for_list_records(const MC_GLOBAL vi4* recs, const BinSet<NR>& bs, Body body) {
  const int total = bs.total, off = bs.delta[0];
  for (int f = (int)threadIdx.x; f < total; f += NT) {
    const vi4 r = recs[f + off];
    body(r);
  }
  __syncthreads();
}

template <int PER, int NT, int NR, class Keep, class Body>
static __device__ __forceinline__ void for_bin_records(const MC_GLOBAL vi4* recs, const BinSet<NR>& bs, vi4* s_list,
                                                       Keep keep, Body body) {
  const int total = bs.total;
  const int lane = __lane_id();
  const unsigned long long below = (1ull << lane) - 1ull;
  vi4* wl = s_list + (threadIdx.x >> 6) * kWaveList;
  int cnt = 0;                                 // wavefront-uniform list length (< 64)
  for (int base = 0; base < total; base += PER * NT) {
    // record indices first, then every load unconditionally (lanes past the
    // end reload the last record and drop it), so all PER loads are in flight
    // together instead of each waiting inside its own branch
    int idx[PER];
    bool k[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int f = base + i * NT + (int)threadIdx.x;
      k[i] = f < total;
      const int fc = k[i] ? f : total - 1;
      int d = bs.delta[0];
#pragma unroll
      for (int j = 1; j < NR; ++j) d = fc >= bs.pre[j] ? bs.delta[j] : d;
      idx[i] = fc + d;
    }
    vi4 r[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) r[i] = recs[idx[i]];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const bool kk = k[i] && keep(r[i]);
      const unsigned long long m = __ballot(kk);
      const int pos = cnt + __popcll(m & below);
      if (kk && pos < kWaveList) wl[pos] = r[i];
      cnt += __popcll(m);
      if (cnt >= kWaveList) {
        wave_sync();
        body(wl[lane]);
        wave_sync();
        if (kk && pos >= kWaveList) wl[pos - kWaveList] = r[i];
        cnt -= kWaveList;
        wave_sync();
      }
    }
  }
  wave_sync();
  if (lane < cnt) body(wl[lane]);
  __syncthreads();
}

// Node -> grid accumulation over a padded window.  A window of side
// S = need + 6 covers grid cells o + c (c in [0, S), o = origin, periodic)
// for a caller that reads the `need` cells [3, 3 + need); a node whose home
// cell is h adds to window cells d + (0..3), d = (h - 1 - o) mod n in [0, n).
// Every contribution lands inside the window, so the inner loops carry no
// bounds or wrap tests:
//   * when need + 3 <= n, a node with d > need + 2 cannot touch the needed
//     cells (its support lies past them, and the part that wraps lands in
//     cells 0..2), so only nodes with d <= need + 2 are kept: their cells
//     reach at most need + 5;
//   * otherwise (small grids, n < need + 3) every node of the bins is kept,
//     its cells reach at most n + 2 < S, and window cells that are the same
//     grid cell are summed when read.
// The first three and last three window cells only catch the spill of nodes
// at the edge of the needed range.

// Window cell sum for needed cell i (window cell 3 + i) on an axis of n cells:
// one term unless the window wraps onto itself.
static __device__ __forceinline__ int first_image(int i, int n) {
  const int c = i + 3;
  return c < n ? c : c % n;
}

// Tile spread: for every node whose 4x4 support meets the tile [x0, x0+tw) x
// [y0, y0+th), add scale * W(c - x_i) * (v[i], v[N + i]) to the window
// accumulators s_x, s_y (64-bit fixed point, side kSpreadSide, origin
// (x0 - 3, y0 - 3)).  Nodes are read from the home-tile bins of the
// neighbourhood.  All threads of the block call it; the accumulators must be
// zeroed (and synchronised) beforehand.  Values whose fixed-point image fits
// 32 bits (|scale v| < 1/8, as nearly all forces) are converted by one
// truncating 32-bit conversion; larger ones by the exact 64-bit split.

// Whether a node with home cell (hx, hy) reaches the spread window of the
// tile at (x0, y0) of size tw x th (the keep rule of tile_spread_vec).  With
// two-layer markers (a world with marker displacements) a node counts if one
// of its markers can: the markers' homes lie within one cell of the node's,
// so the kept homes reach one cell further on every side.
struct SpreadKeep {
  int ox, oy, kx, ky, nx, ny;
  __device__ __forceinline__ SpreadKeep(const WorldDev& w, int x0, int y0, int tw, int th) {
    const int m = w.d_marker ? 1 : 0;
    nx = w.nx;
    ny = w.ny;
    ox = wrap_index(x0 - 3 - m, nx);
    oy = wrap_index(y0 - 3 - m, ny);
    kx = tw + 3 + 2 * m <= nx ? tw + 2 + 2 * m : nx;
    ky = th + 3 + 2 * m <= ny ? th + 2 + 2 * m : ny;
  }
  __device__ __forceinline__ bool operator()(const vi4& r) const {
    return wrap_near((r.x & 0xffff) - 1 - ox, nx) <= kx && wrap_near((r.x >> 16) - 1 - oy, ny) <= ky;
  }
};

// The bin set a tile spread reads: homes in [x0 - 3, x0 + tw + 1] x
// [y0 - 3, y0 + th + 1] (run table kind 1: the homes whose support, or one of
// whose two-layer markers' supports, meets the tile; one-layer readers keep
// the narrower range [x0 - 2, x0 + tw] of it by their keep test).
template <int TILE>
static __device__ __forceinline__ BinFetch spread_fetch(const WorldDev& w, int x0, int y0) {
  constexpr int sh = TileCfg<TILE>::kShift;
  return binset_fetch<TileCfg<TILE>::kRanges>(w, (y0 >> sh) * w.ntx + (x0 >> sh), 1);
}

// One point's 4x4 contribution W * (Vx, Vy) to two 64-bit fixed-point LDS
// windows of row length SIDE at the point's support origin (px, py).
template <int SIDE, bool SCALAR = false>
static __device__ __forceinline__ void spread_point(long long* sx, long long* sy, const float* wx,
                                                    const float* wy, float Vx, float Vy) {
  unsigned long long* px = (unsigned long long*)sx;
  unsigned long long* py = (unsigned long long*)sy;
  if (fmaxf(fabsf(Vx), fabsf(Vy)) < 0.125f) {
    float ax[4], ay[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      ax[a] = (Vx * kFixScale) * wx[a];
      ay[a] = (Vy * kFixScale) * wx[a];
    }
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        atomicAdd(px + b * SIDE + a, (unsigned long long)(long long)(int)(ax[a] * wy[b]));
        if constexpr (!SCALAR) atomicAdd(py + b * SIDE + a, (unsigned long long)(long long)(int)(ay[a] * wy[b]));
      }
  } else {
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const float ww = wx[a] * wy[b];
        atomicAdd(px + b * SIDE + a, (unsigned long long)f32_to_fix(ww * Vx * kFixScale));
        if constexpr (!SCALAR) atomicAdd(py + b * SIDE + a, (unsigned long long)f32_to_fix(ww * Vy * kFixScale));
      }
  }
}

// With s_g (REP), the spread value of a node is its total force: v (the
// elastic force) minus k_rep times the kernel-weighted gradient at its
// support, read from s_g, the gradient staged over the same window; the home
// tile of a node (the one tile holding its home cell) also writes that total
// to w.fel.  The gradient sum runs in the same order as the repulsion gather
// of the node kernels, so the forces are the same.  With LIST, `bins` names
// one range of records that the tile needs, every one of them (its spread
// list), so they skip the keep test.  SCALAR spreads scale * v[i] alone into
// s_x (s_y is not touched and may be null).
template <int TILE, bool REP, bool LIST = false, bool SCALAR = false>
static __device__ void tile_spread_vec(const WorldDev& w, int x0, int y0, int tw, int th,
                                       const MC_GLOBAL float* v, float scale, long long* s_x,
                                       long long* s_y, vi4* s_list, const MC_GLOBAL vi4* recs,
                                       const BinFetch& bins, const vf2* s_g) {
  using C = TileCfg<TILE>;
  constexpr int kSpreadSide = C::kSpreadSide;
  const int nx = w.nx, ny = w.ny, N = w.n_part;
  const auto bs = binset_commit<C::kRanges>(bins);
  const int ox = wrap_index(x0 - 3, nx), oy = wrap_index(y0 - 3, ny);
  const int keep_x = tw + 3 <= nx ? tw + 2 : nx;     // largest kept home offset
  const int keep_y = th + 3 <= ny ? th + 2 : ny;
  const float kr = w.k_rep;
  MC_GLOBAL float* ftot = glb(w.fel);
  const auto keep = [&](const vi4& r) {
    const int dx = wrap_near((r.x & 0xffff) - 1 - ox, nx);
    const int dy = wrap_near((r.x >> 16) - 1 - oy, ny);
    return dx <= keep_x && dy <= keep_y;
  };
  const auto body = [&](const vi4& r) {
    const int dx = wrap_near((r.x & 0xffff) - 1 - ox, nx);
    const int dy = wrap_near((r.x >> 16) - 1 - oy, ny);
    float wx[4], wy[4];
    peskin4(__int_as_float(r.y), wx);
    peskin4(__int_as_float(r.z), wy);
    float Vx, Vy;
    if constexpr (REP) {
      float gx = 0.f, gy = 0.f;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const vf2* row = s_g + (dy + b) * kSpreadSide + dx;
        float ax = 0.f, ay = 0.f;
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          const vf2 t = row[a];
          ax += wx[a] * t.x;
          ay += wx[a] * t.y;
        }
        gx += wy[b] * ax;
        gy += wy[b] * ay;
      }
      Vx = v[r.w] - kr * gx;
      Vy = v[N + r.w] - kr * gy;
      const int hx = r.x & 0xffff, hy = r.x >> 16;
      if (hx >= x0 && hx < x0 + tw && hy >= y0 && hy < y0 + th) {
        ftot[r.w] = Vx;
        ftot[N + r.w] = Vy;
      }
    } else {
      Vx = scale * v[r.w];
      Vy = SCALAR ? 0.f : scale * v[N + r.w];
    }
    spread_point<kSpreadSide, SCALAR>(s_x + dy * kSpreadSide + dx, s_y + dy * kSpreadSide + dx, wx, wy, Vx, Vy);
  };
  if constexpr (LIST) for_list_records<C::kThreads>(recs, bs, body);
  else for_bin_records<4, C::kThreads>(recs, bs, s_list, keep, body);
}

// The tile spread of a two-layer world: each node acts through its markers
// X = x +- d (d from w.d_marker), each taking half of the node's value.  The
// node's value is formed as in tile_spread_vec, with the gradient s_g staged
// over a window one cell wider on every side (side kSpreadSide + 2, origin
// (x0 - 4, y0 - 4)), since a node whose marker reaches the tile can lie one
// cell further out.  The accumulators keep side kSpreadSide and origin
// (x0 - 3, y0 - 3): a marker goes in by the one-layer keep rule applied to
// its own home cell, and the others cannot touch the tile.
template <int TILE, bool REP, bool LIST = false>
static __device__ void tile_spread_markers(const WorldDev& w, int x0, int y0, int tw, int th,
                                           const MC_GLOBAL float* v, float scale, long long* s_x,
                                           long long* s_y, vi4* s_list, const MC_GLOBAL vi4* recs,
                                           const BinFetch& bins, const vf2* s_g) {
  using C = TileCfg<TILE>;
  constexpr int kSpreadSide = C::kSpreadSide, kGSide = C::kSpreadSide + 2;
  const int nx = w.nx, ny = w.ny, N = w.n_part;
  const auto bs = binset_commit<C::kRanges>(bins);
  const int ox = wrap_index(x0 - 3, nx), oy = wrap_index(y0 - 3, ny);
  const int gox = wrap_index(x0 - 4, nx), goy = wrap_index(y0 - 4, ny);
  const int keep_x = tw + 3 <= nx ? tw + 2 : nx;     // markers: largest kept home offset
  const int keep_y = th + 3 <= ny ? th + 2 : ny;
  const int nkeep_x = tw + 5 <= nx ? tw + 4 : nx;    // nodes: one cell more on each side
  const int nkeep_y = th + 5 <= ny ? th + 4 : ny;
  const float kr = w.k_rep;
  MC_GLOBAL float* ftot = glb(w.fel);
  const MC_GLOBAL float* dm = glb(w.d_marker);
  const auto keep = [&](const vi4& r) {
    const int dx = wrap_near((r.x & 0xffff) - 1 - gox, nx);
    const int dy = wrap_near((r.x >> 16) - 1 - goy, ny);
    return dx <= nkeep_x && dy <= nkeep_y;
  };
  const auto body = [&](const vi4& r) {
    const int hx = r.x & 0xffff, hy = r.x >> 16;
    const float fx = __int_as_float(r.y), fy = __int_as_float(r.z);
    float Vx, Vy;
    if constexpr (REP) {
      const int dx = wrap_near(hx - 1 - gox, nx), dy = wrap_near(hy - 1 - goy, ny);
      float wx[4], wy[4];
      peskin4(fx, wx);
      peskin4(fy, wy);
      float gx = 0.f, gy = 0.f;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const vf2* row = s_g + (dy + b) * kGSide + dx;
        float ax = 0.f, ay = 0.f;
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          const vf2 t = row[a];
          ax += wx[a] * t.x;
          ay += wx[a] * t.y;
        }
        gx += wy[b] * ax;
        gy += wy[b] * ay;
      }
      Vx = v[r.w] - kr * gx;
      Vy = v[N + r.w] - kr * gy;
      if (hx >= x0 && hx < x0 + tw && hy >= y0 && hy < y0 + th) {
        ftot[r.w] = Vx;
        ftot[N + r.w] = Vy;
      }
    } else {
      Vx = scale * v[r.w];
      Vy = scale * v[N + r.w];
    }
    const float ddx = dm[r.w], ddy = dm[N + r.w];
    const float hVx = 0.5f * Vx, hVy = 0.5f * Vy;
#pragma unroll
    for (int l = 0; l < 2; ++l) {
      const float sg = l == 0 ? 1.f : -1.f;
      int sx, sy;
      float mx, my;
      marker_shift(fx, sg * ddx, &sx, &mx);
      marker_shift(fy, sg * ddy, &sy, &my);
      const int mdx = wrap_index(hx + sx - 1 - ox, nx), mdy = wrap_index(hy + sy - 1 - oy, ny);
      if (mdx <= keep_x && mdy <= keep_y) {
        float wx[4], wy[4];
        peskin4(mx, wx);
        peskin4(my, wy);
        spread_point<kSpreadSide>(s_x + mdy * kSpreadSide + mdx, s_y + mdy * kSpreadSide + mdx, wx, wy, hVx, hVy);
      }
    }
  };
  if constexpr (LIST) for_list_records<C::kThreads>(recs, bs, body);
  else for_bin_records<4, C::kThreads>(recs, bs, s_list, keep, body);
}

// The accumulated value of tile cell (lx, ly) of a spread window.
template <int TILE>
static __device__ __forceinline__ long long spread_cell(const long long* s, int lx, int ly, int nx, int ny) {
  constexpr int kSpreadSide = TileCfg<TILE>::kSpreadSide;
  const int cx0 = first_image(lx, nx), cy0 = first_image(ly, ny);
  if (cx0 + nx >= kSpreadSide && cy0 + ny >= kSpreadSide) return s[cy0 * kSpreadSide + cx0];
  long long acc = 0;
  for (int cy = cy0; cy < kSpreadSide; cy += ny)
    for (int cx = cx0; cx < kSpreadSide; cx += nx) acc += s[cy * kSpreadSide + cx];
  return acc;
}

template <int TILE>
static inline bool tile_family_present(const Grid& G) {
  return G.tile_blocks[TileCfg<TILE>::kFamily] > 0;
}

// Host side: launch a tile kernel with a one-layer and a two-layer variant
// (template argument MK last) for every tile family present, in the
// variants the grid needs: launch(Int<TILE>, Bool<MK>) launches one.  Each
// variant skips the other's worlds; the two-layer one runs only where a
// binned world has markers, the one-layer one unless every world has them.
template <class L>
static inline void for_tile_variants(const Grid& G, L launch) {
  const bool mk = G.any_markers && G.any_binned, plain = !G.mk_only;
  if (tile_family_present<16>(G)) {
    if (plain) launch(std::integral_constant<int, 16>(), std::false_type());
    if (mk) launch(std::integral_constant<int, 16>(), std::true_type());
  }
  if (tile_family_present<32>(G)) {
    if (plain) launch(std::integral_constant<int, 32>(), std::false_type());
    if (mk) launch(std::integral_constant<int, 32>(), std::true_type());
  }
  if (tile_family_present<64>(G)) {
    if (plain) launch(std::integral_constant<int, 64>(), std::false_type());
    if (mk) launch(std::integral_constant<int, 64>(), std::true_type());
  }
}

}  // namespace mc
