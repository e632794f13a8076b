// Device helpers shared by the forward and adjoint kernels.
#pragma once

#include <math.h>

#include "engine.h"

namespace mc {

constexpr float kPi = 3.14159265358979323846f;
constexpr float kTwoPi = 6.28318530717958647692f;
constexpr double kTwoPiD = 6.28318530717958647692;

static __device__ __forceinline__ int wrap_index(int i, int n) {
  int r = i % n;
  return r < 0 ? r + n : r;
}

static __device__ __forceinline__ int wrap_near(int v, int n) {   // v in [-n, 2n)
  return v < 0 ? v + n : (v >= n ? v - n : v);
}

// Map an angle difference into (-pi, pi].
static __device__ __forceinline__ float wrap_angle(float d) {
  return d - kTwoPi * ceilf((d - kPi) / kTwoPi);
}

// The four 1D weights of Peskin's 4-point function for offsets
// (-1 - f, -f, 1 - f, 2 - f), f in [0, 1): with q = sqrt(1 + 4f - 4f^2) they
// are (3 - 2f - q)/8, (3 - 2f + q)/8, (1 + 2f + q)/8, (1 + 2f - q)/8.
static __device__ __forceinline__ void peskin4(float f, float w[4]) {
  const float q = sqrtf(fmaf(4.0f * f, 1.0f - f, 1.0f));
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
  const float q = sqrtf(fmaf(4.0f * f, 1.0f - f, 1.0f));
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

// D2Q9 lattice: velocity q has components (CX[q], CY[q]); q and q+2 are
// opposite for q = 1, 2, 5, 6.
static __constant__ int kCX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static __constant__ int kCY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

// Distinct tiles (of kTile cells) holding the cells lo..hi of a periodic
// axis of n cells split into ntile tiles.  The ranges used here are at most
// 53 cells wide, so they touch at most 4 tiles.
static __device__ __forceinline__ int tiles_covering(int lo, int hi, int n, int ntile, int t[4]) {
  int cnt = 0;
  if (hi - lo + 1 >= n) {                       // whole axis (then ntile <= 2)
    for (int k = 0; k < ntile && cnt < 4; ++k) t[cnt++] = k;
    return cnt;
  }
  int c = lo;
  while (c <= hi && cnt < 4) {
    const int cc = wrap_index(c, n);
    const int tt = cc / kTile;
    bool seen = false;
    for (int k = 0; k < cnt; ++k) seen |= (t[k] == tt);
    if (!seen) t[cnt++] = tt;
    c += min((tt + 1) * kTile, n) - cc;         // jump to the next tile boundary
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
static __device__ __forceinline__ void lds_fix_add(long long* p, float v) {
  atomicAdd((unsigned long long*)p, (unsigned long long)f32_to_fix(v * kFixScale));
}
static __device__ __forceinline__ float fix_to_float(long long v) {
  const int hi = (int)(v >> 32);
  const unsigned lo = (unsigned)v;
  return (float)((double)hi * 4294967296.0 + (double)lo) * kFixInv;
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

// Block-wide exclusive scan of one int per thread (256 threads), wave
// shuffles plus one LDS exchange.  Returns the exclusive prefix; *total gets
// the block sum.  All threads must call it.
static __device__ __forceinline__ int block_scan256(int v, int* s_wave, int* total) {
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
  for (int k = 0; k < 4; ++k) {
    const int sw = s_wave[k];
    before += (k < wid) ? sw : 0;
    all += sw;
  }
  __syncthreads();
  *total = all;
  return before + x - v;
}


// Records of a set of home-tile bins (the set lives in LDS, built by one
// thread), visited in chunks: the records for which keep(r) holds are first
// compacted into an LDS list (wavefront ballots, one LDS atomic per
// wavefront), then body(r) runs over the dense list, so lanes holding
// irrelevant records do not idle through the work.
constexpr int kListCap = 1024;

struct BinSet {
  int n;
  int start[16];
  int pre[17];
};

// Build the bin set of the tiles tx[ntx] x ty[nty] in LDS: one thread per
// bin loads its range (independent loads, no chain), then a short prefix.
// All threads call it with the same tile lists.
static __device__ __forceinline__ void make_binset(const MC_GLOBAL int* bstart, int tiles_per_row, const int* tx,
                                                   int ntx, const int* ty, int nty, BinSet* bs) {
  const int n = ntx * nty;
  const int i = threadIdx.x;
  if (i < n) {
    const int t = ty[i / ntx] * tiles_per_row + tx[i - (i / ntx) * ntx];
    const int b0 = bstart[t];
    bs->start[i] = b0;
    bs->pre[i + 1] = bstart[t + 1] - b0;      // length, turned into a prefix below
  }
  __syncthreads();
  if (i == 0) {
    bs->n = n;
    bs->pre[0] = 0;
    for (int k = 1; k <= n; ++k) bs->pre[k] += bs->pre[k - 1];
  }
  __syncthreads();
}

template <class Keep, class Body>
static __device__ __forceinline__ void for_bin_records(const MC_GLOBAL vi4* recs, const BinSet& bs, vi4* s_list,
                                                       int* s_count, Keep keep, Body body) {
  constexpr int kPer = kListCap / 256;         // records each thread loads per round
  const int total = bs.pre[bs.n];
  const int lane = __lane_id();
  for (int base = 0; base < total; base += kListCap) {
    if (threadIdx.x == 0) *s_count = 0;
    vi4 r[kPer];
    bool k[kPer];
#pragma unroll
    for (int i = 0; i < kPer; ++i) {           // issue every load before any use
      const int f = base + i * 256 + (int)threadIdx.x;
      k[i] = f < total;
      if (k[i]) {
        int b = 0;
        while (f >= bs.pre[b + 1]) ++b;
        r[i] = recs[bs.start[b] + (f - bs.pre[b])];
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const bool kk = k[i] && keep(r[i]);
      const unsigned long long m = __ballot(kk);
      int base_i = 0;
      if (lane == 0 && m) base_i = atomicAdd(s_count, __popcll(m));
      base_i = __shfl(base_i, 0);
      if (kk) s_list[base_i + __popcll(m & ((1ull << lane) - 1ull))] = r[i];
    }
    __syncthreads();
    const int n = *s_count;
    for (int i = threadIdx.x; i < n; i += blockDim.x) body(s_list[i]);
    __syncthreads();
  }
}

// Add, for every node whose 4x4 support meets the tile [x0, x0+tw) x
// [y0, y0+th), the values scale * W(c - x_i) * (v[i], v[N + i]) to the tile's
// LDS accumulators (64-bit fixed point, row stride kTile).  Nodes are read
// from the home-tile bins of the neighbourhood.  All threads of the block
// call it; accumulators must be zeroed (and synchronised) beforehand.
static __device__ void tile_spread_vec(const WorldDev& w, int x0, int y0, int tw, int th,
                                       const MC_GLOBAL float* v, float scale, long long* s_x,
                                       long long* s_y, vi4* s_list, int* s_count, BinSet* s_bs) {
  const int nx = w.nx, ny = w.ny, N = w.n_part;
  {
    int txs[4], tys[4];
    const int ntxs = tiles_covering(x0 - 2, x0 + tw, nx, w.ntx, txs);
    const int ntys = tiles_covering(y0 - 2, y0 + th, ny, w.nty, tys);
    make_binset(glb(w.bin_start), w.ntx, txs, ntxs, tys, ntys, s_bs);
  }
  for_bin_records(
      glbv<const vi4>(w.bin_rec), *s_bs, s_list, s_count,
      [&](const vi4& r) {
        const int dx = wrap_near((r.x & 0xffff) - 1 - x0, nx);   // home in [0,n), x0 in [0,n)
        const int dy = wrap_near((r.x >> 16) - 1 - y0, ny);
        return !((dx >= tw && dx + 3 < nx) || (dy >= th && dy + 3 < ny));
      },
      [&](const vi4& r) {
        const int dx = wrap_near((r.x & 0xffff) - 1 - x0, nx);
        const int dy = wrap_near((r.x >> 16) - 1 - y0, ny);
        float wx[4], wy[4];
        peskin4(__int_as_float(r.y), wx);
        peskin4(__int_as_float(r.z), wy);
        const float Vx = scale * v[r.w], Vy = scale * v[N + r.w];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          int ly = dy + b;
          ly = ly >= ny ? ly - ny : ly;
          if (ly >= th) continue;
#pragma unroll
          for (int a = 0; a < 4; ++a) {
            int lx = dx + a;
            lx = lx >= nx ? lx - nx : lx;
            if (lx >= tw) continue;
            const float ww = wx[a] * wy[b];
            lds_fix_add(&s_x[ly * kTile + lx], ww * Vx);
            lds_fix_add(&s_y[ly * kTile + lx], ww * Vy);
          }
        }
      });
}

}  // namespace mc
