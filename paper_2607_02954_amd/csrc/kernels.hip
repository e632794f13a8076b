// Forward kernels of the filament-fluid step for gfx950 (CDNA4).
//
// Step order (one launch per sub-step, all worlds of a table at once):
//   k_elastic     S0 actuation + S1 PBD Cosserat projection (Eqs. 1-4) -> node
//                 elastic force; registers each node with the tiles it affects
//   k_bin_scan    per-world prefix over tile counts      (binned transfer)
//   k_bin_fill    node indices into their tile bins      (binned transfer)
//   k_filter      S2 deposit + S3 separable circular Gaussian filter on a
//                 32x32 tile with an R-cell halo, all in LDS; writes s~
//   k_repulse     S4 repulsion from the gradient of s~ -> total node force
//   k_lbm         S5 force spread (in LDS) + S6 D2Q9 TRT/Guo collision and
//                 push streaming on a 32x32 tile; exports u
//   k_integrate   S7 gather u at the nodes and move them
//
// Particle -> grid transfer has three modes, chosen per world:
//   binned  nodes are binned by the 32x32 tiles their (filter-extended)
//           support touches; each tile sums its nodes' contributions in LDS
//           and writes every cell once, so no HBM atomics and no clearing pass
//   sorted  nodes are counting-sorted by home cell and every grid value is a
//           fixed-order sum over the sorted segments of its 4x4 home window:
//           bitwise reproducible
//   direct  global float atomics into HBM accumulators (reference point)
//
// Node kernels run one block per node pack (whole filaments, <= pack nodes,
// filament-contiguous SoA), so neighbour exchange along a chain stays in LDS.
// Positions are an integer cell plus a float fraction, so the quantities the
// physics needs (edge vectors, kernel offsets) are formed from small numbers.
#include "engine.h"

#include <math.h>

namespace mc {

namespace {

constexpr float kPi = 3.14159265358979323846f;
constexpr float kTwoPi = 6.28318530717958647692f;
constexpr double kTwoPiD = 6.28318530717958647692;

__device__ __forceinline__ int wrap_index(int i, int n) {
  int r = i % n;
  return r < 0 ? r + n : r;
}

__device__ __forceinline__ int wrap_near(int v, int n) {   // v in [-n, 2n)
  return v < 0 ? v + n : (v >= n ? v - n : v);
}

// Map an angle difference into (-pi, pi].
__device__ __forceinline__ float wrap_angle(float d) {
  return d - kTwoPi * ceilf((d - kPi) / kTwoPi);
}

// The four 1D weights of Peskin's 4-point function for offsets
// (-1 - f, -f, 1 - f, 2 - f), f in [0, 1): with q = sqrt(1 + 4f - 4f^2) they
// are (3 - 2f - q)/8, (3 - 2f + q)/8, (1 + 2f + q)/8, (1 + 2f - q)/8.
__device__ __forceinline__ void peskin4(float f, float w[4]) {
  const float q = sqrtf(fmaf(4.0f * f, 1.0f - f, 1.0f));
  const float a = 3.0f - 2.0f * f;
  const float b = 1.0f + 2.0f * f;
  w[0] = 0.125f * (a - q);
  w[1] = 0.125f * (a + q);
  w[2] = 0.125f * (b + q);
  w[3] = 0.125f * (b - q);
}

// D2Q9 lattice: velocity q has components (CX[q], CY[q]); q and q+2 are
// opposite for q = 1, 2, 5, 6.
__constant__ int kCX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__constant__ int kCY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

// Distinct tiles (in order) covering cells b+lo .. b+hi (periodic, n cells,
// tiles of kTile cells).  At most 3 because full tiles are wider than any
// extended support (<= 20 cells).
__device__ __forceinline__ int tile_span(int b, int lo, int hi, int n, int t[3]) {
  int cnt = 0;
  int last = -1;
  for (int c = b + lo; c <= b + hi; ++c) {
    const int tt = wrap_index(c, n) / kTile;
    if (tt != last) {
      bool seen = false;
      for (int k = 0; k < cnt; ++k) seen |= (t[k] == tt);
      if (!seen && cnt < 3) t[cnt++] = tt;
      last = tt;
    }
  }
  return cnt;
}

// Wavefront-aggregated atomic increment: lanes that target the same counter
// are served by one atomic from a leader lane.  Returns, for lanes with `has`,
// a distinct slot (the counter's old value plus the lane's rank among the
// matching lanes).  Must be called by every lane of the wavefront.
__device__ __forceinline__ int agg_atomic_inc(int* counters, int key, bool has) {
  const int lane = __lane_id();
  unsigned long long pending = __ballot(has);
  int slot = 0;
  while (pending) {
    const int leader = __ffsll((unsigned long long)pending) - 1;
    const int lkey = __shfl(key, leader);
    const unsigned long long match = __ballot(has && key == lkey) & pending;
    int base = 0;
    if (lane == leader) base = atomicAdd(&counters[lkey], __popcll(match));
    base = __shfl(base, leader);
    if ((match >> lane) & 1ull) slot = base + __popcll(match & ((1ull << lane) - 1ull));
    pending &= ~match;
  }
  return slot;
}

// Block-wide exclusive scan of one int per thread (256 threads), wave
// shuffles plus one LDS exchange.  Returns the exclusive prefix; *total gets
// the block sum.  All threads must call it.
__device__ __forceinline__ int block_scan256(int v, int* s_wave, int* total) {
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

}  // namespace

// ---------------------------------------------------------------------------
// S0 + S1: actuation and PBD elastic force.  Then, by transfer mode: tile-bin
// counts (binned), home-cell key and rank (sorted) or the density deposit
// with global atomics (direct).
// ---------------------------------------------------------------------------
template <int PACK>
__global__ __launch_bounds__(PACK) void k_elastic(const WorldDev* __restrict__ W, Tables T) {
  __shared__ float s_th[PACK];
  __shared__ float s_dx[PACK];
  __shared__ float s_dy[PACK];
  __shared__ int s_off[PACK + 1];

  const int npk = *T.n_packs;
  const int li = threadIdx.x;
  for (int it = blockIdx.x; it < npk; it += gridDim.x) {
    const Pack pk = T.packs[it];
    const WorldDev& w = W[pk.world];
    const Ctl ctl = *w.ctl_src;
    if (ctl.remaining <= 0) continue;           // block-uniform
    const int nf = pk.fil_end - pk.fil_begin;
    for (int k = li; k <= nf; k += PACK) s_off[k] = w.fil_offset[pk.fil_begin + k] - pk.node_begin;
    __syncthreads();

    const int N = w.n_part;
    const int gi = pk.node_begin + li;
    const bool active = gi < pk.node_end;
    // filament of this node: largest f with s_off[f] <= li
    int lo = 0, hi = nf - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (s_off[mid] <= li) lo = mid; else hi = mid - 1;
    }
    const int o = s_off[lo];
    const int n = s_off[lo + 1] - o;
    const int k = li - o;
    const bool has_edge = active && k < n - 1;
    const bool is_joint = active && k >= 1 && k <= n - 2;
    const int j = k - 1;

    int cx = 0, cy = 0;
    float fx = 0.f, fy = 0.f;
    if (active) {
      cx = w.cell_in[gi]; cy = w.cell_in[N + gi];
      fx = w.frac_in[gi]; fy = w.frac_in[N + gi];
    }
    float v0x = 0.f, v0y = 0.f, L = 0.f, th = 0.f;
    if (has_edge) {
      v0x = (float)(w.cell_in[gi + 1] - cx) + (w.frac_in[gi + 1] - fx);
      v0y = (float)(w.cell_in[N + gi + 1] - cy) + (w.frac_in[N + gi + 1] - fy);
      L = w.rest_length[gi];
      th = atan2f(v0y, v0x);
    }
    float th_hat = 0.f;
    if (is_joint) {
      const int f = pk.fil_begin + lo;
      const float amp = w.act_amp[f];
      const float ra = w.rest_angle[gi];
      if (amp != 0.0f) {
        const double arg = kTwoPiD * (double)ctl.t / (double)w.act_period[f] + (double)w.act_phase[f] -
                           kTwoPiD * (double)j / (double)(n - 2);
        th_hat = (float)((double)ra + (double)amp * sin(arg));
      } else {
        th_hat = ra;
      }
    }
    s_th[li] = th;
    s_dx[li] = 0.f;
    s_dy[li] = 0.f;
    __syncthreads();

    const float hb = 0.5f * w.k_bend;
    const float hs = 0.5f * w.k_stretch;
    const float ksh = w.k_shear;
    for (int iter = 0; iter < w.pbd_iters; ++iter) {
      // bending pass (Eq. 1): even joints, then odd joints
      for (int par = 0; par < 2; ++par) {
        if (is_joint && (j & 1) == par) {
          const float t1 = s_th[li - 1];
          const float t2 = s_th[li];
          const float c = wrap_angle(t2 - t1) - th_hat;
          s_th[li - 1] = t1 + hb * c;
          s_th[li] = t2 - hb * c;
        }
        __syncthreads();
      }
      // position pass (Eqs. 2-4): even edges, then odd edges
      for (int par = 0; par < 2; ++par) {
        if (has_edge && (k & 1) == par) {
          const float d0x = s_dx[li], d0y = s_dy[li];
          const float d1x = s_dx[li + 1], d1y = s_dy[li + 1];
          const float vx = v0x + (d1x - d0x);
          const float vy = v0y + (d1y - d0y);
          const float ell = sqrtf(vx * vx + vy * vy);
          const float sc = (ell - L) / ell;
          const float csx = sc * vx, csy = sc * vy;
          float sn, cs;
          sincosf(s_th[li], &sn, &cs);
          const float dx = hs * (csx + ksh * (vx - L * cs - csx));
          const float dy = hs * (csy + ksh * (vy - L * sn - csy));
          s_dx[li] = d0x + dx;
          s_dy[li] = d0y + dy;
          s_dx[li + 1] = d1x - dx;
          s_dy[li + 1] = d1y - dy;
        }
        __syncthreads();
      }
    }

    const int bx = wrap_index(cx, w.nx);
    const int by = wrap_index(cy, w.ny);
    if (active) {
      w.fel[gi] = w.k_el * s_dx[li];
      w.fel[N + gi] = w.k_el * s_dy[li];
    }
    if (w.mode == kBinned) {
      int tx[3], ty[3];
      const int R = w.radius;
      const int ntx = active ? tile_span(bx, -1 - R, 2 + R, w.nx, tx) : 0;
      const int nty = active ? tile_span(by, -1 - R, 2 + R, w.ny, ty) : 0;
      for (int b = 0; b < 3; ++b)
        for (int a = 0; a < 3; ++a) {
          const bool has = a < ntx && b < nty;
          const int tile = has ? ty[b] * w.ntx + tx[a] : 0;
          agg_atomic_inc(w.bin_cnt, tile, has);
        }
    } else if (active && w.mode == kSorted) {
      const int key = by * w.nx + bx;
      w.key[gi] = key;
      w.rank[gi] = atomicAdd(&w.cnt[key], 1);
    } else if (active) {
      float wx[4], wy[4];
      peskin4(fx, wx);
      peskin4(fy, wy);
      int ix[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) ix[a] = wrap_near(bx - 1 + a, w.nx);
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        float* row = w.s + (size_t)wrap_near(by - 1 + b, w.ny) * w.nx;
#pragma unroll
        for (int a = 0; a < 4; ++a) unsafeAtomicAdd(row + ix[a], wx[a] * wy[b]);
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Binned transfer: per-world exclusive scan of tile counts, then every node
// writes its index into each bin it belongs to.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_bin_scan(const WorldDev* __restrict__ W, Tables T) {
  __shared__ int s_wave[4];
  const int nw = *T.n_worlds;
  for (int it = blockIdx.x; it < nw; it += gridDim.x) {
    const WorldDev& w = W[T.worlds[it].x];
    if (w.mode != kBinned || w.ctl_src->remaining <= 0) continue;
    const int nt = w.ntx * w.nty;
    const int per = (nt + 255) / 256;
    const int b0 = threadIdx.x * per;
    int loc = 0;
    for (int k = 0; k < per; ++k) loc += (b0 + k < nt) ? w.bin_cnt[b0 + k] : 0;
    int total;
    int run = block_scan256(loc, s_wave, &total);
    for (int k = 0; k < per; ++k) {
      if (b0 + k < nt) {
        const int v = w.bin_cnt[b0 + k];
        w.bin_start[b0 + k] = run;
        w.bin_cnt[b0 + k] = 0;
        w.bin_fill[b0 + k] = 0;
        run += v;
      }
    }
    if (threadIdx.x == 0) w.bin_start[nt] = total;
  }
}

template <int PACK>
__global__ __launch_bounds__(PACK) void k_bin_fill(const WorldDev* __restrict__ W, Tables T) {
  const int npk = *T.n_packs;
  for (int it = blockIdx.x; it < npk; it += gridDim.x) {
    const Pack pk = T.packs[it];
    const WorldDev& w = W[pk.world];
    if (w.mode != kBinned || w.ctl_src->remaining <= 0) continue;
    const int gi = pk.node_begin + threadIdx.x;
    const bool active = gi < pk.node_end;
    int tx[3], ty[3], ntx = 0, nty = 0;
    if (active) {
      const int R = w.radius;
      ntx = tile_span(wrap_index(w.cell_in[gi], w.nx), -1 - R, 2 + R, w.nx, tx);
      nty = tile_span(wrap_index(w.cell_in[w.n_part + gi], w.ny), -1 - R, 2 + R, w.ny, ty);
    }
    for (int b = 0; b < 3; ++b)
      for (int a = 0; a < 3; ++a) {
        const bool has = a < ntx && b < nty;
        const int tile = has ? ty[b] * w.ntx + tx[a] : 0;
        const int slot = agg_atomic_inc(w.bin_fill, tile, has);
        if (has) w.bin_idx[w.bin_start[tile] + slot] = gi;
      }
  }
}

// ---------------------------------------------------------------------------
// Sorted transfer: exclusive scan of the per-cell counts (three phases over
// (world, 1024-cell block) items), scatter of node indices into their slots,
// and an insertion sort of every multi-node segment by node index, so that
// all later sums run in a fixed order.
// ---------------------------------------------------------------------------
constexpr int kScanBlock = 1024;   // cells per scan item (256 threads x 4)

__global__ __launch_bounds__(256) void k_scan_reduce(const WorldDev* __restrict__ W, Tables T) {
  __shared__ int s_wave[4];
  const int n = *T.n_scan;
  for (int it = blockIdx.x; it < n; it += gridDim.x) {
    const int2 sc = T.scan[it];
    const WorldDev& w = W[sc.x];
    if (w.mode != kSorted || w.ctl_src->remaining <= 0) continue;
    const int ncell = w.nx * w.ny;
    const int c0 = sc.y * kScanBlock + threadIdx.x * 4;
    int v = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) v += (c0 + k < ncell) ? w.cnt[c0 + k] : 0;
    int total;
    block_scan256(v, s_wave, &total);
    if (threadIdx.x == 0) w.part[sc.y] = total;
  }
}

__global__ __launch_bounds__(256) void k_scan_partials(const WorldDev* __restrict__ W, Tables T) {
  __shared__ int s_wave[4];
  const int n = *T.n_worlds;
  for (int it = blockIdx.x; it < n; it += gridDim.x) {
    const WorldDev& w = W[T.worlds[it].x];
    if (w.mode != kSorted || w.ctl_src->remaining <= 0) continue;
    const int ncell = w.nx * w.ny;
    const int nb = (ncell + kScanBlock - 1) / kScanBlock;
    int carry = 0;
    for (int b0 = 0; b0 < nb; b0 += 256) {
      const int b = b0 + threadIdx.x;
      const int v = b < nb ? w.part[b] : 0;
      int total;
      const int ex = block_scan256(v, s_wave, &total);
      if (b < nb) w.part[b] = carry + ex;
      carry += total;
    }
    if (threadIdx.x == 0) w.start[ncell] = carry;
  }
}

__global__ __launch_bounds__(256) void k_scan_down(const WorldDev* __restrict__ W, Tables T) {
  __shared__ int s_wave[4];
  const int n = *T.n_scan;
  for (int it = blockIdx.x; it < n; it += gridDim.x) {
    const int2 sc = T.scan[it];
    const WorldDev& w = W[sc.x];
    if (w.mode != kSorted || w.ctl_src->remaining <= 0) continue;
    const int ncell = w.nx * w.ny;
    const int c0 = sc.y * kScanBlock + threadIdx.x * 4;
    int v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = (c0 + k < ncell) ? w.cnt[c0 + k] : 0;
    int total;
    const int ex = block_scan256(v[0] + v[1] + v[2] + v[3], s_wave, &total);
    int run = w.part[sc.y] + ex;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (c0 + k < ncell) {
        w.start[c0 + k] = run;
        w.cnt[c0 + k] = 0;          // ready for the next step's histogram
      }
      run += v[k];
    }
  }
}

template <int PACK>
__global__ __launch_bounds__(PACK) void k_scatter(const WorldDev* __restrict__ W, Tables T) {
  const int npk = *T.n_packs;
  for (int it = blockIdx.x; it < npk; it += gridDim.x) {
    const Pack pk = T.packs[it];
    const WorldDev& w = W[pk.world];
    if (w.mode != kSorted || w.ctl_src->remaining <= 0) continue;
    const int gi = pk.node_begin + threadIdx.x;
    if (gi >= pk.node_end) continue;
    w.perm[w.start[w.key[gi]] + w.rank[gi]] = gi;
  }
}

template <int PACK>
__global__ __launch_bounds__(PACK) void k_segsort(const WorldDev* __restrict__ W, Tables T) {
  const int npk = *T.n_packs;
  for (int it = blockIdx.x; it < npk; it += gridDim.x) {
    const Pack pk = T.packs[it];
    const WorldDev& w = W[pk.world];
    if (w.mode != kSorted || w.ctl_src->remaining <= 0) continue;
    const int gi = pk.node_begin + threadIdx.x;
    // one thread per segment: the node that drew rank 0 (ranks are never rewritten)
    if (gi >= pk.node_end || w.rank[gi] != 0) continue;
    const int key = w.key[gi];
    const int b = w.start[key], e = w.start[key + 1];
    for (int i = b + 1; i < e; ++i) {
      const int v = w.perm[i];
      int j = i - 1;
      while (j >= b && w.perm[j] > v) {
        w.perm[j + 1] = w.perm[j];
        --j;
      }
      w.perm[j + 1] = v;
    }
    // fractions of the sorted nodes for the density gather of this step
    const int N = w.n_part;
    for (int i = b; i < e; ++i) {
      const int v = w.perm[i];
      w.rec[i] = make_float4(w.frac_in[v], w.frac_in[N + v], 0.f, 0.f);
    }
  }
}

// Fixed-order sums over the sorted segments of the 4x4 home window of cell
// (gx, gy): the node at home cell h contributes weight index c - h + 1.
__device__ __forceinline__ float gather_density(const WorldDev& w, int gx, int gy) {
  float acc = 0.f;
  for (int b = 0; b < 4; ++b) {
    const int hy = wrap_near(gy + 1 - b, w.ny);
    for (int a = 0; a < 4; ++a) {
      const int h = hy * w.nx + wrap_near(gx + 1 - a, w.nx);
      const int e = w.start[h + 1];
      for (int sidx = w.start[h]; sidx < e; ++sidx) {
        const float4 r = w.rec[sidx];
        float wx[4], wy[4];
        peskin4(r.x, wx);
        peskin4(r.y, wy);
        acc += wx[a] * wy[b];
      }
    }
  }
  return acc;
}

__device__ __forceinline__ void gather_force(const WorldDev& w, int gx, int gy, float& Fx, float& Fy) {
  Fx = 0.f;
  Fy = 0.f;
  for (int b = 0; b < 4; ++b) {
    const int hy = wrap_near(gy + 1 - b, w.ny);
    for (int a = 0; a < 4; ++a) {
      const int h = hy * w.nx + wrap_near(gx + 1 - a, w.nx);
      const int e = w.start[h + 1];
      for (int sidx = w.start[h]; sidx < e; ++sidx) {
        const float4 r = w.rec[sidx];
        float wx[4], wy[4];
        peskin4(r.x, wx);
        peskin4(r.y, wy);
        const float ww = wx[a] * wy[b];
        Fx += ww * r.z;
        Fy += ww * r.w;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// S2 + S3: density on a 32x32 tile plus an R-cell halo, staged in LDS, then
// the separable circular Gaussian (x pass into LDS, y pass to HBM).
// ---------------------------------------------------------------------------
constexpr int kRegion = kTile + 2 * kMaxRadius;

__global__ __launch_bounds__(256) void k_filter(const WorldDev* __restrict__ W, Tables T) {
  __shared__ float s_reg[kRegion * kRegion];
  __shared__ float s_mid[kRegion * kTile];
  const int nt = *T.n_tiles;
  const int tid = threadIdx.x;
  for (int it = blockIdx.x; it < nt; it += gridDim.x) {
    const int2 tl = T.tiles[it];
    const WorldDev& w = W[tl.x];
    if (w.ctl_src->remaining <= 0) continue;
    const int R = w.radius;
    const int nx = w.nx, ny = w.ny;
    const int x0 = (tl.y % w.ntx) * kTile;
    const int y0 = (tl.y / w.ntx) * kTile;
    const int reg = kTile + 2 * R;
    const int xo = x0 - R, yo = y0 - R;          // region origin (unwrapped)
    if (w.mode == kBinned) {
      for (int k = tid; k < reg * reg; k += 256) s_reg[k] = 0.f;
      __syncthreads();
      const int tile = tl.y;
      const int e1 = w.bin_start[tile + 1];
      for (int e = w.bin_start[tile] + tid; e < e1; e += 256) {
        const int i = w.bin_idx[e];
        const int bx = wrap_index(w.cell_in[i], nx);
        const int by = wrap_index(w.cell_in[w.n_part + i], ny);
        float wx[4], wy[4];
        peskin4(w.frac_in[i], wx);
        peskin4(w.frac_in[w.n_part + i], wy);
        for (int b = 0; b < 4; ++b) {
          for (int ly = wrap_index(by - 1 + b - yo, ny); ly < reg; ly += ny) {
            for (int a = 0; a < 4; ++a) {
              for (int lx = wrap_index(bx - 1 + a - xo, nx); lx < reg; lx += nx)
                atomicAdd(&s_reg[ly * reg + lx], wx[a] * wy[b]);
            }
          }
        }
      }
    } else {
      for (int k = tid; k < reg * reg; k += 256) {
        const int r = k / reg, c = k - (k / reg) * reg;
        const int gx = wrap_index(xo + c, nx);
        const int gy = wrap_index(yo + r, ny);
        s_reg[k] = w.mode == kSorted ? gather_density(w, gx, gy) : w.s[(size_t)gy * nx + gx];
      }
    }
    __syncthreads();
    for (int k = tid; k < reg * kTile; k += 256) {
      const int r = k / kTile, c = k - (k / kTile) * kTile;
      const float* row = s_reg + r * reg + c + R;
      float acc = w.gtap[0] * row[0];
      for (int m = 1; m <= R; ++m) acc += w.gtap[m] * (row[-m] + row[m]);
      s_mid[r * kTile + c] = acc;
    }
    __syncthreads();
    for (int k = tid; k < kTile * kTile; k += 256) {
      const int r = k / kTile, c = k - (k / kTile) * kTile;
      const float* col = s_mid + (r + R) * kTile + c;
      float acc = w.gtap[0] * col[0];
      for (int m = 1; m <= R; ++m) acc += w.gtap[m] * (col[-m * kTile] + col[m * kTile]);
      const int gx = x0 + c, gy = y0 + r;
      if (gx < nx && gy < ny) w.st[(size_t)gy * nx + gx] = acc;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// S4: repulsion from the central difference of the filtered density and the
// total node force.  Direct mode also spreads it with global atomics; sorted
// mode runs in slot order and stores the node records.
// ---------------------------------------------------------------------------
template <int PACK>
__global__ __launch_bounds__(PACK) void k_repulse(const WorldDev* __restrict__ W, Tables T) {
  const int npk = *T.n_packs;
  for (int it = blockIdx.x; it < npk; it += gridDim.x) {
    const Pack pk = T.packs[it];
    const WorldDev& w = W[pk.world];
    if (w.ctl_src->remaining <= 0) continue;
    const int sl = pk.node_begin + threadIdx.x;      // node index, or sorted slot
    if (sl >= pk.node_end) continue;
    const int gi = w.mode == kSorted ? w.perm[sl] : sl;
    const int N = w.n_part;
    const int nx = w.nx, ny = w.ny;
    const int bx = wrap_index(w.cell_in[gi], nx);
    const int by = wrap_index(w.cell_in[N + gi], ny);
    const float fx = w.frac_in[gi], fy = w.frac_in[N + gi];
    float wx[4], wy[4];
    peskin4(fx, wx);
    peskin4(fy, wy);
    int ix[6], iy[6];
#pragma unroll
    for (int a = 0; a < 6; ++a) {
      ix[a] = wrap_near(bx - 2 + a, nx);
      iy[a] = wrap_near(by - 2 + a, ny);
    }
    float gx = 0.f, gy = 0.f;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const float* rm = w.st + (size_t)iy[b] * nx;
      const float* r0 = w.st + (size_t)iy[b + 1] * nx;
      const float* rp = w.st + (size_t)iy[b + 2] * nx;
      float rx = 0.f, ry = 0.f;
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        rx += wx[a] * (r0[ix[a + 2]] - r0[ix[a]]);
        ry += wx[a] * (rp[ix[a + 1]] - rm[ix[a + 1]]);
      }
      gx += wy[b] * rx;
      gy += wy[b] * ry;
    }
    const float Fx = w.fel[gi] - 0.5f * w.k_rep * gx;
    const float Fy = w.fel[N + gi] - 0.5f * w.k_rep * gy;
    w.fel[gi] = Fx;
    w.fel[N + gi] = Fy;
    if (w.mode == kSorted) {
      w.rec[sl] = make_float4(fx, fy, Fx, Fy);
    } else if (w.mode == kDirect) {
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        float* row0 = w.Fg + (size_t)iy[b + 1] * nx;
        float* row1 = row0 + (size_t)nx * ny;
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          const float ww = wx[a] * wy[b];
          unsafeAtomicAdd(row0 + ix[a + 1], ww * Fx);
          unsafeAtomicAdd(row1 + ix[a + 1], ww * Fy);
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// S5 + S6: grid force of a 32x32 tile (LDS sums over the tile's bin, a
// fixed-order sorted gather, or the HBM accumulator), then the D2Q9
// two-relaxation-time collision with Guo forcing and push streaming.
// Populations are stored shifted (g = f - w_q) so FP32 resolves the small
// deviations from rest.  Writes u; sets the world flag on NaN or |u| > u_max.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_lbm(const WorldDev* __restrict__ W, Tables T) {
  __shared__ float s_fx[kTile * kTile];
  __shared__ float s_fy[kTile * kTile];
  const int nt = *T.n_tiles;
  const int tid = threadIdx.x;
  for (int it = blockIdx.x; it < nt; it += gridDim.x) {
    const int2 tl = T.tiles[it];
    const WorldDev& w = W[tl.x];
    const Ctl cs = *w.ctl_src;
    const bool live = cs.remaining > 0;
    if (tl.y == 0 && tid == 0) {
      Ctl cd = cs;
      if (live) { cd.t += 1; cd.remaining -= 1; }
      *w.ctl_dst = cd;
    }
    if (!live) continue;
    const int nx = w.nx, ny = w.ny;
    const int ncell = nx * ny;
    const int x0 = (tl.y % w.ntx) * kTile;
    const int y0 = (tl.y / w.ntx) * kTile;
    const int tw = min(kTile, nx - x0), th = min(kTile, ny - y0);
    if (w.mode == kBinned) {
      for (int k = tid; k < kTile * kTile; k += 256) {
        s_fx[k] = 0.f;
        s_fy[k] = 0.f;
      }
      __syncthreads();
      const int N = w.n_part;
      const int e1 = w.bin_start[tl.y + 1];
      for (int e = w.bin_start[tl.y] + tid; e < e1; e += 256) {
        const int i = w.bin_idx[e];
        const int bx = wrap_index(w.cell_in[i], nx);
        const int by = wrap_index(w.cell_in[N + i], ny);
        float wx[4], wy[4];
        peskin4(w.frac_in[i], wx);
        peskin4(w.frac_in[N + i], wy);
        const float Fx = w.fel[i], Fy = w.fel[N + i];
        int lx[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) lx[a] = wrap_near(bx - 1 + a, nx) - x0;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const int ly = wrap_near(by - 1 + b, ny) - y0;
          if (ly < 0 || ly >= th) continue;
#pragma unroll
          for (int a = 0; a < 4; ++a) {
            if (lx[a] < 0 || lx[a] >= tw) continue;
            const float ww = wx[a] * wy[b];
            atomicAdd(&s_fx[ly * kTile + lx[a]], ww * Fx);
            atomicAdd(&s_fy[ly * kTile + lx[a]], ww * Fy);
          }
        }
      }
      __syncthreads();
    }
    const float op = w.om_p, om = w.om_m;
    const float sp = 1.0f - 0.5f * op, sm = 1.0f - 0.5f * om;
    for (int k = 0; k < 4; ++k) {
      const int lx = tid & (kTile - 1);
      const int ly = (tid >> 5) + 8 * k;
      if (lx >= tw || ly >= th) continue;
      const int x = x0 + lx, y = y0 + ly;
      const int c = y * nx + x;
      float g[9];
#pragma unroll
      for (int q = 0; q < 9; ++q) g[q] = w.f_src[(size_t)q * ncell + c];
      float Fx, Fy;
      if (w.mode == kBinned) {
        Fx = s_fx[ly * kTile + lx];
        Fy = s_fy[ly * kTile + lx];
      } else if (w.mode == kSorted) {
        gather_force(w, x, y, Fx, Fy);
      } else {
        Fx = w.Fg[c];
        Fy = w.Fg[(size_t)ncell + c];
        w.Fg[c] = 0.f;
        w.Fg[(size_t)ncell + c] = 0.f;
        w.s[c] = 0.f;
      }
      // moments (the lattice weights have zero first moment, so the shift
      // does not change the momentum sum)
      const float drho = ((g[0] + g[1]) + (g[2] + g[3])) + ((g[4] + g[5]) + (g[6] + g[7])) + g[8];
      const float rho = 1.0f + drho;
      const float jx = (g[1] - g[3]) + (g[5] - g[6]) + (g[8] - g[7]);
      const float jy = (g[2] - g[4]) + (g[5] - g[8]) + (g[6] - g[7]);
      const float inv = 1.0f / rho;
      const float ux = (jx + 0.5f * Fx) * inv;
      const float uy = (jy + 0.5f * Fy) * inv;
      const float usq = ux * ux + uy * uy;
      w.u[c] = ux;
      w.u[(size_t)ncell + c] = uy;
      if (!(usq <= w.u_max2)) atomicOr(w.flags, 1u);

      // equilibrium minus weights: w_q (drho + rho (3 cu + 4.5 cu^2 - 1.5 u^2));
      // Guo source: w_q (3 (c - u) + 9 (c.u) c) . F; split into the parts
      // symmetric and antisymmetric under q <-> opposite(q)
      const float base = 1.5f * usq;
      const float uF = ux * Fx + uy * Fy;
      float out[9];
      {
        const float w0 = 4.0f / 9.0f;
        const float geq0 = w0 * (drho - rho * base);
        const float S0 = w0 * (-3.0f * uF);
        out[0] = g[0] - op * (g[0] - geq0) + sp * S0;
      }
#pragma unroll
      for (int pr = 0; pr < 4; ++pr) {
        const int q = pr < 2 ? 1 + pr : 5 + (pr - 2);
        const int qb = q + 2;
        const float wq = pr < 2 ? (1.0f / 9.0f) : (1.0f / 36.0f);
        const float cxq = (float)kCX[q], cyq = (float)kCY[q];
        const float cu = cxq * ux + cyq * uy;
        const float cF = cxq * Fx + cyq * Fy;
        const float eqp = wq * (drho + rho * (4.5f * cu * cu - base));
        const float eqm = wq * rho * 3.0f * cu;
        const float Sp = wq * (9.0f * cu * cF - 3.0f * uF);
        const float Sm = wq * 3.0f * cF;
        const float gp = 0.5f * (g[q] + g[qb]);
        const float gm = 0.5f * (g[q] - g[qb]);
        const float relp = -op * (gp - eqp) + sp * Sp;
        const float relm = -om * (gm - eqm) + sm * Sm;
        out[q] = g[q] + relp + relm;
        out[qb] = g[qb] + relp - relm;
      }
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        const int xn = wrap_near(x + kCX[q], nx);
        const int yn = wrap_near(y + kCY[q], ny);
        w.f_dst[(size_t)q * ncell + (size_t)yn * nx + xn] = out[q];
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// S7: gather the step's fluid velocity at each node and integrate
// (x <- x + sum_c W(c - x) u(c)), carrying the fraction into the cell.
// ---------------------------------------------------------------------------
template <int PACK>
__global__ __launch_bounds__(PACK) void k_integrate(const WorldDev* __restrict__ W, Tables T) {
  const int npk = *T.n_packs;
  for (int it = blockIdx.x; it < npk; it += gridDim.x) {
    const Pack pk = T.packs[it];
    const WorldDev& w = W[pk.world];
    if (w.ctl_src->remaining <= 0) continue;
    const int gi = pk.node_begin + threadIdx.x;
    if (gi >= pk.node_end) continue;
    const int N = w.n_part;
    const int nx = w.nx, ny = w.ny;
    const int cx = w.cell_in[gi], cy = w.cell_in[N + gi];
    const float fx = w.frac_in[gi], fy = w.frac_in[N + gi];
    const int bx = wrap_index(cx, nx), by = wrap_index(cy, ny);
    float wx[4], wy[4];
    peskin4(fx, wx);
    peskin4(fy, wy);
    int ix[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) ix[a] = wrap_near(bx - 1 + a, nx);
    const size_t nc = (size_t)nx * ny;
    float dux = 0.f, duy = 0.f;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const float* r0 = w.u + (size_t)wrap_near(by - 1 + b, ny) * nx;
      const float* r1 = r0 + nc;
      float ax = 0.f, ay = 0.f;
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        ax += wx[a] * r0[ix[a]];
        ay += wx[a] * r1[ix[a]];
      }
      dux += wy[b] * ax;
      duy += wy[b] * ay;
    }
    float nfx = fx + dux, nfy = fy + duy;
    const float flx = floorf(nfx), fly = floorf(nfy);
    int ncx = cx + (int)flx, ncy = cy + (int)fly;
    nfx -= flx;
    nfy -= fly;
    if (nfx >= 1.0f) { nfx = 0.0f; ncx += 1; }
    if (nfy >= 1.0f) { nfy = 0.0f; ncy += 1; }
    w.cell_out[gi] = ncx;
    w.cell_out[N + gi] = ncy;
    w.frac_out[gi] = nfx;
    w.frac_out[N + gi] = nfy;
  }
}

__global__ void k_set_ctl(Ctl* c, long long t, int remaining) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    Ctl v;
    v.t = t;
    v.remaining = remaining;
    v.pad = 0;
    *c = v;
  }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
#define MC_PACK_DISPATCH(KERNEL, G, ...)                                         \
  do {                                                                           \
    if ((G).pack == 256)                                                         \
      KERNEL<256><<<(G).node_blocks, 256, 0, s>>>(__VA_ARGS__);                  \
    else                                                                         \
      KERNEL<1024><<<(G).node_blocks, 1024, 0, s>>>(__VA_ARGS__);                \
  } while (0)

void launch_elastic(const WorldDev* W, const Tables& T, const Grid& G, hipStream_t s) {
  MC_PACK_DISPATCH(k_elastic, G, W, T);
}

void launch_sort(const WorldDev* W, const Tables& T, const Grid& G, hipStream_t s) {
  if (G.any_binned) {
    k_bin_scan<<<G.world_blocks, 256, 0, s>>>(W, T);
    MC_PACK_DISPATCH(k_bin_fill, G, W, T);
  }
  if (G.any_sorted) {
    k_scan_reduce<<<G.scan_blocks, 256, 0, s>>>(W, T);
    k_scan_partials<<<G.world_blocks, 256, 0, s>>>(W, T);
    k_scan_down<<<G.scan_blocks, 256, 0, s>>>(W, T);
    MC_PACK_DISPATCH(k_scatter, G, W, T);
    MC_PACK_DISPATCH(k_segsort, G, W, T);
  }
}

void launch_filter(const WorldDev* W, const Tables& T, const Grid& G, hipStream_t s) {
  k_filter<<<G.tile_blocks, 256, 0, s>>>(W, T);
}

void launch_repulse(const WorldDev* W, const Tables& T, const Grid& G, hipStream_t s) {
  MC_PACK_DISPATCH(k_repulse, G, W, T);
}

void launch_lbm(const WorldDev* W, const Tables& T, const Grid& G, hipStream_t s) {
  k_lbm<<<G.tile_blocks, 256, 0, s>>>(W, T);
}

void launch_integrate(const WorldDev* W, const Tables& T, const Grid& G, hipStream_t s) {
  MC_PACK_DISPATCH(k_integrate, G, W, T);
}

void launch_set_ctl(Ctl* c, long long t, int remaining, hipStream_t s) {
  k_set_ctl<<<1, 64, 0, s>>>(c, t, remaining);
}

}  // namespace mc
