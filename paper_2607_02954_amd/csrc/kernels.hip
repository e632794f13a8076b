// Forward kernels of the filament-fluid step for gfx950 (CDNA4).
//
// Step order (one launch per sub-step, all worlds of a table at once):
//   k_elastic   S0 actuation + S1 PBD Cosserat projection (Eqs. 1-4) -> node
//               force; S2 deposit of the node density onto the grid
//   k_filter    S3 separable circular Gaussian filter, LDS-tiled
//   k_repulse   S4 repulsion from the density gradient + S5 force spread
//   k_lbm       S6 D2Q9 TRT + Guo collision and push streaming; exports u;
//               clears the deposit and force accumulators for the next step
//   k_integrate S7 gather u at the nodes and move them
//
// Node kernels run one block per node pack (whole filaments, <= pack nodes,
// filament-contiguous SoA), so neighbour exchange along a chain stays in LDS.
// Positions are an integer cell plus a float fraction: every quantity the
// physics needs (edge vectors, kernel offsets) is then formed from small
// numbers, which keeps FP32 accurate on 2048^2 grids.
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

// D2Q9 lattice: velocity q has components (CX[q], CY[q]); pairs (q, q+2) for
// q = 1, 2 and (q, q+2) for q = 5, 6 are opposite.
__constant__ int kCX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__constant__ int kCY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

}  // namespace

// ---------------------------------------------------------------------------
// S0 + S1 + S2: actuation, PBD elastic force, density deposit (atomic) or
// home-cell key (sorted transfer).
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

    if (active) {
      w.fel[gi] = w.k_el * s_dx[li];
      w.fel[N + gi] = w.k_el * s_dy[li];
      const int bx = wrap_index(cx, w.nx);
      const int by = wrap_index(cy, w.ny);
      if (w.sorted) {
        const int key = by * w.nx + bx;
        w.key[gi] = key;
        w.rank[gi] = atomicAdd(&w.cnt[key], 1);
      } else {
        float wx[4], wy[4];
        peskin4(fx, wx);
        peskin4(fy, wy);
        int ix[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          int v = bx - 1 + a;
          ix[a] = v < 0 ? v + w.nx : (v >= w.nx ? v - w.nx : v);
        }
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          int iy = by - 1 + b;
          iy = iy < 0 ? iy + w.ny : (iy >= w.ny ? iy - w.ny : iy);
          float* row = w.s + (size_t)iy * w.nx;
#pragma unroll
          for (int a = 0; a < 4; ++a) unsafeAtomicAdd(row + ix[a], wx[a] * wy[b]);
        }
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// S3: separable circular Gaussian filter on a 64x16 output tile with an
// R-cell halo staged in LDS (x pass into LDS, then y pass to HBM).
// In sorted mode the deposit s is formed here, in the tile load, by gathering
// the node records of the sorted home-cell segments (no s array).
// ---------------------------------------------------------------------------
__device__ __forceinline__ float gather_density(const WorldDev& w, int gx, int gy) {
  // s(c) = sum over nodes with home cell h in [c-2, c+1]^2 of W(c - x)
  float acc = 0.f;
  for (int b = 0; b < 4; ++b) {
    const int hy = wrap_index(gy + 1 - b, w.ny);        // c - h_y = b - 1 in {-1,0,1,2}
    for (int a = 0; a < 4; ++a) {
      const int hx = wrap_index(gx + 1 - a, w.nx);
      const int h = hy * w.nx + hx;
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

__global__ __launch_bounds__(256) void k_filter(const WorldDev* __restrict__ W, Tables T) {
  __shared__ float s_in[(kTileY + 2 * kMaxRadius) * (kTileX + 2 * kMaxRadius)];
  __shared__ float s_mid[(kTileY + 2 * kMaxRadius) * kTileX];
  const int nt = *T.n_tiles;
  const int tid = threadIdx.x;
  for (int it = blockIdx.x; it < nt; it += gridDim.x) {
    const int2 tl = T.tiles[it];
    const WorldDev& w = W[tl.x];
    if (w.ctl_src->remaining <= 0) continue;
    const int R = w.radius;
    const int ntx = (w.nx + kTileX - 1) / kTileX;
    const int tx0 = (tl.y % ntx) * kTileX;
    const int ty0 = (tl.y / ntx) * kTileY;
    const int win = kTileX + 2 * R;
    const int hin = kTileY + 2 * R;
    for (int k = tid; k < win * hin; k += 256) {
      const int r = k / win, c = k - (k / win) * win;
      const int gx = wrap_index(tx0 - R + c, w.nx);
      const int gy = wrap_index(ty0 - R + r, w.ny);
      s_in[r * win + c] = w.sorted ? gather_density(w, gx, gy) : w.s[(size_t)gy * w.nx + gx];
    }
    __syncthreads();
    for (int k = tid; k < hin * kTileX; k += 256) {
      const int r = k / kTileX, c = k - (k / kTileX) * kTileX;
      const float* row = s_in + r * win + c + R;
      float acc = w.gtap[0] * row[0];
      for (int m = 1; m <= R; ++m) acc += w.gtap[m] * (row[-m] + row[m]);
      s_mid[r * kTileX + c] = acc;
    }
    __syncthreads();
    for (int k = tid; k < kTileY * kTileX; k += 256) {
      const int r = k / kTileX, c = k - (k / kTileX) * kTileX;
      const float* col = s_mid + (r + R) * kTileX + c;
      float acc = w.gtap[0] * col[0];
      for (int m = 1; m <= R; ++m) acc += w.gtap[m] * (col[-m * kTileX] + col[m * kTileX]);
      const int gx = tx0 + c, gy = ty0 + r;
      if (gx < w.nx && gy < w.ny) w.st[(size_t)gy * w.nx + gx] = acc;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// S4 + S5: repulsion from the central difference of the filtered density,
// total node force, and its spread onto the grid (atomic) or into the sorted
// node records (sorted transfer).
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
    const int gi = w.sorted ? w.perm[sl] : sl;
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
      int v = bx - 2 + a;
      ix[a] = v < 0 ? v + nx : (v >= nx ? v - nx : v);
      int u = by - 2 + a;
      iy[a] = u < 0 ? u + ny : (u >= ny ? u - ny : u);
    }
    float gx = 0.f, gy = 0.f;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const float* rm = w.st + (size_t)iy[b] * nx;       // row y-1 relative to support row
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
    if (w.sorted) {
      w.rec[sl] = make_float4(fx, fy, Fx, Fy);
    } else {
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
// S6: D2Q9 two-relaxation-time collision with Guo forcing and push streaming.
// Populations are stored shifted (g = f - w_q) so that FP32 resolves the small
// deviations from rest.  Reads and clears the force accumulator (and the
// deposit accumulator) and writes u; sets the world flag on NaN or |u| > u_max.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void gather_force(const WorldDev& w, int gx, int gy, float& Fx, float& Fy) {
  Fx = 0.f;
  Fy = 0.f;
  for (int b = 0; b < 4; ++b) {
    const int hy = wrap_index(gy + 1 - b, w.ny);
    for (int a = 0; a < 4; ++a) {
      const int hx = wrap_index(gx + 1 - a, w.nx);
      const int h = hy * w.nx + hx;
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

__global__ __launch_bounds__(256) void k_lbm(const WorldDev* __restrict__ W, Tables T) {
  const int nit = *T.n_items;
  for (int it = blockIdx.x; it < nit; it += gridDim.x) {
    const int2 item = T.items[it];
    const WorldDev& w = W[item.x];
    const Ctl cs = *w.ctl_src;
    const bool live = cs.remaining > 0;
    if (item.y == 0 && threadIdx.x == 0) {
      Ctl cd = cs;
      if (live) { cd.t += 1; cd.remaining -= 1; }
      *w.ctl_dst = cd;
    }
    if (!live) continue;
    const int nx = w.nx, ny = w.ny;
    const int ncell = nx * ny;
    const int c = item.y + threadIdx.x;
    if (c >= ncell) continue;
    const int y = c / nx;
    const int x = c - y * nx;

    float g[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) g[q] = w.f_src[(size_t)q * ncell + c];
    float Fx, Fy;
    if (w.sorted) {
      gather_force(w, x, y, Fx, Fy);
    } else {
      Fx = w.Fg[c];
      Fy = w.Fg[(size_t)ncell + c];
      w.Fg[c] = 0.f;
      w.Fg[(size_t)ncell + c] = 0.f;
      w.s[c] = 0.f;
    }
    // moments (the lattice weights have zero first moment, so shifting does
    // not change the momentum sum)
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

    const float op = w.om_p, om = w.om_m;
    const float sp = 1.0f - 0.5f * op, sm = 1.0f - 0.5f * om;
    const float base = 1.5f * usq;
    // equilibrium minus weights: w_q (drho + rho (3 cu + 4.5 cu^2 - 1.5 u^2))
    // Guo source: w_q (3 (c - u) + 9 (c.u) c) . F
    const float uF = ux * Fx + uy * Fy;
    float out[9];
    {
      const float w0 = 4.0f / 9.0f;
      const float geq0 = w0 * (drho - rho * base);
      const float S0 = w0 * (-3.0f * uF);
      out[0] = g[0] - op * (g[0] - geq0) + sp * S0;
    }
    // pairs (q, qb): (1,3), (2,4), (5,7), (6,8)
#pragma unroll
    for (int pr = 0; pr < 4; ++pr) {
      const int q = pr < 2 ? 1 + pr : 5 + (pr - 2);
      const int qb = q + 2;
      const float wq = pr < 2 ? (1.0f / 9.0f) : (1.0f / 36.0f);
      const float cxq = (float)kCX[q], cyq = (float)kCY[q];
      const float cu = cxq * ux + cyq * uy;
      const float cF = cxq * Fx + cyq * Fy;
      // symmetric / antisymmetric parts over (q, qb): cu -> -cu, cF -> -cF
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
      int xn = x + kCX[q];
      xn = xn < 0 ? xn + nx : (xn >= nx ? xn - nx : xn);
      int yn = y + kCY[q];
      yn = yn < 0 ? yn + ny : (yn >= ny ? yn - ny : yn);
      w.f_dst[(size_t)q * ncell + (size_t)yn * nx + xn] = out[q];
    }
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
    for (int a = 0; a < 4; ++a) {
      int v = bx - 1 + a;
      ix[a] = v < 0 ? v + nx : (v >= nx ? v - nx : v);
    }
    const size_t nc = (size_t)nx * ny;
    float dux = 0.f, duy = 0.f;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      int iy = by - 1 + b;
      iy = iy < 0 ? iy + ny : (iy >= ny ? iy - ny : iy);
      const float* r0 = w.u + (size_t)iy * nx;
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

// ---------------------------------------------------------------------------
// Sorted-segment transfer: exclusive scan of the per-cell counts (three
// phases over (world, 1024-cell block) items), then scatter of node indices
// into their slots and an insertion sort of every multi-node segment by node
// index, so that all later sums run in a fixed order.
// ---------------------------------------------------------------------------
constexpr int kScanBlock = 1024;   // cells per scan item (256 threads x 4)

__device__ __forceinline__ int block_exclusive_scan256(int v, int* s_tmp, int& total) {
  // Hillis-Steele inclusive scan over 256 threads in LDS.
  const int tid = threadIdx.x;
  s_tmp[tid] = v;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const int add = tid >= off ? s_tmp[tid - off] : 0;
    __syncthreads();
    s_tmp[tid] += add;
    __syncthreads();
  }
  total = s_tmp[255];
  const int incl = s_tmp[tid];
  __syncthreads();
  return incl - v;
}

__global__ __launch_bounds__(256) void k_scan_reduce(const WorldDev* __restrict__ W, Tables T) {
  __shared__ int s_tmp[256];
  const int n = *T.n_scan;
  for (int it = blockIdx.x; it < n; it += gridDim.x) {
    const int2 sc = T.scan[it];
    const WorldDev& w = W[sc.x];
    if (!w.sorted || w.ctl_src->remaining <= 0) continue;
    const int ncell = w.nx * w.ny;
    const int c0 = sc.y * kScanBlock + threadIdx.x * 4;
    int v = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) v += (c0 + k < ncell) ? w.cnt[c0 + k] : 0;
    int total;
    block_exclusive_scan256(v, s_tmp, total);
    if (threadIdx.x == 0) w.part[sc.y] = total;
  }
}

__global__ __launch_bounds__(256) void k_scan_partials(const WorldDev* __restrict__ W, Tables T) {
  // one block per world whose scan item index is 0: exclusive scan of partials
  __shared__ int s_tmp[256];
  const int n = *T.n_scan;
  for (int it = blockIdx.x; it < n; it += gridDim.x) {
    const int2 sc = T.scan[it];
    if (sc.y != 0) continue;
    const WorldDev& w = W[sc.x];
    if (!w.sorted || w.ctl_src->remaining <= 0) continue;
    const int ncell = w.nx * w.ny;
    const int nb = (ncell + kScanBlock - 1) / kScanBlock;
    int carry = 0;
    for (int b0 = 0; b0 < nb; b0 += 256) {
      const int b = b0 + threadIdx.x;
      const int v = b < nb ? w.part[b] : 0;
      int total;
      const int ex = block_exclusive_scan256(v, s_tmp, total);
      if (b < nb) w.part[b] = carry + ex;
      carry += total;
    }
    if (threadIdx.x == 0) w.start[ncell] = carry;
  }
}

__global__ __launch_bounds__(256) void k_scan_down(const WorldDev* __restrict__ W, Tables T) {
  __shared__ int s_tmp[256];
  const int n = *T.n_scan;
  for (int it = blockIdx.x; it < n; it += gridDim.x) {
    const int2 sc = T.scan[it];
    const WorldDev& w = W[sc.x];
    if (!w.sorted || w.ctl_src->remaining <= 0) continue;
    const int ncell = w.nx * w.ny;
    const int c0 = sc.y * kScanBlock + threadIdx.x * 4;
    int v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = (c0 + k < ncell) ? w.cnt[c0 + k] : 0;
    int total;
    const int ex = block_exclusive_scan256(v[0] + v[1] + v[2] + v[3], s_tmp, total);
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
    if (!w.sorted || w.ctl_src->remaining <= 0) continue;
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
    if (!w.sorted || w.ctl_src->remaining <= 0) continue;
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

void launch_sort(const WorldDev* W, const Tables& T, const Grid& G, hipStream_t s, bool any_sorted) {
  if (!any_sorted) return;
  k_scan_reduce<<<G.scan_blocks, 256, 0, s>>>(W, T);
  k_scan_partials<<<G.scan_blocks, 256, 0, s>>>(W, T);
  k_scan_down<<<G.scan_blocks, 256, 0, s>>>(W, T);
  MC_PACK_DISPATCH(k_scatter, G, W, T);
  MC_PACK_DISPATCH(k_segsort, G, W, T);
}

void launch_filter(const WorldDev* W, const Tables& T, const Grid& G, hipStream_t s) {
  k_filter<<<G.tile_blocks, 256, 0, s>>>(W, T);
}

void launch_repulse(const WorldDev* W, const Tables& T, const Grid& G, hipStream_t s) {
  MC_PACK_DISPATCH(k_repulse, G, W, T);
}

void launch_lbm(const WorldDev* W, const Tables& T, const Grid& G, hipStream_t s) {
  k_lbm<<<G.cell_blocks, 256, 0, s>>>(W, T);
}

void launch_integrate(const WorldDev* W, const Tables& T, const Grid& G, hipStream_t s) {
  MC_PACK_DISPATCH(k_integrate, G, W, T);
}

void launch_set_ctl(Ctl* c, long long t, int remaining, hipStream_t s) {
  k_set_ctl<<<1, 64, 0, s>>>(c, t, remaining);
}

}  // namespace mc
