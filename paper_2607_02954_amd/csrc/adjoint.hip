// Reverse mode of one filament-fluid step (hand-written adjoint kernels).
//
// The paper differentiates end to end through the PBD solver and the fluid
// (Methods; Experiments, Filament Folding).  Given dL/dx_{t+1} and
// dL/dg_{t+1}, one reversed step produces dL/dx_t, dL/dg_t and accumulates
// dL/d(rest angle), visiting the forward sub-steps backwards:
//   k_adj_spread  S7 (operand 0): u~ = spread(dL/dx_{t+1})     (tile, LDS)
//   k_adj_lbm     S6: streaming^T (pull) and the collision Jacobian^T per
//                     cell -> dL/dg_t, dL/dF_grid
//   (MDF)         S5 with multi-direct forcing: the iterates recomputed,
//                     then reversed iteration by iteration (k_adj_mdf_*)
//   k_adj_force   S5, S4, S7: dL/dF_i = gather(dL/dF_grid); the derivative
//                     terms of the three node gathers/spreads w.r.t. x_t
//                     (at the two-layer markers where a world has them)
//   k_adj_markers two layers: dL/dd through each node's normal to the
//                     neighbours that define it
//   k_adj_spread  S4 (operand 1): dL/dG = -k_rep spread(dL/dF) (tile, LDS)
//   k_adj_filter  S3: dL/ds = G (D^T dL/dG): the central difference and the
//                     symmetric Gaussian transposed                (tile, LDS)
//   k_adj_pbd     S2, S1, S0: the deposit derivative, then the PBD iterations
//                     reversed pass by pass (forward states recomputed and
//                     kept in registers; chains, closed loops, branches),
//                     atan2 of the initial edge angles and the actuation ->
//                     dL/dx_t and dL/d(rest angle)
// Every forward field the adjoint needs (x_t, g_t, G_t, F_t, F_grid, u_t, the
// tile bins of x_t and the filter's spread lists) is taken from the tape
// written by the recomputed forward step; the descriptor passed in points at
// that tape slot.
#include "device_util.h"

namespace mc {

constexpr int kMaxAdjIters = 8;   // most PBD iterations the adjoint keeps in registers

static __device__ __forceinline__ const AdjDev& adj_of(const AdjArg& a, int world) {
  return a.arr ? a.arr[world] : a.one;
}

// ---------------------------------------------------------------------------
// Node -> grid spreads of adjoint node vectors (u~ and G~), tile-binned.
// ---------------------------------------------------------------------------
// out = add + scale S[v], the operands chosen by `which`: 0 u~ = S[x~'],
// 1 G~ = -k_rep S[F~], 2 the MDF iterate F_grid_1 = S[F], 3 the iterate
// F_grid_{k+1} = F_grid_k + S[c_k], 4 the test hook's vector and grid.
template <int TILE>
__global__ __launch_bounds__(TileCfg<TILE>::kThreads) void k_adj_spread(const WorldDev* __restrict__ W, Tables T,
                                                                         AdjArg AA, int which, int k) {
  using C = TileCfg<TILE>;
  constexpr int kThreads = C::kThreads, kSpreadCells = C::kSpreadCells;
  __shared__ __align__(16) long long s_x[kSpreadCells];
  __shared__ __align__(16) long long s_y[kSpreadCells];
  __shared__ vi4 s_list[(kThreads / 64) * kWaveList];
  const int nt = n_tiles<TILE>(T);
  const XcdLoop tiles(nt);
  for (int it = tiles.first; it < tiles.end; it += tiles.step) {
    const int2 tl = tile_entry<TILE>(T, it);
    const WorldDev& w = W[tl.x];
    const AdjDev& A = adj_of(AA, tl.x);
    const int nx = w.nx, ny = w.ny;
    const size_t ncell = (size_t)nx * ny;
    const int x0 = tile_x(tl.y) * TILE;
    const int y0 = tile_y(tl.y) * TILE;
    const int tw = min(TILE, nx - x0), th = min(TILE, ny - y0);
    const float* v = A.dbg_v;
    float scale = 1.0f;
    const float2* add = nullptr;
    float2* out = A.dbg_out;
    if (which == 0) {
      v = A.xbar_in;
      out = A.ubar;
    } else if (which == 1) {
      v = A.Fbar;
      scale = -w.k_rep;
      out = A.Gbar;
    } else if (which == 2) {
      v = A.F;
      out = A.Fgk;
    } else if (which == 3) {
      v = A.mc;
      add = A.Fgk + (size_t)(k - 1) * ncell;
      out = A.Fgk + (size_t)k * ncell;
    }
    zero_lds_u64(s_x, kSpreadCells);
    zero_lds_u64(s_y, kSpreadCells);
    __syncthreads();
    // the step's spread list (written by the recomputed filter into the
    // tape), or the bins if it overflowed (and for the test hook, which runs
    // on a world's own buffers)
    const int tix = tile_y(tl.y) * w.ntx + tile_x(tl.y);
    const int cnt = which != 4 ? glb(w.sp_cnt)[tix] : -1;
    BinFetch lf;
    lf.n = 1;
    lf.b0 = tix * C::kSpreadCap;
    lf.len = __lane_id() == 0 ? cnt : 0;
    const bool list = cnt >= 0 && cnt <= C::kSpreadCap;
    const MC_GLOBAL vi4* lrec = glbv<const vi4>(w.sp_rec);
    const MC_GLOBAL vi4* brec = glbv<const vi4>(w.bin_rec);
    // the transfers of the node<->grid coupling act through two-layer
    // markers where a world has them; the repulsion (G~) stays at the node
    if (w.d_marker && which != 1 && which != 4) {
      if (list)
        tile_spread_markers<TILE, false, true>(w, x0, y0, tw, th, glb(v), scale, s_x, s_y, s_list, lrec, lf, nullptr);
      else
        tile_spread_markers<TILE, false>(w, x0, y0, tw, th, glb(v), scale, s_x, s_y, s_list, brec,
                                         spread_fetch<TILE>(w, x0, y0), nullptr);
    } else if (list && !w.d_marker) {
      tile_spread_vec<TILE, false, true>(w, x0, y0, tw, th, glb(v), scale, s_x, s_y, s_list, lrec, lf, nullptr);
    } else if (list) {                 // a two-layer world's list also holds nodes one cell further out
      tile_spread_vec<TILE, false>(w, x0, y0, tw, th, glb(v), scale, s_x, s_y, s_list, lrec, lf, nullptr);
    } else {
      tile_spread_vec<TILE, false>(w, x0, y0, tw, th, glb(v), scale, s_x, s_y, s_list, brec,
                                   spread_fetch<TILE>(w, x0, y0), nullptr);
    }
    __syncthreads();
    MC_GLOBAL vf2* o = glbv<vf2>(out);
    for (int k = threadIdx.x; k < TILE * TILE; k += kThreads) {
      const int ly = k >> C::kShift, lx = k & (TILE - 1);
      if (lx >= tw || ly >= th) continue;
      const size_t c = (size_t)(y0 + ly) * nx + x0 + lx;
      vf2 val = {0.f, 0.f};
      if (add) val = glbv<const vf2>(add)[c];
      val.x += fix_to_float(spread_cell<TILE>(s_x, lx, ly, nx, ny));
      val.y += fix_to_float(spread_cell<TILE>(s_y, lx, ly, nx, ny));
      o[c] = val;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// S6 reversed: pull-streaming transpose and the TRT/Guo collision Jacobian
// transposed, per cell.  Reads g_t, F_grid_t (tape) and u~ (from k_adj_u).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_adj_lbm(const WorldDev* __restrict__ W, Tables T, AdjArg AA) {
  // (items in XCD-contiguous order, as in the forward fluid kernel; the
  // populations and their adjoint are touched once per reversed step, so
  // their loads and stores bypass the caches' allocation)
  const XcdLoop items(*T.n_items);
  for (int it = items.first; it < items.end; it += items.step) {
    const int2 item = T.items[it];
    const WorldDev& w = W[item.x];
    const AdjDev& A = adj_of(AA, item.x);
    const int nx = w.nx, ny = w.ny;
    const int ncell = nx * ny;
    const int c = item.y + threadIdx.x;
    if (c >= ncell) continue;
    const int y = c / nx;
    const int x = c - y * nx;
    const MC_GLOBAL float* src = glb(w.f_src);
    const MC_GLOBAL float* gin = glb(A.gbar_in);
    float g[9], gs[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      g[q] = __builtin_nontemporal_load((const float*)(src + (size_t)q * ncell + c));
      const int xn = wrap_near(x + kCX[q], nx);
      const int yn = wrap_near(y + kCY[q], ny);
      gs[q] = __builtin_nontemporal_load((const float*)(gin + (size_t)q * ncell + (size_t)yn * nx + xn));   // dL/dg*_q(c)
    }
    const vf2 F = glbv<const vf2>(w.Fg)[c];
    const vf2 ubv = glbv<const vf2>(A.ubar)[c];
    // forward moments
    const float drho = ((g[0] + g[1]) + (g[2] + g[3])) + ((g[4] + g[5]) + (g[6] + g[7])) + g[8];
    const float rho = 1.0f + drho;
    const float jx = (g[1] - g[3]) + (g[5] - g[6]) + (g[8] - g[7]);
    const float jy = (g[2] - g[4]) + (g[5] - g[8]) + (g[6] - g[7]);
    const float inv = 1.0f / rho;
    const float ux = (jx + 0.5f * F.x) * inv;
    const float uy = (jy + 0.5f * F.y) * inv;
    const float usq = ux * ux + uy * uy;
    const float op = w.om_p, om = w.om_m;
    const float ap = 1.0f - 0.5f * op, am = 1.0f - 0.5f * om;
    // g* = g - op P+ (g - geq) - om P- (g - geq) + ap P+ S + am P- S, with
    // self-adjoint projectors P+- onto the parts (anti)symmetric under
    // q <-> opposite(q)
    float gdir[9], geqb[9], Sb[9];
    gdir[0] = gs[0] - op * gs[0];
    geqb[0] = op * gs[0];
    Sb[0] = ap * gs[0];
#pragma unroll
    for (int pr = 0; pr < 4; ++pr) {
      const int q = pr < 2 ? 1 + pr : 5 + (pr - 2);
      const int qb = q + 2;
      const float sp = 0.5f * (gs[q] + gs[qb]);
      const float sm = 0.5f * (gs[q] - gs[qb]);
      gdir[q] = gs[q] - op * sp - om * sm;
      gdir[qb] = gs[qb] - op * sp + om * sm;
      geqb[q] = op * sp + om * sm;
      geqb[qb] = op * sp - om * sm;
      Sb[q] = ap * sp + am * sm;
      Sb[qb] = ap * sp - am * sm;
    }
    // geq_q = w_q (drho + rho (3 cu + 4.5 cu^2 - 1.5 u^2)),
    // S_q = w_q (3 c.F - 3 u.F + 9 (c.u)(c.F))
    float ubx = ubv.x, uby = ubv.y, drb = 0.f, Fbx = 0.f, Fby = 0.f;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      const float wq = q == 0 ? (4.0f / 9.0f) : (q < 5 ? (1.0f / 9.0f) : (1.0f / 36.0f));
      const float cxq = (float)kCX[q], cyq = (float)kCY[q];
      const float cu = cxq * ux + cyq * uy;
      const float cF = cxq * F.x + cyq * F.y;
      const float e = geqb[q] * wq;
      drb += e * (1.0f + 3.0f * cu + 4.5f * cu * cu - 1.5f * usq);
      const float er = e * rho;
      ubx += er * (3.0f * cxq + 9.0f * cu * cxq - 3.0f * ux);
      uby += er * (3.0f * cyq + 9.0f * cu * cyq - 3.0f * uy);
      const float sb = Sb[q] * wq;
      ubx += sb * (-3.0f * F.x + 9.0f * cF * cxq);
      uby += sb * (-3.0f * F.y + 9.0f * cF * cyq);
      Fbx += sb * (3.0f * cxq - 3.0f * ux + 9.0f * cu * cxq);
      Fby += sb * (3.0f * cyq - 3.0f * uy + 9.0f * cu * cyq);
    }
    // u = (j + F/2) / rho
    Fbx += 0.5f * ubx * inv;
    Fby += 0.5f * uby * inv;
    const float jbx = ubx * inv, jby = uby * inv;
    drb -= (ubx * ux + uby * uy) * inv;
    MC_GLOBAL float* gout = glb(A.gbar);
#pragma unroll
    for (int q = 0; q < 9; ++q)
      __builtin_nontemporal_store(gdir[q] + drb + (float)kCX[q] * jbx + (float)kCY[q] * jby,
                                  (float*)(gout + (size_t)q * ncell + c));
    const vf2 fb = {Fbx, Fby};
    glbv<vf2>(A.Fgbar)[c] = fb;
  }
}

// ---------------------------------------------------------------------------
// S5/S4/S7 node terms: dL/dF_i = sum_c W(c - x_i) dL/dF_grid(c), and the
// derivative of the three node<->grid transfers with respect to x_t.  In a
// two-layer world the force spread and the velocity gather act through the
// markers X = x +- d (half weight each): dL/dF_i and both transfers' position
// terms are formed per marker; their sum goes to dL/dx_i and their
// difference (dL/dd) to A.dbar, which k_adj_markers carries through the
// normal d(x_prev, x_next).  The repulsion gather stays at the node.
// ---------------------------------------------------------------------------
template <int TILE, bool MK>
__global__ __launch_bounds__(TileCfg<TILE>::kThreads) void k_adj_force(const WorldDev* __restrict__ W, Tables T,
                                                                        AdjArg AA) {
  // per tile: u, dL/dF_grid and the density gradient staged over the cells
  // the supports of the tile's own nodes (and of their markers: MK) reach,
  // then one thread per node of the tile's bin
  constexpr int kE = MK ? 1 : 0;
  constexpr int kStage = TILE + 3 + 2 * kE, kThreads = TileCfg<TILE>::kThreads, kCells = kStage * kStage;
  __shared__ vf2 s_u[kCells];
  __shared__ vf2 s_fb[kCells];
  __shared__ vf2 s_g[kCells];
  const int nt = n_tiles<TILE>(T);
  const XcdLoop tiles(nt);
  for (int it = tiles.first; it < tiles.end; it += tiles.step) {
    const int2 tl = tile_entry<TILE>(T, it);
    const WorldDev& w = W[tl.x];
    if (MK != (w.d_marker != nullptr)) continue;
    const AdjDev& A = adj_of(AA, tl.x);
    const int N = w.n_part, nx = w.nx, ny = w.ny;
    const int x0 = tile_x(tl.y) * TILE, y0 = tile_y(tl.y) * TILE;
    const MC_GLOBAL vf2* u = glbv<const vf2>(w.u);
    const MC_GLOBAL vf2* Fgb = glbv<const vf2>(A.Fgbar);
    const MC_GLOBAL vf2* Gr = glbv<const vf2>(w.grad);
    {
      constexpr int kIt = (kCells + kThreads - 1) / kThreads;
      vf2 vu[kIt], vf[kIt], vg[kIt];
#pragma unroll
      for (int i = 0; i < kIt; ++i) {          // every load in flight before the stores
        const int k = min((int)threadIdx.x + kThreads * i, kCells - 1);
        const int r = k / kStage, c = k - (k / kStage) * kStage;
        const size_t idx = (size_t)wrap_index(y0 - 1 - kE + r, ny) * nx + wrap_index(x0 - 1 - kE + c, nx);
        vu[i] = u[idx];
        vf[i] = Fgb[idx];
        vg[i] = Gr[idx];
      }
#pragma unroll
      for (int i = 0; i < kIt; ++i) {
        const int k = (int)threadIdx.x + kThreads * i;
        if (k < kCells) {
          s_u[k] = vu[i];
          s_fb[k] = vf[i];
          s_g[k] = vg[i];
        }
      }
    }
    __syncthreads();
    const int tile = tile_y(tl.y) * w.ntx + tile_x(tl.y);
    const int e0 = glb(w.bin_start)[tile], e1 = glb(w.bin_start)[tile + 1];
    const MC_GLOBAL vi4* recs = glbv<const vi4>(w.bin_rec);
    for (int e = e0 + (int)threadIdx.x; e < e1; e += kThreads) {
      const vi4 rec = recs[e];
      const int lx = (rec.x & 0xffff) - x0, ly = (rec.x >> 16) - y0;   // home cell in the tile
      const int gi = rec.w;
      const float nfx = __int_as_float(rec.y), nfy = __int_as_float(rec.z);
      float wx[4], dwx[4], wy[4], dwy[4];
      peskin4_d(nfx, wx, dwx);
      peskin4_d(nfy, wy, dwy);
      const float xbx = A.xbar_in[gi], xby = A.xbar_in[N + gi];
      const float Fx = w.fel[gi], Fy = w.fel[N + gi];
      float fbx = 0.f, fby = 0.f;       // dL/dF_i
      float sux = 0.f, suy = 0.f;       // d/dx of  sum_c W (u_c . xbar')
      float sfx = 0.f, sfy = 0.f;       // d/dx of  sum_c W (F_i . Fgbar_c)
      if constexpr (!MK) {
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
          for (int a = 0; a < 4; ++a) {
            const int q = (ly + b) * kStage + lx + a;
            const vf2 uc = s_u[q];
            const vf2 fc = s_fb[q];
            const float W0 = wx[a] * wy[b], Wx = dwx[a] * wy[b], Wy = wx[a] * dwy[b];
            fbx += W0 * fc.x;
            fby += W0 * fc.y;
            const float pu = uc.x * xbx + uc.y * xby;
            sux += Wx * pu;
            suy += Wy * pu;
            const float pf = Fx * fc.x + Fy * fc.y;
            sfx += Wx * pf;
            sfy += Wy * pf;
          }
      } else {                          // two layers: the transfer terms at the markers
        const float ddx = glb(w.d_marker)[gi], ddy = glb(w.d_marker)[N + gi];
        float dbx = 0.f, dby = 0.f;
#pragma unroll
        for (int l = 0; l < 2; ++l) {
          const float sg = l == 0 ? 1.f : -1.f;
          int shx, shy;
          float mfx, mfy;
          marker_shift(nfx, sg * ddx, &shx, &mfx);
          marker_shift(nfy, sg * ddy, &shy, &mfy);
          float mwx[4], mdwx[4], mwy[4], mdwy[4];
          peskin4_d(mfx, mwx, mdwx);
          peskin4_d(mfy, mwy, mdwy);
          float px = 0.f, py = 0.f;
#pragma unroll
          for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int a = 0; a < 4; ++a) {
              const int q = (ly + shy + 1 + b) * kStage + lx + shx + 1 + a;
              const vf2 uc = s_u[q];
              const vf2 fc = s_fb[q];
              const float W0 = 0.5f * mwx[a] * mwy[b], Wx = 0.5f * mdwx[a] * mwy[b], Wy = 0.5f * mwx[a] * mdwy[b];
              fbx += W0 * fc.x;
              fby += W0 * fc.y;
              const float pp = (uc.x * xbx + uc.y * xby) + (Fx * fc.x + Fy * fc.y);
              px += Wx * pp;
              py += Wy * pp;
            }
          sux += px;                    // dL/dX of each marker moves the node ...
          suy += py;
          dbx += sg * px;               // ... and, with its sign, the displacement
          dby += sg * py;
        }
        A.dbar[gi] = dbx;
        A.dbar[N + gi] = dby;
      }
      float mx = 0.f, my = 0.f;
      if (A.mdf > 1) {                  // U_d = I[j / rho] + F / 2, and the MDF transfers' position terms
        fbx += 0.5f * A.Udbar[gi];
        fby += 0.5f * A.Udbar[N + gi];
        mx = A.xbar_m[gi];
        my = A.xbar_m[N + gi];
      }
      // repulsion F_rep = -k sum_c W G_c : d/dx of (-k sum_c W (G_c . Fbar))
      // (the gradient read from the staged window again: fewer registers)
      float srx = 0.f, sry = 0.f;
#pragma unroll
      for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          const vf2 gc = s_g[(ly + kE + b) * kStage + lx + kE + a];
          const float pg = gc.x * fbx + gc.y * fby;
          srx += dwx[a] * wy[b] * pg;
          sry += wx[a] * dwy[b] * pg;
        }
      const float kr = w.k_rep;
      A.Fbar[gi] = fbx;
      A.Fbar[N + gi] = fby;
      A.xbar[gi] = xbx + sux + sfx - kr * srx + mx;
      A.xbar[N + gi] = xby + suy + sfy - kr * sry + my;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Two-layer markers reversed: d_i = delta n_i with n_i the unit normal
// (-t_y, t_x) / |t| of the tangent t = x_b - x_a (a, b: the node's
// neighbours, or the node itself at a chain end; as in k_markers).  From
// dL/dd (A.dbar, plus the MDF transfers' A.dbar_m): dL/dt = (delta / |t|)
// (I - t^ t^T) (dd~_y, -dd~_x), added to dL/dx_b and subtracted from
// dL/dx_a.  Each node gathers the terms of the nodes whose tangent it ends
// or starts, in a fixed order.
// ---------------------------------------------------------------------------
template <int PACK>
__global__ __launch_bounds__(PACK) void k_adj_markers(const WorldDev* __restrict__ W, Tables T, AdjArg AA) {
  __shared__ int s_off[PACK + 1];
  __shared__ vf2 s_tb[PACK];
  const int npk = *T.n_packs;
  const int li = threadIdx.x;
  for (int it = blockIdx.x; it < npk; it += gridDim.x) {
    const Pack pk = T.packs[it];
    const WorldDev& w = W[pk.world];
    if (!w.d_marker) continue;                                  // block-uniform
    const AdjDev& A = adj_of(AA, pk.world);
    const int nf = pk.fil_end - pk.fil_begin;
    for (int k = li; k <= nf; k += PACK) s_off[k] = glb(w.fil_offset)[pk.fil_begin + k] - pk.node_begin;
    __syncthreads();
    const int gi = pk.node_begin + li;
    const bool live = gi < pk.node_end;
    int o = 0, n = 1, k = 0;
    bool ring = false;
    if (live) {
      int lo = 0, hi = nf - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_off[mid] <= li) lo = mid; else hi = mid - 1;
      }
      o = s_off[lo];
      n = s_off[lo + 1] - o;
      k = li - o;
      ring = w.fil_flags && (glb(w.fil_flags)[pk.fil_begin + lo] & 1) && n >= 3;
      const int first = pk.node_begin + o;
      int a = gi, b = gi;
      if (k > 0) a = gi - 1; else if (ring) a = first + n - 1;
      if (k < n - 1) b = gi + 1; else if (ring) b = first;
      const int N = w.n_part;
      const MC_GLOBAL int* cell = glb(w.cell_in);
      const MC_GLOBAL float* frac = glb(w.frac_in);
      const float tx = (float)(cell[b] - cell[a]) + (frac[b] - frac[a]);
      const float ty = (float)(cell[N + b] - cell[N + a]) + (frac[N + b] - frac[N + a]);
      const float len = sqrtf(tx * tx + ty * ty);
      float dbx = A.dbar[gi], dby = A.dbar[N + gi];
      if (A.mdf > 1) {
        dbx += A.dbar_m[gi];
        dby += A.dbar_m[N + gi];
      }
      vf2 tb = {0.f, 0.f};
      if (len > 0.f) {
        const float inv = 1.0f / len, hx = tx * inv, hy = ty * inv;
        const float vx = dby, vy = -dbx;
        const float dot = hx * vx + hy * vy;
        const float sc = w.marker_offset * inv;
        tb.x = sc * (vx - hx * dot);
        tb.y = sc * (vy - hy * dot);
      }
      s_tb[li] = tb;
    }
    __syncthreads();
    if (live) {
      // + the tangent ending here (the previous node's, or this chain end's
      // own), - the tangent starting here (the next node's, or this chain
      // start's own)
      const int last = o + n - 1;
      float ax = 0.f, ay = 0.f;
      if (k > 0 || ring) {
        const int p = k > 0 ? li - 1 : last;
        ax += s_tb[p].x;
        ay += s_tb[p].y;
      }
      if (k == n - 1 && !ring) {
        ax += s_tb[li].x;
        ay += s_tb[li].y;
      }
      if (k < n - 1 || ring) {
        const int q = k < n - 1 ? li + 1 : o;
        ax -= s_tb[q].x;
        ay -= s_tb[q].y;
      }
      if (k == 0 && !ring) {
        ax -= s_tb[li].x;
        ay -= s_tb[li].y;
      }
      const int N = w.n_part;
      A.xbar[gi] += ax;
      A.xbar[N + gi] += ay;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// S3 reversed: dL/ds = G (D^T dL/dG) on a tile.  dL/dG is staged with an
// (R+1)-cell halo; D^T maps it to an R-cell halo; the symmetric Gaussian
// then runs as in the forward filter.
// ---------------------------------------------------------------------------
template <int TILE>
__global__ __launch_bounds__(TileCfg<TILE>::kThreads) void k_adj_filter(const WorldDev* __restrict__ W, Tables T,
                                                                         AdjArg AA) {
  constexpr int kTile = TILE, kThreads = TileCfg<TILE>::kThreads;
  constexpr int kAdjRing = kTile + 2;
  constexpr int kAdjRegion = kAdjRing + 2 * kMaxRadius;
  constexpr int kAdjInner = kTile + 2 * kMaxRadius;
  __shared__ float s_gx[kAdjRegion * kAdjRegion];
  __shared__ float s_gy[kAdjRegion * kAdjRegion];
  __shared__ float s_in[kAdjInner * kAdjInner];
  __shared__ float s_mid[kAdjInner * kTile];
  const int nt = n_tiles<TILE>(T);
  const int tid = threadIdx.x;
  const XcdLoop tiles(nt);
  for (int it = tiles.first; it < tiles.end; it += tiles.step) {
    const int2 tl = tile_entry<TILE>(T, it);
    const WorldDev& w = W[tl.x];
    const AdjDev& A = adj_of(AA, tl.x);
    const int R = w.radius;
    const int nx = w.nx, ny = w.ny;
    const int x0 = tile_x(tl.y) * kTile;
    const int y0 = tile_y(tl.y) * kTile;
    const int rega = kAdjRing + 2 * R;       // dL/dG region, origin (x0-R-1, y0-R-1)
    const int regb = kTile + 2 * R;          // D^T dL/dG region, origin (x0-R, y0-R)
    const MC_GLOBAL vf2* gb = glbv<const vf2>(A.Gbar);
    for (int k = tid; k < rega * rega; k += kThreads) {
      const int r = k / rega, c = k - (k / rega) * rega;
      const vf2 v = gb[(size_t)wrap_index(y0 - R - 1 + r, ny) * nx + wrap_index(x0 - R - 1 + c, nx)];
      s_gx[k] = v.x;
      s_gy[k] = v.y;
    }
    __syncthreads();
    // (D^T h)(c) = (h_x(c - e_x) - h_x(c + e_x)) / 2 + (h_y(c - e_y) - h_y(c + e_y)) / 2
    for (int k = tid; k < regb * regb; k += kThreads) {
      const int r = k / regb, c = k - (k / regb) * regb;
      const int ra = r + 1, ca = c + 1;
      s_in[k] = 0.5f * (s_gx[ra * rega + ca - 1] - s_gx[ra * rega + ca + 1]) +
                0.5f * (s_gy[(ra - 1) * rega + ca] - s_gy[(ra + 1) * rega + ca]);
    }
    __syncthreads();
    for (int k = tid; k < regb * kTile; k += kThreads) {
      const int r = k / kTile, c = k - (k / kTile) * kTile;
      const float* row = s_in + r * regb + c + R;
      float acc = w.gtap[0] * row[0];
      for (int m = 1; m <= R; ++m) acc += w.gtap[m] * (row[-m] + row[m]);
      s_mid[r * kTile + c] = acc;
    }
    __syncthreads();
    MC_GLOBAL float* sb = glb(A.sbar);
    for (int k = tid; k < kTile * kTile; k += kThreads) {
      const int r = k >> TileCfg<TILE>::kShift, c = k & (kTile - 1);
      const float* col = s_mid + (r + R) * kTile + c;
      float acc = w.gtap[0] * col[0];
      for (int m = 1; m <= R; ++m) acc += w.gtap[m] * (col[-m * kTile] + col[m * kTile]);
      const int gx = x0 + c, gy = y0 + r;
      if (gx < nx && gy < ny) sb[(size_t)gy * nx + gx] = acc;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// S2 + S1 + S0 reversed, one block per node pack.  GEN: the general variant
// of the forward's PBD (closed loops: the joint before node 0 and the
// closing edge, a third colour on loops of odd length; per-edge
// stiffnesses), reversed pass by pass in the same way.  BR: branches too
// (each attached filament's first node c0 owns its attachment: the joints
// at the parent p and at c0, then the edge p -> c0, after the regular
// passes of each kind, with the world's stiffnesses and fixed rest angles).
// IT: the iterations whose states the registers hold (at least every
// world's pbd_iters; 4 for the usual count, kMaxAdjIters otherwise: fewer
// registers, more blocks per CU).
// ---------------------------------------------------------------------------
template <int PACK, bool GEN, bool BR, int IT>
__global__ __launch_bounds__(PACK) void k_adj_pbd(const WorldDev* __restrict__ W, Tables T, AdjArg AA) {
  static_assert(GEN || !BR, "branches take the general variant");
  __shared__ float s_th[PACK];
  __shared__ float s_dx[PACK];
  __shared__ float s_dy[PACK];
  __shared__ float s_gx[PACK];     // dL/dd per node
  __shared__ float s_gy[PACK];
  __shared__ float s_gth[PACK];    // dL/dtheta per edge
  __shared__ float s_ta[BR ? PACK : 1];    // attachment edge angle (owned by c0)
  __shared__ float s_gta[BR ? PACK : 1];   // and its adjoint
  __shared__ int s_off[PACK + 1];
  const int npk = *T.n_packs;
  const int li = threadIdx.x;
  for (int it = blockIdx.x; it < npk; it += gridDim.x) {
    const Pack pk = T.packs[it];
    const WorldDev& w = W[pk.world];
    const AdjDev& A = adj_of(AA, pk.world);
    const int N = w.n_part, nx = w.nx, ny = w.ny;
    const MC_GLOBAL int* cell = glb(w.cell_in);
    const MC_GLOBAL float* frac = glb(w.frac_in);
    const int nf = pk.fil_end - pk.fil_begin;
    for (int k = li; k <= nf; k += PACK) s_off[k] = glb(w.fil_offset)[pk.fil_begin + k] - pk.node_begin;
    __syncthreads();
    const int gi = pk.node_begin + li;
    const bool active = gi < pk.node_end;
    int lo = 0, hi = nf - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (s_off[mid] <= li) lo = mid; else hi = mid - 1;
    }
    const int o = s_off[lo];
    const int n = s_off[lo + 1] - o;
    const int k = li - o;
    const int fil = pk.fil_begin + lo;
    // as in the forward: a closed loop (three nodes or more) closes with the
    // edge from its last node to its first, and every node is a joint
    const bool ring = GEN && active && w.fil_flags && (glb(w.fil_flags)[fil] & 1) && n >= 3;
    const bool has_edge = active && (k < n - 1 || ring);
    const bool is_joint = active && (ring || (k >= 1 && k <= n - 2));
    const int j = ring ? k : k - 1;
    const int m = ring ? n : n - 2;
    const int li_prev = (ring && k == 0) ? o + n - 1 : li - 1;    // edge before the joint
    const int li_next = (ring && k == n - 1) ? o : li + 1;        // far node of the edge
    const int jcol = (ring && (n & 1) && j == n - 1) ? 2 : (j & 1);
    const int ecol = (ring && (n & 1) && k == n - 1) ? 2 : (k & 1);
    int ncol = 2;                                // block-uniform
    if constexpr (GEN) ncol = __syncthreads_or(ring && (n & 1)) ? 3 : 2;

    int cx = 0, cy = 0;
    float fx = 0.f, fy = 0.f;
    if (active) {
      cx = cell[gi]; cy = cell[N + gi];
      fx = frac[gi]; fy = frac[N + gi];
    }
    float v0x = 0.f, v0y = 0.f, L = 0.f, th = 0.f;
    float u0x = 1.f, u0y = 0.f;
    if (has_edge) {
      const int gn = pk.node_begin + li_next;
      v0x = (float)(cell[gn] - cx) + (frac[gn] - fx);
      v0y = (float)(cell[N + gn] - cy) + (frac[N + gn] - fy);
      L = glb(w.rest_length)[gi];
      th = atan2f(v0y, v0x);
      const float l0 = hw_sqrt(v0x * v0x + v0y * v0y);
      if (l0 > 0.f) {
        const float il = hw_rcp(l0);
        u0x = v0x * il;
        u0y = v0y * il;
      }
    }
    float th_hat = 0.f;
    if (is_joint)
      th_hat = actuated_angle(glb(w.rest_angle)[gi], glb(w.act_amp)[fil], glb(w.act_period)[fil],
                              glb(w.act_phase)[fil], w.ctl_src->t, j, m);
    // the attachment this node owns (as in the forward)
    bool att = false, att_cj = false, any_att = false;
    int p_l = 0, in_l = 0;
    float a_vx = 0.f, a_vy = 0.f, a_th = 0.f, a_ux = 1.f, a_uy = 0.f, a_L = 0.f, a_al = 0.f, a_be = 0.f;
    if (BR && w.fil_parent) {                  // block-uniform: the pack's world
      const int par = (active && k == 0) ? glb(w.fil_parent)[fil] : -1;
      att = par >= 0;
      if (att) {
        p_l = par - pk.node_begin;
        int lp = 0, hp = nf - 1;
        while (lp < hp) {
          const int mid = (lp + hp + 1) >> 1;
          if (s_off[mid] <= p_l) lp = mid; else hp = mid - 1;
        }
        in_l = p_l == s_off[lp] ? s_off[lp + 1] - 1 : p_l - 1;   // p's entering edge
        const int F = w.n_fil;
        a_L = glb(w.fil_attach)[fil];
        a_al = glb(w.fil_attach)[F + fil];
        a_be = glb(w.fil_attach)[2 * F + fil];
        a_vx = (float)(cx - cell[par]) + (fx - frac[par]);
        a_vy = (float)(cy - cell[N + par]) + (fy - frac[N + par]);
        a_th = atan2f(a_vy, a_vx);
        const float l0 = hw_sqrt(a_vx * a_vx + a_vy * a_vy);
        if (l0 > 0.f) {
          const float il = hw_rcp(l0);
          a_ux = a_vx * il;
          a_uy = a_vy * il;
        }
        att_cj = n >= 2;
      }
      s_ta[li] = a_th;
      any_att = __syncthreads_or(att);
    }
    const float hb_w = 0.5f * w.k_bend, hs_w = 0.5f * w.k_stretch, ksh_w = w.k_shear;
    // dL/dx_t so far (written by k_adj_force) plus the deposit derivative
    float xbx = 0.f, xby = 0.f;
    if (active) {
      xbx = A.xbar[gi];
      xby = A.xbar[N + gi];
      const int bx = wrap_index(cx, nx), by = wrap_index(cy, ny);
      float wx[4], dwx[4], wy[4], dwy[4];
      peskin4_d(fx, wx, dwx);
      peskin4_d(fy, wy, dwy);
      const MC_GLOBAL float* sb = glb(A.sbar);
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const size_t row = (size_t)wrap_near(by - 1 + b, ny) * nx;
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          const float sv = sb[row + wrap_near(bx - 1 + a, nx)];
          xbx += dwx[a] * wy[b] * sv;
          xby += wx[a] * dwy[b] * sv;
        }
      }
    }

    // forward PBD again, keeping the state each position pass starts from
    const int K = w.pbd_iters;
    // per-edge stiffnesses of the joint and the edge at this node
    const int gs = active ? gi : pk.node_begin;
    const float hb = 0.5f * (w.kb_arr ? glb(w.kb_arr)[gs] : w.k_bend);
    const float hs = 0.5f * (w.ks_arr ? glb(w.ks_arr)[gs] : w.k_stretch);
    const float ksh = w.ksh_arr ? glb(w.ksh_arr)[gs] : w.k_shear;
    constexpr int kCol = GEN ? 3 : 2;
    float d_p_x[kCol][IT], d_p_y[kCol][IT];   // d before each position colour
    float th_p[IT];
    constexpr int kAtt = BR ? IT : 1;
    float ta_p[kAtt], da_x[kAtt], da_y[kAtt];   // attachment angle after the joints; d before its edge pass
    s_th[li] = th;
    s_dx[li] = 0.f;
    s_dy[li] = 0.f;
    __syncthreads();
#pragma unroll
    for (int iter = 0; iter < IT; ++iter) {
      if (iter < K) {
#pragma unroll
        for (int par = 0; par < kCol; ++par) {
          if (par < ncol) {
            if (is_joint && jcol == par) {
              const float t1 = s_th[li_prev];
              const float t2 = s_th[li];
              const float c = wrap_angle(t2 - t1) - th_hat;
              s_th[li_prev] = t1 + hb * c;
              s_th[li] = t2 - hb * c;
            }
            __syncthreads();
          }
        }
        if (BR && any_att) {                   // attachment joints: at p, then at c0
          if (att) {
            const float t1 = s_th[in_l], t2 = s_ta[li];
            const float c = wrap_angle(t2 - t1) - a_al;
            s_th[in_l] = t1 + hb_w * c;
            s_ta[li] = t2 - hb_w * c;
          }
          __syncthreads();
          if (att_cj) {
            const float t1 = s_ta[li], t2 = s_th[li];
            const float c = wrap_angle(t2 - t1) - a_be;
            s_ta[li] = t1 + hb_w * c;
            s_th[li] = t2 - hb_w * c;
          }
          __syncthreads();
        }
        th_p[iter] = s_th[li];
        if constexpr (BR) ta_p[iter] = s_ta[li];
#pragma unroll
        for (int par = 0; par < kCol; ++par) {
          if (par >= ncol) continue;
          d_p_x[par][iter] = s_dx[li];
          d_p_y[par][iter] = s_dy[li];
          __syncthreads();
          if (has_edge && ecol == par) {
            const float d0x = s_dx[li], d0y = s_dy[li];
            const float d1x = s_dx[li_next], d1y = s_dy[li_next];
            const float vx = v0x + (d1x - d0x);
            const float vy = v0y + (d1y - d0y);
            const float ell = hw_sqrt(vx * vx + vy * vy);
            const float sc = (ell - L) * hw_rcp(ell);
            const float csx = sc * vx, csy = sc * vy;
            float sn, cs;
            edge_direction(th_p[iter], th, u0x, u0y, &cs, &sn);
            const float dx = hs * (csx + ksh * (vx - L * cs - csx));
            const float dy = hs * (csy + ksh * (vy - L * sn - csy));
            s_dx[li] = d0x + dx;
            s_dy[li] = d0y + dy;
            s_dx[li_next] = d1x - dx;
            s_dy[li_next] = d1y - dy;
          }
          __syncthreads();
        }
        if (BR && any_att) {                   // attachment edges p -> c0
          if constexpr (BR) {
            da_x[iter] = s_dx[li];
            da_y[iter] = s_dy[li];
          }
          __syncthreads();
          if (att) {
            const float d0x = s_dx[p_l], d0y = s_dy[p_l];
            const float d1x = s_dx[li], d1y = s_dy[li];
            const float vx = a_vx + (d1x - d0x);
            const float vy = a_vy + (d1y - d0y);
            const float ell = hw_sqrt(vx * vx + vy * vy);
            const float sc = (ell - a_L) * hw_rcp(ell);
            const float csx = sc * vx, csy = sc * vy;
            float sn, cs;
            edge_direction(ta_p[BR ? iter : 0], a_th, a_ux, a_uy, &cs, &sn);
            const float dx = hs_w * (csx + ksh_w * (vx - a_L * cs - csx));
            const float dy = hs_w * (csy + ksh_w * (vy - a_L * sn - csy));
            s_dx[p_l] = d0x + dx;
            s_dy[p_l] = d0y + dy;
            s_dx[li] = d1x - dx;
            s_dy[li] = d1y - dy;
          }
          __syncthreads();
        }
      }
    }

    // reverse: F_el = k_el d  ->  dL/dd = k_el dL/dF
    const float kel = w.k_el;
    s_gx[li] = active ? kel * A.Fbar[gi] : 0.f;
    s_gy[li] = active ? kel * A.Fbar[N + gi] : 0.f;
    s_gth[li] = 0.f;
    if constexpr (BR) s_gta[li] = 0.f;
    float v0bx = 0.f, v0by = 0.f, thhb = 0.f;
    float a_v0bx = 0.f, a_v0by = 0.f;          // dL/d(attachment vector), c0 lanes
    __syncthreads();
#pragma unroll
    for (int iter = IT - 1; iter >= 0; --iter) {
      if (iter < K) {
        if (BR && any_att) {                   // attachment edges reversed
          if constexpr (BR) {
            s_dx[li] = da_x[iter];
            s_dy[li] = da_y[iter];
          }
          __syncthreads();
          if (att) {
            const float d0x = s_dx[p_l], d0y = s_dy[p_l];
            const float d1x = s_dx[li], d1y = s_dy[li];
            const float vx = a_vx + (d1x - d0x);
            const float vy = a_vy + (d1y - d0y);
            const float ell = sqrtf(vx * vx + vy * vy);
            const float hx = vx / ell, hy = vy / ell;
            const float Dbx = s_gx[p_l] - s_gx[li];
            const float Dby = s_gy[p_l] - s_gy[li];
            const float a = 1.0f - ksh_w;
            const float lr = a_L / ell;
            const float hd = hx * Dbx + hy * Dby;
            const float mbx = hs_w * (Dbx - a * lr * (Dbx - hx * hd));
            const float mby = hs_w * (Dby - a * lr * (Dby - hy * hd));
            s_gx[p_l] -= mbx;
            s_gy[p_l] -= mby;
            s_gx[li] += mbx;
            s_gy[li] += mby;
            a_v0bx += mbx;
            a_v0by += mby;
            float sn, cs;
            edge_direction(ta_p[BR ? iter : 0], a_th, a_ux, a_uy, &cs, &sn);
            s_gta[li] += -hs_w * ksh_w * a_L * (-sn * Dbx + cs * Dby);
          }
          __syncthreads();
        }
#pragma unroll
        for (int par = kCol - 1; par >= 0; --par) {
          if (par >= ncol) continue;
          s_dx[li] = d_p_x[par][iter];
          s_dy[li] = d_p_y[par][iter];
          __syncthreads();
          if (has_edge && ecol == par) {
            const float d0x = s_dx[li], d0y = s_dy[li];
            const float d1x = s_dx[li_next], d1y = s_dy[li_next];
            const float vx = v0x + (d1x - d0x);
            const float vy = v0y + (d1y - d0y);
            const float ell = sqrtf(vx * vx + vy * vy);
            const float hx = vx / ell, hy = vy / ell;
            const float Dbx = s_gx[li] - s_gx[li_next];
            const float Dby = s_gy[li] - s_gy[li_next];
            // M = hs [(1 - ksh) (I - (L/ell)(I - h h^T)) + ksh I]
            const float a = 1.0f - ksh;
            const float lr = L / ell;
            const float hd = hx * Dbx + hy * Dby;
            const float mbx = hs * (Dbx - a * lr * (Dbx - hx * hd));
            const float mby = hs * (Dby - a * lr * (Dby - hy * hd));
            s_gx[li] -= mbx;
            s_gy[li] -= mby;
            s_gx[li_next] += mbx;
            s_gy[li_next] += mby;
            v0bx += mbx;
            v0by += mby;
            float sn, cs;
            edge_direction(th_p[iter], th, u0x, u0y, &cs, &sn);
            s_gth[li] += -hs * ksh * L * (-sn * Dbx + cs * Dby);
          }
          __syncthreads();
        }
        if (BR && any_att) {                   // attachment joints reversed: at c0, then at p
          if (att_cj) {
            const float cb = hb_w * (s_gta[li] - s_gth[li]);
            s_gta[li] -= cb;
            s_gth[li] += cb;
          }
          __syncthreads();
          if (att) {
            const float cb = hb_w * (s_gth[in_l] - s_gta[li]);
            s_gth[in_l] -= cb;
            s_gta[li] += cb;
          }
          __syncthreads();
        }
#pragma unroll
        for (int par = kCol - 1; par >= 0; --par) {
          if (par >= ncol) continue;
          if (is_joint && jcol == par) {
            const float cb = hb * (s_gth[li_prev] - s_gth[li]);
            s_gth[li_prev] -= cb;
            s_gth[li] += cb;
            thhb -= cb;
          }
          __syncthreads();
        }
      }
    }
    // theta_e = atan2(v0): d theta / d v0 = (-v0y, v0x) / |v0|^2
    if (has_edge) {
      const float r2 = v0x * v0x + v0y * v0y;
      const float tb = s_gth[li];
      v0bx += tb * (-v0y / r2);
      v0by += tb * (v0x / r2);
    }
    __syncthreads();
    // the attachment angle atan2(a_v), a_v = x_c0 - x_p
    if (BR && att) {
      const float r2 = a_vx * a_vx + a_vy * a_vy;
      const float tb = s_gta[li];
      a_v0bx += tb * (-a_vy / r2);
      a_v0by += tb * (a_vx / r2);
    }
    // v0_e = x_next(e) - x_e
    s_dx[li] = has_edge ? v0bx : 0.f;
    s_dy[li] = has_edge ? v0by : 0.f;
    if constexpr (BR) {                        // (dL/dd is no longer needed: it holds -dL/da_v at p)
      s_gx[li] = 0.f;
      s_gy[li] = 0.f;
    }
    __syncthreads();
    if (BR && att) {                           // one child per parent node: a single writer
      s_gx[p_l] = -a_v0bx;
      s_gy[p_l] = -a_v0by;
    }
    if constexpr (BR) __syncthreads();
    if (active) {
      xbx -= s_dx[li];
      xby -= s_dy[li];
      if (k >= 1 || ring) {                     // the edge ending here (a loop's closing edge at node 0)
        xbx += s_dx[li_prev];
        xby += s_dy[li_prev];
      }
      if constexpr (BR) {
        xbx += s_gx[li] + a_v0bx;
        xby += s_gy[li] + a_v0by;
      }
      A.xbar[gi] = xbx;
      A.xbar[N + gi] = xby;
      if (is_joint) A.g_rest[gi] += thhb;     // theta_hat = theta_rest + actuation
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// S5 with multi-direct forcing (binned transfer), forward recomputed and
// reversed; with two layers, I and S act through the markers (the MK
// variants), and the position terms also go to dL/dd.  Forward: F_grid_1 = S[F], U_d = I[j / rho] + F / 2, and for
// k = 1 .. K-1: u_k = (j + F_grid_k / 2) / rho, c_k = 2 (U_d - I[u_k]),
// F_grid_{k+1} = F_grid_k + S[c_k].  Given G~ = dL/dF_grid_{k+1}, iteration k
// reversed: c~ = I[G~]; U_d~ += 2 c~; U_k~ = -2 c~; x~ gets the derivatives
// of S[c_k] and I[u_k] in the node positions; u_k~ = S[U_k~] gives
// G~ += u_k~ / (2 rho), j~ += u_k~ / rho, rho~ -= u_k~ . u_k / rho.  Then U_d:
// F~ += U_d~ / 2 (in k_adj_force), x~ from I[j / rho], v~ = S[U_d~] gives
// j~ += v~ / rho, rho~ -= v~ . (j / rho) / rho, and finally g~_q += rho~ + c_q . j~.
// Node passes gather over each tile's own-bin nodes from fields staged over
// the tile with one cell before it and two after on each axis (one more on
// each side with markers); the spreads are the tile spread in 64-bit
// fixed point.  The recomputed iterates use the forward's arithmetic and sums,
// so they equal the forward's bit for bit.
// ---------------------------------------------------------------------------
// Zero U_d~, the MDF position terms, j~ and rho~ of every world (blockIdx.y:
// the world table entry).
__global__ void k_adj_mdf_zero(const WorldDev* __restrict__ W, Tables T, AdjArg AA) {
  if ((int)blockIdx.y >= *T.n_worlds) return;
  const int wi = T.worlds[blockIdx.y].x;
  const WorldDev& w = W[wi];
  const AdjDev& A = adj_of(AA, wi);
  const size_t n2 = 2 * (size_t)w.n_part, nc = (size_t)w.nx * w.ny;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < 2 * n2 + 3 * nc;
       i += (size_t)gridDim.x * blockDim.x) {
    if (i < n2) A.Udbar[i] = 0.f;
    else if (i < 2 * n2) A.xbar_m[i - n2] = 0.f;
    else if (i < 2 * n2 + 2 * nc) ((float*)A.jbar)[i - 2 * n2] = 0.f;
    else A.rhobar[i - 2 * n2 - 2 * nc] = 0.f;
    if (A.dbar_m && i < n2) A.dbar_m[i] = 0.f;
  }
}

// Cells (x0 - 1 - E + c, y0 - 1 - E + r), c, r in [0, TILE + 3 + 2E), of a
// tile: value(idx) of each (periodic grid index) into st; all loads before
// the stores.  E = 1 reaches the supports of the tile's nodes' two-layer
// markers.
template <int TILE, int E, class V>
static __device__ __forceinline__ void adj_stage(int nx, int ny, int x0, int y0, vf2* st, V value) {
  constexpr int kStage = TILE + 3 + 2 * E, kThreads = TileCfg<TILE>::kThreads;
  constexpr int kIt = (kStage * kStage + kThreads - 1) / kThreads;
  vf2 v[kIt];
#pragma unroll
  for (int i = 0; i < kIt; ++i) {
    const int k = min((int)threadIdx.x + kThreads * i, kStage * kStage - 1);
    const int r = k / kStage, c = k - (k / kStage) * kStage;
    v[i] = value((size_t)wrap_index(y0 - 1 - E + r, ny) * nx + wrap_index(x0 - 1 - E + c, nx));
  }
#pragma unroll
  for (int i = 0; i < kIt; ++i) {
    const int k = (int)threadIdx.x + kThreads * i;
    if (k < kStage * kStage) st[k] = v[i];
  }
}

// The points a tile node acts through, relative to the staged window of
// adj_stage<TILE, MK ? 1 : 0>: the node itself (weight 1), or its two
// markers (weight 1/2 each); f(l, lx, ly, fx, fy, h) is called for each with
// the support origin in the window, the point's fractions and its weight.
template <bool MK, class Fn>
static __device__ __forceinline__ void for_points(const WorldDev& w, int gi, int lx, int ly, float fx, float fy,
                                                  Fn f) {
  if constexpr (MK) {
    const int N = w.n_part;
    const float ddx = glb(w.d_marker)[gi], ddy = glb(w.d_marker)[N + gi];
#pragma unroll
    for (int l = 0; l < 2; ++l) {
      const float sg = l == 0 ? 1.f : -1.f;
      int sx, sy;
      float mx, my;
      marker_shift(fx, sg * ddx, &sx, &mx);
      marker_shift(fy, sg * ddy, &sy, &my);
      f(l, lx + sx + 1, ly + sy + 1, mx, my, 0.5f);
    }
  } else {
    f(0, lx, ly, fx, fy, 1.0f);
  }
}

// U_d (DESIRED) or the correction c_k of the iterate Fgk at the tile's own
// nodes (MK: through their two-layer markers).
template <int TILE, bool DESIRED, bool MK>
__global__ __launch_bounds__(TileCfg<TILE>::kThreads) void k_adj_mdf_fwd_gather(const WorldDev* __restrict__ W,
                                                                                 Tables T, AdjArg AA, int k) {
  constexpr int kE = MK ? 1 : 0;
  constexpr int kStage = TILE + 3 + 2 * kE, kThreads = TileCfg<TILE>::kThreads;
  __shared__ vf2 s_u[kStage * kStage];
  const int nt = n_tiles<TILE>(T);
  const XcdLoop tiles(nt);
  for (int it = tiles.first; it < tiles.end; it += tiles.step) {
    const int2 tl = tile_entry<TILE>(T, it);
    const WorldDev& w = W[tl.x];
    if (MK != (w.d_marker != nullptr)) continue;
    const AdjDev& A = adj_of(AA, tl.x);
    const float2* Fgk = A.Fgk + (size_t)(k > 0 ? k - 1 : 0) * ((size_t)w.nx * w.ny);   // iterate k (k >= 1)
    const int nx = w.nx, ny = w.ny, N = w.n_part;
    const int x0 = tile_x(tl.y) * TILE, y0 = tile_y(tl.y) * TILE;
    const MC_GLOBAL vf4* m = glbv<const vf4>(w.rho_j);
    const MC_GLOBAL vf2* Fg = glbv<const vf2>(Fgk);
    adj_stage<TILE, kE>(nx, ny, x0, y0, s_u, [&](size_t c) {
      const vf4 mv = m[c];
      vf2 u;
      if (DESIRED) {
        u.x = mv.y / mv.x;
        u.y = mv.z / mv.x;
      } else {
        const vf2 fv = Fg[c];
        const float inv = 1.0f / mv.x;
        u.x = (mv.y + 0.5f * fv.x) * inv;
        u.y = (mv.z + 0.5f * fv.y) * inv;
      }
      return u;
    });
    __syncthreads();
    const int tile = tile_y(tl.y) * w.ntx + tile_x(tl.y);
    const int e0 = glb(w.bin_start)[tile], e1 = glb(w.bin_start)[tile + 1];
    const MC_GLOBAL vi4* recs = glbv<const vi4>(w.bin_rec);
    for (int e = e0 + (int)threadIdx.x; e < e1; e += kThreads) {
      const vi4 r = recs[e];
      const int lx = (r.x & 0xffff) - x0, ly = (r.x >> 16) - y0;
      const int gi = r.w;
      float gx = 0.f, gy = 0.f;
      float sx = 0.f, sy = 0.f;
      for_points<MK>(w, gi, lx, ly, __int_as_float(r.y), __int_as_float(r.z),
                     [&](int, int px, int py, float fx, float fy, float) {
        float wx[4], wy[4];
        peskin4(fx, wx);
        peskin4(fy, wy);
        float qx = 0.f, qy = 0.f;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const vf2* row = s_u + (py + b) * kStage + px;
          float ax = 0.f, ay = 0.f;
#pragma unroll
          for (int a = 0; a < 4; ++a) {
            const vf2 t = row[a];
            ax += wx[a] * t.x;
            ay += wx[a] * t.y;
          }
          qx += wy[b] * ax;
          qy += wy[b] * ay;
        }
        sx += qx;
        sy += qy;
      });
      if (MK) {                         // the forward's order: both markers summed, then halved
        gx = 0.5f * sx;
        gy = 0.5f * sy;
      } else {
        gx = sx;
        gy = sy;
      }
      if (DESIRED) {
        A.Ud[gi] = gx + 0.5f * glb(w.fel)[gi];
        A.Ud[N + gi] = gy + 0.5f * glb(w.fel)[N + gi];
      } else {
        A.mc[gi] = 2.0f * (A.Ud[gi] - gx);
        A.mc[N + gi] = 2.0f * (A.Ud[N + gi] - gy);
      }
    }
    __syncthreads();
  }
}

// Reverse node pass.  MODE 0 (iteration k, iterate Fgk): c~ = I[G~],
// U_k~ = -2 c~ (stored), U_d~ += 2 c~, x~ += dI/dx terms of S[c_k] and I[u_k].
// MODE 1 (U_d): x~ += U_d~ . dI[j / rho]/dx.  MK: I and S act through the
// two markers (half weight each); each marker's position term goes to x~
// and, with its sign, to dL/dd (A.dbar_m).
template <int TILE, int MODE, bool MK>
__global__ __launch_bounds__(TileCfg<TILE>::kThreads) void k_adj_mdf_node(const WorldDev* __restrict__ W, Tables T,
                                                                           AdjArg AA, int k) {
  constexpr int kE = MK ? 1 : 0;
  constexpr int kStage = TILE + 3 + 2 * kE, kThreads = TileCfg<TILE>::kThreads;
  __shared__ vf2 s_g[MODE == 0 ? kStage * kStage : 1];
  __shared__ vf2 s_u[kStage * kStage];
  const int nt = n_tiles<TILE>(T);
  const XcdLoop tiles(nt);
  for (int it = tiles.first; it < tiles.end; it += tiles.step) {
    const int2 tl = tile_entry<TILE>(T, it);
    const WorldDev& w = W[tl.x];
    if (MK != (w.d_marker != nullptr)) continue;
    const AdjDev& A = adj_of(AA, tl.x);
    const float2* Fgk = A.Fgk + (size_t)(k > 0 ? k - 1 : 0) * ((size_t)w.nx * w.ny);   // iterate k (k >= 1)
    const int nx = w.nx, ny = w.ny, N = w.n_part;
    const int x0 = tile_x(tl.y) * TILE, y0 = tile_y(tl.y) * TILE;
    const MC_GLOBAL vf4* m = glbv<const vf4>(w.rho_j);
    const MC_GLOBAL vf2* Fg = glbv<const vf2>(Fgk);
    const MC_GLOBAL vf2* Gb = glbv<const vf2>(A.Fgbar);
    if constexpr (MODE == 0) adj_stage<TILE, kE>(nx, ny, x0, y0, s_g, [&](size_t c) { return Gb[c]; });
    adj_stage<TILE, kE>(nx, ny, x0, y0, s_u, [&](size_t c) {
      const vf4 mv = m[c];
      const float inv = 1.0f / mv.x;
      vf2 u;
      if (MODE == 0) {
        const vf2 fv = Fg[c];
        u.x = (mv.y + 0.5f * fv.x) * inv;
        u.y = (mv.z + 0.5f * fv.y) * inv;
      } else {
        u.x = mv.y * inv;
        u.y = mv.z * inv;
      }
      return u;
    });
    __syncthreads();
    const int tile = tile_y(tl.y) * w.ntx + tile_x(tl.y);
    const int e0 = glb(w.bin_start)[tile], e1 = glb(w.bin_start)[tile + 1];
    const MC_GLOBAL vi4* recs = glbv<const vi4>(w.bin_rec);
    for (int e = e0 + (int)threadIdx.x; e < e1; e += kThreads) {
      const vi4 r = recs[e];
      const int lx = (r.x & 0xffff) - x0, ly = (r.x >> 16) - y0;
      const float nfx = __int_as_float(r.y), nfy = __int_as_float(r.z);
      const int gi = r.w;
      // I[G~] and I[u] (the forward's order: the points summed, then halved)
      float cbx = 0.f, cby = 0.f, Ux = 0.f, Uy = 0.f;
      for_points<MK>(w, gi, lx, ly, nfx, nfy, [&](int, int px, int py, float fx, float fy, float) {
        float wx[4], wy[4];
        peskin4(fx, wx);
        peskin4(fy, wy);
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
          for (int a = 0; a < 4; ++a) {
            const int q = (py + b) * kStage + px + a;
            const float W0 = wx[a] * wy[b];
            if (MODE == 0) {
              cbx += W0 * s_g[q].x;
              cby += W0 * s_g[q].y;
            }
            Ux += W0 * s_u[q].x;
            Uy += W0 * s_u[q].y;
          }
      });
      if (MK) {
        cbx *= 0.5f;
        cby *= 0.5f;
        Ux *= 0.5f;
        Uy *= 0.5f;
      }
      float Ubx, Uby;                                            // dL/d(the sampled velocity)
      float cx = 0.f, cy = 0.f;
      if (MODE == 0) {
        Ubx = -2.0f * cbx;
        Uby = -2.0f * cby;
        cx = 2.0f * (A.Ud[gi] - Ux);
        cy = 2.0f * (A.Ud[N + gi] - Uy);
        A.Ukbar[gi] = Ubx;
        A.Ukbar[N + gi] = Uby;
        A.Udbar[gi] += 2.0f * cbx;
        A.Udbar[N + gi] += 2.0f * cby;
      } else {
        Ubx = A.Udbar[gi];
        Uby = A.Udbar[N + gi];
      }
      float sx = 0.f, sy = 0.f, dx = 0.f, dy = 0.f;
      for_points<MK>(w, gi, lx, ly, nfx, nfy, [&](int l, int px, int py, float fx, float fy, float h) {
        float wx[4], dwx[4], wy[4], dwy[4];
        peskin4_d(fx, wx, dwx);
        peskin4_d(fy, wy, dwy);
        float qx = 0.f, qy = 0.f;
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
          for (int a = 0; a < 4; ++a) {
            const int q = (py + b) * kStage + px + a;
            float p = Ubx * s_u[q].x + Uby * s_u[q].y;
            if (MODE == 0) p += cx * s_g[q].x + cy * s_g[q].y;
            qx += dwx[a] * wy[b] * p;
            qy += wx[a] * dwy[b] * p;
          }
        sx += h * qx;
        sy += h * qy;
        if (MK) {
          dx += (l == 0 ? h : -h) * qx;
          dy += (l == 0 ? h : -h) * qy;
        }
      });
      A.xbar_m[gi] += sx;
      A.xbar_m[N + gi] += sy;
      if (MK) {
        A.dbar_m[gi] += dx;
        A.dbar_m[N + gi] += dy;
      }
    }
    __syncthreads();
  }
}

// Reverse cell pass: w~ = S[nodevec] over the tile, then MODE 0 (iterate
// Fgk): G~ += w~ / (2 rho), j~ += w~ / rho, rho~ -= w~ . u_k / rho; MODE 1
// (U_d): j~ += w~ / rho, rho~ -= w~ . (j / rho) / rho, and g~_q += rho~ + c_q . j~.
template <int TILE, int MODE>
__global__ __launch_bounds__(TileCfg<TILE>::kThreads) void k_adj_mdf_cell(const WorldDev* __restrict__ W, Tables T,
                                                                           AdjArg AA, int k) {
  using C = TileCfg<TILE>;
  constexpr int kThreads = C::kThreads, kSpreadCells = C::kSpreadCells;
  __shared__ __align__(16) long long s_x[kSpreadCells];
  __shared__ __align__(16) long long s_y[kSpreadCells];
  __shared__ vi4 s_list[(kThreads / 64) * kWaveList];
  const int nt = n_tiles<TILE>(T);
  const XcdLoop tiles(nt);
  for (int it = tiles.first; it < tiles.end; it += tiles.step) {
    const int2 tl = tile_entry<TILE>(T, it);
    const WorldDev& w = W[tl.x];
    const AdjDev& A = adj_of(AA, tl.x);
    const float2* Fgk = A.Fgk + (size_t)(k > 0 ? k - 1 : 0) * ((size_t)w.nx * w.ny);   // iterate k (k >= 1)
    const float* nodevec = MODE == 0 ? A.Ukbar : A.Udbar;
    const int nx = w.nx, ny = w.ny;
    const int ncell = nx * ny;
    const int x0 = tile_x(tl.y) * TILE, y0 = tile_y(tl.y) * TILE;
    const int tw = min(TILE, nx - x0), th = min(TILE, ny - y0);
    zero_lds_u64(s_x, kSpreadCells);
    zero_lds_u64(s_y, kSpreadCells);
    __syncthreads();
    if (w.d_marker)                     // two layers: the nodes' vectors spread from their markers
      tile_spread_markers<TILE, false>(w, x0, y0, tw, th, glb(nodevec), 1.0f, s_x, s_y, s_list,
                                       glbv<const vi4>(w.bin_rec), spread_fetch<TILE>(w, x0, y0), nullptr);
    else
      tile_spread_vec<TILE, false>(w, x0, y0, tw, th, glb(nodevec), 1.0f, s_x, s_y, s_list,
                                   glbv<const vi4>(w.bin_rec), spread_fetch<TILE>(w, x0, y0), nullptr);
    __syncthreads();
    const MC_GLOBAL vf4* m = glbv<const vf4>(w.rho_j);
    for (int k = threadIdx.x; k < TILE * TILE; k += kThreads) {
      const int ly = k >> C::kShift, lx = k & (TILE - 1);
      if (lx >= tw || ly >= th) continue;
      const size_t c = (size_t)(y0 + ly) * nx + x0 + lx;
      const float wbx = fix_to_float(spread_cell<TILE>(s_x, lx, ly, nx, ny));
      const float wby = fix_to_float(spread_cell<TILE>(s_y, lx, ly, nx, ny));
      const vf4 mv = m[c];
      const float inv = 1.0f / mv.x;
      vf2 u;
      if (MODE == 0) {
        const vf2 fv = glbv<const vf2>(Fgk)[c];
        u.x = (mv.y + 0.5f * fv.x) * inv;
        u.y = (mv.z + 0.5f * fv.y) * inv;
        vf2 gb = glbv<vf2>(A.Fgbar)[c];
        gb.x += 0.5f * wbx * inv;
        gb.y += 0.5f * wby * inv;
        glbv<vf2>(A.Fgbar)[c] = gb;
      } else {
        u.x = mv.y * inv;
        u.y = mv.z * inv;
      }
      vf2 jb = glbv<vf2>(A.jbar)[c];
      jb.x += wbx * inv;
      jb.y += wby * inv;
      const float rb = A.rhobar[c] - (wbx * u.x + wby * u.y) * inv;
      if (MODE == 0) {
        glbv<vf2>(A.jbar)[c] = jb;
        A.rhobar[c] = rb;
      } else {
        MC_GLOBAL float* gout = glb(A.gbar);
#pragma unroll
        for (int q = 0; q < 9; ++q) gout[(size_t)q * ncell + c] += rb + (float)kCX[q] * jb.x + (float)kCY[q] * jb.y;
      }
    }
    __syncthreads();
  }
}

#define MC_ADJ_PACK(KERNEL, G, ...)                                              \
  do {                                                                           \
    if ((G).pack == 256)                                                         \
      KERNEL<256><<<(G).node_blocks, 256, 0, s>>>(__VA_ARGS__);                  \
    else                                                                         \
      KERNEL<1024><<<(G).node_blocks, 1024, 0, s>>>(__VA_ARGS__);                \
  } while (0)

// One launch of a tile kernel per tile family present.
#define MC_ADJ_TILES(KERNEL, G, ...)                                                              \
  do {                                                                                            \
    if ((G).tile_blocks[0] > 0) KERNEL<16><<<(G).tile_blocks[0], TileCfg<16>::kThreads, 0, s>>>(__VA_ARGS__); \
    if ((G).tile_blocks[1] > 0) KERNEL<32><<<(G).tile_blocks[1], TileCfg<32>::kThreads, 0, s>>>(__VA_ARGS__); \
    if ((G).tile_blocks[2] > 0) KERNEL<64><<<(G).tile_blocks[2], TileCfg<64>::kThreads, 0, s>>>(__VA_ARGS__); \
  } while (0)

// A tile kernel with a second template argument, once per tile family present.
#define MC_ADJ_TILES2(KERNEL, ARG, G, ...)                                                        \
  do {                                                                                            \
    if ((G).tile_blocks[0] > 0) KERNEL<16, ARG><<<(G).tile_blocks[0], TileCfg<16>::kThreads, 0, s>>>(__VA_ARGS__); \
    if ((G).tile_blocks[1] > 0) KERNEL<32, ARG><<<(G).tile_blocks[1], TileCfg<32>::kThreads, 0, s>>>(__VA_ARGS__); \
    if ((G).tile_blocks[2] > 0) KERNEL<64, ARG><<<(G).tile_blocks[2], TileCfg<64>::kThreads, 0, s>>>(__VA_ARGS__); \
  } while (0)

// Single linear adjoint sub-steps, for transpose (dot-product) tests:
// 0: out = S[v] (spread of a node vector, the transpose of the gather);
// 1: A.sbar = G D^T A.Gbar (filter and central difference transposed);
// 2: A.gbar = J^T A.gbar_in at the world's populations and grid force (the
//    collision and streaming Jacobian transposed; A.ubar must be zero).
void launch_adjoint_debug(const WorldDev* W, const Tables& T, const Grid& G, int which, const AdjDev& A,
                          const float* v, float2* out, hipStream_t s) {
  AdjArg a{};
  a.arr = nullptr;
  a.one = A;
  a.one.dbg_v = v;
  a.one.dbg_out = out;
  if (which == 0) MC_ADJ_TILES(k_adj_spread, G, W, T, a, 4, 0);
  else if (which == 1) MC_ADJ_TILES(k_adj_filter, G, W, T, a);
  else k_adj_lbm<<<G.item_blocks, 256, 0, s>>>(W, T, a);
}

void launch_adjoint_step(const WorldDev* W, const Tables& T, const Grid& G, const AdjArg& A, int mdf, hipStream_t s) {
  if (G.any_markers) launch_markers(W, T, G, s);    // the step's marker displacements, from x_t
  MC_ADJ_TILES(k_adj_spread, G, W, T, A, 0, 0);
  k_adj_lbm<<<G.item_blocks, 256, 0, s>>>(W, T, A);
  if (mdf > 1) {
    // recompute the step's MDF: moments, U_d, F_grid_1 = S[F], then
    // F_grid_{k+1} = F_grid_k + S[c_k] up to K - 1
    launch_mdf_moments(W, T, G, s);
    k_adj_mdf_zero<<<dim3(32, G.world_blocks), 256, 0, s>>>(W, T, A);
    const auto fwd_gather = [&](auto desired, int k) {
      for_tile_variants(G, [&](auto tile, auto mk) {
        constexpr int TL = decltype(tile)::value;
        k_adj_mdf_fwd_gather<TL, decltype(desired)::value, decltype(mk)::value>
            <<<G.tile_blocks[TileCfg<TL>::kFamily], TileCfg<TL>::kThreads, 0, s>>>(W, T, A, k);
      });
    };
    const auto node_pass = [&](auto mode, int k) {
      for_tile_variants(G, [&](auto tile, auto mk) {
        constexpr int TL = decltype(tile)::value;
        k_adj_mdf_node<TL, decltype(mode)::value, decltype(mk)::value>
            <<<G.tile_blocks[TileCfg<TL>::kFamily], TileCfg<TL>::kThreads, 0, s>>>(W, T, A, k);
      });
    };
    fwd_gather(std::true_type(), 0);
    MC_ADJ_TILES(k_adj_spread, G, W, T, A, 2, 0);
    for (int k = 1; k <= mdf - 2; ++k) {
      fwd_gather(std::false_type(), k);
      MC_ADJ_TILES(k_adj_spread, G, W, T, A, 3, k);
    }
    // reverse: iterations K - 1 .. 1 (the grid-force adjoint becomes dL/dF_grid_k), then U_d
    for (int k = mdf - 1; k >= 1; --k) {
      node_pass(std::integral_constant<int, 0>(), k);
      MC_ADJ_TILES2(k_adj_mdf_cell, 0, G, W, T, A, k);
    }
    node_pass(std::integral_constant<int, 1>(), 0);
    MC_ADJ_TILES2(k_adj_mdf_cell, 1, G, W, T, A, 0);
  }
  for_tile_variants(G, [&](auto tile, auto mk) {
    constexpr int TL = decltype(tile)::value;
    k_adj_force<TL, decltype(mk)::value><<<G.tile_blocks[TileCfg<TL>::kFamily], TileCfg<TL>::kThreads, 0, s>>>(W, T, A);
  });
  if (G.any_markers) MC_ADJ_PACK(k_adj_markers, G, W, T, A);
  MC_ADJ_TILES(k_adj_spread, G, W, T, A, 1, 0);
  MC_ADJ_TILES(k_adj_filter, G, W, T, A);
  const auto pbd = [&](auto gen, auto br, auto it) {
    constexpr bool GN = decltype(gen)::value, B = decltype(br)::value;
    constexpr int I = decltype(it)::value;
    if (G.pack == 256)
      k_adj_pbd<256, GN, B, I><<<G.node_blocks, 256, 0, s>>>(W, T, A);
    else
      k_adj_pbd<1024, GN, B, I><<<G.node_blocks, 1024, 0, s>>>(W, T, A);
  };
  const auto pbd_iters = [&](auto gen, auto br) {
    if (G.pbd_max <= 4)
      pbd(gen, br, std::integral_constant<int, 4>());
    else
      pbd(gen, br, std::integral_constant<int, kMaxAdjIters>());
  };
  using T_ = std::true_type;
  using F_ = std::false_type;
  if (G.branches)
    pbd_iters(T_(), T_());
  else if (G.general)
    pbd_iters(T_(), F_());
  else
    pbd_iters(F_(), F_());
}

}  // namespace mc
