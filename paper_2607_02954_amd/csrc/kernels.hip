// Forward kernels of the filament-fluid step for gfx950 (CDNA4).
//
// Step order (one launch per sub-step, all worlds of a table at once):
//   k_elastic     S0 actuation + S1 PBD Cosserat projection (Eqs. 1-4) -> node
//                 elastic force; writes each node's record into its
//                 home-tile bin (binned transfer)
//   k_filter      S2 deposit + S3 separable circular Gaussian filter on a
//                 32x32 tile with an (R+1)-cell halo, all in LDS; writes the
//                 central difference G = D s~ of the filtered density
//   k_repulse     S4 repulsion -k_rep sum W G -> total node force (sorted
//                 and direct transfers)
//   k_spread      S5 force spread onto a 32x32 tile, summed in LDS; for the
//                 binned transfer it also forms S4 for the nodes it spreads
//   k_lbm         S6 D2Q9 TRT/Guo collision and push streaming over
//                 contiguous cells; exports u
//   k_integrate   S7 gather u at the nodes and move them; counts the nodes
//                 of every home tile at the new positions (binned transfer)
//   k_bin_scan    per-world prefix of those counts: the bin starts of the
//                 next step (binned transfer)
//
// Particle -> grid transfer has three modes, chosen per world:
//   binned  nodes are binned by the 32x32 tile of their home cell; each tile
//           reads the bins of its neighbourhood and sums the contributions in
//           LDS as 64-bit fixed point (integer adds: order-independent, so
//           results are bitwise reproducible, and on this chip integer LDS
//           atomics are far faster than float ones), then writes every cell
//           once: no HBM atomics and no clearing pass
//   sorted  nodes are counting-sorted by home cell and every grid value is a
//           fixed-order sum over the sorted segments of its 4x4 home window:
//           bitwise reproducible
//   direct  global float atomics into HBM accumulators (reference point)
//
// Node kernels run one block per node pack (whole filaments, <= pack nodes,
// filament-contiguous SoA), so neighbour exchange along a chain stays in LDS.
// Positions are an integer cell plus a float fraction, so the quantities the
// physics needs (edge vectors, kernel offsets) are formed from small numbers.
#include <hip/hip_ext.h>

#include "device_util.h"

namespace mc {


// ---------------------------------------------------------------------------
// S0 + S1: actuation and PBD elastic force.  Then, by transfer mode: the
// node's record in its home-tile bin (binned), home-cell key and rank
// (sorted) or the density deposit with global atomics (direct).
// ---------------------------------------------------------------------------
// GEN: worlds may pass closed-loop flags and per-edge stiffness arrays, BR
// (with GEN) branches as well; the plain variant serves open chains with the
// world's scalar stiffnesses.
//
// Branches: the first node c0 of a filament that hangs from node p (of the
// same pack: packs hold whole creatures) owns the attachment edge p -> c0,
// whose angle lives in s_ta at c0's slot, and its two joints; after the
// regular colours of each pass come the joints at the parent nodes, then
// those at the first nodes (bending), and the attachment edges (position).
// A node carries at most one attachment, so each of those phases touches
// every angle and node once at most.
template <int PACK, bool GEN, bool BR>
__global__ __launch_bounds__(PACK) void k_elastic(const WorldDev* __restrict__ W, Tables T) {
  static_assert(GEN || !BR, "branches take the general variant");
  __shared__ float s_th[PACK];
  __shared__ float s_dx[PACK];
  __shared__ float s_dy[PACK];
  __shared__ float s_ta[BR ? PACK : 1];
  __shared__ int s_off[PACK + 1];

  const int npk = *T.n_packs;
  const int li = threadIdx.x;
  for (int it = blockIdx.x; it < npk; it += gridDim.x) {
    const Pack pk = T.packs[it];
    const WorldDev& w = W[pk.world];
    const Ctl ctl = *w.ctl_src;
    if (ctl.remaining <= 0) continue;           // block-uniform
    const int N = w.n_part, nx = w.nx, ny = w.ny, mode = w.mode;
    const MC_GLOBAL int* cell = glb(w.cell_in);
    const MC_GLOBAL float* frac = glb(w.frac_in);
    const MC_GLOBAL int* foff = glb(w.fil_offset);
    const int nf = pk.fil_end - pk.fil_begin;
    // every load this node needs is issued before anything waits: the
    // filament offsets first (they go to LDS), then the node's own data at
    // clamped indices (lanes past the pack's end, and the pack's last node
    // for its successor, read an in-range node and ignore it)
    const int off_a = foff[pk.fil_begin + min(li, nf)];      // nf <= PACK filaments
    const int off_b = foff[pk.fil_begin + nf];
    __builtin_amdgcn_sched_barrier(0);           // keep these two loads ahead of the node loads
    const int gi = pk.node_begin + li;
    const bool active = gi < pk.node_end;
    const int gic = min(gi, pk.node_end - 1);
    const int gin = min(gic + 1, N - 1);
    const int c0x = cell[gic], c0y = cell[N + gic];
    const float f0x = frac[gic], f0y = frac[N + gic];
    int c1x = cell[gin], c1y = cell[N + gin];
    float f1x = frac[gin], f1y = frac[N + gin];
    const float L_r = glb(w.rest_length)[gic];
    const float ra = glb(w.rest_angle)[gic];
    // per-edge stiffnesses (joint and edge at this node), else the world's
    const float kb_i = GEN && w.kb_arr ? glb(w.kb_arr)[gic] : w.k_bend;
    const float ks_i = GEN && w.ks_arr ? glb(w.ks_arr)[gic] : w.k_stretch;
    const float ksh_i = GEN && w.ksh_arr ? glb(w.ksh_arr)[gic] : w.k_shear;
    if (li < nf) s_off[li] = off_a - pk.node_begin;
    if (li == 0) s_off[nf] = off_b - pk.node_begin;
    __syncthreads();

    // filament of this node: largest f with s_off[f] <= li
    int lo = 0, hi = nf - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (s_off[mid] <= li) lo = mid; else hi = mid - 1;
    }
    const int o = s_off[lo];
    const int n = s_off[lo + 1] - o;
    const int k = li - o;
    const int fil = pk.fil_begin + lo;
    // a closed loop (at least three nodes): the last node's edge joins it to
    // the first, and every node is a joint (the first between the closing
    // edge and edge 0)
    const bool ring = GEN && w.fil_flags && (glb(w.fil_flags)[fil] & 1) && n >= 3;
    const bool has_edge = active && (k < n - 1 || ring);
    const bool is_joint = active && (ring || (k >= 1 && k <= n - 2));
    const int j = ring ? k : k - 1;              // joint's local index
    const int m = ring ? n : n - 2;              // joints of the filament
    const int li_prev = (ring && k == 0) ? o + n - 1 : li - 1;    // edge before the joint
    const int li_next = (ring && k == n - 1) ? o : li + 1;        // far node of the edge
    if (ring && k == n - 1) {                    // the closing edge's far node: the first
      const int g0 = pk.node_begin + o;
      c1x = cell[g0];
      c1y = cell[N + g0];
      f1x = frac[g0];
      f1y = frac[N + g0];
    }
    // Gauss-Seidel colours: local parity; on a loop of odd length the last
    // joint and the last edge meet the first ones and take a third colour
    const int jcol = (ring && (n & 1) && j == n - 1) ? 2 : (j & 1);
    const int ecol = (ring && (n & 1) && k == n - 1) ? 2 : (k & 1);
    int ncol = 2;                                // block-uniform
    if constexpr (GEN) ncol = __syncthreads_or(active && ring && (n & 1)) ? 3 : 2;
    const float amp = glb(w.act_amp)[fil], period = glb(w.act_period)[fil], phase = glb(w.act_phase)[fil];

    const int cx = active ? c0x : 0, cy = active ? c0y : 0;
    const float fx = active ? f0x : 0.f, fy = active ? f0y : 0.f;
    float v0x = 0.f, v0y = 0.f, L = 0.f, th = 0.f;
    float u0x = 1.f, u0y = 0.f;                  // unit edge direction, (cos th, sin th)
    if (has_edge) {
      v0x = (float)(c1x - cx) + (f1x - fx);
      v0y = (float)(c1y - cy) + (f1y - fy);
      L = L_r;
      th = atan2f(v0y, v0x);
      const float l0 = hw_sqrt(v0x * v0x + v0y * v0y);
      if (l0 > 0.f) {
        const float il = hw_rcp(l0);
        u0x = v0x * il;
        u0y = v0y * il;
      }
    }
    float th_hat = 0.f;
    if (is_joint) th_hat = actuated_angle(ra, amp, period, phase, ctl.t, j, m);
    s_th[li] = th;
    s_dx[li] = 0.f;
    s_dy[li] = 0.f;
    // branch attachment owned by this node (its filament's first node)
    bool att = false, att_cj = false, any_att = false;
    int p_l = 0, in_l = 0;
    float a_vx = 0.f, a_vy = 0.f, a_th = 0.f, a_ux = 1.f, a_uy = 0.f, a_L = 0.f, a_al = 0.f, a_be = 0.f;
    if (BR && w.fil_parent) {                    // block-uniform: the pack's world
      const int par = (active && k == 0) ? glb(w.fil_parent)[fil] : -1;
      att = par >= 0;
      if (att) {
        p_l = par - pk.node_begin;
        int lp = 0, hp = nf - 1;                   // p's filament: largest f with s_off[f] <= p_l
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
    __syncthreads();
    const float hb_w = 0.5f * w.k_bend, hs_w = 0.5f * w.k_stretch, ksh_w = w.k_shear;

    const float hb = 0.5f * kb_i;
    const float hs = 0.5f * ks_i;
    const float ksh = ksh_i;
    const int iters = w.pbd_iters;
    for (int iter = 0; iter < iters; ++iter) {
      // bending pass (Eq. 1): even joints, then odd joints (then a loop's third colour)
      for (int par = 0; par < ncol; ++par) {
        if (is_joint && jcol == par) {
          const float t1 = s_th[li_prev];
          const float t2 = s_th[li];
          const float c = wrap_angle(t2 - t1) - th_hat;
          s_th[li_prev] = t1 + hb * c;
          s_th[li] = t2 - hb * c;
        }
        __syncthreads();
      }
      if (BR && any_att) {                       // attachment joints: at p, then at c0
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
      // the edge directions of this iteration (the angles change only in the
      // bending passes), for every lane at once rather than per colour
      float cs = 1.f, sn = 0.f;
      if (has_edge) edge_direction(s_th[li], th, u0x, u0y, &cs, &sn);
      float a_cs = 1.f, a_sn = 0.f;
      if (BR && att) edge_direction(s_ta[li], a_th, a_ux, a_uy, &a_cs, &a_sn);
      // position pass (Eqs. 2-4): even edges, then odd edges (then the third colour)
      for (int par = 0; par < ncol; ++par) {
        if (has_edge && ecol == par) {
          const float d0x = s_dx[li], d0y = s_dy[li];
          const float d1x = s_dx[li_next], d1y = s_dy[li_next];
          const float vx = v0x + (d1x - d0x);
          const float vy = v0y + (d1y - d0y);
          const float ell = hw_sqrt(vx * vx + vy * vy);
          const float sc = (ell - L) * hw_rcp(ell);
          const float csx = sc * vx, csy = sc * vy;
          const float dx = hs * (csx + ksh * (vx - L * cs - csx));
          const float dy = hs * (csy + ksh * (vy - L * sn - csy));
          s_dx[li] = d0x + dx;
          s_dy[li] = d0y + dy;
          s_dx[li_next] = d1x - dx;
          s_dy[li_next] = d1y - dy;
        }
        __syncthreads();
      }
      if (BR && any_att) {                       // attachment edges p -> c0
        if (att) {
          const float d0x = s_dx[p_l], d0y = s_dy[p_l];
          const float d1x = s_dx[li], d1y = s_dy[li];
          const float vx = a_vx + (d1x - d0x);
          const float vy = a_vy + (d1y - d0y);
          const float ell = hw_sqrt(vx * vx + vy * vy);
          const float sc = (ell - a_L) * hw_rcp(ell);
          const float csx = sc * vx, csy = sc * vy;
          const float dx = hs_w * (csx + ksh_w * (vx - a_L * a_cs - csx));
          const float dy = hs_w * (csy + ksh_w * (vy - a_L * a_sn - csy));
          s_dx[p_l] = d0x + dx;
          s_dy[p_l] = d0y + dy;
          s_dx[li] = d1x - dx;
          s_dy[li] = d1y - dy;
        }
        __syncthreads();
      }
    }

    const int bx = wrap_index(cx, nx);
    const int by = wrap_index(cy, ny);
    if (active) {
      MC_GLOBAL float* fel = glb(w.fel_el);
      fel[gi] = w.k_el * s_dx[li];
      fel[N + gi] = w.k_el * s_dy[li];
    }
    if (mode == kBinned) {
      // this node's record in its home-tile bin (bins sized by the counts
      // of these positions: the previous step's integrate or the pre-pass)
      const int tile = bin_of(bx, by, w.ntx, w.tile_shift);
      const int slot = agg_atomic_inc(glb(w.bin_fill), tile, active);
      if (active) {
        const MC_GLOBAL int* bstart = glb(w.bin_start);
        const int e = bstart[tile] + slot;
        if (e < bstart[tile + 1]) {
          const vi4 rec = {bx | (by << 16), __float_as_int(fx), __float_as_int(fy), gi};
          glbv<vi4>(w.bin_rec)[e] = rec;
        } else {
          atomicOr((unsigned*)glb(w.flags), kFlagBins);
        }
      }
    } else if (active && mode == kSorted) {
      const int key = by * nx + bx;
      glb(w.key)[gi] = key;
      glb(w.rank)[gi] = atomicAdd((int*)(glb(w.cnt) + key), 1);
    } else if (active) {
      float wx[4], wy[4];
      peskin4(fx, wx);
      peskin4(fy, wy);
      int ix[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) ix[a] = wrap_near(bx - 1 + a, nx);
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        MC_GLOBAL float* row = glb(w.s) + (size_t)wrap_near(by - 1 + b, ny) * nx;
#pragma unroll
        for (int a = 0; a < 4; ++a) unsafeAtomicAdd((float*)(row + ix[a]), wx[a] * wy[b]);
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Binned transfer: per-world exclusive scan of the home-tile counts; every
// node then writes one record (home cell, fractions, index) into its bin.
// ---------------------------------------------------------------------------
// next: write the starts for the next step's bins (bin_start_next; after
// integrate) rather than for the current positions (bin_start; pre-pass).
// Every node has exactly one record, so the counts must add up to the
// world's node count: the starts are clamped to it (no bin range can leave
// the record buffer) and a mismatch raises kFlagBins.
__global__ __launch_bounds__(1024) void k_bin_scan(const WorldDev* __restrict__ W, Tables T, int next) {
  // every thread sums 4 consecutive bins (one 16-byte load), the wavefronts
  // scan those sums with shuffles, one exchange of the 16 wavefront totals;
  // a round covers 4096 bins
  __shared__ int s_tot[16];
  const int nw = *T.n_worlds;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int it = blockIdx.x; it < nw; it += gridDim.x) {
    const WorldDev& w = W[T.worlds[it].x];
    if (w.mode != kBinned || w.ctl_src->remaining <= 0) continue;
    MC_GLOBAL int* cnt = glb(w.bin_cnt);
    MC_GLOBAL int* fill = glb(w.bin_fill);
    MC_GLOBAL int* start = glb(next ? w.bin_start_next : w.bin_start);
    const int nt = w.ntx * w.nty;               // bins (one per tile)
    const int N = w.n_part;
    int carry = 0;
    for (int c0 = 0; c0 < nt; c0 += 4096) {
      const int i0 = c0 + 4 * tid;              // a multiple of 4: 16-byte aligned
      const bool whole = i0 + 3 < nt;
      vi4 v = {0, 0, 0, 0};
      if (whole) {
        v = *(const MC_GLOBAL vi4*)(cnt + i0);
      } else {
        if (i0 < nt) v.x = cnt[i0];
        if (i0 + 1 < nt) v.y = cnt[i0 + 1];
        if (i0 + 2 < nt) v.z = cnt[i0 + 2];
      }
      const int sum = v.x + v.y + v.z + v.w;
      int x = sum;
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(x, off);
        if (lane >= off) x += y;
      }
      if (lane == 63) s_tot[wv] = x;
      __syncthreads();
      int before = carry, all = 0;
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int t = s_tot[j];
        before += j < wv ? t : 0;
        all += t;
      }
      __syncthreads();
      const int e = before + x - sum;           // start of bin i0
      const vi4 st = {min(e, N), min(e + v.x, N), min(e + v.x + v.y, N), min(e + v.x + v.y + v.z, N)};
      const vi4 zero = {0, 0, 0, 0};
      if (whole) {
        *(MC_GLOBAL vi4*)(start + i0) = st;
        *(MC_GLOBAL vi4*)(cnt + i0) = zero;
        *(MC_GLOBAL vi4*)(fill + i0) = zero;
      } else {
        if (i0 < nt) { start[i0] = st.x; cnt[i0] = 0; fill[i0] = 0; }
        if (i0 + 1 < nt) { start[i0 + 1] = st.y; cnt[i0 + 1] = 0; fill[i0 + 1] = 0; }
        if (i0 + 2 < nt) { start[i0 + 2] = st.z; cnt[i0 + 2] = 0; fill[i0 + 2] = 0; }
      }
      carry += all;
    }
    if (tid == 0) {
      start[nt] = min(carry, N);
      if (carry != N) atomicOr((unsigned*)glb(w.flags), kFlagBins);
    }
  }
}

// Pre-pass: tile-bin counts of the current positions (a rollout's first step
// needs them; later steps get them from the previous step's integrate).
template <int PACK>
__global__ __launch_bounds__(PACK) void k_bin_count(const WorldDev* __restrict__ W, Tables T) {
  const int npk = *T.n_packs;
  for (int it = blockIdx.x; it < npk; it += gridDim.x) {
    const Pack pk = T.packs[it];
    const WorldDev& w = W[pk.world];
    if (w.mode != kBinned || w.ctl_src->remaining <= 0) continue;
    const int N = w.n_part;
    const int gi = pk.node_begin + threadIdx.x;
    const bool active = gi < pk.node_end;
    int tile = 0;
    if (active)
      tile = bin_of(wrap_index(glb(w.cell_in)[gi], w.nx), wrap_index(glb(w.cell_in)[N + gi], w.ny), w.ntx, w.tile_shift);
    agg_atomic_inc(glb(w.bin_cnt), tile, active);
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
    const MC_GLOBAL int* cnt = glb(w.cnt);
    const int ncell = w.nx * w.ny;
    const int c0 = sc.y * kScanBlock + threadIdx.x * 4;
    int v = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) v += (c0 + k < ncell) ? cnt[c0 + k] : 0;
    int total;
    block_scan256(v, s_wave, &total);
    if (threadIdx.x == 0) glb(w.part)[sc.y] = total;
  }
}

__global__ __launch_bounds__(256) void k_scan_partials(const WorldDev* __restrict__ W, Tables T) {
  __shared__ int s_wave[4];
  const int n = *T.n_worlds;
  for (int it = blockIdx.x; it < n; it += gridDim.x) {
    const WorldDev& w = W[T.worlds[it].x];
    if (w.mode != kSorted || w.ctl_src->remaining <= 0) continue;
    MC_GLOBAL int* part = glb(w.part);
    const int ncell = w.nx * w.ny;
    const int nb = (ncell + kScanBlock - 1) / kScanBlock;
    int carry = 0;
    for (int b0 = 0; b0 < nb; b0 += 256) {
      const int b = b0 + threadIdx.x;
      const int v = b < nb ? part[b] : 0;
      int total;
      const int ex = block_scan256(v, s_wave, &total);
      if (b < nb) part[b] = carry + ex;
      carry += total;
    }
    if (threadIdx.x == 0) glb(w.start)[ncell] = carry;
  }
}

__global__ __launch_bounds__(256) void k_scan_down(const WorldDev* __restrict__ W, Tables T) {
  __shared__ int s_wave[4];
  const int n = *T.n_scan;
  for (int it = blockIdx.x; it < n; it += gridDim.x) {
    const int2 sc = T.scan[it];
    const WorldDev& w = W[sc.x];
    if (w.mode != kSorted || w.ctl_src->remaining <= 0) continue;
    MC_GLOBAL int* cnt = glb(w.cnt);
    MC_GLOBAL int* start = glb(w.start);
    const int ncell = w.nx * w.ny;
    const int c0 = sc.y * kScanBlock + threadIdx.x * 4;
    int v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = (c0 + k < ncell) ? cnt[c0 + k] : 0;
    int total;
    const int ex = block_scan256(v[0] + v[1] + v[2] + v[3], s_wave, &total);
    int run = glb(w.part)[sc.y] + ex;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (c0 + k < ncell) {
        start[c0 + k] = run;
        cnt[c0 + k] = 0;          // ready for the next step's histogram
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
    glb(w.perm)[glb(w.start)[glb(w.key)[gi]] + glb(w.rank)[gi]] = gi;
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
    if (gi >= pk.node_end || glb(w.rank)[gi] != 0) continue;
    MC_GLOBAL int* perm = glb(w.perm);
    const int key = glb(w.key)[gi];
    const int b = glb(w.start)[key], e = glb(w.start)[key + 1];
    for (int i = b + 1; i < e; ++i) {
      const int v = perm[i];
      int j = i - 1;
      while (j >= b && perm[j] > v) {
        perm[j + 1] = perm[j];
        --j;
      }
      perm[j + 1] = v;
    }
    // fractions of the sorted nodes for the density gather of this step
    const int N = w.n_part;
    const MC_GLOBAL float* frac = glb(w.frac_in);
    MC_GLOBAL vf4* rec = glbv<vf4>(w.rec);
    for (int i = b; i < e; ++i) {
      const int v = perm[i];
      const vf4 r = {frac[v], frac[N + v], 0.f, 0.f};
      rec[i] = r;
    }
  }
}

// Fixed-order sums over the sorted segments of the 4x4 home window of cell
// (gx, gy): the node at home cell h contributes weight index c - h + 1.
__device__ __forceinline__ float gather_density(const MC_GLOBAL int* start, const MC_GLOBAL vf4* rec,
                                                int nx, int ny, int gx, int gy) {
  float acc = 0.f;
  for (int b = 0; b < 4; ++b) {
    const int hy = wrap_near(gy + 1 - b, ny);
    for (int a = 0; a < 4; ++a) {
      const int h = hy * nx + wrap_near(gx + 1 - a, nx);
      const int e = start[h + 1];
      for (int sidx = start[h]; sidx < e; ++sidx) {
        const vf4 r = rec[sidx];
        float wx[4], wy[4];
        peskin4(r.x, wx);
        peskin4(r.y, wy);
        acc += wx[a] * wy[b];
      }
    }
  }
  return acc;
}

__device__ __forceinline__ vf2 gather_force(const MC_GLOBAL int* start, const MC_GLOBAL vf4* rec,
                                               int nx, int ny, int gx, int gy) {
  float Fx = 0.f, Fy = 0.f;
  for (int b = 0; b < 4; ++b) {
    const int hy = wrap_near(gy + 1 - b, ny);
    for (int a = 0; a < 4; ++a) {
      const int h = hy * nx + wrap_near(gx + 1 - a, nx);
      const int e = start[h + 1];
      for (int sidx = start[h]; sidx < e; ++sidx) {
        const vf4 r = rec[sidx];
        float wx[4], wy[4];
        peskin4(r.x, wx);
        peskin4(r.y, wy);
        const float ww = wx[a] * wy[b];
        Fx += ww * r.z;
        Fy += ww * r.w;
      }
    }
  }
  const vf2 out = {Fx, Fy};
  return out;
}

// ---------------------------------------------------------------------------
// S2 + S3: density on a tile (side TILE) plus an (R+1)-cell halo, staged in LDS,
// the separable circular Gaussian (x pass, then y pass, both in LDS) on the
// tile plus a one-cell ring, and the central difference G = D s~ of the
// tile, written as interleaved float2.
//
// Binned mode deposits the neighbourhood's nodes into a padded window (three
// spare cells per side, see the window note with tile_spread_vec) as exact
// integer products of quantised weights, so the sums are order-independent
// and the inner loop is two 24-bit multiplies and an LDS add per cell.
// Dynamic LDS: [window: filter_window_bytes(max radius) | list / density].
// ---------------------------------------------------------------------------
// Window rows are kWinPad elements longer than the window side: an even
// row length of 64-bit words puts vertically adjacent cells, which nodes
// next to each other on a chain often deposit to at once, in the same LDS bank.
constexpr int kWinPad = 1;
template <int TILE>
static __host__ __device__ constexpr int filter_window_bytes(int max_radius) {
  return (TILE + 2 + 2 * max_radius + 6) * (TILE + 2 + 2 * max_radius + 6 + kWinPad) * 8;
}
template <int TILE>
static __host__ __device__ constexpr int filter_list_bytes(int max_radius) {
  return (TILE + 2 + 2 * max_radius) * (TILE + 2 + 2 * max_radius) * 4 > TileCfg<TILE>::kListBytes
             ? (TILE + 2 + 2 * max_radius) * (TILE + 2 + 2 * max_radius) * 4
             : TileCfg<TILE>::kListBytes;
}
// the passes' intermediate rows (region x ring) and the filtered ring fit the window
static_assert(filter_window_bytes<16>(1) >= ((16 + 2 + 2 * kMaxRadius) * 18 + 18 * 18) * 4, "window");
static_assert(filter_window_bytes<32>(1) >= ((32 + 2 + 2 * kMaxRadius) * 34 + 34 * 34) * 4, "window");
static_assert(filter_window_bytes<64>(1) >= ((64 + 2 + 2 * kMaxRadius) * 66 + 66 * 66) * 4, "window");

// q = k / d for 0 <= k < 2^16 and 0 < d <= 64: (k + 1/2) / d is at least
// 1/(2d) away from an integer, far beyond the FP32 rounding of the product.
static __device__ __forceinline__ int div_small(int k, float inv_d) {
  return (int)(((float)k + 0.5f) * inv_d);
}

// The bin set a filter tile reads: homes in [xo - 2, xo + reg] per axis
// (xo = x0 - R - 1, reg = TILE + 2 + 2R), whose supports meet the density
// region (run table kind 0).
template <int TILE>
static __device__ __forceinline__ BinFetch filter_fetch(const WorldDev& w, int tile) {
  return binset_fetch<TileCfg<TILE>::kRanges>(w, tile_y(tile) * w.ntx + tile_x(tile), 0);
}

// Set-up: the runs of bins that the filter and the spread of every tile read
// (they depend on the grid, the tile side and the radius only).
template <int TILE>
__global__ void k_tile_ranges(int nx, int ny, int R, int2* out) {
  const int ntx = (nx + TILE - 1) / TILE, nty = (ny + TILE - 1) / TILE;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < ntx * nty; t += gridDim.x * blockDim.x) {
    const int x0 = (t % ntx) * TILE, y0 = (t / ntx) * TILE;
    const int tw = min(TILE, nx - x0), th = min(TILE, ny - y0);
    const int reg = TILE + 2 + 2 * R, xo = x0 - R - 1, yo = y0 - R - 1;
    tile_runs<TILE>(xo - 2, xo + reg, yo - 2, yo + reg, nx, ny, ntx, out + (size_t)(2 * t) * kRunStride);
    tile_runs<TILE>(x0 - 3, x0 + tw + 1, y0 - 3, y0 + th + 1, nx, ny, ntx, out + (size_t)(2 * t + 1) * kRunStride);
  }
}

// The two passes of the separable Gaussian (radius R) over the density
// region s_regf (reg x reg, reg = ring + 2R) into the filtered tile-plus-ring
// s_st (ring x ring, ring = TILE + 2), through s_mid (reg rows x ring).
// Every thread forms two adjacent outputs from taps read as aligned pairs
// (rows have even lengths); each output is summed in the same order as a
// one-output loop would.  Ends with a barrier.
template <int TILE, int R>
static __device__ __forceinline__ void filter_passes(const float* s_regf, float* s_mid, float* s_st, const float* g) {
  constexpr int kRing = TILE + 2, kThreads = TileCfg<TILE>::kThreads;
  constexpr int reg = kRing + 2 * R, kHalf = kRing / 2;
  const int tid = threadIdx.x;
  for (int k = tid; k < reg * kHalf; k += kThreads) {
    const int r = k / kHalf, c = 2 * (k - (k / kHalf) * kHalf);
    const vf2* row = (const vf2*)(s_regf + r * reg + c);   // cells c .. c + 2R + 1 of row r
    float v[2 * R + 2];
#pragma unroll
    for (int i = 0; i <= R; ++i) {
      const vf2 t = row[i];
      v[2 * i] = t.x;
      v[2 * i + 1] = t.y;
    }
    float a0 = g[0] * v[R], a1 = g[0] * v[R + 1];
#pragma unroll
    for (int m = 1; m <= R; ++m) {
      a0 += g[m] * (v[R - m] + v[R + m]);
      a1 += g[m] * (v[R + 1 - m] + v[R + 1 + m]);
    }
    const vf2 out = {a0, a1};
    *(vf2*)(s_mid + r * kRing + c) = out;
  }
  __syncthreads();
  for (int k = tid; k < kRing * kHalf; k += kThreads) {
    const int r = k / kHalf, c = 2 * (k - (k / kHalf) * kHalf);
    const vf2* col = (const vf2*)(s_mid + (r + R) * kRing + c);
    vf2 t[2 * R + 1];
#pragma unroll
    for (int m = -R; m <= R; ++m) t[m + R] = col[m * kHalf];
    float a0 = g[0] * t[R].x, a1 = g[0] * t[R].y;
#pragma unroll
    for (int m = 1; m <= R; ++m) {
      a0 += g[m] * (t[R - m].x + t[R + m].x);
      a1 += g[m] * (t[R - m].y + t[R + m].y);
    }
    const vf2 out = {a0, a1};
    *(vf2*)(s_st + r * kRing + c) = out;
  }
  __syncthreads();
}

template <int TILE>
__global__ __launch_bounds__(TileCfg<TILE>::kThreads) void k_filter(const WorldDev* __restrict__ W, Tables T,
                                                                     int window_bytes) {
  using C = TileCfg<TILE>;
  constexpr int kRing = TILE + 2, kThreads = C::kThreads, kSpreadCap = C::kSpreadCap;
  extern __shared__ __align__(16) unsigned char smem[];
  unsigned long long* s_win = (unsigned long long*)smem;
  vi4* s_list = (vi4*)(smem + window_bytes);
  float* s_regf = (float*)(smem + window_bytes);
  float* s_mid = (float*)smem;
  __shared__ int s_spn;                          // records appended to the spread list
  const int nt = n_tiles<TILE>(T);
  const int tid = threadIdx.x;
  const XcdLoop tiles(nt);
  for (int it = tiles.first; it < tiles.end; it += tiles.step) {
    const int2 tl = tile_entry<TILE>(T, it);
    const WorldDev& w = W[tl.x];
    if (w.ctl_src->remaining <= 0) continue;
    const int R = w.radius, mode = w.mode;
    const int nx = w.nx, ny = w.ny;
    const int x0 = tile_x(tl.y) * TILE;
    const int y0 = tile_y(tl.y) * TILE;
    const int reg = kRing + 2 * R;
    const float inv_reg = 1.0f / (float)reg;
    const int xo = x0 - R - 1, yo = y0 - R - 1;   // region origin (unwrapped)
    float* s_st = s_mid + reg * kRing;
    if (mode == kBinned) {
      const int S = reg + 6;                      // window side; window origin (xo - 3, yo - 3)
      const int P = S + kWinPad;                  // row pitch
      zero_lds_u64(s_win, S * P);
      if (tid == 0) s_spn = 0;
      const auto bs = binset_commit<C::kRanges>(filter_fetch<TILE>(w, tl.y));
      const int ox = wrap_index(xo - 3, nx), oy = wrap_index(yo - 3, ny);
      const int keep_x = reg + 3 <= nx ? reg + 2 : nx;
      const int keep_y = reg + 3 <= ny ? reg + 2 : ny;
      // the records this tile's spread needs (a subset of the filter's: its
      // window lies inside the filter's) go to the tile's spread list
      const int tix = tile_y(tl.y) * w.ntx + tile_x(tl.y);
      const SpreadKeep sp_keep(w, x0, y0, min(TILE, nx - x0), min(TILE, ny - y0));
      MC_GLOBAL vi4* sp_rec = glbv<vi4>(w.sp_rec) + (size_t)tix * kSpreadCap;
      for_bin_records<4, kThreads>(
          glbv<const vi4>(w.bin_rec), bs, s_list,
          [&](const vi4& r) {
            const int dx = wrap_near((r.x & 0xffff) - 1 - ox, nx);
            const int dy = wrap_near((r.x >> 16) - 1 - oy, ny);
            return dx <= keep_x && dy <= keep_y;
          },
          [&](const vi4& r) {
            const int dx = wrap_near((r.x & 0xffff) - 1 - ox, nx);
            const int dy = wrap_near((r.x >> 16) - 1 - oy, ny);
            unsigned qx[4], qy[4];
            peskin4_quant(__int_as_float(r.y), qx);
            peskin4_quant(__int_as_float(r.z), qy);
            unsigned long long* p = s_win + dy * P + dx;
#pragma unroll
            for (int b = 0; b < 4; ++b)
#pragma unroll
              for (int a = 0; a < 4; ++a) atomicAdd(p + b * P + a, weight_product(qx[a], qy[b]));
            // append to the spread list: one LDS atomic per wavefront
            const bool sp = sp_keep(r);
            const unsigned long long m = __ballot(sp);
            if (m) {
              const int leader = __ffsll((unsigned long long)m) - 1;
              int base = 0;
              if (__lane_id() == leader) base = atomicAdd(&s_spn, __popcll(m));
              base = __shfl(base, leader);
              const int slot = base + __popcll(m & ((1ull << __lane_id()) - 1ull));
              if (sp && slot < kSpreadCap) sp_rec[slot] = r;
            }
          });
      if (tid == 0) glb(w.sp_cnt)[tix] = s_spn;   // (for_bin_records ended with a barrier)
      // (the list area is free again after the barrier that ends for_bin_records)
      const bool single = reg + 3 <= nx && reg + 3 <= ny;   // one image per needed cell
      for (int k = tid; k < reg * reg; k += kThreads) {
        const int r = div_small(k, inv_reg), c = k - r * reg;
        unsigned long long v;
        if (single) {
          v = s_win[(r + 3) * P + c + 3];
        } else {
          v = 0;
          for (int cy = first_image(r, ny); cy < S; cy += ny)
            for (int cx = first_image(c, nx); cx < S; cx += nx) v += s_win[cy * P + cx];
        }
        s_regf[k] = density_to_float(v);
      }
    } else if (mode == kSorted) {
      const MC_GLOBAL int* start = glb(w.start);
      const MC_GLOBAL vf4* rec = glbv<const vf4>(w.rec);
      for (int k = tid; k < reg * reg; k += kThreads) {
        const int r = div_small(k, inv_reg), c = k - r * reg;
        s_regf[k] = gather_density(start, rec, nx, ny, wrap_index(xo + c, nx), wrap_index(yo + r, ny));
      }
    } else {
      const MC_GLOBAL float* sd = glb(w.s);
      for (int k = tid; k < reg * reg; k += kThreads) {
        const int r = div_small(k, inv_reg), c = k - r * reg;
        s_regf[k] = sd[(size_t)wrap_index(yo + r, ny) * nx + wrap_index(xo + c, nx)];
      }
    }
    float g[kMaxRadius + 1];
#pragma unroll
    for (int m = 0; m <= kMaxRadius; ++m) g[m] = w.gtap[m];
    __syncthreads();
    switch (R) {                                  // uniform: the world's radius
      case 1: filter_passes<TILE, 1>(s_regf, s_mid, s_st, g); break;
      case 2: filter_passes<TILE, 2>(s_regf, s_mid, s_st, g); break;
      case 3: filter_passes<TILE, 3>(s_regf, s_mid, s_st, g); break;
      case 4: filter_passes<TILE, 4>(s_regf, s_mid, s_st, g); break;
      case 5: filter_passes<TILE, 5>(s_regf, s_mid, s_st, g); break;
      case 6: filter_passes<TILE, 6>(s_regf, s_mid, s_st, g); break;
      case 7: filter_passes<TILE, 7>(s_regf, s_mid, s_st, g); break;
      default: filter_passes<TILE, 8>(s_regf, s_mid, s_st, g); break;
    }
    MC_GLOBAL vf2* grad = glbv<vf2>(w.grad);
    for (int k = tid; k < TILE * TILE; k += kThreads) {
      const int r = k >> C::kShift, c = k & (TILE - 1);
      const int gx = x0 + c, gy = y0 + r;
      if (gx < nx && gy < ny) {
        const float* p = s_st + (r + 1) * kRing + (c + 1);
        const vf2 gr = {0.5f * (p[1] - p[-1]), 0.5f * (p[kRing] - p[-kRing])};
        grad[(size_t)gy * nx + gx] = gr;
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// S4: repulsion F_rep = -k_rep sum_c W(c - x) G_c and the total node force.
// Direct mode also spreads it with global atomics; sorted mode runs in slot
// order and stores the node records.
// ---------------------------------------------------------------------------
template <int PACK>
__global__ __launch_bounds__(PACK) void k_repulse(const WorldDev* __restrict__ W, Tables T) {
  const int npk = *T.n_packs;
  for (int it = blockIdx.x; it < npk; it += gridDim.x) {
    const Pack pk = T.packs[it];
    const WorldDev& w = W[pk.world];
    if (w.mode == kBinned || w.ctl_src->remaining <= 0) continue;   // binned: in k_spread
    const int sl = pk.node_begin + threadIdx.x;      // node index, or sorted slot
    if (sl >= pk.node_end) continue;
    const int mode = w.mode;
    const int gi = mode == kSorted ? glb(w.perm)[sl] : sl;
    const int N = w.n_part;
    const int nx = w.nx, ny = w.ny;
    const MC_GLOBAL int* cell = glb(w.cell_in);
    const MC_GLOBAL float* frac = glb(w.frac_in);
    const MC_GLOBAL vf2* grad = glbv<const vf2>(w.grad);
    MC_GLOBAL float* fel = glb(w.fel);
    const int bx = wrap_index(cell[gi], nx);
    const int by = wrap_index(cell[N + gi], ny);
    const float fx = frac[gi], fy = frac[N + gi];
    float wx[4], wy[4];
    peskin4(fx, wx);
    peskin4(fy, wy);
    int ix[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) ix[a] = wrap_near(bx - 1 + a, nx);
    float gx = 0.f, gy = 0.f;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const MC_GLOBAL vf2* row = grad + (size_t)wrap_near(by - 1 + b, ny) * nx;
      float rx = 0.f, ry = 0.f;
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const vf2 g = row[ix[a]];
        rx += wx[a] * g.x;
        ry += wx[a] * g.y;
      }
      gx += wy[b] * rx;
      gy += wy[b] * ry;
    }
    const MC_GLOBAL float* fe = glb(w.fel_el);
    const float Fx = fe[gi] - w.k_rep * gx;
    const float Fy = fe[N + gi] - w.k_rep * gy;
    fel[gi] = Fx;
    fel[N + gi] = Fy;
    if (mode == kSorted) {
      const vf4 r = {fx, fy, Fx, Fy};
      glbv<vf4>(w.rec)[sl] = r;
    } else if (mode == kDirect && w.d_marker) {
      // two layers: half of the force from each marker
      const float dx = glb(w.d_marker)[gi], dy = glb(w.d_marker)[N + gi];
      const int cx = cell[gi], cy = cell[N + gi];
#pragma unroll
      for (int sgn = 1; sgn >= -1; sgn -= 2) {
        int hx, hy;
        float mx, my;
        marker_home(cx, fx, sgn * dx, nx, &hx, &mx);
        marker_home(cy, fy, sgn * dy, ny, &hy, &my);
        atomic_spread_vec(glb((float*)w.Fg), nx, ny, hx, hy, mx, my, 0.5f * Fx, 0.5f * Fy);
      }
    } else if (mode == kDirect) {
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        MC_GLOBAL float* row = glb((float*)w.Fg) + 2 * (size_t)wrap_near(by - 1 + b, ny) * nx;
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          const float ww = wx[a] * wy[b];
          unsafeAtomicAdd((float*)(row + 2 * ix[a]), ww * Fx);
          unsafeAtomicAdd((float*)(row + 2 * ix[a] + 1), ww * Fy);
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// S5: grid force of a tile, summed in LDS over the tile's bin (binned)
// or by fixed-order gathers over sorted segments (sorted); every cell of the
// tile is written once.  Direct mode accumulates in k_repulse instead.
// ---------------------------------------------------------------------------
// MK: the two-layer variant (binned worlds with markers, which the plain
// variant skips): the gradient is staged one cell wider on every side and
// the nodes spread through their markers.
template <int TILE, bool MK>
__global__ __launch_bounds__(TileCfg<TILE>::kThreads) void k_spread(const WorldDev* __restrict__ W, Tables T) {
  using C = TileCfg<TILE>;
  constexpr int kThreads = C::kThreads, kSpreadCells = C::kSpreadCells;
  constexpr int kGSide = C::kSpreadSide + (MK ? 2 : 0), kGCells = kGSide * kGSide;
  constexpr int kSpreadCap = C::kSpreadCap;
  __shared__ __align__(16) long long s_fx[kSpreadCells];   // 64-bit fixed point, padded window
  __shared__ __align__(16) long long s_fy[kSpreadCells];
  __shared__ vi4 s_list[(kThreads / 64) * kWaveList];
  __shared__ vf2 s_g[kGCells];                  // gradient over the window (binned)
  const int nt = n_tiles<TILE>(T);
  const int tid = threadIdx.x;
  const XcdLoop tiles(nt);
  for (int it = tiles.first; it < tiles.end; it += tiles.step) {
    const int2 tl = tile_entry<TILE>(T, it);
    const WorldDev& w = W[tl.x];
    if (w.mode == kDirect || w.ctl_src->remaining <= 0) continue;
    if (MK != (w.mode == kBinned && w.d_marker != nullptr)) continue;
    const int mode = w.mode;
    const int nx = w.nx, ny = w.ny;
    const int x0 = tile_x(tl.y) * TILE;
    const int y0 = tile_y(tl.y) * TILE;
    const int tw = min(TILE, nx - x0), th = min(TILE, ny - y0);
    if (mode == kBinned) {
      // S4 repulsion is formed here, per node, from the gradient staged over
      // the window (grid cells (x0 - 3 + i, y0 - 3 + j), periodic); all loads
      // first, then the stores (the barrier in the bin set commit follows)
      {
        constexpr int kIt = (kGCells + kThreads - 1) / kThreads;
        const MC_GLOBAL vf2* grad = glbv<const vf2>(w.grad);
        const int gx0 = wrap_index(x0 - (MK ? 4 : 3), nx), gy0 = wrap_index(y0 - (MK ? 4 : 3), ny);
        vf2 gv[kIt];
#pragma unroll
        for (int i = 0; i < kIt; ++i) {
          const int k = min(tid + kThreads * i, kGCells - 1);
          const int j = k / kGSide, c = k - (k / kGSide) * kGSide;
          gv[i] = grad[(size_t)wrap_index(gy0 + j, ny) * nx + wrap_index(gx0 + c, nx)];
        }
#pragma unroll
        for (int i = 0; i < kIt; ++i) {
          const int k = tid + kThreads * i;
          if (k < kGCells) s_g[k] = gv[i];
        }
      }
      zero_lds_u64(s_fx, kSpreadCells);
      zero_lds_u64(s_fy, kSpreadCells);
      // the tile's record list from the filter (one range), or, if it
      // overflowed, the bins of the neighbourhood
      const int tix = tile_y(tl.y) * w.ntx + tile_x(tl.y);
      const int cnt = glb(w.sp_cnt)[tix];
      if (cnt >= 0 && cnt <= kSpreadCap) {
        BinFetch f;
        f.n = 1;
        f.b0 = tix * kSpreadCap;
        f.len = __lane_id() == 0 ? cnt : 0;
        if constexpr (MK)
          tile_spread_markers<TILE, true, true>(w, x0, y0, tw, th, glb(w.fel_el), 1.0f, s_fx, s_fy, s_list,
                                                glbv<const vi4>(w.sp_rec), f, s_g);
        else
          tile_spread_vec<TILE, true, true>(w, x0, y0, tw, th, glb(w.fel_el), 1.0f, s_fx, s_fy, s_list,
                                            glbv<const vi4>(w.sp_rec), f, s_g);
      } else {
        if constexpr (MK)
          tile_spread_markers<TILE, true>(w, x0, y0, tw, th, glb(w.fel_el), 1.0f, s_fx, s_fy, s_list,
                                          glbv<const vi4>(w.bin_rec), spread_fetch<TILE>(w, x0, y0), s_g);
        else
          tile_spread_vec<TILE, true>(w, x0, y0, tw, th, glb(w.fel_el), 1.0f, s_fx, s_fy, s_list,
                                      glbv<const vi4>(w.bin_rec), spread_fetch<TILE>(w, x0, y0), s_g);
      }
      __syncthreads();
    }
    MC_GLOBAL vf2* Fg = glbv<vf2>(w.Fg);
    const MC_GLOBAL int* start = glb(w.start);
    const MC_GLOBAL vf4* rec = glbv<const vf4>(w.rec);
    for (int k = tid; k < TILE * TILE; k += kThreads) {
      const int ly = k >> C::kShift, lx = k & (TILE - 1);
      if (lx >= tw || ly >= th) continue;
      vf2 F;
      if (mode == kBinned) {
        F.x = fix_to_float(spread_cell<TILE>(s_fx, lx, ly, nx, ny));
        F.y = fix_to_float(spread_cell<TILE>(s_fy, lx, ly, nx, ny));
      } else {
        F = gather_force(start, rec, nx, ny, x0 + lx, y0 + ly);
      }
      Fg[(size_t)(y0 + ly) * nx + x0 + lx] = F;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// S6: D2Q9 two-relaxation-time collision with Guo forcing and push streaming
// over 256 contiguous cells per item.  Populations are stored shifted
// (g = f - w_q) so FP32 resolves the small deviations from rest.  Writes u;
// sets the world flag on NaN or |u| > u_max.  In direct mode it also clears
// the HBM accumulators for the next step.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_lbm(const WorldDev* __restrict__ W, Tables T) {
  constexpr int CPT = kCellsPerItem / 256;      // cells per thread, loaded together
  const XcdLoop items(*T.n_items);
  for (int it = items.first; it < items.end; it += items.step) {
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
    const int ry = item.y / nx;                 // row and column of the item's first cell
    const int rx = item.y - ry * nx;
    const MC_GLOBAL float* src = glb(w.f_src);
    MC_GLOBAL float* dst = glb(w.f_dst);
    float gg[CPT][9];
    vf2 FF[CPT];
#pragma unroll
    for (int h = 0; h < CPT; ++h) {             // every load of every cell first
      const int c = min(item.y + (int)threadIdx.x + 256 * h, ncell - 1);
#pragma unroll
      for (int q = 0; q < 9; ++q)                 // read once per step: no cache allocation
        gg[h][q] = __builtin_nontemporal_load((const float*)(src + (size_t)q * ncell + c));
      FF[h] = glbv<vf2>(w.Fg)[c];
    }
#pragma unroll
    for (int h = 0; h < CPT; ++h) {
      const int c = item.y + (int)threadIdx.x + 256 * h;
      if (c >= ncell) continue;
      int x = rx + (int)threadIdx.x + 256 * h, y = ry;
      while (x >= nx) {                           // items may run over row ends
        x -= nx;
        ++y;
      }
      const float* g = gg[h];
      const vf2 F = FF[h];
      if (w.mode == kDirect) {
        const vf2 zero = {0.f, 0.f};
        glbv<vf2>(w.Fg)[c] = zero;
        glb(w.s)[c] = 0.f;
      }
      const float Fx = F.x, Fy = F.y;
      // moments (the lattice weights have zero first moment, so the shift does
      // not change the momentum sum)
      const float drho = ((g[0] + g[1]) + (g[2] + g[3])) + ((g[4] + g[5]) + (g[6] + g[7])) + g[8];
      const float rho = 1.0f + drho;
      const float jx = (g[1] - g[3]) + (g[5] - g[6]) + (g[8] - g[7]);
      const float jy = (g[2] - g[4]) + (g[5] - g[8]) + (g[6] - g[7]);
      const float inv = 1.0f / rho;
      const float ux = (jx + 0.5f * Fx) * inv;
      const float uy = (jy + 0.5f * Fy) * inv;
      const float usq = ux * ux + uy * uy;
      const vf2 uv = {ux, uy};
      glbv<vf2>(w.u)[c] = uv;
      if (!(usq <= w.u_max2)) atomicOr((unsigned*)glb(w.flags), kFlagUnstable);

      // equilibrium minus weights: w_q (drho + rho (3 cu + 4.5 cu^2 - 1.5 u^2));
      // Guo source: w_q (3 (c - u) + 9 (c.u) c) . F; split into the parts
      // symmetric and antisymmetric under q <-> opposite(q)
      const float op = w.om_p, om = w.om_m;
      const float sp = 1.0f - 0.5f * op, sm = 1.0f - 0.5f * om;
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
        // (non-temporal: the next read is a step away; the caches keep
        // what the following kernels read instead)
        __builtin_nontemporal_store(out[q], (float*)(dst + (size_t)q * ncell + (size_t)yn * nx + xn));
      }
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
    if (w.mode == kBinned || w.ctl_src->remaining <= 0) continue;   // binned: k_integrate_tile
    const int gi = pk.node_begin + threadIdx.x;
    if (gi >= pk.node_end) continue;
    const int N = w.n_part;
    const int nx = w.nx, ny = w.ny;
    const MC_GLOBAL int* cell = glb(w.cell_in);
    const MC_GLOBAL float* frac = glb(w.frac_in);
    const MC_GLOBAL vf2* u = glbv<const vf2>(w.u);
    const int cx = cell[gi], cy = cell[N + gi];
    const float fx = frac[gi], fy = frac[N + gi];
    const int bx = wrap_index(cx, nx), by = wrap_index(cy, ny);
    float wx[4], wy[4];
    peskin4(fx, wx);
    peskin4(fy, wy);
    int ix[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) ix[a] = wrap_near(bx - 1 + a, nx);
    float dux = 0.f, duy = 0.f;
    if (w.d_marker) {
      // two layers: the mean of the markers' interpolated velocities
      const float dx = glb(w.d_marker)[gi], dy = glb(w.d_marker)[N + gi];
#pragma unroll
      for (int sgn = 1; sgn >= -1; sgn -= 2) {
        int hx, hy;
        float mx, my;
        marker_home(cx, fx, sgn * dx, nx, &hx, &mx);
        marker_home(cy, fy, sgn * dy, ny, &hy, &my);
        const vf2 v = gather_vec(u, nx, ny, hx, hy, mx, my);
        dux += 0.5f * v.x;
        duy += 0.5f * v.y;
      }
    } else {
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const MC_GLOBAL vf2* row = u + (size_t)wrap_near(by - 1 + b, ny) * nx;
      float ax = 0.f, ay = 0.f;
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const vf2 v = row[ix[a]];
        ax += wx[a] * v.x;
        ay += wx[a] * v.y;
      }
      dux += wy[b] * ax;
      duy += wy[b] * ay;
    }
    }
    float nfx = fx + dux, nfy = fy + duy;
    const float flx = floorf(nfx), fly = floorf(nfy);
    int ncx = cx + (int)flx, ncy = cy + (int)fly;
    nfx -= flx;
    nfy -= fly;
    if (nfx >= 1.0f) { nfx = 0.0f; ncx += 1; }
    if (nfy >= 1.0f) { nfy = 0.0f; ncy += 1; }
    MC_GLOBAL int* cell_out = glb(w.cell_out);
    MC_GLOBAL float* frac_out = glb(w.frac_out);
    cell_out[gi] = ncx;
    cell_out[N + gi] = ncy;
    frac_out[gi] = nfx;
    frac_out[N + gi] = nfy;
  }
}

// ---------------------------------------------------------------------------
// Binned worlds: the node gather of S7 (u) per tile.  The field is staged in
// LDS for the tile plus the support margin (cells x0-1 .. x0+TILE+1)
// with coalesced loads; every node whose home cell lies in the tile (its bin)
// gathers its 4x4 window from LDS.  (The S4 gather of binned worlds happens
// inside k_spread.)
// ---------------------------------------------------------------------------
// Stage a vector field over the cells (x0 - 1 - E .. x0 + TILE + 1 + E) of
// each axis (side TILE + 3 + 2E): every support of a node whose home lies in
// the tile (E = 0), or of its two-layer markers (E = 1: a marker's home lies
// within one cell of its node's).
template <int TILE, int E = 0>
__device__ __forceinline__ void stage_field(const MC_GLOBAL vf2* f, int nx, int ny, int x0, int y0, vf2* st) {
  constexpr int kStage = TILE + 3 + 2 * E, kThreads = TileCfg<TILE>::kThreads;
  constexpr int kIt = (kStage * kStage + kThreads - 1) / kThreads;
  vf2 v[kIt];
#pragma unroll
  for (int i = 0; i < kIt; ++i) {              // all loads in flight before the stores
    const int k = min((int)threadIdx.x + kThreads * i, kStage * kStage - 1);
    const int r = k / kStage, c = k - (k / kStage) * kStage;
    v[i] = f[(size_t)wrap_index(y0 - 1 - E + r, ny) * nx + wrap_index(x0 - 1 - E + c, nx)];
  }
#pragma unroll
  for (int i = 0; i < kIt; ++i) {
    const int k = (int)threadIdx.x + kThreads * i;
    if (k < kStage * kStage) st[k] = v[i];
  }
}

// 4x4 kernel-weighted sum of a staged vector field (stage_field<TILE, E>)
// at a point whose support starts at staged cell (lx, ly) (a node with home
// cell (lx, ly) of the tile when E = 0; weights wx, wy along x and y).
template <int TILE, int E = 0>
__device__ __forceinline__ vf2 gather_staged(const vf2* st, int lx, int ly, const float* wx, const float* wy) {
  constexpr int kStage = TILE + 3 + 2 * E;
  float gx = 0.f, gy = 0.f;
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const vf2* row = st + (ly + b) * kStage + lx;
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
  const vf2 out = {gx, gy};
  return out;
}

// MK: the two-layer variant (worlds with markers, which the plain variant
// skips): a node moves with the mean of its two markers' velocities.
template <int TILE, bool MK>
__global__ __launch_bounds__(TileCfg<TILE>::kThreads) void k_integrate_tile(const WorldDev* __restrict__ W, Tables T) {
  constexpr int kE = MK ? 1 : 0;
  constexpr int kStage = TILE + 3 + 2 * kE, kThreads = TileCfg<TILE>::kThreads;
  __shared__ vf2 s_u[kStage * kStage];        // staged velocity, x and y interleaved
  const int nt = n_tiles<TILE>(T);
  const XcdLoop tiles(nt);
  for (int it = tiles.first; it < tiles.end; it += tiles.step) {
    const int2 tl = tile_entry<TILE>(T, it);
    const WorldDev& w = W[tl.x];
    if (w.mode != kBinned || w.ctl_src->remaining <= 0) continue;
    if (MK != (w.d_marker != nullptr)) continue;
    const int nx = w.nx, ny = w.ny, N = w.n_part;
    const int x0 = tile_x(tl.y) * TILE;
    const int y0 = tile_y(tl.y) * TILE;
    const MC_GLOBAL vi4* recs = glbv<const vi4>(w.bin_rec);
    const MC_GLOBAL int* cell = glb(w.cell_in);
    MC_GLOBAL int* cell_out = glb(w.cell_out);
    MC_GLOBAL float* frac_out = glb(w.frac_out);
    const int tile = tile_y(tl.y) * w.ntx + tile_x(tl.y);
    const int e0 = glb(w.bin_start)[tile], e1 = glb(w.bin_start)[tile + 1];
    // this thread's first two records and their cells are loaded beside the
    // staged field, unconditionally (record 0 always exists: the record
    // buffer holds at least one; an empty world has no positions at all)
    const int ea = e0 + (int)threadIdx.x, eb = ea + kThreads;
    const bool has0 = ea < e1, has1 = eb < e1;
    const vi4 r0 = recs[has0 ? ea : 0];
    const vi4 r1 = recs[has1 ? eb : 0];
    stage_field<TILE, kE>(glbv<const vf2>(w.u), nx, ny, x0, y0, s_u);
    int c0x = 0, c0y = 0, c1x = 0, c1y = 0;    // in flight across the barrier
    if (N > 0) {
      const int g0 = has0 ? r0.w : 0, g1 = has1 ? r1.w : 0;
      c0x = cell[g0];
      c0y = cell[N + g0];
      c1x = cell[g1];
      c1y = cell[N + g1];
    }
    __syncthreads();
    auto node = [&](const vi4& r, int cxo, int cyo) {
      const int lx = (r.x & 0xffff) - x0, ly = (r.x >> 16) - y0;
      const float fx = __int_as_float(r.y), fy = __int_as_float(r.z);
      const int gi = r.w;
      float dux, duy;
      if constexpr (MK) {
        dux = duy = 0.f;
        const float ddx = glb(w.d_marker)[gi], ddy = glb(w.d_marker)[N + gi];
#pragma unroll
        for (int l = 0; l < 2; ++l) {
          const float sg = l == 0 ? 1.f : -1.f;
          int sx, sy;
          float mx, my;
          marker_shift(fx, sg * ddx, &sx, &mx);
          marker_shift(fy, sg * ddy, &sy, &my);
          float wx[4], wy[4];
          peskin4(mx, wx);
          peskin4(my, wy);
          const vf2 g = gather_staged<TILE, 1>(s_u, lx + sx + 1, ly + sy + 1, wx, wy);
          dux += g.x;
          duy += g.y;
        }
        dux *= 0.5f;
        duy *= 0.5f;
      } else {
        float wx[4], wy[4];
        peskin4(fx, wx);
        peskin4(fy, wy);
        const vf2 du = gather_staged<TILE>(s_u, lx, ly, wx, wy);
        dux = du.x;
        duy = du.y;
      }
      float nfx = fx + dux, nfy = fy + duy;
      const float flx = floorf(nfx), fly = floorf(nfy);
      int ncx = cxo + (int)flx, ncy = cyo + (int)fly;
      nfx -= flx;
      nfy -= fly;
      if (nfx >= 1.0f) { nfx = 0.0f; ncx += 1; }
      if (nfy >= 1.0f) { nfy = 0.0f; ncy += 1; }
      cell_out[gi] = ncx;
      cell_out[N + gi] = ncy;
      frac_out[gi] = nfx;
      frac_out[N + gi] = nfy;
      // next step's tile-bin counts
      agg_atomic_inc(glb(w.bin_cnt), bin_of(wrap_index(ncx, nx), wrap_index(ncy, ny), w.ntx, TileCfg<TILE>::kShift),
                     true);
    };
    // the first two records (already loaded), then any further ones
    if (has0) node(r0, c0x, c0y);
    if (has1) node(r1, c1x, c1y);
    for (int e = eb + kThreads; e < e1; e += kThreads) {
      const vi4 r = recs[e];
      node(r, cell[r.w], cell[N + r.w]);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Energy field: every node senses e_i = sum_c W(c - x_i) E_c at the step's
// starting position and collects rate * e_i, which its filament's total
// gains (summed in node order by the filament's first node) and the field
// loses through the same kernel (k_energy_deplete: tile-binned worlds spread
// it over the spread lists in 64-bit fixed point; others with float atomics).
// ---------------------------------------------------------------------------
template <int PACK>
__global__ __launch_bounds__(PACK) void k_energy_gather(const WorldDev* __restrict__ W, Tables T) {
  __shared__ float s_c[PACK];
  __shared__ int s_off[PACK + 1];
  const int npk = *T.n_packs;
  const int li = threadIdx.x;
  for (int it = blockIdx.x; it < npk; it += gridDim.x) {
    const Pack pk = T.packs[it];
    const WorldDev& w = W[pk.world];
    if (!w.energy || w.ctl_src->remaining <= 0) continue;     // block-uniform
    const int N = w.n_part, nx = w.nx, ny = w.ny;
    const int nf = pk.fil_end - pk.fil_begin;
    for (int k = li; k <= nf; k += PACK) s_off[k] = glb(w.fil_offset)[pk.fil_begin + k] - pk.node_begin;
    const int gi = pk.node_begin + li;
    float c = 0.f;
    if (gi < pk.node_end) {
      const int bx = wrap_index(glb(w.cell_in)[gi], nx), by = wrap_index(glb(w.cell_in)[N + gi], ny);
      float wx[4], wy[4];
      peskin4(glb(w.frac_in)[gi], wx);
      peskin4(glb(w.frac_in)[N + gi], wy);
      const MC_GLOBAL float* E = glb(w.energy);
      float e = 0.f;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const size_t row = (size_t)wrap_near(by - 1 + b, ny) * nx;
        float a = 0.f;
#pragma unroll
        for (int q = 0; q < 4; ++q) a += wx[q] * E[row + wrap_near(bx - 1 + q, nx)];
        e += wy[b] * a;
      }
      glb(w.e_node)[gi] = e;
      if (w.e_sensed) glb(w.e_sensed)[gi] = e;
      c = w.energy_rate * e;
    }
    s_c[li] = c;
    __syncthreads();
    if (w.e_collected && li < nf) {
      // in node order; the loads eight at a time, so that one lane's chain
      // of adds does not wait for each load in turn
      float sum = 0.f;
      int k = s_off[li];
      const int k1 = s_off[li + 1];
      for (; k + 8 <= k1; k += 8) {
        float v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = s_c[k + q];
#pragma unroll
        for (int q = 0; q < 8; ++q) sum += v[q];
      }
      for (; k < k1; ++k) sum += s_c[k];
      glb(w.e_collected)[pk.fil_begin + li] += sum;
    }
    __syncthreads();
  }
}

template <int TILE>
__global__ __launch_bounds__(TileCfg<TILE>::kThreads) void k_energy_deplete(const WorldDev* __restrict__ W,
                                                                             Tables T) {
  using C = TileCfg<TILE>;
  constexpr int kThreads = C::kThreads, kSpreadCells = C::kSpreadCells, kSpreadCap = C::kSpreadCap;
  __shared__ __align__(16) long long s_x[kSpreadCells];
  __shared__ vi4 s_list[(kThreads / 64) * kWaveList];
  const int nt = n_tiles<TILE>(T);
  const XcdLoop tiles(nt);
  for (int it = tiles.first; it < tiles.end; it += tiles.step) {
    const int2 tl = tile_entry<TILE>(T, it);
    const WorldDev& w = W[tl.x];
    if (!w.energy || w.mode != kBinned || w.ctl_src->remaining <= 0) continue;
    const int nx = w.nx, ny = w.ny;
    const int x0 = tile_x(tl.y) * TILE, y0 = tile_y(tl.y) * TILE;
    const int tw = min(TILE, nx - x0), th = min(TILE, ny - y0);
    zero_lds_u64(s_x, kSpreadCells);
    __syncthreads();
    const int tix = tile_y(tl.y) * w.ntx + tile_x(tl.y);
    const int cnt = glb(w.sp_cnt)[tix];
    // the tile's spread list of this step (the records of the step's
    // starting positions), or the bins if it overflowed; a two-layer world's
    // list also holds nodes one cell further out (for their markers), which
    // the keep test drops here
    if (cnt >= 0 && cnt <= kSpreadCap) {
      BinFetch f;
      f.n = 1;
      f.b0 = tix * kSpreadCap;
      f.len = __lane_id() == 0 ? cnt : 0;
      if (w.d_marker)
        tile_spread_vec<TILE, false, false, true>(w, x0, y0, tw, th, glb(w.e_node), -w.energy_rate, s_x, nullptr,
                                                  s_list, glbv<const vi4>(w.sp_rec), f, nullptr);
      else
        tile_spread_vec<TILE, false, true, true>(w, x0, y0, tw, th, glb(w.e_node), -w.energy_rate, s_x, nullptr,
                                                 s_list, glbv<const vi4>(w.sp_rec), f, nullptr);
    } else {
      tile_spread_vec<TILE, false, false, true>(w, x0, y0, tw, th, glb(w.e_node), -w.energy_rate, s_x, nullptr,
                                                s_list, glbv<const vi4>(w.bin_rec), spread_fetch<TILE>(w, x0, y0),
                                                nullptr);
    }
    __syncthreads();
    MC_GLOBAL float* E = glb(w.energy);
    for (int k = threadIdx.x; k < TILE * TILE; k += kThreads) {
      const int ly = k >> C::kShift, lx = k & (TILE - 1);
      if (lx >= tw || ly >= th) continue;
      const size_t c = (size_t)(y0 + ly) * nx + x0 + lx;
      E[c] += fix_to_float(spread_cell<TILE>(s_x, lx, ly, nx, ny));
    }
    __syncthreads();
  }
}

template <int PACK>
__global__ __launch_bounds__(PACK) void k_energy_deplete_atomic(const WorldDev* __restrict__ W, Tables T) {
  const int npk = *T.n_packs;
  for (int it = blockIdx.x; it < npk; it += gridDim.x) {
    const Pack pk = T.packs[it];
    const WorldDev& w = W[pk.world];
    if (!w.energy || w.mode == kBinned || w.ctl_src->remaining <= 0) continue;
    const int gi = pk.node_begin + threadIdx.x;
    if (gi >= pk.node_end) continue;
    const int N = w.n_part, nx = w.nx, ny = w.ny;
    const int bx = wrap_index(glb(w.cell_in)[gi], nx), by = wrap_index(glb(w.cell_in)[N + gi], ny);
    float wx[4], wy[4];
    peskin4(glb(w.frac_in)[gi], wx);
    peskin4(glb(w.frac_in)[N + gi], wy);
    const float c = -w.energy_rate * glb(w.e_node)[gi];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      MC_GLOBAL float* row = glb(w.energy) + (size_t)wrap_near(by - 1 + b, ny) * nx;
#pragma unroll
      for (int q = 0; q < 4; ++q) unsafeAtomicAdd((float*)(row + wrap_near(bx - 1 + q, nx)), c * wx[q] * wy[b]);
    }
  }
}

// Gaussian packets added to a field, every cell (minimum image).
// One block per 32x32 tile: the packets that can reach the tile are listed
// (in index order) and each cell sums only those, in that order.  A packet
// whose nearest distance to the tile (minimum image, less one cell for
// rounding) exceeds sqrt(220) widths has exp(-r^2 / (2 s^2)) below e^-110,
// which is exactly 0 in FP32 (below half the smallest denormal), at every
// cell of the tile, so the sum is the full sum bit for bit.
constexpr int kPacketTile = 32;
constexpr int kPacketChunk = 1024;               // packets listed per pass
__global__ __launch_bounds__(256) void k_energy_packets(int nx, int ny, int n_packets, const float* centres,
                                                        const float* amps, const float* widths, float* field) {
  __shared__ int s_list[kPacketChunk];
  __shared__ int s_wave[4];
  const int ntx = (nx + kPacketTile - 1) / kPacketTile, nty = (ny + kPacketTile - 1) / kPacketTile;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int t = blockIdx.x; t < ntx * nty; t += gridDim.x) {
    const int x0 = (t % ntx) * kPacketTile, y0 = (t / ntx) * kPacketTile;
    const int x1 = min(x0 + kPacketTile, nx) - 1, y1 = min(y0 + kPacketTile, ny) - 1;
    const float hx = 0.5f * (float)(x1 - x0), hy = 0.5f * (float)(y1 - y0);
    const float mx = 0.5f * (float)(x0 + x1), my = 0.5f * (float)(y0 + y1);
    float acc[4] = {0.f, 0.f, 0.f, 0.f};             // cells tid + 256 k of the tile
    for (int p0 = 0; p0 < n_packets; p0 += kPacketChunk) {
      // list this chunk's packets that can reach the tile, in index order:
      // thread tid tests packets p0 + 4 tid .. + 3
      int keep[4];
      int n_keep = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int pi = p0 + 4 * tid + q;
        keep[q] = 0;
        if (pi < n_packets) {
          float dx = centres[pi] - mx, dy = centres[n_packets + pi] - my;
          dx -= (float)nx * floorf(dx / (float)nx + 0.5f);
          dy -= (float)ny * floorf(dy / (float)ny + 0.5f);
          const float ex = fmaxf(fabsf(dx) - hx - 1.0f, 0.f), ey = fmaxf(fabsf(dy) - hy - 1.0f, 0.f);
          const float s = widths[pi];
          keep[q] = ex * ex + ey * ey <= 220.0f * s * s ? 1 : 0;
          n_keep += keep[q];
        }
      }
      // exclusive prefix of n_keep over the block (thread order = packet order)
      int x = n_keep;
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(x, off);
        if (lane >= off) x += y;
      }
      if (lane == 63) s_wave[wv] = x;
      __syncthreads();
      int base = x - n_keep;
      for (int j = 0; j < wv; ++j) base += s_wave[j];
      const int total = s_wave[0] + s_wave[1] + s_wave[2] + s_wave[3];
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (keep[q]) s_list[base++] = p0 + 4 * tid + q;
      __syncthreads();
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int c = tid + 256 * k;
        const int x = x0 + (c & (kPacketTile - 1)), y = y0 + (c >> 5);
        if (x > x1 || y > y1) continue;
        float a = acc[k];
        for (int i = 0; i < total; ++i) {
          const int p = s_list[i];
          float dx = (float)x - centres[p], dy = (float)y - centres[n_packets + p];
          dx -= (float)nx * floorf(dx / (float)nx + 0.5f);
          dy -= (float)ny * floorf(dy / (float)ny + 0.5f);
          const float s = widths[p];
          a += amps[p] * expf(-(dx * dx + dy * dy) / (2.0f * s * s));
        }
        acc[k] = a;
      }
      __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int c = tid + 256 * k;
      const int x = x0 + (c & (kPacketTile - 1)), y = y0 + (c >> 5);
      if (x <= x1 && y <= y1) field[(size_t)y * nx + x] += acc[k];
    }
  }
}

// ---------------------------------------------------------------------------
// Coupling leakage fixes (direct transfer).  Two layers: node i is broadcast
// as markers X = x_i +- d_i, d_i = offset * unit normal (the tangent is
// x_next - x_prev where the node has two neighbours, the edge direction at a
// chain end, none for a lone node).  MDF: desired node velocity
// U_d = I2[j / rho] + F / 2; each further iteration samples
// u = (j + F_grid / 2) / rho at the markers and spreads 2 (U_d - I2[u]).
// ---------------------------------------------------------------------------
template <int PACK>
__global__ __launch_bounds__(PACK) void k_markers(const WorldDev* __restrict__ W, Tables T) {
  __shared__ int s_off[PACK + 1];
  const int npk = *T.n_packs;
  const int li = threadIdx.x;
  for (int it = blockIdx.x; it < npk; it += gridDim.x) {
    const Pack pk = T.packs[it];
    const WorldDev& w = W[pk.world];
    if (!w.d_marker || w.ctl_src->remaining <= 0) continue;     // block-uniform
    const int nf = pk.fil_end - pk.fil_begin;
    for (int k = li; k <= nf; k += PACK) s_off[k] = glb(w.fil_offset)[pk.fil_begin + k] - pk.node_begin;
    __syncthreads();
    const int gi = pk.node_begin + li;
    if (gi < pk.node_end) {
      int lo = 0, hi = nf - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_off[mid] <= li) lo = mid; else hi = mid - 1;
      }
      const int o = s_off[lo], n = s_off[lo + 1] - o, k = li - o;
      const int fil = pk.fil_begin + lo;
      const bool ring = w.fil_flags && (glb(w.fil_flags)[fil] & 1) && n >= 3;
      const int first = pk.node_begin + o;
      int a = gi, b = gi;                         // the nodes the tangent joins
      if (k > 0) a = gi - 1; else if (ring) a = first + n - 1;
      if (k < n - 1) b = gi + 1; else if (ring) b = first;
      const int N = w.n_part;
      const MC_GLOBAL int* cell = glb(w.cell_in);
      const MC_GLOBAL float* frac = glb(w.frac_in);
      const float tx = (float)(cell[b] - cell[a]) + (frac[b] - frac[a]);
      const float ty = (float)(cell[N + b] - cell[N + a]) + (frac[N + b] - frac[N + a]);
      const float len = sqrtf(tx * tx + ty * ty);
      const float sc = len > 0.f ? w.marker_offset / len : 0.f;
      glb(w.d_marker)[gi] = -ty * sc;
      glb(w.d_marker)[N + gi] = tx * sc;
    }
    __syncthreads();
  }
}

// (rho, j) of the step's populations (stored shifted by the weights, whose
// first moment is zero), per cell.
__global__ __launch_bounds__(256) void k_mdf_moments(const WorldDev* __restrict__ W, Tables T) {
  const int nit = *T.n_items;
  for (int it = blockIdx.x; it < nit; it += gridDim.x) {
    const int2 item = T.items[it];
    const WorldDev& w = W[item.x];
    if (w.mdf_iters <= 1 || w.ctl_src->remaining <= 0) continue;
    const int ncell = w.nx * w.ny;
    const int c = item.y + threadIdx.x;
    if (c >= ncell) continue;
    const MC_GLOBAL float* src = glb(w.f_src);
    float g[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) g[q] = src[(size_t)q * ncell + c];
    const float drho = ((g[0] + g[1]) + (g[2] + g[3])) + ((g[4] + g[5]) + (g[6] + g[7])) + g[8];
    const float jx = (g[1] - g[3]) + (g[5] - g[6]) + (g[8] - g[7]);
    const float jy = (g[2] - g[4]) + (g[5] - g[8]) + (g[6] - g[7]);
    const vf4 m = {1.0f + drho, jx, jy, 0.f};
    glbv<vf4>(w.rho_j)[c] = m;
  }
}

// u = (j + F_grid / 2) / rho of the current grid force, per cell.
__global__ __launch_bounds__(256) void k_mdf_velocity(const WorldDev* __restrict__ W, Tables T, int iter) {
  const int nit = *T.n_items;
  for (int it = blockIdx.x; it < nit; it += gridDim.x) {
    const int2 item = T.items[it];
    const WorldDev& w = W[item.x];
    if (w.mode == kBinned || iter >= w.mdf_iters || w.ctl_src->remaining <= 0) continue;
    const int ncell = w.nx * w.ny;
    const int c = item.y + threadIdx.x;
    if (c >= ncell) continue;
    const vf4 m = glbv<const vf4>(w.rho_j)[c];
    const vf2 F = glbv<const vf2>(w.Fg)[c];
    const float inv = 1.0f / m.x;
    const vf2 u = {(m.y + 0.5f * F.x) * inv, (m.z + 0.5f * F.y) * inv};
    glbv<vf2>(w.u_mdf)[c] = u;
  }
}

// Two-layer interpolation of a per-cell quantity at node gi: mean over its
// markers (or the node itself with one layer) of sum_c W(c - X) value(c).
template <class V>
static __device__ __forceinline__ vf2 interp2(const WorldDev& w, int gi, V value) {
  const int N = w.n_part, nx = w.nx, ny = w.ny;
  const int cx = glb(w.cell_in)[gi], cy = glb(w.cell_in)[N + gi];
  const float fx = glb(w.frac_in)[gi], fy = glb(w.frac_in)[N + gi];
  const float dx = w.d_marker ? glb(w.d_marker)[gi] : 0.f, dy = w.d_marker ? glb(w.d_marker)[N + gi] : 0.f;
  float sx = 0.f, sy = 0.f;
  const int layers = w.d_marker ? 2 : 1;
  for (int l = 0; l < layers; ++l) {
    const float sg = l == 0 ? 1.f : -1.f;
    int hx, hy;
    float mx, my;
    marker_home(cx, fx, sg * dx, nx, &hx, &mx);
    marker_home(cy, fy, sg * dy, ny, &hy, &my);
    float wx[4], wy[4];
    peskin4(mx, wx);
    peskin4(my, wy);
    float gx = 0.f, gy = 0.f;
    for (int b = 0; b < 4; ++b) {
      const size_t row = (size_t)wrap_near(hy - 1 + b, ny) * nx;
      float ax = 0.f, ay = 0.f;
      for (int a = 0; a < 4; ++a) {
        const vf2 v = value(row + wrap_near(hx - 1 + a, nx));
        ax += wx[a] * v.x;
        ay += wx[a] * v.y;
      }
      gx += wy[b] * ax;
      gy += wy[b] * ay;
    }
    sx += gx;
    sy += gy;
  }
  const float h = layers == 2 ? 0.5f : 1.0f;
  const vf2 out = {h * sx, h * sy};
  return out;
}

// Spread of (vx, vy) from node gi's markers (half each) or the node.
static __device__ __forceinline__ void spread2_atomic(const WorldDev& w, int gi, float vx, float vy) {
  const int N = w.n_part, nx = w.nx, ny = w.ny;
  const int cx = glb(w.cell_in)[gi], cy = glb(w.cell_in)[N + gi];
  const float fx = glb(w.frac_in)[gi], fy = glb(w.frac_in)[N + gi];
  if (!w.d_marker) {
    atomic_spread_vec(glb((float*)w.Fg), nx, ny, wrap_index(cx, nx), wrap_index(cy, ny), fx, fy, vx, vy);
    return;
  }
  const float dx = glb(w.d_marker)[gi], dy = glb(w.d_marker)[N + gi];
  for (int sg = 1; sg >= -1; sg -= 2) {
    int hx, hy;
    float mx, my;
    marker_home(cx, fx, sg * dx, nx, &hx, &mx);
    marker_home(cy, fy, sg * dy, ny, &hy, &my);
    atomic_spread_vec(glb((float*)w.Fg), nx, ny, hx, hy, mx, my, 0.5f * vx, 0.5f * vy);
  }
}

template <int PACK>
__global__ __launch_bounds__(PACK) void k_mdf_desired(const WorldDev* __restrict__ W, Tables T) {
  const int npk = *T.n_packs;
  for (int it = blockIdx.x; it < npk; it += gridDim.x) {
    const Pack pk = T.packs[it];
    const WorldDev& w = W[pk.world];
    if (w.mode == kBinned || w.mdf_iters <= 1 || w.ctl_src->remaining <= 0) continue;
    const int gi = pk.node_begin + threadIdx.x;
    if (gi >= pk.node_end) continue;
    const MC_GLOBAL vf4* m = glbv<const vf4>(w.rho_j);
    const vf2 us = interp2(w, gi, [&](size_t c) {
      const vf4 v = m[c];
      const vf2 r = {v.y / v.x, v.z / v.x};
      return r;
    });
    const int N = w.n_part;
    glb(w.U_d)[gi] = us.x + 0.5f * glb(w.fel)[gi];
    glb(w.U_d)[N + gi] = us.y + 0.5f * glb(w.fel)[N + gi];
  }
}

template <int PACK>
__global__ __launch_bounds__(PACK) void k_mdf_correct(const WorldDev* __restrict__ W, Tables T, int iter) {
  const int npk = *T.n_packs;
  for (int it = blockIdx.x; it < npk; it += gridDim.x) {
    const Pack pk = T.packs[it];
    const WorldDev& w = W[pk.world];
    if (w.mode == kBinned || iter >= w.mdf_iters || w.ctl_src->remaining <= 0) continue;
    const int gi = pk.node_begin + threadIdx.x;
    if (gi >= pk.node_end) continue;
    const MC_GLOBAL vf2* um = glbv<const vf2>(w.u_mdf);
    const vf2 U = interp2(w, gi, [&](size_t c) { return um[c]; });
    const int N = w.n_part;
    const float cx = 2.0f * (glb(w.U_d)[gi] - U.x);
    const float cy = 2.0f * (glb(w.U_d)[N + gi] - U.y);
    spread2_atomic(w, gi, cx, cy);
  }
}

// Binned transfer: the node passes of MDF as tile passes over the home-tile
// bins, and the correction spread through the tiles' spread lists, summed in
// LDS as 64-bit fixed point like the force spread: deterministic and without
// HBM atomics.
//   k_mdf_gather_tile<TILE, true>   U_d = I[j / rho] + F / 2 at the tile's nodes
//   k_mdf_gather_tile<TILE, false>  c = 2 (U_d - I[(j + F_grid / 2) / rho])
//   k_mdf_spread_tile<TILE>         F_grid += S[c] over the tile
// The velocity is formed per staged cell from the moments and the grid force.
// MK: the two-layer variants (I: the mean over the node's two markers; S:
// half of the value from each marker).
template <int TILE, bool DESIRED, bool MK>
__global__ __launch_bounds__(TileCfg<TILE>::kThreads) void k_mdf_gather_tile(const WorldDev* __restrict__ W, Tables T,
                                                                             int iter) {
  constexpr int kE = MK ? 1 : 0;
  constexpr int kStage = TILE + 3 + 2 * kE, kThreads = TileCfg<TILE>::kThreads;
  constexpr int kIt = (kStage * kStage + kThreads - 1) / kThreads;
  __shared__ vf2 s_u[kStage * kStage];
  const int nt = n_tiles<TILE>(T);
  const XcdLoop tiles(nt);
  for (int it = tiles.first; it < tiles.end; it += tiles.step) {
    const int2 tl = tile_entry<TILE>(T, it);
    const WorldDev& w = W[tl.x];
    if (w.mode != kBinned || w.mdf_iters <= 1 || (!DESIRED && iter >= w.mdf_iters) || w.ctl_src->remaining <= 0)
      continue;
    if (MK != (w.d_marker != nullptr)) continue;
    const int nx = w.nx, ny = w.ny, N = w.n_part;
    const int x0 = tile_x(tl.y) * TILE, y0 = tile_y(tl.y) * TILE;
    const MC_GLOBAL vf4* m = glbv<const vf4>(w.rho_j);
    const MC_GLOBAL vf2* Fg = glbv<const vf2>(w.Fg);
    vf4 mv[kIt];
    vf2 fv[kIt];
#pragma unroll
    for (int i = 0; i < kIt; ++i) {              // all loads in flight before the stores
      const int k = min((int)threadIdx.x + kThreads * i, kStage * kStage - 1);
      const int r = k / kStage, c = k - (k / kStage) * kStage;
      const size_t idx = (size_t)wrap_index(y0 - 1 - kE + r, ny) * nx + wrap_index(x0 - 1 - kE + c, nx);
      mv[i] = m[idx];
      if (!DESIRED) fv[i] = Fg[idx];
    }
#pragma unroll
    for (int i = 0; i < kIt; ++i) {
      const int k = (int)threadIdx.x + kThreads * i;
      if (k < kStage * kStage) {
        const float inv = 1.0f / mv[i].x;
        vf2 u;
        if (DESIRED) {
          u.x = mv[i].y / mv[i].x;
          u.y = mv[i].z / mv[i].x;
        } else {
          u.x = (mv[i].y + 0.5f * fv[i].x) * inv;
          u.y = (mv[i].z + 0.5f * fv[i].y) * inv;
        }
        s_u[k] = u;
      }
    }
    __syncthreads();
    const int tile = tile_y(tl.y) * w.ntx + tile_x(tl.y);
    const int e0 = glb(w.bin_start)[tile], e1 = glb(w.bin_start)[tile + 1];
    const MC_GLOBAL vi4* recs = glbv<const vi4>(w.bin_rec);
    MC_GLOBAL float* Ud = glb(w.U_d);
    for (int e = e0 + (int)threadIdx.x; e < e1; e += kThreads) {
      const vi4 r = recs[e];
      const int lx = (r.x & 0xffff) - x0, ly = (r.x >> 16) - y0;
      const float fx = __int_as_float(r.y), fy = __int_as_float(r.z);
      const int gi = r.w;
      vf2 g;
      if constexpr (MK) {
        g.x = g.y = 0.f;
        const float ddx = glb(w.d_marker)[gi], ddy = glb(w.d_marker)[N + gi];
#pragma unroll
        for (int l = 0; l < 2; ++l) {
          const float sg = l == 0 ? 1.f : -1.f;
          int sx, sy;
          float mx, my;
          marker_shift(fx, sg * ddx, &sx, &mx);
          marker_shift(fy, sg * ddy, &sy, &my);
          float wx[4], wy[4];
          peskin4(mx, wx);
          peskin4(my, wy);
          const vf2 gl = gather_staged<TILE, 1>(s_u, lx + sx + 1, ly + sy + 1, wx, wy);
          g.x += gl.x;
          g.y += gl.y;
        }
        g.x *= 0.5f;
        g.y *= 0.5f;
      } else {
        float wx[4], wy[4];
        peskin4(fx, wx);
        peskin4(fy, wy);
        g = gather_staged<TILE>(s_u, lx, ly, wx, wy);
      }
      if (DESIRED) {
        Ud[gi] = g.x + 0.5f * glb(w.fel)[gi];
        Ud[N + gi] = g.y + 0.5f * glb(w.fel)[N + gi];
      } else {
        glb(w.mdf_c)[gi] = 2.0f * (Ud[gi] - g.x);
        glb(w.mdf_c)[N + gi] = 2.0f * (Ud[N + gi] - g.y);
      }
    }
    __syncthreads();
  }
}

template <int TILE, bool MK>
__global__ __launch_bounds__(TileCfg<TILE>::kThreads) void k_mdf_spread_tile(const WorldDev* __restrict__ W, Tables T,
                                                                             int iter) {
  using C = TileCfg<TILE>;
  constexpr int kThreads = C::kThreads, kSpreadCells = C::kSpreadCells, kSpreadCap = C::kSpreadCap;
  __shared__ __align__(16) long long s_fx[kSpreadCells];
  __shared__ __align__(16) long long s_fy[kSpreadCells];
  __shared__ vi4 s_list[(kThreads / 64) * kWaveList];
  const int nt = n_tiles<TILE>(T);
  const XcdLoop tiles(nt);
  for (int it = tiles.first; it < tiles.end; it += tiles.step) {
    const int2 tl = tile_entry<TILE>(T, it);
    const WorldDev& w = W[tl.x];
    if (w.mode != kBinned || iter >= w.mdf_iters || w.ctl_src->remaining <= 0) continue;
    if (MK != (w.d_marker != nullptr)) continue;
    const int nx = w.nx, ny = w.ny;
    const int x0 = tile_x(tl.y) * TILE, y0 = tile_y(tl.y) * TILE;
    const int tw = min(TILE, nx - x0), th = min(TILE, ny - y0);
    zero_lds_u64(s_fx, kSpreadCells);
    zero_lds_u64(s_fy, kSpreadCells);
    __syncthreads();
    const int tix = tile_y(tl.y) * w.ntx + tile_x(tl.y);
    const int cnt = glb(w.sp_cnt)[tix];
    if (cnt >= 0 && cnt <= kSpreadCap) {
      BinFetch f;
      f.n = 1;
      f.b0 = tix * kSpreadCap;
      f.len = __lane_id() == 0 ? cnt : 0;
      if constexpr (MK)
        tile_spread_markers<TILE, false, true>(w, x0, y0, tw, th, glb(w.mdf_c), 1.0f, s_fx, s_fy, s_list,
                                               glbv<const vi4>(w.sp_rec), f, nullptr);
      else
        tile_spread_vec<TILE, false, true>(w, x0, y0, tw, th, glb(w.mdf_c), 1.0f, s_fx, s_fy, s_list,
                                           glbv<const vi4>(w.sp_rec), f, nullptr);
    } else {
      if constexpr (MK)
        tile_spread_markers<TILE, false>(w, x0, y0, tw, th, glb(w.mdf_c), 1.0f, s_fx, s_fy, s_list,
                                         glbv<const vi4>(w.bin_rec), spread_fetch<TILE>(w, x0, y0), nullptr);
      else
        tile_spread_vec<TILE, false>(w, x0, y0, tw, th, glb(w.mdf_c), 1.0f, s_fx, s_fy, s_list,
                                     glbv<const vi4>(w.bin_rec), spread_fetch<TILE>(w, x0, y0), nullptr);
    }
    __syncthreads();
    MC_GLOBAL vf2* Fg = glbv<vf2>(w.Fg);
    for (int k = threadIdx.x; k < TILE * TILE; k += kThreads) {
      const int ly = k >> C::kShift, lx = k & (TILE - 1);
      if (lx >= tw || ly >= th) continue;
      const size_t c = (size_t)(y0 + ly) * nx + x0 + lx;
      vf2 F = Fg[c];
      F.x += fix_to_float(spread_cell<TILE>(s_fx, lx, ly, nx, ny));
      F.y += fix_to_float(spread_cell<TILE>(s_fy, lx, ly, nx, ny));
      Fg[c] = F;
    }
    __syncthreads();
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
  if (G.branches) {
    if (G.pack == 256)
      k_elastic<256, true, true><<<G.node_blocks, 256, 0, s>>>(W, T);
    else
      k_elastic<1024, true, true><<<G.node_blocks, 1024, 0, s>>>(W, T);
  } else if (G.general) {
    if (G.pack == 256)
      k_elastic<256, true, false><<<G.node_blocks, 256, 0, s>>>(W, T);
    else
      k_elastic<1024, true, false><<<G.node_blocks, 1024, 0, s>>>(W, T);
  } else {
    if (G.pack == 256)
      k_elastic<256, false, false><<<G.node_blocks, 256, 0, s>>>(W, T);
    else
      k_elastic<1024, false, false><<<G.node_blocks, 1024, 0, s>>>(W, T);
  }
}

void launch_bin_prepass(const WorldDev* W, const Tables& T, const Grid& G, hipStream_t s) {
  if (!G.any_binned) return;
  MC_PACK_DISPATCH(k_bin_count, G, W, T);
  k_bin_scan<<<G.world_blocks, 1024, 0, s>>>(W, T, 0);
}

void launch_sort(const WorldDev* W, const Tables& T, const Grid& G, hipStream_t s) {
  if (G.any_sorted) {
    k_scan_reduce<<<G.scan_blocks, 256, 0, s>>>(W, T);
    k_scan_partials<<<G.world_blocks, 256, 0, s>>>(W, T);
    k_scan_down<<<G.scan_blocks, 256, 0, s>>>(W, T);
    MC_PACK_DISPATCH(k_scatter, G, W, T);
    MC_PACK_DISPATCH(k_segsort, G, W, T);
  }
}

// Tile kernels: one launch per tile family present.
template <int TILE>
static void launch_filter_t(const WorldDev* W, const Tables& T, const Grid& G, hipStream_t s) {
  constexpr int f = TileCfg<TILE>::kFamily;
  if (G.tile_blocks[f] <= 0) return;
  // the largest dynamic LDS any launch asks for (64-cell tiles exceed 64 KiB),
  // declared once per process
  static const bool lds_declared = [] {
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_filter<TILE>),
                               hipFuncAttributeMaxDynamicSharedMemorySize,
                               filter_window_bytes<TILE>(kMaxRadius) + filter_list_bytes<TILE>(kMaxRadius)) ==
           hipSuccess;
  }();
  (void)lds_declared;
  const int wb = filter_window_bytes<TILE>(G.max_radius);
  k_filter<TILE><<<G.tile_blocks[f], TileCfg<TILE>::kThreads, wb + filter_list_bytes<TILE>(G.max_radius), s>>>(W, T, wb);
}

void launch_filter(const WorldDev* W, const Tables& T, const Grid& G, hipStream_t s) {
  launch_filter_t<16>(W, T, G, s);
  launch_filter_t<32>(W, T, G, s);
  launch_filter_t<64>(W, T, G, s);
}

void launch_repulse(const WorldDev* W, const Tables& T, const Grid& G, hipStream_t s) {
  if (G.any_node) MC_PACK_DISPATCH(k_repulse, G, W, T);
  // binned worlds form the repulsion inside k_spread
}

// (tile kernels with a one-layer and a two-layer variant: for_tile_variants)
void launch_spread(const WorldDev* W, const Tables& T, const Grid& G, hipStream_t s) {
  for_tile_variants(G, [&](auto tile, auto mk) {
    constexpr int TL = decltype(tile)::value;
    k_spread<TL, decltype(mk)::value><<<G.tile_blocks[TileCfg<TL>::kFamily], TileCfg<TL>::kThreads, 0, s>>>(W, T);
  });
}

void launch_lbm(const WorldDev* W, const Tables& T, const Grid& G, hipStream_t s) {
  k_lbm<<<G.item_blocks, 256, 0, s>>>(W, T);
}

void launch_lbm_timed(const WorldDev* W, const Tables& T, const Grid& G, hipStream_t s, hipEvent_t start,
                      hipEvent_t stop) {
  hipExtLaunchKernelGGL(k_lbm, dim3(G.item_blocks), dim3(256), 0, s, start, stop, 0, W, T);
}

void launch_integrate(const WorldDev* W, const Tables& T, const Grid& G, hipStream_t s) {
  if (G.any_node) MC_PACK_DISPATCH(k_integrate, G, W, T);
  if (G.any_binned) {
    for_tile_variants(G, [&](auto tile, auto mk) {
      constexpr int TL = decltype(tile)::value;
      k_integrate_tile<TL, decltype(mk)::value>
          <<<G.tile_blocks[TileCfg<TL>::kFamily], TileCfg<TL>::kThreads, 0, s>>>(W, T);
    });
    k_bin_scan<<<G.world_blocks, 1024, 0, s>>>(W, T, 1);  // bins of the new positions
  }
}

void launch_markers(const WorldDev* W, const Tables& T, const Grid& G, hipStream_t s) {
  if (G.any_markers) MC_PACK_DISPATCH(k_markers, G, W, T);
}

void launch_mdf_moments(const WorldDev* W, const Tables& T, const Grid& G, hipStream_t s) {
  k_mdf_moments<<<G.item_blocks, 256, 0, s>>>(W, T);
}

void launch_mdf(const WorldDev* W, const Tables& T, const Grid& G, hipStream_t s) {
  if (G.mdf_max <= 1) return;
  k_mdf_moments<<<G.item_blocks, 256, 0, s>>>(W, T);
  if (G.any_node) MC_PACK_DISPATCH(k_mdf_desired, G, W, T);
  if (G.any_binned) {
    for_tile_variants(G, [&](auto tile, auto mk) {
      constexpr int TL = decltype(tile)::value;
      k_mdf_gather_tile<TL, true, decltype(mk)::value>
          <<<G.tile_blocks[TileCfg<TL>::kFamily], TileCfg<TL>::kThreads, 0, s>>>(W, T, 0);
    });
  }
  for (int iter = 1; iter < G.mdf_max; ++iter) {
    if (G.any_node) {
      k_mdf_velocity<<<G.item_blocks, 256, 0, s>>>(W, T, iter);
      MC_PACK_DISPATCH(k_mdf_correct, G, W, T, iter);
    }
    if (G.any_binned) {
      for_tile_variants(G, [&](auto tile, auto mk) {
        constexpr int TL = decltype(tile)::value;
        k_mdf_gather_tile<TL, false, decltype(mk)::value>
            <<<G.tile_blocks[TileCfg<TL>::kFamily], TileCfg<TL>::kThreads, 0, s>>>(W, T, iter);
      });
      for_tile_variants(G, [&](auto tile, auto mk) {
        constexpr int TL = decltype(tile)::value;
        k_mdf_spread_tile<TL, decltype(mk)::value>
            <<<G.tile_blocks[TileCfg<TL>::kFamily], TileCfg<TL>::kThreads, 0, s>>>(W, T, iter);
      });
    }
  }
}

void launch_energy(const WorldDev* W, const Tables& T, const Grid& G, hipStream_t s) {
  if (!G.any_energy) return;
  MC_PACK_DISPATCH(k_energy_gather, G, W, T);
  if (G.any_binned) {
    if (G.tile_blocks[0] > 0) k_energy_deplete<16><<<G.tile_blocks[0], TileCfg<16>::kThreads, 0, s>>>(W, T);
    if (G.tile_blocks[1] > 0) k_energy_deplete<32><<<G.tile_blocks[1], TileCfg<32>::kThreads, 0, s>>>(W, T);
    if (G.tile_blocks[2] > 0) k_energy_deplete<64><<<G.tile_blocks[2], TileCfg<64>::kThreads, 0, s>>>(W, T);
  }
  if (G.any_node) MC_PACK_DISPATCH(k_energy_deplete_atomic, G, W, T);
}

void launch_energy_packets(int nx, int ny, int n_packets, const float* centres, const float* amps,
                           const float* widths, float* field, hipStream_t s) {
  const int nt = ((nx + kPacketTile - 1) / kPacketTile) * ((ny + kPacketTile - 1) / kPacketTile);
  k_energy_packets<<<nt < 8192 ? nt : 8192, 256, 0, s>>>(nx, ny, n_packets, centres, amps, widths, field);
}

void launch_tile_ranges(int nx, int ny, int R, int tile, int2* out, hipStream_t s) {
  const int nt = ((nx + tile - 1) / tile) * ((ny + tile - 1) / tile);
  const int blocks = nt > 0 ? (nt + 255) / 256 : 1;
  if (tile == 16) k_tile_ranges<16><<<blocks, 256, 0, s>>>(nx, ny, R, out);
  else if (tile == 64) k_tile_ranges<64><<<blocks, 256, 0, s>>>(nx, ny, R, out);
  else k_tile_ranges<32><<<blocks, 256, 0, s>>>(nx, ny, R, out);
}

void launch_set_ctl(Ctl* c, long long t, int remaining, hipStream_t s) {
  k_set_ctl<<<1, 64, 0, s>>>(c, t, remaining);
}

}  // namespace mc
