// Objectives and descriptors computed from a world's state.
//
// Folding objective (Experiments, Filament Folding): the node density
// splatted with a Gaussian onto an image that covers the periodic world, its
// mean squared error to a target image, and the gradient of that loss with
// respect to the node positions.  Behavioural descriptors (Experiments, QD
// Search, Eqs. 5-6): bending and stretching effort of a change of the rest
// values, per filament.
//
// Pixel (a, b) of a W x H image is centred at world point
// (-1/2 + (a + 1/2) hx, -1/2 + (b + 1/2) hy), hx = nx / W, hy = ny / H; node i
// adds amp exp(-r^2 / (2 sigma^2)) to every pixel whose centre lies within
// r <= 5 sigma of it (periodic minimum-image distance).
//
//   k_splat_image     per node: its pixels' contributions, summed as 64-bit
//                     fixed point (order-independent: bitwise reproducible)
//   k_image_residual  per pixel: the image, 2 (I - T) / P for the gradient,
//                     and per-block sums of (I - T)^2 in a fixed order
//   k_image_loss      one block: the loss from the block sums (fixed order)
//   k_splat_grad      per node: dL/dx_i = sum over its pixels of
//                     2 (I - T) / P * amp e^{-r^2/2s^2} * (-(x_i - c) / s^2)
#include "device_util.h"

namespace mc {

constexpr float kImgFix = 1099511627776.0f;          // 2^40: image fixed-point scale
constexpr double kImgFixInv = 1.0 / 1099511627776.0;
constexpr int kLossBlock = 256;

struct SplatGeom {
  int nx, ny, n, W, H;
  float hx, hy;          // pixel spacing (cells)
  float inv2s2;          // 1 / (2 sigma^2)
  float inv_s2;          // 1 / sigma^2
  float cut2;            // (5 sigma)^2
  float amp;
  int rx, ry;            // pixel window half-widths; rx < 0: every column once (same for ry)
};

// Minimum-image difference d (|d| < 2n on entry) reduced to [-n/2, n/2).
static __device__ __forceinline__ float wrap_half(float d, float n) {
  if (d >= 0.5f * n) d -= n;
  if (d < -0.5f * n) d += n;
  return d;
}

// The pixels of node (xw, yw) (wrapped world position): calls f(pixel index,
// dx, dy, weight) for every pixel centre within the cutoff, each pixel once.
template <class F>
static __device__ __forceinline__ void for_node_pixels(const SplatGeom& g, float xw, float yw, F f) {
  const int a0 = (int)floorf((xw + 0.5f) / g.hx);      // pixel column holding the node
  const int b0 = (int)floorf((yw + 0.5f) / g.hy);
  const int alo = g.rx < 0 ? 0 : a0 - g.rx, ahi = g.rx < 0 ? g.W - 1 : a0 + g.rx;
  const int blo = g.ry < 0 ? 0 : b0 - g.ry, bhi = g.ry < 0 ? g.H - 1 : b0 + g.ry;
  for (int b = blo; b <= bhi; ++b) {
    const int bw = wrap_index(b, g.H);
    const float dy = wrap_half(yw - (-0.5f + ((float)bw + 0.5f) * g.hy), (float)g.ny);
    for (int a = alo; a <= ahi; ++a) {
      const int aw = wrap_index(a, g.W);
      const float dx = wrap_half(xw - (-0.5f + ((float)aw + 0.5f) * g.hx), (float)g.nx);
      const float r2 = dx * dx + dy * dy;
      if (r2 <= g.cut2) f(bw * g.W + aw, dx, dy, g.amp * expf(-r2 * g.inv2s2));
    }
  }
}

static __device__ __forceinline__ void node_position(const SplatGeom& g, const int* cell, const float* frac, int i,
                                                     float* xw, float* yw) {
  *xw = (float)wrap_index(cell[i], g.nx) + frac[i];
  *yw = (float)wrap_index(cell[g.n + i], g.ny) + frac[g.n + i];
}

__global__ void k_zero_u64(unsigned long long* p, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0ull;
}

__global__ __launch_bounds__(256) void k_splat_image(SplatGeom g, const int* cell, const float* frac,
                                                     unsigned long long* acc) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < g.n; i += gridDim.x * blockDim.x) {
    float xw, yw;
    node_position(g, cell, frac, i, &xw, &yw);
    for_node_pixels(g, xw, yw, [&](int pix, float, float, float v) {
      atomicAdd(acc + pix, (unsigned long long)f32_to_fix(v * kImgFix));
    });
  }
}

__global__ __launch_bounds__(kLossBlock) void k_image_residual(SplatGeom g, const unsigned long long* acc,
                                                               const float* target, float* image, float* resid,
                                                               float* partial) {
  __shared__ float s_sum[kLossBlock];
  const int P = g.W * g.H;
  const int p = blockIdx.x * kLossBlock + threadIdx.x;
  float e2 = 0.f;
  if (p < P) {
    const float I = (float)((double)(long long)acc[p] * kImgFixInv);
    const float r = I - target[p];
    if (image) image[p] = I;
    resid[p] = 2.0f * r / (float)P;
    e2 = r * r;
  }
  s_sum[threadIdx.x] = e2;
  __syncthreads();
  for (int off = kLossBlock / 2; off > 0; off >>= 1) {   // fixed pairing: deterministic
    if ((int)threadIdx.x < off) s_sum[threadIdx.x] += s_sum[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = s_sum[0];
}

__global__ __launch_bounds__(kLossBlock) void k_image_loss(const float* partial, int nblocks, int P, float* loss) {
  __shared__ double s_sum[kLossBlock];
  double acc = 0.0;
  for (int k = threadIdx.x; k < nblocks; k += kLossBlock) acc += (double)partial[k];
  s_sum[threadIdx.x] = acc;
  __syncthreads();
  for (int off = kLossBlock / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) s_sum[threadIdx.x] += s_sum[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = (float)(s_sum[0] / (double)P);
}

__global__ __launch_bounds__(256) void k_splat_grad(SplatGeom g, const int* cell, const float* frac,
                                                    const float* resid, float* g_pos) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < g.n; i += gridDim.x * blockDim.x) {
    float xw, yw;
    node_position(g, cell, frac, i, &xw, &yw);
    float gx = 0.f, gy = 0.f;
    for_node_pixels(g, xw, yw, [&](int pix, float dx, float dy, float v) {
      const float c = resid[pix] * v * g.inv_s2;
      gx -= c * dx;
      gy -= c * dy;
    });
    g_pos[i] = gx;
    g_pos[g.n + i] = gy;
  }
}

// Workspace: accumulator [H*W] u64 | residual [H*W] f32 | block sums.
size_t density_loss_workspace(int W, int H) {
  const size_t P = (size_t)W * H;
  const size_t nb = (P + kLossBlock - 1) / kLossBlock;
  auto al = [](size_t b) { return (b + 255) / 256 * 256; };
  return al(P * 8) + al(P * 4) + al(nb * 4);
}

void launch_density_loss(int nx, int ny, int n, int W, int H, float sigma, float amp, const int* cell,
                         const float* frac, const float* target, float* image, float* loss, float* g_pos,
                         void* ws, hipStream_t s) {
  SplatGeom g;
  g.nx = nx;
  g.ny = ny;
  g.n = n;
  g.W = W;
  g.H = H;
  g.hx = (float)nx / (float)W;
  g.hy = (float)ny / (float)H;
  g.inv2s2 = 1.0f / (2.0f * sigma * sigma);
  g.inv_s2 = 1.0f / (sigma * sigma);
  g.cut2 = 25.0f * sigma * sigma;
  g.amp = amp;
  // a pixel k columns away from the node's own has its centre at least
  // (|k| - 1/2) hx away: columns up to 5 sigma / hx + 1/2 can be inside
  const int rx = (int)floorf(5.0f * sigma / g.hx + 0.5f) + 1;
  const int ry = (int)floorf(5.0f * sigma / g.hy + 0.5f) + 1;
  g.rx = 2 * rx + 1 >= W ? -1 : rx;            // the window would wrap onto itself: all columns once
  g.ry = 2 * ry + 1 >= H ? -1 : ry;
  const int P = W * H;
  const int nb = (P + kLossBlock - 1) / kLossBlock;
  char* base = (char*)ws;
  auto al = [](size_t b) { return (b + 255) / 256 * 256; };
  unsigned long long* acc = (unsigned long long*)base;
  float* resid = (float*)(base + al((size_t)P * 8));
  float* partial = (float*)(base + al((size_t)P * 8) + al((size_t)P * 4));
  const int zb = P / 256 + 1 < 1024 ? P / 256 + 1 : 1024;
  k_zero_u64<<<zb, 256, 0, s>>>(acc, P);
  const int nodeb = n / 256 + 1 < 4096 ? n / 256 + 1 : 4096;
  if (n > 0) k_splat_image<<<nodeb, 256, 0, s>>>(g, cell, frac, acc);
  k_image_residual<<<nb, kLossBlock, 0, s>>>(g, acc, target, image, resid, partial);
  k_image_loss<<<1, kLossBlock, 0, s>>>(partial, nb, P, loss);
  if (g_pos && n > 0) k_splat_grad<<<nodeb, 256, 0, s>>>(g, cell, frac, resid, g_pos);
}

// ---------------------------------------------------------------------------
// Efforts: per filament, sum over its joints of (old - new rest angle)^2 and
// over its edges of (old - new rest length)^2, accumulated into effort[f]
// and effort[F + f].  One block per filament; fixed-order block sums.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_rest_effort(int n_fil, const int* fil_offset, const int* fil_flags,
                                                     const float* old_a, const float* new_a, const float* old_l,
                                                     const float* new_l, float* effort) {
  __shared__ float s_b[256];
  __shared__ float s_p[256];
  for (int f = blockIdx.x; f < n_fil; f += gridDim.x) {
    const int a = fil_offset[f], b = fil_offset[f + 1], n = b - a;
    const bool ring = fil_flags && (fil_flags[f] & 1) && n >= 3;
    const int j0 = ring ? a : a + 1, j1 = ring ? b : b - 1;      // joints [j0, j1)
    const int e1 = ring ? b : b - 1;                               // edges [a, e1)
    float eb = 0.f, ep = 0.f;
    for (int i = j0 + (int)threadIdx.x; i < j1; i += 256) {
      const float d = old_a[i] - new_a[i];
      eb += d * d;
    }
    for (int i = a + (int)threadIdx.x; i < e1; i += 256) {
      const float d = old_l[i] - new_l[i];
      ep += d * d;
    }
    s_b[threadIdx.x] = eb;
    s_p[threadIdx.x] = ep;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
      if ((int)threadIdx.x < off) {
        s_b[threadIdx.x] += s_b[threadIdx.x + off];
        s_p[threadIdx.x] += s_p[threadIdx.x + off];
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      effort[f] += s_b[0];
      effort[n_fil + f] += s_p[0];
    }
    __syncthreads();
  }
}

void launch_rest_effort(int n_fil, const int* fil_offset, const int* fil_flags, const float* old_a,
                        const float* new_a, const float* old_l, const float* new_l, float* effort, hipStream_t s) {
  if (n_fil <= 0) return;
  k_rest_effort<<<n_fil < 8192 ? n_fil : 8192, 256, 0, s>>>(n_fil, fil_offset, fil_flags, old_a, new_a, old_l, new_l,
                                                           effort);
}

}  // namespace mc
