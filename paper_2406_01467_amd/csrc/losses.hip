// Normal-consistency regulariser on the rendered maps (Sec. 3.4, Eq. 24) and
// its gradient, fused into two pixel-parallel kernels (gfx950).
//
// Per view, over interior pixels p (one pixel away from every border):
//   P(q)  = D_med(q) * ((x_q + 1/2 - cx)/fx, (y_q + 1/2 - cy)/fy, 1)
//           (back-projected median depth)
//   c(p)  = (P(p+x) - P(p-x)) x (P(p+y) - P(p-y))   (central differences)
//   n~(p) = s c / |c|, s = +-1 so that n~ faces the camera (n~ . P(p) <= 0)
//   L_n   = weight / n_int * sum_p (A(p) - N(p) . n~(p))
// Eq. 24 writes sum_i w_i (1 - n_i . n~) per pixel; with A = sum_i w_i and
// N = sum_i w_i n_i that is A - N . n~, exactly, from the blended maps.
// The gradient flows into A, N and (through n~, not detached) D_med.
#include <mutex>

#include "common.hpp"

namespace rade {
namespace {

constexpr int kT = 256;

__device__ __forceinline__ int view_of_pixel(const rade_view* views, int V, int64_t pix) {
  int v = 0;
  while (v + 1 < V && views[v + 1].pix_offset <= pix) ++v;
  return v;
}

// The loss and its gradient in one kernel over 32 x 8 pixel blocks of each
// view (blocks of the views back to back).  Per pixel the arithmetic is that
// of the two passes it replaces: the loss term, dL/dA, dL/dN and the
// gradients of the two difference vectors (6 floats) for every interior
// pixel, then dL/dD_med(q) = r(q) . (g_du(q-x) - g_du(q+x) + g_dv(q-y) -
// g_dv(q+y)).  The block computes the difference-vector gradients for itself
// and a one-pixel ring around it (from the median depths of a two-pixel
// ring, staged in LDS), so none of them goes through memory.  ACC adds the
// gradients into the maps; otherwise every pixel's entries are written (0 +
// x, so the bits equal adding into zeroed maps; border pixels and the
// expected-depth plane get 0).  The block's loss sum goes to partial[block].
// A block is 32 x 8 pixels (a row of it is one 128-byte line of a map).
constexpr int kBX = 32, kBY = 8;
constexpr int kGX = kBX + 2, kGY = kBY + 2;  // with the ring of difference-vector gradients
constexpr int kDX = kBX + 4, kDY = kBY + 4;  // with the ring of depths they read
static_assert(kBX * kBY == kT, "one thread per pixel of a block");

__device__ __forceinline__ int nc_blocks_x(const rade_view& vw) { return (vw.width + kBX - 1) / kBX; }
__device__ __forceinline__ int64_t nc_blocks(const rade_view& vw) {
  return (int64_t)nc_blocks_x(vw) * ((vw.height + kBY - 1) / kBY);
}

// View of block b and the view's first block index.
__device__ __forceinline__ int nc_view_of_block(const rade_view* views, int V, int64_t b,
                                                int64_t& first) {
  int64_t acc = 0;
  for (int v = 0; v < V; ++v) {
    const int64_t n = nc_blocks(views[v]);
    if (b < acc + n || v == V - 1) {
      first = acc;
      return v;
    }
    acc += n;
  }
  first = 0;
  return 0;
}

template <bool ACC>
__global__ void __launch_bounds__(kT)
k_nc(const rade_view* __restrict__ views, int V, int64_t nblocks, const float* __restrict__ depth,
     const float* __restrict__ normal, const float* __restrict__ alpha, float weight,
     float* __restrict__ d_depth, float* __restrict__ d_normal, float* __restrict__ d_alpha,
     float* __restrict__ partial) {
  __shared__ float sD[kDX * kDY];
  __shared__ float sG[6][kGX * kGY];
  __shared__ float red[kT / 64];
  const int64_t b = blockIdx.x;
  if (b >= nblocks) return;  // uniform per block
  int64_t first;
  const int v = nc_view_of_block(views, V, b, first);
  const rade_view& vw = views[v];
  const int W = vw.width, H = vw.height;
  const int nbx = nc_blocks_x(vw);
  const int bi = (int)(b - first);
  const int x0 = (bi % nbx) * kBX, y0 = (bi / nbx) * kBY;
  const int64_t o = vw.pix_offset, P = (int64_t)W * H;
  const float* Dm = depth + 2 * o + P;  // median plane
  const float wn = weight / (float)((W - 2) * (H - 2));
  const float ifx = 1.0f / vw.fx, ify = 1.0f / vw.fy;  // one division per block
  // Region pixels (the block and a one-pixel ring) of this thread: i = t and
  // i = t + kT.  Their normals and alphas are loaded first, together with
  // the median depths of the block and a two-pixel ring (0 outside the
  // view), so every global load of the block is in flight at once.
  constexpr int kR = (kGX * kGY + kT - 1) / kT;
  float Nr[kR][3], Ar[kR];
#pragma unroll
  for (int k = 0; k < kR; ++k) {
    const int i = threadIdx.x + k * kT;
    const int gx = i % kGX, gy = i / kGX;
    const int px = x0 - 1 + gx, py = y0 - 1 + gy;
    const bool interior =
        i < kGX * kGY && px >= 1 && py >= 1 && px <= W - 2 && py <= H - 2;
    const bool own = gx >= 1 && gy >= 1 && gx <= kBX && gy <= kBY;
    const int64_t pix = (int64_t)py * W + px;
    Nr[k][0] = interior ? normal[3 * o + pix] : 0.0f;
    Nr[k][1] = interior ? normal[3 * o + P + pix] : 0.0f;
    Nr[k][2] = interior ? normal[3 * o + 2 * P + pix] : 0.0f;
    Ar[k] = interior && own ? alpha[o + pix] : 0.0f;
  }
  for (int i = threadIdx.x; i < kDX * kDY; i += kT) {
    const int x = x0 - 2 + i % kDX, y = y0 - 2 + i / kDX;
    sD[i] = (x >= 0 && y >= 0 && x < W && y < H) ? Dm[(int64_t)y * W + x] : 0.0f;
  }
  __syncthreads();
  float term = 0.0f;
  // pass 1 over the block and the ring; region pixel i = (gx, gy)
#pragma unroll
  for (int k = 0; k < kR; ++k) {
    const int i = threadIdx.x + k * kT;
    if (i >= kGX * kGY) break;
    const int gx = i % kGX, gy = i / kGX;
    const int px = x0 - 1 + gx, py = y0 - 1 + gy;
    const bool own = gx >= 1 && gy >= 1 && gx <= kBX && gy <= kBY && px < W && py < H;
    const bool interior = px >= 1 && py >= 1 && px <= W - 2 && py <= H - 2;
    float gd[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    const int64_t pix = (int64_t)py * W + px;
    if (interior) {
      // central differences of the back-projected points, written through
      // depth differences so FP32 does not cancel |P| ~ D against |dP| ~ D/f:
      // P(p +- x) = D(p +- x) (r(p) +- (1/fx, 0, 0)), r(p) = (rx, ry, 1)
      const float rx = ((float)px + 0.5f - vw.cx) * ifx;
      const float ry = ((float)py + 0.5f - vw.cy) * ify;
      const int c = (gy + 1) * kDX + (gx + 1);  // this pixel in sD
      const float Dl = sD[c - 1], Dr = sD[c + 1];
      const float Du = sD[c - kDX], Dd = sD[c + kDX];
      const float dx_ = Dr - Dl, sx = Dr + Dl;
      const float dy_ = Dd - Du, sy = Dd + Du;
      const float du[3] = {dx_ * rx + sx * ifx, dx_ * ry, dx_};
      const float dv[3] = {dy_ * rx, dy_ * ry + sy * ify, dy_};
      const float Pc[3] = {sD[c] * rx, sD[c] * ry, sD[c]};
      const float cr[3] = {du[1] * dv[2] - du[2] * dv[1], du[2] * dv[0] - du[0] * dv[2],
                           du[0] * dv[1] - du[1] * dv[0]};
      const float cc = cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2];
      const float N0 = Nr[k][0], N1 = Nr[k][1], N2 = Nr[k][2];
      float nt[3] = {0.f, 0.f, 0.f};
      float gc[3] = {0.f, 0.f, 0.f};
      if (cc > 1e-30f) {
        const float inv = rsqrtf(cc);
        const float s = (cr[0] * Pc[0] + cr[1] * Pc[1] + cr[2] * Pc[2]) > 0.0f ? -1.0f : 1.0f;
        const float ch[3] = {cr[0] * inv, cr[1] * inv, cr[2] * inv};
        for (int j = 0; j < 3; ++j) nt[j] = s * ch[j];
        // dL/dc = -wn d(N . n~)/dc = -wn s (N - (N . c^) c^) / |c|
        const float nd = N0 * ch[0] + N1 * ch[1] + N2 * ch[2];
        const float Nv[3] = {N0, N1, N2};
        for (int j = 0; j < 3; ++j) gc[j] = -wn * s * (Nv[j] - nd * ch[j]) * inv;
      }
      // d/d(du) = dv x gc, d/d(dv) = gc x du
      gd[0] = dv[1] * gc[2] - dv[2] * gc[1];
      gd[1] = dv[2] * gc[0] - dv[0] * gc[2];
      gd[2] = dv[0] * gc[1] - dv[1] * gc[0];
      gd[3] = gc[1] * du[2] - gc[2] * du[1];
      gd[4] = gc[2] * du[0] - gc[0] * du[2];
      gd[5] = gc[0] * du[1] - gc[1] * du[0];
      if (own) {
        term += (Ar[k] - (N0 * nt[0] + N1 * nt[1] + N2 * nt[2])) * wn;
        const float a0 = ACC ? d_alpha[o + pix] : 0.0f;
        const float n0 = ACC ? d_normal[3 * o + pix] : 0.0f;
        const float n1 = ACC ? d_normal[3 * o + P + pix] : 0.0f;
        const float n2 = ACC ? d_normal[3 * o + 2 * P + pix] : 0.0f;
        d_alpha[o + pix] = a0 + wn;
        d_normal[3 * o + pix] = n0 - wn * nt[0];
        d_normal[3 * o + P + pix] = n1 - wn * nt[1];
        d_normal[3 * o + 2 * P + pix] = n2 - wn * nt[2];
      }
    } else if (own && !ACC) {
      d_alpha[o + pix] = 0.0f;
      d_normal[3 * o + pix] = 0.0f;
      d_normal[3 * o + P + pix] = 0.0f;
      d_normal[3 * o + 2 * P + pix] = 0.0f;
    }
#pragma unroll
    for (int j = 0; j < 6; ++j) sG[j][i] = gd[j];
  }
  __syncthreads();
  // pass 2 for the block's own pixels
  {
    const int lx = threadIdx.x % kBX, ly = threadIdx.x / kBX;
    const int px = x0 + lx, py = y0 + ly;
    if (px < W && py < H) {
      const int i = (ly + 1) * kGX + (lx + 1);
      float g[3] = {0.f, 0.f, 0.f};
      // a neighbour's entries are zero when it is not interior
      if (px >= 1) for (int k = 0; k < 3; ++k) g[k] += sG[k][i - 1];
      if (px + 1 < W) for (int k = 0; k < 3; ++k) g[k] -= sG[k][i + 1];
      if (py >= 1) for (int k = 0; k < 3; ++k) g[k] += sG[3 + k][i - kGX];
      if (py + 1 < H) for (int k = 0; k < 3; ++k) g[k] -= sG[3 + k][i + kGX];
      const float rx = ((float)px + 0.5f - vw.cx) * ifx;
      const float ry = ((float)py + 0.5f - vw.cy) * ify;
      const int64_t pix = (int64_t)py * W + px;
      const float prev = ACC ? d_depth[2 * o + P + pix] : 0.0f;
      d_depth[2 * o + P + pix] = prev + (g[0] * rx + g[1] * ry + g[2]);
      if constexpr (!ACC) d_depth[2 * o + pix] = 0.0f;
    }
  }
  // the block's loss sum (a thread's terms are those of its own pixels)
  float x = term;
  for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    float t = 0.0f;
    for (int k = 0; k < kT / 64; ++k) t += red[k];
    partial[b] = t;
  }
}

// Loss per view: workgroup v sums view v's block partials and writes loss[v].
__global__ void __launch_bounds__(kT)
k_nc_sum(const rade_view* __restrict__ views, const float* __restrict__ partial,
         float* __restrict__ loss) {
  __shared__ float red[kT / 64];
  int64_t b0 = 0;
  for (int v = 0; v < (int)blockIdx.x; ++v) b0 += nc_blocks(views[v]);
  const int64_t b1 = b0 + nc_blocks(views[blockIdx.x]);
  float x = 0.0f;
#pragma unroll 4
  for (int64_t b = b0 + threadIdx.x; b < b1; b += kT) x += partial[b];
  for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    float t = 0.0f;
    for (int i = 0; i < kT / 64; ++i) t += red[i];
    loss[blockIdx.x] = t;
  }
}

// Gradient of the mean absolute colour difference of each view (3 planes):
// d_color = weight sign(color - target) / (3 W H), written for every pixel.
__global__ void __launch_bounds__(kT)
k_l1_color_grad(const rade_view* __restrict__ views, int V, int64_t total,
                const float* __restrict__ color, const float* __restrict__ target, double weight,
                float* __restrict__ d_color) {
  const int64_t q = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (q >= total) return;
  const rade_view& vw = views[view_of_pixel(views, V, q)];
  const int64_t o = vw.pix_offset, P = (int64_t)vw.width * vw.height;
  const int64_t pix = q - o;
  const float w = (float)(weight / (3.0 * (double)P));
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const int64_t i = 3 * o + c * P + pix;
    const float d = color[i] - target[i];
    const float s = d > 0.0f ? 1.0f : d < 0.0f ? -1.0f : d;  // sign, NaN kept
    d_color[i] = s * w;
  }
}

__global__ void k_zero_f(float* __restrict__ a, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0.0f;
}

}  // namespace

// Number of 32x8 pixel blocks (one loss partial each) over the views.
int64_t normal_consistency_blocks(const rade_view* views_host, int V) {
  int64_t nb = 0;
  for (int v = 0; v < V; ++v)
    nb += (int64_t)((views_host[v].width + kBX - 1) / kBX) * ((views_host[v].height + kBY - 1) / kBY);
  return nb;
}

// One loss partial per block; every block holds at least one pixel.
size_t normal_consistency_workspace(int64_t total_pixels) {
  return (size_t)total_pixels * sizeof(float) + 256;
}

namespace {
// Scratch of the allocation-free entry point: one loss partial per block.
// Host code never passes the array's name to a kernel (on the host it is a
// stand-in, not a device address): it uses the address looked up below.
static __device__ __align__(256) float scratch[RADE_NC_NOALLOC_MAX_BLOCKS];

constexpr int kScratchDevices = 64;
std::mutex scratch_mu;
void* scratch_dev[kScratchDevices];  // per device ordinal, looked up once
}  // namespace

// Device address of `scratch` on the calling thread's current device, looked
// up on the first call made with that device current.
hipError_t nc_scratch_address(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kScratchDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_dev[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    scratch_dev[dev] = p;
  }
  *out = scratch_dev[dev];
  return hipSuccess;
}

hipError_t launch_normal_consistency(const rade_view* views_host, const rade_view* views, int V,
                                     int64_t total, const float* depth, const float* normal,
                                     const float* alpha, float weight, float* loss,
                                     float* d_depth, float* d_normal, float* d_alpha,
                                     bool accumulate, void* ws, hipStream_t st) {
  if (total == 0) {
    hipLaunchKernelGGL(k_zero_f, dim3((V + 255) / 256), dim3(256), 0, st, loss, V);
    return hipGetLastError();
  }
  const int64_t nb = normal_consistency_blocks(views_host, V);
  float* partial = static_cast<float*>(ws);
  if (accumulate)
    hipLaunchKernelGGL(k_nc<true>, dim3((unsigned)nb), dim3(kT), 0, st, views, V, nb, depth,
                       normal, alpha, weight, d_depth, d_normal, d_alpha, partial);
  else
    hipLaunchKernelGGL(k_nc<false>, dim3((unsigned)nb), dim3(kT), 0, st, views, V, nb, depth,
                       normal, alpha, weight, d_depth, d_normal, d_alpha, partial);
  hipLaunchKernelGGL(k_nc_sum, dim3(V), dim3(kT), 0, st, views, partial, loss);
  return hipGetLastError();
}

hipError_t launch_l1_color_grad(const rade_view* views, int V, int64_t total, const float* color,
                                const float* target, double weight, float* d_color,
                                hipStream_t st) {
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_l1_color_grad, dim3((unsigned)((total + kT - 1) / kT)), dim3(kT), 0, st,
                     views, V, total, color, target, weight, d_color);
  return hipGetLastError();
}

}  // namespace rade
