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
#include "common.hpp"

namespace rade {
namespace {

constexpr int kT = 256;

__device__ __forceinline__ int view_of_pixel(const rade_view* views, int V, int64_t pix) {
  int v = 0;
  while (v + 1 < V && views[v + 1].pix_offset <= pix) ++v;
  return v;
}

// Pass 1: per interior pixel, the loss term, dL/dA, dL/dN and the gradients
// of the two difference vectors (6 floats, kept for pass 2).  ACC adds the
// gradients into the maps; otherwise every pixel's entries are written
// (0 + x, so the bits equal adding into zeroed maps; border pixels get 0).
template <bool ACC>
__global__ void __launch_bounds__(kT)
k_nc_pass1(const rade_view* __restrict__ views, int V, int64_t total, const float* __restrict__ depth,
           const float* __restrict__ normal, const float* __restrict__ alpha, float weight,
           float* __restrict__ loss, float* __restrict__ d_normal, float* __restrict__ d_alpha,
           float* __restrict__ gdiff, float* __restrict__ partial) {
  const int64_t q = (int64_t)blockIdx.x * kT + threadIdx.x;
  float term = 0.0f;
  int v = 0;
  if (q < total) {
    v = view_of_pixel(views, V, q);
    const rade_view& vw = views[v];
    const int64_t o = vw.pix_offset, P = (int64_t)vw.width * vw.height;
    const int64_t pix = q - o;
    const int px = (int)(pix % vw.width), py = (int)(pix / vw.width);
    float* gd = gdiff + 6 * q;
    const bool interior = px >= 1 && py >= 1 && px <= vw.width - 2 && py <= vw.height - 2;
    if (!interior) {
      for (int k = 0; k < 6; ++k) gd[k] = 0.0f;
      if constexpr (!ACC) {
        d_alpha[o + pix] = 0.0f;
        d_normal[3 * o + pix] = 0.0f;
        d_normal[3 * o + P + pix] = 0.0f;
        d_normal[3 * o + 2 * P + pix] = 0.0f;
      }
    } else {
      const float wn = weight / (float)((vw.width - 2) * (vw.height - 2));
      const float* Dm = depth + 2 * o + P;  // median plane
      // Central differences of the back-projected points, written through
      // depth differences so FP32 does not cancel |P| ~ D against |dP| ~ D/f:
      // P(p +- x) = D(p +- x) (r(p) +- (1/fx, 0, 0)), r(p) = (rx, ry, 1).
      const float rx = ((float)px + 0.5f - vw.cx) / vw.fx;
      const float ry = ((float)py + 0.5f - vw.cy) / vw.fy;
      const float Dl = Dm[pix - 1], Dr = Dm[pix + 1];
      const float Du = Dm[pix - vw.width], Dd = Dm[pix + vw.width];
      const float dx_ = Dr - Dl, sx = Dr + Dl;
      const float dy_ = Dd - Du, sy = Dd + Du;
      const float du[3] = {dx_ * rx + sx / vw.fx, dx_ * ry, dx_};
      const float dv[3] = {dy_ * rx, dy_ * ry + sy / vw.fy, dy_};
      const float Pc[3] = {Dm[pix] * rx, Dm[pix] * ry, Dm[pix]};
      const float c[3] = {du[1] * dv[2] - du[2] * dv[1], du[2] * dv[0] - du[0] * dv[2],
                          du[0] * dv[1] - du[1] * dv[0]};
      const float cc = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
      const float N0 = normal[3 * o + pix], N1 = normal[3 * o + P + pix],
                  N2 = normal[3 * o + 2 * P + pix];
      const float A = alpha[o + pix];
      float nt[3] = {0.f, 0.f, 0.f};
      float gc[3] = {0.f, 0.f, 0.f};
      if (cc > 1e-30f) {
        const float inv = rsqrtf(cc);
        const float s = (c[0] * Pc[0] + c[1] * Pc[1] + c[2] * Pc[2]) > 0.0f ? -1.0f : 1.0f;
        const float ch[3] = {c[0] * inv, c[1] * inv, c[2] * inv};
        for (int k = 0; k < 3; ++k) nt[k] = s * ch[k];
        // dL/dc = -wn d(N . n~)/dc = -wn s (N - (N . c^) c^) / |c|
        const float nd = N0 * ch[0] + N1 * ch[1] + N2 * ch[2];
        const float Nv[3] = {N0, N1, N2};
        for (int k = 0; k < 3; ++k) gc[k] = -wn * s * (Nv[k] - nd * ch[k]) * inv;
      }
      term = A - (N0 * nt[0] + N1 * nt[1] + N2 * nt[2]);
      // d/d(du) = dv x gc, d/d(dv) = gc x du
      gd[0] = dv[1] * gc[2] - dv[2] * gc[1];
      gd[1] = dv[2] * gc[0] - dv[0] * gc[2];
      gd[2] = dv[0] * gc[1] - dv[1] * gc[0];
      gd[3] = gc[1] * du[2] - gc[2] * du[1];
      gd[4] = gc[2] * du[0] - gc[0] * du[2];
      gd[5] = gc[0] * du[1] - gc[1] * du[0];
      const float a0 = ACC ? d_alpha[o + pix] : 0.0f;
      const float n0 = ACC ? d_normal[3 * o + pix] : 0.0f;
      const float n1 = ACC ? d_normal[3 * o + P + pix] : 0.0f;
      const float n2 = ACC ? d_normal[3 * o + 2 * P + pix] : 0.0f;
      d_alpha[o + pix] = a0 + wn;
      d_normal[3 * o + pix] = n0 - wn * nt[0];
      d_normal[3 * o + P + pix] = n1 - wn * nt[1];
      d_normal[3 * o + 2 * P + pix] = n2 - wn * nt[2];
      term *= wn;
    }
  }
  // loss value: a workgroup inside one view writes its sum to partial[block]
  // (added up per view by k_nc_sum); a workgroup that straddles two views
  // (rare) writes 0 there and adds its terms per lane.
  __shared__ float red[kT / 64];
  const int64_t q0 = (int64_t)blockIdx.x * kT;
  const int64_t q1 = min(total, q0 + kT) - 1;
  const int v0 = view_of_pixel(views, V, q0), v1 = view_of_pixel(views, V, q1);
  if (v0 == v1) {
    float x = term;
    for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
      float t = 0.0f;
      for (int i = 0; i < kT / 64; ++i) t += red[i];
      partial[blockIdx.x] = t;
    }
  } else {
    if (threadIdx.x == 0) partial[blockIdx.x] = 0.0f;
    if (term != 0.0f) atomicAdd(loss + v, term);
  }
}

// Loss per view: workgroup (v, c) sums chunk c of view v's pass-1 partials
// and adds it to loss[v] (kSumChunks atomics per view).
constexpr int kSumChunks = 32;

__global__ void __launch_bounds__(kT)
k_nc_sum(const rade_view* __restrict__ views, const float* __restrict__ partial,
         float* __restrict__ loss) {
  __shared__ float red[kT / 64];
  const rade_view& vw = views[blockIdx.x];
  const int64_t b0 = vw.pix_offset / kT;
  const int64_t b1 = (vw.pix_offset + (int64_t)vw.width * vw.height + kT - 1) / kT;
  const int64_t per = (b1 - b0 + kSumChunks - 1) / kSumChunks;
  const int64_t c0 = b0 + (int64_t)blockIdx.y * per, c1 = min(b1, c0 + per);
  float x = 0.0f;
  for (int64_t b = c0 + threadIdx.x; b < c1; b += kT) x += partial[b];
  for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    float t = 0.0f;
    for (int i = 0; i < kT / 64; ++i) t += red[i];
    if (c0 < c1) atomicAdd(loss + blockIdx.x, t);
  }
}

// Pass 2: dL/dD_med(q) = r(q) . (g_du(q-x) - g_du(q+x) + g_dv(q-y) - g_dv(q+y)).
// Without ACC both depth planes are written (the expected-depth plane gets 0).
template <bool ACC>
__global__ void __launch_bounds__(kT)
k_nc_pass2(const rade_view* __restrict__ views, int V, int64_t total,
           const float* __restrict__ gdiff, float* __restrict__ d_depth) {
  const int64_t q = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (q >= total) return;
  const int v = view_of_pixel(views, V, q);
  const rade_view& vw = views[v];
  const int64_t o = vw.pix_offset, P = (int64_t)vw.width * vw.height;
  const int64_t pix = q - o;
  const int px = (int)(pix % vw.width), py = (int)(pix / vw.width);
  float g[3] = {0.f, 0.f, 0.f};
  // each neighbour's entry is zero when that neighbour is not interior
  if (px >= 1) for (int k = 0; k < 3; ++k) g[k] += gdiff[6 * (q - 1) + k];
  if (px + 1 < vw.width) for (int k = 0; k < 3; ++k) g[k] -= gdiff[6 * (q + 1) + k];
  if (py >= 1) for (int k = 0; k < 3; ++k) g[k] += gdiff[6 * (q - vw.width) + 3 + k];
  if (py + 1 < vw.height) for (int k = 0; k < 3; ++k) g[k] -= gdiff[6 * (q + vw.width) + 3 + k];
  const float rx = ((float)px + 0.5f - vw.cx) / vw.fx;
  const float ry = ((float)py + 0.5f - vw.cy) / vw.fy;
  const float prev = ACC ? d_depth[2 * o + P + pix] : 0.0f;
  d_depth[2 * o + P + pix] = prev + (g[0] * rx + g[1] * ry + g[2]);
  if constexpr (!ACC) d_depth[2 * o + pix] = 0.0f;
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

size_t normal_consistency_workspace(int64_t total_pixels) {
  const int64_t blocks = (total_pixels + kT - 1) / kT;
  return (size_t)total_pixels * 6 * sizeof(float) + (size_t)blocks * sizeof(float) + 256;
}

hipError_t launch_normal_consistency(const rade_view* views, int V, int64_t total,
                                     const float* depth, const float* normal,
                                     const float* alpha, float weight, float* loss,
                                     float* d_depth, float* d_normal, float* d_alpha,
                                     bool accumulate, void* ws, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_f, dim3((V + 255) / 256), dim3(256), 0, st, loss, V);
  if (total == 0) return hipGetLastError();
  float* gdiff = static_cast<float*>(ws);
  const unsigned blocks = (unsigned)((total + kT - 1) / kT);
  float* partial = gdiff + 6 * total;
  if (accumulate)
    hipLaunchKernelGGL(k_nc_pass1<true>, dim3(blocks), dim3(kT), 0, st, views, V, total, depth,
                       normal, alpha, weight, loss, d_normal, d_alpha, gdiff, partial);
  else
    hipLaunchKernelGGL(k_nc_pass1<false>, dim3(blocks), dim3(kT), 0, st, views, V, total, depth,
                       normal, alpha, weight, loss, d_normal, d_alpha, gdiff, partial);
  hipLaunchKernelGGL(k_nc_sum, dim3(V, kSumChunks), dim3(kT), 0, st, views, partial, loss);
  if (accumulate)
    hipLaunchKernelGGL(k_nc_pass2<true>, dim3(blocks), dim3(kT), 0, st, views, V, total, gdiff,
                       d_depth);
  else
    hipLaunchKernelGGL(k_nc_pass2<false>, dim3(blocks), dim3(kT), 0, st, views, V, total, gdiff,
                       d_depth);
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
