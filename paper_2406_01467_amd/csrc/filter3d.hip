// 3D smoothing filter of the Gaussians (the Mip-Splatting filter RaDe-GS
// trains with, Sec. 4.1) (gfx950).
//
// Per Gaussian, the largest sampling rate at which any view sees its centre,
// rate = fx / z (pixels per world unit at the centre's camera depth z), taken
// over the views with z > near whose image, widened by `margin` of its width
// and height on every side, holds the projected centre.  The filter is an
// isotropic 3D Gaussian of variance var = scale / rate^2 (0 when no view sees
// the centre) convolved into the Gaussian:
//   Sigma' = Sigma + var I = R diag(s_k^2 + var) R^T,  s'_k = sqrt(s_k^2 + var),
//   o' = o sqrt(prod s_k^2 / prod s'_k^2)   (the Gaussian's integral is kept).
// var depends on the means and cameras only and is held constant by the
// adjoint (it is recomputed from time to time during training, not learnt).
#include "common.hpp"

namespace rade {
namespace {

constexpr int kT = 256;

__global__ void __launch_bounds__(kT)
k_filter3d_var(const rade_view* __restrict__ views, int V, int64_t N,
               const float* __restrict__ means, double near_plane, float scale, float margin,
               float* __restrict__ var) {
  const int64_t g = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (g >= N) return;
  const double m0 = means[3 * g], m1 = means[3 * g + 1], m2 = means[3 * g + 2];
  double best = 0.0;
  for (int vi = 0; vi < V; ++vi) {
    const rade_view& v = views[vi];
    // camera-space centre (FP32 products are exact in FP64)
    const double x = (double)v.R[0] * m0 + (double)v.R[1] * m1 + (double)v.R[2] * m2 + v.t[0];
    const double y = (double)v.R[3] * m0 + (double)v.R[4] * m1 + (double)v.R[5] * m2 + v.t[1];
    const double z = (double)v.R[6] * m0 + (double)v.R[7] * m1 + (double)v.R[8] * m2 + v.t[2];
    if (!(z > near_plane)) continue;
    const double u = (double)v.fx * x / z + v.cx, w = (double)v.fy * y / z + v.cy;
    const double mx = (double)margin * v.width, my = (double)margin * v.height;
    if (u < -mx || u > v.width + mx || w < -my || w > v.height + my) continue;
    best = fmax(best, (double)v.fx / z);
  }
  var[g] = best > 0.0 ? (float)((double)scale / (best * best)) : 0.0f;
}

__global__ void __launch_bounds__(kT)
k_filter3d_apply(int64_t N, const float* __restrict__ scales, const float* __restrict__ opac,
                 const float* __restrict__ var, float* __restrict__ scales_out,
                 float* __restrict__ opac_out) {
  const int64_t g = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (g >= N) return;
  const float f = var[g];
  float ratio = 1.0f;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float s = scales[3 * g + k];
    const float s2 = s * s;
    const float t2 = s2 + f;
    scales_out[3 * g + k] = sqrtf(t2);
    ratio *= t2 > 0.0f ? s2 / t2 : 1.0f;
  }
  opac_out[g] = opac[g] * sqrtf(ratio);
}

// d s_k = d s'_k s_k / s'_k + d o' o' var / (s_k s'_k^2),  d o = d o' o' / o.
// d_scales / d_opac may alias d_scales_f / d_opac_f (elementwise).
__global__ void __launch_bounds__(kT)
k_filter3d_apply_bwd(int64_t N, const float* __restrict__ scales, const float* __restrict__ opac,
                     const float* __restrict__ var, const float* d_scales_f,
                     const float* d_opac_f, float* d_scales, float* d_opac) {
  const int64_t g = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (g >= N) return;
  const float f = var[g];
  float s[3], t2[3], ratio = 1.0f;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    s[k] = scales[3 * g + k];
    t2[k] = s[k] * s[k] + f;
    ratio *= t2[k] > 0.0f ? s[k] * s[k] / t2[k] : 1.0f;
  }
  const float root = sqrtf(ratio);
  const float go = d_opac_f[g];
  const float o_f = opac[g] * root;  // filtered opacity
  float ds[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float sf = sqrtf(t2[k]);
    const float a = sf > 0.0f ? d_scales_f[3 * g + k] * s[k] / sf : 0.0f;
    const float b = s[k] != 0.0f && t2[k] > 0.0f ? go * o_f * f / (s[k] * t2[k]) : 0.0f;
    ds[k] = a + b;
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) d_scales[3 * g + k] = ds[k];
  d_opac[g] = go * root;
}

}  // namespace

hipError_t launch_filter3d_var(const rade_view* views, int V, int64_t N, const float* means,
                               double near_plane, float scale, float margin, float* var,
                               hipStream_t st) {
  if (N == 0) return hipSuccess;
  hipLaunchKernelGGL(k_filter3d_var, dim3((unsigned)((N + kT - 1) / kT)), dim3(kT), 0, st, views,
                     V, N, means, near_plane, scale, margin, var);
  return hipGetLastError();
}

hipError_t launch_filter3d_apply(int64_t N, const float* scales, const float* opac,
                                 const float* var, float* scales_out, float* opac_out,
                                 hipStream_t st) {
  if (N == 0) return hipSuccess;
  hipLaunchKernelGGL(k_filter3d_apply, dim3((unsigned)((N + kT - 1) / kT)), dim3(kT), 0, st, N,
                     scales, opac, var, scales_out, opac_out);
  return hipGetLastError();
}

hipError_t launch_filter3d_apply_bwd(int64_t N, const float* scales, const float* opac,
                                     const float* var, const float* d_scales_f,
                                     const float* d_opac_f, float* d_scales, float* d_opac,
                                     hipStream_t st) {
  if (N == 0) return hipSuccess;
  hipLaunchKernelGGL(k_filter3d_apply_bwd, dim3((unsigned)((N + kT - 1) / kT)), dim3(kT), 0, st,
                     N, scales, opac, var, d_scales_f, d_opac_f, d_scales, d_opac);
  return hipGetLastError();
}

}  // namespace rade
