// TSDF fusion of rendered median-depth maps (the mesh extraction of
// Sec. 4.1: the depth maps of all views are fused into a truncated signed
// distance field, Curless-Levoy) (gfx950).
//
// One lane per voxel, voxels x-fastest so that a wavefront's voxels project
// to neighbouring pixels (the depth-map gathers stay in L2).  For voxel
// centre X and every view with camera z > near whose projection falls in
// pixel (floor(u), floor(v)) of the image and whose median depth D there is
// positive: s = D - z; views with s >= -trunc add min(1, s / trunc) with
// weight 1.  Output: the mean contribution (0 where none) and the number of
// contributing views.  The camera transform is FP64 (the pixel lookup is a
// discrete decision; FP32 would move it by ~1e-5 px at 1600 px).
#include "common.hpp"
#include "grid.hpp"

namespace rade {
namespace {

constexpr int kT = 256;

__global__ void __launch_bounds__(kT)
k_tsdf_fuse(const rade_view* __restrict__ views, int V, const float* __restrict__ depth,
            double o0, double o1, double o2, double voxel, Grid3 grid, uint32_t nvox,
            double near_plane, float trunc, float* __restrict__ tsdf,
            float* __restrict__ weight) {
  // 64-bit counter: the stride must not wrap near 2^32
  for (uint64_t qq = (uint64_t)blockIdx.x * kT + threadIdx.x; qq < nvox;
       qq += (uint64_t)gridDim.x * kT) {
    const uint32_t q = (uint32_t)qq;
    uint32_t i, j, k;
    grid.split(q, i, j, k);
    const double X0 = o0 + ((double)i + 0.5) * voxel;
    const double X1 = o1 + ((double)j + 0.5) * voxel;
    const double X2 = o2 + ((double)k + 0.5) * voxel;
    float f = 0.0f;
    int w = 0;
    for (int vi = 0; vi < V; ++vi) {
      const rade_view& v = views[vi];
      const double x = (double)v.R[0] * X0 + (double)v.R[1] * X1 + (double)v.R[2] * X2 + v.t[0];
      const double y = (double)v.R[3] * X0 + (double)v.R[4] * X1 + (double)v.R[5] * X2 + v.t[1];
      const double z = (double)v.R[6] * X0 + (double)v.R[7] * X1 + (double)v.R[8] * X2 + v.t[2];
      if (!(z > near_plane)) continue;
      const double iz = 1.0 / z;
      const double u = (double)v.fx * x * iz + v.cx, uv = (double)v.fy * y * iz + v.cy;
      const double px = floor(u), py = floor(uv);
      if (!(px >= 0.0 && px < (double)v.width && py >= 0.0 && py < (double)v.height)) continue;
      const int64_t P = (int64_t)v.width * v.height;
      const float D = depth[2 * v.pix_offset + P + (int64_t)py * v.width + (int64_t)px];
      if (!(D > 0.0f)) continue;
      const double s = (double)D - z;
      if (s < -(double)trunc) continue;
      f += (float)fmin(1.0, s / (double)trunc);
      ++w;
    }
    tsdf[q] = w > 0 ? f / (float)w : 0.0f;
    weight[q] = (float)w;
  }
}

}  // namespace

hipError_t launch_tsdf_fuse(const rade_view* views, int V, const float* depth,
                            const double* origin, double voxel, int64_t nx, int64_t ny,
                            int64_t nz, double near_plane, float trunc, float* tsdf,
                            float* weight, hipStream_t st) {
  // the caller checks nx ny nz <= 2^32 - 1: 32-bit voxel indices
  const int64_t nvox = nx * ny * nz;
  if (nvox == 0) return hipSuccess;
  int64_t blocks = (nvox + kT - 1) / kT;
  if (blocks > (int64_t)1 << 20) blocks = (int64_t)1 << 20;  // grid-stride beyond
  hipLaunchKernelGGL(k_tsdf_fuse, dim3((unsigned)blocks), dim3(kT), 0, st, views, V, depth,
                     origin[0], origin[1], origin[2], voxel, Grid3((uint32_t)nx, (uint32_t)ny),
                     (uint32_t)nvox, near_plane, trunc, tsdf, weight);
  return hipGetLastError();
}

}  // namespace rade
