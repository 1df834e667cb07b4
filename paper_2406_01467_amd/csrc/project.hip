// Projection of 3D Gaussians to screen-space splats and its adjoint (gfx950).
//
// One lane per Gaussian; the lane loops over the views so the parameters
// (up to 59 floats) are read from HBM once per batch of views.  The geometry
// is evaluated in FP64: the splat centre must be known to well under 1e-5 px
// for 1e-5 agreement of the blended maps at 1600 px images, which FP32
// (ulp(1600) = 1.2e-4) cannot provide.  MI355X runs FP64 FMA at the rate of
// FP32 non-packed FMA, and this kernel is bound by memory traffic.
//
// Math (RaDe-GS, arXiv 2406.01467):
//   Sigma = R S S^T R^T (Eq. 1); ray-space covariance Sigma' = J W Sigma W^T
//   J^T (Eq. 2) with the local affine Jacobian J of the map
//   x -> (fx x/z + cx, fy y/z + cy, |x|) (Sec. 3.2.2).  Written here as
//   Sigma' = T T^T with T = J (W R_g) diag(s).
//   Footprint B = Sigma'[0:2,0:2] + dilation I; plane slope
//   q = -Sigma'[0:2,0:2]^-1 Sigma'[0:2,2], which equals the first two entries
//   of v'^T Sigma'^-1 / (v'^T Sigma'^-1 v') (Eq. 13) by the Schur complement;
//   p = (z_c / t_c) q (Eq. 15-17); n = normalize(J^T (-(q, 1))) (Eq. 21-22).
#include "common.hpp"

namespace rade {
namespace {

// Real SH basis up to degree 3 (16 values), Condon-Shortley phase, order
// m = -l..l.  Constants: 1/(2 sqrt(pi)); sqrt(3/(4 pi)); sqrt(15/pi)/2,
// sqrt(5/pi)/4, sqrt(15/pi)/4; sqrt(35/(2 pi))/4, sqrt(105/pi)/2,
// sqrt(21/(2 pi))/4, sqrt(7/pi)/4, sqrt(105/pi)/4.
constexpr double kY0 = 0.28209479177387814;
constexpr double kY1 = 0.48860251190291992;
constexpr double kY2a = 1.0925484305920792;
constexpr double kY2b = 0.31539156525252005;
constexpr double kY2c = 0.54627421529603959;
constexpr double kY3a = 0.59004358992664352;
constexpr double kY3b = 2.8906114426405538;
constexpr double kY3c = 0.45704579946446572;
constexpr double kY3d = 0.37317633259011546;
constexpr double kY3e = 1.4453057213202769;

// FP64: a colour is 1/2 plus a sum of up to 48 products that may cancel, so
// colours near zero need more than FP32 round-off of the terms.
__device__ __forceinline__ void sh_basis(int deg, double x, double y, double z, double* Y) {
  Y[0] = kY0;
  if (deg < 1) return;
  Y[1] = -kY1 * y;
  Y[2] = kY1 * z;
  Y[3] = -kY1 * x;
  if (deg < 2) return;
  const double xx = x * x, yy = y * y, zz = z * z;
  const double xy = x * y, yz = y * z, xz = x * z;
  Y[4] = kY2a * xy;
  Y[5] = -kY2a * yz;
  Y[6] = kY2b * (2.0 * zz - xx - yy);
  Y[7] = -kY2a * xz;
  Y[8] = kY2c * (xx - yy);
  if (deg < 3) return;
  Y[9] = -kY3a * y * (3.0 * xx - yy);
  Y[10] = kY3b * xy * z;
  Y[11] = -kY3c * y * (4.0 * zz - xx - yy);
  Y[12] = kY3d * z * (2.0 * zz - 3.0 * xx - 3.0 * yy);
  Y[13] = -kY3c * x * (4.0 * zz - xx - yy);
  Y[14] = kY3e * z * (xx - yy);
  Y[15] = -kY3a * x * (xx - 3.0 * yy);
}

// Gradient of sum_k c_k Y_k(x, y, z) with respect to (x, y, z) (unit sphere
// constraint not applied).
__device__ __forceinline__ void sh_grad(int deg, double x, double y, double z, const double* c,
                                        double* g) {
  g[0] = g[1] = g[2] = 0.0;
  if (deg < 1) return;
  g[0] += -kY1 * c[3];
  g[1] += -kY1 * c[1];
  g[2] += kY1 * c[2];
  if (deg < 2) return;
  const double xx = x * x, yy = y * y, zz = z * z;
  g[0] += kY2a * y * c[4] - kY2a * z * c[7] - 2.0 * kY2b * x * c[6] + 2.0 * kY2c * x * c[8];
  g[1] += kY2a * x * c[4] - kY2a * z * c[5] - 2.0 * kY2b * y * c[6] - 2.0 * kY2c * y * c[8];
  g[2] += -kY2a * y * c[5] + 4.0 * kY2b * z * c[6] - kY2a * x * c[7];
  if (deg < 3) return;
  // Y9 = -a y (3xx - yy)
  g[0] += -kY3a * 6.0 * x * y * c[9];
  g[1] += -kY3a * (3.0 * xx - 3.0 * yy) * c[9];
  // Y10 = b x y z
  g[0] += kY3b * y * z * c[10];
  g[1] += kY3b * x * z * c[10];
  g[2] += kY3b * x * y * c[10];
  // Y11 = -c y (4zz - xx - yy)
  g[0] += kY3c * 2.0 * x * y * c[11];
  g[1] += -kY3c * (4.0 * zz - xx - 3.0 * yy) * c[11];
  g[2] += -kY3c * 8.0 * y * z * c[11];
  // Y12 = d z (2zz - 3xx - 3yy)
  g[0] += -kY3d * 6.0 * x * z * c[12];
  g[1] += -kY3d * 6.0 * y * z * c[12];
  g[2] += kY3d * (6.0 * zz - 3.0 * xx - 3.0 * yy) * c[12];
  // Y13 = -c x (4zz - xx - yy)
  g[0] += -kY3c * (4.0 * zz - 3.0 * xx - yy) * c[13];
  g[1] += kY3c * 2.0 * x * y * c[13];
  g[2] += -kY3c * 8.0 * x * z * c[13];
  // Y14 = e z (xx - yy)
  g[0] += kY3e * 2.0 * x * z * c[14];
  g[1] += -kY3e * 2.0 * y * z * c[14];
  g[2] += kY3e * (xx - yy) * c[14];
  // Y15 = -a x (xx - 3yy)
  g[0] += -kY3a * (3.0 * xx - 3.0 * yy) * c[15];
  g[1] += kY3a * 6.0 * x * y * c[15];
}

// One Gaussian's 3K SH coefficients (row g of the N x K x 3 array) in
// registers.  VEC: the row is a whole number of 16-byte words and aligned,
// so it moves in dwordx4 loads/stores (a wave's 64 rows are 64 separate
// cache lines per instruction; 4x fewer instructions than dword access).
template <int K, bool VEC>
__device__ __forceinline__ void load_row(const float* __restrict__ p, float (&c)[3 * K]) {
  if constexpr (VEC) {
    const float4* p4 = reinterpret_cast<const float4*>(p);
#pragma unroll
    for (int i = 0; i < 3 * K / 4; ++i) {
      const float4 t = p4[i];
      c[4 * i] = t.x; c[4 * i + 1] = t.y; c[4 * i + 2] = t.z; c[4 * i + 3] = t.w;
    }
  } else {
#pragma unroll
    for (int i = 0; i < 3 * K; ++i) c[i] = p[i];
  }
}

template <int K, bool VEC>
__device__ __forceinline__ void store_row(float* __restrict__ p, const float (&c)[3 * K],
                                          bool accumulate) {
  if constexpr (VEC) {
    float4* p4 = reinterpret_cast<float4*>(p);
#pragma unroll
    for (int i = 0; i < 3 * K / 4; ++i) {
      float4 t = make_float4(c[4 * i], c[4 * i + 1], c[4 * i + 2], c[4 * i + 3]);
      if (accumulate) {
        const float4 o = p4[i];
        t.x += o.x; t.y += o.y; t.z += o.z; t.w += o.w;
      }
      p4[i] = t;
    }
  } else {
#pragma unroll
    for (int i = 0; i < 3 * K; ++i) p[i] = accumulate ? p[i] + c[i] : c[i];
  }
}

template <int K>
__device__ __forceinline__ bool row_finite(const float (&c)[3 * K]) {
  bool ok = true;
#pragma unroll
  for (int i = 0; i < 3 * K; ++i) ok = ok && isfinite(c[i]);
  return ok;
}

// Colour of one view: max(0, sum_k coef_k Y_k(dir) + 1/2) per channel.
// raw[] keeps the unclamped values for the clamp decision of the backward
// pass.
template <int K>
__device__ __forceinline__ void sh_colour(int deg, const double* dir, const float (&coef)[3 * K],
                                          double* raw) {
  double Y[16];
  sh_basis(deg, dir[0], dir[1], dir[2], Y);
  raw[0] = raw[1] = raw[2] = 0.0;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    raw[0] += (double)coef[3 * k + 0] * Y[k];
    raw[1] += (double)coef[3 * k + 1] * Y[k];
    raw[2] += (double)coef[3 * k + 2] * Y[k];
  }
  raw[0] += 0.5; raw[1] += 0.5; raw[2] += 0.5;
}

// Unit viewing direction from the camera centre to the mean; returns 1/|d|.
__device__ __forceinline__ double view_dir(const double* mu, const double* C, double* u) {
  const double d0 = mu[0] - C[0], d1 = mu[1] - C[1], d2 = mu[2] - C[2];
  const double idn = 1.0 / sqrt(d0 * d0 + d1 * d1 + d2 * d2);
  u[0] = d0 * idn; u[1] = d1 * idn; u[2] = d2 * idn;
  return idn;
}

struct ViewD {
  double R[9], t[3], fx, fy, cx, cy, limx, limy, C[3];
  int W, H, tiles_x;
};

__device__ __forceinline__ ViewD load_view(const rade_view& v, double fov_clamp) {
  ViewD o;
  for (int i = 0; i < 9; ++i) o.R[i] = (double)v.R[i];
  for (int i = 0; i < 3; ++i) o.t[i] = (double)v.t[i];
  o.fx = v.fx; o.fy = v.fy; o.cx = v.cx; o.cy = v.cy;
  o.W = v.width; o.H = v.height; o.tiles_x = v.tiles_x;
  o.limx = fov_clamp * (double)v.width / (2.0 * o.fx);
  o.limy = fov_clamp * (double)v.height / (2.0 * o.fy);
  // camera centre in world coordinates: C = -R^T t
  for (int i = 0; i < 3; ++i)
    o.C[i] = -(o.R[i] * o.t[0] + o.R[3 + i] * o.t[1] + o.R[6 + i] * o.t[2]);
  return o;
}

// Everything the forward computes for one (view, Gaussian) and the backward
// needs again.
struct Geo {
  double X, Y, Z, tc;
  double J0[3], J1[3], J2[3];   // rows of J
  bool clx, cly;
  double xi, eta;
  double Wm[9];                 // W R_g diag(s): column k = (W R_g)[:,k] * s_k
  double T[9];                  // J Wm
  double B00, B01, B11, b0, b1; // Sigma' entries (undilated footprint and coupling)
  double D00, D11;              // dilated diagonal (D01 = B01)
  double detD;
  bool degenerate;
  double q0, q1;
  double nr[3], nlen;
};

struct Params {
  double mu[3], s[3], qn[4], qinv, Rg[9];
  float o;
};

__device__ __forceinline__ bool finitef(float x) { return isfinite(x); }

// Quaternion (w,x,y,z), unit -> rotation matrix (row-major).
__device__ __forceinline__ void quat_to_mat(const double* q, double* Rm) {
  const double w = q[0], x = q[1], y = q[2], z = q[3];
  const double xx = x * x, yy = y * y, zz = z * z;
  const double xy = x * y, xz = x * z, yz = y * z, wx = w * x, wy = w * y, wz = w * z;
  Rm[0] = 1.0 - 2.0 * (yy + zz); Rm[1] = 2.0 * (xy - wz);        Rm[2] = 2.0 * (xz + wy);
  Rm[3] = 2.0 * (xy + wz);        Rm[4] = 1.0 - 2.0 * (xx + zz); Rm[5] = 2.0 * (yz - wx);
  Rm[6] = 2.0 * (xz - wy);        Rm[7] = 2.0 * (yz + wx);        Rm[8] = 1.0 - 2.0 * (xx + yy);
}

// Camera-space centre; products of two FP32 numbers are exact in FP64, so the
// left-to-right summation fixes the result bit for bit.
__device__ __forceinline__ void cam_centre(const ViewD& v, const double* mu, double* x) {
  for (int i = 0; i < 3; ++i) {
    double a = __dmul_rn(v.R[3 * i + 0], mu[0]);
    a = __dadd_rn(a, __dmul_rn(v.R[3 * i + 1], mu[1]));
    a = __dadd_rn(a, __dmul_rn(v.R[3 * i + 2], mu[2]));
    x[i] = __dadd_rn(a, v.t[i]);
  }
}

// Forward geometry of one (view, Gaussian); false when culled by depth.
__device__ bool geometry(const ViewD& v, const Params& P, const rade_settings& st, Geo& G) {
  double x[3];
  cam_centre(v, P.mu, x);
  G.X = x[0]; G.Y = x[1]; G.Z = x[2];
  if (!(G.Z > st.near_plane)) return false;
  G.tc = sqrt(G.X * G.X + G.Y * G.Y + G.Z * G.Z);
  const double iz = 1.0 / G.Z;
  double xi = G.X * iz, eta = G.Y * iz;
  G.clx = xi < -v.limx || xi > v.limx;
  G.cly = eta < -v.limy || eta > v.limy;
  xi = fmin(v.limx, fmax(-v.limx, xi));
  eta = fmin(v.limy, fmax(-v.limy, eta));
  G.xi = xi; G.eta = eta;
  G.J0[0] = v.fx * iz; G.J0[1] = 0.0; G.J0[2] = -v.fx * xi * iz;
  G.J1[0] = 0.0; G.J1[1] = v.fy * iz; G.J1[2] = -v.fy * eta * iz;
  const double it = 1.0 / G.tc;
  G.J2[0] = G.X * it; G.J2[1] = G.Y * it; G.J2[2] = G.Z * it;
  // Wm = (R_world * R_g) diag(s)
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 3; ++k) {
      const double a = v.R[3 * i + 0] * P.Rg[0 + k] + v.R[3 * i + 1] * P.Rg[3 + k] +
                       v.R[3 * i + 2] * P.Rg[6 + k];
      G.Wm[3 * i + k] = a * P.s[k];
    }
  // T = J Wm
  const double* Jr[3] = {G.J0, G.J1, G.J2};
  for (int j = 0; j < 3; ++j)
    for (int k = 0; k < 3; ++k)
      G.T[3 * j + k] = Jr[j][0] * G.Wm[k] + Jr[j][1] * G.Wm[3 + k] + Jr[j][2] * G.Wm[6 + k];
  const double* T0 = G.T;
  const double* T1 = G.T + 3;
  const double* T2 = G.T + 6;
  G.B00 = T0[0] * T0[0] + T0[1] * T0[1] + T0[2] * T0[2];
  G.B01 = T0[0] * T1[0] + T0[1] * T1[1] + T0[2] * T1[2];
  G.B11 = T1[0] * T1[0] + T1[1] * T1[1] + T1[2] * T1[2];
  G.b0 = T0[0] * T2[0] + T0[1] * T2[1] + T0[2] * T2[2];
  G.b1 = T1[0] * T2[0] + T1[1] * T2[1] + T1[2] * T2[2];
  G.D00 = G.B00 + st.dilation;
  G.D11 = G.B11 + st.dilation;
  G.detD = G.D00 * G.D11 - G.B01 * G.B01;
  // plane slope q (Schur form of Eq. 13)
  const double det0 = G.B00 * G.B11 - G.B01 * G.B01;
  const double tr0 = G.B00 + G.B11;
  G.degenerate = !(det0 > st.degenerate * tr0 * tr0);
  if (G.degenerate) {
    G.q0 = 0.0; G.q1 = 0.0;
  } else {
    const double id = 1.0 / det0;
    G.q0 = -(G.B11 * G.b0 - G.B01 * G.b1) * id;
    G.q1 = -(G.B00 * G.b1 - G.B01 * G.b0) * id;
  }
  for (int k = 0; k < 3; ++k) G.nr[k] = -(G.q0 * G.J0[k] + G.q1 * G.J1[k] + G.J2[k]);
  G.nlen = sqrt(G.nr[0] * G.nr[0] + G.nr[1] * G.nr[1] + G.nr[2] * G.nr[2]);
  return true;
}

// The stored inputs of one Gaussian (loaded ahead of their use by the
// pipelined kernel).
struct RawGauss {
  float m0, m1, m2, s0, s1, s2, o;
  float4 q;
};

__device__ __forceinline__ RawGauss load_raw(int64_t g, const float* __restrict__ means,
                                             const float* __restrict__ scales,
                                             const float* __restrict__ quats,
                                             const float* __restrict__ opac) {
  RawGauss r;
  r.m0 = means[3 * g]; r.m1 = means[3 * g + 1]; r.m2 = means[3 * g + 2];
  r.s0 = scales[3 * g]; r.s1 = scales[3 * g + 1]; r.s2 = scales[3 * g + 2];
  r.q = *reinterpret_cast<const float4*>(quats + 4 * g);
  r.o = opac[g];
  return r;
}

// The parameters of a loaded Gaussian; false when it is culled (a parameter
// not finite, a zero quaternion, or opacity <= alpha_min, which leaves no
// pixel with alpha >= alpha_min).
__device__ __forceinline__ bool params_of(const RawGauss& r, double alpha_min, Params& P) {
  const float4 q = r.q;
  bool ok = finitef(r.m0) && finitef(r.m1) && finitef(r.m2) && finitef(r.s0) &&
            finitef(r.s1) && finitef(r.s2) && finitef(q.x) && finitef(q.y) && finitef(q.z) &&
            finitef(q.w) && finitef(r.o);
  P.mu[0] = r.m0; P.mu[1] = r.m1; P.mu[2] = r.m2;
  P.s[0] = r.s0; P.s[1] = r.s1; P.s[2] = r.s2;
  P.o = r.o;
  const double qw = q.x, qx = q.y, qy = q.z, qz = q.w;
  const double qq = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
  ok = ok && qq > 0.0 && ((double)r.o > alpha_min);
  P.qinv = ok ? 1.0 / qq : 0.0;
  P.qn[0] = qw * P.qinv; P.qn[1] = qx * P.qinv; P.qn[2] = qy * P.qinv; P.qn[3] = qz * P.qinv;
  quat_to_mat(P.qn, P.Rg);
  return ok;
}

// Loads Gaussian g (params_of's culling).
__device__ __forceinline__ bool load_params(int64_t g, const float* means, const float* scales,
                                            const float* quats, const float* opac,
                                            double alpha_min, Params& P) {
  return params_of(load_raw(g, means, scales, quats, opac), alpha_min, P);
}

__device__ __forceinline__ void store_invisible(rade_splat* out) {
  rade_splat s = {};
  s.rect[0] = 0; s.rect[1] = -1; s.rect[2] = 0; s.rect[3] = -1;
  *out = s;
}

// Exact-depth record of one (view, Gaussian) (Sec. 3.2.1, Eq. 5-7).  The
// camera-space inverse covariance is A = sum_k c_k c_k^T with c_k the k-th
// axis of the Gaussian in camera space divided by its scale (no matrix
// inverse, so flat Gaussians stay well conditioned).  With r_c = (x/z, y/z,
// 1) and D0 = r_c^T A r_c, the ray r = r_c - (dx/fx, dy/fy, 0) through the
// pixel at offset (dx, dy) = (u_c - u, v_c - v) meets the Gaussian's maximum
// at camera z = z (1 - g.d) / (1 - 2 g.d + d^T H d) with g = (A r_c)_{0,1}/D0
// and H = A_{0:2,0:2}/D0, d = (dx/fx, dy/fy); the record stores g and H
// with the focal lengths folded in.
__device__ __forceinline__ void exact_depth_record(const ViewD& v, const Params& P, const Geo& G,
                                                   float4* rec) {
  const double r0 = G.X / G.Z, r1 = G.Y / G.Z;
  double D0 = 0.0, g0 = 0.0, g1 = 0.0, h00 = 0.0, h01 = 0.0, h11 = 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    // camera-space axis k: (R_world R_g)[:, k]
    double c[3];
    for (int i = 0; i < 3; ++i)
      c[i] = v.R[3 * i + 0] * P.Rg[0 + k] + v.R[3 * i + 1] * P.Rg[3 + k] +
             v.R[3 * i + 2] * P.Rg[6 + k];
    const double is = 1.0 / fmax(fabs(P.s[k]), 1e-15);
    c[0] *= is; c[1] *= is; c[2] *= is;
    const double a = c[0] * r0 + c[1] * r1 + c[2];
    D0 += a * a;
    g0 += a * c[0]; g1 += a * c[1];
    h00 += c[0] * c[0]; h01 += c[0] * c[1]; h11 += c[1] * c[1];
  }
  const double i0 = 1.0 / D0;
  const double ifx = 1.0 / v.fx, ify = 1.0 / v.fy;
  rec[0] = make_float4((float)(g0 * i0 * ifx), (float)(g1 * i0 * ify),
                       (float)(h00 * i0 * ifx * ifx), (float)(2.0 * h01 * i0 * ifx * ify));
  rec[1] = make_float4((float)(h11 * i0 * ify * ify), 0.0f, 0.0f, 0.0f);
}

template <int KMAX, bool VEC, bool EXACT>
__global__ void __launch_bounds__(256, EXACT ? 1 : 2)
k_project(rade_settings st, const rade_view* __restrict__ views, int V, int64_t N,
          const float* __restrict__ means, const float* __restrict__ scales,
          const float* __restrict__ quats, const float* __restrict__ opac,
          const float* __restrict__ sh, rade_splat* __restrict__ splats,
          int32_t* __restrict__ tiles_touched, uint4* __restrict__ bin_records,
          float4* __restrict__ depth_quad) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= N) return;
  const int deg = st.sh_degree;
  constexpr int K = KMAX;
  const float* __restrict__ coef_g = sh + 3 * K * g;
  Params P;
  const bool ok = load_params(g, means, scales, quats, opac, st.alpha_min, P);
  // Affine depth: the coefficients are loaded with the parameters, so their
  // latency overlaps the FP64 geometry (the registers fit two waves per
  // SIMD).  Exact depth: they are loaded per view after the geometry, as its
  // extra registers leave no room to hold them across it.
  float coef[3 * K];
  bool rok = true;
  if constexpr (!EXACT) {
    load_row<K, VEC>(coef_g, coef);
    rok = row_finite<K>(coef);
  }
  for (int vi = 0; vi < V; ++vi) {
    const int64_t o = (int64_t)vi * N + g;
    const ViewD v = load_view(views[vi], st.fov_clamp);
    Geo G;
    bool vis = ok && rok && geometry(v, P, st, G) && G.detD > 0.0;
    if constexpr (EXACT) {
      if (vis) {
        load_row<K, VEC>(coef_g, coef);
        vis = row_finite<K>(coef);
      }
    }
    if (!vis) {
      store_invisible(splats + o);
      tiles_touched[o] = 0;
      if (bin_records) bin_records[o] = make_uint4(0u, 0u, 0u, 0u);
      if constexpr (EXACT) {
        depth_quad[2 * o] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        depth_quad[2 * o + 1] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      }
      continue;
    }
    if constexpr (EXACT) exact_depth_record(v, P, G, depth_quad + 2 * o);
    // The record is stored in its five 16-byte words as soon as each is
    // complete (fewer values live at once than with one store at the end).
    float4* rec = reinterpret_cast<float4*>(splats + o);
    const double uc = v.fx * G.X / G.Z + v.cx;
    const double vc = v.fy * G.Y / G.Z + v.cy;
    reinterpret_cast<double2*>(splats + o)[0] = make_double2(uc, vc);
    // support rect: alpha = o e^-power >= alpha_min inside power <= tau
    int x0 = 0, x1 = -1, y0 = 0, y1 = -1;
    {
      const double tau = fmin(st.power_cut, log((double)P.o / st.alpha_min));
      const double rx = sqrt(2.0 * tau * G.D00) * (1.0 + 1e-6) + 1e-3;
      const double ry = sqrt(2.0 * tau * G.D11) * (1.0 + 1e-6) + 1e-3;
      const double xlo = (uc - rx) - 0.5, xhi = (uc + rx) - 0.5;
      const double ylo = (vc - ry) - 0.5, yhi = (vc + ry) - 0.5;
      if (isfinite(xlo) && isfinite(xhi) && isfinite(ylo) && isfinite(yhi) && xhi >= 0.0 &&
          yhi >= 0.0 && xlo <= v.W - 1.0 && ylo <= v.H - 1.0) {
        x0 = max(0, (int)ceil(fmax(xlo, -1.0)));
        x1 = min(v.W - 1, (int)floor(fmin(xhi, (double)v.W)));
        y0 = max(0, (int)ceil(fmax(ylo, -1.0)));
        y1 = min(v.H - 1, (int)floor(fmin(yhi, (double)v.H)));
      }
    }
    // tile sizes are powers of two
    const int lw = __builtin_ctz((unsigned)st.tile_w), lh = __builtin_ctz((unsigned)st.tile_h);
    int32_t nt = 0;
    if (x0 <= x1 && y0 <= y1) {
      nt = ((x1 >> lw) - (x0 >> lw) + 1) * ((y1 >> lh) - (y0 >> lh) + 1);
    } else {
      x0 = 0; x1 = -1; y0 = 0; y1 = -1;
    }
    tiles_touched[o] = nt;
    const float z = (float)G.Z;
    if (bin_records)
      bin_records[o] = nt > 0 ? make_uint4(__float_as_uint(z),
                                           (uint32_t)(x0 >> lw) | ((uint32_t)(y0 >> lh) << 16),
                                           (uint32_t)(x1 >> lw) | ((uint32_t)(y1 >> lh) << 16),
                                           (uint32_t)nt)
                              : make_uint4(0u, 0u, 0u, 0u);
    // Eigen-factored quadratic form of the dilated footprint.
    {
      const double m = 0.5 * (G.D00 + G.D11);
      const double h = 0.5 * (G.D00 - G.D11);
      const double r = sqrt(h * h + G.B01 * G.B01);
      const double l1 = m + r;
      const double l2 = G.detD / l1;
      double ex, ey;
      if (r == 0.0) {
        ex = 1.0; ey = 0.0;
      } else if (h >= 0.0) {
        // (l1 - D11, B01) is well conditioned when D00 >= D11
        ex = l1 - G.D11; ey = G.B01;
      } else {
        ex = G.B01; ey = l1 - G.D00;
      }
      const double en = 1.0 / sqrt(ex * ex + ey * ey);
      ex *= en; ey *= en;
      const double k1 = sqrt(kLog2eD / (2.0 * l1));
      const double k2 = sqrt(kLog2eD / (2.0 * l2));
      rec[1] = make_float4((float)(ex * k1), (float)(ey * k1), (float)(-ey * k2),
                           (float)(ex * k2));
    }
    {
      const double zt = G.Z / G.tc;
      const double inl = 1.0 / G.nlen;
      rec[3] = make_float4(z, (float)(zt * G.q0), (float)(zt * G.q1), (float)(G.nr[0] * inl));
      // normal (y, z) and the rect x0, x1, y0, y1 as 16-bit integers
      const uint32_t rx01 = (uint32_t)(uint16_t)x0 | ((uint32_t)(uint16_t)x1 << 16);
      const uint32_t ry01 = (uint32_t)(uint16_t)y0 | ((uint32_t)(uint16_t)y1 << 16);
      rec[4] = make_float4((float)(G.nr[1] * inl), (float)(G.nr[2] * inl), __uint_as_float(rx01),
                           __uint_as_float(ry01));
    }
    {
      double u[3], raw[3];
      view_dir(P.mu, v.C, u);
      sh_colour<K>(deg, u, coef, raw);
      rec[2] = make_float4(P.o, (float)fmax(raw[0], 0.0), (float)fmax(raw[1], 0.0),
                           (float)fmax(raw[2], 0.0));
    }
  }
}

// Colour part of the projection backward for one view: the gradient of the
// view's SH row, row[3k + c] = g_c Y_k(u) (0 for a clamped channel, the
// forward's decision from the same FP64 colour), and the viewing
// direction's share of the mean gradient, added to gmu.  mu: the mean, C:
// the camera centre, (gr, gg, gb): the colour gradient of the record.
template <int K>
__device__ __forceinline__ void sh_view_bwd(int deg, const double* mu, const double* C,
                                            const float (&coef)[3 * K], float gr, float gg,
                                            float gbl, float (&row)[3 * K], double* gmu) {
  double u[3], raw[3];
  const double idn = view_dir(mu, C, u);
  sh_colour<K>(deg, u, coef, raw);
  {
    // the gradient arithmetic may use fused multiply-adds (the colour whose
    // clamp decisions must match the forward is computed without, above)
#pragma clang fp contract(fast)
    const double g0 = raw[0] < 0.0 ? 0.0 : (double)gr;
    const double g1 = raw[1] < 0.0 ? 0.0 : (double)gg;
    const double g2 = raw[2] < 0.0 ? 0.0 : (double)gbl;
    double Y[16], cw[16];
    sh_basis(deg, u[0], u[1], u[2], Y);
#pragma unroll
    for (int k = 0; k < 16; ++k) cw[k] = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const double c0 = coef[3 * k + 0], c1 = coef[3 * k + 1], c2 = coef[3 * k + 2];
      cw[k] = g0 * c0 + g1 * c1 + g2 * c2;
      row[3 * k + 0] = (float)(g0 * Y[k]);
      row[3 * k + 1] = (float)(g1 * Y[k]);
      row[3 * k + 2] = (float)(g2 * Y[k]);
    }
    double gu[3];
    sh_grad(deg, u[0], u[1], u[2], cw, gu);
    const double ud = u[0] * gu[0] + u[1] * gu[1] + u[2] * gu[2];
    for (int i = 0; i < 3; ++i) gmu[i] += (gu[i] - u[i] * ud) * idn;
  }
}

// Gradient record of one (view, Gaussian) from the render backward, with
// g_o = dL/d opacity per pixel (zero where alpha is clamped):
//   0, 1   sums of g_o dx, g_o dy (first moments of the pixel offset from
//          the centre): the centre gradient through the footprint is -o Q
//          times these, Q the conic
//   2-4    sums of g_o dx^2, g_o dx dy, g_o dy^2: the gradient of the conic
//          (power a dx^2 / 2 + b dx dy + c dy^2 / 2) is -o (s2 / 2, s3, s4 / 2)
//   5      do;  6-8 drgb;  9 dz;  10, 11 dp;  12-14 dn;  15 pad.
constexpr int kGradStride = 16;

// The projection backward comes in two forms.  One view: geometry and colour
// in one kernel (k_project_bwd_pipe), one lane holding both and the SH row
// (one wave per SIMD).  Many views: the geometry (k_project_bwd_geo, no SH
// row, two waves per SIMD) and then the colour (k_project_bwd_sh, which
// keeps its row's gradient in registers over the views).
//
// The first view's gradient record of Gaussian g.
struct Rec0 {
  float4 a, b, c, d;
};

__device__ __forceinline__ Rec0 load_rec0(const float* __restrict__ gsplat, int64_t g) {
  const float4* gr0 = reinterpret_cast<const float4*>(gsplat + g * kGradStride);
  return Rec0{gr0[0], gr0[1], gr0[2], gr0[3]};
}

// Projection backward of Gaussian g from its loaded parameters and first
// record.  (A Gaussian whose SH row is not finite is culled by the forward
// in every view: its records are zero, so every view is skipped and its
// gradients are zero.)
template <int KMAX, bool VEC, bool SH, bool PRE = false>
__device__ __forceinline__ void project_bwd_gauss(
    const rade_settings& st, const rade_view* __restrict__ views, int V, int64_t N, int64_t g,
    const RawGauss& raw, const Rec0& r0, const float* __restrict__ sh,
    const float (&pre_coef)[3 * KMAX],
    const float* __restrict__ gsplat, float* __restrict__ d_means, float* __restrict__ d_scales,
    float* __restrict__ d_quats, float* __restrict__ d_opac, float* __restrict__ d_sh) {
  constexpr int K = KMAX;
  const float* __restrict__ coef_g = SH ? sh + 3 * K * g : nullptr;
  const float4 g0a = r0.a, g0b = r0.b, g0c = r0.c, g0d = r0.d;
  Params P;
  bool ok = params_of(raw, st.alpha_min, P);
  bool sh_written = false;
  double gmu[3] = {0, 0, 0}, gs[3] = {0, 0, 0}, gqn[4] = {0, 0, 0, 0}, go = 0.0;
  for (int vi = 0; ok && vi < V; ++vi) {
    float4 ga = g0a, gb = g0b, gc = g0c, gd = g0d;
    if (vi > 0) {
      const float4* gr = reinterpret_cast<const float4*>(gsplat + ((int64_t)vi * N + g) * kGradStride);
      ga = gr[0]; gb = gr[1]; gc = gr[2]; gd = gr[3];
    }
    // the power gradient is -o g_o: the per-Gaussian factor of the
    // footprint terms
    const double mo = -(double)P.o;
    const double gA = ga.z * mo, gB = ga.w * mo;
    const double gC = gb.x * mo, gO = gb.y;
    const double gZd = gc.y, gp0 = gc.z, gp1 = gc.w;
    const double gn0 = gd.x, gn1 = gd.y, gn2 = gd.z;
    if (ga.x == 0.f && ga.y == 0.f && ga.z == 0.f && ga.w == 0.f && gb.x == 0.f &&
        gb.y == 0.f && gb.z == 0.f && gb.w == 0.f && gc.x == 0.f && gc.y == 0.f &&
        gc.z == 0.f && gc.w == 0.f && gd.x == 0.f && gd.y == 0.f && gd.z == 0.f)
      continue;
    const ViewD v = load_view(views[vi], st.fov_clamp);
    Geo G;
    if (!geometry(v, P, st, G) || !(G.detD > 0.0)) continue;
    go += gO;
    {
    // The backward's own arithmetic may use fused multiply-adds: its
    // results are compared within a tolerance, while the shared pieces
    // whose decisions must match the forward (the geometry, the colour sum
    // for the clamp) are compiled in their own functions without.
#pragma clang fp contract(fast)
    const double X = G.X, Yc = G.Y, Z = G.Z, tc = G.tc;
    const double iz = 1.0 / Z, iz2 = iz * iz;
    // the record's centre gradient leaves out the depth plane's share: the
    // plane depth z + p . (u_c - u) moves with the centre by p, so that share
    // is p times the summed depth gradient
    const double zt = Z / tc;
    // the centre's share through the footprint: the first moments of the
    // offset times the conic (the inverse of the dilated footprint D)
    const double idt = 1.0 / G.detD;
    const double qa = G.D11 * idt, qb = -G.B01 * idt, qc = G.D00 * idt;
    const double guc = mo * (qa * ga.x + qb * ga.y), gvc = mo * (qb * ga.x + qc * ga.y);
    const double gu = guc + zt * G.q0 * gZd, gv = gvc + zt * G.q1 * gZd;
    double gx[3];
    gx[0] = gu * v.fx * iz;
    gx[1] = gv * v.fy * iz;
    gx[2] = -(gu * v.fx * X + gv * v.fy * Yc) * iz2 + gZd;
    // p = (Z / tc) q
    double gq0 = zt * gp0, gq1 = zt * gp1;
    const double pq = gp0 * G.q0 + gp1 * G.q1;
    gx[2] += pq / tc;
    double gtc = -Z * pq / (tc * tc);
    // n = nr / |nr|, nr = -(q0 J0 + q1 J1 + J2)
    double gJ0[3], gJ1[3], gJ2[3];
    {
      const double il = 1.0 / G.nlen;
      const double n[3] = {G.nr[0] * il, G.nr[1] * il, G.nr[2] * il};
      const double nd = n[0] * gn0 + n[1] * gn1 + n[2] * gn2;
      const double gr[3] = {(gn0 - n[0] * nd) * il, (gn1 - n[1] * nd) * il,
                            (gn2 - n[2] * nd) * il};
      gq0 -= G.J0[0] * gr[0] + G.J0[1] * gr[1] + G.J0[2] * gr[2];
      gq1 -= G.J1[0] * gr[0] + G.J1[1] * gr[1] + G.J1[2] * gr[2];
      for (int k = 0; k < 3; ++k) {
        gJ0[k] = -G.q0 * gr[k];
        gJ1[k] = -G.q1 * gr[k];
        gJ2[k] = -gr[k];
      }
    }
    // Gradients of the symmetric Sigma' entries: g00, g11, g01 (the sum over
    // both off-diagonal positions), gb0, gb1.
    double g00 = 0.0, g11 = 0.0, g01 = 0.0, gb0 = 0.0, gb1 = 0.0;
    if (!G.degenerate) {
      const double det0 = G.B00 * G.B11 - G.B01 * G.B01;
      const double id = 1.0 / det0;
      // h = B0^-1 gq
      const double h0 = (G.B11 * gq0 - G.B01 * gq1) * id;
      const double h1 = (G.B00 * gq1 - G.B01 * gq0) * id;
      g00 += -h0 * G.q0;
      g11 += -h1 * G.q1;
      g01 += -(h0 * G.q1 + h1 * G.q0);
      gb0 = -h0;
      gb1 = -h1;
    }
    // conic = D^-1 with D the dilated footprint: gD = -C Gc C.
    {
      const double idt = 1.0 / G.detD;
      const double ca = G.D11 * idt, cb = -G.B01 * idt, cc = G.D00 * idt;
      const double G00 = 0.5 * gA, G01 = 0.5 * gB, G11 = 0.5 * gC;
      const double m00 = ca * G00 + cb * G01, m01 = ca * G01 + cb * G11;
      const double m10 = cb * G00 + cc * G01, m11 = cb * G01 + cc * G11;
      g00 += -(m00 * ca + m01 * cb);
      g11 += -(m10 * cb + m11 * cc);
      g01 += -((m00 * cb + m01 * cc) + (m10 * ca + m11 * cb));
    }
    // Sigma' entries as dot products of rows of T.
    double gT[9];
    for (int k = 0; k < 3; ++k) {
      const double t0 = G.T[k], t1 = G.T[3 + k], t2 = G.T[6 + k];
      gT[k] = 2.0 * g00 * t0 + g01 * t1 + gb0 * t2;
      gT[3 + k] = 2.0 * g11 * t1 + g01 * t0 + gb1 * t2;
      gT[6 + k] = gb0 * t0 + gb1 * t1;
    }
    // T = J Wm: gJ_j += gT_j Wm^T, gWm = J^T gT
    double* gJr[3] = {gJ0, gJ1, gJ2};
    const double* Jr[3] = {G.J0, G.J1, G.J2};
    double gW[9];
    for (int i = 0; i < 3; ++i)
      for (int k = 0; k < 3; ++k) gW[3 * i + k] = 0.0;
    for (int j = 0; j < 3; ++j)
      for (int i = 0; i < 3; ++i) {
        double acc = 0.0;
        for (int k = 0; k < 3; ++k) {
          acc += gT[3 * j + k] * G.Wm[3 * i + k];
          gW[3 * i + k] += Jr[j][i] * gT[3 * j + k];
        }
        gJr[j][i] += acc;
      }
    // Wm = (R Rg) diag(s): gs_k, g(R Rg)
    double gV[9];
    for (int i = 0; i < 9; ++i) gV[i] = gW[i] * P.s[i % 3];
    for (int k = 0; k < 3; ++k) {
      double acc = 0.0;
      for (int i = 0; i < 3; ++i) {
        const double vik = v.R[3 * i] * P.Rg[k] + v.R[3 * i + 1] * P.Rg[3 + k] +
                           v.R[3 * i + 2] * P.Rg[6 + k];
        acc += gW[3 * i + k] * vik;
      }
      gs[k] += acc;
    }
    // gRg = R^T gV
    double gRg[9];
    for (int a = 0; a < 3; ++a)
      for (int k = 0; k < 3; ++k)
        gRg[3 * a + k] = v.R[a] * gV[k] + v.R[3 + a] * gV[3 + k] + v.R[6 + a] * gV[6 + k];
    // rotation matrix -> unit quaternion
    {
      const double w = P.qn[0], x = P.qn[1], y = P.qn[2], z = P.qn[3];
      const double* r = gRg;
      gqn[0] += 2.0 * (-z * r[1] + y * r[2] + z * r[3] - x * r[5] - y * r[6] + x * r[7]);
      gqn[1] += 2.0 * (y * r[1] + z * r[2] + y * r[3] - 2.0 * x * r[4] - w * r[5] + z * r[6] +
                       w * r[7] - 2.0 * x * r[8]);
      gqn[2] += 2.0 * (-2.0 * y * r[0] + x * r[1] + w * r[2] + x * r[3] + z * r[5] - w * r[6] +
                       z * r[7] - 2.0 * y * r[8]);
      gqn[3] += 2.0 * (-2.0 * z * r[0] - w * r[1] + x * r[2] + w * r[3] - 2.0 * z * r[4] +
                       y * r[5] + x * r[6] + y * r[7]);
    }
    // J(x): rows 0,1 (with the x/z, y/z clamps), row 2 = x / tc
    gx[2] += -(gJ0[0] * v.fx + gJ1[1] * v.fy) * iz2;
    if (G.clx) {
      gx[2] += gJ0[2] * v.fx * G.xi * iz2;
    } else {
      gx[0] += -gJ0[2] * v.fx * iz2;
      gx[2] += gJ0[2] * 2.0 * v.fx * X * iz2 * iz;
    }
    if (G.cly) {
      gx[2] += gJ1[2] * v.fy * G.eta * iz2;
    } else {
      gx[1] += -gJ1[2] * v.fy * iz2;
      gx[2] += gJ1[2] * 2.0 * v.fy * Yc * iz2 * iz;
    }
    {
      const double it = 1.0 / tc;
      const double xs[3] = {X * it, Yc * it, Z * it};
      const double dd = gJ2[0] * xs[0] + gJ2[1] * xs[1] + gJ2[2] * xs[2];
      for (int j = 0; j < 3; ++j) gx[j] += (gJ2[j] - xs[j] * dd) * it + gtc * xs[j];
    }
    // x = R mu + t
    for (int i = 0; i < 3; ++i)
      gmu[i] += v.R[i] * gx[0] + v.R[3 + i] * gx[1] + v.R[6 + i] * gx[2];
    if constexpr (SH) {
      float coef[3 * K], row[3 * K];
      if constexpr (PRE) {
#pragma unroll
        for (int i = 0; i < 3 * K; ++i) coef[i] = pre_coef[i];
      } else {
        load_row<K, VEC>(coef_g, coef);
      }
      sh_view_bwd<K>(st.sh_degree, P.mu, v.C, coef, gb.z, gb.w, gc.x, row, gmu);
      store_row<K, VEC>(d_sh + 3 * K * g, row, sh_written);
      sh_written = true;
    }

    }
  }
  // unit quaternion -> raw quaternion
  const double qd = P.qn[0] * gqn[0] + P.qn[1] * gqn[1] + P.qn[2] * gqn[2] + P.qn[3] * gqn[3];
  float4 dq;
  dq.x = (float)((gqn[0] - P.qn[0] * qd) * P.qinv);
  dq.y = (float)((gqn[1] - P.qn[1] * qd) * P.qinv);
  dq.z = (float)((gqn[2] - P.qn[2] * qd) * P.qinv);
  dq.w = (float)((gqn[3] - P.qn[3] * qd) * P.qinv);
  if (!ok) dq = make_float4(0.f, 0.f, 0.f, 0.f);
  *reinterpret_cast<float4*>(d_quats + 4 * g) = dq;
  for (int i = 0; i < 3; ++i) {
    d_means[3 * g + i] = ok ? (float)gmu[i] : 0.0f;
    d_scales[3 * g + i] = ok ? (float)gs[i] : 0.0f;
  }
  d_opac[g] = ok ? (float)go : 0.0f;
  if (SH && !sh_written) {
    float zero[3 * K];
#pragma unroll
    for (int i = 0; i < 3 * K; ++i) zero[i] = 0.0f;
    store_row<K, VEC>(d_sh + 3 * K * g, zero, false);
  }
}

// One lane per Gaussian; the first view's gradient record is loaded together
// with the parameters, so its latency is not paid after theirs.
template <int KMAX, bool VEC, bool SH>
__device__ __forceinline__ void project_bwd_body(
    const rade_settings& st, const rade_view* __restrict__ views, int V, int64_t N,
    const float* __restrict__ means, const float* __restrict__ scales,
    const float* __restrict__ quats, const float* __restrict__ opac,
    const float* __restrict__ sh, const float* __restrict__ gsplat,
    float* __restrict__ d_means, float* __restrict__ d_scales, float* __restrict__ d_quats,
    float* __restrict__ d_opac, float* __restrict__ d_sh) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= N) return;
  const Rec0 r0 = load_rec0(gsplat, g);
  const RawGauss raw = load_raw(g, means, scales, quats, opac);
  float unused[3 * KMAX];
  project_bwd_gauss<KMAX, VEC, SH>(st, views, V, N, g, raw, r0, sh, unused, gsplat, d_means,
                                   d_scales, d_quats, d_opac, d_sh);
}

// One view, software-pipelined over a grid that fits the device at once
// (its registers allow one wave per SIMD, so no other wave hides the load
// latency): lane l takes the Gaussians l, l + S, l + 2 S, ... (S lanes in
// the grid) and issues the loads of its next Gaussian's parameters and
// record before the arithmetic of the current one.
template <int KMAX, bool VEC>
__global__ void __launch_bounds__(256)
k_project_bwd_pipe(rade_settings st, const rade_view* __restrict__ views, int64_t N,
                   const float* __restrict__ means, const float* __restrict__ scales,
                   const float* __restrict__ quats, const float* __restrict__ opac,
                   const float* __restrict__ sh, const float* __restrict__ gsplat,
                   float* __restrict__ d_means, float* __restrict__ d_scales,
                   float* __restrict__ d_quats, float* __restrict__ d_opac,
                   float* __restrict__ d_sh) {
  const int64_t S = (int64_t)gridDim.x * blockDim.x;
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= N) return;
  constexpr int K = KMAX;
  Rec0 ra = load_rec0(gsplat, g), rb = ra;
  RawGauss pa = load_raw(g, means, scales, quats, opac), pb = pa;
  float ca[3 * K], cb[3 * K];
  load_row<K, VEC>(sh + 3 * K * g, ca);
  for (;;) {
    // two Gaussians per trip, so the prefetch buffers alternate without copies
    int64_t gn = g + S;
    if (gn < N) {
      rb = load_rec0(gsplat, gn);
      pb = load_raw(gn, means, scales, quats, opac);
      load_row<K, VEC>(sh + 3 * K * gn, cb);
    }
    project_bwd_gauss<KMAX, VEC, true, true>(st, views, 1, N, g, pa, ra, sh, ca, gsplat, d_means,
                                       d_scales, d_quats, d_opac, d_sh);
    if (gn >= N) break;
    g = gn;
    gn = g + S;
    if (gn < N) {
      ra = load_rec0(gsplat, gn);
      pa = load_raw(gn, means, scales, quats, opac);
      load_row<K, VEC>(sh + 3 * K * gn, ca);
    }
    project_bwd_gauss<KMAX, VEC, true, true>(st, views, 1, N, g, pb, rb, sh, cb, gsplat, d_means,
                                       d_scales, d_quats, d_opac, d_sh);
    if (gn >= N) break;
    g = gn;
  }
}

// The geometry alone at two waves per SIMD: its registers are held to 256
// (a few values spill to scratch memory; measured faster on 16 views than
// one wave per SIMD without spills).
template <int KMAX, bool VEC>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
k_project_bwd_geo(rade_settings st, const rade_view* __restrict__ views, int V, int64_t N,
                  const float* __restrict__ means, const float* __restrict__ scales,
                  const float* __restrict__ quats, const float* __restrict__ opac,
                  const float* __restrict__ gsplat, float* __restrict__ d_means,
                  float* __restrict__ d_scales, float* __restrict__ d_quats,
                  float* __restrict__ d_opac) {
  project_bwd_body<KMAX, VEC, false>(st, views, V, N, means, scales, quats, opac, nullptr,
                                     gsplat, d_means, d_scales, d_quats, d_opac, nullptr);
}

// The colour part of the projection backward, after k_project_bwd_geo: the SH
// coefficient gradients (one row per Gaussian, summed over the views in
// registers and stored once) and the viewing direction's share of the mean
// gradient, added to what k_project_bwd_geo wrote.  A view contributes when its
// colour gradient is not zero; such a record comes from blended pixels, so
// the splat exists in that view and the geometry the fused form would check
// succeeds.  The clamp decisions are the forward's (same FP64 colour).
template <int KMAX, bool VEC>
__global__ void __launch_bounds__(256)
k_project_bwd_sh(rade_settings st, const rade_view* __restrict__ views, int V, int64_t N,
                 const float* __restrict__ means, const float* __restrict__ scales,
                 const float* __restrict__ quats, const float* __restrict__ opac,
                 const float* __restrict__ sh, const float* __restrict__ gsplat,
                 float* __restrict__ d_means, float* __restrict__ d_sh) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= N) return;
  const int deg = st.sh_degree;
  constexpr int K = KMAX;
  Params P;
  bool ok = load_params(g, means, scales, quats, opac, st.alpha_min, P);
  float coef[3 * K], acc[3 * K];
  load_row<K, VEC>(sh + 3 * K * g, coef);
  ok = ok && row_finite<K>(coef);
#pragma unroll
  for (int i = 0; i < 3 * K; ++i) acc[i] = 0.0f;
  double gmu[3] = {0, 0, 0};
  for (int vi = 0; ok && vi < V; ++vi) {
    const float4* gr = reinterpret_cast<const float4*>(gsplat + ((int64_t)vi * N + g) * kGradStride);
    const float4 gb = gr[1], gc = gr[2];
    if (gb.z == 0.f && gb.w == 0.f && gc.x == 0.f) continue;
    double C[3];
    {
      const rade_view& rv = views[vi];
      for (int i = 0; i < 3; ++i)
        C[i] = -((double)rv.R[i] * (double)rv.t[0] + (double)rv.R[3 + i] * (double)rv.t[1] +
                 (double)rv.R[6 + i] * (double)rv.t[2]);
    }
    float row[3 * K];
    sh_view_bwd<K>(deg, P.mu, C, coef, gb.z, gb.w, gc.x, row, gmu);
#pragma unroll
    for (int i = 0; i < 3 * K; ++i) acc[i] += row[i];
  }
  store_row<K, VEC>(d_sh + 3 * K * g, acc, false);
  if (ok)
    for (int i = 0; i < 3; ++i) d_means[3 * g + i] += (float)gmu[i];
}

}  // namespace

hipError_t launch_project(const rade_settings& st, const rade_view* views, int V, int64_t N,
                          const float* means, const float* scales, const float* quats,
                          const float* opac, const float* sh, rade_splat* splats,
                          int32_t* tiles_touched, uint32_t* bin_records, float* depth_quad,
                          hipStream_t stream) {
  if (N == 0) return hipSuccess;
  uint4* br = reinterpret_cast<uint4*>(bin_records);
  const dim3 block(256);
  const dim3 grid((unsigned)((N + 255) / 256));
  EventScope timing(RADE_KERNEL_PROJECT, stream);
  const bool vec = (reinterpret_cast<uintptr_t>(sh) & 15) == 0;
  float4* dq = reinterpret_cast<float4*>(depth_quad);
#define RADE_PROJECT_E(K, V4, E)                                                             \
  hipLaunchKernelGGL((k_project<K, V4, E>), grid, block, 0, stream, st, views, V, N, means,  \
                     scales, quats, opac, sh, splats, tiles_touched, br, dq)
#define RADE_PROJECT(K, V4)                                                                 \
  do {                                                                                      \
    if (dq) RADE_PROJECT_E(K, V4, true); else RADE_PROJECT_E(K, V4, false);                 \
  } while (0)
  switch (st.sh_degree) {
    case 0: RADE_PROJECT(1, false); break;
    case 1: if (vec) RADE_PROJECT(4, true); else RADE_PROJECT(4, false); break;
    case 2: RADE_PROJECT(9, false); break;
    default: if (vec) RADE_PROJECT(16, true); else RADE_PROJECT(16, false); break;
  }
#undef RADE_PROJECT
#undef RADE_PROJECT_E
  return hipGetLastError();
}

hipError_t launch_project_bwd(const rade_settings& st, const rade_view* views, int V, int64_t N,
                              const float* means, const float* scales, const float* quats,
                              const float* opac, const float* sh, const float* gsplat,
                              float* d_means, float* d_scales, float* d_quats, float* d_opac,
                              float* d_sh, hipStream_t stream) {
  if (N == 0) return hipSuccess;
  const dim3 block(256);
  const dim3 grid((unsigned)((N + 255) / 256));
  EventScope timing(RADE_KERNEL_PROJECT_BWD, stream);
  const bool vec = ((reinterpret_cast<uintptr_t>(sh) | reinterpret_cast<uintptr_t>(d_sh)) & 15) == 0;
#define RADE_PROJECT_BWD(K, V4)                                                               \
  do {                                                                                        \
    if (V == 1) {                                                                             \
      static unsigned cached = 0;                                                             \
      const unsigned gp = resident_blocks(k_project_bwd_pipe<K, V4>, 256, grid.x, cached);    \
      hipLaunchKernelGGL((k_project_bwd_pipe<K, V4>), dim3(gp), block, 0, stream, st, views,  \
                         N, means, scales, quats, opac, sh, gsplat, d_means, d_scales,         \
                         d_quats, d_opac, d_sh);                                               \
    } else {                                                                                  \
      hipLaunchKernelGGL((k_project_bwd_geo<K, V4>), grid, block, 0, stream, st, views, V, N,  \
                         means, scales, quats, opac, gsplat, d_means, d_scales, d_quats,       \
                         d_opac);                                                              \
      hipLaunchKernelGGL((k_project_bwd_sh<K, V4>), grid, block, 0, stream, st, views, V, N,  \
                         means, scales, quats, opac, sh, gsplat, d_means, d_sh);             \
    }                                                                                         \
  } while (0)
  switch (st.sh_degree) {
    case 0: RADE_PROJECT_BWD(1, false); break;
    case 1: if (vec) RADE_PROJECT_BWD(4, true); else RADE_PROJECT_BWD(4, false); break;
    case 2: RADE_PROJECT_BWD(9, false); break;
    default: if (vec) RADE_PROJECT_BWD(16, true); else RADE_PROJECT_BWD(16, false); break;
  }
#undef RADE_PROJECT_BWD
  return hipGetLastError();
}

}  // namespace rade
