// FP64 CPU oracle of the RaDe-GS rasterizer (arXiv 2406.01467).
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call this file;
// only the tests, the smoke check and the CPU-baseline leg of the benchmark do.
// It shares no code with the HIP library.
//
// What it computes, step by step, in FP64 on the FP32 inputs:
//   * projection of each 3D Gaussian (Sec. 3.1, Eq. 1-2): covariance from
//     scale and rotation, the local affine (EWA) Jacobian with the ray-space
//     third row (Sec. 3.2.2), the ray-space covariance Sigma';
//   * the depth plane (Sec. 3.2.2, Eq. 13-17): q-hat = third row of Sigma'^-1
//     divided by its (3,3) entry, p = (z_c / t_c) q, per-pixel depth
//     d = z_c + p (u_c - u, v_c - v) (Eq. 4);
//   * the splat normal (Sec. 3.3, Eq. 21-22): n' = -(q, 1), n = J^T n'
//     normalised;
//   * view-dependent colour from real spherical harmonics (Sec. 3.1, Eq. 3);
//   * brute-force front-to-back alpha blending (Eq. 3) of colour, depth,
//     normal and alpha for every requested pixel over ALL Gaussians in
//     ascending (float32(z_c), id) order -- no tiles -- plus the median depth
//     (Sec. 1: depth at which accumulated opacity crosses one half);
//   * the depth-distortion term of Sec. 3.4 (Eq. 23) per pixel,
//     sum_{i,j} w_i w_j (d_i - d_j)^2 over the blended splats, as the plain
//     double sum (the training loss detaches the weights: its adjoint flows
//     through the per-pixel depths d_i only);
//   * the hand-written adjoint of all of the above (FP64);
//   * a binning reference (std::stable_sort of (tile, depth) keys).
//
// Readings where the paper is silent are fixed by the settings vector (see
// oracle/__init__.py) and listed with the design notes of the project.
//
// Build: g++ -O2 -fopenmp -ffp-contract=off -fPIC -shared (oracle/__init__.py builds it).

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <numeric>
#include <vector>

namespace {

// ----------------------------------------------------------------------------
// Settings vector layout (doubles).
enum {
  S_DILATION = 0,   // low-pass added to the 2x2 footprint covariance (px^2)
  S_NEAR = 1,       // near plane (camera z)
  S_ALPHA_MIN = 2,  // blends with alpha below this are skipped
  S_ALPHA_MAX = 3,  // alpha clamp
  S_T_MIN = 4,      // stop when transmittance would fall below this
  S_POWER_CUT = 5,  // skip when 1/2 d^T conic d exceeds this (3 sigma: 4.5)
  S_FOV_CLAMP = 6,  // clamp of x/z, y/z in the Jacobian, times tan(half fov)
  S_DEGEN = 7,      // q := 0 when det(B0) <= S_DEGEN * tr(B0)^2
  S_BG0 = 8, S_BG1 = 9, S_BG2 = 10,
  S_SH_DEGREE = 11,
  S_TILE_W = 12, S_TILE_H = 13,
  S_FRAG_POWER = 14,   // |power - cut| below this flags the pixel
  S_FRAG_ALPHA = 15,   // relative margin around alpha_min
  S_FRAG_T = 16,       // relative margin around t_min
  S_FRAG_MED = 17,     // relative margin around T = 1/2
  S_FRAG_CLAMP = 18,   // relative margin around alpha_max (gradient fragility)
  S_DEPTH_EXACT = 19,  // 1: per-pixel depth of the exact ray maximum (Eq. 7), else Eq. 4
  S_COUNT = 20
};

// View vector layout (doubles): W, H, fx, fy, cx, cy, R[9] (row-major,
// world->camera), t[3].
enum { V_W = 0, V_H = 1, V_FX = 2, V_FY = 3, V_CX = 4, V_CY = 5, V_R = 6, V_T = 15, V_COUNT = 18 };

// Projected record layout (doubles), one per (view, Gaussian).
enum {
  R_UC = 0, R_VC, R_Z, R_TC, R_A, R_B, R_C, R_O, R_R, R_G, R_BL, R_P0, R_P1,
  R_Q0, R_Q1, R_N0, R_N1, R_N2, R_TAU, R_B00, R_B01, R_B11, R_X, R_Y,
  R_AI00, R_AI01, R_AI02, R_AI11, R_AI12, R_AI22,  // camera-space Sigma^-1 (Eq. 7)
  R_COUNT = 30
};

// Per-(view, Gaussian) gradient layout of the projected quantities.
enum {
  G_UC = 0, G_VC, G_A, G_B, G_C, G_O, G_R, G_G, G_BL, G_Z, G_P0, G_P1,
  G_N0, G_N1, G_N2, G_COUNT = 15
};

// Flags per (view, Gaussian).
enum {
  F_CULLED = 1, F_VISIBLE = 2, F_DEGENERATE = 4, F_CLAMP_X = 8, F_CLAMP_Y = 16,
  F_RGB_CLAMP0 = 32, F_RGB_CLAMP1 = 64, F_RGB_CLAMP2 = 128
};

// Per-pixel outputs (doubles).
enum {
  O_R = 0, O_G, O_B, O_DEXP, O_DMED, O_N0, O_N1, O_N2, O_ALPHA, O_TFIN, O_DIST, O_DIST_MAG,
  O_COUNT = 12
};
// Upstream gradients per pixel (doubles): colour 3, expected depth, median
// depth, normal 3, alpha, depth distortion.
constexpr int GOUT = 10;

struct M3 {
  double m[9];
  double& operator()(int i, int j) { return m[3 * i + j]; }
  double operator()(int i, int j) const { return m[3 * i + j]; }
};

M3 zero3() { M3 a; std::memset(a.m, 0, sizeof a.m); return a; }

M3 mul(const M3& a, const M3& b) {
  M3 c = zero3();
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k) c(i, j) += a(i, k) * b(k, j);
  return c;
}

M3 transpose(const M3& a) {
  M3 c;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) c(i, j) = a(j, i);
  return c;
}

M3 add(const M3& a, const M3& b) { M3 c; for (int i = 0; i < 9; ++i) c.m[i] = a.m[i] + b.m[i]; return c; }

// Inverse of a 3x3 matrix through its adjugate.
M3 inverse3(const M3& a) {
  M3 adj;
  adj(0, 0) = a(1, 1) * a(2, 2) - a(1, 2) * a(2, 1);
  adj(0, 1) = a(0, 2) * a(2, 1) - a(0, 1) * a(2, 2);
  adj(0, 2) = a(0, 1) * a(1, 2) - a(0, 2) * a(1, 1);
  adj(1, 0) = a(1, 2) * a(2, 0) - a(1, 0) * a(2, 2);
  adj(1, 1) = a(0, 0) * a(2, 2) - a(0, 2) * a(2, 0);
  adj(1, 2) = a(0, 2) * a(1, 0) - a(0, 0) * a(1, 2);
  adj(2, 0) = a(1, 0) * a(2, 1) - a(1, 1) * a(2, 0);
  adj(2, 1) = a(0, 1) * a(2, 0) - a(0, 0) * a(2, 1);
  adj(2, 2) = a(0, 0) * a(1, 1) - a(0, 1) * a(1, 0);
  double det = a(0, 0) * adj(0, 0) + a(0, 1) * adj(1, 0) + a(0, 2) * adj(2, 0);
  for (int i = 0; i < 9; ++i) adj.m[i] /= det;
  return adj;
}

// ----------------------------------------------------------------------------
// Real spherical harmonics, degree <= 3, in the order m = -l..l per degree
// (16 functions), with the Condon-Shortley phase folded in the way that makes
// Y_{1,-1} = -c1 y, Y_{1,0} = c1 z, Y_{1,1} = -c1 x.  Each function is the
// textbook normalised polynomial in the unit direction (x, y, z); the
// constants are written from their closed forms.
struct SH {
  double y[16];
  double dy[16][3];  // gradient with respect to (x, y, z), unconstrained
};

void eval_sh(int degree, const double d[3], SH& s) {
  const double x = d[0], y = d[1], z = d[2];
  const double pi = 3.14159265358979323846;
  const double c0 = 0.5 * std::sqrt(1.0 / pi);
  const double c1 = std::sqrt(3.0 / (4.0 * pi));
  const double c2a = 0.5 * std::sqrt(15.0 / pi);     // xy, yz, xz
  const double c2b = 0.25 * std::sqrt(5.0 / pi);     // 2z^2 - x^2 - y^2
  const double c2c = 0.25 * std::sqrt(15.0 / pi);    // x^2 - y^2
  const double c3a = 0.25 * std::sqrt(35.0 / (2.0 * pi));   // y(3x^2-y^2), x(x^2-3y^2)
  const double c3b = 0.5 * std::sqrt(105.0 / pi);            // xyz
  const double c3c = 0.25 * std::sqrt(21.0 / (2.0 * pi));   // y(4z^2-x^2-y^2), x(...)
  const double c3d = 0.25 * std::sqrt(7.0 / pi);             // z(2z^2-3x^2-3y^2)
  const double c3e = 0.25 * std::sqrt(105.0 / pi);           // z(x^2-y^2)
  for (int i = 0; i < 16; ++i) { s.y[i] = 0; s.dy[i][0] = s.dy[i][1] = s.dy[i][2] = 0; }
  s.y[0] = c0;
  if (degree < 1) return;
  s.y[1] = -c1 * y; s.dy[1][1] = -c1;
  s.y[2] = c1 * z;  s.dy[2][2] = c1;
  s.y[3] = -c1 * x; s.dy[3][0] = -c1;
  if (degree < 2) return;
  s.y[4] = c2a * x * y;          s.dy[4][0] = c2a * y; s.dy[4][1] = c2a * x;
  s.y[5] = -c2a * y * z;         s.dy[5][1] = -c2a * z; s.dy[5][2] = -c2a * y;
  s.y[6] = c2b * (2 * z * z - x * x - y * y);
  s.dy[6][0] = -2 * c2b * x; s.dy[6][1] = -2 * c2b * y; s.dy[6][2] = 4 * c2b * z;
  s.y[7] = -c2a * x * z;         s.dy[7][0] = -c2a * z; s.dy[7][2] = -c2a * x;
  s.y[8] = c2c * (x * x - y * y); s.dy[8][0] = 2 * c2c * x; s.dy[8][1] = -2 * c2c * y;
  if (degree < 3) return;
  s.y[9] = -c3a * y * (3 * x * x - y * y);
  s.dy[9][0] = -c3a * 6 * x * y; s.dy[9][1] = -c3a * (3 * x * x - 3 * y * y);
  s.y[10] = c3b * x * y * z;
  s.dy[10][0] = c3b * y * z; s.dy[10][1] = c3b * x * z; s.dy[10][2] = c3b * x * y;
  s.y[11] = -c3c * y * (4 * z * z - x * x - y * y);
  s.dy[11][0] = -c3c * (-2 * x * y); s.dy[11][1] = -c3c * (4 * z * z - x * x - 3 * y * y);
  s.dy[11][2] = -c3c * 8 * y * z;
  s.y[12] = c3d * z * (2 * z * z - 3 * x * x - 3 * y * y);
  s.dy[12][0] = c3d * (-6 * x * z); s.dy[12][1] = c3d * (-6 * y * z);
  s.dy[12][2] = c3d * (6 * z * z - 3 * x * x - 3 * y * y);
  s.y[13] = -c3c * x * (4 * z * z - x * x - y * y);
  s.dy[13][0] = -c3c * (4 * z * z - 3 * x * x - y * y); s.dy[13][1] = -c3c * (-2 * x * y);
  s.dy[13][2] = -c3c * 8 * x * z;
  s.y[14] = c3e * z * (x * x - y * y);
  s.dy[14][0] = c3e * 2 * x * z; s.dy[14][1] = -c3e * 2 * y * z; s.dy[14][2] = c3e * (x * x - y * y);
  s.y[15] = -c3a * x * (x * x - 3 * y * y);
  s.dy[15][0] = -c3a * (3 * x * x - 3 * y * y); s.dy[15][1] = -c3a * (-6 * x * y);
}

// Rotation matrix of a unit quaternion (w, x, y, z).
M3 quat_rot(const double q[4]) {
  const double w = q[0], x = q[1], y = q[2], z = q[3];
  M3 r;
  r(0, 0) = 1 - 2 * (y * y + z * z); r(0, 1) = 2 * (x * y - w * z); r(0, 2) = 2 * (x * z + w * y);
  r(1, 0) = 2 * (x * y + w * z); r(1, 1) = 1 - 2 * (x * x + z * z); r(1, 2) = 2 * (y * z - w * x);
  r(2, 0) = 2 * (x * z - w * y); r(2, 1) = 2 * (y * z + w * x); r(2, 2) = 1 - 2 * (x * x + y * y);
  return r;
}

// d R(q) / d q_k for a unit quaternion, as 4 matrices.
void quat_rot_grad(const double q[4], M3 d[4]) {
  const double w = q[0], x = q[1], y = q[2], z = q[3];
  // d/dw
  d[0] = zero3(); d[0](0, 1) = -2 * z; d[0](0, 2) = 2 * y; d[0](1, 0) = 2 * z;
  d[0](1, 2) = -2 * x; d[0](2, 0) = -2 * y; d[0](2, 1) = 2 * x;
  // d/dx
  d[1] = zero3(); d[1](0, 1) = 2 * y; d[1](0, 2) = 2 * z; d[1](1, 0) = 2 * y;
  d[1](1, 1) = -4 * x; d[1](1, 2) = -2 * w; d[1](2, 0) = 2 * z; d[1](2, 1) = 2 * w;
  d[1](2, 2) = -4 * x;
  // d/dy
  d[2] = zero3(); d[2](0, 0) = -4 * y; d[2](0, 1) = 2 * x; d[2](0, 2) = 2 * w;
  d[2](1, 0) = 2 * x; d[2](1, 2) = 2 * z; d[2](2, 0) = -2 * w; d[2](2, 1) = 2 * z;
  d[2](2, 2) = -4 * y;
  // d/dz
  d[3] = zero3(); d[3](0, 0) = -4 * z; d[3](0, 1) = -2 * w; d[3](0, 2) = 2 * x;
  d[3](1, 0) = 2 * w; d[3](1, 1) = -4 * z; d[3](1, 2) = 2 * y; d[3](2, 0) = 2 * x;
  d[3](2, 1) = 2 * y;
}

struct View {
  int W, H;
  double fx, fy, cx, cy;
  M3 R;
  double t[3];
};

View load_view(const double* v) {
  View o;
  o.W = (int)v[V_W]; o.H = (int)v[V_H];
  o.fx = v[V_FX]; o.fy = v[V_FY]; o.cx = v[V_CX]; o.cy = v[V_CY];
  for (int i = 0; i < 9; ++i) o.R.m[i] = v[V_R + i];
  for (int i = 0; i < 3; ++i) o.t[i] = v[V_T + i];
  return o;
}

// All intermediate quantities of one projection (kept for the adjoint).
struct Proj {
  int flags = 0;
  double x[3];           // camera-space centre
  double tc;
  double qn[4], qnorm;
  M3 Rg, Sig, Sc, J, Sp;
  M3 Sci;                // Sc^-1, for the exact ray maximum of Eq. 7
  double B0[3];          // undilated 2x2 footprint (00, 01, 11)
  double B[3];           // dilated
  double conic[3];       // B^-1 as (a, b, c)
  double q[2], p[2];
  double nraw[3], n[3], nlen;
  double uc, vc;
  double dvec[3], dist, dir[3];
  double rgb_raw[3], rgb[3];
  double o, tau;
  int rect[4];
};

bool finite_all(const float* a, int n) {
  for (int i = 0; i < n; ++i) if (!std::isfinite(a[i])) return false;
  return true;
}

// Projection of Gaussian g for one view.  Sec. 3.1 (Eq. 1-3) and Sec. 3.2-3.3
// (Eq. 4, 8, 13-15, 21-22).
void project_one(const View& v, const double* s, int K, const float* mean, const float* scale,
                 const float* quat, float opac, const float* sh, Proj& P) {
  P.flags = 0;
  if (!finite_all(mean, 3) || !finite_all(scale, 3) || !finite_all(quat, 4) ||
      !std::isfinite(opac) || !finite_all(sh, 3 * K)) {
    P.flags = F_CULLED; return;
  }
  const double mu[3] = {mean[0], mean[1], mean[2]};
  // Camera-space centre x = R mu + t; summed left to right (products of two
  // FP32 numbers are exact in FP64, so only this order fixes the result).
  for (int i = 0; i < 3; ++i)
    P.x[i] = ((v.R(i, 0) * mu[0] + v.R(i, 1) * mu[1]) + v.R(i, 2) * mu[2]) + v.t[i];
  const double X = P.x[0], Y = P.x[1], Z = P.x[2];
  if (!(Z > s[S_NEAR])) { P.flags = F_CULLED; return; }
  // alpha = o e^-power >= alpha_min needs o > alpha_min: otherwise the support is empty
  if (!((double)opac > s[S_ALPHA_MIN])) { P.flags = F_CULLED; return; }
  P.o = opac;

  // Eq. 1: Sigma = R S S^T R^T with R from the normalised quaternion.
  P.qnorm = std::sqrt((double)quat[0] * quat[0] + (double)quat[1] * quat[1] +
                      (double)quat[2] * quat[2] + (double)quat[3] * quat[3]);
  if (!(P.qnorm > 0)) { P.flags = F_CULLED; return; }
  for (int i = 0; i < 4; ++i) P.qn[i] = quat[i] / P.qnorm;
  P.Rg = quat_rot(P.qn);
  M3 Msc;
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 3; ++k) Msc(i, k) = P.Rg(i, k) * (double)scale[k];
  P.Sig = mul(Msc, transpose(Msc));
  P.Sc = mul(mul(v.R, P.Sig), transpose(v.R));  // camera frame: W Sigma W^T
  P.Sci = inverse3(P.Sc);

  // Local affine map to ray space (u, v in pixels, t = |x|).
  P.tc = std::sqrt(X * X + Y * Y + Z * Z);
  const double Lx = s[S_FOV_CLAMP] * v.W / (2.0 * v.fx);
  const double Ly = s[S_FOV_CLAMP] * v.H / (2.0 * v.fy);
  double xi = X / Z, eta = Y / Z;
  if (xi < -Lx || xi > Lx) { xi = std::min(Lx, std::max(-Lx, xi)); P.flags |= F_CLAMP_X; }
  if (eta < -Ly || eta > Ly) { eta = std::min(Ly, std::max(-Ly, eta)); P.flags |= F_CLAMP_Y; }
  P.J = zero3();
  P.J(0, 0) = v.fx / Z; P.J(0, 2) = -v.fx * xi / Z;
  P.J(1, 1) = v.fy / Z; P.J(1, 2) = -v.fy * eta / Z;
  P.J(2, 0) = X / P.tc; P.J(2, 1) = Y / P.tc; P.J(2, 2) = Z / P.tc;
  // Eq. 2: Sigma' = J W Sigma W^T J^T.
  P.Sp = mul(mul(P.J, P.Sc), transpose(P.J));
  P.B0[0] = P.Sp(0, 0); P.B0[1] = P.Sp(0, 1); P.B0[2] = P.Sp(1, 1);
  P.B[0] = P.B0[0] + s[S_DILATION]; P.B[1] = P.B0[1]; P.B[2] = P.B0[2] + s[S_DILATION];
  const double detB = P.B[0] * P.B[2] - P.B[1] * P.B[1];
  if (!(detB > 0)) { P.flags = F_CULLED; return; }
  P.conic[0] = P.B[2] / detB; P.conic[1] = -P.B[1] / detB; P.conic[2] = P.B[0] / detB;

  // Eq. 13: q-hat = v'^T Sigma'^-1 / (v'^T Sigma'^-1 v'), v' = (0,0,1); q is
  // its first two entries (its third is one).
  const double det0 = P.B0[0] * P.B0[2] - P.B0[1] * P.B0[1];
  const double tr0 = P.B0[0] + P.B0[2];
  if (det0 <= s[S_DEGEN] * tr0 * tr0) {
    P.q[0] = P.q[1] = 0.0;
    P.flags |= F_DEGENERATE;
  } else {
    M3 A = inverse3(P.Sp);
    P.q[0] = A(2, 0) / A(2, 2);
    P.q[1] = A(2, 1) / A(2, 2);
  }
  // Eq. 15-17: p-hat = (z_c / t_c) q-hat; p is its first two entries.
  P.p[0] = Z / P.tc * P.q[0];
  P.p[1] = Z / P.tc * P.q[1];
  // Eq. 21-22: n' = -(q, 1), n = J^T n' normalised.
  for (int k = 0; k < 3; ++k)
    P.nraw[k] = -(P.q[0] * P.J(0, k) + P.q[1] * P.J(1, k) + P.J(2, k));
  P.nlen = std::sqrt(P.nraw[0] * P.nraw[0] + P.nraw[1] * P.nraw[1] + P.nraw[2] * P.nraw[2]);
  for (int k = 0; k < 3; ++k) P.n[k] = P.nraw[k] / P.nlen;

  // Projected centre in pixels.
  P.uc = v.fx * X / Z + v.cx;
  P.vc = v.fy * Y / Z + v.cy;

  // Colour: SH evaluated along the direction from the camera centre
  // C = -R^T t to the mean, plus 0.5, clamped at zero.
  double C[3];
  for (int i = 0; i < 3; ++i) C[i] = -(v.R(0, i) * v.t[0] + v.R(1, i) * v.t[1] + v.R(2, i) * v.t[2]);
  for (int i = 0; i < 3; ++i) P.dvec[i] = mu[i] - C[i];
  P.dist = std::sqrt(P.dvec[0] * P.dvec[0] + P.dvec[1] * P.dvec[1] + P.dvec[2] * P.dvec[2]);
  for (int i = 0; i < 3; ++i) P.dir[i] = P.dvec[i] / P.dist;
  SH ysh;
  const int degree = (int)s[S_SH_DEGREE];
  eval_sh(degree, P.dir, ysh);
  for (int c = 0; c < 3; ++c) {
    double acc = 0.0;
    for (int j = 0; j < K; ++j) acc += (double)sh[3 * j + c] * ysh.y[j];
    P.rgb_raw[c] = acc + 0.5;
    if (P.rgb_raw[c] < 0.0) { P.rgb[c] = 0.0; P.flags |= (F_RGB_CLAMP0 << c); }
    else P.rgb[c] = P.rgb_raw[c];
  }

  // Support: power <= tau, tau = min(cut, ln(o / alpha_min)) (alpha >= alpha_min
  // there, before the clamp at alpha_max); conservative axis-aligned pixel rect
  // of that ellipse.
  P.tau = std::min(s[S_POWER_CUT], std::log(P.o / s[S_ALPHA_MIN]));
  const double rx = std::sqrt(2.0 * P.tau * P.B[0]) * (1.0 + 1e-6) + 1e-3;
  const double ry = std::sqrt(2.0 * P.tau * P.B[2]) * (1.0 + 1e-6) + 1e-3;
  const double xlo = (P.uc - rx) - 0.5, xhi = (P.uc + rx) - 0.5;
  const double ylo = (P.vc - ry) - 0.5, yhi = (P.vc + ry) - 0.5;
  bool vis = std::isfinite(xlo) && std::isfinite(xhi) && std::isfinite(ylo) && std::isfinite(yhi) &&
             xhi >= 0.0 && yhi >= 0.0 && xlo <= v.W - 1.0 && ylo <= v.H - 1.0;
  if (vis) {
    P.rect[0] = std::max(0, (int)std::ceil(std::max(xlo, -1.0)));
    P.rect[1] = std::min(v.W - 1, (int)std::floor(std::min(xhi, (double)v.W)));
    P.rect[2] = std::max(0, (int)std::ceil(std::max(ylo, -1.0)));
    P.rect[3] = std::min(v.H - 1, (int)std::floor(std::min(yhi, (double)v.H)));
    vis = P.rect[0] <= P.rect[1] && P.rect[2] <= P.rect[3];
  }
  if (vis) P.flags |= F_VISIBLE;
  else { P.rect[0] = 0; P.rect[1] = -1; P.rect[2] = 0; P.rect[3] = -1; }
}

void store_record(const Proj& P, double* r, int* rect, int* flags) {
  std::fill(r, r + R_COUNT, 0.0);
  *flags = P.flags;
  rect[0] = 0; rect[1] = -1; rect[2] = 0; rect[3] = -1;
  if (P.flags & F_CULLED) return;
  r[R_UC] = P.uc; r[R_VC] = P.vc; r[R_Z] = P.x[2]; r[R_TC] = P.tc;
  r[R_A] = P.conic[0]; r[R_B] = P.conic[1]; r[R_C] = P.conic[2]; r[R_O] = P.o;
  r[R_R] = P.rgb[0]; r[R_G] = P.rgb[1]; r[R_BL] = P.rgb[2];
  r[R_P0] = P.p[0]; r[R_P1] = P.p[1]; r[R_Q0] = P.q[0]; r[R_Q1] = P.q[1];
  r[R_N0] = P.n[0]; r[R_N1] = P.n[1]; r[R_N2] = P.n[2]; r[R_TAU] = P.tau;
  r[R_B00] = P.B[0]; r[R_B01] = P.B[1]; r[R_B11] = P.B[2];
  r[R_X] = P.x[0]; r[R_Y] = P.x[1];
  r[R_AI00] = P.Sci(0, 0); r[R_AI01] = P.Sci(0, 1); r[R_AI02] = P.Sci(0, 2);
  r[R_AI11] = P.Sci(1, 1); r[R_AI12] = P.Sci(1, 2); r[R_AI22] = P.Sci(2, 2);
  for (int i = 0; i < 4; ++i) rect[i] = P.rect[i];
}

// Blend order of one view: non-culled Gaussians by ascending (float32(z), id).
std::vector<int64_t> blend_order(int64_t N, const double* rec, const int* flags) {
  std::vector<int64_t> ids;
  ids.reserve(N);
  for (int64_t g = 0; g < N; ++g)
    if (!(flags[g] & F_CULLED)) ids.push_back(g);
  std::stable_sort(ids.begin(), ids.end(), [&](int64_t a, int64_t b) {
    return (float)rec[a * R_COUNT + R_Z] < (float)rec[b * R_COUNT + R_Z];
  });
  return ids;
}

struct Contrib {
  int64_t g;
  double alpha, T, dx, dy, d, gauss;
  bool clamped;
};

struct PixelResult {
  double out[O_COUNT];
  int count;
  int64_t last, median;
  int fragile;
  uint64_t sig;
  std::vector<Contrib> list;
};

inline uint64_t mix64(uint64_t h, uint64_t v) {
  h ^= v + 0x9e3779b97f4a7c15ULL + (h << 6) + (h >> 2);
  return h;
}

// Depth of the point where the ray through the pixel centre meets Gaussian r
// (Sec. 3.2.1, Eq. 5-7): the camera centre is the origin, the ray direction
// the unit vector through the pixel, the intersection the maximum of the
// Gaussian along the ray, t* = v^T Sigma^-1 x_c / (v^T Sigma^-1 v), and the
// depth its camera z, t* v_z.
double exact_ray_depth(const View& v, const double* r, double pcx, double pcy) {
  double dir[3] = {(pcx - v.cx) / v.fx, (pcy - v.cy) / v.fy, 1.0};
  const double len = std::sqrt(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
  for (double& d : dir) d /= len;
  const double xc[3] = {r[R_X], r[R_Y], r[R_Z]};
  M3 A;
  A(0, 0) = r[R_AI00]; A(0, 1) = A(1, 0) = r[R_AI01]; A(0, 2) = A(2, 0) = r[R_AI02];
  A(1, 1) = r[R_AI11]; A(1, 2) = A(2, 1) = r[R_AI12]; A(2, 2) = r[R_AI22];
  double num = 0.0, den = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      num += dir[i] * A(i, j) * xc[j];
      den += dir[i] * A(i, j) * dir[j];
    }
  return num / den * dir[2];
}

// Front-to-back compositing of one pixel over every Gaussian (Eq. 3, Eq. 4;
// with S_DEPTH_EXACT the per-pixel depth of Eq. 7 instead of Eq. 4).
void render_pixel(const double* s, const View& view, const double* rec,
                  const std::vector<int64_t>& order, int px, int py, bool keep_list,
                  PixelResult& R) {
  const bool exact = s[S_DEPTH_EXACT] != 0.0;
  const double cut = s[S_POWER_CUT], amin = s[S_ALPHA_MIN], amax = s[S_ALPHA_MAX];
  const double tmin = s[S_T_MIN];
  double T = 1.0;
  for (int i = 0; i < O_COUNT; ++i) R.out[i] = 0.0;
  R.count = 0; R.last = -1; R.median = -1; R.fragile = 0; R.sig = 1469598103934665603ULL;
  R.list.clear();
  const double pcx = px + 0.5, pcy = py + 0.5;
  int64_t stop_g = -1;
  std::vector<double> ws, ds;  // weight and depth of every blended splat
  for (int64_t g : order) {
    const double* r = rec + g * R_COUNT;
    const double dx = r[R_UC] - pcx, dy = r[R_VC] - pcy;
    const double power = 0.5 * (r[R_A] * dx * dx + 2.0 * r[R_B] * dx * dy + r[R_C] * dy * dy);
    if (std::fabs(power - cut) < s[S_FRAG_POWER]) R.fragile |= 1;
    if (power > cut) continue;
    const double gauss = std::exp(-power);
    const double raw = r[R_O] * gauss;
    if (std::fabs(raw - amax) < s[S_FRAG_CLAMP] * amax) R.fragile |= 2;
    const bool clamped = raw > amax;
    const double alpha = clamped ? amax : raw;
    if (std::fabs(alpha - amin) < s[S_FRAG_ALPHA] * amin) R.fragile |= 1;
    if (alpha < amin) continue;
    const double Tn = T * (1.0 - alpha);
    if (std::fabs(Tn - tmin) < s[S_FRAG_T] * tmin) R.fragile |= 1;
    if (Tn < tmin) { stop_g = g; break; }
    const double w = alpha * T;
    const double d = exact ? exact_ray_depth(view, r, pcx, pcy)
                           : r[R_Z] + r[R_P0] * dx + r[R_P1] * dy;  // Eq. 4, dx = u_c - u
    R.out[O_R] += w * r[R_R]; R.out[O_G] += w * r[R_G]; R.out[O_B] += w * r[R_BL];
    R.out[O_DEXP] += w * d;
    R.out[O_N0] += w * r[R_N0]; R.out[O_N1] += w * r[R_N1]; R.out[O_N2] += w * r[R_N2];
    R.out[O_ALPHA] += w;
    if (std::fabs(T - 0.5) < s[S_FRAG_MED] * 0.5) R.fragile |= 1;
    if (T > 0.5) { R.median = g; R.out[O_DMED] = d; }
    R.count += 1;
    R.last = g;
    R.sig = mix64(R.sig, (uint64_t)g * 2 + (clamped ? 1 : 0));
    if (keep_list) R.list.push_back({g, alpha, T, dx, dy, d, gauss, clamped});
    ws.push_back(w);
    ds.push_back(d);
    T = Tn;
  }
  // Eq. 23: sum over all ordered pairs of blended splats.  dist_mag =
  // sum w_i w_j |d_i - d_j| (|d_i| + |d_j|): when every depth moves by a
  // relative amount of at most eps the sum moves by at most 2 eps dist_mag
  // to first order (attained with two splats moved apart), the round-off
  // scale of an evaluation from depths rounded to a lower precision.
  double dist = 0.0, mag = 0.0;
  for (size_t i = 0; i < ws.size(); ++i)
    for (size_t j = 0; j < ws.size(); ++j) {
      dist += ws[i] * ws[j] * (ds[i] - ds[j]) * (ds[i] - ds[j]);
      mag += ws[i] * ws[j] * std::fabs(ds[i] - ds[j]) * (std::fabs(ds[i]) + std::fabs(ds[j]));
    }
  R.out[O_DIST] = dist;
  R.out[O_DIST_MAG] = mag;
  R.out[O_R] += T * s[S_BG0]; R.out[O_G] += T * s[S_BG1]; R.out[O_B] += T * s[S_BG2];
  R.out[O_TFIN] = T;
  R.sig = mix64(R.sig, (uint64_t)(R.median + 7));
  R.sig = mix64(R.sig, (uint64_t)(stop_g + 11));
}

// Adjoint of one projection: gradient of the projected quantities gP (layout
// G_*) -> parameter gradients (accumulated).
void project_one_bwd(const View& v, const double* s, int K, const float* mean, const float* scale,
                     const float* quat, const float* sh, const Proj& P, const double* gP,
                     double* gmean, double* gscale, double* gquat, double* gopac, double* gsh) {
  const double X = P.x[0], Y = P.x[1], Z = P.x[2];
  double gx[3] = {0, 0, 0};
  double gtc = 0.0;
  M3 gJ = zero3();
  M3 gSp = zero3();

  // Opacity enters alpha directly.
  *gopac += gP[G_O];

  // Colour -> SH coefficients and the view direction.
  {
    SH ysh;
    eval_sh((int)s[S_SH_DEGREE], P.dir, ysh);
    double gdir[3] = {0, 0, 0};
    for (int c = 0; c < 3; ++c) {
      const double gc = (P.flags & (F_RGB_CLAMP0 << c)) ? 0.0 : gP[G_R + c];
      if (gc == 0.0) continue;
      for (int j = 0; j < K; ++j) {
        gsh[3 * j + c] += gc * ysh.y[j];
        for (int k = 0; k < 3; ++k) gdir[k] += gc * (double)sh[3 * j + c] * ysh.dy[j][k];
      }
    }
    const double dd = P.dir[0] * gdir[0] + P.dir[1] * gdir[1] + P.dir[2] * gdir[2];
    for (int k = 0; k < 3; ++k) gmean[k] += (gdir[k] - P.dir[k] * dd) / P.dist;
  }

  // Centre in pixels.
  gx[0] += gP[G_UC] * v.fx / Z;
  gx[1] += gP[G_VC] * v.fy / Z;
  gx[2] += -gP[G_UC] * v.fx * X / (Z * Z) - gP[G_VC] * v.fy * Y / (Z * Z);
  // Depth d = z + p . delta: the z field is the camera z.
  gx[2] += gP[G_Z];

  // p = (Z / tc) q.
  double gq[2] = {Z / P.tc * gP[G_P0], Z / P.tc * gP[G_P1]};
  const double pq = gP[G_P0] * P.q[0] + gP[G_P1] * P.q[1];
  gx[2] += pq / P.tc;
  gtc += -Z * pq / (P.tc * P.tc);

  // n = nraw / |nraw|, nraw = -(q0 J0 + q1 J1 + J2) (rows of J).
  {
    const double gn[3] = {gP[G_N0], gP[G_N1], gP[G_N2]};
    const double nd = P.n[0] * gn[0] + P.n[1] * gn[1] + P.n[2] * gn[2];
    double gnr[3];
    for (int k = 0; k < 3; ++k) gnr[k] = (gn[k] - P.n[k] * nd) / P.nlen;
    for (int k = 0; k < 3; ++k) {
      gq[0] += -P.J(0, k) * gnr[k];
      gq[1] += -P.J(1, k) * gnr[k];
      gJ(0, k) += -P.q[0] * gnr[k];
      gJ(1, k) += -P.q[1] * gnr[k];
      gJ(2, k) += -gnr[k];
    }
  }

  // q = -B0^-1 b (the same function as Eq. 13 written through the Schur
  // complement): gB0 = -B0^-1 gq q^T, gb = -B0^-1 gq.
  if (!(P.flags & F_DEGENERATE)) {
    const double det0 = P.B0[0] * P.B0[2] - P.B0[1] * P.B0[1];
    const double i00 = P.B0[2] / det0, i01 = -P.B0[1] / det0, i11 = P.B0[0] / det0;
    const double h0 = i00 * gq[0] + i01 * gq[1];
    const double h1 = i01 * gq[0] + i11 * gq[1];
    gSp(0, 0) += -h0 * P.q[0]; gSp(0, 1) += -h0 * P.q[1];
    gSp(1, 0) += -h1 * P.q[0]; gSp(1, 1) += -h1 * P.q[1];
    gSp(0, 2) += -h0; gSp(1, 2) += -h1;
  }

  // conic = B^-1, B = B0 + dilation I: gB = -conic G conic.
  {
    const double ca = P.conic[0], cb = P.conic[1], cc = P.conic[2];
    const double G00 = gP[G_A], G01 = 0.5 * gP[G_B], G11 = gP[G_C];
    // C G
    const double t00 = ca * G00 + cb * G01, t01 = ca * G01 + cb * G11;
    const double t10 = cb * G00 + cc * G01, t11 = cb * G01 + cc * G11;
    // (C G) C
    gSp(0, 0) += -(t00 * ca + t01 * cb);
    gSp(0, 1) += -(t00 * cb + t01 * cc);
    gSp(1, 0) += -(t10 * ca + t11 * cb);
    gSp(1, 1) += -(t10 * cb + t11 * cc);
  }

  // Sigma' = J Sc J^T.
  const M3 gSpS = add(gSp, transpose(gSp));
  gJ = add(gJ, mul(mul(gSpS, P.J), P.Sc));
  const M3 gSc = mul(mul(transpose(P.J), gSp), P.J);

  // J(x): rows 0,1 with the x/z, y/z clamp; row 2 = x / tc.
  gx[2] += -gJ(0, 0) * v.fx / (Z * Z) - gJ(1, 1) * v.fy / (Z * Z);
  if (P.flags & F_CLAMP_X) {
    const double xi = -P.J(0, 2) * Z / v.fx;
    gx[2] += gJ(0, 2) * v.fx * xi / (Z * Z);
  } else {
    gx[0] += -gJ(0, 2) * v.fx / (Z * Z);
    gx[2] += gJ(0, 2) * 2.0 * v.fx * X / (Z * Z * Z);
  }
  if (P.flags & F_CLAMP_Y) {
    const double eta = -P.J(1, 2) * Z / v.fy;
    gx[2] += gJ(1, 2) * v.fy * eta / (Z * Z);
  } else {
    gx[1] += -gJ(1, 2) * v.fy / (Z * Z);
    gx[2] += gJ(1, 2) * 2.0 * v.fy * Y / (Z * Z * Z);
  }
  for (int j = 0; j < 3; ++j) {
    double acc = 0.0;
    for (int k = 0; k < 3; ++k) {
      const double dkj = (k == j ? 1.0 : 0.0) - P.x[k] * P.x[j] / (P.tc * P.tc);
      acc += gJ(2, k) * dkj / P.tc;
    }
    gx[j] += acc;
  }
  for (int j = 0; j < 3; ++j) gx[j] += gtc * P.x[j] / P.tc;

  // Camera-space centre -> mean.
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 3; ++k) gmean[i] += v.R(k, i) * gx[k];

  // Sc = R Sigma R^T -> Sigma -> M = Rg diag(s) -> s, Rg -> quaternion.
  const M3 gSig = mul(mul(transpose(v.R), gSc), v.R);
  M3 Msc;
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 3; ++k) Msc(i, k) = P.Rg(i, k) * (double)scale[k];
  const M3 gM = mul(add(gSig, transpose(gSig)), Msc);
  M3 gRg;
  for (int k = 0; k < 3; ++k) {
    double acc = 0.0;
    for (int i = 0; i < 3; ++i) {
      acc += gM(i, k) * P.Rg(i, k);
      gRg(i, k) = gM(i, k) * (double)scale[k];
    }
    gscale[k] += acc;
  }
  M3 dR[4];
  quat_rot_grad(P.qn, dR);
  double gqn[4];
  for (int a = 0; a < 4; ++a) {
    double acc = 0.0;
    for (int i = 0; i < 9; ++i) acc += gRg.m[i] * dR[a].m[i];
    gqn[a] = acc;
  }
  const double qd = P.qn[0] * gqn[0] + P.qn[1] * gqn[1] + P.qn[2] * gqn[2] + P.qn[3] * gqn[3];
  for (int a = 0; a < 4; ++a) gquat[a] += (gqn[a] - P.qn[a] * qd) / P.qnorm;
  (void)mean; (void)quat;
}

}  // namespace

extern "C" {

int oracle_settings_count() { return S_COUNT; }
int oracle_view_count() { return V_COUNT; }
int oracle_record_count() { return R_COUNT; }
int oracle_grad_count() { return G_COUNT; }
int oracle_out_count() { return O_COUNT; }

// Projection of N Gaussians into V views.  rec: V*N*R_COUNT, rect: V*N*4,
// flags: V*N.
int oracle_project(const double* settings, const double* views, int V, int64_t N,
                   const float* means, const float* scales, const float* quats,
                   const float* opac, const float* sh, double* rec, int* rect, int* flags) {
  const int K = ((int)settings[S_SH_DEGREE] + 1) * ((int)settings[S_SH_DEGREE] + 1);
  for (int vi = 0; vi < V; ++vi) {
    const View v = load_view(views + (int64_t)vi * V_COUNT);
#pragma omp parallel for schedule(static)
    for (int64_t g = 0; g < N; ++g) {
      Proj P;
      project_one(v, settings, K, means + 3 * g, scales + 3 * g, quats + 4 * g, opac[g],
                  sh + 3 * K * g, P);
      const int64_t o = (int64_t)vi * N + g;
      store_record(P, rec + o * R_COUNT, rect + 4 * o, flags + o);
    }
  }
  return 0;
}

// Brute-force render of one view from its records.  pix: list of pixel
// indices (py*W+px) or NULL for all W*H pixels.  out: npix*O_COUNT,
// iout: npix*4 = (count, last id, median id, fragile bits), sig: npix.
int oracle_render(const double* settings, const double* view, int64_t N, const double* rec,
                  const int* flags, const int64_t* pix, int64_t npix, double* out, int64_t* iout,
                  uint64_t* sig) {
  const View v = load_view(view);
  const std::vector<int64_t> order = blend_order(N, rec, flags);
  if (!pix) npix = (int64_t)v.W * v.H;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < npix; ++i) {
    const int64_t idx = pix ? pix[i] : i;
    const int px = (int)(idx % v.W), py = (int)(idx / v.W);
    PixelResult R;
    render_pixel(settings, v, rec, order, px, py, false, R);
    for (int k = 0; k < O_COUNT; ++k) out[i * O_COUNT + k] = R.out[k];
    iout[i * 4 + 0] = R.count; iout[i * 4 + 1] = R.last; iout[i * 4 + 2] = R.median;
    iout[i * 4 + 3] = R.fragile;
    if (sig) sig[i] = R.sig;
  }
  return 0;
}

// Adjoint of the compositing of one view: upstream gradients per requested
// pixel, gout: npix*GOUT = (color 3, depth expected, depth median, normal 3,
// alpha, depth distortion) -> gradient of the projected quantities gP:
// N*G_COUNT (accumulated); the distortion term treats the blend weights as
// constants (they are detached in the training loss, Sec. 4.1);
// gP_abs (optional) accumulates, per term, a bound of the magnitudes of the
// quantities it is computed from (the round-off scale of that term).
int oracle_render_bwd(const double* settings, const double* view, int64_t N, const double* rec,
                      const int* flags, const int64_t* pix, int64_t npix, const double* gout,
                      double* gP, double* gP_abs) {
  const View v = load_view(view);
  const std::vector<int64_t> order = blend_order(N, rec, flags);
  if (!pix) npix = (int64_t)v.W * v.H;
  const double bg[3] = {settings[S_BG0], settings[S_BG1], settings[S_BG2]};
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < npix; ++i) {
    const int64_t idx = pix ? pix[i] : i;
    const int px = (int)(idx % v.W), py = (int)(idx / v.W);
    PixelResult R;
    render_pixel(settings, v, rec, order, px, py, true, R);
    const double* g = gout + i * GOUT;
    const double gC[3] = {g[0], g[1], g[2]}, gD = g[3], gM = g[4];
    const double gN[3] = {g[5], g[6], g[7]}, gA = g[8], gL = g[9];
    // Reverse pass: R_acc holds the summed contribution of everything behind
    // the current Gaussian (later blends and the background).
    double Racc = R.out[O_TFIN] * (gC[0] * bg[0] + gC[1] * bg[1] + gC[2] * bg[2]);
    // Magnitude bound of every intermediate (same recursion with absolute
    // values): the scale of round-off of a reduced-precision evaluation.
    double Rabs = R.out[O_TFIN] * (std::fabs(gC[0] * bg[0]) + std::fabs(gC[1] * bg[1]) +
                                   std::fabs(gC[2] * bg[2]));
    for (int64_t k = (int64_t)R.list.size() - 1; k >= 0; --k) {
      const Contrib& c = R.list[k];
      const double* r = rec + c.g * R_COUNT;
      const double w = c.alpha * c.T;
      const double sfeat = gC[0] * r[R_R] + gC[1] * r[R_G] + gC[2] * r[R_BL] + gD * c.d +
                           gN[0] * r[R_N0] + gN[1] * r[R_N1] + gN[2] * r[R_N2] + gA;
      const double galpha = c.T * sfeat - Racc / (1.0 - c.alpha);
      Racc += w * sfeat;
      double gd = w * gD + (c.g == R.median ? gM : 0.0);
      // d/dd_k of sum_{i,j} w_i w_j (d_i - d_j)^2 = 4 w_k sum_j w_j (d_k - d_j)
      double sdist = 0.0, sdist_abs = 0.0;
      if (gL != 0.0) {
        for (const Contrib& o : R.list) {
          sdist += o.alpha * o.T * (c.d - o.d);
          sdist_abs += o.alpha * o.T * (std::fabs(c.d) + std::fabs(o.d));
        }
        gd += gL * 4.0 * w * sdist;
      }
      double gpow = 0.0, go = 0.0;
      if (!c.clamped) {
        gpow = -galpha * c.alpha;  // d alpha / d power = -alpha
        go = galpha * c.gauss;     // d alpha / d o = exp(-power)
      }
      double acc[G_COUNT] = {0};
      // power = 1/2 (a dx^2 + 2 b dx dy + c dy^2), dx = u_c - u.
      acc[G_UC] = gpow * (r[R_A] * c.dx + r[R_B] * c.dy) + gd * r[R_P0];
      acc[G_VC] = gpow * (r[R_B] * c.dx + r[R_C] * c.dy) + gd * r[R_P1];
      acc[G_A] = gpow * 0.5 * c.dx * c.dx;
      acc[G_B] = gpow * c.dx * c.dy;
      acc[G_C] = gpow * 0.5 * c.dy * c.dy;
      acc[G_O] = go;
      acc[G_R] = w * gC[0]; acc[G_G] = w * gC[1]; acc[G_BL] = w * gC[2];
      acc[G_Z] = gd;
      acc[G_P0] = gd * c.dx; acc[G_P1] = gd * c.dy;
      acc[G_N0] = w * gN[0]; acc[G_N1] = w * gN[1]; acc[G_N2] = w * gN[2];
      double mag[G_COUNT] = {0};
      if (gP_abs) {
        const double sabs = std::fabs(gC[0] * r[R_R]) + std::fabs(gC[1] * r[R_G]) +
                            std::fabs(gC[2] * r[R_BL]) + std::fabs(gD * c.d) +
                            std::fabs(gN[0] * r[R_N0]) + std::fabs(gN[1] * r[R_N1]) +
                            std::fabs(gN[2] * r[R_N2]) + std::fabs(gA);
        const double ga_abs = c.T * sabs + Rabs / (1.0 - c.alpha);
        Rabs += w * sabs;
        const double gd_abs = w * std::fabs(gD) + (c.g == R.median ? std::fabs(gM) : 0.0) +
                              std::fabs(gL) * 4.0 * w * sdist_abs;
        const double gp_abs = c.clamped ? 0.0 : ga_abs * c.alpha;
        const double go_abs = c.clamped ? 0.0 : ga_abs * c.gauss;
        mag[G_UC] = gp_abs * (std::fabs(r[R_A] * c.dx) + std::fabs(r[R_B] * c.dy)) +
                    gd_abs * std::fabs(r[R_P0]);
        mag[G_VC] = gp_abs * (std::fabs(r[R_B] * c.dx) + std::fabs(r[R_C] * c.dy)) +
                    gd_abs * std::fabs(r[R_P1]);
        mag[G_A] = gp_abs * 0.5 * c.dx * c.dx;
        mag[G_B] = gp_abs * std::fabs(c.dx * c.dy);
        mag[G_C] = gp_abs * 0.5 * c.dy * c.dy;
        mag[G_O] = go_abs;
        mag[G_R] = w * std::fabs(gC[0]); mag[G_G] = w * std::fabs(gC[1]);
        mag[G_BL] = w * std::fabs(gC[2]);
        mag[G_Z] = gd_abs;
        mag[G_P0] = gd_abs * std::fabs(c.dx); mag[G_P1] = gd_abs * std::fabs(c.dy);
        mag[G_N0] = w * std::fabs(gN[0]); mag[G_N1] = w * std::fabs(gN[1]);
        mag[G_N2] = w * std::fabs(gN[2]);
      }
      for (int j = 0; j < G_COUNT; ++j) {
#pragma omp atomic
        gP[c.g * G_COUNT + j] += acc[j];
        if (gP_abs) {
#pragma omp atomic
          gP_abs[c.g * G_COUNT + j] += mag[j];
        }
      }
    }
  }
  return 0;
}

// Chain the projected-quantity gradients of V views back to the parameters
// (accumulated over views).  gP: V*N*G_COUNT.
int oracle_project_bwd(const double* settings, const double* views, int V, int64_t N,
                       const float* means, const float* scales, const float* quats,
                       const float* opac, const float* sh, const double* gP, double* gmeans,
                       double* gscales, double* gquats, double* gopac, double* gsh) {
  const int K = ((int)settings[S_SH_DEGREE] + 1) * ((int)settings[S_SH_DEGREE] + 1);
  for (int vi = 0; vi < V; ++vi) {
    const View v = load_view(views + (int64_t)vi * V_COUNT);
#pragma omp parallel for schedule(static)
    for (int64_t g = 0; g < N; ++g) {
      Proj P;
      project_one(v, settings, K, means + 3 * g, scales + 3 * g, quats + 4 * g, opac[g],
                  sh + 3 * K * g, P);
      if (P.flags & F_CULLED) continue;
      project_one_bwd(v, settings, K, means + 3 * g, scales + 3 * g, quats + 4 * g,
                      sh + 3 * K * g, P, gP + ((int64_t)vi * N + g) * G_COUNT, gmeans + 3 * g,
                      gscales + 3 * g, gquats + 4 * g, gopac + g, gsh + 3 * K * g);
    }
  }
  return 0;
}

// Binning reference: pairs (view-tile, Gaussian) from the pixel rects,
// ordered by the 64-bit key (global tile << 32 | float bits of z) with a
// stable sort, so equal keys keep ascending Gaussian id.
// rect: V*N*4 (x0,x1,y0,y1, empty when x0>x1), z: V*N float32.
// Returns the pair count; when ids/keys are non-NULL they receive up to
// capacity entries; ranges receives 2 per global tile.
int64_t oracle_bin(const int* dims /* V*2: W,H */, int V, int64_t N, int tile_w, int tile_h,
                   const int* rect, const float* z, uint32_t* ids, uint64_t* keys,
                   int64_t capacity, uint32_t* ranges) {
  std::vector<int64_t> base(V + 1, 0);
  std::vector<int> tiles_x(V);
  for (int vi = 0; vi < V; ++vi) {
    tiles_x[vi] = (dims[2 * vi] + tile_w - 1) / tile_w;
    const int ty = (dims[2 * vi + 1] + tile_h - 1) / tile_h;
    base[vi + 1] = base[vi] + (int64_t)tiles_x[vi] * ty;
  }
  std::vector<std::pair<uint64_t, uint32_t>> pairs;
  for (int vi = 0; vi < V; ++vi) {
    for (int64_t g = 0; g < N; ++g) {
      const int* r = rect + 4 * ((int64_t)vi * N + g);
      if (r[0] > r[1] || r[2] > r[3]) continue;
      uint32_t zb;
      std::memcpy(&zb, &z[(int64_t)vi * N + g], 4);
      for (int ty = r[2] / tile_h; ty <= r[3] / tile_h; ++ty)
        for (int tx = r[0] / tile_w; tx <= r[1] / tile_w; ++tx) {
          const uint64_t tile = (uint64_t)(base[vi] + (int64_t)ty * tiles_x[vi] + tx);
          pairs.push_back({(tile << 32) | zb, (uint32_t)g});
        }
    }
  }
  std::stable_sort(pairs.begin(), pairs.end(),
                   [](const std::pair<uint64_t, uint32_t>& a,
                      const std::pair<uint64_t, uint32_t>& b) { return a.first < b.first; });
  const int64_t M = (int64_t)pairs.size();
  if (ranges) {
    for (int64_t t = 0; t < base[V]; ++t) { ranges[2 * t] = 0; ranges[2 * t + 1] = 0; }
    for (int64_t i = 0; i < M; ++i) {
      const uint64_t t = pairs[i].first >> 32;
      if (i == 0 || (pairs[i - 1].first >> 32) != t) ranges[2 * t] = (uint32_t)i;
      ranges[2 * t + 1] = (uint32_t)(i + 1);
    }
  }
  for (int64_t i = 0; i < M && i < capacity; ++i) {
    if (ids) ids[i] = pairs[i].second;
    if (keys) keys[i] = pairs[i].first;
  }
  return M;
}

}  // extern "C"
