// Shared device-side definitions of the RaDe-GS rasterizer library (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "rade.h"

namespace rade {

constexpr int kWave = 64;            // CDNA wavefront
constexpr float kLog2e = 1.4426950408889634f;
// The render kernels round a splat's centre to FP32 relative to the centre of
// the pixel (px & ~31, py & ~31) of each pixel (px, py); every tile size they
// support (at most 32 pixels per side, powers of two) keeps its pixels inside
// one such 32x32 block, so a tile shares one origin and the rounded offsets do
// not depend on the tile size.
constexpr int kOriginAlign = 32;
constexpr double kLog2eD = 1.4426950408889634;

static_assert(sizeof(rade_splat) == 80, "splat record must be 80 bytes");
// the projection stores the record as five 16-byte words
static_assert(offsetof(rade_splat, w) == 16 && offsetof(rade_splat, opacity) == 32 &&
                  offsetof(rade_splat, rgb) == 36 && offsetof(rade_splat, z) == 48 &&
                  offsetof(rade_splat, p) == 52 && offsetof(rade_splat, n) == 60 &&
                  offsetof(rade_splat, rect) == 72,
              "splat record layout");
static_assert(sizeof(rade_view) == 96, "view record must be 96 bytes");

// Render thresholds in the precision the blend loop uses.  Shared by the
// forward and the backward kernels so both take identical decisions.
struct BlendParams {
  float cut2;        // power_cut * log2(e): skip when the factored power exceeds it
  float alpha_min;
  float alpha_max;
  float t_min;
  float bg[3];
  float log2_alpha_min;  // for the support bound of the staging masks
};

inline BlendParams make_blend_params(const rade_settings& s) {
  BlendParams b;
  b.cut2 = (float)(s.power_cut * kLog2eD);
  b.alpha_min = (float)s.alpha_min;
  b.alpha_max = (float)s.alpha_max;
  b.t_min = (float)s.t_min;
  for (int i = 0; i < 3; ++i) b.bg[i] = (float)s.bg[i];
  b.log2_alpha_min = (float)log2(s.alpha_min);
  return b;
}

// Splat as staged in LDS for one tile: 64 bytes, held as four 16-byte
// quarters in arrays of their own (StagedArrays), so that one address
// register reaches every field of a slot through constant offsets (the
// forward needs the first two quarters before its per-lane decision).
// The centre is split into its FP32 offset (ur, vr) from the pixel centre of
// the tile's 32-pixel-aligned origin and the FP32 remainder (ul, vl) of that
// rounding.  For an integer pixel offset x, ur - x is exact, so (ur - x) + ul
// is the pixel's offset to within one rounding whatever the origin.  The
// remainder enters the two linear forms through the constants of
// StagedForm (t1 = w0 (ur - x) + w1 (vr - y) + c1) and the depth plane
// through zc (the plane at the rounded centre), so the loops use it at no
// extra cost; the remainders themselves are staged (StagedRem) only where a
// loop needs the offset itself (the backward's footprint and plane terms,
// the exact depth).  EXACT staging keeps the centre depth z in zc.
struct alignas(16) StagedSplat {
  float ur, vr, w0, w1;
  float w2, w3, o, zc;
  float r, g, b, p0;
  float p1, n0, n1, n2;
};
struct alignas(8) StagedForm {
  float c1, c2;
};
struct alignas(8) StagedRem {
  float ul, vl;
};

// LDS arrays of B staged splats: quarter k of slot r at q[k * B + r] (k < 4),
// the form constants and the remainder (c1, c2, ul, vl) at q[4 * B + r].
template <int B>
struct StagedArrays {
  float4 q[5 * B];

  __device__ __forceinline__ void put(int r, const StagedSplat& s, const StagedForm& f,
                                      const StagedRem& rm) {
    q[r] = make_float4(s.ur, s.vr, s.w0, s.w1);
    q[B + r] = make_float4(s.w2, s.w3, s.o, s.zc);
    q[2 * B + r] = make_float4(s.r, s.g, s.b, s.p0);
    q[3 * B + r] = make_float4(s.p1, s.n0, s.n1, s.n2);
    q[4 * B + r] = make_float4(f.c1, f.c2, rm.ul, rm.vl);
  }
  __device__ __forceinline__ void get(int r, StagedSplat& s, StagedForm& f,
                                      StagedRem& rm) const {
    const float4 a = q[r], b = q[B + r], c = q[2 * B + r], d = q[3 * B + r], e = q[4 * B + r];
    s = StagedSplat{a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w,
                    c.x, c.y, c.z, c.w, d.x, d.y, d.z, d.w};
    f = StagedForm{e.x, e.y};
    rm = StagedRem{e.z, e.w};
  }
};

// The centre of splat record `sp` relative to the pixel centre (ox + 0.5,
// oy + 0.5), split into FP32 head and remainder: U = ur + ul to within FP64
// rounding (U - ur is exact in FP64).
struct CentreSplit {
  float ur, vr, ul, vl;
};
__device__ __forceinline__ CentreSplit split_centre(double uc, double vc, int ox, int oy) {
  const double U = uc - ((double)ox + 0.5), V = vc - ((double)oy + 0.5);
  CentreSplit c;
  c.ur = (float)U;
  c.vr = (float)V;
  c.ul = (float)(U - (double)c.ur);
  c.vl = (float)(V - (double)c.vr);
  return c;
}

// The depth plane's constant for offsets measured from the rounded centre:
// d = z + p . (dx_head + rem) = (z + p . rem) + p . dx_head.  The remainder
// is below half an FP32 unit of the head, so its product with p is formed in
// FP32 at full relative accuracy; z + p . rem is rounded once.
__device__ __forceinline__ float plane_const(float z, float p0, float p1, float ul, float vl) {
  return z + fmaf(p0, ul, p1 * vl);
}

// The linear-form constant w . rem for the same split (the same argument).
__device__ __forceinline__ float form_const(float wa, float wb, float ul, float vl) {
  return fmaf(wa, ul, wb * vl);
}

// alpha of a splat at offset (dx, dy) = (u_r - u, v_r - v) from its rounded
// centre (the remainder enters through the form constants c1, c2).  Returns false
// when the splat is skipped (outside the cut or below alpha_min).  The
// forward and backward kernels both call exactly this function, compiled
// without floating-point contraction, so their decisions match bit for bit.
// splat_eval computes the pieces and leaves the decision to the caller, which
// must take it as splat_alpha does: pw <= cut2 and alpha >= alpha_min.
__device__ __forceinline__ void splat_eval(const StagedSplat& s, const StagedForm& f, float dx,
                                           float dy, const BlendParams& bp, float& t1, float& t2,
                                           float& pw, float& e, float& alpha, bool& clamped) {
  t1 = fmaf(s.w0, dx, fmaf(s.w1, dy, f.c1));
  t2 = fmaf(s.w2, dx, fmaf(s.w3, dy, f.c2));
  pw = fmaf(t1, t1, t2 * t2);
  // evaluated on every lane (no branch): alpha <= alpha_max < 1 always
  e = __builtin_amdgcn_exp2f(-pw);
  const float raw = s.o * e;
  clamped = raw > bp.alpha_max;
  // min(raw, alpha_max) for raw >= 0 (o > 0, e >= 0), as one median: fminf
  // would re-canonicalise the kernel argument on every call
  alpha = __builtin_amdgcn_fmed3f(raw, 0.0f, bp.alpha_max);
}

__device__ __forceinline__ bool splat_alpha(const StagedSplat& s, const StagedForm& f, float dx,
                                            float dy, const BlendParams& bp, float& t1, float& t2,
                                            float& e, float& alpha, bool& clamped) {
  float pw;
  splat_eval(s, f, dx, dy, bp, t1, t2, pw, e, alpha, clamped);
  return pw <= bp.cut2 && alpha >= bp.alpha_min;
}

// Tile of a global tile index: linear search over the (few) views.
__device__ __forceinline__ int view_of_tile(const rade_view* views, int V, int64_t tile) {
  int v = 0;
  while (v + 1 < V && views[v + 1].tile_offset <= tile) ++v;
  return v;
}

__device__ __forceinline__ uint64_t ballot64(bool p) { return __ballot(p); }

// Optional events recorded around the launches of one kernel kind (set by
// rade_set_kernel_events).
struct KernelEvents {
  hipEvent_t start = nullptr, stop = nullptr;
};
KernelEvents& kernel_events(int kernel);

struct EventScope {
  hipStream_t st;
  KernelEvents& ev;
  EventScope(int kernel, hipStream_t s) : st(s), ev(kernel_events(kernel)) {
    if (ev.start) (void)hipEventRecord(ev.start, st);
  }
  ~EventScope() {
    if (ev.stop) (void)hipEventRecord(ev.stop, st);
  }
};

// Workgroups of `block` threads that fit on the current device at once for a
// kernel; `cached` is the caller's per-kernel cache (0 until first computed).
template <typename K>
unsigned resident_blocks(K kernel, int block, unsigned cap, unsigned& cached) {
  if (cached == 0) {
    int dev = 0, cus = 0, per_cu = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, 0);
    cached = (unsigned)(cus > 0 ? cus : 256) * (unsigned)(per_cu > 0 ? per_cu : 1);
  }
  return cached < cap ? cached : cap;
}

}  // namespace rade
