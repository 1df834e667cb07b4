// Tile rasterizer: forward blending and its adjoint (gfx950).
//
// One workgroup per screen tile; each wavefront owns an 8x8 block of pixels
// of the tile and each lane one pixel.  The tile's list of splats (depth
// order) is walked in batches: every thread stages one splat into LDS (its
// centre made relative to the pixel centre of the tile's 32-pixel-aligned
// origin in FP64 and split into an FP32 head and remainder, so a pixel's
// offset is exact to one rounding; that origin, and so every FP32 operation
// of a pixel, is the same for every tile size), and tests the
// splat's support rect against every wavefront's 8x8 block; a ballot per
// block turns this into a 64-bit mask per (wavefront, stager wavefront), so
// each wavefront only evaluates splats that can touch its pixels.  A
// wavefront leaves the batch loop as soon as all its lanes have stopped, the
// workgroup as soon as all its wavefronts have.
//
// Forward, per pixel (Eq. 3 for colour; Eq. 4 depth; Eq. 22 normal; median
// depth of Sec. 1): T = 1; for each splat in order, skip if its power exceeds
// the cut or alpha < alpha_min; stop if T (1 - alpha) < t_min; otherwise add
// w = alpha T times (rgb, d, n, 1), record the median splat while T > 1/2,
// and set T = T (1 - alpha).
//
// Optionally (template flag DIST) the forward also returns the depth
// distortion of Sec. 3.4 Eq. 23 per pixel, sum_{i,j} w_i w_j (d_i - d_j)^2 =
// 2 A S with A = sum_i w_i and S = sum_i w_i (d_i - m)^2 about the weighted
// mean m, both updated per blend in the weighted incremental form
// S += A w / (A + w) (d - m)^2, m += w / (A + w) (d - m), whose terms are
// all non-negative, unlike A sum w d^2 - (sum w d)^2 which cancels in FP32.
// Its adjoint with the weights held constant (they are detached in the
// training loss, Sec. 4.1) adds 4 g A w_i (d_i - m) to each splat's depth
// gradient, with A and m = D_exp / A read from the forward's maps.
//
// Backward, per pixel, back to front from the last blended splat, with the
// transmittance recovered as T_i = T_{i+1} / (1 - alpha_i) from the saved
// final T (nothing per blend is stored) and the running sum R of what lies
// behind:  dL/dalpha_i = T_i s_i - R / (1 - alpha_i),  R += w_i s_i, where
// s_i = g_C . rgb_i + g_D d_i + g_N . n_i + g_A.  The 15 per-splat gradients
// are summed over the wavefront with a transpose-reduction built on the
// gfx950 lane-swap instructions and DPP, and added with hardware FP32 atomics
// into a per-(view, Gaussian) record.
#include "common.hpp"

namespace rade {
namespace {

// Staging batch parameter of a tile of 8x8 waves with lane masks on every
// wave (one splat staged per thread).
constexpr int kLaneMaskBatch = -1;

// Tile of TW x TH pixels, wavefronts of WW x WH = 64 pixels (row-major in
// the tile), BATCH splats staged per round (0 or kLaneMaskBatch: one per
// thread), in NCH chunks of 64.
template <int TW, int TH, int WW = 8, int BATCH_ = 0>
struct TileGeom {
  static constexpr int WH = 64 / WW;
  static constexpr int LW = WW == 32 ? 5 : WW == 16 ? 4 : 3;
  static constexpr int NWX = TW / WW;
  static constexpr int NWY = TH / WH;
  static constexpr int NW = NWX * NWY;
  static constexpr int BLOCK = 64 * NW;
  static constexpr int BATCH = BATCH_ > 0 ? BATCH_ : BLOCK;
  static constexpr int NCH = BATCH / 64;
  // One wave per tile, or 8x8 waves with kLaneMaskBatch: staging also
  // computes which of each wave's pixels a splat can reach (a 64-bit lane
  // mask per wave), so the loops skip the splats none of their still-active
  // pixels takes.
  static constexpr bool LM = WW == 8 && (NW == 1 || BATCH_ == kLaneMaskBatch);
  static_assert(WW == 8 || WW == 16 || WW == 32, "wave width");
  static_assert(TW % WW == 0 && TH % WH == 0 && BLOCK <= 1024 && BATCH % 64 == 0, "tile");
};

// A value every lane of the wavefront holds alike, moved to scalar registers
// (so loops and LDS addresses driven by it stay scalar).
__device__ __forceinline__ uint64_t uniform_u64(uint64_t x) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(x >> 32));
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ int wave_index() {
  return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
}

struct PixelCtx {
  int v;
  int64_t tile;
  int x0, y0;  // the tile's first pixel
  int ox, oy;  // the 32-pixel-aligned origin splat centres are made relative to
  int lxi, lyi, px, py;
  bool inside;
  int64_t P, poff, pix;
  uint32_t rb, re;
};

struct FwdArgs {
  BlendParams bp;
  const rade_view* views;
  int V;
  int64_t N, tiles;
  const rade_splat* splats;
  const uint32_t* pair_ids;
  const uint32_t* ranges;
  const uint32_t* order;   // tile visiting order (NULL: natural)
  uint32_t* queue;         // work-queue counter of the persistent kernel
  float *color, *depth, *normal, *alpha, *t_final, *distortion;
  int32_t *last, *median, *count, *evals;
  const float4* depth_quad;  // EXACT only: 2 per (view, Gaussian)
  uint64_t* lane_masks;      // LM tiles, optional: the staged pairs' masks
};

struct BwdArgs {
  BlendParams bp;
  const rade_view* views;
  int V;
  int64_t N, tiles;
  const rade_splat* splats;
  const uint32_t* pair_ids;
  const uint32_t* ranges;
  const uint32_t* order;
  uint32_t* queue;
  const float* t_final;
  const int32_t *last, *median;
  const float *d_color, *d_depth, *d_normal, *d_alpha;
  const float *d_distortion, *fwd_depth, *fwd_alpha;  // DIST only
  float* gsplat;
  const uint64_t* lane_masks;  // LM tiles, optional: the forward's masks
};

// Q: an 8x8 tile held by one wave as four 16-lane groups, one per 4x4
// quadrant: lane = 16 q + 4 y + x, quadrant q = 2 (y / 4) + x / 4 (one DPP
// row of 16 lanes per quadrant).
template <int TW, int TH, int WW, int BT, bool Q = false>
__device__ __forceinline__ PixelCtx pixel_ctx(const rade_view* views, int V,
                                              const uint32_t* ranges, int64_t tile) {
  using TG = TileGeom<TW, TH, WW, BT>;
  PixelCtx c;
  c.tile = tile;
  c.v = view_of_tile(views, V, c.tile);
  const rade_view& vw = views[c.v];
  const int64_t lt = c.tile - vw.tile_offset;
  const int tx = (int)(lt % vw.tiles_x), ty = (int)(lt / vw.tiles_x);
  c.x0 = tx * TW;
  c.y0 = ty * TH;
  c.ox = c.x0 & ~(kOriginAlign - 1);
  c.oy = c.y0 & ~(kOriginAlign - 1);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if constexpr (Q) {
    // 8x8 waves, each as four 4x4 quadrants
    const int q = lane >> 4, i = lane & 15;
    c.lxi = 8 * (wave % TG::NWX) + 4 * (q & 1) + (i & 3);
    c.lyi = 8 * (wave / TG::NWX) + 4 * (q >> 1) + (i >> 2);
  } else {
    c.lxi = WW * (wave % TG::NWX) + (lane & (WW - 1));
    c.lyi = TG::WH * (wave / TG::NWX) + (lane >> TG::LW);
  }
  c.px = c.x0 + c.lxi;
  c.py = c.y0 + c.lyi;
  c.inside = c.px < vw.width && c.py < vw.height;
  c.P = (int64_t)vw.width * vw.height;
  c.poff = vw.pix_offset;
  c.pix = (int64_t)c.py * vw.width + c.px;
  c.rb = ranges[2 * c.tile];
  c.re = ranges[2 * c.tile + 1];
  return c;
}

// Does the splat's support reach the block of pixel offsets [bx, bx+bw-1] x
// [by, by+bh-1] (relative to the pixel centre of the origin (ox, oy))?  The factored
// power Q = (w0 dx + w1 dy)^2 + (w2 dx + w3 dy)^2, dx = ur - x, dy = vr - y,
// is convex, so its minimum over the block's rectangle is 0 when the centre
// lies inside and is otherwise reached on an edge, where it is a 1-D
// quadratic minimised in closed form.  The block is kept when that minimum
// is within the support bound tau2 (with a margin far above FP32 round-off:
// skipping a block must never drop a blend the pixel loop would take).
__device__ __forceinline__ bool block_reached(float ur, float vr, float w0, float w1, float w2,
                                              float w3, float A, float B, float C, float invA,
                                              float invC, float tau2, int bx, int by, int bw,
                                              int bh) {
  const float xlo = ur - (float)(bx + bw - 1), xhi = ur - (float)bx;
  const float ylo = vr - (float)(by + bh - 1), yhi = vr - (float)by;
  if (xlo <= 0.0f && xhi >= 0.0f && ylo <= 0.0f && yhi >= 0.0f) return true;
  auto q = [&](float dx, float dy) {
    const float t1 = fmaf(w0, dx, w1 * dy), t2 = fmaf(w2, dx, w3 * dy);
    return fmaf(t1, t1, t2 * t2);
  };
  auto on_x_edge = [&](float X) {  // dx = X, dy free in [ylo, yhi]
    const float dy = fminf(fmaxf(-B * X * invC, ylo), yhi);
    return q(X, dy);
  };
  auto on_y_edge = [&](float Y) {  // dy = Y, dx free in [xlo, xhi]
    const float dx = fminf(fmaxf(-B * Y * invA, xlo), xhi);
    return q(dx, Y);
  };
  const float m = fminf(fminf(on_x_edge(xlo), on_x_edge(xhi)), fminf(on_y_edge(ylo), on_y_edge(yhi)));
  return m <= tau2;
}

// Lane mask in row-major lane order (lane 8 y + x) to the quadrant order of
// pixel_ctx<..., true> (lane 16 q + 4 (y % 4) + x % 4, q = 2 (y / 4) + x / 4):
// per 32-bit half (four pixel rows, one byte each), the low nibbles (x 0-3)
// gather into bits 0-15 and the high nibbles (x 4-7) into bits 16-31.
__device__ __forceinline__ uint32_t nibbles_to_quadrants(uint32_t w) {
  uint32_t l = w & 0x0F0F0F0Fu, h = (w >> 4) & 0x0F0F0F0Fu;
  l = (l | (l >> 4)) & 0x00FF00FFu;
  h = (h | (h >> 4)) & 0x00FF00FFu;
  l = (l | (l >> 8)) & 0x0000FFFFu;
  h = (h | (h >> 8)) & 0x0000FFFFu;
  return l | (h << 16);
}

__device__ __forceinline__ uint64_t to_quadrant_lanes(uint64_t m) {
  return (uint64_t)nibbles_to_quadrants((uint32_t)m) |
         ((uint64_t)nibbles_to_quadrants((uint32_t)(m >> 32)) << 32);
}

// Stage splat `idx` of the tile list into LDS slot `slot` and return the
// bit set of wave blocks its support reaches (support rect first, then the
// exact ellipse-against-block test).
template <int TW, int TH, int WW, int BT, bool EXACT = false, bool QL = false>
__device__ __forceinline__ uint32_t stage(const rade_splat* __restrict__ splats, int64_t vbase,
                                          const uint32_t* __restrict__ pair_ids, uint32_t idx,
                                          int slot, const PixelCtx& c, const BlendParams& bp,
                                          StagedArrays<TileGeom<TW, TH, WW, BT>::BATCH>& st,
                                          uint32_t* sgid, uint64_t* lmask,
                                          uint64_t* __restrict__ lm_out = nullptr,
                                          const uint64_t* __restrict__ lm_in = nullptr) {
  // lmask (LM tiles): the lane mask of wave k at lmask[k * BATCH + slot].
  // lm_out (LM tiles, optional): the masks (row-major lane order) also go to
  // lm_out[idx * NW + k]; lm_in (LM tiles, optional): masks a forward wrote
  // there for the same lists and launch shape, read instead of computed.
  using TG = TileGeom<TW, TH, WW, BT>;
  const uint32_t g = pair_ids[idx];
  const rade_splat& sp = splats[vbase + g];
  StagedSplat s;
  const CentreSplit cs = split_centre(sp.uc, sp.vc, c.ox, c.oy);
  s.ur = cs.ur; s.vr = cs.vr;
  s.w0 = sp.w[0]; s.w1 = sp.w[1]; s.w2 = sp.w[2]; s.w3 = sp.w[3];
  const StagedForm sform{form_const(sp.w[0], sp.w[1], cs.ul, cs.vl),
                         form_const(sp.w[2], sp.w[3], cs.ul, cs.vl)};
  s.o = sp.opacity;
  s.zc = EXACT ? sp.z : plane_const(sp.z, sp.p[0], sp.p[1], cs.ul, cs.vl);
  s.r = sp.rgb[0]; s.g = sp.rgb[1]; s.b = sp.rgb[2];
  s.p0 = sp.p[0]; s.p1 = sp.p[1];
  s.n0 = sp.n[0]; s.n1 = sp.n[1]; s.n2 = sp.n[2];
  st.put(slot, s, sform, StagedRem{cs.ul, cs.vl});
  sgid[slot] = g;
  const int rx0 = sp.rect[0] - c.x0, rx1 = sp.rect[1] - c.x0;
  const int ry0 = sp.rect[2] - c.y0, ry1 = sp.rect[3] - c.y0;
  uint32_t bits = 0;
#pragma unroll
  for (int k = 0; k < TG::NW; ++k) {
    const int bx = WW * (k % TG::NWX), by = TG::WH * (k / TG::NWX);
    if (rx0 <= bx + WW - 1 && rx1 >= bx && ry0 <= by + TG::WH - 1 && ry1 >= by) bits |= 1u << k;
  }
  uint64_t lm[TG::LM ? TG::NW : 1] = {};
  bool loaded = false;
  if constexpr (TG::LM) {
    if (lm_in) {  // uniform
      const uint64_t* src = lm_in + (int64_t)idx * TG::NW;
      if constexpr (TG::NW % 2 == 0) {
#pragma unroll
        for (int k = 0; k < TG::NW; k += 2) {
          const uint4 q = *reinterpret_cast<const uint4*>(src + k);
          lm[k] = ((uint64_t)q.y << 32) | q.x;
          lm[k + 1] = ((uint64_t)q.w << 32) | q.z;
        }
      } else {
#pragma unroll
        for (int k = 0; k < TG::NW; ++k) lm[k] = src[k];
      }
      if constexpr (QL) {
#pragma unroll
        for (int k = 0; k < TG::NW; ++k) lm[k] = to_quadrant_lanes(lm[k]);
      }
      loaded = true;
    }
  }
  if (bits && !loaded) {
    // Support: power <= cut and opacity 2^-power >= alpha_min.  The bound
    // and the tests below carry margins far above the error of the
    // hardware reciprocal, square root and logarithm (about one unit in
    // the last place), so those stand in for the correctly rounded forms.
    const float A = fmaf(s.w0, s.w0, s.w2 * s.w2), B = fmaf(s.w0, s.w1, s.w2 * s.w3);
    const float C = fmaf(s.w1, s.w1, s.w3 * s.w3);
    const float invA = A > 0.0f ? __builtin_amdgcn_rcpf(A) : 0.0f;
    float lo = -1.0f;
    if (s.o >= 1.17549435e-38f && bp.alpha_min >= 1.17549435e-38f)
      lo = __builtin_amdgcn_logf(s.o) - bp.log2_alpha_min;  // no denormal operands
    else if (s.o > 0.0f)
      lo = log2f(s.o / bp.alpha_min);
    const float tau2 = fminf(bp.cut2, lo) * 1.001f + 0.01f;
    // centre relative to the tile's first pixel (x0 - ox is a small integer:
    // exact), so the block offsets below are compile-time constants
    const float ut = s.ur - (float)(c.x0 - c.ox), vt = s.vr - (float)(c.y0 - c.oy);
    if constexpr (!TG::LM) {
      // drop the blocks the ellipse misses (also when the rect touches a
      // single block: one test per staged pair is far cheaper than a wave
      // iteration over a splat that reaches none of its pixels)
      const float invC = C > 0.0f ? __builtin_amdgcn_rcpf(C) : 0.0f;
#pragma unroll
      for (int k = 0; k < TG::NW; ++k) {
        const int bx = WW * (k % TG::NWX), by = TG::WH * (k / TG::NWX);
        if (((bits >> k) & 1u) && !block_reached(ut, vt, s.w0, s.w1, s.w2, s.w3, A, B, C, invA,
                                                 invC, tau2, bx, by, WW, TG::WH))
          bits &= ~(1u << k);
      }
    } else {
      // Lane masks of the 8x8 waves (lane = 8 y + x, or with QL the
      // quadrant layout of pixel_ctx<..., true>), which also stand for the
      // block test: per pixel row of the support rect, the interval of the
      // ellipse A dx^2 + 2 B dx dy + C dy^2 <= tau2 along the row, widened
      // by a margin and rounded outwards (conservative: the loops still test
      // every pixel), split over the waves the row crosses.
      const int x0 = max(rx0, 0), x1 = min(rx1, TW - 1), y0 = max(ry0, 0), y1 = min(ry1, TH - 1);
      // the Gram determinant A C - B^2 >= 0, lowered by more than its FP32
      // rounding (a lower value only widens the intervals)
      const float det = fmaxf(fmaf(A, C, -(B * B)) - 4e-7f * (A * C), 0.0f);
#pragma unroll
      for (int by = 0; by < TG::NWY; ++by) {  // the waves' rows of 8 pixel rows
        for (int y = max(y0, 8 * by); y <= min(y1, 8 * by + 7); ++y) {
          const float dy = vt - (float)y;
          const float disc = fmaf(-det, dy * dy, A * tau2);
          if (disc < 0.0f) continue;
          int xl = x0, xh = x1;
          if (A > 0.0f) {
            // pixels x = ut - dx with dx in -B dy / A -+ sqrt(disc) / A
            const float xc = fmaf(B * dy, invA, ut), half = __builtin_amdgcn_sqrtf(disc) * invA;
            const float m = 2e-3f + 1e-5f * (fabsf(xc) + half);
            xl = max(xl, (int)ceilf(fmaxf(xc - half - m, -1.0f)));
            xh = min(xh, (int)floorf(fminf(xc + half + m, (float)TW)));
          }
          if (xl > xh) continue;
          const int yy = y - 8 * by;
          // pixels xl..xh of the tile row (TW <= 32; the unsigned shifts
          // wrap to the right mask also for xh = 31)
          const uint32_t row = (2u << xh) - (1u << xl);
#pragma unroll
          for (int bx = 0; bx < TG::NWX; ++bx) {
            const uint32_t r8 = (row >> (8 * bx)) & 0xFFu;  // the wave's 8 pixels
            uint64_t bm;
            if constexpr (QL) {
              // x 0-3 to bits 0-3 (quadrant 2 (yy / 4)), x 4-7 to bits
              // 16-19 (quadrant 2 (yy / 4) + 1): r8 + r8 << 12 does not
              // overlap itself; then row yy % 4 of the two quadrants
              const uint32_t q = (r8 * 0x1001u) & 0x000F000Fu;
              bm = (uint64_t)q << (32 * (yy >> 2) + 4 * (yy & 3));
            } else {
              bm = (uint64_t)r8 << (8 * yy);
            }
            lm[by * TG::NWX + bx] |= bm;
          }
        }
      }
    }
  }
  if constexpr (TG::LM) {
    if (!QL && lm_out) {  // uniform; only row-major masks are stored
      uint64_t* dst = lm_out + (int64_t)idx * TG::NW;
      if constexpr (TG::NW % 2 == 0) {
#pragma unroll
        for (int k = 0; k < TG::NW; k += 2)
          *reinterpret_cast<uint4*>(dst + k) =
              make_uint4((uint32_t)lm[k], (uint32_t)(lm[k] >> 32), (uint32_t)lm[k + 1],
                         (uint32_t)(lm[k + 1] >> 32));
      } else {
#pragma unroll
        for (int k = 0; k < TG::NW; ++k) dst[k] = lm[k];
      }
    }
    bits = 0;
#pragma unroll
    for (int k = 0; k < TG::NW; ++k) {
      lmask[k * TG::BATCH + slot] = lm[k];
      if (lm[k]) bits |= 1u << k;
    }
  }
  return bits;
}

// masks[k][chunk]: which splats of a chunk of 64 staged ones reach wave k's
// block (called by whole waves: the ballot needs every lane).
template <int TW, int TH, int WW, int BT>
__device__ __forceinline__ void publish_masks(
    uint32_t bits, int chunk,
    uint64_t (*masks)[TileGeom<TW, TH, WW, BT>::NCH]) {
  using TG = TileGeom<TW, TH, WW, BT>;
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int k = 0; k < TG::NW; ++k) {
    const uint64_t m = __ballot((bits >> k) & 1u);
    if (lane == 0) masks[k][chunk] = m;
  }
}

template <int TW, int TH, bool EXACT, int WW, int BT>
struct FwdShared {
  using TG = TileGeom<TW, TH, WW, BT>;
  StagedArrays<TG::BATCH> st;
  uint32_t sgid[TG::BATCH];
  uint64_t lmask[TG::LM ? TG::NW * TG::BATCH : 1];
  uint64_t masks[TG::NW][TG::NCH];
  // EXACT: the ray-maximum depth terms (g0, g1, H00, H01) and H11
  float4 xq[EXACT ? TG::BATCH : 1];
  float xh[EXACT ? TG::BATCH : 1];
};

// The 16-bit quadrant slices (quadrant layout of pixel_ctx<..., true>) of
// the staged splats' lane masks that hold active lanes, as four chunk masks
// (bit l: staged splat chunk * 64 + l), each lane keeping its own
// quadrant's.  lm: the mask of the splat this lane staged-reads (slot
// chunk * 64 + lane); act: the lanes still working.
__device__ __forceinline__ uint64_t quadrant_chunk_mask(uint64_t lm, uint64_t act, uint64_t m) {
  const uint64_t x = lm & act;
  const uint64_t q0 = __builtin_amdgcn_ballot_w64((x & 0xFFFFull) != 0);
  const uint64_t q1 = __builtin_amdgcn_ballot_w64((x & 0xFFFF0000ull) != 0);
  const uint64_t q2 = __builtin_amdgcn_ballot_w64((x & 0xFFFF00000000ull) != 0);
  const uint64_t q3 = __builtin_amdgcn_ballot_w64((x & 0xFFFF000000000000ull) != 0);
  const int q = (threadIdx.x & 63) >> 4;
  return m & (q == 0 ? q0 : q == 1 ? q1 : q == 2 ? q2 : q3);
}

// Forward blend of one tile (all threads of the workgroup take part).  DIST:
// also the distortion map; CNT: also the blend-count and evaluation-count
// maps (either may be NULL); EXACT: per-pixel
// depth of the ray maximum (Eq. 7) instead of the plane of Eq. 4.
template <int TW, int TH, bool DIST, bool CNT, bool EXACT, int WW, int BT>
__device__ __forceinline__ void fwd_tile(const FwdArgs& a, int64_t tile,
                                         FwdShared<TW, TH, EXACT, WW, BT>& sh) {
  using TG = TileGeom<TW, TH, WW, BT>;
  const BlendParams& bp = a.bp;
  const rade_splat* __restrict__ splats = a.splats;
  const uint32_t* __restrict__ pair_ids = a.pair_ids;
  uint32_t* sgid = sh.sgid;
  auto masks = sh.masks;
  const PixelCtx c = pixel_ctx<TW, TH, WW, BT>(a.views, a.V, a.ranges, tile);
  const int wave = wave_index();
  const int64_t vbase = (int64_t)c.v * a.N;
  // the lane's pixel centre relative to the origin's (exact in FP32)
  const float fx = (float)(c.px - c.ox), fy = (float)(c.py - c.oy);

  float T = 1.0f, C0 = 0.f, C1 = 0.f, C2 = 0.f, D = 0.f, N0 = 0.f, N1 = 0.f, N2 = 0.f, A = 0.f;
  float dmed = 0.f;
  float dmean = 0.f, dvar = 0.f;  // DIST: weighted mean depth and sum w (d - mean)^2
  int cnt = 0, evl = 0, lastp = -1, medp = -1;
  // Lane state of this wave as uniform masks (bit l: lane l), so the
  // per-splat decisions are scalar operations on the compare results and a
  // lane's flag is its bit (inverse ballot): wdone, the lanes that have
  // stopped or lie outside the image.
  uint64_t wdone = __builtin_amdgcn_ballot_w64(!c.inside);

  for (uint32_t b0 = c.rb; b0 < c.re; b0 += TG::BATCH) {
    if (__syncthreads_and(wdone == ~0ull ? 1 : 0)) break;
    // stage the batch: slot = thread + k * BLOCK (each wave's slots share a chunk)
#pragma unroll
    for (int k = 0; k < (TG::BATCH + TG::BLOCK - 1) / TG::BLOCK; ++k) {
      const int slot = (int)threadIdx.x + k * TG::BLOCK;
      if (TG::BATCH % TG::BLOCK != 0 && slot >= TG::BATCH) break;  // wave-uniform
      const uint32_t idx = b0 + (uint32_t)slot;
      uint32_t bits = 0;
      if (idx < c.re) {
        bits = stage<TW, TH, WW, BT, EXACT>(splats, vbase, pair_ids, idx, slot, c, bp, sh.st,
                                            sgid, sh.lmask, a.lane_masks);
        if constexpr (EXACT) {
          const float4* q = a.depth_quad + 2 * (vbase + sgid[slot]);
          sh.xq[slot] = q[0];
          sh.xh[slot] = q[1].x;
        }
      }
      publish_masks<TW, TH, WW, BT>(bits, slot >> 6, masks);
    }
    __syncthreads();
    for (int cw = 0; cw < TG::NCH && wdone != ~0ull; ++cw) {
      uint64_t m = uniform_u64(masks[wave][cw]);
      if constexpr (TG::LM) {
        // drop the chunk's splats whose lane mask holds no pixel still
        // blending (lane l tests staged splat cw * 64 + l)
        m &= __builtin_amdgcn_ballot_w64(
            (sh.lmask[wave * TG::BATCH + cw * 64 + (threadIdx.x & 63)] & ~wdone) != 0);
      }
      while (m && wdone != ~0ull) {
        const int j = __builtin_ctzll(m);
        m &= ~(1ull << j);
        const int r = cw * 64 + j;
        StagedSplat s;
        StagedForm f;
        StagedRem rm;
        sh.st.get(r, s, f, rm);
        const float dx = s.ur - fx, dy = s.vr - fy;
        float t1, t2, pw, e, al;
        bool cl;
        splat_eval(s, f, dx, dy, bp, t1, t2, pw, e, al, cl);
        if constexpr (CNT) evl += __builtin_amdgcn_inverse_ballot_w64(~wdone) ? 1 : 0;
        // the decision of splat_alpha, per lane, as masks
        const uint64_t pass = __builtin_amdgcn_ballot_w64(pw <= bp.cut2) &
                              __builtin_amdgcn_ballot_w64(al >= bp.alpha_min) & ~wdone;
        // one wave per 8x8 tile: skip splats no lane blends (lists whose
        // pixels saturate unevenly); on larger tiles the branch costs more
        // than it saves
        if constexpr (TG::NW == 1) {
          if (!pass) continue;
        }
        // Branch-free blend: lanes that do not take the splat add w = 0
        // (x + 0 * finite = x exactly) and keep their state.
        const float Tn = fmaf(-al, T, T);  // T (1 - alpha), rounded once
        const uint64_t stop = pass & __builtin_amdgcn_ballot_w64(Tn < bp.t_min);
        const uint64_t takes = pass & ~stop;
        wdone |= stop;
        const bool take = __builtin_amdgcn_inverse_ballot_w64(takes);
        const float w = take ? al * T : 0.0f;
        float d;
        if constexpr (EXACT) {
          // z (1 - g.d) / (1 - 2 g.d + H0 dx^2 + H1 dx dy + H2 dy^2), with
          // the offset from the true centre
          const float4 q = sh.xq[r];
          const float h2 = sh.xh[r];
          const float ex = dx + rm.ul, ey = dy + rm.vl;
          const float gd = fmaf(q.y, ey, q.x * ex);
          const float quad = fmaf(h2 * ey, ey, ex * fmaf(q.z, ex, q.w * ey));
          const float den = fmaf(-2.0f, gd, 1.0f) + quad;
          d = s.zc * (1.0f - gd) * __builtin_amdgcn_rcpf(den);
        } else {
          d = fmaf(s.p1, dy, fmaf(s.p0, dx, s.zc));
        }
        C0 = fmaf(w, s.r, C0); C1 = fmaf(w, s.g, C1); C2 = fmaf(w, s.b, C2);
        D = fmaf(w, d, D);
        N0 = fmaf(w, s.n0, N0); N1 = fmaf(w, s.n1, N1); N2 = fmaf(w, s.n2, N2);
        if constexpr (DIST) {
          // m += w/(A+w) delta, S += A w/(A+w) delta^2 (A before this
          // blend): every term of S is a product of non-negative factors, so
          // nothing cancels (the first splat adds exactly 0)
          const float r = take ? __builtin_amdgcn_rcpf(A + w) : 0.0f;
          const float delta = d - dmean;
          const float wr = w * r;
          dmean = fmaf(wr, delta, dmean);
          dvar = fmaf(A * wr, delta * delta, dvar);
        }
        A += w;
        const int pos = (int)(b0 - c.rb) + r;
        const bool med_here =
            __builtin_amdgcn_inverse_ballot_w64(takes & __builtin_amdgcn_ballot_w64(T > 0.5f));
        medp = med_here ? pos : medp;
        if constexpr (EXACT) dmed = med_here ? d : dmed;
        lastp = take ? pos : lastp;
        if constexpr (CNT) cnt += take ? 1 : 0;
        T = take ? Tn : T;
      }
    }
    __syncthreads();
  }
  if (!c.inside) return;
  C0 = fmaf(T, bp.bg[0], C0); C1 = fmaf(T, bp.bg[1], C1); C2 = fmaf(T, bp.bg[2], C2);
  const int64_t P = c.P, pix = c.pix;
  a.color[3 * c.poff + pix] = C0;
  a.color[3 * c.poff + P + pix] = C1;
  a.color[3 * c.poff + 2 * P + pix] = C2;
  a.depth[2 * c.poff + pix] = D;
  if constexpr (!EXACT) {
    // the median splat's plane depth, evaluated once here with the same
    // operations as in the loop (bit-identical to tracking it per blend)
    if (medp >= 0) {
      const rade_splat& sp = splats[vbase + pair_ids[c.rb + medp]];
      const CentreSplit cs = split_centre(sp.uc, sp.vc, c.ox, c.oy);
      const float dx = cs.ur - fx, dy = cs.vr - fy;
      dmed = fmaf(sp.p[1], dy, fmaf(sp.p[0], dx, plane_const(sp.z, sp.p[0], sp.p[1], cs.ul, cs.vl)));
    }
  }
  a.depth[2 * c.poff + P + pix] = medp >= 0 ? dmed : 0.0f;
  a.normal[3 * c.poff + pix] = N0;
  a.normal[3 * c.poff + P + pix] = N1;
  a.normal[3 * c.poff + 2 * P + pix] = N2;
  a.alpha[c.poff + pix] = A;
  a.t_final[c.poff + pix] = T;
  a.last[c.poff + pix] = lastp;
  a.median[c.poff + pix] = medp >= 0 ? (int32_t)pair_ids[c.rb + medp] : -1;
  if constexpr (CNT) {
    if (a.count) a.count[c.poff + pix] = cnt;
    if (a.evals) a.evals[c.poff + pix] = evl;
  }
  if constexpr (DIST) a.distortion[c.poff + pix] = 2.0f * A * dvar;
}

// One workgroup per tile, tiles visited in `order` (or natural) order.
template <int TW, int TH, bool DIST, bool CNT, bool EXACT, int WW, int BT>
__global__ void __launch_bounds__(TW * TH) k_render_fwd(FwdArgs a) {
  __shared__ FwdShared<TW, TH, EXACT, WW, BT> sh;
  const int64_t i = blockIdx.x;
  fwd_tile<TW, TH, DIST, CNT, EXACT, WW, BT>(a, a.order ? (int64_t)a.order[i] : i, sh);
}

// Persistent workgroups pull tiles from a device counter (zeroed before the
// launch) in `order`; every workgroup exits once the counter passes the tile
// count.
template <int TW, int TH, bool DIST, bool CNT, bool EXACT, int WW, int BT>
__global__ void __launch_bounds__(TW * TH) k_render_fwd_persistent(FwdArgs a) {
  __shared__ FwdShared<TW, TH, EXACT, WW, BT> sh;
  __shared__ uint32_t item_s;
  for (;;) {
    if (threadIdx.x == 0) item_s = atomicAdd(a.queue, 1u);
    __syncthreads();
    const uint32_t item = item_s;
    __syncthreads();
    if ((int64_t)item >= a.tiles) break;
    fwd_tile<TW, TH, DIST, CNT, EXACT, WW, BT>(a, a.order ? (int64_t)a.order[item] : (int64_t)item,
                                               sh);
  }
}

template <int CTRL>
__device__ __forceinline__ float dpp(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}

// Pair sums of one transpose-reduction level whose partner lanes lie in the
// other 4-lane bank group of a DPP row: lanes of the banks that hold bit b
// of the lane index clear get a + a(partner), the others b + b(partner).
// Two DPP adds, each writing only its banks (bank_mask), replace the
// select-select-add of the general form.  ror8: partner lane ^ 8 (b = 3,
// banks 0-1 against 2-3); mirror: partner lane ^ 7 within 8 lanes (b = 2,
// banks 0, 2 against 1, 3).  The leading s_nop gives the two wait states a
// DPP read of a vector register needs after the instruction that wrote it.
__device__ __forceinline__ float ror8_pair_sum(float a, float b) {
  float z;
  asm("s_nop 1\n\t"
      "v_add_f32_dpp %0, %1, %1 row_ror:8 row_mask:0xf bank_mask:0x3\n\t"
      "v_add_f32_dpp %0, %2, %2 row_ror:8 row_mask:0xf bank_mask:0xc"
      : "=&v"(z)
      : "v"(a), "v"(b));
  return z;
}

__device__ __forceinline__ float mirror_pair_sum(float a, float b) {
  float z;
  asm("s_nop 1\n\t"
      "v_add_f32_dpp %0, %1, %1 row_half_mirror row_mask:0xf bank_mask:0x5\n\t"
      "v_add_f32_dpp %0, %2, %2 row_half_mirror row_mask:0xf bank_mask:0xa"
      : "=&v"(z)
      : "v"(a), "v"(b));
  return z;
}

// Sum 16 per-lane values over the wavefront by transpose-reduction: every
// level pairs each lane with a partner across one more lane direction, keeps
// half of its values and adds the partner's copy of them, so the number of
// values per lane halves while the set of lanes each value covers doubles.
//   1. v_permlane32_swap(a, b) gives a' = [a.lo32, b.lo32], b' = [a.hi32,
//      b.hi32]: a' + b' is value k in lanes 0-31, value k+8 in lanes 32-63;
//   2. v_permlane16_swap(a, b) gives a' = [a.r0, b.r0, a.r2, b.r2], b' =
//      [a.r1, b.r1, a.r3, b.r3] (16-lane rows): +4 where lane bit 4 is set;
//   3. DPP row_ror:8 (partner = lane ^ 8): +2 where bit 3 is set;
//   4. DPP row_half_mirror (partner = lane ^ 7 within each 8 lanes): +1
//      where bit 2 is set;
//   5. DPP quad_perm xor 1 and xor 2 sum the 4 lanes of each quad.
// The partner directions 32, 16, 8, 7, 1, 2 span all 6 lane bits, so every
// lane is counted once.  On return every lane l holds the total of value
// l >> 2.
__device__ __forceinline__ float wave_sum16(const float (&v)[16]) {
  float u[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[k]),
                                                    __float_as_uint(v[k + 8]), false, false);
    u[k] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
  float w[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(u[k]),
                                                    __float_as_uint(u[k + 4]), false, false);
    w[k] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
  const float x0 = ror8_pair_sum(w[0], w[2]);
  const float x1 = ror8_pair_sum(w[1], w[3]);
  float y = mirror_pair_sum(x0, x1);
  y += dpp<0xB1>(y);
  y += dpp<0x4E>(y);
  return y;
}

// Sum 16 per-lane values over each 16-lane DPP row of the wave by
// transpose-reduction (one level more than the last three of wave_sum16):
// partners lane ^ 8 (row_ror:8), ^ 7 (row_half_mirror), ^ 1 and ^ 2
// (quad_perm), each level keeping half of the values (by the lane bit the
// partner differs in) and adding the partner's copy of them; the partner
// offsets reach all 16 lanes of the row once.  On return lane i of a row
// holds the row's total of value 8 b3 + 4 b2 + 2 b0 + b1 (b_k: bit k of i).
__device__ __forceinline__ float row_sum16(const float (&v)[16]) {
  const int l = (int)threadIdx.x;
  const bool b1 = (l & 2) != 0, b0 = (l & 1) != 0;
  float u[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) u[k] = ror8_pair_sum(v[k], v[k + 8]);
  float w[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) w[k] = mirror_pair_sum(u[k], u[k + 4]);
  float x[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) x[k] = (b0 ? w[k + 2] : w[k]) + dpp<0xB1>(b0 ? w[k] : w[k + 2]);
  return (b1 ? x[1] : x[0]) + dpp<0x4E>(b1 ? x[0] : x[1]);
}

template <int TW, int TH, int WW, int BT>
struct BwdShared {
  using TG = TileGeom<TW, TH, WW, BT>;
  StagedArrays<TG::BATCH> st;
  uint32_t sgid[TG::BATCH];
  uint64_t lmask[TG::LM ? TG::NW * TG::BATCH : 1];
  uint64_t masks[TG::NW][TG::NCH];
  int smax;
};

// Backward pass of one 8x8 tile by one wave as four 16-lane groups, one per
// 4x4 quadrant (pixel_ctx<..., true>): each group walks, from the back, the
// staged splats whose lane mask reaches its pixels that blend at or after
// them, so one step of the wave can take a different splat in every
// quadrant (splats that reach few pixels leave most of a 64-lane step idle
// otherwise), and each group's 15 sums come out of one 16-lane reduction.
// Per pixel the splats, their order and the operations are those of
// bwd_tile.  (The forward keeps one splat per step: its per-splat work is
// small enough that the per-lane bookkeeping of four streams costs more
// than it saves.)
template <int TW, int TH, int BT>
__device__ __forceinline__ void bwd_tile_q(const BwdArgs& a, int64_t tile,
                                           BwdShared<TW, TH, 8, BT>& sh) {
  using TG = TileGeom<TW, TH, 8, BT>;
  const BlendParams& bp = a.bp;
  const rade_splat* __restrict__ splats = a.splats;
  const uint32_t* __restrict__ pair_ids = a.pair_ids;
  float* __restrict__ gsplat = a.gsplat;
  uint32_t* sgid = sh.sgid;
  const PixelCtx c = pixel_ctx<TW, TH, 8, BT, true>(a.views, a.V, a.ranges, tile);
  const int wave = wave_index(), lane = threadIdx.x & 63;
  const int64_t vbase = (int64_t)c.v * a.N;
  // the lane's pixel centre relative to the origin's (exact in FP32)
  const float fx = (float)(c.px - c.ox), fy = (float)(c.py - c.oy);

  float T = 0.f, gC0 = 0.f, gC1 = 0.f, gC2 = 0.f, gD = 0.f, gM = 0.f;
  float gN0 = 0.f, gN1 = 0.f, gN2 = 0.f, gA = 0.f;
  int lastp = -1, med = -1;
  if (c.inside) {
    const int64_t P = c.P, pix = c.pix;
    T = a.t_final[c.poff + pix];
    lastp = a.last[c.poff + pix];
    med = a.median[c.poff + pix];
    if (a.d_color) {
      gC0 = a.d_color[3 * c.poff + pix];
      gC1 = a.d_color[3 * c.poff + P + pix];
      gC2 = a.d_color[3 * c.poff + 2 * P + pix];
    }
    if (a.d_depth) { gD = a.d_depth[2 * c.poff + pix]; gM = a.d_depth[2 * c.poff + P + pix]; }
    if (a.d_normal) {
      gN0 = a.d_normal[3 * c.poff + pix];
      gN1 = a.d_normal[3 * c.poff + P + pix];
      gN2 = a.d_normal[3 * c.poff + 2 * P + pix];
    }
    if (a.d_alpha) gA = a.d_alpha[c.poff + pix];
  }
  float Racc = T * (gC0 * bp.bg[0] + gC1 * bp.bg[1] + gC2 * bp.bg[2]);

  // the furthest last blend of the wave and of the lane's quadrant
  int wlast = lastp;
#pragma unroll
  for (int d = 8; d >= 1; d >>= 1) wlast = max(wlast, __shfl_xor(wlast, d, 64));
  const int qlast = wlast;
  wlast = max(wlast, __shfl_xor(wlast, 16, 64));
  wlast = max(wlast, __shfl_xor(wlast, 32, 64));
  wlast = __builtin_amdgcn_readfirstlane(wlast);
  // records to visit: up to the furthest last blend of the tile (clamped to
  // the list length in case the saved state does not match the lists)
  int tlast = wlast;
  if constexpr (TG::NW > 1) {
    if (threadIdx.x == 0) sh.smax = -1;
    __syncthreads();
    if (lane == 0) atomicMax(&sh.smax, wlast);
    __syncthreads();
    tlast = sh.smax;
  }
  const int nrec = min(tlast + 1, (int)(c.re - c.rb));
  // the sums a lane carries to the splat's record (row_sum16's order)
  const int vi = 8 * ((lane >> 3) & 1) + 4 * ((lane >> 2) & 1) + 2 * (lane & 1) + ((lane >> 1) & 1);

  for (int bend = nrec; bend > 0; bend -= TG::BATCH) {
    const int bstart = bend > TG::BATCH ? bend - TG::BATCH : 0;
#pragma unroll
    for (int k = 0; k < (TG::BATCH + TG::BLOCK - 1) / TG::BLOCK; ++k) {
      const int slot = (int)threadIdx.x + k * TG::BLOCK;
      if (TG::BATCH % TG::BLOCK != 0 && slot >= TG::BATCH) break;  // wave-uniform
      const int li = bstart + slot;
      uint32_t bits = 0;
      if (li < bend)
        bits = stage<TW, TH, 8, BT, false, true>(splats, vbase, pair_ids, c.rb + (uint32_t)li,
                                                 slot, c, bp, sh.st, sgid, sh.lmask, nullptr,
                                                 a.lane_masks);
      publish_masks<TW, TH, 8, BT>(bits, slot >> 6, sh.masks);
    }
    __syncthreads();
    // per chunk, the splats that reach a pixel of the lane's quadrant
    // blending at the chunk's first position or later, at positions up to
    // the quadrant's furthest last blend
    uint64_t qm[TG::NCH];
#pragma unroll
    for (int cw = 0; cw < TG::NCH; ++cw) {
      const int lo = bstart + cw * 64;  // the chunk's first position
      qm[cw] = 0;
      if (wlast < lo) continue;  // nothing at or below a last blend (uniform)
      uint64_t mg = quadrant_chunk_mask(sh.lmask[wave * TG::BATCH + cw * 64 + lane],
                                        __builtin_amdgcn_ballot_w64(lo <= lastp),
                                        uniform_u64(sh.masks[wave][cw]));
      const int ql = qlast - lo;
      qm[cw] = ql < 0 ? 0ull : ql < 63 ? mg & ((2ull << ql) - 1) : mg;
    }
    // Each quadrant walks the batch's chunks from the back on its own (a
    // wave step ends when every quadrant has run out of splats in the whole
    // batch, not in each chunk): cw, the quadrant's current chunk, mg, what
    // is left of it.
    int cw = TG::NCH - 1;
    uint64_t mg = qm[TG::NCH - 1];
    for (;;) {
      if (TG::NCH > 1 && mg == 0) {
        // the next chunk down that holds splats of the quadrant, if any
        int nc = -1;
        uint64_t nm = 0;
#pragma unroll
        for (int k = 0; k < TG::NCH - 1; ++k)
          if (k < cw && qm[k] != 0) { nc = k; nm = qm[k]; }
        cw = nc;
        mg = nm;
      }
      const bool work = mg != 0;
      if (!__any(work)) break;
      {
        int j = 0;
        if (work) {
          j = 63 - __builtin_clzll(mg);
          mg &= ~(1ull << j);
        }
        const int r = (work ? cw * 64 : 0) + j;
        const int pos = bstart + r;
        StagedSplat s;
        StagedForm f;
        StagedRem rm;
        sh.st.get(r, s, f, rm);
        const int gid = (int)sgid[r];
        const float dx = s.ur - fx, dy = s.vr - fy;
        float t1, t2, e, al;
        bool cl;
        const bool has =
            work && splat_alpha(s, f, dx, dy, bp, t1, t2, e, al, cl) && pos <= lastp;
        if (!__any(has)) continue;
        // the operations of bwd_tile's branch-free adjoint (lanes of a
        // quadrant without a splat this step read slot 0, a staged one, and
        // contribute zeros to their own row only)
        const float inv = __builtin_amdgcn_rcpf(1.0f - al);
        const float Ti = T * inv;
        const float w = al * Ti;
        const float d = fmaf(s.p1, dy, fmaf(s.p0, dx, s.zc));
        const float ex = dx + rm.ul, ey = dy + rm.vl;
        float sfm = fmaf(gC0, s.r, gA);
        sfm = fmaf(gC1, s.g, sfm);
        sfm = fmaf(gC2, s.b, sfm);
        sfm = fmaf(gD, d, sfm);
        sfm = fmaf(gN0, s.n0, sfm);
        sfm = fmaf(gN1, s.n1, sfm);
        sfm = fmaf(gN2, s.n2, sfm);
        const float ga = fmaf(Ti, sfm, -(Racc * inv));
        T = has ? Ti : T;
        const float wg = has ? w : 0.0f;
        Racc = fmaf(wg, sfm, Racc);  // + 0 x (finite) where the lane has no blend
        const float gd = fmaf(wg, gD, (has && gid == med) ? gM : 0.0f);
        const float gop = (has && !cl) ? ga * e : 0.0f;
        float g[16];
        const float gpx = gop * ex, gpy = gop * ey;
        g[0] = gpx; g[1] = gpy;
        g[2] = gpx * ex;
        g[3] = gpx * ey;
        g[4] = gpy * ey;
        g[5] = gop;
        g[6] = wg * gC0; g[7] = wg * gC1; g[8] = wg * gC2;
        g[9] = gd;
        g[10] = gd * ex; g[11] = gd * ey;
        g[12] = wg * gN0; g[13] = wg * gN1; g[14] = wg * gN2;
        g[15] = 0.0f;
        const float tot = row_sum16(g);
        if (work && vi < 15 && tot != 0.0f) atomicAdd(gsplat + (vbase + gid) * 16 + vi, tot);
      }
    }
    __syncthreads();
  }
}

// Backward pass of one tile (all threads of the workgroup take part).
template <int TW, int TH, bool DIST, int WW, int BT>
__device__ __forceinline__ void bwd_tile(const BwdArgs& a, int64_t tile,
                                         BwdShared<TW, TH, WW, BT>& sh) {
  using TG = TileGeom<TW, TH, WW, BT>;
  if constexpr (TG::LM && !DIST) {
    bwd_tile_q<TW, TH, BT>(a, tile, sh);
    return;
  }
  const BlendParams& bp = a.bp;
  const rade_splat* __restrict__ splats = a.splats;
  const uint32_t* __restrict__ pair_ids = a.pair_ids;
  const float* __restrict__ t_final = a.t_final;
  const int32_t* __restrict__ last = a.last;
  const int32_t* __restrict__ median = a.median;
  const float* __restrict__ d_color = a.d_color;
  const float* __restrict__ d_depth = a.d_depth;
  const float* __restrict__ d_normal = a.d_normal;
  const float* __restrict__ d_alpha = a.d_alpha;
  float* __restrict__ gsplat = a.gsplat;
  uint32_t* sgid = sh.sgid;
  auto masks = sh.masks;
  int& smax = sh.smax;
  const PixelCtx c = pixel_ctx<TW, TH, WW, BT>(a.views, a.V, a.ranges, tile);
  const int wave = wave_index(), lane = threadIdx.x & 63;
  const int64_t vbase = (int64_t)c.v * a.N;
  // the lane's pixel centre relative to the origin's (exact in FP32)
  const float fx = (float)(c.px - c.ox), fy = (float)(c.py - c.oy);

  float T = 0.f, gC0 = 0.f, gC1 = 0.f, gC2 = 0.f, gD = 0.f, gM = 0.f;
  float gN0 = 0.f, gN1 = 0.f, gN2 = 0.f, gA = 0.f;
  float kdist = 0.f, mdist = 0.f;  // DIST: 4 g A and the weighted mean depth
  int lastp = -1, med = -1;
  if (c.inside) {
    const int64_t P = c.P, pix = c.pix;
    T = t_final[c.poff + pix];
    lastp = last[c.poff + pix];
    med = median[c.poff + pix];
    if (d_color) {
      gC0 = d_color[3 * c.poff + pix];
      gC1 = d_color[3 * c.poff + P + pix];
      gC2 = d_color[3 * c.poff + 2 * P + pix];
    }
    if (d_depth) { gD = d_depth[2 * c.poff + pix]; gM = d_depth[2 * c.poff + P + pix]; }
    if (d_normal) {
      gN0 = d_normal[3 * c.poff + pix];
      gN1 = d_normal[3 * c.poff + P + pix];
      gN2 = d_normal[3 * c.poff + 2 * P + pix];
    }
    if (d_alpha) gA = d_alpha[c.poff + pix];
    if constexpr (DIST) {
      const float Am = a.fwd_alpha[c.poff + pix];
      kdist = 4.0f * a.d_distortion[c.poff + pix] * Am;
      mdist = Am > 0.0f ? a.fwd_depth[2 * c.poff + pix] / Am : 0.0f;
    }
  }
  float Racc = T * (gC0 * bp.bg[0] + gC1 * bp.bg[1] + gC2 * bp.bg[2]);

  if (threadIdx.x == 0) smax = -1;
  __syncthreads();
  atomicMax(&smax, lastp);
  int wlast = lastp;
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) wlast = max(wlast, __shfl_xor(wlast, d, 64));
  wlast = __builtin_amdgcn_readfirstlane(wlast);
  __syncthreads();
  // records to visit: up to the furthest last blend of the tile (clamped to
  // the list length in case the saved state does not match the lists)
  const int nrec = min(smax + 1, (int)(c.re - c.rb));

  for (int bend = nrec; bend > 0; bend -= TG::BATCH) {
    const int bstart = bend > TG::BATCH ? bend - TG::BATCH : 0;
#pragma unroll
    for (int k = 0; k < (TG::BATCH + TG::BLOCK - 1) / TG::BLOCK; ++k) {
      const int slot = (int)threadIdx.x + k * TG::BLOCK;
      if (TG::BATCH % TG::BLOCK != 0 && slot >= TG::BATCH) break;  // wave-uniform
      const int li = bstart + slot;
      uint32_t bits = 0;
      if (li < bend)
        bits = stage<TW, TH, WW, BT>(splats, vbase, pair_ids, c.rb + (uint32_t)li, slot, c, bp,
                                     sh.st, sgid, sh.lmask, nullptr, a.lane_masks);
      publish_masks<TW, TH, WW, BT>(bits, slot >> 6, masks);
    }
    __syncthreads();
    for (int cw = TG::NCH - 1; cw >= 0; --cw) {
      const int lim = wlast - (bstart + cw * 64);  // wave-uniform
      if (lim < 0) continue;  // nothing at or below our last blend
      uint64_t m = uniform_u64(masks[wave][cw]);
      if (lim < 63) m &= (2ull << lim) - 1;  // positions up to wlast
      if constexpr (TG::LM) {
        // drop the chunk's splats whose lane mask holds no pixel that blends
        // at the chunk's first position or later (lane l tests staged splat
        // cw * 64 + l)
        const uint64_t live = __builtin_amdgcn_ballot_w64(bstart + cw * 64 <= lastp);
        m &= __builtin_amdgcn_ballot_w64((sh.lmask[wave * TG::BATCH + cw * 64 + lane] & live) != 0);
      }
      // the chunk's Gaussian ids, one per lane; a splat's id is read from
      // its lane
      const int cgid = (int)sgid[cw * 64 + lane];
      while (m) {
        const int j = 63 - __builtin_clzll(m);
        m &= ~(1ull << j);
        const int r = cw * 64 + j;
        const int pos = bstart + r;
        StagedSplat s;
        StagedForm f;
        StagedRem rm;
        sh.st.get(r, s, f, rm);
        const float dx = s.ur - fx, dy = s.vr - fy;
        float t1, t2, e, al;
        bool cl;
        const bool has = splat_alpha(s, f, dx, dy, bp, t1, t2, e, al, cl) && pos <= lastp;
        // all 16-byte reads are issued before the branch below (left to
        // itself the compiler splits the second half into 4-byte reads inside
        // it, each needing its own address register)
        asm volatile("" ::"v"(s.r), "v"(s.g), "v"(s.b), "v"(s.p0), "v"(s.p1), "v"(s.n0),
                     "v"(s.n1), "v"(s.n2), "v"(rm.ul), "v"(rm.vl));
        if (!__any(has)) continue;
        // Branch-free adjoint: every lane evaluates, lanes without this
        // splat contribute zeros and keep their state (alpha <= alpha_max,
        // so 1 / (1 - alpha) is finite on every lane).
        const float inv = __builtin_amdgcn_rcpf(1.0f - al);
        const float Ti = T * inv;
        const float w = al * Ti;
        const float d = fmaf(s.p1, dy, fmaf(s.p0, dx, s.zc));
        // the offset from the true centre (footprint and plane terms below)
        const float ex = dx + rm.ul, ey = dy + rm.vl;
        // explicit FMAs (the file compiles without contraction so that the
        // alpha decisions above match the forward bit for bit)
        float sf = fmaf(gC0, s.r, gA);
        sf = fmaf(gC1, s.g, sf);
        sf = fmaf(gC2, s.b, sf);
        sf = fmaf(gD, d, sf);
        sf = fmaf(gN0, s.n0, sf);
        sf = fmaf(gN1, s.n1, sf);
        sf = fmaf(gN2, s.n2, sf);
        const float ga = fmaf(Ti, sf, -(Racc * inv));
        T = has ? Ti : T;
        const int gid = __builtin_amdgcn_readlane(cgid, j);
        const float wg = has ? w : 0.0f;
        // lanes without the blend add 0 x sf (sf is finite: a sum of finite
        // products), which leaves Racc unchanged
        Racc = fmaf(wg, sf, Racc);
        float gd = fmaf(wg, gD, (has && gid == med) ? gM : 0.0f);
        if constexpr (DIST) gd = fmaf(kdist * wg, d - mdist, gd);
        // opacity gradient ga e.  Where alpha is not clamped, alpha = o e, so
        // the gradient of the power p = (dx, dy) Q (dx, dy)^T / 2 (Q the
        // conic) is -ga alpha = -o (ga e): the footprint terms below are
        // sums of ga e times the moments 1, dx, dy, dx^2, dx dy, dy^2 of the
        // offset, and the projection backward applies the per-Gaussian
        // factor -o and, for the centre, the conic (d p / d(dx, dy) =
        // Q (dx, dy)^T).
        const float gop = (has && !cl) ? ga * e : 0.0f;
        float g[16];
        // first moments (centre gradient through the footprint; the depth
        // plane's share, p times the summed g[9], is added by the
        // projection backward) and second moments (conic terms)
        const float gpx = gop * ex, gpy = gop * ey;
        g[0] = gpx; g[1] = gpy;
        g[2] = gpx * ex;
        g[3] = gpx * ey;
        g[4] = gpy * ey;
        g[5] = gop;
        g[6] = wg * gC0; g[7] = wg * gC1; g[8] = wg * gC2;
        g[9] = gd;
        g[10] = gd * ex; g[11] = gd * ey;
        g[12] = wg * gN0; g[13] = wg * gN1; g[14] = wg * gN2;
        g[15] = 0.0f;
        {
          const float tot = wave_sum16(g);
          const int vi = lane >> 2;
          if ((lane & 3) == 0 && vi < 15 && tot != 0.0f)
            atomicAdd(gsplat + (vbase + gid) * 16 + vi, tot);
        }
      }
    }
    __syncthreads();
  }
}

// One workgroup per tile, in `order` (or natural) order.
template <int TW, int TH, bool DIST, int WW, int BT>
__global__ void __launch_bounds__(TW * TH) k_render_bwd(BwdArgs a) {
  __shared__ BwdShared<TW, TH, WW, BT> sh;
  const int64_t i = blockIdx.x;
  bwd_tile<TW, TH, DIST, WW, BT>(a, a.order ? (int64_t)a.order[i] : i, sh);
}

// Persistent workgroups over a device work queue (see k_render_fwd_persistent).
template <int TW, int TH, bool DIST, int WW, int BT>
__global__ void __launch_bounds__(TW * TH) k_render_bwd_persistent(BwdArgs a) {
  __shared__ BwdShared<TW, TH, WW, BT> sh;
  __shared__ uint32_t item_s;
  for (;;) {
    if (threadIdx.x == 0) item_s = atomicAdd(a.queue, 1u);
    __syncthreads();
    const uint32_t item = item_s;
    __syncthreads();
    if ((int64_t)item >= a.tiles) break;
    bwd_tile<TW, TH, DIST, WW, BT>(a, a.order ? (int64_t)a.order[item] : (int64_t)item, sh);
  }
}

// Clears n4 16-byte words (grid-stride, one 16-byte store per iteration).
constexpr int kZeroThreads = 256;
constexpr int64_t kZeroBlocks = 4096;
__global__ void __launch_bounds__(kZeroThreads) k_zero(float4* __restrict__ a, int64_t n4) {
  for (int64_t i = (int64_t)blockIdx.x * kZeroThreads + threadIdx.x; i < n4;
       i += (int64_t)gridDim.x * kZeroThreads)
    a[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

__global__ void k_zero_u32(uint32_t* __restrict__ a) { *a = 0u; }

template <int TW, int TH, bool DIST, bool CNT, bool EXACT, int WW = 8, int BT = 0>
void launch_fwd_d(const FwdArgs& a, int schedule, hipStream_t st) {
  constexpr int B = TileGeom<TW, TH, WW, BT>::BLOCK;
  if (schedule == RADE_SCHEDULE_PERSISTENT) {
    static unsigned cached = 0;
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, st, a.queue);
    const unsigned g = resident_blocks(k_render_fwd_persistent<TW, TH, DIST, CNT, EXACT, WW, BT>,
                                       B, (unsigned)a.tiles, cached);
    hipLaunchKernelGGL((k_render_fwd_persistent<TW, TH, DIST, CNT, EXACT, WW, BT>), dim3(g),
                       dim3(B), 0, st, a);
  } else {
    hipLaunchKernelGGL((k_render_fwd<TW, TH, DIST, CNT, EXACT, WW, BT>),
                       dim3((unsigned)a.tiles), dim3(B), 0, st, a);
  }
}

template <int TW, int TH, bool EXACT>
void launch_fwd_e(const FwdArgs& a, int schedule, hipStream_t st) {
  const bool cnt = a.count || a.evals;
  if (a.distortion) {
    if (cnt) launch_fwd_d<TW, TH, true, true, EXACT>(a, schedule, st);
    else launch_fwd_d<TW, TH, true, false, EXACT>(a, schedule, st);
  } else {
    if (cnt) launch_fwd_d<TW, TH, false, true, EXACT>(a, schedule, st);
    else launch_fwd_d<TW, TH, false, false, EXACT>(a, schedule, st);
  }
}

template <int TW, int TH, bool DIST, int WW = 8, int BT = 0>
void launch_bwd_d(const BwdArgs& a, int schedule, hipStream_t st) {
  constexpr int B = TileGeom<TW, TH, WW, BT>::BLOCK;
  if (schedule == RADE_SCHEDULE_PERSISTENT) {
    static unsigned cached = 0;
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, st, a.queue);
    const unsigned g = resident_blocks(k_render_bwd_persistent<TW, TH, DIST, WW, BT>, B,
                                       (unsigned)a.tiles, cached);
    hipLaunchKernelGGL((k_render_bwd_persistent<TW, TH, DIST, WW, BT>), dim3(g), dim3(B), 0, st,
                       a);
  } else {
    hipLaunchKernelGGL((k_render_bwd<TW, TH, DIST, WW, BT>), dim3((unsigned)a.tiles), dim3(B), 0,
                       st, a);
  }
}

// Wave shapes and batches other than the default (8x8 waves, one splat per
// thread) are compiled for the plain forward and backward only (no
// distortion, blend count or exact depth); the caller checks this.
constexpr bool shape_fits(int tw, int th, int ww) { return tw % ww == 0 && th % (64 / ww) == 0; }

// Tiles of several 8x8 waves with lane masks on each (lane_masks = 1).
inline bool lane_mask_shape(int tw, int th, int wave_w, int batch, int lane_masks) {
  return lane_masks == 1 && (wave_w == 0 || wave_w == 8) && batch == 0 && tw * th > 64;
}

inline bool default_shape(int tw, int th, int wave_w, int batch) {
  return (wave_w == 0 || wave_w == 8) && (batch == 0 || batch == tw * th);
}

template <int TW, int TH, int WW>
bool launch_fwd_shape_b(const FwdArgs& a, int schedule, int batch, hipStream_t st) {
  if constexpr (shape_fits(TW, TH, WW)) {
    switch (batch) {
      case 0: launch_fwd_d<TW, TH, false, false, false, WW, 0>(a, schedule, st); return true;
      case 64: launch_fwd_d<TW, TH, false, false, false, WW, 64>(a, schedule, st); return true;
      case 128: launch_fwd_d<TW, TH, false, false, false, WW, 128>(a, schedule, st); return true;
      case 256: launch_fwd_d<TW, TH, false, false, false, WW, 256>(a, schedule, st); return true;
      default: return false;
    }
  }
  return false;
}

template <int TW, int TH, int WW>
bool launch_bwd_shape_b(const BwdArgs& a, int schedule, int batch, hipStream_t st) {
  if constexpr (shape_fits(TW, TH, WW)) {
    switch (batch) {
      case 0: launch_bwd_d<TW, TH, false, WW, 0>(a, schedule, st); return true;
      case 64: launch_bwd_d<TW, TH, false, WW, 64>(a, schedule, st); return true;
      case 128: launch_bwd_d<TW, TH, false, WW, 128>(a, schedule, st); return true;
      case 256: launch_bwd_d<TW, TH, false, WW, 256>(a, schedule, st); return true;
      default: return false;
    }
  }
  return false;
}

template <int TW, int TH>
hipError_t launch_fwd_t(const FwdArgs& a, int schedule, int wave_w, int batch, int lane_masks,
                        hipStream_t st) {
  EventScope timing(RADE_KERNEL_RENDER_FWD, st);
  if (lane_mask_shape(TW, TH, wave_w, batch, lane_masks)) {
    if (a.depth_quad || a.distortion || a.count || a.evals) return hipErrorInvalidValue;
    if constexpr (TW * TH > 64)
      launch_fwd_d<TW, TH, false, false, false, 8, kLaneMaskBatch>(a, schedule, st);
    return hipSuccess;
  }
  if (default_shape(TW, TH, wave_w, batch)) {
    if (a.depth_quad) launch_fwd_e<TW, TH, true>(a, schedule, st);
    else launch_fwd_e<TW, TH, false>(a, schedule, st);
    return hipSuccess;
  }
  if (a.depth_quad || a.distortion || a.count || a.evals) return hipErrorInvalidValue;
  bool ok = false;
  if (wave_w == 0 || wave_w == 8) ok = launch_fwd_shape_b<TW, TH, 8>(a, schedule, batch, st);
  else if (wave_w == 16) ok = launch_fwd_shape_b<TW, TH, 16>(a, schedule, batch, st);
  else if (wave_w == 32) ok = launch_fwd_shape_b<TW, TH, 32>(a, schedule, batch, st);
  return ok ? hipSuccess : hipErrorInvalidValue;
}

template <int TW, int TH>
hipError_t launch_bwd_t(const BwdArgs& a, int schedule, int wave_w, int batch, int lane_masks,
                        hipStream_t st) {
  EventScope timing(RADE_KERNEL_RENDER_BWD, st);
  if (lane_mask_shape(TW, TH, wave_w, batch, lane_masks)) {
    if (a.d_distortion) return hipErrorInvalidValue;
    if constexpr (TW * TH > 64) launch_bwd_d<TW, TH, false, 8, kLaneMaskBatch>(a, schedule, st);
    return hipSuccess;
  }
  if (default_shape(TW, TH, wave_w, batch)) {
    if (a.d_distortion) launch_bwd_d<TW, TH, true>(a, schedule, st);
    else launch_bwd_d<TW, TH, false>(a, schedule, st);
    return hipSuccess;
  }
  if (a.d_distortion) return hipErrorInvalidValue;
  bool ok = false;
  if (wave_w == 0 || wave_w == 8) ok = launch_bwd_shape_b<TW, TH, 8>(a, schedule, batch, st);
  else if (wave_w == 16) ok = launch_bwd_shape_b<TW, TH, 16>(a, schedule, batch, st);
  else if (wave_w == 32) ok = launch_bwd_shape_b<TW, TH, 32>(a, schedule, batch, st);
  return ok ? hipSuccess : hipErrorInvalidValue;
}

}  // namespace

// Wave shapes a tile can hold: ww x (64 / ww) blocks tiling it exactly.
bool wave_shape_supported(int tw, int th, int wave_w) {
  const int ww = wave_w > 0 ? wave_w : 8;
  if (ww != 8 && ww != 16 && ww != 32) return false;
  return shape_fits(tw, th, ww);
}

// 64-bit lane masks per pair that the forward can store for the backward:
// one per 8x8 wave of the tile where the launch shape keeps lane masks (8x8
// tiles of 8x8 waves, or lane_masks on larger ones), else none.
int lane_masks_per_pair(int tw, int th, int wave_w, int batch, int lane_masks) {
  if (lane_mask_shape(tw, th, wave_w, batch, lane_masks)) return (tw / 8) * (th / 8);
  if (tw == 8 && th == 8 && (wave_w == 0 || wave_w == 8)) return 1;
  return 0;
}

bool render_shape_is_default(int tw, int th, int wave_w, int batch, int lane_masks) {
  return default_shape(tw, th, wave_w, batch) &&
         !lane_mask_shape(tw, th, wave_w, batch, lane_masks);
}

bool tile_supported(int tw, int th) {
  return (tw == 8 && th == 8) || (tw == 16 && th == 16) || (tw == 16 && th == 32) ||
         (tw == 32 && th == 16) || (tw == 16 && th == 8) || (tw == 8 && th == 16);
}

#define RADE_TILE_DISPATCH(FN, ARGS)                                     \
  hipError_t de = hipErrorInvalidValue;                                  \
  if (s.tile_w == 8 && s.tile_h == 8) de = FN<8, 8> ARGS;                \
  else if (s.tile_w == 16 && s.tile_h == 16) de = FN<16, 16> ARGS;       \
  else if (s.tile_w == 16 && s.tile_h == 32) de = FN<16, 32> ARGS;       \
  else if (s.tile_w == 32 && s.tile_h == 16) de = FN<32, 16> ARGS;       \
  else if (s.tile_w == 16 && s.tile_h == 8) de = FN<16, 8> ARGS;         \
  else if (s.tile_w == 8 && s.tile_h == 16) de = FN<8, 16> ARGS;         \
  if (de != hipSuccess) return de;

hipError_t launch_render_fwd(const rade_settings& s, const rade_view* views, int V, int64_t N,
                             int64_t tiles, const rade_splat* splats, const uint32_t* ids,
                             const uint32_t* ranges, const uint32_t* order, float* color,
                             float* depth, float* normal, float* alpha, float* tf,
                             int32_t* last, int32_t* med, int32_t* cnt, int32_t* evals,
                             float* distortion, const float* depth_quad, uint64_t* lane_masks,
                             hipStream_t st) {
  if (tiles == 0) return hipSuccess;
  FwdArgs a;
  a.bp = make_blend_params(s);
  a.views = views; a.V = V; a.N = N; a.tiles = tiles;
  a.splats = splats; a.pair_ids = ids; a.ranges = ranges;
  a.order = s.schedule == RADE_SCHEDULE_TILE ? nullptr : order;
  a.queue = order ? const_cast<uint32_t*>(order) + tiles : nullptr;
  a.color = color; a.depth = depth; a.normal = normal; a.alpha = alpha; a.t_final = tf;
  a.last = last; a.median = med; a.count = cnt; a.evals = evals; a.distortion = distortion;
  a.depth_quad = reinterpret_cast<const float4*>(depth_quad);
  a.lane_masks = lane_masks;
  RADE_TILE_DISPATCH(launch_fwd_t, (a, s.schedule, s.wave_w, s.batch, s.lane_masks, st))
  return hipGetLastError();
}

hipError_t launch_render_bwd(const rade_settings& s, const rade_view* views, int V, int64_t N,
                             int64_t tiles, const rade_splat* splats, const uint32_t* ids,
                             const uint32_t* ranges, const uint32_t* order, const float* tf,
                             const int32_t* last, const int32_t* med, const float* dc,
                             const float* dd, const float* dn, const float* da,
                             const float* ddist, const float* fwd_depth, const float* fwd_alpha,
                             float* gsplat, const uint64_t* lane_masks, hipStream_t st) {
  const int64_t ng4 = (int64_t)V * N * 4;  // 16 floats per (view, Gaussian)
  if (ng4 > 0) {
    const int64_t blocks = (ng4 + kZeroThreads - 1) / kZeroThreads;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)(blocks < kZeroBlocks ? blocks : kZeroBlocks)),
                       dim3(kZeroThreads), 0, st, reinterpret_cast<float4*>(gsplat), ng4);
  }
  if (tiles == 0) return hipGetLastError();
  BwdArgs a;
  a.bp = make_blend_params(s);
  a.views = views; a.V = V; a.N = N; a.tiles = tiles;
  a.splats = splats; a.pair_ids = ids; a.ranges = ranges;
  a.order = s.schedule == RADE_SCHEDULE_TILE ? nullptr : order;
  a.queue = order ? const_cast<uint32_t*>(order) + tiles : nullptr;
  a.t_final = tf; a.last = last; a.median = med;
  a.d_color = dc; a.d_depth = dd; a.d_normal = dn; a.d_alpha = da;
  a.d_distortion = ddist; a.fwd_depth = fwd_depth; a.fwd_alpha = fwd_alpha;
  a.gsplat = gsplat;
  a.lane_masks = lane_masks;
  RADE_TILE_DISPATCH(launch_bwd_t, (a, s.schedule, s.wave_w, s.batch, s.lane_masks, st))
  return hipGetLastError();
}

}  // namespace rade
