// Tile rasterizer: forward blending and its adjoint (gfx950).
//
// One workgroup per screen tile; each wavefront owns an 8x8 block of pixels
// of the tile and each lane one pixel.  The tile's list of splats (depth
// order) is walked in batches: every thread stages one splat into LDS (its
// centre made tile-relative in FP64 before rounding to FP32), and tests the
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
// Backward, per pixel, back to front from the last blended splat, with the
// transmittance recovered as T_i = T_{i+1} / (1 - alpha_i) from the saved
// final T (nothing per blend is stored) and the running sum R of what lies
// behind:  dL/dalpha_i = T_i s_i - R / (1 - alpha_i),  R += w_i s_i, where
// s_i = g_C . rgb_i + g_D d_i + g_N . n_i + g_A.  The 15 per-splat gradients
// are summed over the wavefront with a transpose-reduction and added with
// hardware FP32 atomics into a per-(view, Gaussian) record.
#include "common.hpp"

namespace rade {
namespace {

template <int TW, int TH>
struct TileGeom {
  static constexpr int NWX = TW / 8;
  static constexpr int NWY = TH / 8;
  static constexpr int NW = NWX * NWY;
  static constexpr int BLOCK = 64 * NW;
  static_assert(TW % 8 == 0 && TH % 8 == 0 && BLOCK <= 1024, "tile");
};

struct PixelCtx {
  int v;
  int64_t tile;
  int x0, y0;
  int lxi, lyi, px, py;
  bool inside;
  int64_t P, poff, pix;
  uint32_t rb, re;
};

template <int TW, int TH>
__device__ __forceinline__ PixelCtx pixel_ctx(const rade_view* views, int V,
                                              const uint32_t* ranges) {
  using TG = TileGeom<TW, TH>;
  PixelCtx c;
  c.tile = blockIdx.x;
  c.v = view_of_tile(views, V, c.tile);
  const rade_view& vw = views[c.v];
  const int64_t lt = c.tile - vw.tile_offset;
  const int tx = (int)(lt % vw.tiles_x), ty = (int)(lt / vw.tiles_x);
  c.x0 = tx * TW;
  c.y0 = ty * TH;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  c.lxi = 8 * (wave % TG::NWX) + (lane & 7);
  c.lyi = 8 * (wave / TG::NWX) + (lane >> 3);
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

// Stage splat `idx` of the tile list into LDS slot threadIdx.x and return
// the bit set of 8x8 blocks its support rect touches.
template <int TW, int TH>
__device__ __forceinline__ uint32_t stage(const rade_splat* __restrict__ splats, int64_t vbase,
                                          const uint32_t* __restrict__ pair_ids, uint32_t idx,
                                          const PixelCtx& c, StagedSplat* ss, uint32_t* sgid) {
  using TG = TileGeom<TW, TH>;
  const uint32_t g = pair_ids[idx];
  const rade_splat& sp = splats[vbase + g];
  StagedSplat s;
  s.ur = (float)(sp.uc - ((double)c.x0 + 0.5));
  s.vr = (float)(sp.vc - ((double)c.y0 + 0.5));
  s.w0 = sp.w[0]; s.w1 = sp.w[1]; s.w2 = sp.w[2]; s.w3 = sp.w[3];
  s.o = sp.opacity; s.z = sp.z;
  s.r = sp.rgb[0]; s.g = sp.rgb[1]; s.b = sp.rgb[2];
  s.p0 = sp.p[0]; s.p1 = sp.p[1];
  s.n0 = sp.n[0]; s.n1 = sp.n[1]; s.n2 = sp.n[2];
  ss[threadIdx.x] = s;
  sgid[threadIdx.x] = g;
  const int rx0 = sp.rect[0] - c.x0, rx1 = sp.rect[1] - c.x0;
  const int ry0 = sp.rect[2] - c.y0, ry1 = sp.rect[3] - c.y0;
  uint32_t bits = 0;
#pragma unroll
  for (int k = 0; k < TG::NW; ++k) {
    const int bx = 8 * (k % TG::NWX), by = 8 * (k / TG::NWX);
    if (rx0 <= bx + 7 && rx1 >= bx && ry0 <= by + 7 && ry1 >= by) bits |= 1u << k;
  }
  return bits;
}

template <int TW, int TH>
__device__ __forceinline__ void publish_masks(uint32_t bits, uint64_t (*masks)[TileGeom<TW, TH>::NW]) {
  using TG = TileGeom<TW, TH>;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int k = 0; k < TG::NW; ++k) {
    const uint64_t m = __ballot((bits >> k) & 1u);
    if (lane == 0) masks[k][wave] = m;
  }
}

template <int TW, int TH>
__global__ void __launch_bounds__(TW * TH)
k_render_fwd(BlendParams bp, const rade_view* __restrict__ views, int V, int64_t N,
             const rade_splat* __restrict__ splats, const uint32_t* __restrict__ pair_ids,
             const uint32_t* __restrict__ ranges, float* __restrict__ color,
             float* __restrict__ depth, float* __restrict__ normal, float* __restrict__ alpha,
             float* __restrict__ t_final, int32_t* __restrict__ last,
             int32_t* __restrict__ median, int32_t* __restrict__ count) {
  using TG = TileGeom<TW, TH>;
  __shared__ StagedSplat ss[TG::BLOCK];
  __shared__ uint32_t sgid[TG::BLOCK];
  __shared__ uint64_t masks[TG::NW][TG::NW];
  const PixelCtx c = pixel_ctx<TW, TH>(views, V, ranges);
  const int wave = threadIdx.x >> 6;
  const int64_t vbase = (int64_t)c.v * N;
  const float fx = (float)c.lxi, fy = (float)c.lyi;

  float T = 1.0f, C0 = 0.f, C1 = 0.f, C2 = 0.f, D = 0.f, N0 = 0.f, N1 = 0.f, N2 = 0.f, A = 0.f;
  float dmed = 0.f;
  int cnt = 0, lastp = -1, medp = -1;
  bool done = !c.inside;

  for (uint32_t b0 = c.rb; b0 < c.re; b0 += TG::BLOCK) {
    if (__syncthreads_and(done ? 1 : 0)) break;
    const uint32_t idx = b0 + threadIdx.x;
    uint32_t bits = 0;
    if (idx < c.re) bits = stage<TW, TH>(splats, vbase, pair_ids, idx, c, ss, sgid);
    publish_masks<TW, TH>(bits, masks);
    __syncthreads();
    bool wave_live = !__all(done);
    for (int cw = 0; cw < TG::NW && wave_live; ++cw) {
      uint64_t m = masks[wave][cw];
      while (m) {
        const int j = __builtin_ctzll(m);
        m &= m - 1;
        const int r = cw * 64 + j;
        const StagedSplat s = ss[r];
        const float dx = s.ur - fx, dy = s.vr - fy;
        float t1, t2, e, al;
        bool cl;
        if (!done && splat_alpha(s, dx, dy, bp, t1, t2, e, al, cl)) {
          const float Tn = T * (1.0f - al);
          if (Tn < bp.t_min) {
            done = true;
          } else {
            const float w = al * T;
            const float d = fmaf(s.p1, dy, fmaf(s.p0, dx, s.z));
            C0 = fmaf(w, s.r, C0); C1 = fmaf(w, s.g, C1); C2 = fmaf(w, s.b, C2);
            D = fmaf(w, d, D);
            N0 = fmaf(w, s.n0, N0); N1 = fmaf(w, s.n1, N1); N2 = fmaf(w, s.n2, N2);
            A += w;
            const int pos = (int)(b0 - c.rb) + r;
            if (T > 0.5f) { medp = pos; dmed = d; }
            lastp = pos;
            ++cnt;
            T = Tn;
          }
        }
        if (__all(done)) { wave_live = false; break; }
      }
    }
    __syncthreads();
  }
  if (!c.inside) return;
  C0 = fmaf(T, bp.bg[0], C0); C1 = fmaf(T, bp.bg[1], C1); C2 = fmaf(T, bp.bg[2], C2);
  const int64_t P = c.P, pix = c.pix;
  color[3 * c.poff + pix] = C0;
  color[3 * c.poff + P + pix] = C1;
  color[3 * c.poff + 2 * P + pix] = C2;
  depth[2 * c.poff + pix] = D;
  depth[2 * c.poff + P + pix] = medp >= 0 ? dmed : 0.0f;
  normal[3 * c.poff + pix] = N0;
  normal[3 * c.poff + P + pix] = N1;
  normal[3 * c.poff + 2 * P + pix] = N2;
  alpha[c.poff + pix] = A;
  t_final[c.poff + pix] = T;
  last[c.poff + pix] = lastp;
  median[c.poff + pix] = medp >= 0 ? (int32_t)pair_ids[c.rb + medp] : -1;
  if (count) count[c.poff + pix] = cnt;
}

// Sum 16 per-lane values over the wavefront.  On return lane l holds the
// total of value index ((l>>5)&1)*8 + ((l>>4)&1)*4 + ((l>>3)&1)*2 + ((l>>2)&1).
__device__ __forceinline__ float wave_transpose_sum16(float (&v)[16]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int half = 8, mask = 32; half >= 1; half >>= 1, mask >>= 1) {
    const bool up = lane & mask;
#pragma unroll
    for (int k = 0; k < half; ++k) {
      const float send = up ? v[k] : v[k + half];
      const float keep = up ? v[k + half] : v[k];
      v[k] = keep + __shfl_xor(send, mask, 64);
    }
  }
  float s = v[0];
  s += __shfl_xor(s, 2, 64);
  s += __shfl_xor(s, 1, 64);
  return s;
}

constexpr float kTwoOverLog2e = 2.0f / kLog2e;

template <int TW, int TH>
__global__ void __launch_bounds__(TW * TH)
k_render_bwd(BlendParams bp, const rade_view* __restrict__ views, int V, int64_t N,
             const rade_splat* __restrict__ splats, const uint32_t* __restrict__ pair_ids,
             const uint32_t* __restrict__ ranges, const float* __restrict__ t_final,
             const int32_t* __restrict__ last, const int32_t* __restrict__ median,
             const float* __restrict__ d_color, const float* __restrict__ d_depth,
             const float* __restrict__ d_normal, const float* __restrict__ d_alpha,
             float* __restrict__ gsplat) {
  using TG = TileGeom<TW, TH>;
  __shared__ StagedSplat ss[TG::BLOCK];
  __shared__ uint32_t sgid[TG::BLOCK];
  __shared__ uint64_t masks[TG::NW][TG::NW];
  __shared__ int smax;
  const PixelCtx c = pixel_ctx<TW, TH>(views, V, ranges);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t vbase = (int64_t)c.v * N;
  const float fx = (float)c.lxi, fy = (float)c.lyi;

  float T = 0.f, gC0 = 0.f, gC1 = 0.f, gC2 = 0.f, gD = 0.f, gM = 0.f;
  float gN0 = 0.f, gN1 = 0.f, gN2 = 0.f, gA = 0.f;
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
  }
  float Racc = T * (gC0 * bp.bg[0] + gC1 * bp.bg[1] + gC2 * bp.bg[2]);

  if (threadIdx.x == 0) smax = -1;
  __syncthreads();
  atomicMax(&smax, lastp);
  int wlast = lastp;
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) wlast = max(wlast, __shfl_xor(wlast, d, 64));
  __syncthreads();
  // records to visit: up to the furthest last blend of the tile (clamped to
  // the list length in case the saved state does not match the lists)
  const int nrec = min(smax + 1, (int)(c.re - c.rb));

  for (int bend = nrec; bend > 0; bend -= TG::BLOCK) {
    const int bstart = bend > TG::BLOCK ? bend - TG::BLOCK : 0;
    const int li = bstart + (int)threadIdx.x;
    uint32_t bits = 0;
    if (li < bend) bits = stage<TW, TH>(splats, vbase, pair_ids, c.rb + (uint32_t)li, c, ss, sgid);
    publish_masks<TW, TH>(bits, masks);
    __syncthreads();
    for (int cw = TG::NW - 1; cw >= 0; --cw) {
      if (bstart + cw * 64 > wlast) continue;  // wave-uniform: nothing at or below our last
      uint64_t m = masks[wave][cw];
      while (m) {
        const int j = 63 - __builtin_clzll(m);
        m &= ~(1ull << j);
        const int r = cw * 64 + j;
        const int pos = bstart + r;
        if (pos > wlast) continue;
        const StagedSplat s = ss[r];
        const float dx = s.ur - fx, dy = s.vr - fy;
        float t1, t2, e, al;
        bool cl;
        float g[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) g[k] = 0.f;
        bool has = false;
        if (pos <= lastp && splat_alpha(s, dx, dy, bp, t1, t2, e, al, cl)) {
          has = true;
          const float inv = __builtin_amdgcn_rcpf(1.0f - al);
          T = T * inv;
          const float w = al * T;
          const float d = fmaf(s.p1, dy, fmaf(s.p0, dx, s.z));
          const float sf = gC0 * s.r + gC1 * s.g + gC2 * s.b + gD * d + gN0 * s.n0 +
                           gN1 * s.n1 + gN2 * s.n2 + gA;
          const float ga = T * sf - Racc * inv;
          Racc = fmaf(w, sf, Racc);
          const float gd = w * gD + ((int)sgid[r] == med ? gM : 0.0f);
          const float gp = cl ? 0.0f : -ga * al;
          const float dpdx = (t1 * s.w0 + t2 * s.w2) * kTwoOverLog2e;
          const float dpdy = (t1 * s.w1 + t2 * s.w3) * kTwoOverLog2e;
          g[0] = gp * dpdx + gd * s.p0;
          g[1] = gp * dpdy + gd * s.p1;
          g[2] = 0.5f * gp * dx * dx;
          g[3] = gp * dx * dy;
          g[4] = 0.5f * gp * dy * dy;
          g[5] = cl ? 0.0f : ga * e;
          g[6] = w * gC0; g[7] = w * gC1; g[8] = w * gC2;
          g[9] = gd;
          g[10] = gd * dx; g[11] = gd * dy;
          g[12] = w * gN0; g[13] = w * gN1; g[14] = w * gN2;
        }
        if (__any(has)) {
          const float tot = wave_transpose_sum16(g);
          const int vi = ((lane >> 5) & 1) * 8 + ((lane >> 4) & 1) * 4 + ((lane >> 3) & 1) * 2 +
                         ((lane >> 2) & 1);
          if ((lane & 3) == 0 && vi < 15 && tot != 0.0f)
            atomicAdd(gsplat + (vbase + sgid[r]) * 16 + vi, tot);
        }
      }
    }
    __syncthreads();
  }
}

__global__ void k_zero(float* __restrict__ a, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0.0f;
}

template <int TW, int TH>
void launch_fwd_t(const BlendParams& bp, const rade_view* views, int V, int64_t N,
                  int64_t tiles, const rade_splat* splats, const uint32_t* ids,
                  const uint32_t* ranges, float* color, float* depth, float* normal,
                  float* alpha, float* tf, int32_t* last, int32_t* med, int32_t* cnt,
                  hipStream_t st) {
  EventScope timing(RADE_KERNEL_RENDER_FWD, st);
  hipLaunchKernelGGL((k_render_fwd<TW, TH>), dim3((unsigned)tiles),
                     dim3(TileGeom<TW, TH>::BLOCK), 0, st, bp, views, V, N, splats, ids, ranges,
                     color, depth, normal, alpha, tf, last, med, cnt);
}

template <int TW, int TH>
void launch_bwd_t(const BlendParams& bp, const rade_view* views, int V, int64_t N,
                  int64_t tiles, const rade_splat* splats, const uint32_t* ids,
                  const uint32_t* ranges, const float* tf, const int32_t* last,
                  const int32_t* med, const float* dc, const float* dd, const float* dn,
                  const float* da, float* gs, hipStream_t st) {
  EventScope timing(RADE_KERNEL_RENDER_BWD, st);
  hipLaunchKernelGGL((k_render_bwd<TW, TH>), dim3((unsigned)tiles),
                     dim3(TileGeom<TW, TH>::BLOCK), 0, st, bp, views, V, N, splats, ids, ranges,
                     tf, last, med, dc, dd, dn, da, gs);
}

}  // namespace

bool tile_supported(int tw, int th) {
  return (tw == 8 && th == 8) || (tw == 16 && th == 16) || (tw == 16 && th == 32) ||
         (tw == 32 && th == 16) || (tw == 16 && th == 8) || (tw == 8 && th == 16);
}

hipError_t launch_render_fwd(const rade_settings& s, const rade_view* views, int V, int64_t N,
                             int64_t tiles, const rade_splat* splats, const uint32_t* ids,
                             const uint32_t* ranges, float* color, float* depth,
                             float* normal, float* alpha, float* tf, int32_t* last,
                             int32_t* med, int32_t* cnt, hipStream_t st) {
  if (tiles == 0) return hipSuccess;
  const BlendParams bp = make_blend_params(s);
#define RADE_FWD(TW, TH)                                                                      \
  if (s.tile_w == TW && s.tile_h == TH) {                                                     \
    launch_fwd_t<TW, TH>(bp, views, V, N, tiles, splats, ids, ranges, color, depth, normal, \
                         alpha, tf, last, med, cnt, st);                                      \
    return hipGetLastError();                                                                 \
  }
  RADE_FWD(8, 8)
  RADE_FWD(16, 16)
  RADE_FWD(16, 32)
  RADE_FWD(32, 16)
  RADE_FWD(16, 8)
  RADE_FWD(8, 16)
#undef RADE_FWD
  return hipErrorInvalidValue;
}

hipError_t launch_render_bwd(const rade_settings& s, const rade_view* views, int V, int64_t N,
                             int64_t tiles, const rade_splat* splats, const uint32_t* ids,
                             const uint32_t* ranges, const float* tf, const int32_t* last,
                             const int32_t* med, const float* dc, const float* dd,
                             const float* dn, const float* da, float* gsplat,
                             hipStream_t st) {
  const int64_t ng = (int64_t)V * N * 16;
  if (ng > 0)
    hipLaunchKernelGGL(k_zero, dim3((unsigned)((ng + 255) / 256)), dim3(256), 0, st, gsplat, ng);
  if (tiles == 0) return hipGetLastError();
  const BlendParams bp = make_blend_params(s);
#define RADE_BWD(TW, TH)                                                                    \
  if (s.tile_w == TW && s.tile_h == TH) {                                                   \
    launch_bwd_t<TW, TH>(bp, views, V, N, tiles, splats, ids, ranges, tf, last, med, dc, dd, \
                         dn, da, gsplat, st);                                               \
    return hipGetLastError();                                                               \
  }
  RADE_BWD(8, 8)
  RADE_BWD(16, 16)
  RADE_BWD(16, 32)
  RADE_BWD(32, 16)
  RADE_BWD(16, 8)
  RADE_BWD(8, 16)
#undef RADE_BWD
  return hipErrorInvalidValue;
}

}  // namespace rade
