// Binning of splats into screen tiles and the sort that orders each tile's
// list by depth (gfx950).
//
// RaDe-GS blends splats in the order of their centre depth (Sec. 3.1, the
// sort before Eq. 3).  Each tile's list must hold every splat whose support
// rect touches the tile, ordered by (float32 depth, Gaussian id).  Instead of
// one long radix sort over (tile, depth) 64-bit keys, the visible splats are
// first sorted by depth (V*N items, 4 passes of 8 bits), then their pairs are
// emitted in that order and stably sorted by tile (M items, ceil(log2 T)/8
// passes).  Both sorts are stable, so the result equals the stable sort of
// the 64-bit keys (tile << 32 | bits(z)) over pairs emitted in Gaussian
// order, at a fraction of the passes over the (larger) pair array.
//
// All item counts that depend on the data live in device memory; every
// kernel is launched with a grid sized for the capacity and its surplus
// blocks exit, so the whole sequence can be captured in a HIP graph.
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "scan.hpp"

namespace rade {
namespace {

constexpr int kThreads = kScanThreads;
constexpr int kItems = kScanItems;              // items per thread
constexpr int kTile = kScanTile;                // items per block (2048)
constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;

// Inputs of the scans, as functors over the item index.
struct FlagInput {  // 1 when the splat touches at least one tile
  const int32_t* tt;
  __device__ uint32_t operator()(int64_t i) const { return tt[i] > 0 ? 1u : 0u; }
};
struct GatherCount {  // tiles touched by the j-th depth-sorted splat
  const int32_t* tt;
  const uint32_t* vals;
  __device__ uint64_t operator()(int64_t j) const { return (uint64_t)tt[vals[j]]; }
};

// ---------------------------------------------------------------------------
// Compaction of visible splats with their depth keys.
__global__ void __launch_bounds__(kThreads)
k_compact(const int32_t* __restrict__ tt, const uint32_t* __restrict__ pos,
          const rade_splat* __restrict__ splats, int64_t n, uint32_t* __restrict__ keys,
          uint32_t* __restrict__ vals) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= n || tt[i] <= 0) return;
  const uint32_t p = pos[i];
  keys[p] = __float_as_uint(splats[i].z);  // z > near > 0: bits order like values
  vals[p] = (uint32_t)i;
}

// ---------------------------------------------------------------------------
// LSD radix sort pass, 8-bit digit at `shift`, stable.
__device__ __forceinline__ uint32_t digit_of(uint32_t k, int shift) {
  return (k >> shift) & (kRadix - 1);
}

__global__ void __launch_bounds__(kThreads)
k_radix_hist(const uint32_t* __restrict__ keys, const uint32_t* __restrict__ n_dev,
             int shift, int64_t nblocks, uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[kRadix];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t n = *n_dev;
  const int64_t base = (int64_t)blockIdx.x * kTile;
#pragma unroll
  for (int r = 0; r < kItems; ++r) {
    const int64_t i = base + (int64_t)r * kThreads + threadIdx.x;
    if (i < n) atomicAdd(&h[digit_of(keys[i], shift)], 1u);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// Exclusive scan of one digit's row of per-block counts (one workgroup per
// digit, rows are digit-major) and the digit's total.  Together with the
// scan of the 256 totals in the scatter's prologue this replaces a global
// scan of the whole count matrix.
__global__ void __launch_bounds__(kThreads)
k_radix_colscan(uint32_t* __restrict__ hist, int64_t nblocks, uint32_t* __restrict__ dtot) {
  __shared__ uint32_t lw[kThreads / 64];
  uint32_t* row = hist + (int64_t)blockIdx.x * nblocks;
  uint32_t carry = 0;
  for (int64_t b0 = 0; b0 < nblocks; b0 += kTile) {  // uniform trip count
    const int64_t base = b0 + (int64_t)threadIdx.x * kItems;
    uint32_t v[kItems], s = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
      v[k] = base + k < nblocks ? row[base + k] : 0u;
      s += v[k];
    }
    uint32_t tot;
    uint32_t run = carry + block_exclusive_scan<uint32_t>(s, lw, tot);
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
      if (base + k < nblocks) row[base + k] = run;
      run += v[k];
    }
    carry += tot;
  }
  if (threadIdx.x == 0) dtot[blockIdx.x] = carry;
}

// Shared memory of one sorting workgroup.
struct RankShared {
  uint32_t cnt[kRadix];                  // per-digit count of the tile
  uint32_t wcnt[kThreads / 64][kRadix];  // per-round per-wave counts
  uint32_t lstart[kRadix];               // first local position of each digit
  uint32_t dbase[kRadix];                // global position of each digit's run
  uint32_t skey[kTile];
  uint32_t sval[kTile];
  uint32_t lw[kThreads / 64];
};

// Stable ranks of the tile's items [base, min(base + kTile, n)) among equal
// digits (wave match masks: 8 ballots per item), the per-digit counts in
// sh.cnt and the local digit starts in sh.lstart.  On return the items sit
// in key/val with their local sorted positions in pos.
__device__ __forceinline__ void rank_tile(const uint32_t* __restrict__ kin,
                                          const uint32_t* __restrict__ vin, int64_t base,
                                          int64_t n, int shift, RankShared& sh,
                                          uint32_t (&key)[kItems], uint32_t (&val)[kItems],
                                          uint32_t (&pos)[kItems]) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  sh.cnt[threadIdx.x] = 0;
#pragma unroll
  for (int w = 0; w < kThreads / 64; ++w) sh.wcnt[w][threadIdx.x] = 0;
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kItems; ++r) {
    const int64_t i = base + (int64_t)r * kThreads + threadIdx.x;
    const bool valid = i < n;
    key[r] = valid ? kin[i] : 0u;
    val[r] = valid ? vin[i] : 0u;
    const uint32_t d = digit_of(key[r], shift);
    // lanes of this wave holding the same digit
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < kRadixBits; ++b) {
      const uint64_t m = __ballot((d >> b) & 1u);
      peers &= ((d >> b) & 1u) ? m : ~m;
    }
    const uint32_t lr = (uint32_t)__popcll(peers & lt);
    if (valid && lr == 0) sh.wcnt[wave][d] = (uint32_t)__popcll(peers);
    __syncthreads();
    uint32_t pre = sh.cnt[d];
    for (int w = 0; w < wave; ++w) pre += sh.wcnt[w][d];
    pos[r] = pre + lr;
    __syncthreads();
    {
      uint32_t add = 0;
#pragma unroll
      for (int w = 0; w < kThreads / 64; ++w) {
        add += sh.wcnt[w][threadIdx.x];
        sh.wcnt[w][threadIdx.x] = 0;
      }
      sh.cnt[threadIdx.x] += add;
    }
    __syncthreads();
  }
  {
    uint32_t tot;
    sh.lstart[threadIdx.x] = block_exclusive_scan<uint32_t>(sh.cnt[threadIdx.x], sh.lw, tot);
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kItems; ++r) pos[r] += sh.lstart[digit_of(key[r], shift)];
}

// Local sort in LDS, then each digit's run written out contiguously at
// sh.dbase[digit].
__device__ __forceinline__ void scatter_tile(int64_t base, int64_t n, int shift,
                                             RankShared& sh, const uint32_t (&key)[kItems],
                                             const uint32_t (&val)[kItems],
                                             const uint32_t (&pos)[kItems],
                                             uint32_t* __restrict__ kout,
                                             uint32_t* __restrict__ vout) {
#pragma unroll
  for (int r = 0; r < kItems; ++r) {
    const int64_t i = base + (int64_t)r * kThreads + threadIdx.x;
    if (i < n) {
      sh.skey[pos[r]] = key[r];
      sh.sval[pos[r]] = val[r];
    }
  }
  __syncthreads();
  const int64_t nb = (n - base) < kTile ? (n - base) : kTile;
  for (int64_t i = threadIdx.x; i < nb; i += kThreads) {
    const uint32_t k = sh.skey[i];
    const uint32_t d = digit_of(k, shift);
    const uint64_t dst = (uint64_t)sh.dbase[d] + (uint64_t)(i - sh.lstart[d]);
    kout[dst] = k;
    vout[dst] = sh.sval[i];
  }
}

// Scatter of the multi-kernel pass: the global position of digit d's run of
// this block is the exclusive scan of the digit totals at d plus the
// row-scanned count of the blocks before it.
__global__ void __launch_bounds__(kThreads)
k_radix_scatter(const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin,
                uint32_t* __restrict__ kout, uint32_t* __restrict__ vout,
                const uint32_t* __restrict__ n_dev, int shift, int64_t nblocks,
                const uint32_t* __restrict__ offsets, const uint32_t* __restrict__ dtot) {
  __shared__ RankShared sh;
  const int64_t n = *n_dev;
  const int64_t base = (int64_t)blockIdx.x * kTile;
  if (base >= n) return;  // uniform per block
  uint32_t key[kItems], val[kItems], pos[kItems];
  rank_tile(kin, vin, base, n, shift, sh, key, val, pos);
  {
    uint32_t tot;
    const uint32_t dstart = block_exclusive_scan<uint32_t>(dtot[threadIdx.x], sh.lw, tot);
    sh.dbase[threadIdx.x] = dstart + offsets[(int64_t)threadIdx.x * nblocks + blockIdx.x];
  }
  __syncthreads();
  scatter_tile(base, n, shift, sh, key, val, pos, kout, vout);
}

// ---------------------------------------------------------------------------
// Pair emission, four consecutive pairs per thread: pair p belongs to the
// depth-sorted splat j with offs[j] <= p < offs[j + 1] and is its
// (p - offs[j])-th tile in row-major order of its tile rect.  A block covers
// kEmitPairs consecutive pairs, hence at most kEmitPairs consecutive splats
// (each has >= 1 pair): their offsets are staged in LDS.  Writes are
// coalesced and the work is balanced whatever the splat sizes.
constexpr int kEmitPairs = 1024;
constexpr int kEmitPerThread = kEmitPairs / kThreads;  // 4 consecutive pairs
static_assert(kEmitPerThread == 4, "emit stores four pairs as one 16-byte word");

__global__ void __launch_bounds__(kThreads)
k_emit(const uint32_t* __restrict__ svals, const uint64_t* __restrict__ offs,
       const uint32_t* __restrict__ n_dev, const uint64_t* __restrict__ m_dev,
       int64_t capacity, const rade_splat* __restrict__ splats,
       const rade_view* __restrict__ views, int64_t N, int tile_w, int tile_h,
       uint32_t* __restrict__ tkeys, uint32_t* __restrict__ pids, int vec_stores) {
  __shared__ uint64_t win[kEmitPairs + 1];
  __shared__ int64_t j0_s;
  const uint64_t M = *m_dev;
  const int64_t nvis = *n_dev;
  const uint64_t P0 = (uint64_t)blockIdx.x * kEmitPairs;
  if (P0 >= M || M > (uint64_t)capacity) return;  // uniform per block
  if (threadIdx.x == 0) {
    // last j with offs[j] <= P0
    int64_t lo = 0, hi = nvis - 1;
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) >> 1;
      if (offs[mid] <= P0) lo = mid; else hi = mid - 1;
    }
    j0_s = lo;
  }
  __syncthreads();
  const int64_t j0 = j0_s;
  for (int w = threadIdx.x; w <= kEmitPairs; w += kThreads) {
    const int64_t j = j0 + w;
    win[w] = j < nvis ? offs[j] : M;
  }
  __syncthreads();
  // Four consecutive pairs per thread: the first one's splat by binary
  // search in the window, the next ones by stepping forward (every listed
  // splat has at least one pair, so this is at most one step per pair); one
  // 16-byte store per output array when all four exist.
  const uint64_t pb = P0 + (uint64_t)kEmitPerThread * threadIdx.x;
  if (pb >= M) return;
  int lo = 0, hi = kEmitPairs;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (win[mid] <= pb) lo = mid; else hi = mid - 1;
  }
  uint32_t tk[kEmitPerThread], pg[kEmitPerThread];
  int cur = -1;
  int tx0 = 0, ty0 = 0, ty1 = 0;
  uint32_t nx = 1, g = 0, toff = 0, tiles_x = 0;
#pragma unroll
  for (int r = 0; r < kEmitPerThread; ++r) {
    const uint64_t p = pb + r;
    tk[r] = 0u;
    pg[r] = 0u;
    if (p >= M) continue;
    while (lo < kEmitPairs && win[lo + 1] <= p) ++lo;
    if (lo != cur) {
      cur = lo;
      // V*N < 2^32 (32-bit ids): 32-bit divisions
      const uint32_t i = svals[j0 + lo];
      const uint32_t v = i / (uint32_t)N;
      g = i - v * (uint32_t)N;
      const rade_splat& sp = splats[i];
      tx0 = sp.rect[0] / tile_w;
      const int tx1 = sp.rect[1] / tile_w;
      ty0 = sp.rect[2] / tile_h;
      ty1 = sp.rect[3] / tile_h;
      nx = (uint32_t)(tx1 - tx0 + 1);
      toff = (uint32_t)views[v].tile_offset;
      tiles_x = (uint32_t)views[v].tiles_x;
    }
    // pair k of the splat is its k-th tile in row-major order of its rect (a
    // splat covers fewer than 2^31 tiles); stay inside the rect even if
    // tiles_touched disagrees with it
    const uint32_t k = (uint32_t)(p - win[lo]);
    const uint32_t row = k / nx;
    const int ty = min(ty0 + (int)row, ty1);
    const int tx = tx0 + (int)(k - row * nx);
    tk[r] = toff + (uint32_t)ty * tiles_x + (uint32_t)tx;
    pg[r] = g;
  }
  if (vec_stores && pb + kEmitPerThread <= M) {
    *reinterpret_cast<uint4*>(tkeys + pb) = make_uint4(tk[0], tk[1], tk[2], tk[3]);
    *reinterpret_cast<uint4*>(pids + pb) = make_uint4(pg[0], pg[1], pg[2], pg[3]);
  } else {
#pragma unroll
    for (int r = 0; r < kEmitPerThread; ++r)
      if (pb + r < M) {
        tkeys[pb + r] = tk[r];
        pids[pb + r] = pg[r];
      }
  }
}

__global__ void __launch_bounds__(kThreads)
k_fill_u32(uint32_t* __restrict__ a, int64_t n, uint32_t value) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i < n) a[i] = value;
}

__global__ void k_finish_counts(const uint64_t* __restrict__ m_dev, int64_t capacity,
                                uint32_t* __restrict__ m32, int64_t* __restrict__ n_pairs_out) {
  const uint64_t m = *m_dev;
  *m32 = m > (uint64_t)capacity ? 0u : (uint32_t)m;  // items the tile sort processes
  *n_pairs_out = (int64_t)m;
}

__global__ void __launch_bounds__(kThreads)
k_ranges(const uint32_t* __restrict__ tkeys, const uint32_t* __restrict__ m32,
         uint32_t* __restrict__ ranges) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int64_t m = *m32;
  if (i >= m) return;
  const uint32_t t = tkeys[i];
  if (i == 0 || tkeys[i - 1] != t) ranges[2 * (int64_t)t] = (uint32_t)i;
  if (i == m - 1 || tkeys[i + 1] != t) ranges[2 * (int64_t)t + 1] = (uint32_t)(i + 1);
}

__global__ void __launch_bounds__(kThreads)
k_keys(const uint32_t* __restrict__ tkeys, const uint32_t* __restrict__ pids,
       const uint32_t* __restrict__ m32, const rade_splat* __restrict__ splats,
       const rade_view* __restrict__ views, int V, int64_t N, uint64_t* __restrict__ keys) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= (int64_t)*m32) return;
  const uint32_t t = tkeys[i];
  const int v = view_of_tile(views, V, t);
  const float z = splats[(int64_t)v * N + pids[i]].z;
  keys[i] = ((uint64_t)t << 32) | (uint64_t)__float_as_uint(z);
}

inline unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

// Sorts (keys, vals) of *n_dev items (at most n_max) by the low `bits` bits
// of the keys; on return the sorted data are in (k0, v0) when the number of
// passes is even, else in (k1, v1).  Returns the number of passes.
int radix_sort(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1, int64_t n_max,
               const uint32_t* n_dev, int bits, uint32_t* hist, uint32_t* hist_sums,
               hipStream_t st) {
  const int64_t nb = n_max > 0 ? (n_max + kTile - 1) / kTile : 1;
  const int passes = (bits + kRadixBits - 1) / kRadixBits;
  for (int p = 0; p < passes; ++p) {
    const int shift = p * kRadixBits;
    uint32_t* ki = (p & 1) ? k1 : k0;
    uint32_t* vi = (p & 1) ? v1 : v0;
    uint32_t* ko = (p & 1) ? k0 : k1;
    uint32_t* vo = (p & 1) ? v0 : v1;
    hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)nb), dim3(kThreads), 0, st, ki, n_dev, shift,
                       nb, hist);
    hipLaunchKernelGGL(k_radix_colscan, dim3(kRadix), dim3(kThreads), 0, st, hist, nb,
                       hist_sums);
    hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)nb), dim3(kThreads), 0, st, ki, vi, ko, vo,
                       n_dev, shift, nb, hist, (const uint32_t*)hist_sums);
  }
  return passes;
}

inline size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

struct Layout {
  size_t vis_pos, dkeys0, dvals0, dkeys1, dvals1, offs, tkeys0, tkeys1, pids1, hist, sums, scal;
  size_t total;
};

int ceil_log2(int64_t x) {
  int b = 0;
  while (((int64_t)1 << b) < x) ++b;
  return b;
}

Layout layout(int64_t VN, int64_t capacity) {
  Layout L;
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t at = o; o = align_up(o + bytes); return at; };
  const int64_t nmax = VN > capacity ? VN : capacity;
  const int64_t nb = (nmax + kTile - 1) / kTile + 1;
  const int64_t hist_n = nb * kRadix;
  const int64_t scan_n = (hist_n > nmax ? hist_n : nmax);
  L.vis_pos = take(sizeof(uint32_t) * VN);
  L.dkeys0 = take(sizeof(uint32_t) * VN);
  L.dvals0 = take(sizeof(uint32_t) * VN);
  L.dkeys1 = take(sizeof(uint32_t) * VN);
  L.dvals1 = take(sizeof(uint32_t) * VN);
  L.offs = take(sizeof(uint64_t) * VN);
  L.tkeys0 = take(sizeof(uint32_t) * capacity);
  L.tkeys1 = take(sizeof(uint32_t) * capacity);
  L.pids1 = take(sizeof(uint32_t) * capacity);
  L.hist = take(sizeof(uint32_t) * hist_n);
  // block sums of the scans, and the 256 digit totals of a radix pass
  const size_t sums_bytes = sizeof(uint64_t) * ((scan_n + kTile - 1) / kTile + 1);
  L.sums = take(sums_bytes > sizeof(uint32_t) * kRadix ? sums_bytes : sizeof(uint32_t) * kRadix);
  L.scal = take(64);
  L.total = o;
  return L;
}

// Scan block sums (unused by the radix passes now) or the 256 digit totals.
inline size_t tile_order_sums_bytes(int64_t nb) {
  const size_t a = sizeof(uint64_t) * (size_t)(nb * kRadix / kTile + 2);
  const size_t b = sizeof(uint32_t) * kRadix;
  return a > b ? a : b;
}

// Order key of a tile: 255 - 16 log2(len + 1), so longer lists come first.
__global__ void __launch_bounds__(kThreads)
k_order_keys(const uint32_t* __restrict__ ranges, int64_t tiles, uint32_t* __restrict__ keys,
             uint32_t* __restrict__ vals, uint32_t* __restrict__ count) {
  const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (t == 0) *count = (uint32_t)tiles;
  if (t >= tiles) return;
  const uint32_t len = ranges[2 * t + 1] - ranges[2 * t];
  const int b = len == 0 ? 0 : min(255, (int)(16.0f * __log2f((float)len + 1.0f)));
  keys[t] = (uint32_t)(255 - b);
  vals[t] = (uint32_t)t;
}

}  // namespace

size_t tile_order_workspace(int64_t tiles) {
  const int64_t nb = (tiles + kTile - 1) / kTile + 1;
  return align_up(sizeof(uint32_t) * tiles) * 3 + align_up(sizeof(uint32_t) * nb * kRadix) +
         align_up(tile_order_sums_bytes(nb)) + 256;
}

hipError_t launch_tile_order(const uint32_t* ranges, int64_t tiles, uint32_t* order, void* ws,
                             hipStream_t st) {
  char* w = static_cast<char*>(ws);
  const int64_t nb = (tiles + kTile - 1) / kTile + 1;
  uint32_t* k0 = (uint32_t*)w;
  uint32_t* v0 = (uint32_t*)(w + align_up(sizeof(uint32_t) * tiles));
  uint32_t* k1 = (uint32_t*)(w + 2 * align_up(sizeof(uint32_t) * tiles));
  uint32_t* hist = (uint32_t*)(w + 3 * align_up(sizeof(uint32_t) * tiles));
  uint32_t* sums = (uint32_t*)((char*)hist + align_up(sizeof(uint32_t) * nb * kRadix));
  uint32_t* cnt = (uint32_t*)((char*)sums + align_up(tile_order_sums_bytes(nb)));
  hipLaunchKernelGGL(k_order_keys, dim3(blocks_for(tiles > 0 ? tiles : 1, kThreads)),
                     dim3(kThreads), 0, st, ranges, tiles, k0, v0, cnt);
  // one 8-bit pass: the result lands in (k1, order)
  radix_sort(k0, v0, k1, order, tiles, cnt, 8, hist, sums, st);
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(kThreads), 0, st, order + tiles, 1, 0u);
  return hipGetLastError();
}

size_t bin_sort_workspace(int64_t VN, int64_t capacity) { return layout(VN, capacity).total; }

hipError_t launch_bin_sort(const rade_settings& s, const rade_view* views_host,
                           const rade_view* views_dev, int V, int64_t N,
                           const rade_splat* splats, const int32_t* tt, uint32_t* pair_ids,
                           uint32_t* ranges, uint64_t* keys, int64_t capacity,
                           int64_t* n_pairs_dev, int64_t* n_pairs_host, void* ws,
                           hipStream_t st, int* capacity_exceeded) {
  *capacity_exceeded = 0;
  const int64_t VN = (int64_t)V * N;
  const Layout L = layout(VN, capacity);
  char* w = static_cast<char*>(ws);
  uint32_t* vis_pos = (uint32_t*)(w + L.vis_pos);
  uint32_t* dk0 = (uint32_t*)(w + L.dkeys0);
  uint32_t* dv0 = (uint32_t*)(w + L.dvals0);
  uint32_t* dk1 = (uint32_t*)(w + L.dkeys1);
  uint32_t* dv1 = (uint32_t*)(w + L.dvals1);
  uint64_t* offs = (uint64_t*)(w + L.offs);
  uint32_t* tk0 = (uint32_t*)(w + L.tkeys0);
  uint32_t* tk1 = (uint32_t*)(w + L.tkeys1);
  uint32_t* pid1 = (uint32_t*)(w + L.pids1);
  uint32_t* hist = (uint32_t*)(w + L.hist);
  void* sums = (void*)(w + L.sums);
  uint32_t* n_vis = (uint32_t*)(w + L.scal);
  uint64_t* m64 = (uint64_t*)(w + L.scal + 8);
  uint32_t* m32 = (uint32_t*)(w + L.scal + 16);

  int64_t total_tiles = 0;
  for (int v = 0; v < V; ++v)
    total_tiles += (int64_t)views_host[v].tiles_x * views_host[v].tiles_y;

  // 1. visible splats -> compact (depth key, index) list
  if (VN > 0) {
    scan<uint32_t>(FlagInput{tt}, VN, nullptr, vis_pos, (uint32_t*)sums, n_vis, st);
    hipLaunchKernelGGL(k_compact, dim3(blocks_for(VN, kThreads)), dim3(kThreads), 0, st, tt,
                       vis_pos, splats, VN, dk0, dv0);
  } else {
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(kThreads), 0, st, n_vis, 1, 0u);
  }
  // 2. depth sort
  const int dpasses = radix_sort(dk0, dv0, dk1, dv1, VN, n_vis, 32, hist, (uint32_t*)sums, st);
  uint32_t* sv = (dpasses & 1) ? dv1 : dv0;
  // 3. pair offsets in depth order
  if (VN > 0) {
    scan<uint64_t>(GatherCount{tt, sv}, VN, n_vis, offs, (uint64_t*)sums, m64, st);
  } else {
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(kThreads), 0, st, (uint32_t*)m64, 2, 0u);
  }
  hipLaunchKernelGGL(k_finish_counts, dim3(1), dim3(1), 0, st, m64, capacity, m32, n_pairs_dev);
  if (n_pairs_host) {
    hipError_t e = hipMemcpyAsync(n_pairs_host, n_pairs_dev, sizeof(int64_t),
                                  hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e;
    if (*n_pairs_host > capacity) {
      *capacity_exceeded = 1;
      hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for(2 * total_tiles, kThreads)), dim3(kThreads),
                         0, st, ranges, 2 * total_tiles, 0u);
      return hipGetLastError();
    }
  }
  // 4. emit pairs; the tile sort's passes alternate buffers, so emit into
  // the buffer that makes the last pass land in pair_ids.
  const int tbits = total_tiles > 1 ? ceil_log2(total_tiles) : 1;
  const int tpasses = (tbits + kRadixBits - 1) / kRadixBits;
  uint32_t* ek = tk0;
  uint32_t* ev = (tpasses & 1) ? pid1 : pair_ids;
  uint32_t* ok_ = tk1;
  uint32_t* ov = (tpasses & 1) ? pair_ids : pid1;
  if (VN > 0 && capacity > 0)
    hipLaunchKernelGGL(k_emit, dim3(blocks_for(capacity, kEmitPairs)), dim3(kThreads), 0, st, sv,
                       offs, n_vis, m64, capacity, splats, views_dev, N, s.tile_w, s.tile_h, ek,
                       ev, (((uintptr_t)ek | (uintptr_t)ev) & 15) == 0 ? 1 : 0);
  // 5. stable sort by tile
  radix_sort(ek, ev, ok_, ov, capacity, m32, tbits, hist, (uint32_t*)sums, st);
  uint32_t* sk = (tpasses & 1) ? ok_ : ek;
  // 6. tile ranges
  hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for(2 * total_tiles, kThreads)), dim3(kThreads), 0,
                     st, ranges, 2 * total_tiles, 0u);
  if (capacity > 0)
    hipLaunchKernelGGL(k_ranges, dim3(blocks_for(capacity, kThreads)), dim3(kThreads), 0, st, sk,
                       m32, ranges);
  // 7. optional 64-bit keys
  if (keys && capacity > 0)
    hipLaunchKernelGGL(k_keys, dim3(blocks_for(capacity, kThreads)), dim3(kThreads), 0, st, sk,
                       pair_ids, m32, splats, views_dev, V, N, keys);
  return hipGetLastError();
}

}  // namespace rade
