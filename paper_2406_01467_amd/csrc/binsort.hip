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
#include "grid.hpp"
#include "scan.hpp"

namespace rade {
namespace {

constexpr int kThreads = kScanThreads;
constexpr int kItems = kScanItems;              // items per thread
constexpr int kTile = kScanTile;                // items per block (2048)
constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;
// Widest digit of a pass: 9 bits where that saves a pass (17 or 18 key bits,
// e.g. the tile keys of many views of small tiles, sort in two 9-bit passes
// instead of three 8-bit ones).
constexpr int kMaxRadix = 512;

constexpr int kEmitPairs = kTile;                // pairs per emission block (one radix block)

// Compaction of the visible splats (tiles touched > 0), read in index order:
// the depth sort's keys (bits of the float32 view depth, from the splat's
// 16-byte binning record) and values (the splat's index).  The depth sort's
// last pass gathers the binning records into depth order (the index in
// place of the depth word), so the pair emission reads them in order
// instead of gathering records by index.
struct Visible {
  const int32_t* tt;
  __device__ uint32_t operator()(int64_t i) const { return tt[i] > 0 ? 1u : 0u; }
};
struct VisibleOut {
  const uint4* brecs;
  uint32_t* keys;
  uint32_t* vals;
  __device__ void operator()(int64_t i, uint32_t p, uint32_t) const {
    keys[p] = brecs[i].x;  // z > near > 0: bits order like values
    vals[p] = (uint32_t)i;
  }
};

// Tiles touched by the j-th depth-sorted splat (its record's count, which
// the depth sort's last pass also writes to an array of its own, so the
// scans read 4 bytes per splat rather than the 16-byte records).
struct SortedCount {
  const uint32_t* cnt;
  __device__ uint64_t operator()(int64_t j) const { return (uint64_t)cnt[j]; }
};
// Total pair count: stored as 64 bits, as the count the tile sort processes
// (0 when it exceeds the capacity, so nothing is written) and as the
// caller's pair count.
struct PairsTotal {
  uint64_t* m64;
  uint32_t* m32;
  int64_t capacity;
  int64_t* n_pairs_out;
  __device__ void operator()(uint64_t m) const {
    *m64 = m;
    *m32 = m > (uint64_t)capacity ? 0u : (uint32_t)m;
    *n_pairs_out = (int64_t)m;
  }
};

// Pair offsets of the depth-sorted splats, and for every emission block the
// splat that holds its first pair: block b starts in splat j when
// offs[j] <= b * kEmitPairs < offs[j] + count[j].
struct OffsetsOut {
  uint64_t* offs;
  uint32_t* starts;
  int64_t nstarts;
  __device__ void operator()(int64_t j, uint64_t off, uint64_t cnt) const {
    offs[j] = off;
    const uint64_t end = off + cnt;
    for (uint64_t b = (off + kEmitPairs - 1) / kEmitPairs;
         b * kEmitPairs < end && b < (uint64_t)nstarts; ++b)
      starts[b] = (uint32_t)j;
  }
};

// ---------------------------------------------------------------------------
// LSD radix sort, RB-bit digits (8, or 9 where that saves a pass), stable.
// Each pass counts the digits of every block of kTile consecutive items
// (k_radix_hist, counts stored digit-major: hist[d * nblocks + block]), scans
// each digit's row of counts (k_radix_colscan) and scatters
// (k_radix_scatter).
//
// Workgroups are dealt to the XCDs round-robin, so the sort kernels remap
// the workgroup index to a block index such that each XCD takes one
// contiguous run of blocks: the counts of neighbouring blocks (which share
// cache lines of the digit-major rows) then meet in one L2 instead of up to
// eight.
template <int RB = kRadixBits>
__device__ __forceinline__ uint32_t digit_of(uint32_t k, int shift) {
  return (k >> shift) & ((1u << RB) - 1u);
}

constexpr int kXcds = 8;

__device__ __forceinline__ int64_t xcd_block(int64_t wg, int64_t grid) {
  const int64_t x = wg % kXcds, k = wg / kXcds;
  const int64_t q = grid / kXcds, r = grid % kXcds;
  return x * q + (x < r ? x : r) + k;
}

// Items of a radix block: wave w holds the kItems rounds of 64 consecutive
// items [base + w*64*kItems, base + (w+1)*64*kItems), round r at offset
// r*64 + lane.  Block order is then (wave, round, lane), so ranks counted
// per wave, round after round, and combined across waves in wave order are
// stable.  All loads of a thread are issued before any ranking.
constexpr int kWaves = kThreads / 64;
static_assert(kRadix == kThreads && kMaxRadix == 2 * kThreads,
              "one or two digits per thread in the block-wide steps");

__device__ __forceinline__ int64_t item_index(int64_t base, int r) {
  return base + (int64_t)(threadIdx.x >> 6) * (64 * kItems) + (int64_t)r * 64 +
         (threadIdx.x & 63);
}

// Lanes of the wave whose item is valid and has digit d: one ballot per
// digit bit, each lane keeping the lanes that agree with its own bit.  With
// s = 0 or ~0 from the lane's bit, the lanes that agree are ~(m ^ s); the
// halves are kept apart so the selection stays a few 32-bit logic ops.
template <int RB = kRadixBits>
__device__ __forceinline__ uint64_t digit_peers(uint32_t d, bool valid) {
  const uint64_t v = __ballot(valid);
  uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
#pragma unroll
  for (int b = 0; b < RB; ++b) {
    const uint32_t s = (uint32_t)((int32_t)(d << (31 - b)) >> 31);
    const uint64_t m = __builtin_amdgcn_ballot_w64(s != 0u);
    lo &= ~((uint32_t)m ^ s);
    hi &= ~((uint32_t)(m >> 32) ^ s);
  }
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t lanes_below() {
  const int lane = threadIdx.x & 63;
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Per-block digit counts (LDS atomics; lanes that hit one counter are
// serialised by the LDS, not by vector instructions).  The top digit of
// 32-bit keys (the sign and exponent byte of the float depths) takes few
// values: there the lanes of one digit are matched by ballots (digit_peers)
// and their lowest lane adds their number, one LDS atomic per distinct digit
// of a wave (elsewhere the ballots cost more than the contention they save).
template <int RB>
__global__ void __launch_bounds__(kThreads)
k_radix_hist(const uint32_t* __restrict__ keys, const uint32_t* __restrict__ n_dev,
             int64_t n_max, int shift, int64_t nblocks, uint32_t* __restrict__ hist) {
  constexpr int R = 1 << RB;
  __shared__ uint32_t h[R];
  const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
  const int64_t base = blk * kTile;
  // the loads are bounded by the buffer size, so they need not wait for
  // the item count; items past it are not counted
  uint32_t key[kItems];
#pragma unroll
  for (int r = 0; r < kItems; ++r) {
    const int64_t i = item_index(base, r);
    key[r] = i < n_max ? keys[i] : 0u;
  }
  const int64_t n = *n_dev;
#pragma unroll
  for (int d = threadIdx.x; d < R; d += kThreads) h[d] = 0;
  __syncthreads();
  if (shift + RB >= 32) {  // uniform
    const uint64_t lt = lanes_below();
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
      const bool valid = item_index(base, r) < n;
      const uint32_t d = digit_of<RB>(key[r], shift);
      const uint64_t peers = digit_peers<RB>(d, valid);
      if (valid && (peers & lt) == 0) atomicAdd(&h[d], (uint32_t)__popcll(peers));
    }
  } else {
#pragma unroll
    for (int r = 0; r < kItems; ++r)
      if (item_index(base, r) < n) atomicAdd(&h[digit_of<RB>(key[r], shift)], 1u);
  }
  __syncthreads();
#pragma unroll
  for (int d = threadIdx.x; d < R; d += kThreads) hist[(int64_t)d * nblocks + blk] = h[d];
}

// Exclusive scan of one digit's row of per-block counts (one workgroup per
// digit) and the digit's total.  Together with the scan of the digit totals
// in the scatter's prologue this replaces a global scan of the whole count
// matrix.
__global__ void __launch_bounds__(kThreads)
k_radix_colscan(uint32_t* __restrict__ hist, int64_t nblocks, uint32_t* __restrict__ dtot) {
  __shared__ uint32_t lw[kWaves];
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
template <int R>
struct RankShared {
  uint32_t wcnt[kWaves][R];  // per-wave digit counts, then per-wave digit starts
  uint32_t lstart[R];        // first local position of each digit
  uint32_t dbase[R];         // global position of each digit's run
  uint32_t skey[kTile];
  uint32_t sval[kTile];
  uint64_t lw[kWaves];
};

// Scatter of one pass.  The block is ranked stably: each wave counts its
// rounds' digits in its own LDS row (a running count, so no block barrier
// between rounds), one pass per digit turns the rows into per-wave starts,
// and one block scan of (digit total << 32 | local count) gives both the
// start of each digit's region in the output and the block's local digit
// starts (the local counts sum to at most kTile, so the halves never carry
// into each other).  The block is then sorted in LDS and each digit's run
// written contiguously at its region start plus the row-scanned count of
// the blocks before this one.  GATHER: each item also carries the record
// gsrc[value] (values index gsrc), written to gout in the sorted order, and
// its last word to cout.  Thread t takes digits DPT t .. DPT t + DPT - 1 in
// the block-wide steps (DPT = 2 for 9-bit digits).
template <bool GATHER, int RB>
__global__ void __launch_bounds__(kThreads)
k_radix_scatter(const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin,
                uint32_t* __restrict__ kout, uint32_t* __restrict__ vout,
                const uint32_t* __restrict__ n_dev, int64_t n_max, int shift, int64_t nblocks,
                const uint32_t* __restrict__ offsets, const uint32_t* __restrict__ dtot,
                const uint4* __restrict__ gsrc, uint4* __restrict__ gout,
                uint32_t* __restrict__ cout) {
  constexpr int R = 1 << RB, DPT = R / kThreads;
  __shared__ RankShared<R> sh;
  const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
  const int64_t base = blk * kTile;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  // all loads are issued before the item count is known (bounded by the
  // buffer size instead)
  uint32_t key[kItems], val[kItems], pos[kItems];
#pragma unroll
  for (int r = 0; r < kItems; ++r) {
    const int64_t i = item_index(base, r);
    const bool inb = i < n_max;
    key[r] = inb ? kin[i] : 0u;
    val[r] = inb ? vin[i] : 0u;
  }
  uint32_t dtot_d[DPT], goff_d[DPT];
#pragma unroll
  for (int k = 0; k < DPT; ++k) {
    const int d = DPT * (int)threadIdx.x + k;
    dtot_d[k] = dtot[d];
    goff_d[k] = offsets[(int64_t)d * nblocks + blk];
  }
  const int64_t n = *n_dev;
  if (base >= n) return;  // uniform per block
  uint32_t* wc = sh.wcnt[wave];
#pragma unroll
  for (int k = 0; k < R / 64; ++k) wc[k * 64 + lane] = 0;
  const uint64_t lt = lanes_below();
#pragma unroll
  for (int r = 0; r < kItems; ++r) {
    const bool valid = item_index(base, r) < n;
    const uint32_t d = digit_of<RB>(key[r], shift);
    const uint64_t peers = digit_peers<RB>(d, valid);
    // LDS operations of one wave complete in issue order; the leader's
    // store depends on the value every lane read
    const uint32_t pre = wc[d];
    pos[r] = pre + (uint32_t)__popcll(peers & lt);
    if (valid && (peers & lt) == 0) wc[d] = pre + (uint32_t)__popcll(peers);
  }
  __syncthreads();
  {
    uint64_t dc[DPT], sum = 0;
#pragma unroll
    for (int k = 0; k < DPT; ++k) {
      const int d = DPT * (int)threadIdx.x + k;
      uint32_t c = 0;
#pragma unroll
      for (int w = 0; w < kWaves; ++w) {
        const uint32_t x = sh.wcnt[w][d];
        sh.wcnt[w][d] = c;
        c += x;
      }
      dc[k] = ((uint64_t)dtot_d[k] << 32) | c;
      sum += dc[k];
    }
    uint64_t tot;
    uint64_t ex = block_exclusive_scan<uint64_t>(sum, sh.lw, tot);
#pragma unroll
    for (int k = 0; k < DPT; ++k) {
      const int d = DPT * (int)threadIdx.x + k;
      sh.lstart[d] = (uint32_t)ex;
      sh.dbase[d] = (uint32_t)(ex >> 32) + goff_d[k];
      ex += dc[k];
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kItems; ++r) {
    if (item_index(base, r) < n) {
      const uint32_t d = digit_of<RB>(key[r], shift);
      const uint32_t p = pos[r] + sh.lstart[d] + sh.wcnt[wave][d];
      sh.skey[p] = key[r];
      sh.sval[p] = val[r];
    }
  }
  __syncthreads();
  const int nb = (n - base) < kTile ? (int)(n - base) : kTile;
#pragma unroll
  for (int r = 0; r < kItems; ++r) {  // unrolled: the gathers are issued together
    const int i = (int)threadIdx.x + r * kThreads;
    if (i < nb) {
      const uint32_t k = sh.skey[i];
      const uint32_t v = sh.sval[i];
      const uint32_t d = digit_of<RB>(k, shift);
      const uint32_t dst = sh.dbase[d] + ((uint32_t)i - sh.lstart[d]);
      kout[dst] = k;
      vout[dst] = v;
      if constexpr (GATHER) {
        const uint4 rec = gsrc[v];
        gout[dst] = make_uint4(v, rec.y, rec.z, rec.w);
        cout[dst] = rec.w;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Pair emission, four consecutive pairs per thread: pair p belongs to the
// depth-sorted splat j with offs[j] <= p < offs[j + 1] and is its
// (p - offs[j])-th tile in row-major order of its tile rect.  Block b (a
// radix block of the tile sort, remapped like the sort's blocks) covers
// kEmitPairs consecutive pairs, hence at most kEmitPairs consecutive splats
// (each has >= 1 pair), starting with starts[b]: their offsets and ids are
// staged in LDS.  Writes are coalesced and the work is balanced whatever the
// splat sizes.  The block also counts the low RB bits of its tile keys, the
// per-block digit counts of the tile sort's first pass.
constexpr int kEmitThreads = 512;
constexpr int kEmitPerThread = kEmitPairs / kEmitThreads;  // 4 consecutive pairs
static_assert(kEmitPerThread == 4, "emit stores four pairs as one 16-byte word");

template <int RB>
__global__ void __launch_bounds__(kEmitThreads)
k_emit(const uint4* __restrict__ drecs, const uint64_t* __restrict__ offs,
       const uint32_t* __restrict__ starts, const uint32_t* __restrict__ n_dev,
       const uint64_t* __restrict__ m_dev, int64_t capacity,
       const rade_view* __restrict__ views, FastDiv div_n, uint32_t* __restrict__ tkeys,
       uint32_t* __restrict__ pids, int vec_stores, int64_t nblocks, uint32_t* __restrict__ hist) {
  constexpr int R = 1 << RB;
  __shared__ uint64_t win[kEmitPairs + 1];
  __shared__ uint32_t h[R];
  const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
  const uint64_t M = *m_dev;
  const int64_t nvis = *n_dev;
  const int64_t j0 = starts[blk];
  const uint64_t P0 = (uint64_t)blk * kEmitPairs;
  for (int d = threadIdx.x; d < R; d += kEmitThreads) h[d] = 0u;
  if (P0 >= M || M > (uint64_t)capacity) {  // uniform per block
    for (int d = threadIdx.x; d < R; d += kEmitThreads) hist[(int64_t)d * nblocks + blk] = 0u;
    return;
  }
  // The block's pairs belong to the splats j0 .. j1, j1 the splat of the next
  // block's first pair (starts[blk + 1], written when that pair exists); the
  // window holds their offsets and the one after (at most kEmitPairs + 1
  // entries: every splat has at least one pair).
  const int64_t j1 = P0 + kEmitPairs >= M ? nvis - 1 : (int64_t)starts[blk + 1];
  const int nwin = (int)min((int64_t)kEmitPairs, j1 - j0 + 1);
  for (int w = threadIdx.x; w <= nwin; w += kEmitThreads) {
    const int64_t j = j0 + w;
    const bool in = j < nvis;
    win[w] = in ? offs[j] : M;
  }
  __syncthreads();
  // The first pair's splat by binary search in the window, the next ones by
  // stepping forward (every listed splat has at least one pair, so this is
  // at most one step per pair).
  const uint64_t pb = P0 + (uint64_t)kEmitPerThread * threadIdx.x;
  uint32_t tk[kEmitPerThread], pg[kEmitPerThread];
  if (pb < M) {
    int lo = 0, hi = nwin;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (win[mid] <= pb) lo = mid; else hi = mid - 1;
    }
    int cur = -1;
    uint32_t tx0 = 0, ty0 = 0, ty1 = 0, nx = 1, g = 0, toff = 0, tiles_x = 0, row = 0, col = 0;
#pragma unroll
    for (int r = 0; r < kEmitPerThread; ++r) {
      const uint64_t p = pb + r;
      tk[r] = 0u;
      pg[r] = 0u;
      if (p >= M) continue;
      while (lo < nwin && win[lo + 1] <= p) ++lo;
      if (lo != cur) {
        cur = lo;
        // the splat's record in depth order (index, tile rect); V*N < 2^32
        // (32-bit ids)
        const uint4 rec = drecs[j0 + lo];
        const uint32_t i = rec.x;
        const uint32_t v = div_n.div(i);
        g = i - v * div_n.d;
        tx0 = rec.y & 0xFFFFu;
        ty0 = rec.y >> 16;
        const uint32_t tx1 = rec.z & 0xFFFFu;
        ty1 = rec.z >> 16;
        nx = tx1 - tx0 + 1;
        toff = (uint32_t)views[v].tile_offset;
        tiles_x = (uint32_t)views[v].tiles_x;
        // pair k of the splat is its k-th tile in row-major order of its
        // rect (k > 0 only for the thread's first pair)
        const uint32_t k = (uint32_t)(p - win[lo]);
        row = k / nx;
        col = k - row * nx;
      } else if (++col == nx) {
        col = 0;
        ++row;
      }
      // stay inside the rect even if tiles_touched disagrees with it
      const uint32_t ty = min(ty0 + row, ty1);
      tk[r] = toff + ty * tiles_x + tx0 + col;
      pg[r] = g;
      atomicAdd(&h[tk[r] & (R - 1)], 1u);
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
  __syncthreads();
  for (int d = threadIdx.x; d < R; d += kEmitThreads) hist[(int64_t)d * nblocks + blk] = h[d];
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

// Tile ranges from the sorted tile keys: [first, end) of each tile's run of
// pairs, [0, 0) for a tile without pairs.  Item boundary i (0 <= i <= m)
// sits between the tiles prev = key[i - 1] (-1 for i = 0) and cur = key[i]
// (`tiles` for i = m); where they differ it ends prev's range, starts cur's
// and clears the tiles in between.  Each thread takes four boundaries.
__device__ __forceinline__ void range_edge(uint32_t* __restrict__ ranges, int64_t i, int64_t m,
                                           int64_t prev, int64_t cur) {
  if (prev == cur) return;
  if (prev >= 0) ranges[2 * prev + 1] = (uint32_t)i;
  if (i < m) ranges[2 * cur] = (uint32_t)i;
  for (int64_t t = prev + 1; t < cur; ++t) {
    ranges[2 * t] = 0u;
    ranges[2 * t + 1] = 0u;
  }
}

// Keys per thread of k_ranges (four 16-byte loads; consecutive threads take
// consecutive runs, so a thread's previous key is its left neighbour's last).
constexpr int kRangeKeys = 16;

__global__ void __launch_bounds__(kThreads)
k_ranges(const uint32_t* __restrict__ tkeys, const uint32_t* __restrict__ m32, int64_t tiles,
         uint32_t* __restrict__ ranges) {
  const int64_t g = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int64_t m = *m32;
  if (m == 0) {  // no pairs (or too many for the capacity): every range empty
    for (int64_t t = g; t < tiles; t += (int64_t)gridDim.x * kThreads) {
      ranges[2 * t] = 0u;
      ranges[2 * t + 1] = 0u;
    }
    return;
  }
  const int64_t i0 = (int64_t)kRangeKeys * g;
  // the key before a wave's first run, loaded with the runs (not after the
  // shuffle below, which would add a second memory latency to every wave)
  const bool first_lane = (threadIdx.x & 63) == 0;
  const uint32_t before = first_lane && i0 > 0 && i0 <= m ? tkeys[i0 - 1] : 0u;
  uint32_t k[kRangeKeys];
  if (i0 + kRangeKeys <= m) {  // tkeys is 16-byte aligned
#pragma unroll
    for (int q = 0; q < kRangeKeys / 4; ++q) {
      const uint4 v = *reinterpret_cast<const uint4*>(tkeys + i0 + 4 * q);
      k[4 * q] = v.x; k[4 * q + 1] = v.y; k[4 * q + 2] = v.z; k[4 * q + 3] = v.w;
    }
  } else {
#pragma unroll
    for (int r = 0; r < kRangeKeys; ++r) k[r] = i0 + r < m ? tkeys[i0 + r] : 0u;
  }
  // the previous key: the left lane's last one (whole waves take part in
  // the shuffle; lane 0 of a wave reads it)
  const uint32_t left = (uint32_t)__shfl_up((int)k[kRangeKeys - 1], 1, 64);
  if (i0 > m) return;
  int64_t prev;
  if (i0 == 0) prev = -1;
  else if (!first_lane) prev = (int64_t)left;
  else prev = (int64_t)before;
#pragma unroll
  for (int r = 0; r < kRangeKeys; ++r) {
    const int64_t i = i0 + r;
    if (i > m) break;
    const int64_t cur = i < m ? (int64_t)k[r] : tiles;
    range_edge(ranges, i, m, prev, cur);
    prev = cur;
  }
}

__global__ void __launch_bounds__(kThreads)
k_keys(const uint32_t* __restrict__ tkeys, const uint32_t* __restrict__ pids,
       const uint32_t* __restrict__ m32, const uint4* __restrict__ brecs,
       const rade_view* __restrict__ views, int V, int64_t N, uint64_t* __restrict__ keys) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= (int64_t)*m32) return;
  const uint32_t t = tkeys[i];
  const int v = view_of_tile(views, V, t);
  const uint32_t zbits = brecs[(int64_t)v * N + pids[i]].x;  // bits of the float32 depth
  keys[i] = ((uint64_t)t << 32) | (uint64_t)zbits;
}

inline unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

inline size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

// Work space of one radix sort of at most n_max items: the digit-major
// per-block counts and the digit totals (room for 9-bit digits).
struct SortSpace {
  uint32_t* hist;
  uint32_t* dtot;
};

inline int64_t sort_blocks(int64_t n_max) { return n_max > 0 ? (n_max + kTile - 1) / kTile : 1; }

inline size_t sort_space_bytes(int64_t n_max) {
  return align_up(sizeof(uint32_t) * sort_blocks(n_max) * kMaxRadix) +
         align_up(sizeof(uint32_t) * kMaxRadix);
}

inline SortSpace sort_space(char* w, int64_t n_max) {
  SortSpace sp;
  sp.hist = (uint32_t*)w;
  sp.dtot = (uint32_t*)(w + align_up(sizeof(uint32_t) * sort_blocks(n_max) * kMaxRadix));
  return sp;
}

// Digit width of a sort by `bits` key bits: 9 where that takes fewer passes
// than 8 (17-18 or 25-27 bits), else 8.
inline int digit_bits(int bits) {
  return (bits + 8) / 9 < (bits + 7) / 8 ? 9 : kRadixBits;
}

// Sorts (keys, vals) of *n_dev items (at most n_max < 2^32) by the low
// `bits` bits of the keys, in passes of digit_bits(bits) bits; on return the
// sorted data are in (k0, v0) when the number of passes is even, else in
// (k1, v1).  Returns the number of passes.  first_counted: the first pass's
// per-block counts (of digits that wide) are already in sp.hist.
// gsrc: the last pass also writes the record gsrc[value] of every item (the
// values index gsrc), in the sorted order and with the value in place of
// its first word, to gout, and its last word to cout.
template <int RB>
int radix_sort_rb(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1, int64_t n_max,
                  const uint32_t* n_dev, int bits, const SortSpace& sp, hipStream_t st,
                  bool first_counted, const uint4* gsrc, uint4* gout, uint32_t* cout) {
  const int64_t nb = sort_blocks(n_max);
  const int passes = bits > RB ? (bits + RB - 1) / RB : 1;
  for (int p = 0; p < passes; ++p) {
    const int shift = p * RB;
    uint32_t* ki = (p & 1) ? k1 : k0;
    uint32_t* vi = (p & 1) ? v1 : v0;
    uint32_t* ko = (p & 1) ? k0 : k1;
    uint32_t* vo = (p & 1) ? v0 : v1;
    if (p > 0 || !first_counted)
      hipLaunchKernelGGL(k_radix_hist<RB>, dim3((unsigned)nb), dim3(kThreads), 0, st, ki, n_dev,
                         n_max, shift, nb, sp.hist);
    hipLaunchKernelGGL(k_radix_colscan, dim3(1u << RB), dim3(kThreads), 0, st, sp.hist, nb,
                       sp.dtot);
    if (gsrc && p == passes - 1)
      hipLaunchKernelGGL((k_radix_scatter<true, RB>), dim3((unsigned)nb), dim3(kThreads), 0, st,
                         ki, vi, ko, vo, n_dev, n_max, shift, nb, (const uint32_t*)sp.hist,
                         (const uint32_t*)sp.dtot, gsrc, gout, cout);
    else
      hipLaunchKernelGGL((k_radix_scatter<false, RB>), dim3((unsigned)nb), dim3(kThreads), 0, st,
                         ki, vi, ko, vo, n_dev, n_max, shift, nb, (const uint32_t*)sp.hist,
                         (const uint32_t*)sp.dtot, (const uint4*)nullptr, (uint4*)nullptr,
                         (uint32_t*)nullptr);
  }
  return passes;
}

int radix_sort(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1, int64_t n_max,
               const uint32_t* n_dev, int bits, const SortSpace& sp, hipStream_t st,
               bool first_counted = false, const uint4* gsrc = nullptr,
               uint4* gout = nullptr, uint32_t* cout = nullptr) {
  if (digit_bits(bits) == 9)
    return radix_sort_rb<9>(k0, v0, k1, v1, n_max, n_dev, bits, sp, st, first_counted, gsrc,
                            gout, cout);
  return radix_sort_rb<kRadixBits>(k0, v0, k1, v1, n_max, n_dev, bits, sp, st, first_counted,
                                   gsrc, gout, cout);
}

struct Layout {
  size_t starts, dkeys0, dvals0, dkeys1, dvals1, drec, dcnt, offs, tkeys0, tkeys1, pids1,
      sort, sums, scal;
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
  L.starts = take(sizeof(uint32_t) * ((capacity + kEmitPairs - 1) / kEmitPairs + 1));
  L.dkeys0 = take(sizeof(uint32_t) * VN);
  L.dvals0 = take(sizeof(uint32_t) * VN);
  L.dkeys1 = take(sizeof(uint32_t) * VN);
  L.dvals1 = take(sizeof(uint32_t) * VN);
  L.drec = take(sizeof(uint4) * VN);
  L.dcnt = take(sizeof(uint32_t) * VN);
  L.offs = take(sizeof(uint64_t) * VN);
  L.tkeys0 = take(sizeof(uint32_t) * capacity);
  L.tkeys1 = take(sizeof(uint32_t) * capacity);
  L.pids1 = take(sizeof(uint32_t) * capacity);
  L.sort = take(sort_space_bytes(nmax));  // the depth sort's, then the tile sort's
  // block sums of the scans
  L.sums = take(sizeof(uint64_t) * ((nmax + kTile - 1) / kTile + 1));
  L.scal = take(64);
  L.total = o;
  return L;
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

// Heavy-first order of up to kOrderOneBlock tiles in one workgroup: a stable
// counting sort by the order key (the same key as k_order_keys).  The tiles
// are taken in chunks of 1024, wave w holding tiles [64 w, 64 w + 64) of a
// chunk, so ranks counted per wave and combined in wave order are stable.
constexpr int kOrderThreads = 1024;
constexpr int kOrderWaves = kOrderThreads / 64;
constexpr int64_t kOrderOneBlock = 16384;

__device__ __forceinline__ uint32_t order_key(const uint32_t* __restrict__ ranges, int64_t t) {
  const uint32_t len = ranges[2 * t + 1] - ranges[2 * t];
  const int b = len == 0 ? 0 : min(255, (int)(16.0f * __log2f((float)len + 1.0f)));
  return (uint32_t)(255 - b);
}

__global__ void __launch_bounds__(kOrderThreads)
k_tile_order(const uint32_t* __restrict__ ranges, int64_t tiles, uint32_t* __restrict__ order) {
  __shared__ uint32_t base[kRadix];                 // next position of each key
  __shared__ uint32_t wcnt[kOrderWaves][kRadix];    // per-wave key counts of a chunk
  __shared__ uint8_t keys[kOrderOneBlock];          // every tile's key, computed once
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (threadIdx.x < kRadix) base[threadIdx.x] = 0u;
  __syncthreads();
#pragma unroll 8
  for (int64_t t = threadIdx.x; t < tiles; t += kOrderThreads) {
    const uint32_t k = order_key(ranges, t);
    keys[t] = (uint8_t)k;
    atomicAdd(&base[k], 1u);
  }
  __syncthreads();
  if (threadIdx.x < 64) {  // exclusive scan of the 256 key counts by wave 0
    uint32_t c[4], s = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) { c[k] = base[4 * lane + k]; s += c[k]; }
    uint32_t x = s;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t y = __shfl_up(x, d, 64);
      if (lane >= d) x += y;
    }
    uint32_t run = x - s;
#pragma unroll
    for (int k = 0; k < 4; ++k) { base[4 * lane + k] = run; run += c[k]; }
  }
  const uint64_t lt = lanes_below();
  for (int64_t c0 = 0; c0 < tiles; c0 += kOrderThreads) {
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kRadix / 64; ++k) wcnt[wave][k * 64 + lane] = 0u;
    const int64_t t = c0 + threadIdx.x;
    const bool valid = t < tiles;
    const uint32_t d = valid ? (uint32_t)keys[t] : 0u;
    const uint64_t peers = digit_peers(d, valid);
    const uint32_t rank = (uint32_t)__popcll(peers & lt);
    if (valid && rank == 0) wcnt[wave][d] = (uint32_t)__popcll(peers);
    __syncthreads();
    if (threadIdx.x < kRadix) {  // per-wave starts of each key in this chunk
      uint32_t run = base[threadIdx.x];
      for (int w = 0; w < kOrderWaves; ++w) {
        const uint32_t x = wcnt[w][threadIdx.x];
        wcnt[w][threadIdx.x] = run;
        run += x;
      }
      base[threadIdx.x] = run;
    }
    __syncthreads();
    if (valid) order[wcnt[wave][d] + rank] = (uint32_t)t;
  }
  if (threadIdx.x == 0) order[tiles] = 0u;  // the work-queue counter's slot
}

}  // namespace

size_t tile_order_workspace(int64_t tiles) {
  return align_up(sizeof(uint32_t) * tiles) * 3 + sort_space_bytes(tiles) + 256;
}

hipError_t launch_tile_order(const uint32_t* ranges, int64_t tiles, uint32_t* order, void* ws,
                             hipStream_t st) {
  char* w = static_cast<char*>(ws);
  uint32_t* k0 = (uint32_t*)w;
  uint32_t* v0 = (uint32_t*)(w + align_up(sizeof(uint32_t) * tiles));
  uint32_t* k1 = (uint32_t*)(w + 2 * align_up(sizeof(uint32_t) * tiles));
  char* sw = w + 3 * align_up(sizeof(uint32_t) * tiles);
  uint32_t* cnt = (uint32_t*)(sw + sort_space_bytes(tiles));
  if (tiles <= kOrderOneBlock) {
    hipLaunchKernelGGL(k_tile_order, dim3(1), dim3(kOrderThreads), 0, st, ranges, tiles, order);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_order_keys, dim3(blocks_for(tiles > 0 ? tiles : 1, kThreads)),
                     dim3(kThreads), 0, st, ranges, tiles, k0, v0, cnt);
  // one 8-bit pass: the result lands in (k1, order)
  radix_sort(k0, v0, k1, order, tiles, cnt, 8, sort_space(sw, tiles), st);
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(kThreads), 0, st, order + tiles, 1, 0u);
  return hipGetLastError();
}

size_t bin_sort_workspace(int64_t VN, int64_t capacity) { return layout(VN, capacity).total; }

hipError_t launch_bin_sort(const rade_settings& s, const rade_view* views_host,
                           const rade_view* views_dev, int V, int64_t N,
                           const int32_t* tt, const uint32_t* bin_records, uint32_t* pair_ids,
                           uint32_t* ranges, uint64_t* keys, int64_t capacity,
                           int64_t* n_pairs_dev, int64_t* n_pairs_host, void* ws,
                           hipStream_t st, int* capacity_exceeded) {
  *capacity_exceeded = 0;
  const int64_t VN = (int64_t)V * N;
  const Layout L = layout(VN, capacity);
  char* w = static_cast<char*>(ws);
  uint32_t* starts = (uint32_t*)(w + L.starts);
  uint32_t* dk0 = (uint32_t*)(w + L.dkeys0);
  uint32_t* dv0 = (uint32_t*)(w + L.dvals0);
  uint32_t* dk1 = (uint32_t*)(w + L.dkeys1);
  uint32_t* dv1 = (uint32_t*)(w + L.dvals1);
  const uint4* brecs = reinterpret_cast<const uint4*>(bin_records);
  uint4* drec = (uint4*)(w + L.drec);
  uint32_t* dcnt = (uint32_t*)(w + L.dcnt);
  uint64_t* offs = (uint64_t*)(w + L.offs);
  uint32_t* tk0 = (uint32_t*)(w + L.tkeys0);
  uint32_t* tk1 = (uint32_t*)(w + L.tkeys1);
  uint32_t* pid1 = (uint32_t*)(w + L.pids1);
  char* sortw = w + L.sort;
  void* sums = (void*)(w + L.sums);
  uint32_t* n_vis = (uint32_t*)(w + L.scal);
  uint64_t* m64 = (uint64_t*)(w + L.scal + 8);
  uint32_t* m32 = (uint32_t*)(w + L.scal + 16);

  int64_t total_tiles = 0;
  for (int v = 0; v < V; ++v)
    total_tiles += (int64_t)views_host[v].tiles_x * views_host[v].tiles_y;

  // 1. visible splats -> compact (depth key, index) list
  if (VN > 0) {
    scan_emit<uint32_t>(Visible{tt}, VN, (uint32_t*)sums, n_vis,
                        VisibleOut{brecs, dk0, dv0},
                        st);
  } else {
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(kThreads), 0, st, n_vis, 1, 0u);
  }
  // 2. depth sort
  radix_sort(dk0, dv0, dk1, dv1, VN, n_vis, 32, sort_space(sortw, VN), st, false, brecs, drec,
             dcnt);
  // 3. pair offsets in depth order (and the pair counts)
  if (VN > 0) {
    scan_to<uint64_t>(SortedCount{dcnt}, VN, n_vis,
                      OffsetsOut{offs, starts, (capacity + kEmitPairs - 1) / kEmitPairs},
                      (uint64_t*)sums, PairsTotal{m64, m32, capacity, n_pairs_dev}, st);
  } else {
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(kThreads), 0, st, (uint32_t*)m64, 2, 0u);
    hipLaunchKernelGGL(k_finish_counts, dim3(1), dim3(1), 0, st, m64, capacity, m32, n_pairs_dev);
  }
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
  const int trb = digit_bits(tbits);
  const int tpasses = tbits > trb ? (tbits + trb - 1) / trb : 1;
  uint32_t* ek = tk0;
  uint32_t* ev = (tpasses & 1) ? pid1 : pair_ids;
  uint32_t* ok_ = tk1;
  uint32_t* ov = (tpasses & 1) ? pair_ids : pid1;
  // (the emission also counts the tile sort's first digits, per block)
  const SortSpace tsp = sort_space(sortw, capacity);
  const bool emitted = VN > 0 && capacity > 0;
  static_assert(kEmitPairs == kTile, "emission blocks are the tile sort's blocks");
  if (emitted) {
    const int vec = (((uintptr_t)ek | (uintptr_t)ev) & 15) == 0 ? 1 : 0;
    const FastDiv divn((uint32_t)(N > 0 ? N : 1));
    if (trb == 9)
      hipLaunchKernelGGL(k_emit<9>, dim3((unsigned)sort_blocks(capacity)), dim3(kEmitThreads), 0,
                         st, (const uint4*)drec, offs, starts, n_vis, m64, capacity, views_dev,
                         divn, ek, ev, vec, sort_blocks(capacity), tsp.hist);
    else
      hipLaunchKernelGGL(k_emit<kRadixBits>, dim3((unsigned)sort_blocks(capacity)),
                         dim3(kEmitThreads), 0, st, (const uint4*)drec, offs, starts, n_vis, m64,
                         capacity, views_dev, divn, ek, ev, vec, sort_blocks(capacity), tsp.hist);
  }
  // 5. stable sort by tile
  radix_sort(ek, ev, ok_, ov, capacity, m32, tbits, tsp, st, emitted);
  uint32_t* sk = (tpasses & 1) ? ok_ : ek;
  // 6. tile ranges
  if (capacity > 0)
    hipLaunchKernelGGL(k_ranges, dim3(blocks_for(capacity + 1, kRangeKeys * kThreads)),
                       dim3(kThreads), 0, st, sk, m32, total_tiles, ranges);
  else
    hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for(2 * total_tiles, kThreads)), dim3(kThreads), 0,
                       st, ranges, 2 * total_tiles, 0u);
  // 7. optional 64-bit keys
  if (keys && capacity > 0)
    hipLaunchKernelGGL(k_keys, dim3(blocks_for(capacity, kThreads)), dim3(kThreads), 0, st, sk,
                       pair_ids, m32, brecs, views_dev, V, N, keys);
  return hipGetLastError();
}

}  // namespace rade
