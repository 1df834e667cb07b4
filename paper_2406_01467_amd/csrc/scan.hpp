// Three-kernel exclusive scan (reduce, scan of the block sums, down-sweep)
// over an item functor, shared by the binning sort and mesh extraction
// (gfx950).  Item counts may live in device memory (n_dev), so a sequence of
// scans can be captured in a HIP graph: grids are sized for the capacity
// and surplus blocks exit.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace rade {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;                              // items per thread
constexpr int kScanTile = kScanThreads * kScanItems;       // items per block

// ---------------------------------------------------------------------------
// Block-wide exclusive scan of one value per thread (256 threads, 4 waves).
template <typename T>
__device__ __forceinline__ T block_exclusive_scan(T v, T* lds_waves, T& total) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  T x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const T y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) lds_waves[wave] = x;
  __syncthreads();
  T pre = 0;
  total = 0;
#pragma unroll
  for (int w = 0; w < kScanThreads / 64; ++w) {
    const T s = lds_waves[w];
    if (w < wave) pre += s;
    total += s;
  }
  __syncthreads();
  return pre + x - v;
}

// Sum of sums[0..b) by the whole workgroup (every thread gets it): the
// exclusive prefix of block b among the block sums, for scans whose blocks
// are few enough that each can add up those before it (kFoldBlocks), which
// saves the separate kernel that scans the block sums.
constexpr int64_t kFoldBlocks = 1024;

template <typename T>
__device__ __forceinline__ T block_prefix(const T* __restrict__ sums, int64_t b, T* lds_waves) {
  T s = 0;
#pragma unroll 4
  for (int64_t i = threadIdx.x; i < b; i += kScanThreads) s += sums[i];
  T tot;
  block_exclusive_scan<T>(s, lds_waves, tot);
  return tot;
}

// Where a scan's total goes.
template <typename T>
struct TotalStore {
  T* p;
  __device__ void operator()(T t) const {
    if (p) *p = t;
  }
};

struct PlainInput64 {
  const uint64_t* a;
  __device__ uint64_t operator()(int64_t i) const { return a[i]; }
};
struct PlainInput {
  const uint32_t* a;
  __device__ uint32_t operator()(int64_t i) const { return a[i]; }
};

// Phase 1: per-block sums.
template <typename T, typename In>
__global__ void __launch_bounds__(kScanThreads)
k_scan_reduce(In in, int64_t n_max, const uint32_t* n_dev, T* block_sums) {
  __shared__ T lw[kScanThreads / 64];
  const int64_t n = n_dev ? (int64_t)*n_dev : n_max;
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  T s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k)
    if (base + k < n) s += in(base + k);
  T total;
  block_exclusive_scan<T>(s, lw, total);
  if (threadIdx.x == 0) block_sums[blockIdx.x] = total;
}

// Phase 2: exclusive scan of the block sums in one block; writes the total.
template <typename T>
__global__ void __launch_bounds__(kScanThreads)
k_scan_top(T* block_sums, int64_t nb, T* total_out) {
  __shared__ T lw[kScanThreads / 64];
  T carry = 0;
  for (int64_t base = 0; base < nb; base += kScanThreads) {
    const int64_t i = base + threadIdx.x;
    const T v = i < nb ? block_sums[i] : 0;
    T tot;
    const T ex = block_exclusive_scan<T>(v, lw, tot);
    if (i < nb) block_sums[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0 && total_out) *total_out = carry;
}

// Phase 3: per-block exclusive scan plus the block's offset, handed to
// out(item, offset, count).
template <typename T>
struct StoreOut {
  T* a;
  __device__ void operator()(int64_t i, T offset, T) const { a[i] = offset; }
};

template <typename T, typename In, typename Out, typename Tot>
__global__ void __launch_bounds__(kScanThreads)
k_scan_down(In in, int64_t n_max, const uint32_t* n_dev, const T* block_sums, int fold, Out out,
            Tot total) {
  __shared__ T lw[kScanThreads / 64];
  const int64_t n = n_dev ? (int64_t)*n_dev : n_max;
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  if (n == 0) {
    if (blockIdx.x == 0 && threadIdx.x == 0) total(T(0));
    return;
  }
  if ((int64_t)blockIdx.x * kScanTile >= n) return;  // uniform per block
  T v[kScanItems];
  T s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = (base + k < n) ? in(base + k) : 0;
    s += v[k];
  }
  T sum;
  const T ex = block_exclusive_scan<T>(s, lw, sum);
  const T pre = fold ? block_prefix<T>(block_sums, blockIdx.x, lw) : block_sums[blockIdx.x];
  T run = ex + pre;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    if (base + k < n) out(base + k, run, v[k]);
    run += v[k];
  }
  // the block holding the last item has the total
  if (threadIdx.x == 0 && (int64_t)blockIdx.x == (n - 1) / kScanTile) total(pre + sum);
}

// Exclusive scan of in(0..n) handed to out (n = *n_dev, or n_max when n_dev
// is NULL), the total handed to total().  Two kernels when the blocks are
// few enough (kFoldBlocks), else three.  Launch errors are left pending for
// the caller's final hipGetLastError.
template <typename T, typename In, typename Out, typename Tot>
void scan_to(In in, int64_t n_max, const uint32_t* n_dev, Out out, T* block_sums, Tot total,
             hipStream_t st) {
  const int64_t nb = n_max > 0 ? (n_max + kScanTile - 1) / kScanTile : 1;
  const int fold = nb <= kFoldBlocks ? 1 : 0;
  hipLaunchKernelGGL((k_scan_reduce<T, In>), dim3((unsigned)nb), dim3(kScanThreads), 0, st, in,
                     n_max, n_dev, block_sums);
  if (!fold)
    hipLaunchKernelGGL((k_scan_top<T>), dim3(1), dim3(kScanThreads), 0, st, block_sums, nb,
                       (T*)nullptr);
  hipLaunchKernelGGL((k_scan_down<T, In, Out, Tot>), dim3((unsigned)nb), dim3(kScanThreads), 0, st,
                     in, n_max, n_dev, (const T*)block_sums, fold, out, total);
}

// The same, stored into out[0..n).
template <typename T, typename In>
void scan(In in, int64_t n_max, const uint32_t* n_dev, T* out, T* block_sums, T* total,
          hipStream_t st) {
  scan_to<T>(in, n_max, n_dev, StoreOut<T>{out}, block_sums, TotalStore<T>{total}, st);
}

// Compaction: the exclusive scan of in() is handed, for every item with a
// nonzero count, to emit(item, offset, count) instead of being stored.  The
// counts are evaluated twice (reduce and emit) and never stored.  A fixed
// grid of at most kCompactBlocks workgroups each walks a contiguous chunk of
// items in rounds of 256 consecutive items, one per thread (so a wave's
// loads are coalesced), kCompactBatch rounds at a time: all their counts are
// loaded first, scanned within each wave by shuffles, and combined across
// the four waves after one barrier; a batch whose counts are all zero is
// skipped after a single block-wide vote.  The running offset is carried from
// batch to batch; the scan of the per-workgroup sums stays short for any
// item count.
constexpr int64_t kCompactBlocks = 8192;
constexpr int64_t kCompactRound = kScanThreads;
constexpr int kCompactBatch = 8;
constexpr int64_t kCompactStep = kCompactRound * kCompactBatch;

template <typename T, typename In>
__global__ void __launch_bounds__(kScanThreads)
k_compact_reduce(In in, int64_t n, int64_t chunk, T* block_sums) {
  __shared__ T lw[kScanThreads / 64];
  const int64_t lo = (int64_t)blockIdx.x * chunk;
  const int64_t hi = lo + chunk < n ? lo + chunk : n;
  T s = 0;
  for (int64_t r = lo; r < hi; r += kCompactStep) {
    T v[kCompactBatch];
#pragma unroll
    for (int k = 0; k < kCompactBatch; ++k) {
      const int64_t i = r + k * kCompactRound + threadIdx.x;
      v[k] = i < hi ? in(i) : 0;
    }
#pragma unroll
    for (int k = 0; k < kCompactBatch; ++k) s += v[k];
  }
  T total;
  block_exclusive_scan<T>(s, lw, total);
  if (threadIdx.x == 0) block_sums[blockIdx.x] = total;
}

template <typename T, typename In, typename Emit>
__global__ void __launch_bounds__(kScanThreads)
k_compact_emit(In in, int64_t n, int64_t chunk, const T* block_sums, int fold, Emit emit,
               T* total) {
  constexpr int W = kScanThreads / 64;
  __shared__ T lw[kCompactBatch][W];
  __shared__ T lwp[W];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t lo = (int64_t)blockIdx.x * chunk;
  const int64_t hi = lo + chunk < n ? lo + chunk : n;
  T carry = fold ? block_prefix<T>(block_sums, blockIdx.x, lwp) : block_sums[blockIdx.x];
  for (int64_t r = lo; r < hi; r += kCompactStep) {  // uniform trip count
    T v[kCompactBatch], incl[kCompactBatch];
    int any = 0;
#pragma unroll
    for (int k = 0; k < kCompactBatch; ++k) {
      const int64_t i = r + k * kCompactRound + threadIdx.x;
      v[k] = i < hi ? in(i) : 0;
      any |= v[k] != 0 ? 1 : 0;
    }
    // a batch of zero counts (most of a sparse surface's grid) emits nothing
    if (!__syncthreads_or(any)) continue;
#pragma unroll
    for (int k = 0; k < kCompactBatch; ++k) {
      T x = v[k];
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const T y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
      }
      incl[k] = x;
      if (lane == 63) lw[k][wave] = x;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kCompactBatch; ++k) {
      T round_total = 0, before = 0;
#pragma unroll
      for (int w = 0; w < W; ++w) {
        const T t = lw[k][w];
        round_total += t;
        if (w < wave) before += t;
      }
      if (v[k]) emit(r + k * kCompactRound + threadIdx.x, carry + before + incl[k] - v[k], v[k]);
      carry += round_total;
    }
    __syncthreads();
  }
  // the last workgroup's carry is the total
  if (total && threadIdx.x == 0 && blockIdx.x == gridDim.x - 1) *total = carry;
}

// Workgroups and block-sum entries a compaction of n items uses.
inline int64_t compact_blocks(int64_t n) {
  const int64_t steps = (n + kCompactStep - 1) / kCompactStep;
  return steps < kCompactBlocks ? (steps > 0 ? steps : 1) : kCompactBlocks;
}

// Enqueues the compaction of in(0..n): total into *total, emit for every
// item with a nonzero count.  block_sums holds compact_blocks(n) entries.
// Two kernels when the workgroups are few enough (kFoldBlocks), else three.
// Launch errors are left pending.
template <typename T, typename In, typename Emit>
void scan_emit(In in, int64_t n, T* block_sums, T* total, Emit emit, hipStream_t st) {
  const int64_t nb = compact_blocks(n);
  const int64_t steps = (n + kCompactStep - 1) / kCompactStep;
  const int64_t chunk = ((steps + nb - 1) / nb) * kCompactStep;
  const int fold = nb <= kFoldBlocks ? 1 : 0;
  hipLaunchKernelGGL((k_compact_reduce<T, In>), dim3((unsigned)nb), dim3(kScanThreads), 0, st,
                     in, n, chunk, block_sums);
  if (!fold)
    hipLaunchKernelGGL((k_scan_top<T>), dim3(1), dim3(kScanThreads), 0, st, block_sums, nb,
                       (T*)nullptr);
  hipLaunchKernelGGL((k_compact_emit<T, In, Emit>), dim3((unsigned)nb), dim3(kScanThreads), 0, st,
                     in, n, chunk, (const T*)block_sums, fold, emit, total);
}

}  // namespace rade
