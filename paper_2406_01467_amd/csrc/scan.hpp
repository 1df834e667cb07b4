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

// Phase 3: per-block exclusive scan plus the block's offset.
template <typename T, typename In>
__global__ void __launch_bounds__(kScanThreads)
k_scan_down(In in, int64_t n_max, const uint32_t* n_dev, const T* block_sums, T* out) {
  __shared__ T lw[kScanThreads / 64];
  const int64_t n = n_dev ? (int64_t)*n_dev : n_max;
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  if ((int64_t)blockIdx.x * kScanTile >= n) return;  // uniform per block
  T v[kScanItems];
  T s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = (base + k < n) ? in(base + k) : 0;
    s += v[k];
  }
  T total;
  T run = block_exclusive_scan<T>(s, lw, total) + block_sums[blockIdx.x];
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    if (base + k < n) out[base + k] = run;
    run += v[k];
  }
}

// Exclusive scan of in(0..n) into out (n = *n_dev, or n_max when n_dev is
// NULL), total into *total.  Launch errors are left pending for the
// caller's final hipGetLastError.
template <typename T, typename In>
void scan(In in, int64_t n_max, const uint32_t* n_dev, T* out, T* block_sums, T* total,
          hipStream_t st) {
  const int64_t nb = n_max > 0 ? (n_max + kScanTile - 1) / kScanTile : 1;
  hipLaunchKernelGGL((k_scan_reduce<T, In>), dim3((unsigned)nb), dim3(kScanThreads), 0, st, in,
                     n_max, n_dev, block_sums);
  hipLaunchKernelGGL((k_scan_top<T>), dim3(1), dim3(kScanThreads), 0, st, block_sums, nb, total);
  hipLaunchKernelGGL((k_scan_down<T, In>), dim3((unsigned)nb), dim3(kScanThreads), 0, st, in, n_max,
                     n_dev, block_sums, out);
}

}  // namespace rade
