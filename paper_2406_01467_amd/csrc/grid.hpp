// Index arithmetic of dense voxel grids (x fastest) with 32-bit linear
// indices (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace rade {

// Division of 32-bit unsigned integers by an invariant divisor with one
// high multiply, a subtraction and two shifts: the round-up method of
// Granlund and Montgomery, "Division by invariant integers using
// multiplication" (PLDI 1994).  With l = ceil(log2 d) and
// m = floor(2^32 (2^l - d) / d) + 1, t = mulhi(m, n) and
// n / d = (t + ((n - t) >> 1)) >> (l - 1) for every n < 2^32 (d > 1).
struct FastDiv {
  uint32_t d = 1, m = 1;
  int l = 0;
  constexpr FastDiv() = default;
  constexpr explicit FastDiv(uint32_t divisor) : d(divisor), m(1), l(0) {
    while (l < 32 && ((uint64_t)1 << l) < (uint64_t)d) ++l;
    m = (uint32_t)((((uint64_t)1 << 32) * (((uint64_t)1 << l) - d)) / d + 1);
  }
  __host__ __device__ constexpr uint32_t div(uint32_t n) const {
    if (l == 0) return n;  // d == 1
    const uint32_t t = (uint32_t)(((uint64_t)m * n) >> 32);
    return (t + ((n - t) >> 1)) >> (l - 1);
  }
};

constexpr bool fastdiv_selfcheck() {
  const uint32_t ds[] = {1u, 2u, 3u, 5u, 7u, 64u, 100u, 310u, 433u, 511u, 1000u, 65535u,
                         65537u, 2147483647u, 2147483648u, 2147483649u, 4294967295u};
  const uint32_t ns[] = {0u, 1u, 2u, 3u, 63u, 64u, 65u, 999u, 1000u, 123456789u, 2147483647u,
                         2147483648u, 3000000000u, 4294967294u, 4294967295u};
  for (uint32_t d : ds) {
    const FastDiv f(d);
    for (uint32_t n : ns) {
      if (f.div(n) != n / d) return false;
      if (n >= 1 && f.div(n - 1) != (n - 1) / d) return false;
    }
    // around multiples of d
    for (uint64_t k = 1; k < 4; ++k) {
      const uint64_t x = k * (uint64_t)d;
      if (x <= 0xFFFFFFFFull) {
        if (f.div((uint32_t)x) != (uint32_t)(x / d)) return false;
        if (f.div((uint32_t)(x - 1)) != (uint32_t)((x - 1) / d)) return false;
      }
    }
  }
  return true;
}
static_assert(fastdiv_selfcheck(), "division by invariant integers");

// (i, j, k) of linear index q = (k ny + j) nx + i.
struct Grid3 {
  FastDiv fx, fy;  // divisions by nx and ny
  uint32_t nx = 1, ny = 1;
  Grid3() = default;
  Grid3(uint32_t nx_, uint32_t ny_) : fx(nx_), fy(ny_), nx(nx_), ny(ny_) {}
  __device__ __forceinline__ void split(uint32_t q, uint32_t& i, uint32_t& j,
                                        uint32_t& k) const {
    const uint32_t r = fx.div(q);
    i = q - r * nx;
    k = fy.div(r);
    j = r - k * ny;
  }
};

}  // namespace rade
