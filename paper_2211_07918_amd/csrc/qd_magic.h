// Division of 32-bit unsigned integers by a run-time invariant divisor through one multiply-high,
// after Granlund and Montgomery, "Division by invariant integers using multiplication" (PLDI 1994),
// Sec. 4 (the round-up method for N = 32 with the two-step shift that avoids a 33-bit multiplier).
//
// For every divisor 1 <= d < 2^32 and every n < 2^32:
//   l  = ceil(log2 d),  mul = floor(2^32 (2^l - d) / d) + 1,
//   t  = mulhi(mul, n),  n / d = (t + ((n - t) >> min(l, 1))) >> max(l - 1, 0).
//
// Plain C++ on the host (testable with any C++ compiler), inlined into kernels on the device.
#pragma once

#include <cstdint>

#if defined(__HIPCC__)
#define QD_HD __host__ __device__ __forceinline__
#else
#define QD_HD inline
#endif

namespace qd {

struct Magic32 {
  uint32_t mul;
  uint32_t sh1;
  uint32_t sh2;
  uint32_t d;
};

inline Magic32 make_magic32(uint32_t d) {
  Magic32 m{};
  m.d = d;
  uint32_t l = 0;
  while (l < 32 && (uint64_t(1) << l) < uint64_t(d)) ++l;
  const uint64_t two_l = uint64_t(1) << l;                 // 2^l, l <= 32
  // floor(2^32 * (2^l - d) / d) + 1 fits in 32 bits because 2^l - d < d.
  const unsigned __int128 num = (unsigned __int128)(two_l - d) << 32;
  m.mul = uint32_t(uint64_t(num / d) + 1);
  m.sh1 = l < 1 ? l : 1;
  m.sh2 = l > 1 ? l - 1 : 0;
  return m;
}

QD_HD uint32_t mulhi32(uint32_t a, uint32_t b) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __umulhi(a, b);
#else
  return uint32_t((uint64_t(a) * uint64_t(b)) >> 32);
#endif
}

QD_HD uint32_t magic_div(uint32_t n, const Magic32& m) {
  const uint32_t t = mulhi32(m.mul, n);
  return (t + ((n - t) >> m.sh1)) >> m.sh2;
}

}  // namespace qd
