// tc_field.hpp -- arithmetic modulo p = 2^64 - 2^32 + 1, the field of the
// number-theoretic transform that forms leaf products (section 5's FFT
// product under a Toom-Cook level).
//
// 2^64 = 2^32 - 1 (mod p) and 2^96 = -1 (mod p), so a 128-bit product
// hi 2^64 + lo with hi = h1 2^32 + h0 reduces to lo + h0 (2^32 - 1) - h1:
// two 64-bit additions with their wrap-arounds folded back in, and one final
// conditional subtraction.  Every function takes and returns values below p.
#pragma once
#include <stdint.h>

#ifndef TC_HD
#define TC_HD __host__ __device__ __forceinline__
#endif

namespace tc {

constexpr uint64_t kFieldP = 0xFFFFFFFF00000001ull;
constexpr uint64_t kFieldEps = 0xFFFFFFFFull;  // 2^64 - p = 2^64 mod p

TC_HD uint64_t fp_add(uint64_t a, uint64_t b) {
  uint64_t s = a + b;
  if (s < a) s += kFieldEps;  // a + b >= 2^64: 2^64 = 2^32 - 1 (mod p)
  if (s >= kFieldP) s -= kFieldP;
  return s;
}

TC_HD uint64_t fp_sub(uint64_t a, uint64_t b) {
  uint64_t d = a - b;
  if (a < b) d -= kFieldEps;  // a - b + 2^64, minus (2^64 - p)
  return d;
}

TC_HD uint64_t fp_mulhi(uint64_t a, uint64_t b) {
#ifdef __HIP_DEVICE_COMPILE__
  return __umul64hi(a, b);
#else
  return (uint64_t)(((unsigned __int128)a * b) >> 64);
#endif
}

TC_HD uint64_t fp_mul(uint64_t a, uint64_t b) {
  const uint64_t lo = a * b, hi = fp_mulhi(a, b);
  const uint64_t h1 = hi >> 32, h0 = hi & kFieldEps;
  uint64_t t = lo - h1;
  if (lo < h1) t -= kFieldEps;       // borrow: add p
  const uint64_t m = (h0 << 32) - h0;  // h0 (2^32 - 1), below 2^64
  uint64_t r = t + m;
  if (r < m) r += kFieldEps;          // carry: 2^64 = 2^32 - 1 (mod p)
  if (r >= kFieldP) r -= kFieldP;
  return r;
}

}  // namespace tc
