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

// The 128-bit product from four 32 x 32 -> 64 multiply-adds (each partial
// sum fits 64 bits: (2^32-1)^2 + 2 (2^32-1) = 2^64 - 1).
TC_HD void fp_mul128(uint64_t a, uint64_t b, uint64_t& lo, uint64_t& hi) {
  const uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32);
  const uint32_t b0 = (uint32_t)b, b1 = (uint32_t)(b >> 32);
  const uint64_t p00 = (uint64_t)a0 * b0;
  const uint64_t t = (uint64_t)a0 * b1 + (p00 >> 32);
  const uint64_t u = (uint64_t)a1 * b0 + (uint32_t)t;
  lo = (p00 & kFieldEps) | (u << 32);
  hi = (uint64_t)a1 * b1 + (t >> 32) + (u >> 32);
}

TC_HD uint64_t fp_mul(uint64_t a, uint64_t b) {
  uint64_t lo, hi;
  fp_mul128(a, b, lo, hi);
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
