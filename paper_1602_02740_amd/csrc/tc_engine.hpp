// tc_engine.hpp -- wave-level carry engine for long limb arrays (gfx950).
//
// Every linear pass of the Toom-Cook path (evaluation, the even-odd combine,
// the Newton loops, recomposition) has the same shape: limb p of the result
// is a small signed combination delta_p of input limbs, the sum
// sum_p delta_p 2^(32p) must then be normalised (carries), possibly divided
// exactly by one or two odd words and by a power of two, and written out.
// One 64-lane wavefront streams a value from its low limb to its high limb in
// tiles of 64*LPT limbs:
//
//   1. pre-normalise: e_p = lo32(delta_p) + (delta_{p-1} >> 32), so that every
//      carry of the following chain is -1, 0 or +1;
//   2. carries: each lane runs its LPT limbs with carry-in 0 and summarises
//      the outcome as a table {-1,0,1} -> {-1,0,1}; a Kogge-Stone scan of the
//      tables over the wave gives every lane its true carry-in;
//   3. exact division by an odd d (section 3's divided differences are exact,
//      and section 6 keeps each divisor within a 32-bit word): 2-adic
//      (Hensel) division, q_p = (x_p - r_p) d^-1 mod 2^32 with a residue
//      r_p in [0, d).  Over L limbs the residue map is affine,
//      r -> r M^L + K with M = 2^-32 mod d, so a scan of (K) with the
//      precomputed powers M^j gives every lane its incoming residue;
//   4. exact right shift by shr < 64 bits, using the next lane's first limbs
//      (lane 63 computes the next tile's first limbs itself);
//   5. store through the source's sink.
//
// Exactness is asserted, never assumed: bits shifted out must be zero and the
// final residue of each division must be 0 (non-negative quotient) or d-1
// (negative quotient in two's complement).
#pragma once
#include <hip/hip_runtime.h>

#include "tc_types.hpp"

namespace tc {

#define TC_DEV __device__ __forceinline__

TC_DEV int lane_id() { return (int)(threadIdx.x & 63u); }

// ---------------------------------------------------------------- carry tables
// A table maps a carry-in c in {-1,0,1} to a carry-out in {-1,0,1}; two bits
// per input hold out+1.
constexpr uint32_t TAB_ID = 0u | (1u << 2) | (2u << 4);

TC_DEV int tab_apply(uint32_t f, int c) { return (int)((f >> (2 * (c + 1))) & 3u) - 1; }

TC_DEV uint32_t tab_make(int fm, int f0, int fp) {
  return (uint32_t)(fm + 1) | ((uint32_t)(f0 + 1) << 2) | ((uint32_t)(fp + 1) << 4);
}

// f first, then g
TC_DEV uint32_t tab_then(uint32_t f, uint32_t g) {
  return tab_make(tab_apply(g, tab_apply(f, -1)), tab_apply(g, tab_apply(f, 0)),
                  tab_apply(g, tab_apply(f, 1)));
}

// ---------------------------------------------------------------- modular helpers
// a * M^j mod d by Shoup's method with the precomputed companion.
TC_DEV uint32_t mulmod_pw(uint32_t a, const DivEntry* de, int j) {
  const uint32_t w = de->pw[j], wp = de->pws[j], d = de->d;
  const uint32_t q = __umulhi(a, wp);
  const uint64_t r = (uint64_t)a * w - (uint64_t)q * d;
  return (uint32_t)(r >= d ? r - d : r);
}

TC_DEV uint32_t addmod(uint32_t a, uint32_t b, uint32_t d) {
  const uint64_t s = (uint64_t)a + b;
  return (uint32_t)(s >= d ? s - d : s);
}

// One limb of 2-adic exact division; r is the running residue in [0, d).
TC_DEV uint32_t hensel_step(uint32_t x, uint32_t& r, uint32_t d, uint32_t dinv) {
  const uint32_t q = (x - r) * dinv;
  const uint32_t hi = __umulhi(q, d);
  r = hi + (x < r ? 1u : 0u);
  return q;
}

struct EngCfg {
  int64_t Y;                 // limbs computed
  const DivEntry* div[2];    // odd divisors, nullptr = none
  int32_t shr;               // exact right shift, < 64
  bool is_signed;            // two's complement result (else unsigned)
  bool prenorm;              // split delta into lo/hi (|delta| may exceed 2^32)
  bool check_carry;          // unsigned: carry out of limb Y-1 must be 0
};

// Runs one value through the engine on the calling wavefront.  Src provides
//   int64_t delta(int64_t p)          for 0 <= p < Y
//   void    store(int64_t p, uint32_t o, uint32_t& errbits)
// Returns the result's limb Y-1 (all lanes).
template <int LPT, class Src>
TC_DEV uint32_t engine_run(Src& src, const EngCfg& cfg, uint32_t& errbits) {
  static_assert(LPT >= 2, "shift lookahead needs two limbs per lane");
  const int lane = lane_id();
  constexpr int T = 64 * LPT;
  const int64_t Y = cfg.Y;
  const int sq = cfg.shr >> 5, sr = cfg.shr & 31;
  const int E = sq + (sr ? 1 : 0);
  int carry = 0;
  uint32_t rin0 = 0, rin1 = 0;
  uint32_t top_out = 0;

  for (int64_t p0 = 0; p0 < Y; p0 += T) {
    const int64_t pt = p0 + (int64_t)lane * LPT;
    const int64_t rem = Y - pt;
    const int nown = rem <= 0 ? 0 : (rem >= LPT ? LPT : (int)rem);

    // 1. pre-normalised limbs
    int64_t e[LPT];
    int64_t dlast;
    {
      int64_t dprev = (cfg.prenorm && nown > 0 && pt > 0) ? src.delta(pt - 1) : 0;
#pragma unroll
      for (int i = 0; i < LPT; i++) {
        const int64_t d = i < nown ? src.delta(pt + i) : 0;
        e[i] = cfg.prenorm ? ((d & 0xffffffffll) + (dprev >> 32)) : d;
        dprev = d;
      }
      dlast = dprev;
    }

    // 2. carries
    uint32_t x[LPT];
    int cout;
    {
      int c = 0;
      bool ones = true, zeros = true;
#pragma unroll
      for (int i = 0; i < LPT; i++) {
        if (i < nown) {
          const int64_t s = e[i] + c;
          x[i] = (uint32_t)s;
          c = (int)(s >> 32);
          ones = ones && x[i] == 0xffffffffu;
          zeros = zeros && x[i] == 0u;
        }
      }
      const uint32_t tab = nown ? tab_make(c - (zeros ? 1 : 0), c, c + (ones ? 1 : 0)) : TAB_ID;
      uint32_t inc = tab;
#pragma unroll
      for (int dist = 1; dist < 64; dist <<= 1) {
        const uint32_t y = __shfl_up(inc, dist);
        if (lane >= dist) inc = tab_then(y, inc);
      }
      uint32_t exc = __shfl_up(inc, 1);
      if (lane == 0) exc = TAB_ID;
      const int cin = tab_apply(exc, carry);
      const int next_carry = tab_apply(__shfl(inc, 63), carry);
      c = cin;
#pragma unroll
      for (int i = 0; i < LPT; i++) {
        if (i < nown) {
          const int64_t s = e[i] + c;
          x[i] = (uint32_t)s;
          c = (int)(s >> 32);
        }
      }
      cout = c;
      carry = next_carry;
      if (cfg.check_carry && nown > 0 && pt + nown == Y && c != 0) errbits |= ERRBIT_RANGE;
    }

    // 3. exact divisions by odd words
    uint32_t rcur0 = 0, rcur1 = 0;
#pragma unroll
    for (int dv = 0; dv < 2; dv++) {
      const DivEntry* de = cfg.div[dv];
      if (!de) continue;
      const uint32_t d = de->d, dinv = de->dinv;
      uint32_t K = 0;
#pragma unroll
      for (int i = 0; i < LPT; i++)
        if (i < nown) (void)hensel_step(x[i], K, d, dinv);
#pragma unroll
      for (int dist = 1; dist < 64; dist <<= 1) {
        const uint32_t Ky = __shfl_up(K, dist);
        if (lane >= dist) K = addmod(mulmod_pw(Ky, de, dist * LPT), K, d);
      }
      uint32_t Kx = __shfl_up(K, 1);
      if (lane == 0) Kx = 0;
      const uint32_t K63 = __shfl(K, 63);
      const uint32_t rt = dv == 0 ? rin0 : rin1;
      uint32_t r = addmod(mulmod_pw(rt, de, lane * LPT), Kx, d);
      const uint32_t rnext = addmod(mulmod_pw(rt, de, 64 * LPT), K63, d);
#pragma unroll
      for (int i = 0; i < LPT; i++)
        if (i < nown) x[i] = hensel_step(x[i], r, d, dinv);
      // the last limb of the value: the quotient's sign decides the residue
      if (nown > 0 && pt + nown == Y) {
        uint32_t qtop = 0;
#pragma unroll
        for (int i = 0; i < LPT; i++)
          if (i == nown - 1) qtop = x[i];
        const uint32_t want = (qtop >> 31) ? d - 1u : 0u;
        if (r != want) errbits |= ERRBIT_DIV;
      }
      if (dv == 0) {
        rcur0 = r;
        rin0 = rnext;
      } else {
        rcur1 = r;
        rin1 = rnext;
      }
    }

    // 4. lookahead: lane 63 continues into the next tile for the shift
    uint32_t la0 = 0, la1 = 0;
    if (E > 0 && p0 + T < Y && lane == 63) {
      int64_t dprev = dlast;
      int c = cout;
      uint32_t r0 = rcur0, r1 = rcur1;
      for (int i = 0; i < E; i++) {
        const int64_t p = p0 + T + i;
        if (p >= Y) break;
        const int64_t d = src.delta(p);
        const int64_t ee = cfg.prenorm ? ((d & 0xffffffffll) + (dprev >> 32)) : d;
        dprev = d;
        const int64_t s = ee + c;
        uint32_t xx = (uint32_t)s;
        c = (int)(s >> 32);
        if (cfg.div[0]) xx = hensel_step(xx, r0, cfg.div[0]->d, cfg.div[0]->dinv);
        if (cfg.div[1]) xx = hensel_step(xx, r1, cfg.div[1]->d, cfg.div[1]->dinv);
        if (i == 0) la0 = xx; else la1 = xx;
      }
    }

    // sign extension of the result's top limb, for positions >= Y
    uint32_t sext = 0;
    if (cfg.is_signed && Y - 1 < p0 + T + E) {
      uint32_t mine = 0;
#pragma unroll
      for (int i = 0; i < LPT; i++)
        if (pt + i == Y - 1) mine = x[i];
      uint32_t topq;
      if (Y - 1 < p0 + T) {
        topq = __shfl(mine, (int)((Y - 1 - p0) / LPT));
      } else {
        const uint32_t l = (Y - 1 - (p0 + T)) == 0 ? la0 : la1;
        topq = __shfl(l, 63);
      }
      sext = (topq >> 31) ? 0xffffffffu : 0u;
    }

    // 5. shift and store
    uint32_t nx0 = __shfl_down(x[0], 1);
    uint32_t nx1 = __shfl_down(x[1], 1);
    if (lane == 63) {
      nx0 = la0;
      nx1 = la1;
    }
    if (pt + LPT >= Y) nx0 = sext;
    if (pt + LPT + 1 >= Y) nx1 = sext;
    uint32_t q[LPT + 2];
#pragma unroll
    for (int i = 0; i < LPT; i++) q[i] = (pt + i < Y) ? x[i] : sext;
    q[LPT] = nx0;
    q[LPT + 1] = nx1;
    if (pt == 0 && cfg.shr > 0) {
      // section 3's divisions are exact: the bits shifted out are zero
      const uint32_t low = sq ? q[1] : q[0];
      if ((sq && q[0] != 0u) || (sr && (low & ((1u << sr) - 1u)) != 0u)) errbits |= ERRBIT_SHIFT;
    }
#pragma unroll
    for (int i = 0; i < LPT; i++) {
      if (i < nown) {
        const uint32_t lo = sq ? q[i + 1] : q[i];
        const uint32_t hi = sq ? q[i + 2] : q[i + 1];
        const uint32_t o = sr ? ((lo >> sr) | (hi << (32 - sr))) : lo;
        src.store(pt + i, o, errbits);
        if (pt + i == Y - 1) top_out = o;
      }
    }
  }
  // broadcast limb Y-1 of the result from its owner
  const int64_t owner_tile0 = ((Y - 1) / T) * T;
  return __shfl(top_out, (int)((Y - 1 - owner_tile0) / LPT));
}

}  // namespace tc
