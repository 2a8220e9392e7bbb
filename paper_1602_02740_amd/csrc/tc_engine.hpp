// tc_engine.hpp -- wave-level carry engine for long limb arrays (gfx950).
//
// Every linear pass of the Toom-Cook path (evaluation, the even-odd combine,
// the Newton loops, recomposition) has the same shape: limb p of the result
// is a small signed combination delta_p of input limbs; the sum
// sum_p delta_p 2^(32p) must be normalised (carries), possibly divided
// exactly by one or two odd words and by a power of two, and written out.
//
// A value of Y limbs is cut into chunks of T = 64*LPT limbs; one 64-lane
// wavefront owns one chunk, LPT consecutive limbs per lane:
//
//   1. pre-normalise: e_p = lo32(delta_p) + (delta_{p-1} >> 32), so every
//      carry of the following chain is -1, 0 or +1;
//   2. carries: each lane runs its limbs with carry-in 0 and summarises the
//      result as a table {-1,0,1} -> {-1,0,1}; a Kogge-Stone scan of the
//      tables over the wave gives every lane its carry-in relative to the
//      chunk's;
//   3. exact division by an odd d (section 3's divided differences are exact;
//      section 6 keeps each divisor within a 32-bit word): 2-adic (Hensel)
//      division q_p = (x_p - r_p) d^-1 mod 2^32 with a residue r_p in [0, d).
//      Over L limbs the residue map is affine, r -> r M^L + K with
//      M = 2^-32 mod d, so a scan of K with precomputed powers M^j gives every
//      lane its residue;
//   4. exact right shift by shr < 64 bits, using the next lane's first limbs
//      (lane 63 computes the next chunk's first limbs itself);
//   5. store through the source's sink.
//
// Chunks of one value exchange their carry and residues by decoupled
// look-back: a chunk publishes its aggregate (carry table, residue K) as
// soon as it is known, looks back over its predecessors' aggregates until it
// meets an inclusive value, and publishes its own inclusive value.  Chunk
// indices are handed out per value by an atomic ticket, so every predecessor
// a chunk waits on is already running; every wait is bounded.
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

// ---------------------------------------------------------------- global memory
// Pointers that reach a kernel through descriptors are generic; accessed as
// such they compile to flat_* instructions, which also hold the LDS/scalar
// counter, so every scalar-load wait would wait for them too.  These helpers
// access them in the global address space.  Runs of limbs move as 16- and
// 8-byte accesses that need only dword alignment.
typedef __attribute__((address_space(1))) uint32_t g_u32;
typedef uint32_t tc_u4 __attribute__((ext_vector_type(4)));
typedef uint32_t tc_u2 __attribute__((ext_vector_type(2)));
struct __attribute__((packed, aligned(4))) tc_p4 { tc_u4 v; };
struct __attribute__((packed, aligned(4))) tc_p2 { tc_u2 v; };
typedef __attribute__((address_space(1))) tc_p4 g_p4;
typedef __attribute__((address_space(1))) tc_p2 g_p2;

TC_DEV uint32_t gld(const uint32_t* p) { return *(const g_u32*)p; }

// Wave-uniform reads of memory that earlier launches wrote: scalar loads
// through the constant address space (the scalar cache is invalidated at
// each launch), issued back to back instead of one vector load per value.
typedef __attribute__((address_space(4))) const uint32_t c_u32;
TC_DEV uint32_t sld(const uint32_t* p) { return *(c_u32*)p; }
// Device form of resolve: the per-item pointer table of a batch is read by
// scalar loads, so every resolved address stays wave-uniform.
TC_DEV uint8_t* resolve_d(const Bases& b, DPtr d) {
  if (d.buf >= BUF_TABLE0) {
    const uint32_t* t = reinterpret_cast<const uint32_t*>(b.table + (d.buf - BUF_TABLE0));
    const uint64_t lo = sld(t), hi = sld(t + 1);
    return reinterpret_cast<uint8_t*>((uintptr_t)((hi << 32) | lo)) + d.off;
  }
  uint8_t* base = d.buf == BUF_SCRATCH ? b.scratch
                  : d.buf == BUF_U     ? b.p[0]
                  : d.buf == BUF_V     ? b.p[1]
                                       : b.p[2];
  return base + d.off;
}
TC_DEV uint32_t sld_byte(const uint8_t* p) {
  const uintptr_t a = (uintptr_t)p;
  const uint32_t w = *(c_u32*)(a & ~(uintptr_t)3);
  return (w >> (8u * (uint32_t)(a & 3u))) & 0xffu;
}
TC_DEV void gst(uint32_t* p, uint32_t v) { *(g_u32*)p = v; }

// w[0..N) = p[0..N)
template <int N>
TC_DEV void gld_run(const uint32_t* p, uint32_t* w) {
  const g_u32* g = (const g_u32*)p;
#pragma unroll
  for (int i = 0; i + 4 <= N; i += 4) {
    const tc_u4 v = ((const g_p4*)(g + i))->v;
    w[i] = v.x;
    w[i + 1] = v.y;
    w[i + 2] = v.z;
    w[i + 3] = v.w;
  }
  constexpr int b = N & ~3;
  if constexpr ((N & 3) >= 2) {
    const tc_u2 v = ((const g_p2*)(g + b))->v;
    w[b] = v.x;
    w[b + 1] = v.y;
  }
  if constexpr (N & 1) w[N - 1] = g[N - 1];
}

// p[0..N) = w[0..N)
template <int N>
TC_DEV void gst_run(uint32_t* p, const uint32_t* w) {
  g_u32* g = (g_u32*)p;
#pragma unroll
  for (int i = 0; i + 4 <= N; i += 4) {
    tc_u4 v;
    v.x = w[i];
    v.y = w[i + 1];
    v.z = w[i + 2];
    v.w = w[i + 3];
    ((g_p4*)(g + i))->v = v;
  }
  constexpr int b = N & ~3;
  if constexpr ((N & 3) >= 2) {
    tc_u2 v;
    v.x = w[b];
    v.y = w[b + 1];
    ((g_p2*)(g + b))->v = v;
  }
  if constexpr (N & 1) g[N - 1] = w[N - 1];
}

// ---------------------------------------------------------------- carry tables
// A table maps a carry-in c in {-1,0,1} to a carry-out in {-1,0,1}: byte c+1
// holds out+1.  Composition is then a byte permutation: (g after f) has byte
// i = byte f_i of g, one v_perm_b32.  Byte 3 is don't-care.
constexpr uint32_t TAB_ID = 0x00020100u;
constexpr uint32_t TAB_MASK = 0x00ffffffu;

TC_DEV int tab_apply(uint32_t f, int c) { return (int)((f >> (8 * (c + 1))) & 0xffu) - 1; }

TC_DEV uint32_t tab_make(int fm, int f0, int fp) {
  return (uint32_t)(fm + 1) | ((uint32_t)(f0 + 1) << 8) | ((uint32_t)(fp + 1) << 16);
}

// f first, then g
TC_DEV uint32_t tab_then(uint32_t f, uint32_t g) {
  return __builtin_amdgcn_perm(0u, g, f & TAB_MASK);
}

// ---------------------------------------------------------------- modular helpers
// a * M^j mod d by Shoup's method with the precomputed companion.
TC_DEV uint32_t mulmod_pw(uint32_t a, const DivEntry* de, int j) {
  const uint32_t w = de->pw[j], wp = de->pws[j], d = de->d;
  const uint32_t q = __umulhi(a, wp);
  const uint64_t r = (uint64_t)a * w - (uint64_t)q * d;
  return (uint32_t)(r >= d ? r - d : r);
}

// a * w mod d with w's Shoup companion wp = floor(w 2^32 / d).
TC_DEV uint32_t mulmod_c(uint32_t a, uint32_t w, uint32_t wp, uint32_t d) {
  const uint32_t q = __umulhi(a, wp);
  const uint64_t r = (uint64_t)a * w - (uint64_t)q * d;
  return (uint32_t)(r >= d ? r - d : r);
}

// a * b mod d for a, b < d (a few times per chunk).
TC_DEV uint32_t mulmod64_32(uint32_t a, uint32_t b, uint32_t d) {
  return (uint32_t)(((uint64_t)a * b) % d);
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

// ---------------------------------------------------------------- wave scans
// Wave-wide scans on the DPP network (no LDS traffic): row_shr by 1, 2, 4, 8
// within each 16-lane row, then row_bcast:15 and row_bcast:31 across rows.
// Lanes whose DPP source is outside its range keep `old`, the identity.
constexpr int kDppRowShr = 0x110;   // + distance 1..15
constexpr int kDppWaveShl1 = 0x130;
constexpr int kDppWaveShr1 = 0x138;
constexpr int kDppBcast15 = 0x142;
constexpr int kDppBcast31 = 0x143;

template <int CTRL, int ROWMASK = 0xf>
TC_DEV uint32_t dpp(uint32_t old, uint32_t x) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)x, CTRL, ROWMASK, 0xf, false);
}

TC_DEV uint32_t readlane(uint32_t x, int l) { return (uint32_t)__builtin_amdgcn_readlane((int)x, l); }

// Inclusive scan of carry tables over the wave (earlier lanes applied first).
TC_DEV uint32_t scan_tab(uint32_t t) {
  t = tab_then(dpp<kDppRowShr + 1>(TAB_ID, t), t);
  t = tab_then(dpp<kDppRowShr + 2>(TAB_ID, t), t);
  t = tab_then(dpp<kDppRowShr + 4>(TAB_ID, t), t);
  t = tab_then(dpp<kDppRowShr + 8>(TAB_ID, t), t);
  t = tab_then(dpp<kDppBcast15, 0xa>(TAB_ID, t), t);
  t = tab_then(dpp<kDppBcast31, 0xc>(TAB_ID, t), t);
  return t;
}

// Inclusive scan of affine residue maps r -> r W^LPT + K over the wave
// (W = M mod d, each lane spanning LPT limbs).  A combined segment of s lanes
// multiplies the earlier part by W^(s LPT): s = d within rows, s = l%16 + 1
// for the row_bcast:15 step and s = l - 31 for the row_bcast:31 step.
template <int LPT>
TC_DEV uint32_t scan_residue(uint32_t K, const DivEntry* de, int lane) {
  const uint32_t d = de->d;
  const int j1 = ((lane & 15) + 1) * LPT, j2 = (lane >= 32 ? lane - 31 : 0) * LPT;
  const uint32_t w1 = de->pw[j1], w1s = de->pws[j1], w2 = de->pw[j2], w2s = de->pws[j2];
  K = addmod(mulmod_c(dpp<kDppRowShr + 1>(0u, K), de->pw[LPT], de->pws[LPT], d), K, d);
  K = addmod(mulmod_c(dpp<kDppRowShr + 2>(0u, K), de->pw[2 * LPT], de->pws[2 * LPT], d), K, d);
  K = addmod(mulmod_c(dpp<kDppRowShr + 4>(0u, K), de->pw[4 * LPT], de->pws[4 * LPT], d), K, d);
  K = addmod(mulmod_c(dpp<kDppRowShr + 8>(0u, K), de->pw[8 * LPT], de->pws[8 * LPT], d), K, d);
  K = addmod(mulmod_c(dpp<kDppBcast15, 0xa>(0u, K), w1, w1s, d), K, d);
  K = addmod(mulmod_c(dpp<kDppBcast31, 0xc>(0u, K), w2, w2s, d), K, d);
  return K;
}

// ---------------------------------------------------------------- look-back
// Status word: bits 63..62 flag (0 empty, 1 aggregate, 2 inclusive), 31..0
// value.  Flag and value travel in one 64-bit word, so relaxed atomics at
// device scope suffice (no fences, no cache maintenance).
constexpr uint64_t LB_AGG = 1ull << 62;
constexpr uint64_t LB_INC = 2ull << 62;
constexpr int kSpinLimit = 1 << 22;

// v holds bits 61..0 of the word (the flag goes to bits 63..62).
TC_DEV void lb_publish(uint64_t* w, uint64_t flag, uint64_t v) {
  if (lane_id() == 0)
    __hip_atomic_store(w, flag | v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

TC_DEV uint64_t lb_load(uint64_t* w) {
  return __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Loads the window of look-back words st[hi-63] .. st[hi] (lane l holds
// st[hi-63+l], the nearest chunk in lane 63) and waits until every word from
// the nearest inclusive one up to st[hi] has been published.  Words before
// the value's first chunk read as an inclusive `before`.  Returns the lane
// of the nearest inclusive word, or -1 if the window has none.
TC_DEV int lb_window(uint64_t* st, int64_t hi, uint64_t before, uint64_t& x, uint32_t& errbits) {
  const int64_t j = hi - 63 + lane_id();
  x = j >= 0 ? lb_load(&st[j]) : before;
  for (int spins = 0;; spins++) {
    const uint64_t inc = __ballot((x >> 62) == 2);
    const int k = inc ? 63 - __builtin_clzll((unsigned long long)inc) : -1;
    const uint64_t need = k <= 0 ? ~0ull : ~((1ull << k) - 1ull);  // lanes k..63
    const uint64_t empty = __ballot((x >> 62) == 0);
    if (!(empty & need)) return k;
    if (spins >= kSpinLimit) {
      errbits |= ERRBIT_HANG;
      return k;
    }
    __builtin_amdgcn_s_sleep(1);
    if ((x >> 62) == 0 && j >= 0) x = lb_load(&st[j]);
  }
}

// Sum of the lanes' residues modulo d (each below d), by the DPP scan; the
// total is in lane 63.
TC_DEV uint32_t sum_mod_wave(uint32_t w, uint32_t d) {
  w = addmod(w, dpp<kDppRowShr + 1>(0u, w), d);
  w = addmod(w, dpp<kDppRowShr + 2>(0u, w), d);
  w = addmod(w, dpp<kDppRowShr + 4>(0u, w), d);
  w = addmod(w, dpp<kDppRowShr + 8>(0u, w), d);
  w = addmod(w, dpp<kDppBcast15, 0xa>(0u, w), d);
  w = addmod(w, dpp<kDppBcast31, 0xc>(0u, w), d);
  return readlane(w, 63);
}

// Packed look-back word of the carry chain and the first division:
//   aggregate: flag AGG | carry table (2 bits per carry-in) << 32 | K
//   inclusive: flag INC | (carry out + 1) << 32 | rho out
// where rho = r - c is the division residue minus the carry at the same
// boundary (both are published by one store, so a reader sees them together).
TC_DEV uint64_t tab_pack6(uint32_t tab) {
  return (uint64_t)((tab & 3u) | ((tab >> 6) & 0xcu) | ((tab >> 12) & 0x30u));
}
TC_DEV uint32_t tab_unpack6(uint32_t v) {
  return (v & 3u) | ((v & 0xcu) << 6) | ((v & 0x30u) << 12);
}

// Carry and adjusted residue rho entering chunk c (c >= 1).  Chunk j maps the
// carry by its table t_j and rho by rho -> rho W + K_j with W = M^T mod d
// (de == nullptr: no division, rho stays 0).  Lane l of a window holds chunk
// hi - 63 + l, at distance 63 - l from hi; with the nearest inclusive word in
// lane k, the carry leaving chunk hi is the tables of lanes k+1 .. 63 applied
// in lane order to the carry of lane k (one DPP scan), and rho leaving it is
// sum over lanes l >= k of (value of lane l) W^(63-l), every weight read
// from the table.
template <int LPT>
TC_DEV void lb_state(uint64_t* st, int64_t c, const DivEntry* de, int& cin, uint32_t& rho,
                     uint32_t& errbits) {
  constexpr int kind = chunk_kind(LPT);
  const int lane = lane_id();
  const uint32_t d = de ? de->d : 1u;
  const uint32_t wl = de ? de->cw[kind][63 - lane] : 0u;
  const uint32_t wls = de ? de->cws[kind][63 - lane] : 0u;
  uint32_t A = TAB_ID;            // carry after chunk hi -> carry into chunk c
  uint32_t AK = 0, Am = 1u % d;   // rho after chunk hi -> rho into chunk c
  for (int64_t hi = c - 1;; hi -= 64) {
    uint64_t x;
    const int k = lb_window(st, hi, LB_INC | (1ull << 32), x, errbits);
    const uint32_t F =
        readlane(scan_tab(lane > k ? tab_unpack6((uint32_t)(x >> 32) & 63u) : TAB_ID), 63);
    uint32_t S = 0;
    if (de) S = sum_mod_wave(lane >= k ? mulmod_c((uint32_t)x, wl, wls, d) : 0u, d);
    if (k >= 0) {
      const int cinc = (int)(readlane((uint32_t)(x >> 32), k) & 3u) - 1;
      cin = tab_apply(A, tab_apply(F, cinc));
      if (hi == c - 1) rho = S;
      else rho = addmod(mulmod64_32(S, Am, d), AK, d);
      return;
    }
    // no inclusive word in this window: fold it into the composite
    A = tab_then(F, A);
    if (de) {
      AK = addmod(mulmod64_32(S, Am, d), AK, d);
      Am = mulmod_c(Am, de->cw[kind][64], de->cws[kind][64], d);
    }
    if (errbits & ERRBIT_HANG) {
      cin = 0;
      rho = 0;
      return;
    }
  }
}

// Residue entering chunk c (c >= 1) of the second division, whose look-back
// words carry the residue alone (flag | K, or flag | r when inclusive): the
// weighted sum of lb_state without the carry.
template <int LPT>
TC_DEV uint32_t lb_residue(uint64_t* st, int64_t c, const DivEntry* de, uint32_t& errbits) {
  constexpr int kind = chunk_kind(LPT);
  const int lane = lane_id();
  const uint32_t d = de->d;
  const uint32_t wl = de->cw[kind][63 - lane], wls = de->cws[kind][63 - lane];
  uint32_t AK = 0, Am = 1u % d;  // composite of the windows passed: r -> r W^(64 n) + AK
  for (int64_t hi = c - 1;; hi -= 64) {
    uint64_t x;
    const int k = lb_window(st, hi, LB_INC, x, errbits);
    const uint32_t S = sum_mod_wave(lane >= k ? mulmod_c((uint32_t)x, wl, wls, d) : 0u, d);
    if (k >= 0) {
      if (hi == c - 1) return S;
      return addmod(mulmod64_32(S, Am, d), AK, d);
    }
    AK = addmod(mulmod64_32(S, Am, d), AK, d);
    Am = mulmod_c(Am, de->cw[kind][64], de->cws[kind][64], d);
    if (errbits & ERRBIT_HANG) return 0;
  }
}

// Default vector form of Src::delta: dd[0] = delta(pt-1) when pt > 0,
// dd[1+i] = delta(pt+i) for i < nown.
template <int LPT, class Src>
TC_DEV void deltas_by_limb(const Src& s, int64_t pt, int nown, int64_t* dd) {
  if (pt > 0) dd[0] = s.delta(pt - 1);
#pragma unroll
  for (int i = 0; i < LPT; i++)
    if (i < nown) dd[i + 1] = s.delta(pt + i);
}

struct EngCfg {
  int64_t Y;                 // limbs computed
  const DivEntry* div[2];    // odd divisors, nullptr = none
  int32_t shr;               // exact right shift, < 64
  bool is_signed;            // two's complement result (else unsigned)
  bool prenorm;              // split delta into lo/hi (|delta| may exceed 2^32)
  bool check_carry;          // unsigned: carry out of limb Y-1 must be 0
};

// State between consecutive chunks when one wave runs a whole value.
struct EngState {
  int carry;
  uint32_t r[2];
};

// Result of one chunk, broadcast to all lanes.
struct ChunkOut {
  uint32_t top;      // result limb Y-1 if this chunk holds it
  int64_t lowest_nz; // lowest limb index with a non-zero stored result, or -1
};

// Runs chunk c (of nch) of one value on the calling wavefront.  st holds the
// value's look-back words: [carry and first division, packed x nch]
// [second division x nch] (unused when nch == 1).  Src provides
//   int64_t delta(int64_t p)                             for 0 <= p < Y
//   void    deltas<LPT>(pt, nown, dd)                    dd[0] = delta(pt-1), dd[1+i] = delta(pt+i)
//                                                        (i < LPT, or i < LPT+2 if kWide)
//   bool    kWide                                        deltas covers the shift lookahead
//   bool    store(int64_t p, uint32_t o, uint32_t& err)  returns true if stored
// c must be wave-uniform.  FULL: every lane owns LPT limbs below Y (no
// per-limb bounds).
template <int LPT, bool FULL, class Src>
TC_DEV ChunkOut engine_chunk_impl(Src& src, const EngCfg& cfg, int64_t c, int64_t nch,
                                  uint64_t* st, uint32_t& errbits, EngState* carried) {
  static_assert(LPT >= 2, "shift lookahead needs two limbs per lane");
  const int lane = lane_id();
  constexpr int T = 64 * LPT;
  const int64_t Y = cfg.Y;
  const int sq = cfg.shr >> 5, sr = cfg.shr & 31;
  const int E = sq + (sr ? 1 : 0);
  const int64_t p0 = c * T;
  const int64_t pt = p0 + (int64_t)lane * LPT;
  const int64_t rem = Y - pt;
  const int nown = FULL ? LPT : (rem <= 0 ? 0 : (rem >= LPT ? LPT : (int)rem));
  const bool last = c + 1 >= nch;
#define TC_OWN(i) (FULL || (i) < nown)

  // 1. pre-normalised limbs; dd[0] = delta(pt-1), dd[1+i] = delta(pt+i)
  int64_t e[LPT];
  int64_t dlast;
  int64_t la_d[2] = {0, 0};  // wide sources: delta(pt+LPT), delta(pt+LPT+1)
  {
    constexpr int ND = Src::kWide ? LPT + 3 : LPT + 1;
    int64_t dd[ND];
#pragma unroll
    for (int i = 0; i < ND; i++) dd[i] = 0;
    if (FULL || nown > 0) src.template deltas<LPT>(pt, nown, dd);
    if constexpr (Src::kWide) {
      la_d[0] = dd[LPT + 1];
      la_d[1] = dd[LPT + 2];
    }
    int64_t dprev = (cfg.prenorm && pt > 0) ? dd[0] : 0;
#pragma unroll
    for (int i = 0; i < LPT; i++) {
      const int64_t d = TC_OWN(i) ? dd[i + 1] : 0;
      e[i] = cfg.prenorm ? ((d & 0xffffffffll) + (dprev >> 32)) : d;
      dprev = d;
    }
    dlast = dprev;
  }

  // 2. local carries with carry-in 0: the lane's table and its limbs
  uint32_t x[LPT];
  uint32_t tab;
  int t0;  // the lane's carry out for carry-in 0
  {
    int cc = 0;
    bool ones = true, zeros = true;
#pragma unroll
    for (int i = 0; i < LPT; i++) {
      if (TC_OWN(i)) {
        const int64_t s = e[i] + cc;
        x[i] = (uint32_t)s;
        cc = (int)(s >> 32);
        ones = ones && x[i] == 0xffffffffu;
        zeros = zeros && x[i] == 0u;
      }
    }
    tab = (FULL || nown) ? tab_make(cc - (zeros ? 1 : 0), cc, cc + (ones ? 1 : 0)) : TAB_ID;
    t0 = cc;
  }
  const uint32_t inc = scan_tab(tab);
  const uint32_t exc = dpp<kDppWaveShr1>(TAB_ID, inc);
  const uint32_t chunk_tab = readlane(inc, 63);

  // 3. first division, local part.  With carry-in c and residue r the lane's
  // limbs are X(c) = X(0) + c - (t(c) - t(0)) 2^(32 LPT), and its residue out
  // is (r - X(c)) M^LPT mod d; so rho = r - c obeys rho' = rho M^LPT + K'
  // with K' = K(0) - t(0), whatever the carry.  The scan of K' over the wave
  // (and the look-back over chunks) thus needs no carries.
  const DivEntry* de0 = cfg.div[0];
  uint32_t Kx = 0, chunk_K = 0;
  uint32_t pw_l = 0, pws_l = 0, pw_t = 0, pws_t = 0;
  if (de0) {
    const uint32_t d = de0->d, dinv = de0->dinv;
    pw_l = de0->pw[lane * LPT];
    pws_l = de0->pws[lane * LPT];
    pw_t = de0->pw[T];
    pws_t = de0->pws[T];
    uint32_t K = 0;
#pragma unroll
    for (int i = 0; i < LPT; i++)
      if (TC_OWN(i)) (void)hensel_step(x[i], K, d, dinv);
    // K' = K - t(0) mod d
    K = t0 > 0 ? (K == 0 ? d - 1u : K - 1u) : (t0 < 0 ? (K + 1u == d ? 0u : K + 1u) : K);
    K = scan_residue<LPT>(K, de0, lane);
    Kx = dpp<kDppWaveShr1>(0u, K);
    chunk_K = readlane(K, 63);
  }

  // chunk state in: carry and rho
  int carry_in = 0;
  uint32_t rho_in = 0;
  const uint32_t d0 = de0 ? de0->d : 1u;
  if (carried) {
    if (c > 0) {
      carry_in = carried->carry;
      rho_in = de0 ? (uint32_t)(((int64_t)carried->r[0] - carry_in + d0) % d0) : 0u;
    }
    const int cout_chunk = tab_apply(chunk_tab, carry_in);
    carried->carry = cout_chunk;
    if (de0) {
      const uint32_t rho_out = addmod(mulmod_c(rho_in, pw_t, pws_t, d0), chunk_K, d0);
      carried->r[0] = (uint32_t)(((int64_t)rho_out + cout_chunk + d0) % d0);
    }
  } else {
    if (c > 0) {
      lb_publish(&st[c], LB_AGG, ((uint64_t)tab_pack6(chunk_tab) << 32) | chunk_K);
      lb_state<LPT>(st, c, de0, carry_in, rho_in, errbits);
    }
    if (!last) {
      const uint32_t rho_out = de0 ? addmod(mulmod_c(rho_in, pw_t, pws_t, d0), chunk_K, d0) : 0u;
      lb_publish(&st[c], LB_INC,
                 ((uint64_t)(tab_apply(chunk_tab, carry_in) + 1) << 32) | rho_out);
    }
  }

  // final limbs with the lane's carry-in
  int cout;
  int cl;
  {
    int cc = tab_apply(exc, carry_in);
    cl = cc;
#pragma unroll
    for (int i = 0; i < LPT; i++) {
      if (TC_OWN(i)) {
        const int64_t s = e[i] + cc;
        x[i] = (uint32_t)s;
        cc = (int)(s >> 32);
      }
    }
    cout = cc;
    if (!FULL && cfg.check_carry && nown > 0 && pt + nown == Y && cc != 0) errbits |= ERRBIT_RANGE;
  }

  // 3'. exact divisions: the first with r = rho + c at the lane's first limb
  uint32_t rcur0 = 0, rcur1 = 0;
  if (de0) {
    const uint32_t d = d0, dinv = de0->dinv;
    const uint32_t rho_l = addmod(mulmod_c(rho_in, pw_l, pws_l, d), Kx, d);
    uint32_t r = cl > 0 ? (rho_l + 1u == d ? 0u : rho_l + 1u)
                        : (cl < 0 ? (rho_l == 0 ? d - 1u : rho_l - 1u) : rho_l);
#pragma unroll
    for (int i = 0; i < LPT; i++)
      if (TC_OWN(i)) x[i] = hensel_step(x[i], r, d, dinv);
    if (!FULL && nown > 0 && pt + nown == Y) {
      uint32_t qtop = 0;
#pragma unroll
      for (int i = 0; i < LPT; i++)
        if (i == nown - 1) qtop = x[i];
      const uint32_t want = (qtop >> 31) ? d - 1u : 0u;
      if (r != want) errbits |= ERRBIT_DIV;
    }
    rcur0 = r;
  }
  // the second division works on the quotient of the first: its own scan
  // and look-back (words st[nch .. 2 nch))
  if (const DivEntry* de = cfg.div[1]) {
    const uint32_t d = de->d, dinv = de->dinv;
    const uint32_t pl = de->pw[lane * LPT], pls = de->pws[lane * LPT];
    const uint32_t ptt = de->pw[T], ptts = de->pws[T];
    uint32_t K = 0;
#pragma unroll
    for (int i = 0; i < LPT; i++)
      if (TC_OWN(i)) (void)hensel_step(x[i], K, d, dinv);
    K = scan_residue<LPT>(K, de, lane);
    const uint32_t K1x = dpp<kDppWaveShr1>(0u, K);
    const uint32_t cK = readlane(K, 63);
    uint32_t rin = 0;
    if (carried) {
      rin = c > 0 ? carried->r[1] : 0u;
      carried->r[1] = addmod(mulmod_c(rin, ptt, ptts, d), cK, d);
    } else {
      uint64_t* sw = st + nch;
      if (c > 0) {
        lb_publish(&sw[c], LB_AGG, cK);
        rin = lb_residue<LPT>(sw, c, de, errbits);
      }
      if (!last) lb_publish(&sw[c], LB_INC, addmod(mulmod_c(rin, ptt, ptts, d), cK, d));
    }
    uint32_t r = addmod(mulmod_c(rin, pl, pls, d), K1x, d);
#pragma unroll
    for (int i = 0; i < LPT; i++)
      if (TC_OWN(i)) x[i] = hensel_step(x[i], r, d, dinv);
    if (!FULL && nown > 0 && pt + nown == Y) {
      uint32_t qtop = 0;
#pragma unroll
      for (int i = 0; i < LPT; i++)
        if (i == nown - 1) qtop = x[i];
      const uint32_t want = (qtop >> 31) ? d - 1u : 0u;
      if (r != want) errbits |= ERRBIT_DIV;
    }
    rcur1 = r;
  }

  // 4. lookahead: lane 63 continues into the next chunk for the shift
  uint32_t la0 = 0, la1 = 0;
  if (E > 0 && !last && lane == 63) {
    int64_t dprev = dlast;
    int cc = cout;
    uint32_t r0 = rcur0, r1 = rcur1;
    for (int i = 0; i < E; i++) {
      const int64_t p = p0 + T + i;
      if (p >= Y) break;
      int64_t d;
      if constexpr (Src::kWide) d = i == 0 ? la_d[0] : la_d[1];
      else d = src.delta(p);
      const int64_t ee = cfg.prenorm ? ((d & 0xffffffffll) + (dprev >> 32)) : d;
      dprev = d;
      const int64_t s = ee + cc;
      uint32_t xx = (uint32_t)s;
      cc = (int)(s >> 32);
      if (cfg.div[0]) xx = hensel_step(xx, r0, cfg.div[0]->d, cfg.div[0]->dinv);
      if (cfg.div[1]) xx = hensel_step(xx, r1, cfg.div[1]->d, cfg.div[1]->dinv);
      if (i == 0) la0 = xx;
      else la1 = xx;
    }
  }

  // sign extension of the result's top limb, for positions >= Y
  uint32_t sext = 0;
  if (!FULL && cfg.is_signed && Y - 1 < p0 + T + E) {
    uint32_t mine = 0;
#pragma unroll
    for (int i = 0; i < LPT; i++)
      if (pt + i == Y - 1) mine = x[i];
    uint32_t topq;
    if (Y - 1 < p0 + T) {
      topq = readlane(mine, (int)((Y - 1 - p0) / LPT));
    } else {
      const uint32_t l = (Y - 1 - (p0 + T)) == 0 ? la0 : la1;
      topq = readlane(l, 63);
    }
    sext = (topq >> 31) ? 0xffffffffu : 0u;
  }

  // 5. shift and store
  uint32_t nx0 = dpp<kDppWaveShl1>(0u, x[0]);
  uint32_t nx1 = dpp<kDppWaveShl1>(0u, x[1]);
  if (lane == 63) {
    nx0 = la0;
    nx1 = la1;
  }
  if (!FULL) {
    if (pt + LPT >= Y) nx0 = sext;
    if (pt + LPT + 1 >= Y) nx1 = sext;
  }
  uint32_t q[LPT + 2];
#pragma unroll
  for (int i = 0; i < LPT; i++) q[i] = (FULL || pt + i < Y) ? x[i] : sext;
  q[LPT] = nx0;
  q[LPT + 1] = nx1;
  if (pt == 0 && cfg.shr > 0) {
    // section 3's divisions are exact: the bits shifted out are zero
    const uint32_t low = sq ? q[1] : q[0];
    if ((sq && q[0] != 0u) || (sr && (low & ((1u << sr) - 1u)) != 0u)) errbits |= ERRBIT_SHIFT;
  }
  uint32_t o[LPT];
#pragma unroll
  for (int i = 0; i < LPT; i++) {
    const uint32_t lo = sq ? q[i + 1] : q[i];
    const uint32_t hi = sq ? q[i + 2] : q[i + 1];
    o[i] = sr ? ((lo >> sr) | (hi << (32 - sr))) : lo;
  }
  uint32_t top = 0;
  int64_t lownz = -1;
  if (FULL) {
    // every limb lies below Y: one run of wide stores
    src.template store_run<LPT>(pt, o, errbits);
#pragma unroll
    for (int i = LPT - 1; i >= 0; i--)
      if (o[i] != 0u) lownz = pt + i;
  } else {
#pragma unroll
    for (int i = LPT - 1; i >= 0; i--) {
      if (TC_OWN(i)) {
        if (src.store(pt + i, o[i], errbits) && o[i] != 0u) lownz = pt + i;
        if (pt + i == Y - 1) top = o[i];
      }
    }
  }
  ChunkOut res;
  res.top = 0;
  if (!FULL && Y - 1 >= p0 && Y - 1 < p0 + T) res.top = readlane(top, (int)((Y - 1 - p0) / LPT));
  // lowest non-zero stored limb: the first lane that stored one holds it
  const uint64_t nz = __ballot(lownz >= 0);
  if (nz) {
    const int l = __ffsll((unsigned long long)nz) - 1;
    res.lowest_nz = (int64_t)(((uint64_t)readlane((uint32_t)((uint64_t)lownz >> 32), l) << 32) |
                              readlane((uint32_t)lownz, l));
  } else {
    res.lowest_nz = -1;
  }
#undef TC_OWN
  return res;
}

// Runs chunk c of a value; picks the variant without per-limb bounds when
// the chunk and the two limbs its shift looks ahead at all lie below the
// value's top limb Y-1 (that chunk needs the sign of limb Y-1 and the sign
// extension above it).
template <int LPT, class Src>
TC_DEV ChunkOut engine_chunk(Src& src, const EngCfg& cfg, int64_t c, int64_t nch, uint64_t* st,
                             uint32_t& errbits, EngState* carried = nullptr) {
  if ((c + 1) * 64 * LPT + 2 < cfg.Y)
    return engine_chunk_impl<LPT, true>(src, cfg, c, nch, st, errbits, carried);
  return engine_chunk_impl<LPT, false>(src, cfg, c, nch, st, errbits, carried);
}

// Runs a whole value on the calling wavefront, chunk after chunk.
template <int LPT, class Src>
TC_DEV ChunkOut engine_value(Src& src, const EngCfg& cfg, uint32_t& errbits) {
  constexpr int64_t T = 64 * LPT;
  const int64_t nch = (cfg.Y + T - 1) / T;
  EngState s;
  s.carry = 0;
  s.r[0] = s.r[1] = 0u;
  ChunkOut res;
  res.top = 0;
  res.lowest_nz = -1;
  for (int64_t c = 0; c < nch; c++) {
    const ChunkOut o = engine_chunk<LPT>(src, cfg, c, nch, nullptr, errbits, &s);
    res.top = o.top;
    if (res.lowest_nz < 0) res.lowest_nz = o.lowest_nz;
  }
  return res;
}

}  // namespace tc
