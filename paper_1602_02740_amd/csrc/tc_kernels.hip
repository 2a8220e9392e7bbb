// tc_kernels.hip -- the HIP kernels of the Toom-Cook path (gfx950, wave64).
//
//   k_eval    evaluation of one operand at one point (section 1, 4, 6)
//   k_step    one exact linear step of the interpolation: the even-odd
//             combine (section 4) and the two Newton loops (section 3)
//   k_recomp  recomposition w = sum_k w_k 2^(b k) (section 1)
//   k_leaf    batched schoolbook products at the leaves of the recursion
//
// A launch covers many independent values (all nodes of a recursion level,
// both polynomials, every m of a Newton round): one wavefront per value, four
// per workgroup, no workgroup barriers in the linear passes.
#include <hip/hip_runtime.h>

#include "tc_engine.hpp"
#include "tc_internal.hpp"

namespace tc {

// ---------------------------------------------------------------- sources
// G: the source's arrays live in global memory (every kernel but the fused
// bottom node, whose intermediate values sit in LDS and use generic access).

template <bool G>
TC_DEV uint32_t ldx(const uint32_t* p) {
  if constexpr (G) return gld(p);
  else return *p;
}
template <bool G, int N>
TC_DEV void ldx_run(const uint32_t* p, uint32_t* w) {
  if constexpr (G) {
    gld_run<N>(p, w);
  } else {
#pragma unroll
    for (int i = 0; i < N; i++) w[i] = p[i];
  }
}
template <bool G>
TC_DEV void stx(uint32_t* p, uint32_t v) {
  if constexpr (G) gst(p, v);
  else *p = v;
}
template <bool G, int N>
TC_DEV void stx_run(uint32_t* p, const uint32_t* w) {
  if constexpr (G) {
    gst_run<N>(p, w);
  } else {
#pragma unroll
    for (int i = 0; i < N; i++) p[i] = w[i];
  }
}

// One term of a step, compacted to five scalar registers.  The term's limb
// p is bits of (limb(p-k) : limb(p-k-1)) >> sh, one v_alignbit (k = q and
// sh = 32 - r for a left shift of 32 q + r bits, r > 0; k = q - 1, sh = 0 for
// r = 0).  A negated term adds (~v) mul, and the step adds the constant
// mul - mul 2^32 per negated term to every limb: -v mul = (~v) mul + mul - mul 2^32.
template <bool G>
struct Term {
  const uint32_t* ptr;
  int32_t width;
  uint32_t f;     // bit 0 negative, bit 1 absent, bit 2 ones past the width,
                  // bits 3..7 sh, bits 8..31 k + 1
  uint32_t mul;   // odd multiplier, 1 = none

  TC_DEV int k() const { return (int)(f >> 8) - 1; }
  TC_DEV uint32_t sh() const { return (f >> 3) & 31u; }
  TC_DEV uint32_t nmask() const { return (f & 1u) ? 0xffffffffu : 0u; }
  TC_DEV uint32_t limb(int64_t i) const {
    if (i < 0) return 0u;
    if (i < width) return ldx<G>(ptr + i);
    return (f & 4u) ? 0xffffffffu : 0u;
  }
  TC_DEV int64_t at(int64_t p) const {
    const uint32_t v = __builtin_amdgcn_alignbit(limb(p - k()), limb(p - k() - 1), sh());
    const int64_t m = (int64_t)((uint64_t)v * mul);
    return (f & 1u) ? -m : m;
  }
  // acc[i] += term at limb pt-1+i (negated terms: without their constant),
  // i = 0..N-1, from the window of N+1 limbs at pt-2-k
  template <int N>
  TC_DEV void add_window(int64_t pt, uint64_t* acc) const {
    uint32_t w[N + 1];
    const int64_t base = pt - 2 - k();
    if (base >= 0 && base + N + 1 <= width) {
      ldx_run<G, N + 1>(ptr + base, w);
    } else {
#pragma unroll
      for (int i = 0; i < N + 1; i++) w[i] = limb(base + i);
    }
    mac<N>(w, acc);
  }
  // the window known to lie inside the stored limbs
  template <int N>
  TC_DEV void add_window_in(int64_t pt, uint64_t* acc) const {
    uint32_t w[N + 1];
    ldx_run<G, N + 1>(ptr + (pt - 2 - k()), w);
    mac<N>(w, acc);
  }
  // any window: one load per limb from a clamped index, then zero below limb
  // 0 and the extension past the width (no branches, so several terms' loads
  // can be in flight)
  template <int N>
  TC_DEV void add_window_clamped(int64_t pt, uint64_t* acc) const {
    uint32_t w[N + 1];
    const int64_t base = pt - 2 - k();
    const int64_t top = width > 0 ? width - 1 : 0;
    const uint32_t ext = (f & 4u) ? 0xffffffffu : 0u;
#pragma unroll
    for (int i = 0; i < N + 1; i++) {
      const int64_t j = base + i;
      const uint32_t v = ldx<G>(ptr + (j < 0 ? 0 : (j > top ? top : j)));
      w[i] = j < 0 ? 0u : (j >= width ? ext : v);
    }
    mac<N>(w, acc);
  }
  template <int N>
  TC_DEV void mac(const uint32_t* w, uint64_t* acc) const {
    const uint32_t s = sh(), nm = nmask();
#pragma unroll
    for (int i = 0; i < N; i++) {
      const uint32_t v = __builtin_amdgcn_alignbit(w[i + 1], w[i], s) ^ nm;
      acc[i] += (uint64_t)v * mul;
    }
  }
  // constant added per limb: mul - mul 2^32 for a negated term
  TC_DEV uint64_t bias() const {
    return (f & 1u) ? (uint64_t)mul - ((uint64_t)mul << 32) : 0ull;
  }
};

// Packs a term descriptor (left shift below 2^29 bits, checked by the
// planner).  flip: the product's sign negates the term; ones: the limbs past
// the width read as all ones (a negative two's-complement value).
template <bool G>
TC_DEV void make_term(Term<G>& t, const TermDesc& d, const uint32_t* ptr, bool neg, bool ones) {
  const int q = d.shl >> 5, r = d.shl & 31;
  const int k = r ? q : q - 1;
  const uint32_t sh = r ? (uint32_t)(32 - r) : 0u;
  t.ptr = ptr;
  t.width = d.width;
  t.f = (neg ? 1u : 0u) | (ones ? 4u : 0u) | (sh << 3) | ((uint32_t)(k + 1) << 8);
  t.mul = d.mul > 1u ? d.mul : 1u;
}

// hi_limb bounds the limbs the wave reads (exclusive); the sign-extension
// limb is loaded only when that passes the term's width.
TC_DEV void load_term(Term<true>& t, const TermDesc& d, const Bases& b, int64_t node,
                      int64_t hi_limb) {
  // kind and neg share a dword of the descriptor: one scalar load
  const uint32_t kn = sld(reinterpret_cast<const uint32_t*>(&d.kind));
  const int kind = (int)(int8_t)(kn & 0xffu);
  if (kind == TERM_NONE) {
    t.ptr = nullptr;
    t.width = 0;
    t.f = 2u;
    t.mul = 1u;
    return;
  }
  const uint32_t* ptr = reinterpret_cast<const uint32_t*>(resolve_d(b, d.ptr)) + node * d.stride;
  bool neg = ((kn >> 8) & 0xffu) != 0u;
  if (kind == TERM_SM) {
    // sign of a product = sign(U(x)) xor sign(V(x)); sv may be absent
    const uint32_t s1 = sld_byte(resolve_d(b, d.su) + node * d.sstride);
    const uint32_t s2 = d.sv.buf >= 0 ? sld_byte(resolve_d(b, d.sv) + node * d.svstride) : 0u;
    if (s1 ^ s2) neg = !neg;
  }
  const bool ones = kind == TERM_TC && d.width > 0 && hi_limb > d.width &&
                    (sld(ptr + d.width - 1) >> 31);
  make_term(t, d, ptr, neg, ones);
}

template <bool G>
struct StepSrc {
  Term<G> t[kStepTerms];
  int n;
  bool present;  // no absent term among the first n
  uint32_t* out;
  TC_DEV int64_t delta(int64_t p) const {
    int64_t d = 0;
#pragma unroll
    for (int i = 0; i < kStepTerms; i++)
      if (i < n && !(t[i].f & 2u)) d += t[i].at(p);
    return d;
  }
  // Wide windows: dd[LPT+1], dd[LPT+2] = delta(pt+LPT), delta(pt+LPT+1), the
  // lookahead of a right shift.  Limbs past Y are never stored, so the
  // window may include them.
  static constexpr bool kWide = true;
  static_assert(kStepTerms == 8, "deltas switches over up to eight terms");
  template <int LPT, int K>
  TC_DEV void sum_in(int64_t pt, uint64_t* acc) const {
#pragma unroll
    for (int i = 0; i < K; i++) t[i].template add_window_in<LPT + 3>(pt, acc);
  }
  template <int LPT>
  TC_DEV void deltas(int64_t pt, int, int64_t* dd) const {
    constexpr int N = LPT + 3;
    uint64_t acc[N];
#pragma unroll
    for (int i = 0; i < N; i++) acc[i] = 0;
    // the wave's windows span limbs p0-2-k .. p0+64 LPT+1-k of each term
    const int64_t pl = pt - (int64_t)lane_id() * LPT;  // the same in every lane
    const int64_t p0 = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane(
                                      (int)(uint32_t)((uint64_t)pl >> 32)) << 32) |
                                  (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)pl));
    bool inside = present;
    uint64_t bias = 0;
#pragma unroll
    for (int i = 0; i < kStepTerms; i++) {
      if (i < n) {
        const int64_t lo = p0 - 2 - t[i].k(), hi = p0 + 64 * LPT + 2 - t[i].k();
        inside = inside && lo >= 0 && hi <= t[i].width;
        bias += t[i].bias();
      }
    }
    if (inside) {
      // one straight-line block per term count: every load can be in flight
      switch (n) {
        case 0: break;
        case 1: sum_in<LPT, 1>(pt, acc); break;
        case 2: sum_in<LPT, 2>(pt, acc); break;
        case 3: sum_in<LPT, 3>(pt, acc); break;
        case 4: sum_in<LPT, 4>(pt, acc); break;
        case 5: sum_in<LPT, 5>(pt, acc); break;
        case 6: sum_in<LPT, 6>(pt, acc); break;
        case 7: sum_in<LPT, 7>(pt, acc); break;
        case 8: sum_in<LPT, 8>(pt, acc); break;
        default: break;
      }
    } else {
      // the value's first or last chunk: bounds per limb, without branches
#pragma unroll
      for (int i = 0; i < kStepTerms; i++)
        if (i < n && !(t[i].f & 2u)) t[i].template add_window_clamped<N>(pt, acc);
    }
#pragma unroll
    for (int i = 0; i < N; i++) dd[i] += (int64_t)(acc[i] + bias);
  }
  TC_DEV bool store(int64_t p, uint32_t o, uint32_t&) {
    stx<G>(out + p, o);
    return true;
  }
  // limbs pt .. pt+LPT-1, all below Y
  template <int LPT>
  TC_DEV void store_run(int64_t pt, const uint32_t* o, uint32_t&) {
    stx_run<G, LPT>(out + pt, o);
  }
};

// Base address of a plain buffer (scratch, U, V or W) by scalar selects.
TC_DEV const uint8_t* base_of(const Bases& b, int buf) {
  return buf == BUF_SCRATCH ? b.scratch : buf == BUF_U ? b.p[0] : buf == BUF_V ? b.p[1] : b.p[2];
}

// The step's terms from its precomputed records, as straight-line code: every
// record, sign byte and top limb is requested before any is used.  Lane l
// reads the sign bytes of the node's point product l; a product term takes
// its sign by v_readlane.  Absent terms (i >= n) read a safe address.
TC_DEV void setup_terms(StepSrc<true>& s, const StepDesc& D, const Bases& b, int64_t node) {
  const int lane = lane_id();
  const int n = D.nterms;
  uint32_t sgx = 0;
  if (D.nsgn > 0 && lane < D.nsgn) {
    const int64_t o = node * D.sgn_stride + lane;
    uint32_t x = *(const __attribute__((address_space(1))) uint8_t*)(base_of(b, D.sgn_u_buf) +
                                                                       D.sgn_u_off + o);
    if (D.sgn_v_buf >= 0)
      x ^= *(const __attribute__((address_space(1))) uint8_t*)(base_of(b, D.sgn_v_buf) +
                                                                 D.sgn_v_off +
                                                                 node * D.sgn_v_stride + lane);
    sgx = x;
  }
  const uint32_t* ptr[kStepTerms];
  uint32_t top[kStepTerms];
  // a record as eight dwords of scalar loads (its byte fields in the last)
  uint32_t misc[kStepTerms];
#pragma unroll
  for (int i = 0; i < kStepTerms; i++) {
    const uint32_t* r = reinterpret_cast<const uint32_t*>(&D.c[i]);
    const int64_t off = (int64_t)(((uint64_t)sld(r + 1) << 32) | sld(r));
    const int64_t stride = (int64_t)(((uint64_t)sld(r + 3) << 32) | sld(r + 2));
    const int32_t width = (int32_t)sld(r + 4);
    misc[i] = sld(r + 7);
    const int buf = (int)(int8_t)(misc[i] & 0xffu);
    const bool tc = ((misc[i] >> 8) & 0xffu) != 0u;
    ptr[i] = reinterpret_cast<const uint32_t*>(base_of(b, buf) + off) + node * stride;
    const bool want = i < n && tc && width > 0;
    top[i] = sld(want ? ptr[i] + (width - 1) : reinterpret_cast<const uint32_t*>(&D));
    s.t[i].width = width;
    s.t[i].f = sld(r + 5);
    s.t[i].mul = sld(r + 6);
  }
  s.n = n;
  s.present = true;
#pragma unroll
  for (int i = 0; i < kStepTerms; i++) {
    const int si = (int)(int16_t)(misc[i] >> 16);
    const bool tc = ((misc[i] >> 8) & 0xffu) != 0u;
    const uint32_t flip = si >= 0 ? readlane(sgx, si) & 1u : 0u;
    const bool ones = tc && s.t[i].width > 0 && (top[i] >> 31);
    s.t[i].ptr = ptr[i];
    s.t[i].f = (s.t[i].f ^ flip) | (ones ? 4u : 0u);
  }
}

template <bool G>
struct EvalSrc {
  static constexpr bool kWide = false;
  const uint32_t* src;
  int64_t W, bl;
  int B, j, oddneg, copy;
  int rev;  // block t shifted by (B-1-t) j rather than t j
  uint32_t* out;
  int64_t nout;

  TC_DEV uint32_t blk(int t, int64_t q) const {
    if (q < 0 || q >= bl) return 0u;
    const int64_t g = (int64_t)t * bl + q;
    return g < W ? ldx<G>(src + g) : 0u;
  }
  TC_DEV int64_t delta(int64_t p) const {
    if (copy >= 0) return (int64_t)blk(copy, p);
    int64_t d = 0;
    for (int t = 0; t < B; t++) {
      const int s = (rev ? B - 1 - t : t) * j, q = s >> 5, r = s & 31;
      const uint32_t hi = blk(t, p - q);
      const uint32_t v = r ? ((hi << r) | (blk(t, p - q - 1) >> (32 - r))) : hi;
      d += ((t & 1) && oddneg) ? -(int64_t)v : (int64_t)v;
    }
    return d;
  }
  // w[0..LPT+2) = block t's limbs base .. base+LPT+1 (zero outside the block)
  template <int LPT>
  TC_DEV void window(int t, int64_t base, uint32_t* w) const {
    const int64_t g0 = (int64_t)t * bl + base;
    if (base >= 0 && base + LPT + 2 <= bl && g0 + LPT + 2 <= W) {
      ldx_run<G, LPT + 2>(src + g0, w);
    } else {
#pragma unroll
      for (int i = 0; i < LPT + 2; i++) w[i] = blk(t, base + i);
    }
  }
  // Whether every lane's window of every block lies inside the stored limbs
  // (wave-uniform: then the windows load as plain runs, four blocks at a time).
  // PAIRED: block t shifted by t j (the paired evaluation ignores rev).
  template <int LPT, bool PAIRED>
  TC_DEV bool windows_inside(int64_t pt) const {
    bool ok = true;
    for (int t = 0; t < B; t++) {
      const int s = (!PAIRED && rev ? B - 1 - t : t) * j, q = s >> 5;
      const int64_t base = pt - 2 - q;
      ok = ok && base >= 0 && base + LPT + 2 <= bl && (int64_t)t * bl + base + LPT + 2 <= W;
    }
    return __ballot(!ok) == 0;
  }
  // Adds block t's window (shifted left by r bits) into dd[0..LPT].
  template <int LPT>
  TC_DEV static void add_shifted(const uint32_t* w, int r, bool neg, int64_t* dd) {
#pragma unroll
    for (int i = 0; i <= LPT; i++) {
      const uint32_t v = r ? ((w[i + 1] << r) | (w[i] >> (32 - r))) : w[i + 1];
      dd[i] += neg ? -(int64_t)v : (int64_t)v;
    }
  }
  // Blocks t .. t+3 (those below B): all four windows are requested before
  // any is added, so their latencies overlap.  ODD_SPLIT (paired evaluation,
  // shifts t j): odd blocks go to dodd; else they go to dd, negated when
  // oddneg.
  template <int LPT, bool ODD_SPLIT>
  TC_DEV void group4(int t, int64_t pt, int64_t* dd, int64_t* dodd) const {
    uint32_t w[4][LPT + 2];
    int r[4];
#pragma unroll
    for (int u = 0; u < 4; u++) {
      r[u] = 0;
      if (t + u < B) {
        const int sft = (!ODD_SPLIT && rev ? B - 1 - (t + u) : t + u) * j;
        r[u] = sft & 31;
        ldx_run<G, LPT + 2>(src + (int64_t)(t + u) * bl + (pt - 2 - (sft >> 5)), w[u]);
      }
    }
#pragma unroll
    for (int u = 0; u < 4; u++) {
      if (t + u < B) {
        const bool odd = ((t + u) & 1) != 0;
        if (ODD_SPLIT) add_shifted<LPT>(w[u], r[u], false, odd ? dodd : dd);
        else add_shifted<LPT>(w[u], r[u], odd && oddneg, dd);
      }
    }
  }
  template <int LPT>
  TC_DEV void deltas(int64_t pt, int, int64_t* dd) const {
    if (copy < 0 && windows_inside<LPT, false>(pt)) {
      for (int t = 0; t < B; t += 4) group4<LPT, false>(t, pt, dd, nullptr);
      return;
    }
    for (int t = (copy >= 0 ? copy : 0); t < (copy >= 0 ? copy + 1 : B); t++) {
      const int s = copy >= 0 ? 0 : (rev ? B - 1 - t : t) * j, q = s >> 5, r = s & 31;
      const bool neg = copy < 0 && (t & 1) && oddneg;
      uint32_t w[LPT + 2];
      window<LPT>(t, pt - 2 - q, w);
      add_shifted<LPT>(w, r, neg, dd);
    }
  }
  // dd of the even blocks and of the odd blocks separately (all added), so
  // one pass over the blocks serves both U(+2^j) = E + O and U(-2^j) = E - O
  template <int LPT>
  TC_DEV void deltas_split(int64_t pt, int64_t* de, int64_t* dodd) const {
    if (windows_inside<LPT, true>(pt)) {
      for (int t = 0; t < B; t += 4) group4<LPT, true>(t, pt, de, dodd);
      return;
    }
    for (int t = 0; t < B; t++) {
      const int s = t * j, q = s >> 5, r = s & 31;
      uint32_t w[LPT + 2];
      window<LPT>(t, pt - 2 - q, w);
      add_shifted<LPT>(w, r, false, (t & 1) ? dodd : de);
    }
  }
  TC_DEV bool store(int64_t p, uint32_t o, uint32_t&) {
    if (p < nout) stx<G>(out + p, o);
    return p < nout;
  }
  template <int LPT>
  TC_DEV void store_run(int64_t pt, const uint32_t* o, uint32_t&) {
    stx_run<G, LPT>(out + pt, o);
  }
};

// Deltas already in registers (dd[0] = delta(pt-1), dd[1+i] = delta(pt+i)),
// for passes without a right shift (no lookahead past the chunk).
template <int LPT>
struct RegSrc {
  static constexpr bool kWide = false;
  const int64_t* dd;
  uint32_t* out;
  int64_t nout;
  TC_DEV int64_t delta(int64_t) const { return 0; }
  template <int L>
  TC_DEV void deltas(int64_t, int, int64_t* d) const {
#pragma unroll
    for (int i = 0; i <= LPT; i++) d[i] = dd[i];
  }
  TC_DEV bool store(int64_t p, uint32_t o, uint32_t&) {
    if (p < nout) gst(out + p, o);
    return p < nout;
  }
  template <int L>
  TC_DEV void store_run(int64_t pt, const uint32_t* o, uint32_t&) {
    gst_run<L>(out + pt, o);
  }
};

// In-place two's-complement negation modulo 2^(32 n) (own limbs only).
template <bool G>
struct NegSrc {
  static constexpr bool kWide = false;
  uint32_t* v;
  TC_DEV int64_t delta(int64_t p) const { return -(int64_t)ldx<G>(v + p); }
  template <int LPT>
  TC_DEV void deltas(int64_t pt, int nown, int64_t* dd) const {
#pragma unroll
    for (int i = 0; i < LPT; i++)
      if (i < nown) dd[i + 1] = -(int64_t)ldx<G>(v + pt + i);
  }
  TC_DEV bool store(int64_t p, uint32_t o, uint32_t&) {
    stx<G>(v + p, o);
    return true;
  }
  template <int LPT>
  TC_DEV void store_run(int64_t pt, const uint32_t* o, uint32_t&) {
    stx_run<G, LPT>(v + pt, o);
  }
};

template <bool G>
struct RecompSrc {
  static constexpr bool kWide = false;
  const uint32_t* const* w;  // per-wave LDS array of nk coefficient pointers
  int nk;
  int64_t bl, wread;
  uint32_t* out;
  int64_t nstore;
  TC_DEV int64_t delta(int64_t p) const {
    int64_t kmax = p / bl;
    if (kmax > nk - 1) kmax = nk - 1;
    const int64_t kmin = p >= wread ? (p - wread) / bl + 1 : 0;
    int64_t d = 0;
    for (int64_t k = kmin; k <= kmax; k++) d += (int64_t)ldx<G>(w[k] + (p - k * bl));
    return d;
  }
  // dd[j] += w_k limbs at pt-1+j, j = 0..LPT, for every coefficient k whose
  // span [k bl, k bl + wread) meets the window: one run of loads per k
  template <int LPT>
  TC_DEV void deltas(int64_t pt, int, int64_t* dd) const {
    const int64_t lo = pt - 1, hi = pt + LPT - 1;  // window limbs lo..hi
    int64_t kmax = hi / bl;
    if (kmax > nk - 1) kmax = nk - 1;
    const int64_t kmin = lo >= wread ? (lo - wread) / bl + 1 : 0;
    for (int64_t k = kmin; k <= kmax; k++) {
      const uint32_t* src = w[k];
      const int64_t o = lo - k * bl;
      if (o >= 0 && o + LPT < wread) {
        uint32_t v[LPT + 1];
        ldx_run<G, LPT + 1>(src + o, v);
#pragma unroll
        for (int j = 0; j <= LPT; j++) dd[j] += (int64_t)v[j];
      } else {
#pragma unroll
        for (int j = 0; j <= LPT; j++) {
          const int64_t idx = o + j;
          if (idx >= 0 && idx < wread) dd[j] += (int64_t)ldx<G>(src + idx);
        }
      }
    }
  }
  TC_DEV bool store(int64_t p, uint32_t o, uint32_t& err) {
    if (p < nstore) stx<G>(out + p, o);
    else if (o != 0u) err |= ERRBIT_RANGE;
    return p < nstore;
  }
  template <int LPT>
  TC_DEV void store_run(int64_t pt, const uint32_t* o, uint32_t& err) {
    if (pt + LPT <= nstore) {
      stx_run<G, LPT>(out + pt, o);
    } else {
#pragma unroll
      for (int i = 0; i < LPT; i++) (void)store(pt + i, o[i], err);
    }
  }
};

// ---------------------------------------------------------------- helpers

// Index of the calling wave in its workgroup, as a wave-uniform (scalar)
// value: everything derived from it -- descriptors, pointers, divisors --
// then lives in scalar registers and is fetched by scalar loads.
TC_DEV int wave_in_block() { return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)); }

// Index of the descriptor holding global wave gw: descriptors carry their
// first wave index in `wave0` order (ascending).
template <class D>
TC_DEV int find_desc(const D* descs, int ndesc, const int64_t* wave0, int64_t gw) {
  int lo = 0, hi = ndesc - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (wave0[mid] <= gw) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// As find_desc; per_desc > 0 says every descriptor of the launch holds
// per_desc waves, so the index is a division (no dependent loads).
template <class D>
TC_DEV int find_desc_u(const D* descs, int ndesc, const int64_t* wave0, int64_t per_desc,
                       int64_t gw) {
  if (per_desc > 0) return (int)((uint32_t)gw / (uint32_t)per_desc);
  return find_desc(descs, ndesc, wave0, gw);
}

// The error word of a descriptor's product: its own word in a batch that
// reports per-item status, else the device's sticky word.
TC_DEV uint32_t* item_err(const Bases& b, int item) { return b.err + (int64_t)item * b.err_stride; }

TC_DEV void flag_error(uint32_t* err, uint32_t bits) {
  // one atomic per wave
  const uint64_t any = __ballot(bits != 0u);
  if (any) {
    uint32_t all = bits;
    for (int dist = 32; dist >= 1; dist >>= 1) all |= __shfl_xor(all, dist);
    if (lane_id() == 0) atomicOr(err, all);
  }
}

// ---------------------------------------------------------------- kernels

// The chunk a wave works on.  Waves [wave0 + node*nch, wave0 + (node+1)*nch)
// belong to one value; each takes a ticket from the value's counter, so the
// chunks it may wait on were claimed by waves that are already running.
struct WaveWork {
  int di;
  int64_t node, chunk;
  uint64_t* st;
};

// per_desc < 0: every descriptor has the same count and chunks, and waves go
// chunk position by chunk position over all values of the launch; within a
// position, -1 takes descriptor by descriptor (each over all nodes), -2 node
// by node (each over all descriptors, which read the same node's inputs).
TC_DEV void position_major(int64_t per_desc, uint32_t cnt, int ndesc, int64_t gw, int* di,
                           int64_t* node) {
  const uint32_t r = (uint32_t)gw % ((uint32_t)ndesc * cnt);
  if (per_desc == -2) {
    *di = (int)(r % (uint32_t)ndesc);
    *node = (int64_t)(r / (uint32_t)ndesc);
  } else {
    *di = (int)(r / cnt);
    *node = (int64_t)(r % cnt);
  }
}

// The descriptor and node of global wave gw (its chunk still unassigned).
template <class D>
TC_DEV WaveWork wave_locate(const D* descs, const int64_t* wave0, int ndesc, int64_t per_desc,
                            int64_t gw) {
  WaveWork w;
  if (per_desc < 0) {
    position_major(per_desc, (uint32_t)descs[0].count, ndesc, gw, &w.di, &w.node);
  } else {
    w.di = find_desc_u(descs, ndesc, wave0, per_desc, gw);
    const int64_t local = per_desc > 0 ? gw - (int64_t)w.di * per_desc : gw - wave0[w.di];
    w.node = (int64_t)((uint32_t)local / (uint32_t)descs[w.di].nchunks);
  }
  w.chunk = 0;
  w.st = nullptr;
  return w;
}

// wave_work for a launch whose block of four waves may take its tickets
// together: when all four waves are in the launch and belong to one value,
// wave 0 takes four consecutive chunks with one atomic (a value of a thousand
// chunks whose waves all start at once otherwise queues a thousand atomics on
// one word, about 12 ns each); else every wave takes its own.  Node by node,
// a value's waves are consecutive, so the block's first and last waves
// decide; position by position, consecutive waves go to different values
// unless the launch has only one.  The choice is the same for the whole
// block, so the block's barrier is reached by all four waves or by none.
// tk: one word of LDS.
template <class D>
TC_DEV WaveWork wave_work_block(const D* descs, const int64_t* wave0, int ndesc, int64_t per_desc,
                                int64_t total, uint64_t* status, unsigned long long* tk) {
  const int64_t gb = (int64_t)blockIdx.x * 4;
  const int64_t gw = gb + wave_in_block();
  WaveWork w = wave_locate(descs, wave0, ndesc, per_desc, gw);
  bool together = gb + 3 < total;
  if (together) {
    if (per_desc < 0) {
      together = ndesc == 1 && descs[0].count == 1 && descs[0].nchunks > 1;
    } else {
      const WaveWork a = wave_locate(descs, wave0, ndesc, per_desc, gb);
      const WaveWork b = wave_locate(descs, wave0, ndesc, per_desc, gb + 3);
      together = a.di == b.di && a.node == b.node && descs[a.di].nchunks > 1;
    }
  }
  if (!together) return wave_work(descs, wave0, ndesc, per_desc, gw, status);
  const D& d = descs[w.di];
  const int64_t nch = d.nchunks;
  w.st = status + d.status_off + w.node * lb_words(nch);
  if (threadIdx.x == 0)
    *tk = atomicAdd(reinterpret_cast<unsigned long long*>(&w.st[lb_ticket(nch)]), 4ull);
  __syncthreads();
  w.chunk = (int64_t)*tk + wave_in_block();
  return w;
}

template <class D>
TC_DEV WaveWork wave_work(const D* descs, const int64_t* wave0, int ndesc, int64_t per_desc,
                          int64_t gw, uint64_t* status) {
  WaveWork w = wave_locate(descs, wave0, ndesc, per_desc, gw);
  const D& d = descs[w.di];
  const int64_t nch = d.nchunks;
  w.chunk = 0;
  w.st = nullptr;
  if (nch > 1) {
    w.st = status + d.status_off + w.node * lb_words(nch);
    unsigned long long t = 0;
    if (lane_id() == 0) t = atomicAdd(reinterpret_cast<unsigned long long*>(&w.st[lb_ticket(nch)]), 1ull);
    w.chunk = (int64_t)readlane((uint32_t)t, 0);  // uniform: scalar chunk index
  }
  return w;
}

template <int LPT>
__global__ __launch_bounds__(256, 4) void k_step(const StepDesc* __restrict__ descs,
                                              const int64_t* __restrict__ wave0, int ndesc,
                                              int64_t total, int64_t per_desc, const Bases* __restrict__ bp,
                                              const DivEntry* __restrict__ divtab,
                                              uint64_t* status) {
  const Bases bases = *bp;
  const int64_t gw = (int64_t)blockIdx.x * 4 + wave_in_block();
  if (gw >= total) return;
  int di;
  int64_t node;
  if (per_desc < 0) {
    // every descriptor has the same count and chunks: waves go chunk position
    // by chunk position over all values (the chunk itself is the ticket)
    position_major(per_desc, (uint32_t)descs[0].count, ndesc, gw, &di, &node);
  } else {
    di = find_desc_u(descs, ndesc, wave0, per_desc, gw);
    const int64_t local = per_desc > 0 ? gw - (int64_t)di * per_desc : gw - wave0[di];
    node = (int64_t)((uint32_t)local / (uint32_t)descs[di].nchunks);
  }
  const StepDesc& D = descs[di];
  const int64_t nch = D.nchunks;
  // the chunk ticket is requested first and read last: the term set-up below
  // does not depend on it
  uint64_t* st = nullptr;
  unsigned long long tk = 0;
  if (nch > 1) {
    st = status + D.status_off + node * lb_words(nch);
    // an increment (not an add): its result is waited for only where it is read
    if (lane_id() == 0) tk = atomicInc(reinterpret_cast<unsigned int*>(&st[lb_ticket(nch)]), ~0u);
  }
  StepSrc<true> s;
  if (D.fast) {
    setup_terms(s, D, bases, node);
  } else {
    s.n = D.nterms;
    s.present = true;
#pragma unroll
    for (int i = 0; i < kStepTerms; i++)
      if (i < s.n) {
        load_term(s.t[i], D.t[i], bases, node, INT64_MAX);
        s.present = s.present && !(s.t[i].f & 2u);
      }
  }
  s.out = reinterpret_cast<uint32_t*>(resolve_d(bases, D.out)) + node * D.out_stride;
  const int64_t chunk = nch > 1 ? (int64_t)readlane((uint32_t)tk, 0) : 0;
  uint32_t eb = 0;
  if (chunk < nch) {
    EngCfg cfg;
    cfg.Y = D.Y;
    cfg.div[0] = D.div[0] >= 0 ? divtab + D.div[0] : nullptr;
    cfg.div[1] = D.div[1] >= 0 ? divtab + D.div[1] : nullptr;
    cfg.shr = D.shr;
    cfg.is_signed = true;
    cfg.prenorm = true;
    cfg.check_carry = false;
    (void)engine_chunk<LPT>(s, cfg, chunk, nch, st, eb);
  } else {
    eb |= ERRBIT_HANG;
  }
  flag_error(item_err(bases, D.item), eb);
}

// Source of a recomposing step: the node's shifted point products, each
// term's record read by scalar loads as the wave comes to it; terms whose
// shifted limbs miss the wave's windows are skipped.
struct RStepSrc {
  static constexpr bool kWide = true;
  const RStepDesc* D;
  const Bases* b;
  int64_t node;
  int n;
  uint32_t sgx;  // lane l: the sign of the node's point product l
  uint32_t* out;
  int64_t nstore;
  TC_DEV int64_t delta(int64_t) const { return 0; }
  // Terms go in groups of G: the group's records, then all its windows, are
  // requested before any is used, so their latencies overlap.  Launches of
  // few waves (2-limb lanes) take groups of four; wide launches one term at
  // a time, which keeps their registers, and occupancy, as they are
  // (measured: grouping every width slowed the 2^19- and 2^25-limb
  // products by 8 % and 4 %).
  template <int LPT>
  TC_DEV void deltas(int64_t pt, int, int64_t* dd) const {
    constexpr int N = LPT + 3;
    constexpr int G = LPT <= 2 ? 4 : 1;
    uint64_t acc[N];
#pragma unroll
    for (int i = 0; i < N; i++) acc[i] = 0;
    uint64_t bias = 0;
    const int64_t pl = pt - (int64_t)lane_id() * LPT;  // the same in every lane
    const int64_t p0 = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane(
                                      (int)(uint32_t)((uint64_t)pl >> 32)) << 32) |
                                  (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)pl));
    for (int i0 = 0; i0 < n; i0 += G) {
      uint32_t rec[G][8];
#pragma unroll
      for (int j = 0; j < G; j++) {
        const uint32_t* r = reinterpret_cast<const uint32_t*>(&D->c[i0 + j < n ? i0 + j : i0]);
#pragma unroll
        for (int q = 0; q < 8; q++) rec[j][q] = sld(r + q);
      }
      Term<true> t[G];
      bool use[G], in[G];
#pragma unroll
      for (int j = 0; j < G; j++) {
        const uint32_t f = rec[j][5];
        const int k = (int)(f >> 8) - 1;
        const int32_t width = (int32_t)rec[j][4];
        // the wave's windows span limbs p0-2-k .. p0+64 LPT+1-k of the term
        use[j] = i0 + j < n && p0 + 64 * LPT + 2 - k > 0 && p0 - 2 - k < width;
        in[j] = p0 - 2 - k >= 0 && p0 + 64 * LPT + 2 - k <= width;
        const int64_t off = (int64_t)(((uint64_t)rec[j][1] << 32) | rec[j][0]);
        const int64_t stride = (int64_t)(((uint64_t)rec[j][3] << 32) | rec[j][2]);
        const int si = (int)(int16_t)(rec[j][7] >> 16);
        t[j].ptr = reinterpret_cast<const uint32_t*>(base_of(*b, (int)(int8_t)(rec[j][7] & 0xffu)) +
                                                     off) + node * stride;
        t[j].width = width;
        t[j].f = f ^ (si >= 0 ? (readlane(sgx, si) & 1u) : 0u);
        t[j].mul = rec[j][6];
      }
      uint32_t w[G][N + 1];
#pragma unroll
      for (int j = 0; j < G; j++) {
        if (!use[j]) continue;
        const int64_t base = pt - 2 - t[j].k();
        if (in[j]) {
          gld_run<N + 1>(t[j].ptr + base, w[j]);
        } else {
          const int64_t top = t[j].width > 0 ? t[j].width - 1 : 0;
#pragma unroll
          for (int q = 0; q < N + 1; q++) {
            const int64_t x = base + q;
            const uint32_t v = gld(t[j].ptr + (x < 0 ? 0 : (x > top ? top : x)));
            w[j][q] = (x < 0 || x >= t[j].width) ? 0u : v;  // products: zero past the width
          }
        }
      }
#pragma unroll
      for (int j = 0; j < G; j++) {
        if (!use[j]) continue;
        t[j].template mac<N>(w[j], acc);
        bias += t[j].bias();
      }
    }
#pragma unroll
    for (int i = 0; i < N; i++) dd[i] += (int64_t)(acc[i] + bias);
  }
  TC_DEV bool store(int64_t p, uint32_t o, uint32_t& err) {
    if (p < nstore) gst(out + p, o);
    else if (o != 0u) err |= ERRBIT_RANGE;  // the product fits nstore limbs
    return p < nstore;
  }
  template <int LPT>
  TC_DEV void store_run(int64_t pt, const uint32_t* o, uint32_t& err) {
    if (pt + LPT <= nstore) {
      gst_run<LPT>(out + pt, o);
    } else {
#pragma unroll
      for (int i = 0; i < LPT; i++) (void)store(pt + i, o[i], err);
    }
  }
};

template <int LPT>
__global__ __launch_bounds__(256, 4) void k_rstep(const RStepDesc* __restrict__ descs,
                                               const int64_t* __restrict__ wave0, int ndesc,
                                               int64_t total, int64_t per_desc,
                                               const Bases* __restrict__ bp,
                                               const DivEntry* __restrict__ divtab,
                                               uint64_t* status) {
  const Bases bases = *bp;
  const int64_t gw = (int64_t)blockIdx.x * 4 + wave_in_block();
  if (gw >= total) return;
  const int di = find_desc_u(descs, ndesc, wave0, per_desc, gw);
  const int64_t local = per_desc > 0 ? gw - (int64_t)di * per_desc : gw - wave0[di];
  const RStepDesc& D = descs[di];
  const int64_t nch = D.nchunks;
  const int64_t node = (int64_t)((uint64_t)local / (uint64_t)nch);
  uint64_t* st = nullptr;
  unsigned long long tk = 0;
  if (nch > 1) {
    st = status + D.status_off + node * lb_words(nch);
    if (lane_id() == 0) tk = atomicInc(reinterpret_cast<unsigned int*>(&st[lb_ticket(nch)]), ~0u);
  }
  RStepSrc s;
  s.D = &D;
  s.b = &bases;
  s.node = node;
  s.n = D.nterms;
  s.nstore = D.nstore;
  s.out = reinterpret_cast<uint32_t*>(resolve_d(bases, D.out)) + node * D.out_stride;
  s.sgx = 0;
  const int lane = lane_id();
  if (lane < D.nsgn) {
    uint32_t x = *(const __attribute__((address_space(1))) uint8_t*)(base_of(bases, D.sgn_u_buf) +
                                                                       D.sgn_u_off +
                                                                       node * D.sgn_stride + lane);
    if (D.sgn_v_buf >= 0)
      x ^= *(const __attribute__((address_space(1))) uint8_t*)(base_of(bases, D.sgn_v_buf) +
                                                                 D.sgn_v_off +
                                                                 node * D.sgn_v_stride + lane);
    s.sgx = x;
  }
  const int64_t chunk = nch > 1 ? (int64_t)readlane((uint32_t)tk, 0) : 0;
  uint32_t eb = 0;
  if (chunk < nch) {
    EngCfg cfg;
    cfg.Y = D.Y;
    cfg.div[0] = D.div[0] >= 0 ? divtab + D.div[0] : nullptr;
    cfg.div[1] = D.div[1] >= 0 ? divtab + D.div[1] : nullptr;
    cfg.shr = D.shr;
    cfg.is_signed = true;
    cfg.prenorm = true;
    cfg.check_carry = false;
    (void)engine_chunk<LPT>(s, cfg, chunk, nch, st, eb);
  } else {
    eb |= ERRBIT_HANG;
  }
  flag_error(item_err(bases, D.item), eb);
}

// Sign of an evaluation, after the chunk's engine pass: one chunk turns a
// negative value into its magnitude in the same wave; several chunks leave
// that to k_evalneg, which needs the lowest non-zero limb.
template <int LPT>
TC_DEV void eval_finish(const ChunkOut& o, uint32_t* out, int64_t nout, uint8_t* sg,
                        uint64_t* st, int64_t chunk, int64_t nch, uint32_t& eb) {
  const int64_t Y = nout + 1;
  if (chunk + 1 == nch) {
    // The sign limb is 0 or all ones; anything else means the value overflowed
    // the child width.
    if (o.top != 0u && o.top != 0xffffffffu) eb |= ERRBIT_RANGE;
  }
  if (nch == 1) {
    const bool neg = o.top != 0u;
    if (neg) {
      NegSrc<true> ns;
      ns.v = out;
      EngCfg c2;
      c2.Y = nout;
      c2.div[0] = c2.div[1] = nullptr;
      c2.shr = 0;
      c2.is_signed = false;
      c2.prenorm = false;
      c2.check_carry = false;
      (void)engine_chunk<LPT>(ns, c2, 0, 1, nullptr, eb);
    }
    if (lane_id() == 0) *(__attribute__((address_space(1))) uint8_t*)sg = neg ? 1 : 0;
  } else {
    if (o.lowest_nz >= 0 && lane_id() == 0)
      atomicMax(reinterpret_cast<unsigned long long*>(&st[lb_marker(nch)]),
                (unsigned long long)(Y - o.lowest_nz));
    if (chunk + 1 == nch && lane_id() == 0) *sg = o.top != 0u ? 1 : 0;
  }
}

template <int LPT>
__global__ __launch_bounds__(256) void k_eval(const EvalDesc* __restrict__ descs,
                                              const int64_t* __restrict__ wave0, int ndesc,
                                              int64_t total, int64_t per_desc, const Bases* __restrict__ bp, uint64_t* status) {
  const Bases bases = *bp;
  const int64_t gw = (int64_t)blockIdx.x * 4 + wave_in_block();
  if (gw >= total) return;
  const WaveWork w = wave_work(descs, wave0, ndesc, per_desc, gw, status);
  const EvalDesc& D = descs[w.di];
  const int64_t nch = D.nchunks;
  uint32_t eb = 0;
  if (w.chunk >= nch) {
    flag_error(item_err(bases, D.item), ERRBIT_HANG);
    return;
  }
  EvalSrc<true> s;
  s.src = reinterpret_cast<const uint32_t*>(resolve_d(bases, D.src)) + w.node * D.src_stride;
  s.W = D.src_width;
  s.bl = D.bl;
  s.B = D.B;
  s.j = D.j;
  s.oddneg = D.odd_neg;
  s.copy = D.copy_block;
  s.rev = D.rev;
  s.out = reinterpret_cast<uint32_t*>(resolve_d(bases, D.out)) + w.node * D.out_stride;
  s.nout = D.nout;
  EngCfg cfg;
  cfg.Y = (int64_t)D.nout + 1;  // magnitude plus a sign limb
  cfg.div[0] = cfg.div[1] = nullptr;
  cfg.shr = 0;
  cfg.is_signed = true;
  cfg.prenorm = true;
  cfg.check_carry = false;
  uint8_t* sg = resolve_d(bases, D.sign) + w.node * D.sign_stride;
  if (!D.paired) {
    const ChunkOut o = engine_chunk<LPT>(s, cfg, w.chunk, nch, w.st, eb);
    eval_finish<LPT>(o, s.out, D.nout, sg, w.st, w.chunk, nch, eb);
  } else {
    // U(+2^j) = E + O and U(-2^j) = E - O from one pass over the blocks
    const int64_t pt = w.chunk * 64 * LPT + (int64_t)lane_id() * LPT;
    int64_t de[LPT + 1], dodd[LPT + 1], dd[LPT + 1];
#pragma unroll
    for (int i = 0; i <= LPT; i++) de[i] = dodd[i] = 0;
    s.template deltas_split<LPT>(pt, de, dodd);
    RegSrc<LPT> r;
    r.dd = dd;
    r.nout = D.nout;
#pragma unroll
    for (int i = 0; i <= LPT; i++) dd[i] = de[i] + dodd[i];
    r.out = s.out;
    const ChunkOut o1 = engine_chunk<LPT>(r, cfg, w.chunk, nch, w.st, eb);
    eval_finish<LPT>(o1, r.out, D.nout, sg, w.st, w.chunk, nch, eb);
#pragma unroll
    for (int i = 0; i <= LPT; i++) dd[i] = de[i] - dodd[i];
    r.out = reinterpret_cast<uint32_t*>(resolve_d(bases, D.out2)) + w.node * D.out_stride;
    // the second value's chunks follow the first's ticket order, so the
    // chunks its look-back waits on belong to waves already past their first
    uint64_t* st2 = nch > 1 ? status + D.status_off2 + w.node * lb_words(nch) : nullptr;
    uint8_t* sg2 = resolve_d(bases, D.sign2) + w.node * D.sign_stride;
    const ChunkOut o2 = engine_chunk<LPT>(r, cfg, w.chunk, nch, st2, eb);
    eval_finish<LPT>(o2, r.out, D.nout, sg2, st2, w.chunk, nch, eb);
  }
  flag_error(item_err(bases, D.item), eb);
}

// Magnitudes of the negative multi-chunk evaluations: with z the lowest
// non-zero limb of the two's complement x, -x has limbs 0 below z, -x_z at z
// and ~x_p above.
template <int LPT>
__global__ __launch_bounds__(256) void k_evalneg(const EvalDesc* __restrict__ descs,
                                                 const int64_t* __restrict__ wave0, int ndesc,
                                                 int64_t total, int64_t per_desc, const Bases* __restrict__ bp, uint64_t* status) {
  const Bases bases = *bp;
  const int64_t gw = (int64_t)blockIdx.x * 4 + wave_in_block();
  if (gw >= total) return;
  const int di = find_desc_u(descs, ndesc, wave0, per_desc, gw);
  const EvalDesc& D = descs[di];
  const int64_t nch = D.nchunks;
  const int64_t local = per_desc > 0 ? gw - (int64_t)di * per_desc : gw - wave0[di];
  const int64_t node = local / nch, c = local % nch;
  const uint8_t sg = *(resolve_d(bases, D.sign) + node * D.sign_stride);
  if (!sg) return;
  const uint64_t* st = status + D.status_off + node * lb_words(nch);
  const int64_t Y = (int64_t)D.nout + 1;
  const int64_t z = Y - (int64_t)st[lb_marker(nch)];
  uint32_t* out = reinterpret_cast<uint32_t*>(resolve_d(bases, D.out)) + node * D.out_stride;
  const int64_t pt = c * 64 * LPT + (int64_t)lane_id() * LPT;
  if (pt + LPT <= D.nout) {
    uint32_t x[LPT];
    gld_run<LPT>(out + pt, x);
#pragma unroll
    for (int i = 0; i < LPT; i++) {
      const int64_t p = pt + i;
      x[i] = p < z ? 0u : (p == z ? 0u - x[i] : ~x[i]);
    }
    gst_run<LPT>(out + pt, x);
  } else {
#pragma unroll
    for (int i = 0; i < LPT; i++) {
      const int64_t p = pt + i;
      if (p < D.nout) {
        const uint32_t x = gld(out + p);
        gst(out + p, p < z ? 0u : (p == z ? 0u - x : ~x));
      }
    }
  }
}

template <int LPT>
__global__ __launch_bounds__(256) void k_recomp(const RecompDesc* __restrict__ descs,
                                                const int64_t* __restrict__ wave0, int ndesc,
                                                int64_t total, int64_t per_desc, const Bases* __restrict__ bp, uint64_t* status) {
  const Bases bases = *bp;
  __shared__ const uint32_t* wptr[4][kMaxPts];
  __shared__ unsigned long long tk;
  const int64_t gw = (int64_t)blockIdx.x * 4 + wave_in_block();
  const int wv = threadIdx.x >> 6;
  if (gw >= total) return;
  const WaveWork w = wave_work_block(descs, wave0, ndesc, per_desc, total, status, &tk);
  const RecompDesc& D = descs[w.di];
  if (w.chunk >= D.nchunks) {
    flag_error(item_err(bases, D.item), ERRBIT_HANG);
    return;
  }
  const int lane = lane_id();
  if (lane < D.nk)
    wptr[wv][lane] = reinterpret_cast<const uint32_t*>(resolve_d(bases, D.w[lane])) +
                     w.node * D.w_stride;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  RecompSrc<true> s;
  s.w = wptr[wv];
  s.nk = D.nk;
  s.bl = D.bl;
  s.wread = D.wread;
  s.out = reinterpret_cast<uint32_t*>(resolve_d(bases, D.out)) + w.node * D.out_stride;
  s.nstore = D.nstore;
  EngCfg cfg;
  cfg.Y = D.ncompute;
  cfg.div[0] = cfg.div[1] = nullptr;
  cfg.shr = 0;
  cfg.is_signed = false;
  cfg.prenorm = true;
  cfg.check_carry = true;
  uint32_t eb = 0;
  (void)engine_chunk<LPT>(s, cfg, w.chunk, D.nchunks, w.st, eb);
  if (w.chunk == 0 && D.wlimbs > D.wread) {
    // every coefficient is non-negative and fits wread limbs (section 1's
    // w_k are sums of products of blocks): the limbs above must be zero, and
    // a set sign bit in the top limb means the interpolation gave a negative
    // value
    for (int k = 0; k < D.nk; k++)
      for (int64_t p = D.wread + lane; p < D.wlimbs; p += 64) {
        const uint32_t x = gld(wptr[wv][k] + p);
        if (x != 0u) eb |= (p == D.wlimbs - 1 && (x >> 31)) ? ERRBIT_SIGN : ERRBIT_RANGE;
      }
  }
  flag_error(item_err(bases, D.item), eb);
}

// Per-item status of a batch: 0 for a clean item, `code` for one whose
// error word is set.
__global__ void k_item_status(const uint32_t* __restrict__ item_err, int32_t* __restrict__ status,
                              int64_t n, int32_t code) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) status[i] = item_err[i] ? code : 0;
}

// Fault injection for tests of the exactness checks: flips bit 0 of each
// target limb (a point product between the leaves and its interpolation).
__global__ void k_flip(const DPtr* __restrict__ targets, int n, const Bases* __restrict__ bp) {
  const Bases b = *bp;
  const int i = (int)threadIdx.x;
  if (i < n) atomicXor(reinterpret_cast<uint32_t*>(resolve_d(b, targets[i])), 1u);
}

// Takes the device's sticky error word and clears it in one atomic step.
__global__ void k_take_error(uint32_t* err, uint32_t* out) {
  if (threadIdx.x == 0) *out = atomicExch(err, 0u);
}

// Several ranges in one launch: blockIdx.y picks range r, which clears
// ranges[2r + 1] 64-bit words from byte offset ranges[2r] of base.
__global__ void k_fill_ranges(uint8_t* base, const int64_t* ranges) {
  const int64_t off = ranges[2 * blockIdx.y], n = ranges[2 * blockIdx.y + 1];
  uint64_t* p = reinterpret_cast<uint64_t*>(base + off);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0ull;
}

// Schoolbook leaves.  `tpl` lanes (a power of two <= 64, inside one wave)
// share a leaf of n <= tpl*R limbs; lane l sums the columns of groups l and
// 2*tpl-1-l (R columns each), which balances the triangle of the column
// lengths.  Column sums are kept as a 32-bit low word plus a 64-bit high sum:
// t = u*v + lo (no overflow), lo = low(t), hi += high(t).  The tpl lanes then
// turn the columns into limbs with the same carry-table scan as the engine
// (segment width tpl).  us holds u (zero past n); vs[j + R] = v_j with R
// zeros on either side.  clo/chi: 2*tpl*R column words each.
TC_DEV void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int R>
// sq: u = v (vs holds u's limbs).  Column k of a square is then twice the
// sum of u_i u_(k-i) over i < k - i, plus u_(k/2)^2 when k is even: the pairs
// below the diagonal are formed once, about half the multiplications.
TC_DEV void leaf_core(const uint32_t* us, const uint32_t* vs, int n, int tpl, int l,
                      uint32_t* clo, uint64_t* chi, uint32_t* P, int p_width, bool active,
                      bool sq, uint32_t& eb) {
  const int C = 2 * tpl * R;  // columns covered (>= 2n)
  if (active) {
#pragma unroll
    for (int side = 0; side < 2; side++) {
      const int g = side == 0 ? l : 2 * tpl - 1 - l;
      const int k0 = g * R;
      uint32_t lo[R];
      uint64_t hi[R];
#pragma unroll
      for (int r = 0; r < R; r++) {
        lo[r] = 0u;
        hi[r] = 0u;
      }
      int ilo = k0 - n + 1;
      if (ilo < 0) ilo = 0;
      int ihi = k0 + R - 1;
      if (ihi > n - 1) ihi = n - 1;
      if (sq && ihi > (k0 + R - 1) / 2) ihi = (k0 + R - 1) / 2;
      for (int i = ilo; i <= ihi; i++) {
        const uint32_t a = us[i];
#pragma unroll
        for (int r = 0; r < R; r++) {
          uint32_t b = vs[k0 + r - i + R];
          if (sq && 2 * i >= k0 + r) b = 0u;  // on or above the diagonal
          const uint64_t t = (uint64_t)a * b + lo[r];
          lo[r] = (uint32_t)t;
          hi[r] += (uint32_t)(t >> 32);
        }
      }
      if (sq) {
#pragma unroll
        for (int r = 0; r < R; r++) {
          // lo + hi 2^32 doubled, then the diagonal square added
          hi[r] = (hi[r] << 1) | (lo[r] >> 31);
          lo[r] <<= 1;
          const int k = k0 + r;
          if ((k & 1) == 0 && k / 2 < n) {
            const uint64_t d = (uint64_t)us[k / 2] * us[k / 2];
            const uint64_t t = (uint64_t)lo[r] + (uint32_t)d;
            lo[r] = (uint32_t)t;
            hi[r] += (t >> 32) + (d >> 32);
          }
        }
      }
#pragma unroll
      for (int r = 0; r < R; r++) {
        clo[k0 + r] = lo[r];
        chi[k0 + r] = hi[r];
      }
    }
  }
  wave_sync();
  // columns -> limbs: z_k = lo_k + hi_{k-1}; e_k = lo32(z_k) + (z_{k-1} >> 32)
  constexpr int LP = 2 * R;
  const int k0 = l * LP;
  auto z = [&](int k) -> uint64_t {
    if (k < 0 || k >= C) return 0ull;
    return (uint64_t)clo[k] + (k > 0 ? chi[k - 1] : 0ull);
  };
  int64_t e[LP];
  uint32_t x[LP];
  {
    uint64_t zp = z(k0 - 1);
#pragma unroll
    for (int i = 0; i < LP; i++) {
      const uint64_t zc = z(k0 + i);
      e[i] = (int64_t)(zc & 0xffffffffull) + (int64_t)(zp >> 32);
      zp = zc;
    }
  }
  int c = 0;
  bool ones = true, zeros = true;
#pragma unroll
  for (int i = 0; i < LP; i++) {
    const int64_t s = e[i] + c;
    x[i] = (uint32_t)s;
    c = (int)(s >> 32);
    ones = ones && x[i] == 0xffffffffu;
    zeros = zeros && x[i] == 0u;
  }
  uint32_t inc = tab_make(c - (zeros ? 1 : 0), c, c + (ones ? 1 : 0));
  for (int dist = 1; dist < tpl; dist <<= 1) {
    const uint32_t y = __shfl_up(inc, dist, tpl);
    if (l >= dist) inc = tab_then(y, inc);
  }
  uint32_t exc = __shfl_up(inc, 1, tpl);
  if (l == 0) exc = TAB_ID;
  c = tab_apply(exc, 0);
#pragma unroll
  for (int i = 0; i < LP; i++) {
    const int64_t s = e[i] + c;
    x[i] = (uint32_t)s;
    c = (int)(s >> 32);
  }
  if (active) {
#pragma unroll
    for (int i = 0; i < LP; i++) {
      const int k = k0 + i;
      if (k < p_width) P[k] = x[i];
      else if (x[i] != 0u) eb |= ERRBIT_RANGE;
    }
    if (l == tpl - 1 && c != 0) eb |= ERRBIT_RANGE;
  }
}

template <int R>
__global__ __launch_bounds__(256) void k_leaf(const LeafDesc* __restrict__ descs,
                                              const int64_t* __restrict__ wg0, int ndesc,
                                              const Bases* __restrict__ bp, int tpl) {
  const Bases bases = *bp;
  extern __shared__ uint32_t smem[];
  const int lpw = 256 / tpl;
  const int lid = threadIdx.x / tpl, l = threadIdx.x % tpl;
  const int di = find_desc(descs, ndesc, wg0, (int64_t)blockIdx.x);
  const LeafDesc& D = descs[di];
  const int64_t leaf = ((int64_t)blockIdx.x - wg0[di]) * lpw + lid;
  const bool active = leaf < D.count;
  const int n = D.n;
  const int C = 2 * tpl * R;
  // per-leaf LDS: us[tpl*R], vs[tpl*R + 2R] (v shifted by R), lo[C], hi[2C]
  const int per = tpl * R + (tpl * R + 2 * R) + C + 2 * C;
  uint32_t* us = smem + lid * per;
  uint32_t* vs = us + tpl * R;
  uint32_t* clo = vs + tpl * R + 2 * R;
  uint64_t* chi = reinterpret_cast<uint64_t*>(clo + C);
  const uint32_t* U = reinterpret_cast<const uint32_t*>(resolve_d(bases, D.U)) + leaf * D.u_stride;
  const uint32_t* V = reinterpret_cast<const uint32_t*>(resolve_d(bases, D.V)) + leaf * D.v_stride;
  // a square: both operands at one address with one width (uniform: every
  // leaf of a descriptor shares the strides)
  const bool sq = resolve_d(bases, D.U) == resolve_d(bases, D.V) && D.u_stride == D.v_stride &&
                  D.u_width == D.v_width;
  for (int i = l; i < tpl * R; i += tpl) us[i] = (active && i < D.u_width) ? U[i] : 0u;
  for (int i = l; i < tpl * R + 2 * R; i += tpl) {
    const int j = i - R;
    vs[i] = (active && j >= 0 && j < D.v_width) ? V[j] : 0u;
  }
  __syncthreads();
  uint32_t eb = 0;
  uint32_t* P = reinterpret_cast<uint32_t*>(resolve_d(bases, D.P)) + leaf * D.p_stride;
  leaf_core<R>(us, vs, n, tpl, l, clo, chi, P, D.p_width, active, sq, eb);
  if (eb) atomicOr(item_err(bases, D.item), eb);
}

// ---------------------------------------------------------------- MFMA leaves
// Exact schoolbook product of wide leaves on the matrix cores.  The limbs of
// both operands are recoded into signed base-256 digits d_i in [-128, 127]
// (u = sum d_i 256^i; one carry scan), so the column sums
// c_k = sum_i a_i b_{k-i} are exact in int32 and u v = sum_k c_k 256^k.  With
// 32-byte blocks, c_{32K+r} = sum_J sum_s T_J[r][s] a_{32(K-J)+s} where
// T_J[r][s] = b_{32J+r-s}: for a tile of 32 output blocks this is a sum over J
// of 32x32x32 int8 products of the Toeplitz band T_J (from b's digits stored
// reversed) with 32 consecutive 32-byte blocks of a.  Lane (row r, half h)
// of the A operand holds T_J[r][16h..16h+15]; lane (column c, half h) of the
// B operand holds a's bytes 32(K0+c-J)+16h..+15; accumulator register v of
// lane l is row 8(v/4)+4(l/32)+v%4, column l%32.
//
// Registers 4q..4q+3 of lane (c, h) are thus the four digits of limb
// 8(K0+c)+2q+h of the product: each tile folds into 64-bit limb sums
// z_L = sum_e c_{4L+e} 2^(8e) straight from the accumulators, and one
// workgroup-wide carry pass turns the z_L into limbs.
typedef int tc_v4i __attribute__((ext_vector_type(4)));
typedef int tc_v16i __attribute__((ext_vector_type(16)));

struct MLeafShape {
  int Np;     // digits per operand, padded to a multiple of 32 (>= 4n+1)
  int NB;     // Np / 32
  int Y;      // product limbs covered by the column sums: Np / 2
  int oA, oR, oZ, oS;  // byte offsets in LDS
  int bytes;
};

// Register tiling of the band products for leaves of up to n limbs: a wave
// forms, for one band residue j, the products of SM bands of v (J = j + 32 s)
// with DM diagonals of u (d = t - s), into output tiles t = s + d.
struct MLeafTiling {
  int SM, DM, NTT;  // bands, diagonals, tiles touched (SM + DM - 1)
};
TC_HD MLeafTiling mleaf_tiling_of(int n) {
  const int NB = ((4 * n + 1) + 31) / 32;
  MLeafTiling t;
  t.SM = NB / 32 + 1;
  t.DM = (NB + 30) / 32 + 1;
  t.NTT = t.SM + t.DM - 1;
  return t;
}

// ntt: tiles of column sums the launch accumulates (its tiling's NTT).
TC_HD MLeafShape mleaf_shape_of(int n, int ntt) {
  MLeafShape s;
  s.Np = ((4 * n + 1) + 31) / 32 * 32;
  s.NB = s.Np / 32;
  s.Y = s.Np / 2;
  s.oA = 0;                          // 1024 zero bytes, Np digits, 3072 zero bytes
  s.oR = s.oA + 1024 + s.Np + 3072;  // reversed v: R[Np+31-i] = v_i, size Np+96
  s.oZ = (s.oR + s.Np + 96 + 15) / 16 * 16;  // limb sums z_L, 256 per tile
  s.oS = s.oZ + ntt * 264 * 8;       // scan scratch (Z padded: see zidx)
  s.bytes = s.oS + 64;
  return s;
}

// Exclusive workgroup scan of two carry tables at once (256 threads, DPP
// within each wave); returns the tables of all earlier threads.  tmp: 8 words
// of LDS.
TC_DEV void wg_exclusive_tab2(uint32_t& ta, uint32_t& tb, uint32_t* tmp) {
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  const uint32_t ia = scan_tab(ta), ib = scan_tab(tb);
  uint32_t ea = dpp<kDppWaveShr1>(TAB_ID, ia), eb = dpp<kDppWaveShr1>(TAB_ID, ib);
  if (lane == 63) {
    tmp[wave] = ia;
    tmp[4 + wave] = ib;
  }
  __syncthreads();
  uint32_t pa = TAB_ID, pb = TAB_ID;
  for (int w = 0; w < wave; w++) {
    pa = tab_then(pa, tmp[w]);
    pb = tab_then(pb, tmp[4 + w]);
  }
  __syncthreads();
  ta = tab_then(pa, ea);
  tb = tab_then(pb, eb);
}

// Index of limb sum L in the leaf's column-sum array: one spare entry per 32.
// An MFMA update touches limbs 8 r + c (lanes r = 0..31, c fixed), whose
// entries 8 r + r / 4 then fall on 32 distinct 8-byte bank pairs.
TC_DEV int zidx(int L) { return L + (L >> 5); }

// Signed base-256 digits of both n-limb operands.  With c_0 = 0 and
// c_{i+1} = [b_i + c_i >= 128] over the bytes b_i, digit d_i = b_i + c_i -
// 256 c_{i+1} and digit 4n = c_{4n}; the c_i are the carries of adding 0x80
// to every byte, and d_i is byte i of that sum minus 128.  So a limb x with
// carry-in c gives the four digits of x + 0x80808080 + c (each byte xor
// 0x80) and carry-out bit 32; a workgroup scan of the carry tables links the
// threads.  u's digits go to A8[i], v's reversed to R8[Np + 31 - i] (limbs
// past the widths are zero).
constexpr int kRecodeMaxL = 8;  // limbs per thread, n <= 2048

// This thread's limbs [t LP, (t+1) LP) of both operands (zero past the widths).
TC_DEV void recode_load(const uint32_t* U, int uw, const uint32_t* V, int vw, int n,
                        uint32_t (&xu)[kRecodeMaxL], uint32_t (&xv)[kRecodeMaxL]) {
  const int LP = (n + 255) / 256;
  const int l0 = threadIdx.x * LP;
#pragma unroll
  for (int i = 0; i < kRecodeMaxL; i++) {
    const int L = l0 + i;
    xu[i] = (i < LP && L < n && L < uw) ? gld(U + L) : 0u;
    xv[i] = (i < LP && L < n && L < vw) ? gld(V + L) : 0u;
  }
}

TC_DEV void recode_pair(const uint32_t (&xu)[kRecodeMaxL], const uint32_t (&xv)[kRecodeMaxL],
                        int n, int Np, int8_t* A8, int8_t* R8, uint32_t* tmp) {
  constexpr int MAXL = kRecodeMaxL;
  const int LP = (n + 255) / 256;
  const int l0 = threadIdx.x * LP;
  // carry out of this thread's limbs for carry-in 0 and 1
  uint32_t cu[2], cv[2];
#pragma unroll
  for (int cin = 0; cin < 2; cin++) {
    uint32_t a = (uint32_t)cin, b = (uint32_t)cin;
#pragma unroll
    for (int i = 0; i < MAXL; i++) {
      if (i < LP && l0 + i < n) {
        a = (uint32_t)(((uint64_t)xu[i] + 0x80808080u + a) >> 32);
        b = (uint32_t)(((uint64_t)xv[i] + 0x80808080u + b) >> 32);
      }
    }
    cu[cin] = a;
    cv[cin] = b;
  }
  uint32_t ta = tab_make((int)cu[0], (int)cu[0], (int)cu[1]);
  uint32_t tb = tab_make((int)cv[0], (int)cv[0], (int)cv[1]);
  wg_exclusive_tab2(ta, tb, tmp);
  uint32_t a = (uint32_t)tab_apply(ta, 0), b = (uint32_t)tab_apply(tb, 0);
  uint32_t* A32 = reinterpret_cast<uint32_t*>(A8);
  uint32_t* R32 = reinterpret_cast<uint32_t*>(R8 + Np + 28);  // dword of v digits 4L..4L+3
#pragma unroll
  for (int i = 0; i < MAXL; i++) {
    const int L = l0 + i;
    if (i < LP && L < n) {
      const uint64_t su = (uint64_t)xu[i] + 0x80808080u + a;
      const uint64_t sv = (uint64_t)xv[i] + 0x80808080u + b;
      a = (uint32_t)(su >> 32);
      b = (uint32_t)(sv >> 32);
      A32[L] = (uint32_t)su ^ 0x80808080u;
      R32[-L] = __builtin_bswap32((uint32_t)sv ^ 0x80808080u);
      if (L == n - 1) {
        A8[4 * n] = (int8_t)a;
        R8[Np + 31 - 4 * n] = (int8_t)b;
      }
    }
  }
}

// Carry propagation of Y signed 64-bit limb sums z (LDS, at zidx) by one
// workgroup: thread t owns limbs [t LP, (t+1) LP).  Pre-normalised limbs
// e_p = lo32(z_p) + (z_{p-1} >> 32) keep every carry in {-1, 0, 1}, so each
// thread summarises its limbs as a carry table and one workgroup scan gives
// every thread its carry-in.  The limbs are staged in LDS (stage, 4 Y bytes,
// may overlap nothing the pass reads) and leave as 16-byte stores; limbs
// p >= nstore must be zero, and so must the carry out of limb Y-1.
TC_DEV void wg_carry_store(const int64_t* z, int Y, uint32_t* stage, uint32_t* out, int nstore,
                           uint32_t* tmp, uint32_t& eb) {
  const int LP = (Y + 255) / 256;
  const int p0 = (int)threadIdx.x * LP;
  const int nown = Y - p0 <= 0 ? 0 : (Y - p0 >= LP ? LP : Y - p0);
  const int64_t zin = (p0 > 0 && nown > 0) ? z[zidx(p0 - 1)] : 0;
  int cc = 0;
  bool ones = true, zeros = true;
  int64_t zprev = zin;
  for (int i = 0; i < nown; i++) {
    const int64_t zz = z[zidx(p0 + i)];
    const int64_t s = (zz & 0xffffffffll) + (zprev >> 32) + cc;
    zprev = zz;
    const uint32_t x = (uint32_t)s;
    cc = (int)(s >> 32);
    ones = ones && x == 0xffffffffu;
    zeros = zeros && x == 0u;
  }
  uint32_t tab = nown ? tab_make(cc - (zeros ? 1 : 0), cc, cc + (ones ? 1 : 0)) : TAB_ID;
  uint32_t unused = TAB_ID;
  wg_exclusive_tab2(tab, unused, tmp);
  cc = tab_apply(tab, 0);
  zprev = zin;
  for (int i = 0; i < nown; i++) {
    const int p = p0 + i;
    const int64_t zz = z[zidx(p)];
    const int64_t s = (zz & 0xffffffffll) + (zprev >> 32) + cc;
    zprev = zz;
    const uint32_t x = (uint32_t)s;
    cc = (int)(s >> 32);
    stage[p] = x;
    if (p >= nstore && x != 0u) eb |= ERRBIT_RANGE;
  }
  if (nown > 0 && p0 + nown == Y && (cc != 0 || (zprev >> 32) != 0)) eb |= ERRBIT_RANGE;
  __syncthreads();
  const int ns = nstore < Y ? nstore : Y;
  for (int q = 4 * (int)threadIdx.x; q < ns; q += 1024) {
    if (q + 4 <= ns) {
      gst_run<4>(out + q, stage + q);
    } else {
      for (int i = q; i < ns; i++) gst(out + i, stage[i]);
    }
  }
}

// The digit convolution of one leaf on the matrix cores.  Column c of the
// convolution, c = 32 (32 t + col) + row, is tile t's MFMA output (row, col);
// band J of the reversed v (A operand) and diagonal d = t - J/32 of u (B
// operand) meet in tile t.  Writing J = j + 32 s, the A fragment depends on
// (j, s) and the B fragment on (j, d) only, so for each residue j a wave loads
// SM bands and DM diagonals once and issues all SM x DM products (tile
// t = s + d).  Waves split the 32 residues; their partial column sums meet in
// LDS by 64-bit atomic adds.  Bands and diagonals beyond the leaf's digits
// read zero pads.  Tiles are accumulated in passes of at most six, so three
// workgroups fit a CU by registers.
template <int SM, int DM>
__global__ __launch_bounds__(256, 3) void k_mleaf(const LeafDesc* __restrict__ descs,
                                                  const int64_t* __restrict__ wg0, int ndesc,
                                                  const Bases* __restrict__ bp) {
  constexpr int NTT = SM + DM - 1;
  constexpr int P = (NTT + 5) / 6;             // passes of at most six tiles
  constexpr int TP = (NTT + P - 1) / P;        // tiles per pass
  const Bases bases = *bp;
  extern __shared__ __attribute__((aligned(16))) uint8_t ml[];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int di = find_desc(descs, ndesc, wg0, (int64_t)blockIdx.x);
  const LeafDesc& D = descs[di];
  const int64_t leaf = (int64_t)blockIdx.x - wg0[di];
  const int n = D.n;
  const MLeafShape S = mleaf_shape_of(n, NTT);
  int8_t* A8 = reinterpret_cast<int8_t*>(ml + S.oA) + 1024;
  int8_t* R8 = reinterpret_cast<int8_t*>(ml + S.oR);
  int64_t* Z = reinterpret_cast<int64_t*>(ml + S.oZ);
  uint32_t* tmp = reinterpret_cast<uint32_t*>(ml + S.oS);
  // the operands are requested first; their latency covers the zeroing of
  // the digit areas (pads included) and of the column sums
  uint32_t xu[kRecodeMaxL], xv[kRecodeMaxL];
  {
    const uint32_t* U = reinterpret_cast<const uint32_t*>(resolve_d(bases, D.U)) + leaf * D.u_stride;
    const uint32_t* V = reinterpret_cast<const uint32_t*>(resolve_d(bases, D.V)) + leaf * D.v_stride;
    recode_load(U, D.u_width, V, D.v_width, n, xu, xv);
  }
  {
    tc_u4 z4;
    z4.x = z4.y = z4.z = z4.w = 0u;
    for (int i = tid; i < (S.oS - S.oA) / 16; i += 256) reinterpret_cast<tc_u4*>(ml + S.oA)[i] = z4;
  }
  __syncthreads();
  recode_pair(xu, xv, n, S.Np, A8, R8, tmp);
  __syncthreads();

  const int r = lane & 31, h = lane >> 5;
  const uint32_t* R32 = reinterpret_cast<const uint32_t*>(R8);
  // lane (r, h) of band J reads 16 bytes of R at o0 - 32 J; o0 mod 4 does
  // not depend on J
  const int o0 = S.Np + 31 - r + 16 * h;
  const uint32_t sh = (uint32_t)(o0 & 3);
  const int wv = __builtin_amdgcn_readfirstlane(wave);  // uniform: scalar loop control
  // digit weights 2^8, 2^16, 2^24, kept opaque so that the products stay
  // multiply-adds instead of becoming 64-bit shifts and adds
  int kw[4] = {1, 1 << 8, 1 << 16, 1 << 24};
#pragma unroll
  for (int e = 1; e < 4; e++) asm volatile("" : "+s"(kw[e]));
#pragma unroll
  for (int p = 0; p < P; p++) {
    tc_v16i acc[TP];
#pragma unroll
    for (int q = 0; q < TP; q++)
#pragma unroll
      for (int v = 0; v < 16; v++) acc[q][v] = 0;
    for (int j = wv; j < 32; j += 4) {
      tc_v4i a[SM];
      // band j + 32 sb starts 256 sb dwords below band j: one base per j (the
      // lowest band's), every fragment at a constant offset from it
      const uint32_t* Rj = R32 + (((o0 - 32 * j) >> 2) - 256 * (SM - 1));
#pragma unroll
      for (int sb = 0; sb < SM; sb++) {
        if (sb + DM - 1 < p * TP || sb > p * TP + TP - 1) continue;  // no tile of this pass
        uint32_t w[5];
#pragma unroll
        for (int k = 0; k < 5; k++) w[k] = Rj[256 * (SM - 1 - sb) + k];
#pragma unroll
        for (int k = 0; k < 4; k++) a[sb][k] = (int)__builtin_amdgcn_alignbyte(w[k + 1], w[k], sh);
      }
      // diagonal d: half h of the 32 digits from 32 (32 d + r - j)
      const int8_t* Bj = A8 + 32 * (r - j) + 16 * h;
#pragma unroll
      for (int d = 0; d < DM; d++) {
        if (d + SM - 1 < p * TP || d > p * TP + TP - 1) continue;
        const tc_v4i b = *reinterpret_cast<const tc_v4i*>(Bj + 1024 * d);
#pragma unroll
        for (int sb = 0; sb < SM; sb++) {
          const int t = sb + d - p * TP;
          if (t < 0 || t >= TP) continue;
          acc[t] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[sb], b, acc[t], 0, 0, 0);
        }
      }
    }
    // limb 8(32t+c)+2q+h gets digits 4q..4q+3 of this lane's registers
#pragma unroll
    for (int tt = 0; tt < TP; tt++) {
      const int t = p * TP + tt;
      if (t >= NTT) continue;
#pragma unroll
      for (int q = 0; q < 4; q++) {
        // sum of acc_e 2^(8e) as three 32 x 32 -> 64 signed multiply-adds
        int64_t zz = (int64_t)acc[tt][4 * q];
#pragma unroll
        for (int e = 1; e < 4; e++) zz += (int64_t)acc[tt][4 * q + e] * (int64_t)kw[e];
        atomicAdd(reinterpret_cast<unsigned long long*>(&Z[zidx(8 * (32 * t + r) + 2 * q + h)]),
                  (unsigned long long)zz);
      }
    }
  }
  __syncthreads();

  uint32_t eb = 0;
  uint32_t* P32 = reinterpret_cast<uint32_t*>(resolve_d(bases, D.P)) + leaf * D.p_stride;
  // the digit areas below Z are free now: they stage the limbs (4 Y <= oZ bytes)
  wg_carry_store(Z, S.Y, reinterpret_cast<uint32_t*>(ml), P32, (int)D.p_width, tmp, eb);
  flag_error(item_err(bases, D.item), eb);
}

// ---------------------------------------------------------------- launchers

static inline unsigned grid_for(int64_t waves) { return (unsigned)((waves + 3) / 4); }

hipError_t launch_step(int lpt, const StepDesc* d, const int64_t* w0, int nd, int64_t waves,
                       int64_t per_desc,
                       const Bases* b, const DivEntry* divtab, uint64_t* status,
                       hipStream_t st) {
  if (waves <= 0) return hipSuccess;
  dim3 g(grid_for(waves)), blk(256);
  switch (lpt) {
    case 2: hipLaunchKernelGGL(k_step<2>, g, blk, 0, st, d, w0, nd, waves, per_desc, b, divtab, status); break;
    case 4: hipLaunchKernelGGL(k_step<4>, g, blk, 0, st, d, w0, nd, waves, per_desc, b, divtab, status); break;
    case 16: hipLaunchKernelGGL(k_step<16>, g, blk, 0, st, d, w0, nd, waves, per_desc, b, divtab, status); break;
    default: hipLaunchKernelGGL(k_step<8>, g, blk, 0, st, d, w0, nd, waves, per_desc, b, divtab, status); break;
  }
  return hipGetLastError();
}

hipError_t launch_rstep(int lpt, const RStepDesc* d, const int64_t* w0, int nd, int64_t waves,
                        int64_t per_desc, const Bases* b, const DivEntry* divtab, uint64_t* status,
                        hipStream_t st) {
  if (waves <= 0) return hipSuccess;
  dim3 g(grid_for(waves)), blk(256);
  switch (lpt) {
    case 2: hipLaunchKernelGGL(k_rstep<2>, g, blk, 0, st, d, w0, nd, waves, per_desc, b, divtab, status); break;
    case 4: hipLaunchKernelGGL(k_rstep<4>, g, blk, 0, st, d, w0, nd, waves, per_desc, b, divtab, status); break;
    case 16: hipLaunchKernelGGL(k_rstep<16>, g, blk, 0, st, d, w0, nd, waves, per_desc, b, divtab, status); break;
    default: hipLaunchKernelGGL(k_rstep<8>, g, blk, 0, st, d, w0, nd, waves, per_desc, b, divtab, status); break;
  }
  return hipGetLastError();
}

hipError_t launch_eval(int lpt, bool neg_pass, const EvalDesc* d, const int64_t* w0, int nd,
                       int64_t waves, int64_t per_desc, const Bases* b, uint64_t* status,
                       hipStream_t st) {
  if (waves <= 0) return hipSuccess;
  dim3 g(grid_for(waves)), blk(256);
  if (neg_pass) {
    switch (lpt) {
      case 2: hipLaunchKernelGGL(k_evalneg<2>, g, blk, 0, st, d, w0, nd, waves, per_desc, b, status); break;
      case 4: hipLaunchKernelGGL(k_evalneg<4>, g, blk, 0, st, d, w0, nd, waves, per_desc, b, status); break;
      case 16: hipLaunchKernelGGL(k_evalneg<16>, g, blk, 0, st, d, w0, nd, waves, per_desc, b, status); break;
      default: hipLaunchKernelGGL(k_evalneg<8>, g, blk, 0, st, d, w0, nd, waves, per_desc, b, status); break;
    }
    return hipGetLastError();
  }
  switch (lpt) {
    case 2: hipLaunchKernelGGL(k_eval<2>, g, blk, 0, st, d, w0, nd, waves, per_desc, b, status); break;
    case 4: hipLaunchKernelGGL(k_eval<4>, g, blk, 0, st, d, w0, nd, waves, per_desc, b, status); break;
    case 16: hipLaunchKernelGGL(k_eval<16>, g, blk, 0, st, d, w0, nd, waves, per_desc, b, status); break;
    default: hipLaunchKernelGGL(k_eval<8>, g, blk, 0, st, d, w0, nd, waves, per_desc, b, status); break;
  }
  return hipGetLastError();
}

hipError_t launch_recomp(int lpt, const RecompDesc* d, const int64_t* w0, int nd, int64_t waves,
                         int64_t per_desc, const Bases* b, uint64_t* status, hipStream_t st) {
  if (waves <= 0) return hipSuccess;
  dim3 g(grid_for(waves)), blk(256);
  switch (lpt) {
    case 2: hipLaunchKernelGGL(k_recomp<2>, g, blk, 0, st, d, w0, nd, waves, per_desc, b, status); break;
    case 4: hipLaunchKernelGGL(k_recomp<4>, g, blk, 0, st, d, w0, nd, waves, per_desc, b, status); break;
    case 16: hipLaunchKernelGGL(k_recomp<16>, g, blk, 0, st, d, w0, nd, waves, per_desc, b, status); break;
    default: hipLaunchKernelGGL(k_recomp<8>, g, blk, 0, st, d, w0, nd, waves, per_desc, b, status); break;
  }
  return hipGetLastError();
}

int mleaf_lds_bytes(int n) { return mleaf_shape_of(n, mleaf_tiling_of(n).NTT).bytes; }

// The instantiation for a launch whose widest leaf has n limbs (DM is SM or
// SM + 1 for every n in (0, 2048]).
#define TC_MLEAF_CASES(X) X(1, 2) X(2, 2) X(2, 3) X(3, 3) X(3, 4) X(4, 4) X(4, 5) X(5, 5) X(5, 6) X(6, 6) X(6, 7) \
  X(7, 7) X(7, 8) X(8, 8) X(8, 9) X(9, 9)

typedef void (*MLeafFn)(const LeafDesc*, const int64_t*, int, const Bases*);
static MLeafFn mleaf_fn(int n) {
  const MLeafTiling t = mleaf_tiling_of(n);
#define TC_MLEAF_PICK(a, b) \
  if (t.SM == a && t.DM == b) return &k_mleaf<a, b>;
  TC_MLEAF_CASES(TC_MLEAF_PICK)
#undef TC_MLEAF_PICK
  return nullptr;
}

hipError_t launch_mleaf(int n, const LeafDesc* d, const int64_t* wg0, int nd, int64_t wgs,
                        const Bases* b, hipStream_t st) {
  if (wgs <= 0) return hipSuccess;
  const MLeafFn fn = mleaf_fn(n);
  if (!fn) return hipErrorInvalidValue;
  const MLeafShape s = mleaf_shape_of(n, mleaf_tiling_of(n).NTT);
  dim3 g((unsigned)wgs), blk(256);
  hipLaunchKernelGGL(fn, g, blk, (size_t)s.bytes, st, d, wg0, nd, b);
  return hipGetLastError();
}

hipError_t set_mleaf_lds_limit(size_t bytes) {
#define TC_MLEAF_ATTR(a, b)                                                                    \
  {                                                                                            \
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_mleaf<a, b>),  \
                                             hipFuncAttributeMaxDynamicSharedMemorySize,       \
                                             (int)bytes);                                      \
    if (e != hipSuccess) return e;                                                             \
  }
  TC_MLEAF_CASES(TC_MLEAF_ATTR)
#undef TC_MLEAF_ATTR
  return hipSuccess;
}

hipError_t launch_fill_ranges(uint8_t* base, const int64_t* ranges, int nr, int64_t max_words,
                              hipStream_t st) {
  if (nr <= 0 || max_words <= 0) return hipSuccess;
  if (nr > 65535) return hipErrorInvalidValue;
  int64_t blocks = (max_words + 255) / 256;
  if (blocks > 2048) blocks = 2048;
  hipLaunchKernelGGL(k_fill_ranges, dim3((unsigned)blocks, (unsigned)nr), dim3(256), 0, st, base,
                     ranges);
  return hipGetLastError();
}

hipError_t launch_item_status(const uint32_t* item_err, int32_t* status, int64_t n, int32_t code,
                              hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_item_status, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, item_err,
                     status, n, code);
  return hipGetLastError();
}

hipError_t launch_flip(const DPtr* targets, int n, const Bases* b, hipStream_t st) {
  if (n <= 0 || n > 256) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_flip, dim3(1), dim3(256), 0, st, targets, n, b);
  return hipGetLastError();
}

hipError_t launch_take_error(uint32_t* err, uint32_t* out, hipStream_t st) {
  hipLaunchKernelGGL(k_take_error, dim3(1), dim3(64), 0, st, err, out);
  return hipGetLastError();
}

LeafShape leaf_shape(int n) {
  LeafShape s;
  s.R = n <= 64 * 4 ? 4 : 8;
  int tpl = 1;
  while (tpl * s.R < n) tpl <<= 1;
  if (tpl < 4) tpl = 4;
  s.tpl = tpl;
  const int C = 2 * tpl * s.R;
  const int per = tpl * s.R + (tpl * s.R + 2 * s.R) + C + 2 * C;
  s.lds_bytes = (size_t)(256 / tpl) * per * sizeof(uint32_t);
  return s;
}

hipError_t launch_leaf(const LeafShape& s, const LeafDesc* d, const int64_t* wg0, int nd,
                       int64_t wgs, const Bases* b, hipStream_t st) {
  if (wgs <= 0) return hipSuccess;
  if (s.tpl > 64 || s.tpl < 4) return hipErrorInvalidValue;
  dim3 g((unsigned)wgs), blk(256);
  if (s.R == 4)
    hipLaunchKernelGGL(k_leaf<4>, g, blk, s.lds_bytes, st, d, wg0, nd, b, s.tpl);
  else
    hipLaunchKernelGGL(k_leaf<8>, g, blk, s.lds_bytes, st, d, wg0, nd, b, s.tpl);
  return hipGetLastError();
}

}  // namespace tc
