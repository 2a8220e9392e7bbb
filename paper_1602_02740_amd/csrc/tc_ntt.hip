// tc_ntt.hip -- leaves formed by an exact number-theoretic transform on
// gfx950: section 5's Toom-Cook over an FFT product, with the FFT replaced by
// a transform over p = 2^64 - 2^32 + 1 (exact, so the product is bit-exact).
//
// A leaf P = U V cuts both operands into pieces of `bits` bits, transforms
// them (length N = R C, four steps), multiplies pointwise, transforms back and
// adds the coefficients at their bit offsets with carry.  With the array read
// as R rows of C elements, x[r C + c]:
//
//   k_ntt_cols<false>  per column c: R-point transform over r (decimation in
//                      frequency, so row p holds index jr = rev_R(p)), then
//                      the twiddle w_N^(c jr); the pieces are read from the
//                      limbs here
//   k_ntt_rows<0>      per row: C-point transform of the U arrays
//   k_ntt_rows<1>      per row: C-point transform of the V arrays, the
//                      pointwise product with the U row and N^-1, the
//                      inverse C-point transform (decimation in time, back
//                      to natural order) and the inverse twiddle
//   k_ntt_cols<true>   per column: inverse R-point transform, natural order
//   k_ntt_carry        limb sums of the coefficients (staged in LDS), carry
//                      look-back
//
// Position (p, q) of a forward transform holds X[rev_R(p) + R rev_C(q)]; the
// pointwise product does not care, and the inverse steps undo the order.
// With R = 1 (N <= 8192) the row kernels read the pieces themselves.  The
// R- and C-point transforms run in LDS, two stages per pass (one workgroup
// holds a row, or a tile of R x 8192/R column elements), with roots w_8192^k
// from a table.
#include <hip/hip_runtime.h>

#include "tc_engine.hpp"
#include "tc_field.hpp"
#include "tc_internal.hpp"

namespace tc {
namespace ntt {

TC_DEV uint32_t* item_err(const Bases& b, int item) { return b.err + (int64_t)item * b.err_stride; }

TC_DEV void flag_error(uint32_t* err, uint32_t bits) {
  const uint64_t any = __ballot(bits != 0u);
  if (any) {
    uint32_t all = bits;
    for (int dist = 32; dist >= 1; dist >>= 1) all |= __shfl_xor(all, dist);
    if (lane_id() == 0) atomicOr(err, all);
  }
}

// Descriptor of unit u: descriptors carry their first unit in `u0`.
TC_DEV int find_unit(const int64_t* u0, int nd, int64_t u) {
  int lo = 0, hi = nd - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (u0[mid] <= u) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Piece i of an operand of `width` limbs: bits [bits i, bits i + bits).
TC_DEV uint64_t piece(const uint32_t* u, int64_t width, int bits, int64_t i) {
  const int64_t o = (int64_t)bits * i;
  const int64_t L = o >> 5;
  const uint32_t lo = L < width ? gld(u + L) : 0u;
  const uint32_t hi = L + 1 < width ? gld(u + L + 1) : 0u;
  return ((((uint64_t)hi << 32) | lo) >> (o & 31)) & ((1ull << bits) - 1);
}

// w_N^e for e < N = 2^logN <= 2^24, from w_2^24^(E mod 4096) w_2^24^(4096 floor(E/4096)),
// E = e 2^(24 - logN); inv: the inverse root.
TC_DEV uint64_t twiddle(const uint64_t* roots, uint64_t e, int logN, bool inv) {
  const uint64_t E = e << (24 - logN);
  const uint64_t lo = roots[(inv ? kNttLoInv : kNttLo) + (E & 4095u)];
  const uint64_t hi = roots[(inv ? kNttHiInv : kNttHi) + (E >> 12)];
  return fp_mul(lo, hi);
}

// ncol transforms of length 2^logL (1 <= logL <= 13), column-major in X.
// Forward: decimation in frequency (natural order in, bit-reversed out);
// INV: decimation in time with the inverse roots (bit-reversed in, natural
// out).  A stage with half-blocks of h = 2^lh uses w_2h^i = w_8192^(i 2^(12 - lh)),
// read from the stage's own contiguous table (consecutive threads, consecutive
// entries: one request per cache line rather than one per lane).
// Stages run in pairs (radix 4: a thread takes the quad a, a + h, a + 2h,
// a + 3h of two consecutive stages, so one LDS round trip and one barrier
// serve both); an odd stage count adds one radix-2 stage (the first stage
// forward, the last inverse).
template <bool INV>
TC_DEV void lds_transform(uint64_t* X, int logL, int ncol, const uint64_t* roots) {
  const uint64_t* T4 = roots + (INV ? kNttTw4Inv : kNttTw4Fwd);
  const uint64_t* T2 = roots + (INV ? kNttTw2Inv : kNttTw2Fwd);
  const int nthr = (int)blockDim.x, tid = (int)threadIdx.x;
  auto radix2 = [&](int lh) {
    const int half = 1 << (logL - 1), h = 1 << lh;
    const int nb = half * ncol;
    for (int b = tid; b < nb; b += nthr) {
      const int col = b >> (logL - 1);
      const int bb = b & (half - 1);
      const int i = bb & (h - 1);
      const int at = (col << logL) + ((bb >> lh) << (lh + 1)) + i;
      const uint64_t w = T2[h - 1 + i];
      const uint64_t a = X[at], c = X[at + h];
      if (!INV) {
        X[at] = fp_add(a, c);
        X[at + h] = fp_mul(fp_sub(a, c), w);
      } else {
        const uint64_t cw = fp_mul(c, w);
        X[at] = fp_add(a, cw);
        X[at + h] = fp_sub(a, cw);
      }
    }
    __syncthreads();
  };
  // quads of the stage pair with half-blocks 2^lo and 2^(lo + 1)
  auto radix4 = [&](int lo) {
    const int q4 = 1 << (logL - 2), h = 1 << lo;
    const int nq = q4 * ncol;
    for (int b = tid; b < nq; b += nthr) {
      const int col = b >> (logL - 2);
      const int bb = b & (q4 - 1);
      const int i = bb & (h - 1);
      const int at = (col << logL) + ((bb >> lo) << (lo + 2)) + i;
      const uint64_t* T = T4 + 3 * (h - 1);
      const uint64_t wh0 = T[i];          // w_4h^i
      const uint64_t wh1 = T[h + i];      // w_4h^(i+h)
      const uint64_t wl = T[2 * h + i];   // w_2h^i
      const uint64_t x0 = X[at], x1 = X[at + h], x2 = X[at + 2 * h], x3 = X[at + 3 * h];
      if (!INV) {
        // stage lo+1 (pairs at distance 2h), then stage lo (distance h)
        const uint64_t y0 = fp_add(x0, x2), y2 = fp_mul(fp_sub(x0, x2), wh0);
        const uint64_t y1 = fp_add(x1, x3), y3 = fp_mul(fp_sub(x1, x3), wh1);
        X[at] = fp_add(y0, y1);
        X[at + h] = fp_mul(fp_sub(y0, y1), wl);
        X[at + 2 * h] = fp_add(y2, y3);
        X[at + 3 * h] = fp_mul(fp_sub(y2, y3), wl);
      } else {
        // stage lo (distance h), then stage lo+1 (distance 2h)
        const uint64_t c1 = fp_mul(x1, wl), c3 = fp_mul(x3, wl);
        const uint64_t y0 = fp_add(x0, c1), y1 = fp_sub(x0, c1);
        const uint64_t y2 = fp_add(x2, c3), y3 = fp_sub(x2, c3);
        const uint64_t d2 = fp_mul(y2, wh0), d3 = fp_mul(y3, wh1);
        X[at] = fp_add(y0, d2);
        X[at + 2 * h] = fp_sub(y0, d2);
        X[at + h] = fp_add(y1, d3);
        X[at + 3 * h] = fp_sub(y1, d3);
      }
    }
    __syncthreads();
  };
  // octets of three stages with half-blocks 4h, 2h, h (h = 2^lo): a thread
  // takes x[m] = X[at + m h], m < 8, so one LDS round trip and one barrier
  // serve three stages; stage 2^s h pairs elements 2^s apart in the octet,
  // with the twiddle of the pair's position i + (m mod 2^s) h in its half-block
  auto radix8 = [&](int lo) {
    const int q8 = 1 << (logL - 3), h = 1 << lo;
    const int nq = q8 * ncol;
    for (int b = tid; b < nq; b += nthr) {
      const int col = b >> (logL - 3);
      const int bb = b & (q8 - 1);
      const int i = bb & (h - 1);
      const int at = (col << logL) + ((bb >> lo) << (lo + 3)) + i;
      uint64_t x[8];
#pragma unroll
      for (int m = 0; m < 8; m++) x[m] = X[at + m * h];
      const uint64_t* t4 = T2 + (4 * h - 1) + i;  // w_8h^(i + m h)
      const uint64_t* t2 = T2 + (2 * h - 1) + i;  // w_4h^(i + m h)
      const uint64_t w1 = T2[h - 1 + i];          // w_2h^i
      if (!INV) {
#pragma unroll
        for (int m = 0; m < 4; m++) {
          const uint64_t a = x[m], c = x[m + 4];
          x[m] = fp_add(a, c);
          x[m + 4] = fp_mul(fp_sub(a, c), t4[m * h]);
        }
#pragma unroll
        for (int g = 0; g < 8; g += 4)
#pragma unroll
          for (int m = 0; m < 2; m++) {
            const uint64_t a = x[g + m], c = x[g + m + 2];
            x[g + m] = fp_add(a, c);
            x[g + m + 2] = fp_mul(fp_sub(a, c), t2[m * h]);
          }
#pragma unroll
        for (int g = 0; g < 8; g += 2) {
          const uint64_t a = x[g], c = x[g + 1];
          x[g] = fp_add(a, c);
          x[g + 1] = fp_mul(fp_sub(a, c), w1);
        }
      } else {
#pragma unroll
        for (int g = 0; g < 8; g += 2) {
          const uint64_t c = fp_mul(x[g + 1], w1);
          x[g + 1] = fp_sub(x[g], c);
          x[g] = fp_add(x[g], c);
        }
#pragma unroll
        for (int g = 0; g < 8; g += 4)
#pragma unroll
          for (int m = 0; m < 2; m++) {
            const uint64_t c = fp_mul(x[g + m + 2], t2[m * h]);
            x[g + m + 2] = fp_sub(x[g + m], c);
            x[g + m] = fp_add(x[g + m], c);
          }
#pragma unroll
        for (int m = 0; m < 4; m++) {
          const uint64_t c = fp_mul(x[m + 4], t4[m * h]);
          x[m + 4] = fp_sub(x[m], c);
          x[m] = fp_add(x[m], c);
        }
      }
#pragma unroll
      for (int m = 0; m < 8; m++) X[at + m * h] = x[m];
    }
    __syncthreads();
  };
  // forward: the largest half-blocks first, three stages at a time, then
  // the one or two smallest; inverse: the mirror image
  if (!INV) {
    int lh = logL - 1;
    for (; lh >= 2; lh -= 3) radix8(lh - 2);
    if (lh == 1) radix4(0);
    else if (lh == 0) radix2(0);
  } else {
    int lh = 0;
    if (logL % 3 == 1) radix2(lh++);
    else if (logL % 3 == 2) { radix4(0); lh = 2; }
    for (; lh < logL; lh += 3) radix8(lh);
  }
}

TC_DEV uint32_t bit_reverse(uint32_t x, int bits) { return bits ? __brev(x) >> (32 - bits) : 0u; }

// Column tile of a descriptor: 2^logT columns with R 2^logT <= 8192.
TC_DEV int tile_log(const NttDesc& D) {
  const int t = 13 - D.logR;
  return D.logC < t ? D.logC : t;
}

}  // namespace ntt

using namespace ntt;

// Threads of a transform workgroup: sixteen waves share one 64 KiB row or
// tile, so even a transform of a few hundred rows keeps every SIMD busy.  The
// kernels are held to eight waves per SIMD (64 VGPRs), so that two such
// workgroups, LDS permitting, share a CU.
constexpr int kNttThreads = 1024;

// One workgroup per (array, column tile).  Forward: arrays are the U arrays
// then the V arrays (U only for squares) and the input is the pieces; inverse:
// the product arrays (V arrays, U for squares), in place.
template <bool INV>
__global__ __launch_bounds__(kNttThreads, 8) void k_ntt_cols(const NttDesc* __restrict__ descs,
                                                  const int64_t* __restrict__ wg0, int nd,
                                                  const Bases* __restrict__ bp,
                                                  const uint64_t* __restrict__ roots) {
  extern __shared__ __attribute__((aligned(16))) uint64_t X[];
  const Bases bases = *bp;
  const int di = find_unit(wg0, nd, (int64_t)blockIdx.x);
  const NttDesc& D = descs[di];
  const int64_t local = (int64_t)blockIdx.x - wg0[di];
  const int logR = D.logR, logC = D.logC, logT = tile_log(D);
  const int R = 1 << logR, C = 1 << logC;
  const int64_t tiles = (int64_t)1 << (logC - logT);
  const int64_t arr = local / tiles;
  const int c0 = (int)(local % tiles) << logT;
  const int64_t N = (int64_t)1 << (logR + logC);
  uint64_t* base = reinterpret_cast<uint64_t*>(resolve(bases, D.X));
  const int64_t slot = INV ? (D.square ? arr : D.count + arr) : arr;
  uint64_t* A = base + slot * N;
  const int nel = R << logT;
  const uint32_t* src = nullptr;
  int64_t width = 0;
  if (!INV) {
    const bool isv = arr >= D.count;
    const int64_t leaf = isv ? arr - D.count : arr;
    src = reinterpret_cast<const uint32_t*>(resolve(bases, isv ? D.V : D.U)) +
          leaf * (isv ? D.v_stride : D.u_stride);
    width = isv ? D.v_width : D.u_width;
  }
  for (int e = (int)threadIdx.x; e < nel; e += kNttThreads) {
    const int r = e >> logT, c = e & ((1 << logT) - 1);
    const int64_t g = ((int64_t)r << logC) + c0 + c;
    X[(c << logR) + r] = INV ? A[g] : piece(src, width, D.bits, g);
  }
  __syncthreads();
  lds_transform<INV>(X, logR, 1 << logT, roots);
  for (int e = (int)threadIdx.x; e < nel; e += kNttThreads) {
    const int p = e >> logT, c = e & ((1 << logT) - 1);
    uint64_t x = X[(c << logR) + p];
    if (!INV)
      x = fp_mul(x, twiddle(roots, (uint64_t)(c0 + c) * bit_reverse((uint32_t)p, logR),
                            logR + logC, false));
    A[((int64_t)p << logC) + c0 + c] = x;
  }
}

// One workgroup per (leaf, row).  MODE 0: forward C-point transform of the U
// arrays (not launched for squares).  MODE 1: forward transform of the V
// arrays (U for squares), pointwise product with the transformed U row (the
// row itself for squares) times N^-1, inverse C-point transform and, with
// R > 1, the inverse twiddle w_N^-(c jr).
template <int MODE>
__global__ __launch_bounds__(kNttThreads, 8) void k_ntt_rows(const NttDesc* __restrict__ descs,
                                                  const int64_t* __restrict__ wg0, int nd,
                                                  const Bases* __restrict__ bp,
                                                  const uint64_t* __restrict__ roots) {
  extern __shared__ __attribute__((aligned(16))) uint64_t X[];
  const Bases bases = *bp;
  const int di = find_unit(wg0, nd, (int64_t)blockIdx.x);
  const NttDesc& D = descs[di];
  const int64_t local = (int64_t)blockIdx.x - wg0[di];
  const int logR = D.logR, logC = D.logC;
  const int C = 1 << logC;
  const int64_t leaf = local >> logR;
  const int p = (int)(local & ((1 << logR) - 1));
  const int64_t N = (int64_t)1 << (logR + logC);
  uint64_t* base = reinterpret_cast<uint64_t*>(resolve(bases, D.X));
  uint64_t* Ua = base + leaf * N;
  uint64_t* Va = D.square ? Ua : base + (D.count + leaf) * N;
  uint64_t* A = MODE == 0 ? Ua : Va;
  const int64_t row = (int64_t)p << logC;
  if (logR == 0) {
    // no column pass: this row is the whole array, read from the pieces
    const bool isv = MODE == 1 && !D.square;
    const uint32_t* src = reinterpret_cast<const uint32_t*>(resolve(bases, isv ? D.V : D.U)) +
                          leaf * (isv ? D.v_stride : D.u_stride);
    const int64_t width = isv ? D.v_width : D.u_width;
    for (int q = (int)threadIdx.x; q < C; q += kNttThreads) X[q] = piece(src, width, D.bits, q);
  } else {
    for (int q = (int)threadIdx.x; q < C; q += kNttThreads) X[q] = A[row + q];
  }
  __syncthreads();
  lds_transform<false>(X, logC, 1, roots);
  if (MODE == 0) {
    for (int q = (int)threadIdx.x; q < C; q += kNttThreads) A[row + q] = X[q];
    return;
  }
  for (int q = (int)threadIdx.x; q < C; q += kNttThreads) {
    const uint64_t y = D.square ? X[q] : Ua[row + q];
    X[q] = fp_mul(fp_mul(X[q], y), D.ninv);
  }
  __syncthreads();
  lds_transform<true>(X, logC, 1, roots);
  const uint32_t jr = bit_reverse((uint32_t)p, logR);
  for (int c = (int)threadIdx.x; c < C; c += kNttThreads) {
    uint64_t x = X[c];
    if (logR > 0) x = fp_mul(x, twiddle(roots, (uint64_t)c * jr, logR + logC, true));
    A[row + c] = x;
  }
}

// The product limbs from the convolution coefficients c_k (natural order,
// below p): limb p receives bits [32 p, 32 p + 32) of every c_k 2^(bits k),
// at most ceil(95 / bits) + 1 terms below 2^32 each, so the limb sums stay
// far below 2^63 and the engine's pre-normalised carry applies.
// The chunk's coefficients are staged in LDS (S[k - k0]) by the wave first.
TC_DEV int64_t ntt_kmin(int64_t p, int bits) {
  const int64_t lo = 32 * p - 63;  // c_k reaches limb p when bits k > 32 p - 64
  return lo <= 0 ? 0 : (lo + bits - 1) / bits;
}

struct NttCarrySrc {
  static constexpr bool kWide = false;
  const uint64_t* S;  // LDS: coefficients k0 .. of the chunk's limbs
  int64_t k0;
  int64_t ncoef;
  int bits;
  uint32_t* out;
  int64_t nstore;
  // bits [32 p, 32 p + 32) of the coefficients k in [kmin, kmax]; every index
  // is below 2^31 (N <= 2^24 coefficients, under 2^26 limbs)
  TC_DEV int64_t sum(int p, int kmin, int kmax) const {
    int64_t d = 0;
    for (int k = kmin; k <= kmax; k++) {
      const uint64_t v = S[k - (int)k0];
      const int s = bits * k - 32 * p;  // -64 < s < 32
      d += (int64_t)(uint32_t)(s >= 0 ? (v << s) : (v >> (-s)));
    }
    return d;
  }
  TC_DEV int64_t delta(int64_t p) const {
    int kmax = (int)((32 * p + 31) / bits);
    if (kmax > ncoef - 1) kmax = (int)ncoef - 1;
    return sum((int)p, (int)ntt_kmin(p, bits), kmax);
  }
  // The lane's limbs pt-1 .. pt+LPT-1 in order: the coefficient bounds move
  // by at most two per limb, so they advance by comparison rather than by
  // dividing again.
  template <int LPT>
  TC_DEV void deltas(int64_t pt, int nown, int64_t* dd) const {
    const int first = pt > 0 ? (int)pt - 1 : (int)pt;
    int kmin = (int)ntt_kmin(first, bits);
    int kend = (int)((32 * (int64_t)first + 31) / bits);  // unclamped kmax
    const int klast = (int)ncoef - 1;
#pragma unroll
    for (int j = 0; j <= LPT; j++) {
      const int p = (int)pt - 1 + j;
      if (p < first || j > nown) continue;
      if (p > first) {
        while (bits * kmin <= 32 * p - 64) kmin++;
        while (bits * (kend + 1) <= 32 * p + 31) kend++;
      }
      dd[j] = sum(p, kmin, kend < klast ? kend : klast);
    }
  }
  TC_DEV bool store(int64_t p, uint32_t o, uint32_t& err) {
    if (p < nstore) gst(out + p, o);
    else if (o != 0u) err |= ERRBIT_RANGE;
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

// Coefficients one wave stages: limbs [p0 - 1, p0 + 64 LPT) meet at most
// (32 (64 LPT) + 62) / bits + 2 of them, 1029 for LPT = 8 and bits >= 16.
constexpr int kCarryStage = 1040;

// One wavefront per chunk of a leaf's product; chunks are handed out by a
// per-leaf ticket, so every chunk a wave waits on is already running.  The
// wave first copies the coefficients its limbs meet into LDS with coalesced
// loads; the limb sums then read them from there.
template <int LPT>
__global__ __launch_bounds__(256) void k_ntt_carry(const NttDesc* __restrict__ descs,
                                                   const int64_t* __restrict__ wave0, int nd,
                                                   int64_t total, const Bases* __restrict__ bp,
                                                   uint64_t* status) {
  const Bases bases = *bp;
  const int64_t gw = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  if (gw >= total) return;
  const int di = find_unit(wave0, nd, gw);
  const NttDesc& D = descs[di];
  const int64_t nch = D.nchunks;
  const int64_t leaf = (gw - wave0[di]) / nch;
  int64_t chunk = 0;
  uint64_t* st = nullptr;
  if (nch > 1) {
    st = status + D.status_off + leaf * lb_words(nch);
    unsigned long long t = 0;
    if (lane_id() == 0) t = atomicAdd(reinterpret_cast<unsigned long long*>(&st[lb_ticket(nch)]), 1ull);
    chunk = (int64_t)readlane((uint32_t)t, 0);
    if (chunk >= nch) {
      flag_error(item_err(bases, D.item), ERRBIT_HANG);
      return;
    }
  }
  static_assert(LPT <= 8, "the staging buffer holds the coefficients of 512 limbs");
  __shared__ uint64_t stage[4][kCarryStage];
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int64_t N = (int64_t)1 << (D.logR + D.logC);
  const uint64_t* base = reinterpret_cast<const uint64_t*>(resolve(bases, D.X));
  const uint64_t* coef = base + (D.square ? leaf : D.count + leaf) * N;
  const int64_t p0 = chunk * 64 * LPT;
  const int64_t k0 = ntt_kmin(p0 > 0 ? p0 - 1 : 0, D.bits);
  int64_t k1 = (32 * (p0 + 64 * LPT - 1) + 31) / D.bits;
  if (k1 > D.ncoef - 1) k1 = D.ncoef - 1;
  const int64_t cnt = k1 >= k0 ? k1 - k0 + 1 : 0;
  if (cnt > kCarryStage) {
    flag_error(item_err(bases, D.item), ERRBIT_RANGE);
    return;
  }
  for (int64_t j = lane_id(); j < cnt; j += 64) stage[wv][j] = coef[k0 + j];
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  NttCarrySrc s;
  s.S = stage[wv];
  s.k0 = k0;
  s.ncoef = D.ncoef;
  s.bits = D.bits;
  s.out = reinterpret_cast<uint32_t*>(resolve(bases, D.P)) + leaf * D.p_stride;
  s.nstore = D.p_width;
  EngCfg cfg;
  cfg.Y = D.ncompute;
  cfg.div[0] = cfg.div[1] = nullptr;
  cfg.shr = 0;
  cfg.is_signed = false;
  cfg.prenorm = true;
  cfg.check_carry = true;
  uint32_t eb = 0;
  (void)engine_chunk<LPT>(s, cfg, chunk, nch, st, eb);
  flag_error(item_err(bases, D.item), eb);
}

hipError_t launch_ntt(int which, const NttDesc* d, const int64_t* u0, int nd, int64_t units,
                      int lpt, size_t lds, const Bases* b, const uint64_t* roots,
                      uint64_t* status, hipStream_t st) {
  if (units <= 0) return hipSuccess;
  const dim3 blk(256), tblk(kNttThreads);
  switch (which) {
    case kNttColFwd:
      hipLaunchKernelGGL(k_ntt_cols<false>, dim3((unsigned)units), tblk, lds, st, d, u0, nd, b, roots);
      break;
    case kNttRowFwd:
      hipLaunchKernelGGL(k_ntt_rows<0>, dim3((unsigned)units), tblk, lds, st, d, u0, nd, b, roots);
      break;
    case kNttRowMul:
      hipLaunchKernelGGL(k_ntt_rows<1>, dim3((unsigned)units), tblk, lds, st, d, u0, nd, b, roots);
      break;
    case kNttColInv:
      hipLaunchKernelGGL(k_ntt_cols<true>, dim3((unsigned)units), tblk, lds, st, d, u0, nd, b, roots);
      break;
    default: {
      const dim3 g((unsigned)((units + 3) / 4));
      switch (lpt) {
        case 2: hipLaunchKernelGGL(k_ntt_carry<2>, g, blk, 0, st, d, u0, nd, units, b, status); break;
        case 4: hipLaunchKernelGGL(k_ntt_carry<4>, g, blk, 0, st, d, u0, nd, units, b, status); break;
        case 8: hipLaunchKernelGGL(k_ntt_carry<8>, g, blk, 0, st, d, u0, nd, units, b, status); break;
        default: return hipErrorInvalidValue;  // the staging holds at most 512 limbs' coefficients
      }
    }
  }
  return hipGetLastError();
}

}  // namespace tc

// ------------------------------------------------ throughput of the multiplier

namespace tc {
namespace {

// Eight independent chains of x = lo32(x) c + hi32(x) per lane: one 32 x 32 +
// 32 -> 64 multiply-add each (v_mad_u64_u32), the operation the transform's
// field products and the vector-ALU leaves are built from.
__global__ __launch_bounds__(256) void k_mad_rate(uint64_t* out, uint32_t c, int iters) {
  uint64_t x[8];
#pragma unroll
  for (int j = 0; j < 8; j++) x[j] = threadIdx.x + 977u * (uint32_t)j + blockIdx.x;
  for (int it = 0; it < iters; it++) {
#pragma unroll
    for (int j = 0; j < 8; j++) x[j] = (uint64_t)(uint32_t)x[j] * c + (x[j] >> 32);
  }
  uint64_t s = 0;
#pragma unroll
  for (int j = 0; j < 8; j++) s ^= x[j];
  out[(size_t)blockIdx.x * 256 + threadIdx.x] = s;
}

}  // namespace

hipError_t measure_mad_rate(double* per_s) {
  const int blocks = 4096, iters = 4096;
  uint64_t* d = nullptr;
  hipEvent_t a = nullptr, b = nullptr;
  hipError_t e = hipMalloc(&d, (size_t)blocks * 256 * sizeof(uint64_t));
  if (e == hipSuccess) e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&b);
  float best = 0.f;
  for (int rep = 0; rep < 3 && e == hipSuccess; rep++) {
    (void)hipEventRecord(a, nullptr);
    hipLaunchKernelGGL(k_mad_rate, dim3(blocks), dim3(256), 0, nullptr, d, 0x9E3779B9u, iters);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipEventRecord(b, nullptr);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
    if (e == hipSuccess && (rep == 0 || ms < best)) best = ms;
  }
  if (e == hipSuccess) *per_s = (double)blocks * 256 * iters * 8 / (best * 1e-3);
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  if (d) (void)hipFree(d);
  return e;
}

}  // namespace tc
