// tc_types.hpp -- descriptors shared by the host planner and the HIP kernels.
//
// Every device address in a descriptor is a (buffer, byte offset) pair that a
// kernel resolves against the Bases it is launched with, so a compiled plan
// can be replayed with new operand, result and scratch addresses.
#pragma once
#include <stdint.h>

#ifndef TC_HD
#define TC_HD __host__ __device__ __forceinline__
#endif

namespace tc {

constexpr int kMaxB = 32;              // largest split
constexpr int kMaxPts = 2 * kMaxB - 1; // evaluation points
constexpr int kPowMax = 1024;          // powers of 2^-32 kept per divisor
constexpr int kMaxDivs = 512;          // divisor table capacity (filled on demand)

// Buffer ids of DPtr.buf
enum : int32_t { BUF_SCRATCH = 0, BUF_U = 1, BUF_V = 2, BUF_W = 3, BUF_TABLE0 = 4 };

struct DPtr {
  int64_t off;  // bytes
  int32_t buf;
  int32_t pad;
};

struct Bases {
  uint8_t* scratch;
  uint8_t* p[3];               // u, v, w of a single product
  uint8_t* const* table;       // per-item pointers of a batch (buf >= BUF_TABLE0)
  uint32_t* err;               // error words: item i's at err[i * err_stride]
  int64_t err_stride;          // 0: one word for every item (the device's sticky word)
};

// Selects rather than an indexed array read, so a kernel's copy of Bases
// stays in registers.
TC_HD uint8_t* resolve(const Bases& b, DPtr d) {
  uint8_t* base = d.buf == BUF_SCRATCH ? b.scratch
                  : d.buf == BUF_U     ? b.p[0]
                  : d.buf == BUF_V     ? b.p[1]
                  : d.buf == BUF_W     ? b.p[2]
                                       : b.table[d.buf - BUF_TABLE0];
  return base + d.off;
}

// Chunk widths T = 64 LPT of the carry engine (LPT = 2, 4, 8, 16).
constexpr int kChunkKinds = 4;
constexpr int kWindow = 64;  // look-back words examined at once

// Precomputed constants of an odd divisor d > 1: its inverse mod 2^32, the
// powers M^j mod d of M = 2^-32 mod d with Shoup companions floor(M^j 2^32 / d),
// and, per chunk width T, the chunk weights M^(T l) for l = 0..64 (with
// companions) that combine up to 64 chunk residues at once.
struct DivEntry {
  uint32_t d;
  uint32_t dinv;
  uint32_t pw[kPowMax + 1];
  uint32_t pws[kPowMax + 1];
  uint32_t cw[kChunkKinds][kWindow + 1];
  uint32_t cws[kChunkKinds][kWindow + 1];
};

constexpr int chunk_kind(int lpt) { return lpt <= 2 ? 0 : lpt <= 4 ? 1 : lpt <= 8 ? 2 : 3; }

// ---------------------------------------------------------------------------
// Linear step: out = (sum_i s_i m_i (T_i << sh_i)) / (2^shr * d1 * d2),
// exact, in Y-limb two's complement, for up to kStepTerms terms with signs
// s_i and odd multipliers m_i.  One descriptor covers `count` nodes.
// ---------------------------------------------------------------------------
enum : int8_t { TERM_NONE = 0, TERM_TC = 1, TERM_SM = 2 };

struct TermDesc {
  DPtr ptr;         // node 0's value
  int64_t stride;   // limbs between nodes
  DPtr su, sv;      // TERM_SM: sign of node i is su[i*sstride] ^ sv[i*svstride]
  int64_t sstride;  // (sv.buf < 0: su alone)
  int32_t svstride;
  int32_t width;    // stored limbs (TC: sign-extends past it; SM: zero past it)
  int32_t shl;      // left shift in bits
  int8_t kind;
  int8_t neg;       // multiply by -1
  int16_t sidx;     // TERM_SM: index of the point product (its sign byte), else -1
  uint32_t mul;     // odd multiplier (0 or 1: none)
};
// kernels read kind and neg together as one aligned dword
static_assert(__builtin_offsetof(TermDesc, kind) % 4 == 0 && sizeof(TermDesc) % 4 == 0,
              "TermDesc: kind must start an aligned dword");

// A step term as the kernel's prologue reads it (32 bytes, one scalar load):
// limb p of the term is bits of (v[p-k] : v[p-k-1]) >> sh of its value v,
// times mul, negated per bit 0 of f (and by the product's sign).
struct TermC {
  int64_t off;     // bytes: node 0's value in its buffer
  int64_t stride;  // limbs between nodes
  int32_t width;   // stored limbs
  uint32_t f;      // bit 0 negative, bits 3..7 sh, bits 8..31 k + 1
  uint32_t mul;    // odd multiplier, 1 = none
  int8_t buf;      // BUF_SCRATCH, BUF_U, BUF_V or BUF_W
  int8_t tc;       // two's complement: ones past the width when negative
  int16_t sidx;    // product index of the sign byte, -1: none
};
static_assert(sizeof(TermC) == 32, "TermC is one 32-byte scalar load");

// A linear step combines at most this many terms (merged Newton-to-monomial
// rounds, section 3, take up to five).
constexpr int kStepTerms = 8;

// Chunked values: a value of more than one chunk keeps lb_words(nchunks)
// look-back words at status_off + node * lb_words(nchunks) of the status
// region: per chunk a word of the carry and first division, per chunk a word
// of the second division, then a ticket counter and the evaluation's
// lowest-nonzero limb marker.
TC_HD int64_t lb_words(int64_t nch) { return 2 * nch + 2; }
TC_HD int64_t lb_ticket(int64_t nch) { return 2 * nch; }
TC_HD int64_t lb_marker(int64_t nch) { return 2 * nch + 1; }
struct StepDesc {
  DPtr out;
  int64_t out_stride;
  int64_t count;
  int64_t status_off;
  int32_t nchunks;
  int32_t item;     // product of a batch the descriptor belongs to (its error word)
  int32_t Y;        // output width in limbs
  int32_t shr;      // exact right shift in bits
  int32_t div[2];   // divisor table ids or -1
  int32_t nterms;
  int32_t fast;     // c[] and the sign fields below are valid (see fill_fast)
  TermDesc t[kStepTerms];
  // The terms precomputed for the kernel's straight-line prologue: buffers
  // U, V, W or scratch only; the signs of product terms are bytes
  // sgn_u[node * sgn_stride + sidx] xor sgn_v[node * sgn_v_stride + sidx]
  // (sgn_v_buf < 0: no v).
  TermC c[kStepTerms];
  int64_t sgn_u_off, sgn_v_off, sgn_stride;
  int32_t sgn_u_buf, sgn_v_buf;
  int32_t nsgn;     // sign bytes per node read (largest sidx + 1)
  int32_t sgn_v_stride;
};
static_assert(__builtin_offsetof(StepDesc, t) % 4 == 0, "StepDesc: terms dword-aligned");

// ---------------------------------------------------------------------------
// Recomposing step: a Toom level whose interpolation is one round (every
// coefficient w_k = (sum_i a_ki y_i) / D_k is an exact combination of the
// point products) forms the node's product directly.  With L a common
// multiple of the D_k, L W = sum_k (L / D_k) (sum_i a_ki y_i) beta^(k bl):
// one linear pass over the shifted point products (a term per pair (k, i),
// its shift k bl limbs plus the power of two of its weight), then one exact
// division by L = 2^shr d1 d2.  A term whose shifted limbs miss a wave's
// limbs is skipped.  Limbs [nstore, Y) of the result must be zero.
// ---------------------------------------------------------------------------
constexpr int kRTerms = 32;
struct RStepDesc {
  DPtr out;
  int64_t out_stride;
  int64_t count;
  int64_t status_off;
  int32_t nchunks;
  int32_t item;
  int32_t Y;        // limbs computed
  int32_t nstore;   // limbs of the node's product stored
  int32_t shr;
  int32_t div[2];
  int32_t nterms;
  // product signs: sgn_u[node * sgn_stride + sidx] ^ sgn_v[node * sgn_v_stride + sidx]
  int64_t sgn_u_off, sgn_v_off, sgn_stride;
  int32_t sgn_u_buf, sgn_v_buf;  // sgn_v_buf < 0: none
  int32_t nsgn;
  int32_t sgn_v_stride;
  TermC c[kRTerms];
};

// ---------------------------------------------------------------------------
// Evaluation: one point value of one operand of `count` parent nodes.
// value = sum_t s_t * (block_t << (t*j)) with s_t = +1 for even t and
// (odd_neg ? -1 : +1) for odd t (rev: block_t << ((B-1-t)*j), the value at
// 2^-j times 2^((B-1)j)); or a copy of block `copy_block`.
// The magnitude goes to out (nout limbs), the sign to sign[].
// ---------------------------------------------------------------------------
struct EvalDesc {
  int64_t status_off;
  int32_t nchunks;
  int32_t item;     // product of a batch the descriptor belongs to (its error word)
  DPtr src;
  int64_t src_stride;  // limbs between parent nodes
  int64_t src_width;   // limbs of a parent that exist (past it: zero)
  int64_t bl;
  DPtr out;
  int64_t out_stride;
  DPtr sign;           // uint8 per child
  int64_t sign_stride;
  int64_t count;
  int32_t nout;
  int32_t B;
  int32_t j;
  int32_t odd_neg;
  int32_t copy_block;  // >= 0: copy that block
  int32_t paired;      // 1: also the value at -2^j (odd blocks negated), below
  int32_t rev;         // 1: block t shifted by (B-1-t) j (homogeneous value at 2^-j)
  int32_t pad1;
  DPtr out2;           // paired: its values, signs and look-back words
  DPtr sign2;
  int64_t status_off2;
};

// ---------------------------------------------------------------------------
// Recomposition: out = sum_k w_k * 2^(32*bl*k), k < nk; w_k read in wread limbs.
// Limbs [nstore, ncompute) must be zero, and so must limbs [wread, wlimbs) of
// every w_k (a coefficient is non-negative and fits wread limbs).
// ---------------------------------------------------------------------------
struct RecompDesc {
  int64_t status_off;
  int32_t nchunks;
  int32_t item;     // product of a batch the descriptor belongs to (its error word)
  DPtr w[kMaxPts];
  int64_t w_stride;
  int64_t bl;
  DPtr out;
  int64_t out_stride;
  int64_t count;
  int64_t ncompute;
  int64_t nstore;
  int32_t nk;
  int32_t wread;
  int32_t wlimbs;   // limbs each w_k holds; limbs [wread, wlimbs) must be zero
  int32_t pad;
};

// ---------------------------------------------------------------------------
// Schoolbook leaves: P[i] (2n limbs) = U[i] * V[i] (n limbs each).
// ---------------------------------------------------------------------------
struct LeafDesc {
  DPtr U, V, P;
  int64_t u_stride, v_stride, p_stride;
  int64_t count;
  int32_t n;        // leaf width (operands zero-extended to it)
  int32_t u_width;  // limbs of U that exist
  int32_t v_width;
  int32_t p_width;  // limbs of P written; the rest of 2n must be zero
  int32_t item;     // product of a batch the descriptor belongs to (its error word)
  int32_t pad;
};

// ---------------------------------------------------------------------------
// Leaves formed by a number-theoretic transform (section 5's FFT product
// under a Toom-Cook level): P[i] = U[i] * V[i] through pieces of `bits` bits,
// the transform of length N = R C over p = 2^64 - 2^32 + 1 (four steps:
// R-point column transforms, twiddles w_N^(c jr), C-point row transforms),
// the pointwise product, the inverse, and a carry pass.
// ---------------------------------------------------------------------------
constexpr int kNttLogRowMax = 13;  // C <= 8192: a row fills 64 KiB of LDS
constexpr int kNttLogColMax = 11;  // R <= 2048
constexpr int kNttTileElems = 8192;  // column tiles: R x (8192 / R) elements
// root table layout (u64 entries): w_8192^k and w_8192^-k for k < 4096, then
// w_2^24^i, w_2^24^(4096 i) and their inverses for i < 4096; then the twiddles
// of each in-LDS stage stored contiguously, so the threads of a stage read
// consecutive entries: for the radix-4 stage pair with half-blocks h = 2^lo
// (lo = 0..11), at kNttTw4 + 3 (h - 1), w_4h^i, then w_4h^(i+h), then w_2h^i
// for i < h; for a radix-2 stage with half-blocks h = 2^lh (lh = 0..12), at
// kNttTw2 + h - 1, w_2h^i for i < h (forward roots, then the inverse ones).
constexpr int kNttRootFwd = 0, kNttRootInv = 4096, kNttLo = 8192, kNttHi = 12288,
              kNttLoInv = 16384, kNttHiInv = 20480;
constexpr int kNttTw4Len = 3 * 4095, kNttTw2Len = 8191;
constexpr int kNttTw4Fwd = 24576, kNttTw4Inv = kNttTw4Fwd + kNttTw4Len,
              kNttTw2Fwd = kNttTw4Inv + kNttTw4Len, kNttTw2Inv = kNttTw2Fwd + kNttTw2Len,
              kNttRootEntries = kNttTw2Inv + kNttTw2Len;

struct NttDesc {
  DPtr U, V, P;       // limb operands of leaf 0 and its product
  int64_t u_stride, v_stride, p_stride;  // limbs between leaves
  int64_t count;      // leaves
  DPtr X;             // transforms: count arrays for U, then count for V (N u64 each)
  int32_t u_width, v_width, p_width;
  int32_t bits;       // piece width
  int32_t logR, logC; // N = 2^(logR + logC); logR = 0: rows only
  int32_t square;     // V is U: one transform per leaf, in the U arrays
  int32_t item;
  uint64_t ninv;      // N^-1 mod p
  int64_t ncoef;      // convolution coefficients (pieces of U + pieces of V - 1)
  int64_t ncompute;   // limbs the carry pass forms (>= p_width; the rest must be 0)
  int32_t nchunks;    // carry pass: chunks of 64 LPT limbs
  int32_t pad;
  int64_t status_off; // carry pass look-back words
};

// Device error bits (sticky).
enum : uint32_t {
  ERRBIT_DIV = 1u,      // exact division had a remainder
  ERRBIT_SHIFT = 2u,    // exact right shift dropped set bits
  ERRBIT_RANGE = 4u,    // a value did not fit its width
  ERRBIT_SIGN = 8u,     // a coefficient that must be >= 0 was negative
  ERRBIT_HANG = 16u     // a look-back wait gave up (bounded spin)
};

}  // namespace tc
