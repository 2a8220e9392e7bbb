/*
 * toomref.h -- CPU oracle for B-way Toom-Cook multiplication of unsigned
 * integers held as 32-bit limbs (M.J. Kronenburg, "Toom-Cook Multiplication:
 * Some Theoretical and Practical Aspects", arXiv:1602.02740).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the checker: it is plain, slow
 * and written to be compared with the paper by eye.  Only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg load it.  The GPU library
 * shares no source, header, table or helper with it; the two agree only on
 * the data conventions written below.
 *
 * Conventions (shared by agreement, not by code):
 *  - An integer is a little-endian array of uint32_t limbs, limb 0 least
 *    significant.  Lengths are in limbs.
 *  - A node of nominal width n limbs is split into B blocks of
 *    bl = ceil(n / B) limbs (section 1: u = U(2^b) with b = 32*bl); block t
 *    holds limbs [t*bl, (t+1)*bl) and is zero where that range passes n.
 *  - Evaluation points, even-odd variant (section 6 point set used as +/-
 *    pairs, section 4): index 0 is x = 0, index 2j+1 is x = +2^j and index
 *    2j+2 is x = -2^j, for j = 0 .. B-2.  That is 2B-1 points.
 *  - Infinity variant (B = 3 only; not in the paper): points
 *    [0, +1, -1, +2, inf] with U(inf) = the top block.
 *  - Plain variant (test baseline, section 4 "without the even-odd method"):
 *    same points as the even-odd variant, interpolated as one polynomial of
 *    degree 2n with the Newton loops of section 3.
 *  - Half variant (B = 4 only; not in the paper's experiments): points
 *    [0, +1, -1, +2, -2, 1/2, inf].  The value at 1/2 is homogeneous,
 *    2^(B-1) U(1/2) = sum_t u_t 2^(B-1-t), so a point product there is
 *    2^(2B-2) W(1/2); U(inf) is the top block.  The coefficients are
 *    recovered as c = V^-1 y with V the 7 x 7 matrix of these point rows,
 *    section 3's closing remark on a fixed n, the inverse taken exactly in
 *    rationals.
 *  - Odd-direct variant (the other reading of section 4's handling of the
 *    odd polynomial): same points and even polynomial as the even-odd
 *    variant; W_o is interpolated directly with degree n-1 at X = 4^j,
 *    j = 0 .. n-1, instead of X W_o(X) with degree n at X = 0, 4^j.
 *  - A child node has width n' = bl + g(B), where g is the evaluation growth
 *    in limbs (tcref_growth_limbs).  A node's product has width 2n.
 *  - Signed values crossing the API are sign-magnitude: a magnitude array plus
 *    an int8 sign (0 = non-negative, 1 = negative; zero is always 0).
 *  - The interpolated coefficients w_k (k = 0 .. 2B-2) are non-negative and
 *    are written in nw limbs each (2*bl + 1 suffices).
 *  - Interpolation width: with point products of ny limbs, every intermediate
 *    of the Newton loops must fit a signed two's-complement value of ny + 2
 *    limbs (inside tcref_mul_toom, ny = 2n'); the oracle checks this.
 *
 * Every function returns TCREF_OK or a negative TCREF_ERR_* code.  An
 * exactness failure (a division with a remainder, an odd value before a
 * halving, a negative coefficient, a value that does not fit its width) is
 * reported, never rounded away.
 */
#ifndef TOOMREF_H
#define TOOMREF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TCREF_MAX_LEVELS 16

enum {
  TCREF_OK = 0,
  TCREF_ERR_ARG = -1,     /* bad argument (null pointer, unsupported B, ...) */
  TCREF_ERR_INEXACT = -2, /* a division or halving that must be exact was not */
  TCREF_ERR_RANGE = -3,   /* a value does not fit the width it must fit */
  TCREF_ERR_NOMEM = -4
};

enum {
  TCREF_VAR_EVENODD = 0, /* the paper's method: points 0, +/-2^j; even-odd Newton */
  TCREF_VAR_INF = 1,     /* B = 3 with points 0, 1, -1, 2, inf */
  TCREF_VAR_PLAIN = 2,   /* points 0, +/-2^j; one Newton interpolation of degree 2n */
  TCREF_VAR_ODD_DIRECT = 3, /* as EVENODD, but W_o itself (degree n-1) is
                              interpolated at the n non-zero nodes X = 4^j from
                              W_o(4^j) = (W(2^j) - W(-2^j)) / 2^(j+1) */
  TCREF_VAR_HALF = 4     /* B = 4 with points 0, 1, -1, 2, -2, 1/2, inf,
                            interpolated by the fixed-n matrix inverse */
};

/* A multiplication plan: `levels` Toom levels, then schoolbook leaves. */
typedef struct {
  int levels;
  int B[TCREF_MAX_LEVELS];       /* 2 .. 32 */
  int variant[TCREF_MAX_LEVELS]; /* TCREF_VAR_* */
  int threads;                   /* threads for the top-level products (section 2,
                                    P <= 2B-1); 0 or 1 runs serially */
  int leaf_ntt_bits;             /* 0: schoolbook leaves; else leaves formed by
                                    tcref_mul_ntt with pieces of this many bits
                                    (section 5: Toom-Cook over an FFT product) */
} tcref_plan;

/* Nominal operation counts (see tcref_counts_get). */
typedef struct {
  uint64_t leaves;        /* schoolbook leaf products */
  uint64_t leaf_mults;    /* sum over leaves of (leaf width)^2 */
  uint64_t toom_nodes;    /* Toom nodes (interpolations) */
  uint64_t eval_limbs;    /* limbs written by evaluations */
  uint64_t interp_steps;  /* Newton steps (both loops of section 3) */
  uint64_t interp_limbs;  /* sum over Newton steps of the value width */
  uint64_t recomp_limbs;  /* limbs written by recompositions */
} tcref_counts;

/* Evaluation growth g(B) in limbs for a variant (child width = bl + g). */
size_t tcref_growth_limbs(int B, int variant);
/* Block width bl = ceil(n / B). */
size_t tcref_block_limbs(size_t n, int B);

/* w (nu+nv limbs) = u * v by schoolbook column products. */
int tcref_mul_school(uint32_t *w, const uint32_t *u, size_t nu,
                     const uint32_t *v, size_t nv);

/* w (nu+nv limbs) = u * v by recursive Toom-Cook following `plan`, with
 * nominal top width max(nu, nv). */
int tcref_mul_toom(uint32_t *w, const uint32_t *u, size_t nu,
                   const uint32_t *v, size_t nv, const tcref_plan *plan);

/* Evaluation of one operand (u, nu limbs) split into B blocks of bl limbs at
 * the 2B-1 points of `variant`.  out: (2B-1) x nout magnitudes; sign: 2B-1. */
int tcref_eval(int B, int variant, const uint32_t *u, size_t nu, size_t bl,
               size_t nout, uint32_t *out, int8_t *sign);

/* Interpolation: from the 2B-1 signed point products y (ny limbs each) to the
 * coefficients w_0 .. w_{2B-2} (nw limbs each). */
int tcref_interp(int B, int variant, size_t ny, const uint32_t *y,
                 const int8_t *sign, size_t nw, uint32_t *w);

/* Recomposition: out (nout limbs) = sum_k w_k * 2^(32*bl*k). */
int tcref_recompose(int B, size_t bl, size_t nw, const uint32_t *w,
                    size_t nout, uint32_t *out);

/* Newton interpolation of section 3 on arbitrary distinct int64 nodes x[0..n]
 * and signed values y (nl limbs each).  phase 1 leaves the divided
 * differences alpha_k; phase 2 also runs the Newton-to-monomial loop and
 * leaves the monomial coefficients c_0 .. c_n.  Every division must be exact. */
int tcref_newton(int n, const int64_t *x, size_t nl, const uint32_t *ymag,
                 const int8_t *ysign, uint32_t *cmag, int8_t *csign, int phase);

/* Number-theoretic transform over p = 2^64 - 2^32 + 1 (nttref.c), the
 * exact FFT product that section 5 puts under a Toom-Cook top level.
 * tcref_ntt_root: w_N = 7^((p-1)/N) for a power of two N <= 2^32 (0 if not).
 * tcref_ntt: in place, X[j] = sum_i x[i] w_N^(i j); inverse != 0 gives
 * x[i] = N^-1 sum_j X[j] w_N^(-i j).  Entries must be below p.
 * tcref_ntt_pieces: out[i] = floor(u / 2^(bits i)) mod 2^bits, i < nout.
 * tcref_mul_ntt: w (nu+nv limbs) = u v through pieces of `bits` bits, the
 * transform of the smallest power-of-two length that holds the acyclic
 * convolution, the pointwise product and the inverse; TCREF_ERR_RANGE when
 * a coefficient could reach p ((2^bits-1)^2 min(pieces) >= p). */
uint64_t tcref_ntt_root(uint64_t N);
int tcref_ntt(uint64_t *x, size_t N, int inverse);
size_t tcref_ntt_npieces(size_t n, int bits);
int tcref_ntt_pieces(const uint32_t *u, size_t nu, int bits, uint64_t *out, size_t nout);
int tcref_mul_ntt(uint32_t *w, const uint32_t *u, size_t nu, const uint32_t *v, size_t nv,
                  int bits);

/* Operation counters, summed over all calls since the last reset. */
void tcref_counts_reset(void);
void tcref_counts_get(tcref_counts *out);
/* The same counts for one tcref_mul_toom of nominal width n, computed from
 * the plan's sizes alone (no arithmetic). */
int tcref_plan_counts(size_t n, const tcref_plan *plan, tcref_counts *out);

#ifdef __cplusplus
}
#endif
#endif /* TOOMREF_H */
