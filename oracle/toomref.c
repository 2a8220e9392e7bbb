/*
 * toomref.c -- CPU oracle for B-way Toom-Cook multiplication.
 *
 * TEST INFRASTRUCTURE ONLY (see toomref.h).  Written for checking by eye
 * against M.J. Kronenburg, "Toom-Cook Multiplication: Some Theoretical and
 * Practical Aspects" (arXiv:1602.02740):
 *   section 1  integers as polynomials u = U(2^b), w = W(2^b) = uv;
 *   section 2  recursion T(N) = (2B-1) T(N/B) and the top-level products on
 *              P <= 2B-1 processors;
 *   section 3  Newton interpolation: the divided-difference loop (Theorem 3.2)
 *              and the Newton-to-monomial loop (Theorem 3.3);
 *   section 4  the even-odd method, W(x) = W_e(x^2) + x W_o(x^2);
 *   section 6  points 0, 1, 2, 4, ..., 2^(n-1) (used here as +/- pairs), all
 *              divisions exact.
 *
 * The arithmetic is a small sign-magnitude bignum of our own.  Nothing here is
 * blocked, fused or reordered beyond what the paper states.  Exact divisions
 * are done top-down by long division with a 128-bit remainder and the
 * remainder is checked to be zero.
 */
#include "toomref.h"

#include <pthread.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------- */
/* Sticky error per thread                                                    */
/* ------------------------------------------------------------------------- */

static __thread int t_err = TCREF_OK;

static void set_err(int e) {
  if (t_err == TCREF_OK) t_err = e;
}

/* ------------------------------------------------------------------------- */
/* Counters                                                                   */
/* ------------------------------------------------------------------------- */

static tcref_counts g_counts;

static void count_add(uint64_t *field, uint64_t v) {
  __atomic_fetch_add(field, v, __ATOMIC_RELAXED);
}

void tcref_counts_reset(void) { memset(&g_counts, 0, sizeof g_counts); }

void tcref_counts_get(tcref_counts *out) {
  out->leaves = __atomic_load_n(&g_counts.leaves, __ATOMIC_RELAXED);
  out->leaf_mults = __atomic_load_n(&g_counts.leaf_mults, __ATOMIC_RELAXED);
  out->toom_nodes = __atomic_load_n(&g_counts.toom_nodes, __ATOMIC_RELAXED);
  out->eval_limbs = __atomic_load_n(&g_counts.eval_limbs, __ATOMIC_RELAXED);
  out->interp_steps = __atomic_load_n(&g_counts.interp_steps, __ATOMIC_RELAXED);
  out->interp_limbs = __atomic_load_n(&g_counts.interp_limbs, __ATOMIC_RELAXED);
  out->recomp_limbs = __atomic_load_n(&g_counts.recomp_limbs, __ATOMIC_RELAXED);
}

/* ------------------------------------------------------------------------- */
/* Sign-magnitude bignum                                                      */
/* ------------------------------------------------------------------------- */

typedef struct {
  int neg;     /* 1 if negative; never set for zero */
  size_t len;  /* limbs in use; d[len-1] != 0 unless len == 0 */
  size_t cap;
  uint32_t *d;
} bn;

static void bn_init(bn *a) {
  a->neg = 0;
  a->len = 0;
  a->cap = 0;
  a->d = NULL;
}

static void bn_free(bn *a) {
  free(a->d);
  bn_init(a);
}

static void bn_reserve(bn *a, size_t cap) {
  if (cap > a->cap) {
    uint32_t *p = (uint32_t *)realloc(a->d, (cap ? cap : 1) * sizeof(uint32_t));
    if (!p) abort();
    a->d = p;
    a->cap = cap;
  }
}

static void bn_trim(bn *a) {
  while (a->len > 0 && a->d[a->len - 1] == 0) a->len--;
  if (a->len == 0) a->neg = 0;
}

static void bn_zero(bn *a) {
  a->len = 0;
  a->neg = 0;
}

static void bn_move(bn *dst, bn *src) {
  bn_free(dst);
  *dst = *src;
  bn_init(src);
}

static void bn_copy(bn *r, const bn *a) {
  if (r == a) return;
  bn_reserve(r, a->len);
  if (a->len) memcpy(r->d, a->d, a->len * sizeof(uint32_t));
  r->len = a->len;
  r->neg = a->neg;
}

/* r = magnitude p[0..n) (non-negative). */
static void bn_set_limbs(bn *r, const uint32_t *p, size_t n) {
  bn_reserve(r, n);
  if (n) memcpy(r->d, p, n * sizeof(uint32_t));
  r->len = n;
  r->neg = 0;
  bn_trim(r);
}

/* Write |a| into out[0..n); error if it does not fit. */
static void bn_get_limbs(const bn *a, uint32_t *out, size_t n) {
  if (a->len > n) {
    set_err(TCREF_ERR_RANGE);
    return;
  }
  if (a->len) memcpy(out, a->d, a->len * sizeof(uint32_t));
  if (n > a->len) memset(out + a->len, 0, (n - a->len) * sizeof(uint32_t));
}

static int mag_cmp(const bn *a, const bn *b) {
  if (a->len != b->len) return a->len < b->len ? -1 : 1;
  for (size_t i = a->len; i-- > 0;) {
    if (a->d[i] != b->d[i]) return a->d[i] < b->d[i] ? -1 : 1;
  }
  return 0;
}

/* r = |a| + |b| (new storage, r may alias a or b through the caller). */
static void mag_add(bn *r, const bn *a, const bn *b) {
  const bn *x = a->len >= b->len ? a : b;
  const bn *y = a->len >= b->len ? b : a;
  bn t;
  bn_init(&t);
  bn_reserve(&t, x->len + 1);
  uint64_t carry = 0;
  for (size_t i = 0; i < x->len; i++) {
    uint64_t s = (uint64_t)x->d[i] + (i < y->len ? y->d[i] : 0) + carry;
    t.d[i] = (uint32_t)s;
    carry = s >> 32;
  }
  t.d[x->len] = (uint32_t)carry;
  t.len = x->len + 1;
  bn_trim(&t);
  bn_move(r, &t);
}

/* r = |a| - |b| where |a| >= |b|. */
static void mag_sub(bn *r, const bn *a, const bn *b) {
  bn t;
  bn_init(&t);
  bn_reserve(&t, a->len);
  int64_t borrow = 0;
  for (size_t i = 0; i < a->len; i++) {
    int64_t s = (int64_t)a->d[i] - (int64_t)(i < b->len ? b->d[i] : 0) - borrow;
    borrow = s < 0;
    t.d[i] = (uint32_t)(s + (borrow ? ((int64_t)1 << 32) : 0));
  }
  t.len = a->len;
  bn_trim(&t);
  bn_move(r, &t);
}

/* r = a + (negate_b ? -b : b) */
static void bn_addsub(bn *r, const bn *a, const bn *b, int negate_b) {
  int an = a->neg;
  int bneg = b->len ? (b->neg ^ negate_b) : 0;
  if (an == bneg) {
    mag_add(r, a, b);
    r->neg = r->len ? an : 0;
  } else if (mag_cmp(a, b) >= 0) {
    mag_sub(r, a, b);
    r->neg = r->len ? an : 0;
  } else {
    mag_sub(r, b, a);
    r->neg = r->len ? bneg : 0;
  }
}

static void bn_add(bn *r, const bn *a, const bn *b) { bn_addsub(r, a, b, 0); }
static void bn_sub(bn *r, const bn *a, const bn *b) { bn_addsub(r, a, b, 1); }

/* r = a * 2^s */
static void bn_shl(bn *r, const bn *a, size_t s) {
  if (a->len == 0) {
    bn_zero(r);
    return;
  }
  size_t q = s / 32, b = s % 32;
  bn t;
  bn_init(&t);
  bn_reserve(&t, a->len + q + 1);
  memset(t.d, 0, (a->len + q + 1) * sizeof(uint32_t));
  for (size_t i = 0; i < a->len; i++) {
    uint64_t x = (uint64_t)a->d[i] << b;
    t.d[i + q] |= (uint32_t)x;
    t.d[i + q + 1] |= (uint32_t)(x >> 32);
  }
  t.len = a->len + q + 1;
  t.neg = a->neg;
  bn_trim(&t);
  bn_move(r, &t);
}

/* r = a / 2^s, which must be exact (the low s bits of |a| are zero). */
static void bn_shr_exact(bn *r, const bn *a, size_t s) {
  size_t q = s / 32, b = s % 32;
  for (size_t i = 0; i < q && i < a->len; i++) {
    if (a->d[i]) set_err(TCREF_ERR_INEXACT);
  }
  if (b && q < a->len && (a->d[q] & ((1u << b) - 1))) set_err(TCREF_ERR_INEXACT);
  if (a->len <= q) {
    bn_zero(r);
    return;
  }
  bn t;
  bn_init(&t);
  size_t n = a->len - q;
  bn_reserve(&t, n);
  for (size_t i = 0; i < n; i++) {
    uint64_t lo = a->d[i + q];
    uint64_t hi = (i + q + 1 < a->len) ? a->d[i + q + 1] : 0;
    t.d[i] = (uint32_t)(((hi << 32) | lo) >> b);
  }
  t.len = n;
  t.neg = a->neg;
  bn_trim(&t);
  bn_move(r, &t);
}

/* r = a * s for a small signed s (|s| < 2^63). */
static void bn_mul_si(bn *r, const bn *a, int64_t s) {
  if (s == 0 || a->len == 0) {
    bn_zero(r);
    return;
  }
  uint64_t m = s < 0 ? (uint64_t)(-(s + 1)) + 1 : (uint64_t)s;
  bn t;
  bn_init(&t);
  bn_reserve(&t, a->len + 2);
  unsigned __int128 carry = 0;
  for (size_t i = 0; i < a->len; i++) {
    unsigned __int128 p = (unsigned __int128)a->d[i] * m + carry;
    t.d[i] = (uint32_t)p;
    carry = p >> 32;
  }
  t.d[a->len] = (uint32_t)carry;
  t.d[a->len + 1] = (uint32_t)(carry >> 32);
  t.len = a->len + 2;
  t.neg = a->neg ^ (s < 0);
  bn_trim(&t);
  bn_move(r, &t);
}

/* r = a / s for a small signed s != 0; the division must be exact.
 * Long division from the most significant limb down (remainder < |s|). */
static void bn_divexact_si(bn *r, const bn *a, int64_t s) {
  if (s == 0) {
    set_err(TCREF_ERR_ARG);
    return;
  }
  uint64_t d = s < 0 ? (uint64_t)(-(s + 1)) + 1 : (uint64_t)s;
  bn t;
  bn_init(&t);
  bn_reserve(&t, a->len);
  unsigned __int128 rem = 0;
  for (size_t i = a->len; i-- > 0;) {
    unsigned __int128 cur = (rem << 32) | a->d[i];
    t.d[i] = (uint32_t)(cur / d);
    rem = cur % d;
  }
  if (rem != 0) set_err(TCREF_ERR_INEXACT);
  t.len = a->len;
  t.neg = a->neg ^ (s < 0);
  bn_trim(&t);
  bn_move(r, &t);
}

/* r = a * b, schoolbook: every limb of a times every limb of b. */
static void bn_mul(bn *r, const bn *a, const bn *b) {
  if (a->len == 0 || b->len == 0) {
    bn_zero(r);
    return;
  }
  bn t;
  bn_init(&t);
  bn_reserve(&t, a->len + b->len);
  memset(t.d, 0, (a->len + b->len) * sizeof(uint32_t));
  for (size_t i = 0; i < a->len; i++) {
    uint64_t carry = 0;
    for (size_t j = 0; j < b->len; j++) {
      uint64_t p = (uint64_t)a->d[i] * b->d[j] + t.d[i + j] + carry;
      t.d[i + j] = (uint32_t)p;
      carry = p >> 32;
    }
    t.d[i + b->len] = (uint32_t)carry;
  }
  t.len = a->len + b->len;
  t.neg = a->neg ^ b->neg;
  bn_trim(&t);
  bn_move(r, &t);
}

/* ------------------------------------------------------------------------- */
/* Sizes                                                                      */
/* ------------------------------------------------------------------------- */

/* Bits by which |U(x)| can exceed the block bound 2^(32 bl) at the points of
 * a variant.  For x = +/-2^j, j <= B-2: |U(x)| <= (2^(32bl)-1) sum_t 2^(tj)
 * < 2^(32bl) 2^((B-1)(B-2)+1).  B = 2 has only x = +/-1: < 2^(32bl+1).
 * The infinity variant's largest value is U(2) < 7 * 2^(32bl). */
static size_t growth_bits(int B, int variant) {
  if (variant == TCREF_VAR_INF) return 3;
  /* the half variant's largest values are U(+-2) and 8 U(1/2), below 15 2^(32bl) */
  if (variant == TCREF_VAR_HALF) return 4;
  if (B == 2) return 1;
  return (size_t)(B - 1) * (size_t)(B - 2) + 1;
}

size_t tcref_growth_limbs(int B, int variant) {
  return (growth_bits(B, variant) + 31) / 32;
}

size_t tcref_block_limbs(size_t n, int B) { return (n + (size_t)B - 1) / (size_t)B; }

static int plan_level_ok(int B, int variant) {
  if (variant == TCREF_VAR_INF) return B == 3;
  if (variant == TCREF_VAR_HALF) return B == 4;
  if (variant == TCREF_VAR_EVENODD || variant == TCREF_VAR_PLAIN ||
      variant == TCREF_VAR_ODD_DIRECT)
    return B >= 2 && B <= 32;
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Evaluation (sections 1, 4, 6)                                              */
/* ------------------------------------------------------------------------- */

/* Block t of u (nu limbs): limbs [t*bl, (t+1)*bl), zero past nu. */
static void get_block(bn *r, const uint32_t *u, size_t nu, size_t bl, int t) {
  size_t lo = (size_t)t * bl;
  if (lo >= nu) {
    bn_zero(r);
    return;
  }
  size_t hi = lo + bl < nu ? lo + bl : nu;
  bn_set_limbs(r, u + lo, hi - lo);
}

/* With U(x) = U_e(x^2) + x U_o(x^2) (section 4):
 *   E = U_e(4^j)     = sum_k u_{2k} 2^(2jk)
 *   O = 2^j U_o(4^j) = sum_k u_{2k+1} 2^(j(2k+1))
 * so U(+2^j) = E + O and U(-2^j) = E - O. */
static void eval_pm(bn *plus, bn *minus, const bn *blk, int B, int j) {
  bn E, O, t;
  bn_init(&E);
  bn_init(&O);
  bn_init(&t);
  for (int k = 0; 2 * k < B; k++) {
    bn_shl(&t, &blk[2 * k], (size_t)(2 * j * k));
    bn_add(&E, &E, &t);
  }
  for (int k = 0; 2 * k + 1 < B; k++) {
    bn_shl(&t, &blk[2 * k + 1], (size_t)(j * (2 * k + 1)));
    bn_add(&O, &O, &t);
  }
  bn_add(plus, &E, &O);
  bn_sub(minus, &E, &O);
  bn_free(&E);
  bn_free(&O);
  bn_free(&t);
}

/* All 2B-1 point values of one operand in the variant's point order. */
static void eval_points(bn *val, const bn *blk, int B, int variant) {
  if (variant == TCREF_VAR_HALF) {
    bn t;
    bn_init(&t);
    bn_copy(&val[0], &blk[0]);            /* U(0) = u_0 */
    eval_pm(&val[1], &val[2], blk, 4, 0); /* U(+1), U(-1) */
    eval_pm(&val[3], &val[4], blk, 4, 1); /* U(+2), U(-2) */
    bn_zero(&val[5]);                     /* 2^3 U(1/2) = sum_t u_t 2^(3-t) */
    for (int k = 0; k < 4; k++) {
      bn_shl(&t, &blk[k], (size_t)(3 - k));
      bn_add(&val[5], &val[5], &t);
    }
    bn_copy(&val[6], &blk[3]);            /* U(inf) = u_3 */
    bn_free(&t);
    return;
  }
  if (variant == TCREF_VAR_INF) {
    bn unused;
    bn_init(&unused);
    bn_copy(&val[0], &blk[0]);            /* U(0)   = u_0 */
    eval_pm(&val[1], &val[2], blk, 3, 0); /* U(+1), U(-1) */
    eval_pm(&val[3], &unused, blk, 3, 1); /* U(2) */
    bn_copy(&val[4], &blk[2]);            /* U(inf) = u_2 */
    bn_free(&unused);
    return;
  }
  bn_copy(&val[0], &blk[0]); /* U(0) = u_0 */
  for (int j = 0; j <= B - 2; j++) eval_pm(&val[2 * j + 1], &val[2 * j + 2], blk, B, j);
}

/* ------------------------------------------------------------------------- */
/* Newton interpolation (section 3)                                           */
/* ------------------------------------------------------------------------- */

/* Every Newton intermediate must fit a signed two's-complement value of
 * `width` limbs: |c| < 2^(32 width - 1).  The GPU path computes in exactly
 * that fixed width, so this is the bound it relies on. */
static void check_width(const bn *c, size_t width) {
  if (c->len > width || (c->len == width && (c->d[width - 1] >> 31)))
    set_err(TCREF_ERR_RANGE);
}

/* Divided differences, Theorem 3.2 made into an in-place loop:
 *   for k = 1..n, for m = n down to k: c[m] = (c[m] - c[m-1]) / (x[m] - x[m-k]).
 * Afterwards c[k] = alpha_k.  All divisions are exact for the integer data here. */
static void newton_divided_differences(int n, const int64_t *x, bn *c, size_t width) {
  for (int k = 1; k <= n; k++) {
    for (int m = n; m >= k; m--) {
      bn_sub(&c[m], &c[m], &c[m - 1]);
      check_width(&c[m], width);
      bn_divexact_si(&c[m], &c[m], x[m] - x[m - k]);
      count_add(&g_counts.interp_steps, 1);
      count_add(&g_counts.interp_limbs, width);
    }
  }
}

/* Newton form to monomial form, Theorem 3.3 as a loop:
 *   for m = n-1 down to 0, for k = m..n-1: c[k] -= x[m] * c[k+1]. */
static void newton_to_monomial(int n, const int64_t *x, bn *c, size_t width) {
  bn t;
  bn_init(&t);
  for (int m = n - 1; m >= 0; m--) {
    for (int k = m; k <= n - 1; k++) {
      bn_mul_si(&t, &c[k + 1], x[m]);
      bn_sub(&c[k], &c[k], &t);
      check_width(&c[k], width);
      count_add(&g_counts.interp_steps, 1);
      count_add(&g_counts.interp_limbs, width);
    }
  }
  bn_free(&t);
}

int tcref_newton(int n, const int64_t *x, size_t nl, const uint32_t *ymag,
                 const int8_t *ysign, uint32_t *cmag, int8_t *csign, int phase) {
  if (n < 0 || n > 64 || !x || !ymag || !ysign || !cmag || !csign) return TCREF_ERR_ARG;
  for (int i = 0; i <= n; i++)
    for (int j = 0; j < i; j++)
      if (x[i] == x[j]) return TCREF_ERR_ARG;
  t_err = TCREF_OK;
  bn *c = (bn *)calloc((size_t)n + 1, sizeof(bn));
  if (!c) return TCREF_ERR_NOMEM;
  for (int i = 0; i <= n; i++) {
    bn_init(&c[i]);
    bn_set_limbs(&c[i], ymag + (size_t)i * nl, nl);
    c[i].neg = c[i].len ? (ysign[i] != 0) : 0;
  }
  newton_divided_differences(n, x, c, nl);
  if (phase >= 2) newton_to_monomial(n, x, c, nl);
  for (int i = 0; i <= n; i++) {
    bn_get_limbs(&c[i], cmag + (size_t)i * nl, nl);
    csign[i] = (int8_t)c[i].neg;
    bn_free(&c[i]);
  }
  free(c);
  return t_err;
}

/* ------------------------------------------------------------------------- */
/* Interpolation of the 2B-1 products (sections 3, 4)                         */
/* ------------------------------------------------------------------------- */

/* Exact rationals for the fixed-n inverse (entries stay small). */
typedef struct {
  __int128 num, den; /* den > 0, reduced */
} frac;

static __int128 gcd128(__int128 a, __int128 b) {
  if (a < 0) a = -a;
  if (b < 0) b = -b;
  while (b) {
    __int128 t = a % b;
    a = b;
    b = t;
  }
  return a;
}

static frac fr_make(__int128 n, __int128 d) {
  if (d < 0) {
    n = -n;
    d = -d;
  }
  __int128 g = gcd128(n, d);
  if (g > 1) {
    n /= g;
    d /= g;
  }
  frac f = {n, d};
  return f;
}

static frac fr_sub(frac a, frac b) { return fr_make(a.num * b.den - b.num * a.den, a.den * b.den); }
static frac fr_mul(frac a, frac b) { return fr_make(a.num * b.num, a.den * b.den); }
static frac fr_div(frac a, frac b) { return fr_make(a.num * b.den, a.den * b.num); }

/* The inverse of the half variant's 7 x 7 point matrix, by Gauss-Jordan
 * elimination in exact rationals: row i of V holds the weights of w_k in the
 * point value y_i. */
static void half_inverse(frac inv[7][7]) {
  frac a[7][14];
  const int64_t xs[5] = {0, 1, -1, 2, -2};
  for (int i = 0; i < 7; i++)
    for (int k = 0; k < 14; k++) a[i][k] = fr_make(k - 7 == i ? 1 : 0, 1);
  for (int i = 0; i < 5; i++) {
    int64_t p = 1; /* x^k */
    for (int k = 0; k < 7; k++) {
      a[i][k] = fr_make(i == 0 ? (k == 0) : p, 1);
      p *= xs[i];
    }
  }
  for (int k = 0; k < 7; k++) a[5][k] = fr_make((int64_t)1 << (6 - k), 1); /* 2^6 W(1/2) */
  for (int k = 0; k < 7; k++) a[6][k] = fr_make(k == 6, 1);                /* W(inf) = w_6 */
  for (int col = 0; col < 7; col++) {
    int piv = col;
    while (a[piv][col].num == 0) piv++;
    for (int k = 0; k < 14; k++) {
      frac t = a[col][k];
      a[col][k] = a[piv][k];
      a[piv][k] = t;
    }
    const frac pv = a[col][col];
    for (int k = 0; k < 14; k++) a[col][k] = fr_div(a[col][k], pv);
    for (int i = 0; i < 7; i++) {
      if (i == col || a[i][col].num == 0) continue;
      const frac f = a[i][col];
      for (int k = 0; k < 14; k++) a[i][k] = fr_sub(a[i][k], fr_mul(f, a[col][k]));
    }
  }
  for (int i = 0; i < 7; i++)
    for (int k = 0; k < 7; k++) inv[i][k] = a[i][k + 7];
}

/* y: the 2B-1 point products in point order; w: the 2B-1 coefficients. */
static void interp_values(int B, int variant, bn *y, bn *w, size_t width) {
  int n = B - 1;
  if (variant == TCREF_VAR_HALF) {
    /* w = V^-1 y: per coefficient, the row over a common denominator D,
     * then one exact division by D */
    frac inv[7][7];
    half_inverse(inv);
    bn acc, t;
    bn_init(&acc);
    bn_init(&t);
    for (int k = 0; k < 7; k++) {
      __int128 D = 1;
      for (int i = 0; i < 7; i++) D = D / gcd128(D, inv[k][i].den) * inv[k][i].den;
      bn_zero(&acc);
      for (int i = 0; i < 7; i++) {
        const __int128 c = inv[k][i].num * (D / inv[k][i].den);
        bn_mul_si(&t, &y[i], (int64_t)c);
        bn_add(&acc, &acc, &t);
      }
      check_width(&acc, width);
      bn_divexact_si(&w[k], &acc, (int64_t)D);
      count_add(&g_counts.interp_steps, 1);
      count_add(&g_counts.interp_limbs, width);
    }
    bn_free(&acc);
    bn_free(&t);
    return;
  }
  if (variant == TCREF_VAR_INF) {
    /* w_4 = W(inf) = u_2 v_2.  Remove w_4 x^4 from the finite points and
     * interpolate the remaining cubic at x = 0, 1, -1, 2. */
    int64_t x[4] = {0, 1, -1, 2};
    int64_t x4[4] = {0, 1, 1, 16};
    bn c[4], t;
    bn_init(&t);
    for (int i = 0; i < 4; i++) {
      bn_init(&c[i]);
      bn_mul_si(&t, &y[4], x4[i]);
      bn_sub(&c[i], &y[i], &t);
    }
    newton_divided_differences(3, x, c, width);
    newton_to_monomial(3, x, c, width);
    for (int i = 0; i < 4; i++) {
      bn_copy(&w[i], &c[i]);
      bn_free(&c[i]);
    }
    bn_copy(&w[4], &y[4]);
    bn_free(&t);
    return;
  }
  if (variant == TCREF_VAR_PLAIN) {
    /* W(x) of degree 2n directly at all 2n+1 points (no even-odd split). */
    int64_t x[65];
    x[0] = 0;
    for (int j = 0; j < n; j++) {
      x[2 * j + 1] = (int64_t)1 << j;
      x[2 * j + 2] = -((int64_t)1 << j);
    }
    for (int i = 0; i <= 2 * n; i++) bn_copy(&w[i], &y[i]);
    newton_divided_differences(2 * n, x, w, width);
    newton_to_monomial(2 * n, x, w, width);
    return;
  }
  /* Even-odd (section 4).  From W(x) and W(-x) at x = 2^j:
   *   W_e(x^2)        = (W(x) + W(-x)) / 2
   *   x^2 W_o(x^2)    = x (W(x) - W(-x)) / 2
   * Both are polynomials of degree n in X = x^2, at X = 0, 1, 4, ..., 4^(n-1);
   * at X = 0 they take the values W(0) = y_0 and 0. */
  bn *ce = (bn *)calloc((size_t)n + 1, sizeof(bn));
  bn *co = (bn *)calloc((size_t)n + 1, sizeof(bn));
  if (!ce || !co) abort();
  int64_t X[33];
  X[0] = 0;
  for (int m = 1; m <= n; m++) X[m] = (int64_t)1 << (2 * (m - 1));
  for (int i = 0; i <= n; i++) {
    bn_init(&ce[i]);
    bn_init(&co[i]);
  }
  bn_copy(&ce[0], &y[0]);
  bn_zero(&co[0]);
  for (int j = 0; j < n; j++) {
    const bn *yp = &y[2 * j + 1], *ym = &y[2 * j + 2];
    bn_add(&ce[j + 1], yp, ym);
    bn_shr_exact(&ce[j + 1], &ce[j + 1], 1);
    bn_sub(&co[j + 1], yp, ym);
    bn_shr_exact(&co[j + 1], &co[j + 1], 1);
    bn_shl(&co[j + 1], &co[j + 1], (size_t)j);
  }
  newton_divided_differences(n, X, ce, width);
  newton_to_monomial(n, X, ce, width);
  for (int k = 0; k <= n; k++) bn_copy(&w[2 * k], &ce[k]);
  if (variant == TCREF_VAR_ODD_DIRECT) {
    /* W_o(4^j) = x (W(x) - W(-x)) / 2 / x^2 = (W(x) - W(-x)) / 2^(j+1): the
     * values above divided by 4^j exactly; W_o has degree n-1, interpolated
     * at the n nodes X = 4^0 .. 4^(n-1) (entries 1 .. n of X and co). */
    for (int j = 0; j < n; j++) bn_shr_exact(&co[j + 1], &co[j + 1], (size_t)(2 * j));
    newton_divided_differences(n - 1, X + 1, co + 1, width);
    newton_to_monomial(n - 1, X + 1, co + 1, width);
    for (int k = 0; k < n; k++) bn_copy(&w[2 * k + 1], &co[k + 1]);
  } else {
    newton_divided_differences(n, X, co, width);
    newton_to_monomial(n, X, co, width);
    if (co[0].len != 0) set_err(TCREF_ERR_INEXACT); /* x^2 W_o(x^2) has no constant term */
    for (int k = 0; k < n; k++) bn_copy(&w[2 * k + 1], &co[k + 1]);
  }
  for (int i = 0; i <= n; i++) {
    bn_free(&ce[i]);
    bn_free(&co[i]);
  }
  free(ce);
  free(co);
}

/* ------------------------------------------------------------------------- */
/* Recursive multiplication (sections 1, 2)                                   */
/* ------------------------------------------------------------------------- */

static void toom_rec(bn *w, const bn *u, const bn *v, size_t n, const tcref_plan *p,
                     int level);

typedef struct {
  const bn *uv;   /* evaluations of u */
  const bn *vv;   /* evaluations of v */
  bn *y;          /* products */
  size_t width;   /* child nominal width */
  const tcref_plan *plan;
  int level;
  int first, step, count;
  int err;
} prod_job;

static void *prod_worker(void *arg) {
  prod_job *j = (prod_job *)arg;
  t_err = TCREF_OK;
  for (int k = j->first; k < j->count; k += j->step)
    toom_rec(&j->y[k], &j->uv[k], &j->vv[k], j->width, j->plan, j->level);
  j->err = t_err;
  return NULL;
}

/* w = u * v for |u|, |v| < 2^(32 n).  Signs are handled by the caller. */
static void toom_rec(bn *w, const bn *u, const bn *v, size_t n, const tcref_plan *p,
                     int level) {
  if (level >= p->levels) {
    count_add(&g_counts.leaves, 1);
    count_add(&g_counts.leaf_mults, (uint64_t)n * (uint64_t)n);
    if (p->leaf_ntt_bits > 0 && u->len > 0 && v->len > 0) {
      /* section 5: the pointwise products by an FFT (here an exact NTT) */
      bn_reserve(w, u->len + v->len);
      int rc = tcref_mul_ntt(w->d, u->d, u->len, v->d, v->len, p->leaf_ntt_bits);
      if (rc != TCREF_OK) set_err(rc);
      w->len = u->len + v->len;
      w->neg = 0;
      bn_trim(w);
      return;
    }
    bn_mul(w, u, v);
    return;
  }
  int B = p->B[level], variant = p->variant[level];
  int npts = 2 * B - 1;
  size_t bl = tcref_block_limbs(n, B);
  size_t nc = bl + tcref_growth_limbs(B, variant);
  size_t width = 2 * nc + 2;
  count_add(&g_counts.toom_nodes, 1);

  /* Section 1: split into B blocks of b = 32 bl bits. */
  bn *ub = (bn *)calloc((size_t)B, sizeof(bn));
  bn *vb = (bn *)calloc((size_t)B, sizeof(bn));
  bn *uv = (bn *)calloc((size_t)npts, sizeof(bn));
  bn *vv = (bn *)calloc((size_t)npts, sizeof(bn));
  bn *y = (bn *)calloc((size_t)npts, sizeof(bn));
  bn *wk = (bn *)calloc((size_t)npts, sizeof(bn));
  if (!ub || !vb || !uv || !vv || !y || !wk) abort();
  for (int t = 0; t < B; t++) {
    bn_init(&ub[t]);
    bn_init(&vb[t]);
    get_block(&ub[t], u->d, u->len, bl, t);
    get_block(&vb[t], v->d, v->len, bl, t);
  }
  for (int k = 0; k < npts; k++) {
    bn_init(&uv[k]);
    bn_init(&vv[k]);
    bn_init(&y[k]);
    bn_init(&wk[k]);
  }
  /* Evaluate U(x_k), V(x_k); every value must fit the child width. */
  eval_points(uv, ub, B, variant);
  eval_points(vv, vb, B, variant);
  for (int k = 0; k < npts; k++) {
    if (uv[k].len > nc || vv[k].len > nc) set_err(TCREF_ERR_RANGE);
  }
  count_add(&g_counts.eval_limbs, 2 * (uint64_t)npts * nc);

  /* Section 1: the 2B-1 independent products; section 2: the top-level ones
   * on P <= 2B-1 threads. */
  bn *um = (bn *)calloc((size_t)npts, sizeof(bn));
  bn *vm = (bn *)calloc((size_t)npts, sizeof(bn));
  if (!um || !vm) abort();
  for (int k = 0; k < npts; k++) {
    bn_init(&um[k]);
    bn_init(&vm[k]);
    bn_copy(&um[k], &uv[k]);
    um[k].neg = 0;
    bn_copy(&vm[k], &vv[k]);
    vm[k].neg = 0;
  }
  int P = (level == 0 && p->threads > 1) ? p->threads : 1;
  if (P > npts) P = npts;
  if (P > 1) {
    pthread_t th[64];
    prod_job jobs[64];
    for (int i = 0; i < P; i++) {
      jobs[i] = (prod_job){um, vm, y, nc, p, level + 1, i, P, npts, TCREF_OK};
      if (pthread_create(&th[i], NULL, prod_worker, &jobs[i]) != 0) abort();
    }
    for (int i = 0; i < P; i++) {
      pthread_join(th[i], NULL);
      if (jobs[i].err != TCREF_OK) set_err(jobs[i].err);
    }
  } else {
    for (int k = 0; k < npts; k++) toom_rec(&y[k], &um[k], &vm[k], nc, p, level + 1);
  }
  for (int k = 0; k < npts; k++) y[k].neg = y[k].len ? (uv[k].neg ^ vv[k].neg) : 0;

  /* Sections 3 and 4: interpolate the coefficients w_k. */
  interp_values(B, variant, y, wk, width);

  /* Section 1: recompose w = W(2^b) = sum_k w_k 2^(b k). */
  bn_zero(w);
  bn t;
  bn_init(&t);
  for (int k = 0; k < npts; k++) {
    if (wk[k].neg) set_err(TCREF_ERR_INEXACT);
    if (wk[k].len > 2 * bl + 1) set_err(TCREF_ERR_RANGE);
    bn_shl(&t, &wk[k], 32 * bl * (size_t)k);
    bn_add(w, w, &t);
  }
  if (w->len > 2 * n) set_err(TCREF_ERR_RANGE);
  count_add(&g_counts.recomp_limbs, 2 * (uint64_t)n);
  bn_free(&t);

  for (int t2 = 0; t2 < B; t2++) {
    bn_free(&ub[t2]);
    bn_free(&vb[t2]);
  }
  for (int k = 0; k < npts; k++) {
    bn_free(&uv[k]);
    bn_free(&vv[k]);
    bn_free(&um[k]);
    bn_free(&vm[k]);
    bn_free(&y[k]);
    bn_free(&wk[k]);
  }
  free(ub);
  free(vb);
  free(uv);
  free(vv);
  free(um);
  free(vm);
  free(y);
  free(wk);
}

static int plan_ok(const tcref_plan *p) {
  if (!p || p->levels < 0 || p->levels > TCREF_MAX_LEVELS) return 0;
  for (int i = 0; i < p->levels; i++)
    if (!plan_level_ok(p->B[i], p->variant[i])) return 0;
  return p->threads <= 64 && p->leaf_ntt_bits >= 0 && p->leaf_ntt_bits <= 32;
}

/* ------------------------------------------------------------------------- */
/* Public entry points                                                        */
/* ------------------------------------------------------------------------- */

int tcref_mul_school(uint32_t *w, const uint32_t *u, size_t nu, const uint32_t *v,
                     size_t nv) {
  if (!w || !u || !v || nu == 0 || nv == 0) return TCREF_ERR_ARG;
  t_err = TCREF_OK;
  bn a, b, r;
  bn_init(&a);
  bn_init(&b);
  bn_init(&r);
  bn_set_limbs(&a, u, nu);
  bn_set_limbs(&b, v, nv);
  bn_mul(&r, &a, &b);
  bn_get_limbs(&r, w, nu + nv);
  bn_free(&a);
  bn_free(&b);
  bn_free(&r);
  return t_err;
}

int tcref_mul_toom(uint32_t *w, const uint32_t *u, size_t nu, const uint32_t *v,
                   size_t nv, const tcref_plan *plan) {
  if (!w || !u || !v || nu == 0 || nv == 0 || !plan_ok(plan)) return TCREF_ERR_ARG;
  t_err = TCREF_OK;
  bn a, b, r;
  bn_init(&a);
  bn_init(&b);
  bn_init(&r);
  bn_set_limbs(&a, u, nu);
  bn_set_limbs(&b, v, nv);
  toom_rec(&r, &a, &b, nu > nv ? nu : nv, plan, 0);
  bn_get_limbs(&r, w, nu + nv);
  bn_free(&a);
  bn_free(&b);
  bn_free(&r);
  return t_err;
}

int tcref_eval(int B, int variant, const uint32_t *u, size_t nu, size_t bl, size_t nout,
               uint32_t *out, int8_t *sign) {
  if (!plan_level_ok(B, variant) || !u || !out || !sign || bl == 0) return TCREF_ERR_ARG;
  t_err = TCREF_OK;
  int npts = 2 * B - 1;
  bn *blk = (bn *)calloc((size_t)B, sizeof(bn));
  bn *val = (bn *)calloc((size_t)npts, sizeof(bn));
  if (!blk || !val) abort();
  for (int t = 0; t < B; t++) {
    bn_init(&blk[t]);
    get_block(&blk[t], u, nu, bl, t);
  }
  for (int k = 0; k < npts; k++) bn_init(&val[k]);
  eval_points(val, blk, B, variant);
  for (int k = 0; k < npts; k++) {
    bn_get_limbs(&val[k], out + (size_t)k * nout, nout);
    sign[k] = (int8_t)val[k].neg;
    bn_free(&val[k]);
  }
  for (int t = 0; t < B; t++) bn_free(&blk[t]);
  free(blk);
  free(val);
  return t_err;
}

int tcref_interp(int B, int variant, size_t ny, const uint32_t *y, const int8_t *sign,
                 size_t nw, uint32_t *w) {
  if (!plan_level_ok(B, variant) || !y || !sign || !w) return TCREF_ERR_ARG;
  t_err = TCREF_OK;
  int npts = 2 * B - 1;
  bn *yv = (bn *)calloc((size_t)npts, sizeof(bn));
  bn *wv = (bn *)calloc((size_t)npts, sizeof(bn));
  if (!yv || !wv) abort();
  for (int k = 0; k < npts; k++) {
    bn_init(&yv[k]);
    bn_init(&wv[k]);
    bn_set_limbs(&yv[k], y + (size_t)k * ny, ny);
    yv[k].neg = yv[k].len ? (sign[k] != 0) : 0;
  }
  interp_values(B, variant, yv, wv, ny + 2);
  for (int k = 0; k < npts; k++) {
    if (wv[k].neg) set_err(TCREF_ERR_INEXACT);
    bn_get_limbs(&wv[k], w + (size_t)k * nw, nw);
    bn_free(&yv[k]);
    bn_free(&wv[k]);
  }
  free(yv);
  free(wv);
  return t_err;
}

int tcref_recompose(int B, size_t bl, size_t nw, const uint32_t *w, size_t nout,
                    uint32_t *out) {
  if (B < 2 || B > 32 || !w || !out) return TCREF_ERR_ARG;
  t_err = TCREF_OK;
  bn acc, t, c;
  bn_init(&acc);
  bn_init(&t);
  bn_init(&c);
  for (int k = 0; k < 2 * B - 1; k++) {
    bn_set_limbs(&c, w + (size_t)k * nw, nw);
    bn_shl(&t, &c, 32 * bl * (size_t)k);
    bn_add(&acc, &acc, &t);
  }
  bn_get_limbs(&acc, out, nout);
  bn_free(&acc);
  bn_free(&t);
  bn_free(&c);
  return t_err;
}

/* Dry run of toom_rec's sizes: every child of a node has the same width, so
 * one child's counts times 2B-1 gives the node's. */
static void plan_counts_rec(size_t n, const tcref_plan *p, int level, tcref_counts *c) {
  if (level >= p->levels) {
    c->leaves += 1;
    c->leaf_mults += (uint64_t)n * (uint64_t)n;
    return;
  }
  int B = p->B[level], variant = p->variant[level];
  uint64_t npts = 2 * (uint64_t)B - 1;
  size_t bl = tcref_block_limbs(n, B);
  size_t nc = bl + tcref_growth_limbs(B, variant);
  uint64_t width = 2 * nc + 2;
  tcref_counts child;
  memset(&child, 0, sizeof child);
  plan_counts_rec(nc, p, level + 1, &child);
  uint64_t steps;
  int deg = B - 1;
  if (variant == TCREF_VAR_INF)
    steps = 6 + 6; /* cubic: 3+2+1 divided differences, 3+2+1 monomial steps */
  else if (variant == TCREF_VAR_HALF)
    steps = 7; /* one row of the inverse per coefficient */
  else if (variant == TCREF_VAR_PLAIN)
    steps = (uint64_t)(2 * deg) * (2 * deg + 1) / 2 + (uint64_t)(2 * deg) * (2 * deg + 1) / 2;
  else
    steps = 2 * ((uint64_t)deg * (deg + 1) / 2 + (uint64_t)deg * (deg + 1) / 2);
  c->leaves += npts * child.leaves;
  c->leaf_mults += npts * child.leaf_mults;
  c->toom_nodes += 1 + npts * child.toom_nodes;
  c->eval_limbs += 2 * npts * nc + npts * child.eval_limbs;
  c->interp_steps += steps + npts * child.interp_steps;
  c->interp_limbs += steps * width + npts * child.interp_limbs;
  c->recomp_limbs += 2 * (uint64_t)n + npts * child.recomp_limbs;
}

int tcref_plan_counts(size_t n, const tcref_plan *plan, tcref_counts *out) {
  if (!out || !plan_ok(plan) || n == 0) return TCREF_ERR_ARG;
  memset(out, 0, sizeof *out);
  plan_counts_rec(n, plan, 0, out);
  return TCREF_OK;
}
