/*
 * nttref.c -- CPU oracle for products formed by a number-theoretic transform
 * (the FFT multiplier that section 5 places under a Toom-Cook top level).
 *
 * TEST INFRASTRUCTURE ONLY (see toomref.h).  Plain and slow on purpose:
 * field arithmetic is 128-bit multiplication followed by the % operator, and
 * the transform is the textbook recursive radix-2 split of the discrete
 * Fourier transform X[j] = sum_i x[i] w^(i j).
 *
 * Conventions (shared by agreement with the GPU library, not by code):
 *  - The field is Z/pZ with p = 2^64 - 2^32 + 1.
 *  - The root of order N (a power of two, N <= 2^32) is w_N = 7^((p-1)/N).
 *  - An operand of n limbs is cut into pieces of `bits` bits: piece i is
 *    floor(u / 2^(bits i)) mod 2^bits, for i < ceil(32 n / bits).
 *  - The product of pieces a, b is the cyclic convolution of length
 *    N >= len(a) + len(b) - 1, which is the acyclic one; it is exact when
 *    every coefficient is below p, i.e. (2^bits - 1)^2 min(len a, len b) < p.
 *  - The result is sum_k c_k 2^(bits k), written in nu + nv limbs.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "toomref.h"

#define P_FIELD 0xFFFFFFFF00000001ull

typedef unsigned __int128 u128;

static uint64_t f_add(uint64_t a, uint64_t b) { return (uint64_t)(((u128)a + b) % P_FIELD); }
static uint64_t f_sub(uint64_t a, uint64_t b) { return a >= b ? a - b : a + (P_FIELD - b); }
static uint64_t f_mul(uint64_t a, uint64_t b) { return (uint64_t)(((u128)a * b) % P_FIELD); }

static uint64_t f_pow(uint64_t a, uint64_t e) {
  uint64_t r = 1;
  while (e) {
    if (e & 1) r = f_mul(r, a);
    a = f_mul(a, a);
    e >>= 1;
  }
  return r;
}

uint64_t tcref_ntt_root(uint64_t N) {
  if (N == 0 || (N & (N - 1)) || N > ((uint64_t)1 << 32)) return 0;
  return f_pow(7, (P_FIELD - 1) / N);
}

/* X[j] = sum_i x[i] w^(i j), j < n, by X[j] = E[j] + w^j O[j] and
 * X[j + n/2] = E[j] - w^j O[j], where E and O are the transforms of the even-
 * and odd-indexed inputs with the root w^2. */
static void dft_rec(uint64_t *x, size_t n, uint64_t w) {
  if (n == 1) return;
  size_t h = n / 2;
  uint64_t *e = (uint64_t *)malloc(h * sizeof(uint64_t));
  uint64_t *o = (uint64_t *)malloc(h * sizeof(uint64_t));
  if (!e || !o) abort();
  for (size_t i = 0; i < h; i++) {
    e[i] = x[2 * i];
    o[i] = x[2 * i + 1];
  }
  uint64_t w2 = f_mul(w, w);
  dft_rec(e, h, w2);
  dft_rec(o, h, w2);
  uint64_t t = 1;
  for (size_t j = 0; j < h; j++) {
    uint64_t a = e[j], b = f_mul(t, o[j]);
    x[j] = f_add(a, b);
    x[j + h] = f_sub(a, b);
    t = f_mul(t, w);
  }
  free(e);
  free(o);
}

int tcref_ntt(uint64_t *x, size_t N, int inverse) {
  uint64_t w = tcref_ntt_root(N);
  if (!x || w == 0) return TCREF_ERR_ARG;
  for (size_t i = 0; i < N; i++)
    if (x[i] >= P_FIELD) return TCREF_ERR_RANGE;
  if (inverse) w = f_pow(w, P_FIELD - 2);
  dft_rec(x, N, w);
  if (inverse) {
    uint64_t ninv = f_pow((uint64_t)N % P_FIELD, P_FIELD - 2);
    for (size_t i = 0; i < N; i++) x[i] = f_mul(x[i], ninv);
  }
  return TCREF_OK;
}

size_t tcref_ntt_npieces(size_t n, int bits) {
  return bits <= 0 ? 0 : (32 * n + (size_t)bits - 1) / (size_t)bits;
}

/* bit t of u (0 beyond its n limbs) */
static unsigned bit_of(const uint32_t *u, size_t n, uint64_t t) {
  uint64_t L = t / 32;
  return L < n ? (u[L] >> (t % 32)) & 1u : 0u;
}

int tcref_ntt_pieces(const uint32_t *u, size_t nu, int bits, uint64_t *out, size_t nout) {
  if (!u || !out || bits < 1 || bits > 32) return TCREF_ERR_ARG;
  for (size_t i = 0; i < nout; i++) {
    uint64_t a = 0;
    for (int b = bits - 1; b >= 0; b--) a = 2 * a + bit_of(u, nu, (uint64_t)bits * i + b);
    out[i] = a;
  }
  return TCREF_OK;
}

int tcref_mul_ntt(uint32_t *w, const uint32_t *u, size_t nu, const uint32_t *v, size_t nv,
                  int bits) {
  if (!w || !u || !v || nu == 0 || nv == 0 || bits < 1 || bits > 32) return TCREF_ERR_ARG;
  size_t pa = tcref_ntt_npieces(nu, bits), pb = tcref_ntt_npieces(nv, bits);
  /* exactness: every convolution coefficient below p */
  u128 mx = ((u128)1 << bits) - 1;
  if (mx * mx * (u128)(pa < pb ? pa : pb) >= (u128)P_FIELD) return TCREF_ERR_RANGE;
  size_t N = 1;
  while (N < pa + pb - 1) N *= 2;
  if (N > ((size_t)1 << 32)) return TCREF_ERR_ARG;
  uint64_t *a = (uint64_t *)calloc(N, sizeof(uint64_t));
  uint64_t *b = (uint64_t *)calloc(N, sizeof(uint64_t));
  if (!a || !b) abort();
  tcref_ntt_pieces(u, nu, bits, a, pa);
  tcref_ntt_pieces(v, nv, bits, b, pb);
  /* convolution theorem: c = inverse(forward(a) . forward(b)) */
  tcref_ntt(a, N, 0);
  tcref_ntt(b, N, 0);
  for (size_t j = 0; j < N; j++) a[j] = f_mul(a[j], b[j]);
  tcref_ntt(a, N, 1);
  /* w = sum_k c_k 2^(bits k): add each coefficient at its bit offset */
  size_t nw = nu + nv;
  memset(w, 0, nw * sizeof(uint32_t));
  int err = TCREF_OK;
  for (size_t k = 0; k < pa + pb - 1; k++) {
    uint64_t off = (uint64_t)bits * k;
    size_t L = (size_t)(off / 32);
    u128 add = (u128)a[k] << (off % 32);
    uint64_t carry = 0;
    for (size_t q = L; add != 0 || carry != 0; q++) {
      if (q >= nw) {
        err = TCREF_ERR_RANGE;
        break;
      }
      uint64_t s = (uint64_t)w[q] + (uint64_t)(add & 0xFFFFFFFFu) + carry;
      w[q] = (uint32_t)s;
      carry = s >> 32;
      add >>= 32;
    }
  }
  for (size_t k = pa + pb - 1; k < N; k++)
    if (a[k] != 0) err = TCREF_ERR_INEXACT; /* a cyclic wrap: cannot happen when exact */
  free(a);
  free(b);
  return err;
}
