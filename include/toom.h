/*
 * toom.h -- C ABI of libtoom.so: B-way Toom-Cook multiplication of large
 * unsigned integers on AMD Instinct MI355X (gfx950).
 *
 * Method: M.J. Kronenburg, "Toom-Cook Multiplication: Some Theoretical and
 * Practical Aspects" (arXiv:1602.02740).  A product w = u v is computed as
 * W(2^b) = U(2^b) V(2^b) (section 1): both operands are split into B blocks,
 * evaluated at 2B-1 small points, the 2B-1 point products are formed
 * recursively (section 2) down to schoolbook leaves, the coefficients w_k are
 * recovered by the even-odd method (section 4) and the Newton loops of
 * section 3 with exact divisions, and w is recomposed with full carry
 * propagation.
 *
 * Data: an integer is a little-endian array of 32-bit limbs (tc_limb), limb 0
 * least significant; lengths count limbs.  Unless a function says otherwise,
 * limb pointers are DEVICE pointers owned by the caller; the library never
 * frees them and does not keep them after the work completes.
 *
 * Streams: every call that takes a stream enqueues its work on that stream
 * and returns without waiting (unless stated).  Inputs must stay unchanged,
 * and outputs untouched, until the stream has passed the work.
 *
 * Errors: functions return TC_OK (0) or a negative TC_ERR_* code.  Argument
 * errors are detected on the host before anything is enqueued.  Errors found
 * by the kernels (an exact division with a remainder, a value that overflows
 * its width, a coefficient that comes out negative) are sticky per device and
 * are returned by the next tc_sync() or tc_get_error() as TC_ERR_INEXACT; a
 * batch given a status array gets them per item instead.  The affected
 * results are undefined.  No C++ exception crosses this interface.
 */
#ifndef TOOM_H
#define TOOM_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef uint32_t tc_limb;

#define TC_OK 0
#define TC_ERR_INVALID (-1)     /* null pointer, zero length, aliasing, bad plan */
#define TC_ERR_NOMEM (-2)       /* device or host allocation failed */
#define TC_ERR_HIP (-3)         /* a HIP runtime call failed (see tc_hip_error_string) */
#define TC_ERR_AGAIN (-4)       /* serving queue full: retry later */
#define TC_ERR_NOT_READY (-5)   /* serving: request still pending */
#define TC_ERR_INEXACT (-6)     /* a device exactness check failed (internal fault) */
#define TC_ERR_UNSUPPORTED (-7) /* valid request outside what the library handles */
#define TC_ERR_WORKSPACE (-8)   /* tc_mul_noalloc: the product needs more than the
                                   fixed workspace (tc_noalloc_capacity) */

#define TC_MAX_LEVELS 16

/* Point sets of one recursion level. */
#define TC_VAR_EVENODD 0 /* points 0, +/-2^j (j < B-1): section 6's set used in
                            +/- pairs, interpolated by section 4's even-odd
                            method; 2 <= B <= 32 */
#define TC_VAR_INF 1     /* B = 3 with points 0, 1, -1, 2 and infinity */
#define TC_VAR_HALF 2    /* B = 4 with points 0, 1, -1, 2, -2, 1/2 (the homogeneous
                            value 2^3 U(1/2)) and infinity, interpolated by the
                            fixed-n inverse of section 3's closing remark */

/* How the leaves of a plan form their products. */
#define TC_LEAF_SCHOOL 0 /* schoolbook: vector ALUs up to 32 limbs, exact int8
                            digit convolutions on the matrix cores up to 2048 */
#define TC_LEAF_NTT 1    /* section 5's Toom-Cook over an FFT product: an exact
                            number-theoretic transform over p = 2^64 - 2^32 + 1
                            (see tc_ntt_params); leaves up to about 4 million
                            limbs */

/* A multiplication plan: `levels` Toom levels (level 0 splits the operands),
 * then leaves of kind `leaf` (TC_LEAF_*; 0 is schoolbook).  A level of
 * nominal width n uses blocks of bl = ceil(n / B) limbs and hands its
 * children width bl + g(B).  `chunk` scales the chunk width of the linear
 * passes (evaluation, interpolation, recomposition: 64 LPT limbs a wave) by
 * 2^chunk against the library's rule, with LPT kept within 2..16
 * (-2 <= chunk <= 2; 0 is the rule); the autotuner picks it per size
 * class.  It changes speed only. */
typedef struct {
  int levels;
  int B[TC_MAX_LEVELS];
  int variant[TC_MAX_LEVELS];
  int leaf;
  int chunk;
} tc_plan;

/* ------------------------------------------------------------------ setup */

/* Creates the per-device state (divisor tables, error word) of the current
 * HIP device.  Optional: every call does it on first use.  Synchronous. */
int tc_init(void);

/* Last HIP error string seen by the library in this thread ("" if none). */
const char *tc_hip_error_string(void);

/* Human-readable text of a TC_* code. */
const char *tc_strerror(int code);

/* ------------------------------------------------------------- products */

/* w (nu+nv limbs, device) = u (nu limbs) * v (nv limbs).  nu, nv >= 1.
 * u and v may alias each other (squaring); w must not overlap either.
 * Leading zero limbs are allowed.  Scratch memory belongs to the library's
 * compiled plan of this shape (allocated on its first use, then kept in a
 * per-device cache, see tc_set_cache_limit).  Section 1 defines the product; sections
 * 2-4 and 6 the method.  Balanced sizes (max(nu, nv) < 2 min(nu, nv)) use
 * tc_plan_default(nu, nv).  Unbalanced ones are cut: with s = min(nu, nv),
 * the longer operand's s-limb pieces times the shorter operand are balanced
 * products (plan tc_plan_default(s, s); a shorter last piece is cut again
 * while unbalanced), summed with carry at offsets of s limbs.  The paper's
 * products are balanced; the cut is this library's. */
int tc_mul(tc_limb *w, const tc_limb *u, size_t nu, const tc_limb *v, size_t nv,
           hipStream_t stream);

/* As tc_mul with an explicit plan (host pointer, copied) for blocks of
 * max(nu, nv) limbs; a shorter operand has zero blocks (no cut).  Schoolbook
 * leaves must be at most 2048 limbs wide, transform leaves within
 * tc_ntt_params' range; otherwise TC_ERR_UNSUPPORTED.  Schoolbook leaves up
 * to 32 limbs run on the vector ALUs, wider ones on the matrix cores (exact
 * int8 digit convolutions).  A plan of no level with TC_LEAF_NTT is one
 * transform product of the whole operands. */
int tc_mul_plan(tc_limb *w, const tc_limb *u, size_t nu, const tc_limb *v, size_t nv,
                const tc_plan *plan, hipStream_t stream);

/* The plan tc_mul uses for balanced sizes (host pointer out): the plan
 * tc_autotune measured for their size class if there is one, else no Toom
 * level up to a 2048-limb leaf, and above a 16-way (32-way from 2^22 limbs)
 * top level with 3-way levels until the leaves fit 2048 limbs.  A split is
 * used only when its blocks hold at least 8 g(B) limbs. */
int tc_plan_default(size_t nu, size_t nv, tc_plan *out);

/* Autotuner: times candidate plans for an nu x nv product on the current
 * device (one leaf; or a first split B in {2,3,4,8,16,32}, or Toom-4 on the
 * TC_VAR_HALF points, followed by 3- or 16-way levels down to 512- or
 * 2048-limb leaves; then the fastest with half and double the chunk width of
 * its linear passes, tc_plan::chunk; the minimum of several timed runs each,
 * as a batch of one, on a private stream, with temporary operands) and makes
 * the fastest the default for max(nu, nv)'s size class (a quarter octave),
 * process-wide.  Section 2: any plan yields the same product, so the choice
 * affects speed only.  flags must be 0.  best and ms (host) may be null.
 * Synchronous; allocates and frees device memory. */
int tc_autotune(size_t nu, size_t nv, int flags, tc_plan *best, double *ms);

/* Forgets every tuned plan (back to the built-in defaults). */
int tc_autotune_clear(void);

/* The tuning table, persisted: tc_autotune_save writes every tuned size
 * class (its plan and measured milliseconds) as JSON to `path`, keyed by the
 * current device's architecture and compute-unit count; tc_autotune_load
 * reads such a file and makes its plans the defaults of their classes
 * (TC_ERR_UNSUPPORTED, nothing loaded, if it was tuned on another kind of
 * device; TC_ERR_INVALID for a missing or malformed file).
 * tc_autotune_count returns the number of tuned classes. */
int tc_autotune_save(const char *path);
int tc_autotune_load(const char *path);
int tc_autotune_count(void);

/* Device scratch bytes tc_mul (and tc_mul_plan with `plan`) takes for these
 * sizes: the children's operands and products and the interpolation buffers
 * of every level, the two partial sums of a cut product, and the look-back
 * and error words.  Section 6 gives the extra memory of its sequential
 * scheme as about 6 times the argument size (growing with the threads); the
 * level-synchronous scheme here holds every node of a level at once, about
 * 6 to 8 times the operands for B = 16.  The serving loop admits requests by
 * this figure.  0 for invalid arguments.  Plans only (nothing runs), so it
 * answers without a usable device too. */
size_t tc_workspace_bytes(size_t nu, size_t nv);
size_t tc_workspace_bytes_plan(size_t nu, size_t nv, const tc_plan *plan);

/* tc_mul for callers that cannot allocate device memory: code under HIP
 * stream capture, tight serving loops, harnesses that forbid allocation.
 * Same arguments, rules and result as tc_mul (same plans, bit-identical
 * products), but every buffer beyond the inputs and output lies in a fixed
 * workspace that each device holds for the life of the process
 * (tc_noalloc_capacity() bytes: 64 MiB, enough for products up to about
 * 2^17 x 2^17 limbs).  Calls no hipMalloc, hipFree or other allocating
 * routine: it copies the product's descriptors from host memory into the
 * workspace and launches the kernels directly (no graph).  tc_init() must
 * have been called on the current device first (it looks the workspace up);
 * otherwise TC_ERR_INVALID.  A product whose plan needs more than the
 * workspace returns TC_ERR_WORKSPACE with nothing enqueued.  Every call on a
 * device shares that device's workspace: calls in one stream run one after
 * the other, but calls that overlap on one device (other streams, other
 * threads) race and give undefined results.  Exactness failures set the
 * sticky error word as for tc_mul. */
int tc_mul_noalloc(tc_limb *w, const tc_limb *u, size_t nu, const tc_limb *v, size_t nv,
                   hipStream_t stream);

/* Bytes of tc_mul_noalloc's fixed workspace per device. */
size_t tc_noalloc_capacity(void);

/* One item of a batch: device pointers as for tc_mul. */
typedef struct {
  tc_limb *w;
  const tc_limb *u;
  size_t nu;
  const tc_limb *v;
  size_t nv;
} tc_mul_desc;

/* count independent products of any sizes (host array of descriptors,
 * copied before return; 1 <= count <= 2^24).  Their recursion levels are
 * merged, so each kernel launch serves every item at that level (section 2:
 * the products of a level are independent, and the paper spreads them over
 * its processors).  Each item is computed as tc_mul does (cut when
 * unbalanced).  Same rules per item as tc_mul; in addition no item's output
 * may overlap another item's output or any item's input (TC_ERR_INVALID,
 * checked on the host).
 *
 * status_or_null: null, or count int32 slots (device memory, or host memory;
 * for pageable host memory the call waits for the batch).  When given, each
 * item's exactness failures are kept apart: after the batch, in stream
 * order, status[i] = TC_OK or TC_ERR_INEXACT for item i, and the device's
 * sticky error word is not touched.  When null, failures set the sticky word
 * as for tc_mul. */
int tc_mul_batch(const tc_mul_desc *d, size_t count, int32_t *status_or_null,
                 hipStream_t stream);

/* As tc_mul_batch, each item with its plan plans[i] (host array, copied) as
 * tc_mul_plan does. */
int tc_mul_batch_plan(const tc_mul_desc *d, size_t count, const tc_plan *plans,
                      int32_t *status_or_null, hipStream_t stream);

/* Waits for `stream` and returns the device's sticky error (then clears it). */
int tc_sync(hipStream_t stream);

/* Returns and clears the sticky device error without waiting for the
 * caller's streams (one atomic exchange on the device: an error set by
 * work still running is reported by a later call, never lost). */
int tc_get_error(void);

/* ---------------------------------------------- single phases (parity tests)
 * Each runs one phase of one Toom level on the GPU, with the layouts below,
 * and waits for `stream` before returning. */

/* Evaluation (sections 1, 4, 6): u (nu limbs) split into B blocks of bl
 * limbs, evaluated at the 2B-1 points of `variant` in the order
 *   EVENODD: 0, +2^0, -2^0, +2^1, -2^1, ..., +2^(B-2), -2^(B-2)
 *   INF:     0, +1, -1, +2, infinity
 *   HALF:    0, +1, -1, +2, -2, 2^3 U(1/2), infinity.
 * out: (2B-1) x nout magnitudes; sign: 2B-1 bytes (1 = negative). */
int tc_eval(tc_limb *out, uint8_t *sign, const tc_limb *u, size_t nu, int B, int variant,
            size_t bl, size_t nout, hipStream_t stream);

/* Interpolation (sections 3, 4): the 2B-1 point products y ((2B-1) x ny
 * magnitudes, same point order) with signs `sign` (2B-1 bytes) to the
 * coefficients w_0 .. w_{2B-2} ((2B-1) x nw limbs).  Intermediates are kept
 * in ny+4 limbs of two's complement; consecutive rounds of section 3's loops
 * are composed exactly into shared passes where the combined weights allow.
 * Values that no product can give (a division of section 3 with a
 * remainder, an odd value before a halving) set the sticky error. */
int tc_interp(tc_limb *w, size_t nw, const tc_limb *y, const uint8_t *sign, size_t ny, int B,
              int variant, hipStream_t stream);

/* Recomposition (section 1): out (nout limbs) = sum_k w_k 2^(32 bl k) over
 * the 2B-1 coefficients w ((2B-1) x nw limbs).  A non-zero carry or limb
 * beyond nout sets the sticky error (TC_ERR_INEXACT at tc_sync). */
int tc_recompose(tc_limb *out, size_t nout, const tc_limb *w, size_t nw, int B, size_t bl,
                 hipStream_t stream);

/* Schoolbook leaves: p[i] (2n limbs) = u[i] * v[i] (n limbs each) for
 * i < count, arrays packed back to back.  n <= 2048 (n > 512: matrix cores). */
int tc_school(tc_limb *p, const tc_limb *u, const tc_limb *v, size_t n, size_t count,
              hipStream_t stream);

/* Transform leaves (TC_LEAF_NTT; section 5 multiplies its Toom-Cook pieces
 * with an FFT product).  The field is Z/pZ, p = 2^64 - 2^32 + 1, and the
 * root of order N is w_N = 7^((p-1)/N).  A product of na x nb limbs cuts
 * each operand into pieces of `bits` bits (piece i = floor(u / 2^(bits i))
 * mod 2^bits) and takes the cyclic convolution of length N = 2^logN, which
 * is the acyclic one; it is exact because every coefficient stays below p.
 *
 * tc_ntt_params (host only, no device work): the library's choice for an
 * na x nb product -- the smallest N (2^6 <= N <= 2^24) for which a width
 * 16 <= bits <= 30 fits the convolution (pieces(na) + pieces(nb) - 1 <= N)
 * and keeps it exact ((2^bits - 1)^2 min(pieces) < p), with the narrowest
 * such width -- and its row length C = 2^min(logN, 13) (N = R C).  Any output
 * may be null.  TC_ERR_UNSUPPORTED when no N <= 2^24 fits.
 *
 * tc_ntt_forward: X (N uint64_t, device) = the forward transform of the
 * pieces of u (nu limbs, device) for the (bits, N) of tc_ntt_params, in the
 * library's order: with R = N / C, entry p C + q holds
 * X[rev_R(p) + R rev_C(q)], X[j] = sum_i piece_i w_N^(i j) mod p, rev_M
 * reversing log2 M bits and C = 2^min(log2 N, 13).  Waits for `stream`.
 * TC_ERR_INVALID for a null pointer, nu == 0, bits outside 16..30, N not a
 * power of two in [2^6, 2^24], or more than N pieces in u. */
int tc_ntt_params(size_t na, size_t nb, int *bits, size_t *N, size_t *C);
int tc_ntt_forward(uint64_t *X, const tc_limb *u, size_t nu, int bits, size_t N,
                   hipStream_t stream);

/* Measurement: the issue rate of the 32 x 32 + 32 -> 64 multiply-add
 * (v_mad_u64_u32) on the current device, in operations per second (host
 * pointer out), from a throughput probe of about 2 ms (eight independent
 * chains per lane, 4096 workgroups; the fastest of three runs).  It is the
 * unit the transform leaves' field products (four per product) and the
 * vector-ALU leaves are built from, so their rooflines divide by it.
 * Synchronous; allocates and frees a small device buffer. */
int tc_measure_mad_rate(double *per_s);

/* Strictness of the exactness checks (off by default).  A Toom level whose
 * interpolation is one round (3-way, Karatsuba, TC_VAR_HALF) normally forms
 * its node products in one recomposing step: L W as one combination of the
 * shifted point products, then one exact division by L, the least common
 * multiple of the coefficients' denominators.  That asserts the division by
 * L and that W fits its limbs, but a corrupted point product can change W
 * by a multiple of L and pass.  With strict on, such levels compute every
 * coefficient in its own exact step (each division of section 3 asserted)
 * and recompose separately, at some cost in speed.  Results are identical
 * either way.  Affects plans compiled afterwards on the current device. */
int tc_set_strict(int on);

/* Fault injection, for tests of the exactness checks.  item >= 0: products
 * run after this call (batch item `item`, or a single product for item 0)
 * flip bit 0 of the first limb of their top node's point product at x = +1
 * between the level below and the top interpolation; the even-odd combine
 * of section 4 then halves an odd value, the kernels detect it and report
 * TC_ERR_INEXACT for that item (nothing faults; with tc_set_strict off, a
 * top level computed by a recomposing step may not notice).  Products
 * without a Toom level are unaffected.  item = -1 turns the hook off.  Plans compiled with
 * the hook are cached apart from the others. */
int tc_debug_fault(int item);

/* ------------------------------------------------------------- timing */

/* Kernel classes timed by tc_timing. */
#define TC_KERNEL_EVAL 0
#define TC_KERNEL_LEAF 1
#define TC_KERNEL_STEP 2
#define TC_KERNEL_RECOMP 3
#define TC_KERNEL_CLASSES 4

/* With timing on, every launch of the library is bracketed by HIP events on
 * its stream.  tc_timing_read waits for those events and returns, per kernel
 * class, the number of launches and their summed duration in milliseconds
 * since the last read (arrays of TC_KERNEL_CLASSES entries, host memory). */
int tc_timing_enable(int on);
int tc_timing_read(int64_t *launches, double *ms);

/* Algorithmic work of one tc_mul_plan(nu, nv, plan) (plan NULL: of one
 * tc_mul(nu, nv)) per kernel class: the
 * number of launches, the HBM bytes each class must move (inputs read once,
 * outputs written once, per value), and the limb products of the leaves.  For
 * roofline accounting; nothing is run. */
typedef struct {
  int64_t launches[TC_KERNEL_CLASSES];
  double bytes[TC_KERNEL_CLASSES];
  double leaf_limb_products;
} tc_plan_cost;
/* Plans only, so it answers without a usable device too (out: host). */
int tc_plan_cost_get(size_t nu, size_t nv, const tc_plan *plan, tc_plan_cost *out);

/* Device bytes the cached compiled plans of the current device may hold
 * (persistent scratch of their instances).  Beyond it, least-recently-used
 * plans with no work in flight are released.  Default 32 GiB. */
int tc_set_cache_limit(size_t bytes);

/* ------------------------------------------------------------- serving
 * A request loop on the current device with continuous batching: requests
 * wait in a FIFO queue; whenever one of the server's streams is free and the
 * HBM budget allows, the oldest request is launched together with the queued
 * requests of the same size as one merged product launch (section 2: the
 * products are independent), so batches overlap on the device and requests
 * that arrive meanwhile are admitted as streams and memory free up.
 * Admission counts each request's plan scratch (tc_workspace_bytes) against
 * the budget; that scratch stays device-resident between requests.  Results
 * are bit-identical to tc_mul of the same operands.  All functions are
 * thread-safe; a device exactness error is reported in the status of exactly
 * the request that had it (each batch has per-item status), and the device's
 * sticky error word is not touched. */
typedef struct tc_server tc_server;

typedef struct {
  size_t hbm_budget;   /* plan scratch bytes of in-flight work (0: a quarter of free memory) */
  size_t max_inflight; /* requests on the device at once (0: 256) */
  size_t max_queued;   /* waiting requests; beyond it tc_submit returns TC_ERR_AGAIN (0: 4096) */
  int streams;         /* HIP streams (default priority) batches overlap on (0: 4) */
  int max_batch;       /* requests merged into one launch (0: 64) */
} tc_server_cfg;

typedef struct {
  int status;       /* TC_OK or the error of the request's batch */
  double submit_us; /* host times in microseconds since the server was created */
  double start_us;  /* batch launched */
  double finish_us; /* completion seen by the server */
} tc_result;

typedef struct {
  uint64_t submitted, completed, rejected, batches;
  uint64_t queued, inflight;
  size_t inflight_bytes;
  double p50_us, p99_us;    /* submit -> completion latency of completed requests */
  double limb_mults_per_s;  /* sum of nu*nv completed / window */
  double window_s;          /* first submit -> last completion */
} tc_stats;

/* Creates a server (cfg may be null: all defaults) and its scheduler thread.
 * Idle plans stay cached (with their scratch) up to tc_set_cache_limit. */
int tc_server_create(const tc_server_cfg *cfg, tc_server **out);

/* Queues w = u * v (device pointers, rules of tc_mul; the caller keeps them
 * valid and untouched until the request completes).  Non-blocking; writes
 * the request's ticket.  TC_ERR_AGAIN: queue full; TC_ERR_NOMEM: the request
 * alone exceeds the budget. */
int tc_submit(tc_server *s, tc_limb *w, const tc_limb *u, size_t nu, const tc_limb *v, size_t nv,
              uint64_t *ticket);

/* TC_OK with *r filled once the request has completed (each ticket is
 * reported once); TC_ERR_NOT_READY while it is queued or running;
 * TC_ERR_INVALID for an unknown or already reported ticket. */
int tc_poll(tc_server *s, uint64_t ticket, tc_result *r);

/* Counters and latency percentiles since creation or the last reset. */
int tc_server_stats(tc_server *s, tc_stats *out);
int tc_server_reset_stats(tc_server *s);

/* Completes all queued and running requests, then frees the server. */
int tc_server_destroy(tc_server *s);

#ifdef __cplusplus
}
#endif
#endif /* TOOM_H */
