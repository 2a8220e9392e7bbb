// tc_host.hip -- host runtime of libtoom.so: per-device state, the planner,
// the descriptor compiler that turns a plan into merged level-synchronous
// kernel launches, the executor, and the C ABI of include/toom.h.
//
// Execution model.  A product (or a batch of products) is compiled once per
// shape into a list of launches:
//   down:  for each recursion depth d, one evaluation launch for every node of
//          every item at depth d (both operands, all 2B-1 points);
//   leaf:  one schoolbook launch per leaf shape;
//   up:    for each depth from the deepest up, the even-odd combine
//          (section 4), the Newton divided-difference rounds and the
//          Newton-to-monomial rounds (section 3), then the recomposition.
// Within a round of the Newton loops every update reads only values of the
// previous round (the paper's loops run m downwards, or k upwards, exactly so
// that no value is read after it is overwritten), so a round is one launch;
// each value has two buffers used alternately.  Compiled plans are cached
// per shape; addresses are (buffer, offset) pairs resolved at run time.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/toom.h"
#include "tc_field.hpp"
#include "tc_internal.hpp"

using namespace tc;

// The fixed workspace of tc_mul_noalloc, for callers that cannot allocate:
// the Bases record, the descriptors and the scratch of one product.  Every
// device the library runs on holds its own copy until the process ends.
// Host code must not use this name as an address: it reaches the current
// device's copy only through the pointer hipGetSymbolAddress returned when
// the device's context was set up (Ctx::na_ptr).
constexpr size_t kNoAllocBytes = (size_t)64 << 20;
static __device__ __align__(256) uint8_t scratch[kNoAllocBytes];

namespace {

thread_local std::string g_hip_err;

int hip_fail(hipError_t e) {
  g_hip_err = hipGetErrorString(e);
  (void)hipGetLastError();
  return e == hipErrorOutOfMemory ? TC_ERR_NOMEM : TC_ERR_HIP;
}

#define HIPCHK(x)                              \
  do {                                         \
    hipError_t e_ = (x);                       \
    if (e_ != hipSuccess) return hip_fail(e_); \
  } while (0)

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// ------------------------------------------------------------------ divisors

uint32_t inv_mod_2_32(uint32_t d) {
  uint32_t x = d;  // correct to 3 bits for odd d; each step doubles
  for (int i = 0; i < 5; i++) x *= 2u - d * x;
  return x;
}

uint64_t inv_mod(uint64_t a, uint64_t m) {
  int64_t t = 0, nt = 1;
  int64_t r = (int64_t)m, nr = (int64_t)(a % m);
  while (nr != 0) {
    const int64_t q = r / nr;
    int64_t tmp = t - q * nt;
    t = nt;
    nt = tmp;
    tmp = r - q * nr;
    r = nr;
    nr = tmp;
  }
  if (t < 0) t += (int64_t)m;
  return (uint64_t)t;
}

void make_div(DivEntry& e, uint32_t d) {
  e.d = d;
  e.dinv = inv_mod_2_32(d);
  const uint64_t M = inv_mod((1ull << 32) % d, d);  // 2^-32 mod d
  uint64_t p = 1 % d;
  for (int j = 0; j <= kPowMax; j++) {
    e.pw[j] = (uint32_t)p;
    e.pws[j] = (uint32_t)((p << 32) / d);
    p = p * M % d;
  }
  for (int kind = 0; kind < kChunkKinds; kind++) {
    const int T = 64 * (2 << kind);  // LPT = 2, 4, 8, 16
    uint64_t MT = 1 % d;
    for (int j = 0; j < T; j++) MT = MT * M % d;
    uint64_t w = 1 % d;
    for (int l = 0; l <= kWindow; l++) {
      e.cw[kind][l] = (uint32_t)w;
      e.cws[kind][l] = (uint32_t)((w << 32) / d);
      w = w * MT % d;
    }
  }
}

// The odd divisors of the Newton loops: X_m - X_{m-k} = 4^(m-k-1) (4^k - 1)
// for the even-odd nodes X = 0, 1, 4, ..., 4^(B-2), plus 3 for the infinity
// variant.  4^k - 1 fits a word for k <= 15; beyond, its coprime factors
// 2^k - 1 and 2^k + 1 are used one after the other.
std::vector<uint32_t> divisor_set() {
  std::vector<uint32_t> v;
  for (int k = 1; k <= 15; k++) v.push_back((uint32_t)((1ull << (2 * k)) - 1));
  for (int k = 16; k <= 31; k++) {
    v.push_back((uint32_t)((1ull << k) - 1));
    v.push_back((uint32_t)((1ull << k) + 1));
  }
  return v;
}

// ------------------------------------------------------------------ context

struct TimedLaunch {
  int kind;
  hipEvent_t a, b;
};

struct Compiled;

struct Ctx {
  int dev = 0;
  DivEntry* d_div = nullptr;      // kMaxDivs entries; the first div_n are filled
  uint64_t* d_ntt = nullptr;      // roots of the transform leaves (kNttRootEntries)
  std::map<uint32_t, int> div_id;
  int div_n = 0;
  std::mutex div_mu;
  uint32_t* d_err = nullptr;      // the sticky error word of single products
  uint32_t* h_err = nullptr;      // pinned: where tc_get_error takes the word to
  hipStream_t err_stream = nullptr;
  // Host-to-device uploads of tables and plan blobs: a non-blocking stream of
  // the library's own, so they never touch the legacy stream (another
  // thread's graph capture would make such a copy fail).
  hipStream_t up_stream = nullptr;
  std::mutex err_mu;
  std::mutex mu;
  std::map<std::string, std::shared_ptr<Compiled>> cache;
  uint64_t use_clock = 0;                   // for least-recently-used eviction
  size_t cache_limit = (size_t)32 << 30;    // device bytes cached plans may hold
  bool timing = false;
  std::vector<TimedLaunch> timed;
  std::vector<hipEvent_t> event_pool;
  bool graphs = true;        // replay captured graphs (off while timing)
  int fault_item = -1;       // tc_debug_fault: the item whose plans flip a product bit
  bool strict = false;       // tc_set_strict: no recomposing steps (every coefficient checked)
  // tc_mul_noalloc: this device's copy of the fixed workspace, the host-side
  // compiled plans that run from it, and the Bases record staged into it
  uint8_t* na_ptr = nullptr;
  std::map<std::string, std::shared_ptr<Compiled>> na_cache;
  Bases na_bases{};
  std::mutex na_mu;
  hipStream_t capture_stream = nullptr;
};

std::mutex g_ctx_mu;
std::map<int, std::unique_ptr<Ctx>> g_ctx;

// ------------------------------------------------------------------ transform leaves

using u128 = unsigned __int128;

uint64_t field_pow(uint64_t a, uint64_t e) {
  uint64_t r = 1;
  while (e) {
    if (e & 1) r = fp_mul(r, a);
    a = fp_mul(a, a);
    e >>= 1;
  }
  return r;
}

// The roots of the transform leaves in the layout of tc_types.hpp: powers of
// w_8192 = 7^((p-1)/8192) and of w_2^24 = 7^((p-1)/2^24), and of their
// inverses (7 is not a square modulo p, so w_M has order exactly M).
std::vector<uint64_t> ntt_roots() {
  const uint64_t w13 = field_pow(7, (kFieldP - 1) >> 13), w24 = field_pow(7, (kFieldP - 1) >> 24);
  const uint64_t w13i = field_pow(w13, kFieldP - 2), w24i = field_pow(w24, kFieldP - 2);
  const uint64_t step[6] = {w13, w13i, w24, field_pow(w24, 4096), w24i, field_pow(w24i, 4096)};
  const int at[6] = {kNttRootFwd, kNttRootInv, kNttLo, kNttHi, kNttLoInv, kNttHiInv};
  std::vector<uint64_t> t(kNttRootEntries);
  for (int j = 0; j < 6; j++) {
    uint64_t x = 1;
    for (int k = 0; k < 4096; k++) {
      t[(size_t)(at[j] + k)] = x;
      x = fp_mul(x, step[j]);
    }
  }
  // per-stage copies of w_8192^k: w_2h^i = w_8192^(i 8192 / 2h)
  for (int inv = 0; inv < 2; inv++) {
    const uint64_t* W = t.data() + (inv ? kNttRootInv : kNttRootFwd);
    for (int lo = 0; lo <= 11; lo++) {
      const int h = 1 << lo;
      uint64_t* T = t.data() + (inv ? kNttTw4Inv : kNttTw4Fwd) + 3 * (h - 1);
      for (int i = 0; i < h; i++) {
        T[i] = W[i << (11 - lo)];            // w_4h^i
        T[h + i] = W[(i + h) << (11 - lo)];  // w_4h^(i+h)
        T[2 * h + i] = W[i << (12 - lo)];    // w_2h^i
      }
    }
    for (int lh = 0; lh <= 12; lh++) {
      const int h = 1 << lh;
      uint64_t* T = t.data() + (inv ? kNttTw2Inv : kNttTw2Fwd) + (h - 1);
      for (int i = 0; i < h; i++) T[i] = W[i << (12 - lh)];
    }
  }
  return t;
}

int64_t ntt_pieces(int64_t n, int bits) { return (32 * n + bits - 1) / bits; }

// Piece width and transform length of an na x nb transform leaf: the
// smallest N = 2^logN (2^6 .. 2^24) for which a width 16 <= bits <= 30 holds
// the convolution (pieces(na) + pieces(nb) - 1 <= N) and keeps it exact
// (every coefficient below p: (2^bits - 1)^2 min(pieces) < p), with the
// narrowest such width.
bool ntt_choose(int64_t na, int64_t nb, int* bits, int* logN) {
  for (int k = 6; k <= 24; k++)
    for (int w = 16; w <= 30; w++) {
      const int64_t pa = ntt_pieces(na, w), pb = ntt_pieces(nb, w);
      if (pa + pb - 1 > ((int64_t)1 << k)) continue;
      const u128 mx = ((u128)1 << w) - 1;
      if (mx * mx * (u128)std::min(pa, pb) >= (u128)kFieldP) continue;
      *bits = w;
      *logN = k;
      return true;
    }
  return false;
}

// n bytes from host memory at src to device memory at dst, complete on return.
hipError_t upload(Ctx* c, void* dst, const void* src, size_t n) {
  hipError_t e = hipMemcpyAsync(dst, src, n, hipMemcpyHostToDevice, c->up_stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->up_stream);
  return e;
}

int get_ctx(Ctx** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_ctx_mu);
  auto it = g_ctx.find(dev);
  if (it != g_ctx.end()) {
    *out = it->second.get();
    return TC_OK;
  }
  auto c = std::make_unique<Ctx>();
  c->dev = dev;
  const std::vector<uint32_t> ds = divisor_set();
  std::vector<DivEntry> tab(ds.size());
  for (size_t i = 0; i < ds.size(); i++) {
    make_div(tab[i], ds[i]);
    c->div_id[ds[i]] = (int)i;
  }
  c->div_n = (int)ds.size();
  HIPCHK(hipStreamCreateWithFlags(&c->up_stream, hipStreamNonBlocking));
  HIPCHK(hipMalloc(&c->d_div, (size_t)kMaxDivs * sizeof(DivEntry)));
  HIPCHK(upload(c.get(), c->d_div, tab.data(), tab.size() * sizeof(DivEntry)));
  {
    const std::vector<uint64_t> roots = ntt_roots();
    HIPCHK(hipMalloc(&c->d_ntt, roots.size() * sizeof(uint64_t)));
    HIPCHK(upload(c.get(), c->d_ntt, roots.data(), roots.size() * sizeof(uint64_t)));
  }
  HIPCHK(hipMalloc(&c->d_err, sizeof(uint32_t)));
  {
    const uint32_t zero = 0;
    HIPCHK(upload(c.get(), c->d_err, &zero, sizeof(uint32_t)));
  }
  HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&c->h_err), sizeof(uint32_t), hipHostMallocDefault));
  HIPCHK(hipStreamCreateWithFlags(&c->err_stream, hipStreamNonBlocking));
  int lds = 0;
  if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
      lds > 0)
    (void)set_mleaf_lds_limit((size_t)lds - 1024);  // room for the kernel's static LDS
  {
    // this device's copy of the fixed workspace (tc_mul_noalloc)
    void* sp = nullptr;
    if (hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch)) == hipSuccess) c->na_ptr = static_cast<uint8_t*>(sp);
    else (void)hipGetLastError();
  }
  hipMemPool_t pool;
  if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
    uint64_t thr = UINT64_MAX;
    (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
  }
  (void)hipGetLastError();
  *out = c.get();
  g_ctx[dev] = std::move(c);
  return TC_OK;
}

// The context of the current device if it has been set up (nothing is
// created).
int find_ctx(Ctx** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_ctx_mu);
  auto it = g_ctx.find(dev);
  if (it == g_ctx.end()) return TC_ERR_INVALID;
  *out = it->second.get();
  return TC_OK;
}

// Planning-only queries (costs, workspace sizes) also work without a usable
// device: they then plan against a host context whose divisor table stays
// on the host.  Nothing is run through it.
int get_plan_ctx(Ctx** out) {
  if (get_ctx(out) == TC_OK) return TC_OK;
  (void)hipGetLastError();
  static std::unique_ptr<Ctx> host;
  std::lock_guard<std::mutex> lk(g_ctx_mu);
  if (!host) {
    auto c = std::make_unique<Ctx>();
    c->dev = -1;
    const std::vector<uint32_t> ds = divisor_set();
    for (size_t i = 0; i < ds.size(); i++) c->div_id[ds[i]] = (int)i;
    c->div_n = (int)ds.size();
    host = std::move(c);
  }
  *out = host.get();
  return TC_OK;
}

// ------------------------------------------------------------------ planning

int64_t growth_limbs(int B, int var) {
  if (var == TC_VAR_INF || var == TC_VAR_HALF) return 1;  // below 7 and 15 times 2^(32 bl)
  if (B == 2) return 1;
  const int64_t bits = (int64_t)(B - 1) * (B - 2) + 1;
  return (bits + 31) / 32;
}

bool plan_ok(const tc_plan& p) {
  if (p.levels < 0 || p.levels > TC_MAX_LEVELS) return false;
  if (p.leaf != TC_LEAF_SCHOOL && p.leaf != TC_LEAF_NTT) return false;
  if (p.chunk < -2 || p.chunk > 2) return false;
  for (int i = 0; i < p.levels; i++) {
    if (p.variant[i] == TC_VAR_INF) {
      if (p.B[i] != 3) return false;
    } else if (p.variant[i] == TC_VAR_HALF) {
      if (p.B[i] != 4) return false;
    } else if (p.variant[i] == TC_VAR_EVENODD) {
      if (p.B[i] < 2 || p.B[i] > kMaxB) return false;
    } else {
      return false;
    }
  }
  return true;
}

int64_t leaf_width(int64_t n, const tc_plan& p) {
  for (int i = 0; i < p.levels; i++) n = (n + p.B[i] - 1) / p.B[i] + growth_limbs(p.B[i], p.variant[i]);
  return n;
}

// The leaves of p for nominal width n are within what their kind handles.
bool leaves_fit(int64_t n, const tc_plan& p) {
  const int64_t w = leaf_width(n, p);
  int bits, logN;
  return p.leaf == TC_LEAF_NTT ? ntt_choose(w, w, &bits, &logN) : w <= kLeafMax;
}

// The plan tc_mul uses: no Toom level up to a leaf (vector ALUs to 512
// limbs, matrix cores to 2048); above, a wide top level (16- or 32-way,
// section 2's lower exponent) and 3-way levels until the children fit a
// matrix-core leaf.  A split needs blocks of at least 8 g(B) limbs.
// A split applies when its blocks hold at least 8 g(B) limbs.
bool split_ok(int64_t n, int B, int var) {
  return (n + B - 1) / B >= 8 * growth_limbs(B, var);
}

// Plans chosen by measurement (tc_autotune), per quarter-octave size class
// of max(nu, nv); process-wide.
std::mutex g_tune_mu;
std::map<int, tc_plan> g_tuned;
std::map<int, double> g_tuned_ms;  // the winner's measured time, for the saved table

int size_class(int64_t n) { return (int)std::floor(4.0 * std::log2((double)n)); }

// The tuned plan of n's class, if its splits apply to n and its leaves fit.
bool tuned_plan(int64_t n, tc_plan* out) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tuned.find(size_class(n));
  if (it == g_tuned.end()) return false;
  const tc_plan& p = it->second;
  int64_t w = n;
  for (int i = 0; i < p.levels; i++) {
    if (!split_ok(w, p.B[i], p.variant[i])) return false;
    w = (w + p.B[i] - 1) / p.B[i] + growth_limbs(p.B[i], p.variant[i]);
  }
  if (w > kLeafMax) return false;
  *out = p;
  return true;
}

tc_plan default_plan(int64_t n) {
  tc_plan p;
  std::memset(&p, 0, sizeof p);
  if (tuned_plan(n, &p)) return p;
  while (n > kLeafMax && p.levels < TC_MAX_LEVELS) {
    int B = 3;
    if (p.levels == 0 && n >= (int64_t)1 << 22) B = 32;
    else if (p.levels == 0 && n >= (int64_t)1 << 15) B = 16;
    while (B > 3 && !split_ok(n, B, TC_VAR_EVENODD)) B /= 2;
    p.B[p.levels] = B;
    p.variant[p.levels] = TC_VAR_EVENODD;
    p.levels++;
    n = (n + B - 1) / B + growth_limbs(B, TC_VAR_EVENODD);
  }
  return p;
}

// ------------------------------------------------------------------ compiled plans

struct Launch {
  int kind;          // TC_KERNEL_*
  int lpt;           // engine limbs per lane
  int neg_pass;      // TC_KERNEL_EVAL: the sign fix-up of multi-chunk values
  LeafShape leaf;    // TC_KERNEL_LEAF
  int mleaf_n;       // TC_KERNEL_LEAF on the matrix cores: the leaf width
  size_t desc_off, w0_off;
  int nd;
  int64_t units;     // waves (leaf: workgroups)
  size_t lds;        // transform leaves: dynamic LDS bytes
  int64_t per_desc;  // > 0: every descriptor holds this many units; -1, -2
                     // (steps, evaluations): every descriptor has the same
                     // count and chunks, and waves run chunk position by
                     // chunk position (-2: node by node within a position)
};

// One set of device resources a compiled plan runs with: persistent scratch,
// the device copy of the run's base addresses (written before each run), the
// batch pointer table, and the captured graph of all launches.  A run may
// reuse an instance once the previous run on it has completed (`done`).
struct Instance {
  hipGraphExec_t exec = nullptr;
  Bases* d_bases = nullptr;
  Bases* h_bases = nullptr;  // pinned staging
  uint8_t* scratch = nullptr;
  void** d_table = nullptr;
  void** h_table = nullptr;  // pinned staging
  hipEvent_t done = nullptr;
  ~Instance() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (d_bases) (void)hipFree(d_bases);
    if (h_bases) (void)hipHostFree(h_bases);
    if (scratch) (void)hipFree(scratch);
    if (d_table) (void)hipFree(d_table);
    if (h_table) (void)hipHostFree(h_table);
    if (done) (void)hipEventDestroy(done);
  }
};

constexpr size_t kMaxInstances = 4;

struct Compiled {
  std::vector<Launch> launches;
  uint8_t* d_blob = nullptr;
  std::vector<uint8_t> h_blob;  // host copy, for plans that run from the fixed workspace
  size_t scratch_bytes = 0;
  size_t status_off = 0;     // bytes into scratch
  int64_t status_words = 0;  // look-back words, zeroed before every run
  // ranges cleared before every run (the look-back words and the Builder's
  // zeroed ranges): (byte offset into scratch, 64-bit words) pairs in the blob
  size_t fill_off = 0;
  int nfill = 0;
  int64_t fill_max = 0;
  size_t table_n = 0;        // batch pointer table entries (3 per item)
  int64_t items = 1;         // products (batch items)
  size_t item_err_off = 0;   // bytes into scratch: one error word per item
  size_t item_stat_off = 0;  // bytes into scratch: one int32 status per item
  tc_plan_cost cost{};       // algorithmic work per kernel class
  uint64_t last_use = 0;
  std::vector<std::unique_ptr<Instance>> inst;
  size_t device_bytes() const { return inst.size() * scratch_bytes; }
  bool idle() const {
    for (auto& i : inst)
      if (hipEventQuery(i->done) != hipSuccess) return false;
    return true;
  }
  ~Compiled() {
    for (auto& i : inst)
      if (i->done) (void)hipEventSynchronize(i->done);
    inst.clear();
    if (d_blob) (void)hipFree(d_blob);
  }
};

int lpt_for(int64_t Y) {
  if (Y <= 128) return 2;
  if (Y <= 256) return 4;
  return 8;
}

// Interpolation steps of very wide values take 1024-limb chunks: half the
// per-chunk work (scans, look-back) per limb, with launches that still fill
// the device.  In a single product, levels of many nodes keep 512-limb
// chunks up to 4096 limbs (measured faster for the 3-way bottom levels, with
// values of about 2500 limbs); `wide` is the log2 width from which 1024-limb
// chunks are taken.
int wide_from(int64_t nodes, bool single) { return single && nodes >= 64 ? 12 : 11; }
int lpt_for_step(int64_t Y, int wide) { return Y > ((int64_t)1 << wide) ? 16 : lpt_for(Y); }

// Recompositions likewise.
int lpt_for_recomp(int64_t Y, int wide) { return Y > ((int64_t)1 << wide) ? 16 : lpt_for(Y); }

// Descriptors of one launch, before layout.
struct PhaseDescs {
  int kind = 0;
  int lpt = 0;
  LeafShape leaf{};
  std::vector<StepDesc> steps;
  std::vector<EvalDesc> evals;
  std::vector<RecompDesc> recomps;
  std::vector<LeafDesc> leaves;
  int mleaf_n = 0;   // matrix-core leaves of this width
  std::vector<DPtr> flips;  // kFaultKind: limbs whose bit 0 is flipped
  std::vector<RStepDesc> rsteps;  // kRStepKind
  std::vector<NttDesc> ntts;      // kNttKind0 + kNtt*
};

// Launch kind of the fault-injection hook (not a kernel class of the cost
// accounting).
constexpr int kFaultKind = 100;
// Launch kind of the recomposing steps (timed and costed as TC_KERNEL_STEP).
constexpr int kRStepKind = 102;
// Launch kinds of the transform leaves, kNttKind0 + kNttColFwd .. kNttCarry
// (timed and costed as TC_KERNEL_LEAF).
constexpr int kNttKind0 = 110;
bool ntt_kind(int kind) { return kind >= kNttKind0 && kind <= kNttKind0 + kNttCarry; }

DPtr dptr(int buf, int64_t off) {
  DPtr d;
  d.off = off;
  d.buf = buf;
  d.pad = 0;
  return d;
}

DPtr dadd(DPtr d, int64_t bytes) {
  d.off += bytes;
  return d;
}

DPtr none_ptr() { return dptr(-1, 0); }

TermDesc term_none() {
  TermDesc t;
  std::memset(&t, 0, sizeof t);
  t.kind = TERM_NONE;
  t.su = t.sv = none_ptr();
  t.sidx = -1;
  return t;
}

TermDesc term_tc(DPtr p, int64_t stride, int64_t width, bool neg, int shl) {
  TermDesc t = term_none();
  t.kind = TERM_TC;
  t.ptr = p;
  t.stride = stride;
  t.width = (int32_t)width;
  t.neg = neg ? 1 : 0;
  t.shl = shl;
  return t;
}

TermDesc term_sm(DPtr p, int64_t stride, int64_t width, DPtr su, DPtr sv, int64_t sstride,
                 bool neg, int shl) {
  TermDesc t = term_none();
  t.kind = TERM_SM;
  t.ptr = p;
  t.stride = stride;
  t.width = (int32_t)width;
  t.su = su;
  t.sv = sv;
  t.sstride = sstride;
  t.svstride = (int32_t)sstride;
  t.neg = neg ? 1 : 0;
  t.shl = shl;
  return t;
}

// Phase ordering keys: stage, depth and round, then the engine width.
enum : int64_t { ST_EVAL = 0, ST_LEAF = 1, ST_UP = 2 };
using PhaseKey = std::pair<int64_t, int>;

PhaseKey key_eval(int depth, int lpt) { return {ST_EVAL * 1000000000LL + depth, lpt}; }
PhaseKey key_leaf(const LeafShape& s) { return {ST_LEAF * 1000000000LL + s.R * 1000 + s.tpl, 0}; }
// up-pass: deeper first; within a depth: combine, Newton rounds, monomial
// rounds, recomposition
PhaseKey key_up(int depth, int sub, int lpt) {
  return {ST_UP * 1000000000LL + (int64_t)(TC_MAX_LEVELS - depth) * 100000 + sub, lpt};
}
// interpolation launches: SUB_COMBINE + group; recomposing steps; recompositions
constexpr int SUB_COMBINE = 0, SUB_RSTEP = 99998, SUB_RECOMP = 99999;

struct Builder {
  Ctx* ctx;
  size_t scratch = 0;
  std::map<PhaseKey, PhaseDescs> phases;
  // the batch item whose descriptors are being generated, and the item count
  // (one error word each)
  int32_t item = 0;
  int64_t items = 1;
  // single-round levels interpolate and recompose in one recomposing step
  bool fuse_recomp = true;
  // the current plan's chunk scale (tc_plan::chunk): LPT times 2^chunk
  int chunk = 0;
  int lpt(int rule) const {
    int l = chunk >= 0 ? rule << chunk : rule >> -chunk;
    return l < 2 ? 2 : l > 16 ? 16 : l;
  }
  // tc_debug_fault: the item whose first Toom node gets a flipped product bit
  int fault_item = -1;
  bool fault_done = false;
  // one product (tc_mul, tc_mul_plan) rather than a batch: batches, which
  // serving runs on several streams at once, keep wider chunks (measured:
  // higher request throughput)
  bool single = true;
  int err = TC_OK;
  // algorithmic HBM bytes per kernel class: every phase reads its inputs once
  // and writes its outputs once (the plan's minimum, whatever the passes)
  double alg_bytes[TC_KERNEL_CLASSES] = {0, 0, 0, 0};

  // scratch ranges (bytes offset, 64-bit words) cleared before every run
  std::vector<std::pair<int64_t, int64_t>> zeros;

  int64_t alloc(size_t bytes) {
    const size_t o = align_up(scratch, 256);
    scratch = o + bytes;
    return (int64_t)o;
  }
  // Clears limbs [off, off + n) of scratch buffer p before every run, in
  // whole 64-bit words (the buffer must allow rounding out to 8 bytes).
  void zero(DPtr p, int64_t off, int64_t n) {
    const int64_t lo = (p.off + off * 4) & ~(int64_t)7;
    const int64_t hi = (p.off + (off + n) * 4 + 7) & ~(int64_t)7;
    zeros.push_back({lo, (hi - lo) / 8});
  }
  PhaseDescs& phase(PhaseKey k, int kind, int lpt) {
    auto it = phases.find(k);
    if (it != phases.end() && it->second.kind != kind) err = TC_ERR_UNSUPPORTED;  // keys never mix kinds
    PhaseDescs& p = phases[k];
    p.kind = kind;
    p.lpt = lpt;
    return p;
  }
  // Table id of the odd divisor d (1 < d < 2^32), adding it on first use.
  // Entries never move, so compiled plans keep valid ids.
  int div_for(uint32_t d) {
    std::lock_guard<std::mutex> lk(ctx->div_mu);
    auto it = ctx->div_id.find(d);
    if (it != ctx->div_id.end()) return it->second;
    if (ctx->div_n >= kMaxDivs) return -1;
    auto e = std::make_unique<DivEntry>();
    make_div(*e, d);
    const int id = ctx->div_n;
    if (ctx->d_div && upload(ctx, ctx->d_div + id, e.get(), sizeof(DivEntry)) != hipSuccess) {
      (void)hipGetLastError();  // the caller's thread keeps no error of ours
      return -1;
    }
    ctx->div_id[d] = id;
    ctx->div_n = id + 1;
    return id;
  }
  // (neg, shr, div ids) of dividing by a small signed integer delta
  bool divspec(int64_t delta, bool* neg, int* shr, int* d0, int* d1) {
    *neg = delta < 0;
    uint64_t a = delta < 0 ? (uint64_t)(-delta) : (uint64_t)delta;
    if (a == 0) return false;
    int s = 0;
    while (!(a & 1)) {
      a >>= 1;
      s++;
    }
    *shr = s;
    *d0 = *d1 = -1;
    if (a == 1) return true;
    if (a < (1ull << 32)) {
      *d0 = div_for((uint32_t)a);
      return *d0 >= 0;
    }
    for (int k = 16; k <= 31; k++) {
      if (a == (1ull << (2 * k)) - 1) {
        *d0 = div_for((uint32_t)((1ull << k) - 1));
        *d1 = div_for((uint32_t)((1ull << k) + 1));
        return *d0 >= 0 && *d1 >= 0;
      }
    }
    return false;
  }
};

using i128 = __int128;

i128 i128_gcd(i128 a, i128 b) {
  if (a < 0) a = -a;
  if (b < 0) b = -b;
  while (b != 0) {
    const i128 t = a % b;
    a = b;
    b = t;
  }
  return a;
}

// The inverse of the matrix whose row i gives the point value y_i of the
// half point set (0, 1, -1, 2, -2, 2^6 W(1/2), W(inf)) from w_0 .. w_6, as
// reduced fractions num/den (den > 0), by Gauss-Jordan elimination.
bool half_point_inverse(i128 num[7][7], i128 den[7][7]) {
  struct Q {
    i128 n, d;
  };
  auto mk = [](i128 n, i128 d) {
    if (d < 0) {
      n = -n;
      d = -d;
    }
    const i128 g = i128_gcd(n, d);
    if (g > 1) {
      n /= g;
      d /= g;
    }
    return Q{n, d};
  };
  Q a[7][14];
  const int64_t xs[5] = {0, 1, -1, 2, -2};
  for (int i = 0; i < 7; i++)
    for (int k = 0; k < 14; k++) a[i][k] = mk(k == i + 7 ? 1 : 0, 1);
  for (int i = 0; i < 5; i++) {
    i128 p = 1;
    for (int k = 0; k < 7; k++) {
      a[i][k] = mk(xs[i] == 0 ? (k == 0 ? 1 : 0) : p, 1);
      p *= xs[i];
    }
  }
  for (int k = 0; k < 7; k++) a[5][k] = mk((i128)1 << (6 - k), 1);
  for (int k = 0; k < 7; k++) a[6][k] = mk(k == 6 ? 1 : 0, 1);
  for (int col = 0; col < 7; col++) {
    int piv = col;
    while (piv < 7 && a[piv][col].n == 0) piv++;
    if (piv == 7) return false;
    for (int k = 0; k < 14; k++) std::swap(a[col][k], a[piv][k]);
    const Q pv = a[col][col];
    for (int k = 0; k < 14; k++) a[col][k] = mk(a[col][k].n * pv.d, a[col][k].d * pv.n);
    for (int i = 0; i < 7; i++) {
      if (i == col || a[i][col].n == 0) continue;
      const Q f = a[i][col];
      for (int k = 0; k < 14; k++) {
        const Q m = mk(f.n * a[col][k].n, f.d * a[col][k].d);
        a[i][k] = mk(a[i][k].n * m.d - m.n * a[i][k].d, a[i][k].d * m.d);
      }
    }
  }
  for (int i = 0; i < 7; i++)
    for (int k = 0; k < 7; k++) {
      num[i][k] = a[i][k + 7].n;
      den[i][k] = a[i][k + 7].d;
    }
  return true;
}

// Interpolation values are kept in Y = (product width) + kInterpHeadroom
// limbs of two's complement: two limbs above the largest intermediate
// (section 3's values fit the product width plus two limbs), two more for a
// merged step's value before its right shift of up to 63 bits.
constexpr int64_t kInterpHeadroom = 4;

// Layout of one Toom node's interpolation buffers: [poly][value][version][Y].
struct InterpLayout {
  DPtr base;
  int64_t node_stride;  // limbs
  int npoly, nvals;
  int64_t Y;
  DPtr slot(int poly, int val, int ver) const {
    return dadd(base, ((((int64_t)poly * nvals + val) * 2 + ver) * Y) * 4);
  }
};

// Odd primes (with multiplicity) packed into at most two words (w0, w1);
// false if they do not fit.
bool pack_odd_divisors(const std::map<uint32_t, int>& D, uint32_t* w0, uint32_t* w1) {
  std::vector<uint64_t> f;
  for (auto& kv : D)
    for (int i = 0; i < kv.second; i++) f.push_back(kv.first);
  std::sort(f.rbegin(), f.rend());
  uint64_t a = 1, c = 1;
  for (uint64_t x : f) {
    if (a * x < (1ull << 32) && (a <= c || c * x >= (1ull << 32))) a *= x;
    else if (c * x < (1ull << 32)) c *= x;
    else return false;
  }
  *w0 = (uint32_t)a;
  *w1 = (uint32_t)c;
  return true;
}

// A coefficient of a single-round interpolation as an exact combination of
// the point products: w_k = (sum_j a_j y_{point_j}) / (2^S D).
struct FusedCoef {
  std::vector<std::pair<int, __int128>> terms;  // (point index, weight a_j)
  int S = 0;
  std::map<uint32_t, int> D;  // odd primes -> exponents
};

// The interpolation of one level for `count` nodes: combine, Newton rounds,
// monomial rounds.  prod(k) is the term of point product k.  Returns, per
// coefficient k, the slot that holds w_k.
// emit(sub, step) receives every step with its round key (SUB_*).
// fused != nullptr: when the rounds compose into one launch (every
// coefficient still a combination of the point products), the coefficients
// go to *fused instead and nothing is emitted.
template <class ProdFn, class Emit>
bool gen_interp(Builder& b, int B, int var, int64_t count, const InterpLayout& L, ProdFn prod,
                Emit emit, std::vector<DPtr>* wslots, std::vector<FusedCoef>* fused = nullptr) {
  const int n = B - 1;
  const int64_t Y = L.Y;
  auto step = [&](DPtr out, const TermDesc& a, const TermDesc& bb, int shr, int d0, int d1) {
    StepDesc s;
    std::memset(&s, 0, sizeof s);
    s.out = out;
    s.out_stride = L.node_stride;
    s.count = count;
    s.Y = (int32_t)Y;
    s.item = b.item;
    s.shr = shr;
    s.div[0] = d0;
    s.div[1] = d1;
    s.nterms = 2;
    s.t[0] = a;
    s.t[1] = bb;
    for (int i = 2; i < kStepTerms; i++) s.t[i] = term_none();
    return s;
  };
  auto slot_term = [&](int poly, int val, int ver, bool neg, int shl) {
    return term_tc(L.slot(poly, val, ver), L.node_stride, Y, neg, shl);
  };
  // ---- the paper's rounds on exact rational values ----
  // Every value of the interpolation is kept as an exact rational combination
  // (sum_i a_i s_i) / (2^S D) of materialized sources s_i: the point products,
  // or slot versions written by earlier launches.  D is odd and kept as prime
  // powers.  The rounds of section 4 (even-odd combine) and section 3
  // (divided differences, Theorem 3.2's loop; Newton to monomial, Theorem
  // 3.3's loop) are applied to these combinations, each round updating its
  // values from the values before it.  A launch is emitted only when a value
  // would no longer fit one step: at most kStepTerms terms whose odd weights
  // sum below 2^30, a right shift below 64 bits, and an odd divisor that
  // splits into at most two words.  So several rounds share one pass over the
  // data, and the launch computes exactly what the rounds compute.
  using i128 = __int128;
  struct Src {
    bool prod;
    int k;           // point product k
    int p, v, ver;   // slot (polynomial, value, version)
  };
  struct Val {
    std::vector<std::pair<int, i128>> t;  // (source id, coefficient), non-zero
    int S = 0;
    std::map<uint32_t, int> D;  // odd prime -> exponent
    bool ident_of(int src) const {
      return t.size() == 1 && t[0].first == src && t[0].second == 1 && S == 0 && D.empty();
    }
  };
  std::vector<Src> srcs;
  auto ipow = [](i128 b, int e, i128* out) {
    i128 r = 1;
    for (int i = 0; i < e; i++)
      if (__builtin_mul_overflow(r, b, &r)) return false;
    *out = r;
    return true;
  };
  // odd a -> primes (a < 2^64; a >= 2^32 only as 4^k - 1 = (2^k-1)(2^k+1))
  auto factor_odd = [](uint64_t a, std::map<uint32_t, int>* out) {
    auto f32 = [&](uint64_t x) {
      for (uint64_t q = 3; q * q <= x && q < 65536; q += 2)
        while (x % q == 0) {
          (*out)[(uint32_t)q]++;
          x /= q;
        }
      if (x > 1) (*out)[(uint32_t)x]++;  // below 2^32 with no factor below 2^16: prime
    };
    if (a < (1ull << 32)) {
      f32(a);
      return true;
    }
    for (int k = 16; k <= 31; k++)
      if (a == (1ull << (2 * k)) - 1) {
        f32((1ull << k) - 1);
        f32((1ull << k) + 1);
        return true;
      }
    return false;
  };
  // odd primes (with multiplicity) into at most two words; false if not
  auto pack_divisors = pack_odd_divisors;
  auto reduce = [](Val* v) {
    std::vector<std::pair<int, i128>> t;
    for (auto& x : v->t)
      if (x.second != 0) t.push_back(x);
    v->t = t;
    if (v->t.empty()) {
      v->S = 0;
      v->D.clear();
      return;
    }
    auto all_div = [&](i128 q) {
      for (auto& x : v->t)
        if (x.second % q != 0) return false;
      return true;
    };
    while (v->S > 0 && all_div(2)) {
      for (auto& x : v->t) x.second /= 2;
      v->S--;
    }
    for (auto it = v->D.begin(); it != v->D.end();) {
      while (it->second > 0 && all_div((i128)it->first)) {
        for (auto& x : v->t) x.second /= (i128)it->first;
        it->second--;
      }
      if (it->second == 0) it = v->D.erase(it);
      else ++it;
    }
  };
  // out = (sum_j w_j V_j) / (2^s d), d odd (as primes)
  auto lin = [&](const std::vector<std::pair<const Val*, i128>>& parts, int s,
                 const std::map<uint32_t, int>& d, Val* out) {
    Val r;
    for (auto& pp : parts) {
      r.S = std::max(r.S, pp.first->S);
      for (auto& kv : pp.first->D) r.D[kv.first] = std::max(r.D[kv.first], kv.second);
    }
    std::map<int, i128> acc;
    for (auto& pp : parts) {
      i128 scale = 0;
      if (!ipow(2, r.S - pp.first->S, &scale)) return false;
      for (auto& kv : r.D) {
        auto it = pp.first->D.find(kv.first);
        const int e = kv.second - (it == pp.first->D.end() ? 0 : it->second);
        i128 f;
        if (!ipow((i128)kv.first, e, &f) || __builtin_mul_overflow(scale, f, &scale)) return false;
      }
      i128 ws;
      if (__builtin_mul_overflow(scale, pp.second, &ws)) return false;
      for (auto& x : pp.first->t) {
        i128 m, sum;
        if (__builtin_mul_overflow(ws, x.second, &m) ||
            __builtin_add_overflow(acc[x.first], m, &sum))
          return false;
        acc[x.first] = sum;
      }
    }
    for (auto& kv : acc) r.t.push_back(kv);
    r.S += s;
    for (auto& kv : d) r.D[kv.first] += kv.second;
    reduce(&r);
    *out = r;
    return true;
  };
  // can one step compute v?
  auto fits = [&](const Val& v) {
    if ((int)v.t.size() > kStepTerms || v.S > 63) return false;
    i128 odd_sum = 0;
    for (auto& x : v.t) {
      i128 a = x.second < 0 ? -x.second : x.second;
      int sh = 0;
      while (!(a & 1)) {
        a >>= 1;
        sh++;
      }
      if (sh > 200) return false;
      odd_sum += a;
      if (odd_sum >= ((i128)1 << 30)) return false;
    }
    uint32_t w0, w1;
    return pack_divisors(v.D, &w0, &w1);
  };

  // the interpolation nodes of each polynomial
  std::vector<std::vector<int64_t>> X;
  if (var == TC_VAR_INF) {
    X.push_back({0, 1, -1, 2});  // the cubic W(x) - w_4 x^4
  } else if (var == TC_VAR_HALF) {
    X.push_back(std::vector<int64_t>(7, 0));  // W itself, by the fixed-n inverse (no nodes)
  } else {
    std::vector<int64_t> x(n + 1);
    x[0] = 0;
    for (int m = 1; m <= n; m++) x[m] = (int64_t)1 << (2 * (m - 1));  // X = x^2 = 4^(m-1)
    X.push_back(x);
    X.push_back(x);
  }
  const int npoly = (int)X.size();
  const int deg = (int)X[0].size() - 1;
  const int nvals = var == TC_VAR_INF ? 5 : deg + 1;  // INF keeps w_4 as value 4
  std::vector<std::vector<int>> ver(npoly, std::vector<int>(nvals, 0));
  std::vector<std::vector<int>> src_of(npoly, std::vector<int>(nvals, -1));
  std::vector<std::vector<Val>> cur(npoly, std::vector<Val>(nvals));
  std::vector<std::vector<bool>> dirty(npoly, std::vector<bool>(nvals, false));
  int group = 0;

  auto prod_src = [&](int k) {
    srcs.push_back(Src{true, k, 0, 0, 0});
    Val v;
    v.t.push_back({(int)srcs.size() - 1, 1});
    return v;
  };
  // emits one launch writing every dirty value; they become sources
  auto materialize = [&](bool finals) {
    const int sub = SUB_COMBINE + group;
    bool any = false;
    for (int p = 0; p < npoly; p++)
      for (int i = 0; i < nvals; i++) {
        const Val& v = cur[p][i];
        const bool need = dirty[p][i] || (finals && (src_of[p][i] < 0 || !v.ident_of(src_of[p][i])));
        if (!need) continue;
        if (!finals && v.t.empty()) continue;  // a zero stays virtual until needed
        StepDesc st = step(L.slot(p, i, (ver[p][i] + 1) % 2), term_none(), term_none(), 0, -1, -1);
        int nt = 0;
        for (auto& x : v.t) {
          i128 a = x.second < 0 ? -x.second : x.second;
          int sh = 0;
          while (!(a & 1)) {
            a >>= 1;
            sh++;
          }
          const Src& sr = srcs[(size_t)x.first];
          TermDesc td = sr.prod ? prod(sr.k, x.second < 0, sh)
                                : slot_term(sr.p, sr.v, sr.ver, x.second < 0, sh);
          td.mul = (uint32_t)a;
          st.t[nt++] = td;
        }
        st.nterms = nt;
        st.shr = v.S;
        uint32_t w0 = 1, w1 = 1;
        if (!pack_divisors(v.D, &w0, &w1)) return false;
        st.div[0] = w0 > 1 ? b.div_for(w0) : -1;
        st.div[1] = w1 > 1 ? b.div_for(w1) : -1;
        if ((w0 > 1 && st.div[0] < 0) || (w1 > 1 && st.div[1] < 0)) return false;
        if (st.div[0] < 0 && st.div[1] >= 0) std::swap(st.div[0], st.div[1]);
        emit(sub, st);
        any = true;
        ver[p][i] = (ver[p][i] + 1) % 2;
        srcs.push_back(Src{false, 0, p, i, ver[p][i]});
        src_of[p][i] = (int)srcs.size() - 1;
        Val id;
        id.t.push_back({src_of[p][i], 1});
        cur[p][i] = id;
        dirty[p][i] = false;
      }
    if (any) group++;
    return true;
  };
  // applies one round: upd(p, i, cur) -> new value of (p, i) or false when
  // (p, i) is not updated; merges into the pending launch when it fits
  auto round = [&](auto upd) {
    for (int attempt = 0; attempt < 2; attempt++) {
      std::vector<std::vector<Val>> nxt = cur;
      std::vector<std::vector<bool>> nd = dirty;
      bool ok = true;
      for (int p = 0; p < npoly && ok; p++)
        for (int i = 0; i < nvals && ok; i++) {
          Val v;
          int r = upd(p, i, &v);
          if (r < 0) ok = false;   // arithmetic overflow
          if (r == 1) {
            nxt[p][i] = v;
            nd[p][i] = true;
          }
        }
      for (int p = 0; p < npoly && ok; p++)
        for (int i = 0; i < nvals && ok; i++)
          if (nd[p][i] && !fits(nxt[p][i])) ok = false;
      if (ok) {
        cur = nxt;
        dirty = nd;
        return true;
      }
      if (attempt == 1) return false;  // one round must fit one launch
      if (!materialize(false)) return false;
    }
    return false;
  };

  // ---- combine (section 4) ----
  if (var == TC_VAR_HALF) {
    // section 3's closing remark: for a fixed n, c = V^-1 y.  Each
    // coefficient is its row of the inverse of the 7 x 7 point matrix (exact
    // rationals) over a common denominator 2^S D, one exact step.
    i128 num[7][7], den[7][7];
    if (!half_point_inverse(num, den)) return false;
    std::vector<Val> y;
    for (int k = 0; k < 7; k++) y.push_back(prod_src(k));
    if (!round([&](int, int k, Val* out) {
          i128 D = 1;
          for (int i = 0; i < 7; i++) D = D / i128_gcd(D, den[k][i]) * den[k][i];
          std::vector<std::pair<const Val*, i128>> parts;
          for (int i = 0; i < 7; i++)
            if (num[k][i] != 0) parts.push_back({&y[i], num[k][i] * (D / den[k][i])});
          int S = 0;
          while (D % 2 == 0) {
            D /= 2;
            S++;
          }
          std::map<uint32_t, int> d;
          if (D >= ((i128)1 << 32) || !factor_odd((uint64_t)D, &d)) return -1;
          return lin(parts, S, d, out) ? 1 : -1;
        }))
      return false;
  } else if (var == TC_VAR_INF) {
    // w_4 = W(inf); the cubic W(x) - w_4 x^4 at x = 0, 1, -1, 2
    std::vector<Val> y;
    for (int k = 0; k < 5; k++) y.push_back(prod_src(k));
    const std::map<uint32_t, int> none;
    if (!round([&](int, int i, Val* out) {
          if (i == 0) return *out = y[0], 1;
          if (i == 4) return *out = y[4], 1;
          const i128 w = i == 3 ? 16 : 1;  // x^4 at x = 1, -1, 2
          return lin({{&y[i], 1}, {&y[4], -w}}, 0, none, out) ? 1 : -1;
        }))
      return false;
  } else {
    // W_e(4^j) = (W(2^j) + W(-2^j)) / 2 ; 4^j W_o(4^j) = 2^j (W(2^j) - W(-2^j)) / 2
    std::vector<Val> y;
    for (int k = 0; k < 2 * n + 1; k++) y.push_back(prod_src(k));
    const std::map<uint32_t, int> none;
    if (!round([&](int p, int i, Val* out) {
          if (i == 0) {
            if (p == 0) return *out = y[0], 1;
            return *out = Val(), 1;  // the odd polynomial's extra point X = 0 has value 0
          }
          const int j = i - 1;
          if (p == 0) return lin({{&y[2 * j + 1], 1}, {&y[2 * j + 2], 1}}, 1, none, out) ? 1 : -1;
          i128 pw = 0;
          if (!ipow(2, j, &pw)) return -1;
          return lin({{&y[2 * j + 1], pw}, {&y[2 * j + 2], -pw}}, 1, none, out) ? 1 : -1;
        }))
      return false;
  }
  // ---- divided differences (Theorem 3.2's loop): round k updates m = k..deg ----
  for (int k = 1; k <= deg && var != TC_VAR_HALF; k++) {
    if (!round([&](int p, int m, Val* out) {
          if (m < k || m > deg) return 0;
          const int64_t dl = X[p][m] - X[p][m - k];
          if (dl == 0) return -1;
          uint64_t a = dl < 0 ? (uint64_t)(-dl) : (uint64_t)dl;
          int sh = 0;
          while (!(a & 1)) {
            a >>= 1;
            sh++;
          }
          std::map<uint32_t, int> d;
          if (!factor_odd(a, &d)) return -1;
          const i128 sg = dl < 0 ? -1 : 1;
          return lin({{&cur[p][m], sg}, {&cur[p][m - 1], -sg}}, sh, d, out) ? 1 : -1;
        }))
      return false;
  }
  // ---- Newton to monomial (Theorem 3.3's loop): round m updates k = m..deg-1 ----
  for (int mm = deg - 1; mm >= 0 && var != TC_VAR_HALF; mm--) {
    bool any = false;
    for (int p = 0; p < npoly; p++) any = any || X[p][mm] != 0;
    if (!any) continue;
    if (!round([&](int p, int k, Val* out) {
          if (k < mm || k > deg - 1 || X[p][mm] == 0) return 0;
          const std::map<uint32_t, int> none;
          return lin({{&cur[p][k], 1}, {&cur[p][k + 1], -(i128)X[p][mm]}}, 0, none, out) ? 1 : -1;
        }))
      return false;
  }
  if (fused && group == 0) {
    // no value was materialized: every coefficient is still a combination of
    // the point products
    fused->assign(2 * B - 1, FusedCoef());
    for (int k = 0; k < 2 * B - 1; k++) {
      int p = 0, i = k;
      if (var == TC_VAR_EVENODD) {
        p = k % 2;
        i = k % 2 == 0 ? k / 2 : (k + 1) / 2;
      }
      const Val& v = cur[p][i];
      FusedCoef& fc = (*fused)[k];
      for (auto& x : v.t) {
        if (!srcs[(size_t)x.first].prod) return false;
        fc.terms.push_back({srcs[(size_t)x.first].k, x.second});
      }
      fc.S = v.S;
      fc.D = v.D;
    }
    return true;
  }
  if (!materialize(true)) return false;

  // ---- where each coefficient ended up ----
  wslots->assign(2 * B - 1, DPtr{});
  if (var == TC_VAR_INF || var == TC_VAR_HALF) {
    for (int k = 0; k < 2 * B - 1; k++) (*wslots)[k] = L.slot(0, k, ver[0][k]);
  } else {
    for (int k = 0; k <= n; k++) (*wslots)[2 * k] = L.slot(0, k, ver[0][k]);
    for (int k = 0; k < n; k++) (*wslots)[2 * k + 1] = L.slot(1, k + 1, ver[1][k + 1]);
  }
  return true;
}

EvalDesc eval_desc(DPtr src, int64_t src_stride, int64_t src_width, int64_t bl, DPtr out,
                   int64_t out_stride, DPtr sign, int64_t sign_stride, int64_t count, int64_t nout,
                   int B, int var, int k) {
  EvalDesc e;
  std::memset(&e, 0, sizeof e);
  e.src = src;
  e.src_stride = src_stride;
  e.src_width = src_width;
  e.bl = bl;
  e.out = out;
  e.out_stride = out_stride;
  e.sign = sign;
  e.sign_stride = sign_stride;
  e.count = count;
  e.nout = (int32_t)nout;
  e.B = B;
  e.copy_block = -1;
  if (k == 0) {
    e.copy_block = 0;
  } else if (var == TC_VAR_INF) {
    if (k == 1) e.j = 0, e.odd_neg = 0;
    else if (k == 2) e.j = 0, e.odd_neg = 1;
    else if (k == 3) e.j = 1, e.odd_neg = 0;
    else e.copy_block = B - 1;
  } else if (var == TC_VAR_HALF) {
    // 0, +1, -1, +2, -2, 2^3 U(1/2) = sum_t u_t 2^(3-t), infinity
    if (k <= 4) e.j = (k - 1) / 2, e.odd_neg = (k % 2 == 0) ? 1 : 0;
    else if (k == 5) e.j = 1, e.rev = 1;
    else e.copy_block = B - 1;
  } else {
    e.j = (k - 1) / 2;
    e.odd_neg = (k % 2 == 0) ? 1 : 0;
  }
  return e;
}

RecompDesc recomp_desc(const std::vector<DPtr>& w, int64_t w_stride, int64_t bl, int64_t wread,
                       DPtr out, int64_t out_stride, int64_t count, int64_t nstore) {
  RecompDesc r;
  std::memset(&r, 0, sizeof r);
  for (size_t k = 0; k < w.size(); k++) r.w[k] = w[k];
  r.nk = (int32_t)w.size();
  r.w_stride = w_stride;
  r.bl = bl;
  r.wread = (int32_t)wread;
  r.out = out;
  r.out_stride = out_stride;
  r.count = count;
  r.nstore = nstore;
  r.ncompute = std::max<int64_t>((int64_t)(w.size() - 1) * bl + wread, nstore);
  r.wlimbs = (int32_t)wread;
  return r;
}

// Leaves up to kLeafVmax limbs go to the vector kernel (grouped by shape),
// wider ones to the matrix-core kernel (grouped by width).
void add_leaf_desc(Builder& b, const LeafDesc& d) {
  if (d.n > kLeafVmax) {
    // one launch per 256-limb width class; each workgroup reads its own n
    // and the launch reserves the LDS of the widest
    PhaseDescs& ph =
        b.phase({ST_LEAF * 1000000000LL + 700000 + (d.n + 255) / 256, 0}, TC_KERNEL_LEAF, 0);
    ph.mleaf_n = std::max<int>(ph.mleaf_n, d.n);
    ph.leaves.push_back(d);
    return;
  }
  const LeafShape s = leaf_shape(d.n);
  PhaseDescs& ph = b.phase(key_leaf(s), TC_KERNEL_LEAF, 0);
  ph.leaf = s;
  ph.leaves.push_back(d);
}

// Transform leaves: P[i] = U[i] V[i] (count leaves of uw x vw limbs, pw
// product limbs) through the launches of tc_ntt.hip; sq: V is U.
bool add_ntt_leaves(Builder& b, DPtr U, DPtr V, DPtr P, int64_t ustride, int64_t vstride,
                    int64_t pstride, int64_t count, int64_t uw, int64_t vw, int64_t pw, bool sq) {
  int bits = 0, logN = 0;
  if (!ntt_choose(uw, vw, &bits, &logN)) return false;
  NttDesc d;
  std::memset(&d, 0, sizeof d);
  d.U = U;
  d.V = sq ? U : V;
  d.P = P;
  d.u_stride = ustride;
  d.v_stride = sq ? ustride : vstride;
  d.p_stride = pstride;
  d.count = count;
  d.u_width = (int32_t)uw;
  d.v_width = (int32_t)(sq ? uw : vw);
  d.p_width = (int32_t)pw;
  d.bits = bits;
  d.logC = std::min(logN, kNttLogRowMax);
  d.logR = logN - d.logC;
  d.square = sq ? 1 : 0;
  d.item = b.item;
  const int64_t N = (int64_t)1 << logN;
  d.ninv = field_pow((uint64_t)N, kFieldP - 2);
  d.ncoef = ntt_pieces(uw, bits) + ntt_pieces(d.v_width, bits) - 1;
  // the top coefficient reaches bit bits (ncoef - 1) + 64
  d.ncompute = std::max<int64_t>(pw, ((int64_t)bits * (d.ncoef - 1) + 64 + 31) / 32);
  d.X = dptr(BUF_SCRATCH, b.alloc((size_t)(count * (sq ? 1 : 2) * N) * 8));
  for (int which = kNttColFwd; which <= kNttCarry; which++) {
    if ((which == kNttColFwd || which == kNttColInv) && d.logR == 0) continue;
    if (which == kNttRowFwd && sq) continue;
    b.phase({ST_LEAF * 1000000000LL + 800000 + which, 0}, kNttKind0 + which, 0).ntts.push_back(d);
  }
  return true;
}

// The interpolation and recomposition of a level whose interpolation is one
// round, as one recomposing step per node (RStepDesc): with L = 2^S D the
// least common multiple of the coefficients' denominators,
//   L W = sum_k sum_j (a_kj L / (2^S_k D_k)) y_{point_kj} beta^(k bl),
// every term a point product shifted left by k bl limbs and by the power of
// two of its weight, then one exact division by L.  Returns false (nothing
// added) when the terms or L do not fit one step.
bool gen_rstep(Builder& b, int depth, int64_t nodes, DPtr out, int64_t pstride, int64_t nstore,
               DPtr cP, DPtr csu, DPtr csv, int64_t nc, int npts, bool vshared, int64_t bl,
               int wide, const std::vector<FusedCoef>& fc) {
  using i128 = __int128;
  int S = 0;
  std::map<uint32_t, int> D;
  for (const FusedCoef& f : fc) {
    S = std::max(S, f.S);
    for (auto& kv : f.D) D[kv.first] = std::max(D[kv.first], kv.second);
  }
  if (S >= 64) return false;
  uint32_t d0 = 1, d1 = 1;
  if (!pack_odd_divisors(D, &d0, &d1)) return false;
  RStepDesc r;
  std::memset(&r, 0, sizeof r);
  int nt = 0;
  i128 odd_sum = 0;
  for (int k = 0; k < (int)fc.size(); k++) {
    // this coefficient's weights times L / (2^S_k D_k)
    i128 scale = (i128)1 << (S - fc[(size_t)k].S);
    for (auto& kv : D) {
      auto it = fc[(size_t)k].D.find(kv.first);
      for (int e = kv.second - (it == fc[(size_t)k].D.end() ? 0 : it->second); e > 0; e--) {
        if (__builtin_mul_overflow(scale, (i128)kv.first, &scale)) return false;
      }
    }
    for (auto& t : fc[(size_t)k].terms) {
      i128 a;
      if (__builtin_mul_overflow(t.second, scale, &a) || a == 0) return false;
      const bool neg = a < 0;
      if (neg) a = -a;
      int tz = 0;
      while (!(a & 1)) {
        a >>= 1;
        tz++;
      }
      odd_sum += a;
      if (nt >= kRTerms || odd_sum >= ((i128)1 << 30)) return false;
      const int64_t shl = (int64_t)tz + 32 * (int64_t)k * bl;
      if (shl >= ((int64_t)1 << 29)) return false;
      const int q = (int)(shl >> 5), rr = (int)(shl & 31);
      const int kk = rr ? q : q - 1;
      TermC& c = r.c[nt++];
      c.off = cP.off + (int64_t)t.first * 2 * nc * 4;
      c.stride = (int64_t)npts * 2 * nc;
      c.width = (int32_t)(2 * nc);
      c.f = (neg ? 1u : 0u) | ((rr ? (uint32_t)(32 - rr) : 0u) << 3) | ((uint32_t)(kk + 1) << 8);
      c.mul = (uint32_t)a;
      c.buf = (int8_t)cP.buf;
      c.tc = 0;
      c.sidx = (int16_t)t.first;
    }
  }
  r.out = out;
  r.out_stride = pstride;
  r.count = nodes;
  r.item = b.item;
  r.nstore = (int32_t)nstore;
  r.Y = (int32_t)(nstore + 2);  // L W < 2^(32 nstore) L, L below 2^64
  r.shr = S;
  r.div[0] = d0 > 1 ? b.div_for(d0) : -1;
  r.div[1] = d1 > 1 ? b.div_for(d1) : -1;
  if ((d0 > 1 && r.div[0] < 0) || (d1 > 1 && r.div[1] < 0)) return false;
  if (r.div[0] < 0 && r.div[1] >= 0) std::swap(r.div[0], r.div[1]);
  r.nterms = nt;
  r.sgn_u_buf = csu.buf;
  r.sgn_u_off = csu.off;
  r.sgn_stride = npts;
  r.sgn_v_buf = csv.buf;
  r.sgn_v_off = csv.off;
  r.sgn_v_stride = vshared ? 0 : npts;
  r.nsgn = npts;
  // the widest chunks that still give the launch enough waves to fill the
  // device (each wave sums every point product its limbs meet)
  (void)wide;
  int lpt = 2;
  for (const int l : {16, 8, 4})
    if (nodes * ((r.Y + 64 * l - 1) / (64 * l)) >= 2048) {
      lpt = l;
      break;
    }
  lpt = b.lpt(lpt);
  // a key of its own: batch items whose level at this depth interpolates in
  // several rounds use the SUB_COMBINE keys for their steps
  b.phase(key_up(depth, SUB_RSTEP, lpt), kRStepKind, lpt).rsteps.push_back(r);
  // read the 2B-1 point products, write the node's product
  b.alg_bytes[TC_KERNEL_STEP] += 4.0 * (double)nodes * ((double)npts * 2 * nc + (double)nstore);
  return true;
}

// `nodes` products of one shape through the whole recursion: product i
// multiplies U + i*ustride (uw limbs) by V + i*vstride (vw limbs) into
// P + i*pstride (pw = uw + vw limbs); n = max(uw, vw).  Strides in limbs.
// U == V (same address, width and stride) makes every node a square: each
// level evaluates the operand once, and its children are squares again.
struct Root {
  int64_t nodes, n;
  DPtr U, V, P;
  int64_t uw, vw, pw, ustride, vstride, pstride;
};

bool gen_product(Builder& b, const Root& root, const tc_plan& P) {
  b.chunk = P.chunk;
  struct Lv {
    int64_t nodes, n;
    DPtr U, V, su, sv, P;
    int64_t uw, vw, pw, ustride, vstride, pstride;
  };
  const int L = P.levels;
  std::vector<Lv> lv(L + 1);
  lv[0].nodes = root.nodes;
  lv[0].n = root.n;
  lv[0].U = root.U;
  lv[0].V = root.V;
  lv[0].P = root.P;
  lv[0].uw = root.uw;
  lv[0].vw = root.vw;
  lv[0].pw = root.pw;
  lv[0].ustride = root.ustride;
  lv[0].vstride = root.vstride;
  lv[0].pstride = root.pstride;
  const bool sq = root.U.buf == root.V.buf && root.U.off == root.V.off && root.uw == root.vw &&
                  root.ustride == root.vstride;
  // Nodes that share one V (stride 0: the pieces of a cut product) over a
  // single level evaluate V once; their children's V values and signs are
  // then indexed by point only.
  const bool vshared = !sq && root.nodes > 1 && root.vstride == 0 && L == 1;
  for (int l = 0; l < L; l++) {
    const int B = P.B[l], var = P.variant[l], npts = 2 * B - 1;
    const int64_t bl = (lv[l].n + B - 1) / B;
    const int64_t nc = bl + growth_limbs(B, var);
    Lv& c = lv[l + 1];
    c.nodes = lv[l].nodes * npts;
    c.n = nc;
    const int64_t vnodes = vshared ? npts : c.nodes;
    c.U = dptr(BUF_SCRATCH, b.alloc((size_t)(c.nodes * nc) * 4));
    c.V = sq ? c.U : dptr(BUF_SCRATCH, b.alloc((size_t)(vnodes * nc) * 4));
    c.su = dptr(BUF_SCRATCH, b.alloc((size_t)c.nodes));
    c.sv = sq ? c.su : dptr(BUF_SCRATCH, b.alloc((size_t)vnodes));
    c.P = dptr(BUF_SCRATCH, b.alloc((size_t)(c.nodes * 2 * nc) * 4));
    c.uw = c.vw = nc;
    c.pw = 2 * nc;
    c.ustride = c.vstride = nc;
    c.pstride = 2 * nc;
  }
  // down: evaluations
  for (int l = 0; l < L; l++) {
    const int B = P.B[l], var = P.variant[l], npts = 2 * B - 1;
    const int64_t bl = (lv[l].n + B - 1) / B;
    const Lv& c = lv[l + 1];
    // read both operands, write 2B-1 values (magnitude + sign limb) of each
    // (of the one operand of a square)
    const int nops = sq ? 1 : 2;
    const double per_op = (double)npts * (c.n + 1);
    b.alg_bytes[TC_KERNEL_EVAL] += 4.0 * (double)lv[l].nodes * ((double)lv[l].uw + per_op);
    if (!sq)
      b.alg_bytes[TC_KERNEL_EVAL] +=
          4.0 * (vshared ? 1.0 : (double)lv[l].nodes) * ((double)lv[l].vw + per_op);
    const int lpt = b.lpt(lpt_for(c.n + 1));
    PhaseDescs& ph = b.phase(key_eval(l, lpt), TC_KERNEL_EVAL, lpt);
    for (int op = 0; op < nops; op++) {
      const DPtr src = op ? lv[l].V : lv[l].U;
      const int64_t sstride = op ? lv[l].vstride : lv[l].ustride;
      const int64_t swidth = op ? lv[l].vw : lv[l].uw;
      const DPtr out = op ? c.V : c.U;
      const DPtr sg = op ? c.sv : c.su;
      for (int k = 0; k < npts; k++) {
        const int64_t count = op && vshared ? 1 : lv[l].nodes;
        EvalDesc e = eval_desc(src, sstride, swidth, bl, dadd(out, (int64_t)k * c.n * 4),
                               npts * c.n, dadd(sg, k), npts, count, c.n, B, var, k);
        e.item = b.item;
        // +2^j and -2^j share their pass over the blocks (E + O and E - O)
        const bool plus = e.copy_block < 0 && e.odd_neg == 0 && k + 1 < npts &&
                          (var == TC_VAR_INF ? k == 1
                                             : var == TC_VAR_HALF ? (k == 1 || k == 3)
                                                                  : (k % 2 == 1));
        if (plus) {
          e.paired = 1;
          e.out2 = dadd(out, (int64_t)(k + 1) * c.n * 4);
          e.sign2 = dadd(sg, k + 1);
          k++;
        }
        ph.evals.push_back(e);
      }
    }
  }
  if (P.leaf == TC_LEAF_NTT) {
    const Lv& f = lv[L];
    if (!vshared) {
      if (!add_ntt_leaves(b, f.U, f.V, f.P, f.ustride, f.vstride, f.pstride, f.nodes, f.uw, f.vw,
                          f.pw, sq))
        return false;
    } else {
      // the nodes' k-th children all use the one evaluated V at k
      const int npts = 2 * P.B[0] - 1;
      for (int k = 0; k < npts; k++)
        if (!add_ntt_leaves(b, dadd(f.U, (int64_t)k * f.ustride * 4), dadd(f.V, (int64_t)k * f.n * 4),
                            dadd(f.P, (int64_t)k * f.pstride * 4), npts * f.ustride, 0,
                            npts * f.pstride, lv[0].nodes, f.uw, f.vw, f.pw, false))
          return false;
    }
  } else {
    const Lv& f = lv[L];
    if (f.n > kLeafMax) return false;
    LeafDesc d;
    std::memset(&d, 0, sizeof d);
    d.U = f.U;
    d.V = f.V;
    d.P = f.P;
    d.u_stride = f.ustride;
    d.v_stride = f.vstride;
    d.p_stride = f.pstride;
    d.count = f.nodes;
    d.n = (int32_t)f.n;
    d.u_width = (int32_t)f.uw;
    d.v_width = (int32_t)f.vw;
    d.p_width = (int32_t)f.pw;
    d.item = b.item;
    if (!vshared) {
      add_leaf_desc(b, d);
    } else {
      // one descriptor per point k: the nodes' k-th children, all with the
      // one evaluated V at k
      const int npts = 2 * P.B[0] - 1;
      d.count = lv[0].nodes;
      d.u_stride = npts * f.ustride;
      d.v_stride = 0;
      d.p_stride = npts * f.pstride;
      for (int k = 0; k < npts; k++) {
        LeafDesc e = d;
        e.U = dadd(f.U, (int64_t)k * f.ustride * 4);
        e.V = dadd(f.V, (int64_t)k * f.n * 4);
        e.P = dadd(f.P, (int64_t)k * f.pstride * 4);
        add_leaf_desc(b, e);
      }
    }
  }
  // test hook: one bit of the top node's product at the second point flips
  // between the level below and the top interpolation, which then cannot be
  // exact (the combine halves y(+x) + y(-x))
  if (L >= 1 && b.fault_item == b.item && !b.fault_done) {
    b.fault_done = true;
    const int64_t nc = lv[1].n;
    PhaseDescs& ph = b.phase({ST_UP * 1000000000LL + (int64_t)TC_MAX_LEVELS * 100000 - 1, 99},
                             kFaultKind, 0);
    ph.flips.push_back(dadd(lv[1].P, 1 * 2 * nc * 4));
  }
  // up: interpolation and recomposition
  for (int l = L - 1; l >= 0; l--) {
    const int B = P.B[l], var = P.variant[l], npts = 2 * B - 1;
    const int64_t bl = (lv[l].n + B - 1) / B;
    const Lv& c = lv[l + 1];
    const int64_t nc = c.n;
    InterpLayout IL;
    IL.npoly = var == TC_VAR_EVENODD ? 2 : 1;
    IL.nvals = var == TC_VAR_EVENODD ? B : 2 * B - 1;
    IL.Y = 2 * nc + kInterpHeadroom;
    IL.node_stride = (int64_t)IL.npoly * IL.nvals * 2 * IL.Y;
    IL.base = dptr(BUF_SCRATCH, 0);  // allocated below, unless the level is one recomposing step
    auto prod = [&](int k, bool neg, int shl) {
      TermDesc t = term_sm(dadd(c.P, (int64_t)k * 2 * nc * 4), (int64_t)npts * 2 * nc, 2 * nc,
                           dadd(c.su, k), dadd(c.sv, k), npts, neg, shl);
      t.sidx = (int16_t)k;
      if (vshared) t.svstride = 0;  // one V sign per point
      return t;
    };
    std::vector<DPtr> ws;
    const int wide = wide_from(lv[l].nodes, b.single);
    // a single-round interpolation and the recomposition: one recomposing step
    if (b.fuse_recomp) {
      std::vector<FusedCoef> fc;
      auto none = [](int, const StepDesc&) {};
      if (gen_interp(b, B, var, lv[l].nodes, IL, prod, none, &ws, &fc) && !fc.empty() &&
          gen_rstep(b, l, lv[l].nodes, lv[l].P, lv[l].pstride, lv[l].pw, c.P, c.su, c.sv, nc, npts,
                    vshared, bl, wide, fc))
        continue;
      ws.clear();
    }
    IL.base = dptr(BUF_SCRATCH, b.alloc((size_t)(lv[l].nodes * IL.node_stride) * 4));
    const int lpt = b.lpt(lpt_for_step(IL.Y, wide));
    auto emit = [&](int sub, const StepDesc& st) {
      b.phase(key_up(l, sub, lpt), TC_KERNEL_STEP, lpt).steps.push_back(st);
    };
    if (!gen_interp(b, B, var, lv[l].nodes, IL, prod, emit, &ws)) return false;
    const int64_t wread = std::min<int64_t>(2 * bl + 1, IL.Y);
    const int64_t nstore = lv[l].pw;
    // interpolation: read the 2B-1 point products, write 2B-1 coefficients;
    // recomposition: read the coefficients, write the node's product
    b.alg_bytes[TC_KERNEL_STEP] += 4.0 * (double)lv[l].nodes * npts * (double)(2 * nc + IL.Y);
    b.alg_bytes[TC_KERNEL_RECOMP] +=
        4.0 * (double)lv[l].nodes * ((double)npts * wread + (double)nstore);
    RecompDesc r = recomp_desc(ws, IL.node_stride, bl, wread, lv[l].P, lv[l].pstride,
                               lv[l].nodes, nstore);
    r.item = b.item;
    r.wlimbs = (int32_t)IL.Y;
    const int rlpt = b.lpt(lpt_for_recomp(r.ncompute, wide));
    b.phase(key_up(l, SUB_RECOMP, rlpt), TC_KERNEL_RECOMP, rlpt).recomps.push_back(r);
  }
  return true;
}

// One product; ub/vb/wb are the buffer ids of its operands and result.
bool gen_product(Builder& b, size_t nu, size_t nv, const tc_plan& P, int ub, int vb, int wb) {
  Root r;
  r.nodes = 1;
  r.n = (int64_t)std::max(nu, nv);
  r.U = dptr(ub, 0);
  r.V = dptr(vb, 0);
  r.P = dptr(wb, 0);
  r.uw = (int64_t)nu;
  r.vw = (int64_t)nv;
  r.pw = (int64_t)(nu + nv);
  r.ustride = r.vstride = r.pstride = 0;
  return gen_product(b, r, P);
}

// Unbalanced products (the longer operand at least twice the shorter) are
// cut into balanced ones: with a the longer operand, c the shorter one (s
// limbs) and a_i the s-limb pieces of a, a c = sum_i (a_i c) beta^(i s).
// Pieces of even index write disjoint, adjacent ranges of one buffer E,
// pieces of odd index of another, O, shifted down by s limbs, so the sum is
// one two-term recomposition E + O beta^s with carry.  The full pieces share
// their shape and run as one multi-node product; a shorter last piece is a
// product of its own (cut again if it is unbalanced).  Section 2's plans
// are for balanced operands; the paper's products are balanced.
constexpr int64_t kChunkRatio = 2;

// Cut when unbalanced; the final sum reads its two partial sums over
// nu + nv limbs, a 32-bit width, so longer products keep the zero blocks.
bool cut(int64_t nu, int64_t nv) {
  return std::max(nu, nv) >= kChunkRatio * std::min(nu, nv) && nu + nv < ((int64_t)1 << 31);
}

// Phases of the sums: after every level of every product, innermost first.
PhaseKey key_acc(int nest, int lpt) {
  return {ST_UP * 1000000000LL + (int64_t)(TC_MAX_LEVELS + 1) * 100000 + (1000 - nest), lpt};
}

bool gen_mul_default(Builder& b, DPtr u, int64_t nu, DPtr v, int64_t nv, DPtr w, int nest) {
  if (!cut(nu, nv)) {
    Root r;
    r.nodes = 1;
    r.n = std::max(nu, nv);
    r.U = u;
    r.V = v;
    r.P = w;
    r.uw = nu;
    r.vw = nv;
    r.pw = nu + nv;
    r.ustride = r.vstride = r.pstride = 0;
    return gen_product(b, r, default_plan(r.n));
  }
  if (nest >= 64) return false;  // lengths at least halve per nesting level
  if (nu < nv) {
    std::swap(u, v);
    std::swap(nu, nv);
  }
  const int64_t s = nv, T = nu + nv;
  const int64_t m = (nu + s - 1) / s;  // pieces, >= 2
  const int64_t r = nu - (m - 1) * s;  // last piece, 1..s limbs
  const int64_t full = r == s ? m : m - 1;
  const DPtr E = dptr(BUF_SCRATCH, b.alloc((size_t)(T + 2) * 4));
  const DPtr O = dptr(BUF_SCRATCH, b.alloc((size_t)(T + 2) * 4));
  // piece i's product goes to E + i s (even i) or O + (i - 1) s (odd i)
  auto dest = [&](int64_t i) {
    return i % 2 == 0 ? dadd(E, i * s * 4) : dadd(O, (i - 1) * s * 4);
  };
  const tc_plan P = default_plan(s);
  for (int par = 0; par < 2; par++) {
    const int64_t cnt = full > par ? (full - par + 1) / 2 : 0;
    if (cnt == 0) continue;
    Root R;
    R.nodes = cnt;
    R.n = s;
    R.U = dadd(u, par * s * 4);
    R.V = v;
    R.P = dest(par);
    R.uw = R.vw = s;
    R.pw = 2 * s;
    R.ustride = 2 * s;
    R.vstride = 0;
    R.pstride = 2 * s;
    if (!gen_product(b, R, P)) return false;
  }
  if (r < s && !gen_mul_default(b, dadd(u, (m - 1) * s * 4), r, v, s, dest(m - 1), nest + 1))
    return false;
  // the tails no piece writes: E beyond the last even piece, O beyond the
  // last odd one (O's top s limbs always)
  auto piece_end = [&](int64_t i) { return i * s + (i == m - 1 ? r : s) + s; };
  const int64_t ie = (m - 1) % 2 == 0 ? m - 1 : m - 2;
  const int64_t io = (m - 1) % 2 == 1 ? m - 1 : m - 2;
  const int64_t e_end = piece_end(ie), o_end = piece_end(io) - s;
  if (e_end < T) b.zero(E, e_end, T - e_end);
  if (o_end < T) b.zero(O, o_end, T - o_end);
  // E + O beta^s: both read over T limbs, T stored, the s limbs above T zero
  RecompDesc rd = recomp_desc({E, O}, 0, s, T, w, 0, 1, T);
  rd.item = b.item;
  b.alg_bytes[TC_KERNEL_RECOMP] += 4.0 * 3.0 * (double)T;
  const int lpt = b.lpt(lpt_for_recomp(rd.ncompute, wide_from(1, b.single)));
  b.phase(key_acc(nest, lpt), TC_KERNEL_RECOMP, lpt).recomps.push_back(rd);
  return true;
}

// Precomputes a step's term records for the kernel's straight-line prologue
// (StepDesc::c); fast = 0 keeps the kernel on the general path (per-item
// batch buffers, LDS terms, or product signs not in one per-node array).
void fill_fast(StepDesc& d) {
  d.fast = 0;
  d.nsgn = 0;
  d.sgn_u_buf = d.sgn_v_buf = -1;
  d.sgn_u_off = d.sgn_v_off = d.sgn_stride = 0;
  d.sgn_v_stride = 0;
  std::memset(d.c, 0, sizeof d.c);
  for (int i = 0; i < kStepTerms; i++) d.c[i].sidx = -1;
  auto plain = [](int buf) { return buf >= BUF_SCRATCH && buf < BUF_TABLE0; };
  if (d.nterms < 0 || d.nterms > kStepTerms || !plain(d.out.buf)) return;
  bool have_sgn = false;
  for (int i = 0; i < d.nterms; i++) {
    const TermDesc& t = d.t[i];
    TermC& c = d.c[i];
    if (t.kind == TERM_NONE || !plain(t.ptr.buf) || t.shl < 0 || t.shl >= (1 << 29)) return;
    const int q = t.shl >> 5, r = t.shl & 31;
    const int k = r ? q : q - 1;
    const uint32_t sh = r ? (uint32_t)(32 - r) : 0u;
    c.off = t.ptr.off;
    c.stride = t.stride;
    c.width = t.width;
    c.f = (t.neg ? 1u : 0u) | (sh << 3) | ((uint32_t)(k + 1) << 8);
    c.mul = t.mul > 1u ? t.mul : 1u;
    c.buf = (int8_t)t.ptr.buf;
    c.tc = t.kind == TERM_TC ? 1 : 0;
    c.sidx = -1;
    if (t.kind == TERM_SM) {
      if (t.sidx < 0 || t.sidx >= 64 || !plain(t.su.buf)) return;
      if (t.sv.buf >= 0 && !plain(t.sv.buf)) return;
      const int64_t uo = t.su.off - t.sidx;
      const int64_t vo = t.sv.buf >= 0 ? t.sv.off - t.sidx : 0;
      if (!have_sgn) {
        have_sgn = true;
        d.sgn_u_buf = t.su.buf;
        d.sgn_u_off = uo;
        d.sgn_v_buf = t.sv.buf >= 0 ? t.sv.buf : -1;
        d.sgn_v_off = vo;
        d.sgn_stride = t.sstride;
        d.sgn_v_stride = t.svstride;
      } else if (d.sgn_u_buf != t.su.buf || d.sgn_u_off != uo ||
                 d.sgn_v_buf != (t.sv.buf >= 0 ? t.sv.buf : -1) || d.sgn_v_off != vo ||
                 d.sgn_stride != t.sstride || d.sgn_v_stride != t.svstride) {
        return;
      }
      c.sidx = t.sidx;
      d.nsgn = std::max(d.nsgn, (int32_t)t.sidx + 1);
    }
  }
  d.fast = 1;
}

// Lays the phases out into one device blob and a launch list.  Values longer
// than one chunk (64*lpt limbs) get look-back words in the status region.
int finish(Builder& b, std::shared_ptr<Compiled>* out, bool to_device = true) {
  if (b.err != TC_OK) return b.err;
  auto cp = std::make_shared<Compiled>();
  for (int k = 0; k < TC_KERNEL_CLASSES; k++) cp->cost.bytes[k] = b.alg_bytes[k];
  std::vector<uint8_t> blob;
  int64_t status_words = 0;
  auto put = [&](const void* p, size_t bytes) {
    const size_t o = align_up(blob.size(), 64);
    blob.resize(o + bytes);
    if (bytes) std::memcpy(blob.data() + o, p, bytes);
    return o;
  };
  // chunking of one descriptor; returns its waves
  auto chunk = [&](auto& d, int64_t Y, int lpt) -> int64_t {
    const int64_t T = 64LL * lpt;
    d.nchunks = (int32_t)((Y + T - 1) / T);
    d.status_off = 0;
    if (d.nchunks > 1) {
      d.status_off = status_words;
      status_words += d.count * lb_words(d.nchunks);
    }
    return d.count * d.nchunks;
  };
  auto emit = [&](Launch L, const void* descs, size_t bytes, const std::vector<int64_t>& w0,
                  int64_t tot) {
    L.desc_off = put(descs, bytes);
    L.w0_off = put(w0.data(), w0.size() * sizeof(int64_t));
    L.nd = (int)w0.size();
    L.units = tot;
    L.per_desc = 0;
    if (!w0.empty() && tot % (int64_t)w0.size() == 0) {
      const int64_t u = tot / (int64_t)w0.size();
      bool same = u > 0 && u < ((int64_t)1 << 31);
      for (size_t i = 0; same && i < w0.size(); i++) same = w0[i] == (int64_t)i * u;
      if (same) L.per_desc = u;
    }
    if (L.nd > 0 && tot > 0) {
      cp->launches.push_back(L);
      cp->cost.launches[L.kind] += 1;
    }
  };
  for (auto& kv : b.phases) {
    PhaseDescs& ph = kv.second;
    Launch L;
    std::memset(&L, 0, sizeof L);
    L.kind = ph.kind;
    L.lpt = ph.lpt;
    L.leaf = ph.leaf;
    std::vector<int64_t> w0;
    int64_t tot = 0;
    if (ph.kind == TC_KERNEL_STEP) {
      for (auto& d : ph.steps) {
        // kernels pack a term's limb shift into 24 bits
        for (int i = 0; i < d.nterms; i++)
          if (d.t[i].shl < 0 || d.t[i].shl >= (1 << 29)) return TC_ERR_UNSUPPORTED;
        fill_fast(d);
        w0.push_back(tot);
        tot += chunk(d, d.Y, ph.lpt);
      }
      const size_t before = cp->launches.size();
      emit(L, ph.steps.data(), ph.steps.size() * sizeof(StepDesc), w0, tot);
      // equal shapes with long values or several nodes: the waves take
      // chunk position 0 of every value, then position 1, ..., and within a
      // position node by node over the outputs, so outputs that share terms
      // read them close together in time (measured: 95 -> 68 ms for the
      // 2^25-limb product, 1 % for the 2^19-limb one)
      bool same = !ph.steps.empty() && tot < ((int64_t)1 << 31);
      for (auto& d : ph.steps)
        same = same && d.count == ph.steps[0].count && d.nchunks == ph.steps[0].nchunks;
      same = same && (ph.steps[0].nchunks >= 128 || ph.steps[0].count >= 2);
      if (same && cp->launches.size() == before + 1) cp->launches.back().per_desc = -2;
    } else if (ph.kind == TC_KERNEL_EVAL) {
      std::vector<EvalDesc> multi;
      std::vector<int64_t> mw0;
      int64_t mtot = 0;
      for (auto& d : ph.evals) {
        w0.push_back(tot);
        tot += chunk(d, (int64_t)d.nout + 1, ph.lpt);
        d.status_off2 = 0;
        if (d.paired && d.nchunks > 1) {
          d.status_off2 = status_words;
          status_words += d.count * lb_words(d.nchunks);
        }
        if (d.nchunks > 1) {
          // the sign fix-up pass takes each value of a pair on its own
          EvalDesc a = d;
          a.paired = 0;
          multi.push_back(a);
          mw0.push_back(mtot);
          mtot += d.count * d.nchunks;
          if (d.paired) {
            EvalDesc b2 = a;
            b2.out = d.out2;
            b2.sign = d.sign2;
            b2.status_off = d.status_off2;
            multi.push_back(b2);
            mw0.push_back(mtot);
            mtot += d.count * d.nchunks;
          }
        }
      }
      const size_t before = cp->launches.size();
      emit(L, ph.evals.data(), ph.evals.size() * sizeof(EvalDesc), w0, tot);
      // the points of one operand read the same blocks: chunk position by
      // chunk position and node by node when values are long or nodes
      // several (as for steps)
      bool same = !ph.evals.empty() && tot < ((int64_t)1 << 31);
      for (auto& d : ph.evals)
        same = same && d.count == ph.evals[0].count && d.nchunks == ph.evals[0].nchunks;
      same = same && (ph.evals[0].nchunks >= 128 || ph.evals[0].count >= 2);
      if (same && cp->launches.size() == before + 1) cp->launches.back().per_desc = -2;
      if (!multi.empty()) {
        Launch N = L;
        N.neg_pass = 1;
        emit(N, multi.data(), multi.size() * sizeof(EvalDesc), mw0, mtot);
      }
    } else if (ph.kind == kRStepKind) {
      for (auto& d : ph.rsteps) {
        w0.push_back(tot);
        tot += chunk(d, d.Y, ph.lpt);
      }
      L.desc_off = put(ph.rsteps.data(), ph.rsteps.size() * sizeof(RStepDesc));
      L.w0_off = put(w0.data(), w0.size() * sizeof(int64_t));
      L.nd = (int)w0.size();
      L.units = tot;
      L.per_desc = 0;
      if (!w0.empty() && tot % (int64_t)w0.size() == 0) {
        const int64_t u = tot / (int64_t)w0.size();
        bool same = u > 0 && u < ((int64_t)1 << 31);
        for (size_t i = 0; same && i < w0.size(); i++) same = w0[i] == (int64_t)i * u;
        if (same) L.per_desc = u;
      }
      if (L.nd > 0 && tot > 0) {
        cp->launches.push_back(L);
        cp->cost.launches[TC_KERNEL_STEP] += 1;
      }
    } else if (ntt_kind(ph.kind)) {
      const int which = ph.kind - kNttKind0;
      size_t lds = 0;
      int lpt = 0;
      if (which == kNttCarry) {
        int64_t Y = 0;
        for (auto& d : ph.ntts) Y = std::max(Y, d.ncompute);
        lpt = std::min(lpt_for(Y), 8);  // the carry pass stages 512 limbs' coefficients at most
      }
      for (auto& d : ph.ntts) {
        const int logT = std::min(d.logC, kNttLogRowMax - d.logR);
        const size_t tile = (size_t)8 << (d.logR + logT), row = (size_t)8 << d.logC;
        int64_t units = 0;
        switch (which) {
          case kNttColFwd:
            units = (d.square ? 1 : 2) * (d.count << (d.logC - logT));
            lds = std::max(lds, tile);
            break;
          case kNttColInv:
            units = d.count << (d.logC - logT);
            lds = std::max(lds, tile);
            break;
          case kNttRowFwd:
          case kNttRowMul:
            units = d.count << d.logR;
            lds = std::max(lds, row);
            break;
          default:
            units = chunk(d, d.ncompute, lpt);
            // the leaves read their operands and write their products once
            cp->cost.bytes[TC_KERNEL_LEAF] +=
                (double)d.count * 4.0 * ((double)d.u_width + (d.square ? 0 : d.v_width) + d.p_width);
            break;
        }
        w0.push_back(tot);
        tot += units;
      }
      L.lpt = lpt;
      L.lds = lds;
      L.desc_off = put(ph.ntts.data(), ph.ntts.size() * sizeof(NttDesc));
      L.w0_off = put(w0.data(), w0.size() * sizeof(int64_t));
      L.nd = (int)w0.size();
      L.units = tot;
      L.per_desc = 0;
      if (L.nd > 0 && tot > 0) {
        cp->launches.push_back(L);
        cp->cost.launches[TC_KERNEL_LEAF] += 1;
      }
    } else if (ph.kind == kFaultKind) {
      L.desc_off = put(ph.flips.data(), ph.flips.size() * sizeof(DPtr));
      L.nd = (int)ph.flips.size();
      L.units = L.nd;
      cp->launches.push_back(L);
    } else if (ph.kind == TC_KERNEL_RECOMP) {
      for (auto& d : ph.recomps) {
        w0.push_back(tot);
        tot += chunk(d, d.ncompute, ph.lpt);
      }
      emit(L, ph.recomps.data(), ph.recomps.size() * sizeof(RecompDesc), w0, tot);
    } else if (ph.mleaf_n > 0) {
      for (auto& d : ph.leaves) {
        w0.push_back(tot);
        tot += d.count;
        cp->cost.bytes[TC_KERNEL_LEAF] +=
            (double)d.count * 4.0 * ((double)d.u_width + d.v_width + d.p_width);
        cp->cost.leaf_limb_products += (double)d.count * (double)d.n * d.n;
      }
      L.mleaf_n = ph.mleaf_n;
      emit(L, ph.leaves.data(), ph.leaves.size() * sizeof(LeafDesc), w0, tot);
    } else {
      const int lpw = 256 / ph.leaf.tpl;
      for (auto& d : ph.leaves) {
        w0.push_back(tot);
        tot += (d.count + lpw - 1) / lpw;
        cp->cost.bytes[TC_KERNEL_LEAF] +=
            (double)d.count * 4.0 * ((double)d.u_width + d.v_width + d.p_width);
        cp->cost.leaf_limb_products += (double)d.count * (double)d.n * d.n;
      }
      emit(L, ph.leaves.data(), ph.leaves.size() * sizeof(LeafDesc), w0, tot);
    }
  }
  cp->status_off = align_up(b.scratch, 256);
  cp->status_words = status_words;
  // per-item error words (cleared with the look-back words), then the
  // per-item status a batch reports
  cp->items = b.items;
  cp->item_err_off = cp->status_off + (size_t)status_words * 8;
  const int64_t err_words = (b.items + 1) / 2;
  cp->item_stat_off = cp->item_err_off + (size_t)err_words * 8;
  {
    std::vector<int64_t> fr;
    auto add = [&](int64_t off, int64_t words) {
      if (words <= 0) return;
      fr.push_back(off);
      fr.push_back(words);
      cp->fill_max = std::max(cp->fill_max, words);
    };
    add((int64_t)cp->status_off, status_words + err_words);
    for (const auto& z : b.zeros) add(z.first, z.second);
    cp->nfill = (int)(fr.size() / 2);
    if (cp->nfill > 0) cp->fill_off = put(fr.data(), fr.size() * sizeof(int64_t));
  }
  cp->scratch_bytes = cp->item_stat_off + (size_t)b.items * 4;
  if (to_device && !blob.empty()) {
    HIPCHK(hipMalloc(&cp->d_blob, blob.size()));
    HIPCHK(upload(b.ctx, cp->d_blob, blob.data(), blob.size()));
  }
  if (!to_device) cp->h_blob = std::move(blob);
  *out = cp;
  return TC_OK;
}

hipEvent_t pool_event(Ctx* c) {
  if (!c->event_pool.empty()) {
    hipEvent_t e = c->event_pool.back();
    c->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}

// Enqueues every launch of a compiled plan; `bases` is the instance's device
// copy of the base addresses, `scratch` its scratch buffer.
// `blob` is the device copy of the plan's descriptors (cp.d_blob, or the
// copy in the fixed workspace).
int launch_all(Ctx* c, const Compiled& cp, const uint8_t* blob, const Bases* bases,
               uint8_t* scratch, bool timed, hipStream_t st) {
  uint64_t* status = reinterpret_cast<uint64_t*>(scratch + cp.status_off);
  if (cp.nfill > 0) {
    const hipError_t e =
        launch_fill_ranges(scratch, reinterpret_cast<const int64_t*>(blob + cp.fill_off),
                           cp.nfill, cp.fill_max, st);
    if (e != hipSuccess) return hip_fail(e);
  }
  for (const Launch& L : cp.launches) {
    hipEvent_t ea = nullptr, eb = nullptr;
    const bool tl = timed && (L.kind < TC_KERNEL_CLASSES || L.kind == kRStepKind || ntt_kind(L.kind));
    if (tl) {
      ea = pool_event(c);
      eb = pool_event(c);
      HIPCHK(hipEventRecord(ea, st));
    }
    const uint8_t* d = blob + L.desc_off;
    const int64_t* w0 = reinterpret_cast<const int64_t*>(blob + L.w0_off);
    hipError_t e = hipSuccess;
    if (ntt_kind(L.kind)) {
      e = launch_ntt(L.kind - kNttKind0, reinterpret_cast<const NttDesc*>(d), w0, L.nd, L.units,
                     L.lpt, L.lds, bases, c->d_ntt, status, st);
      if (e != hipSuccess) return hip_fail(e);
      if (tl) {
        HIPCHK(hipEventRecord(eb, st));
        c->timed.push_back({TC_KERNEL_LEAF, ea, eb});
      }
      continue;
    }
    switch (L.kind) {
      case TC_KERNEL_STEP:
        e = launch_step(L.lpt, reinterpret_cast<const StepDesc*>(d), w0, L.nd, L.units, L.per_desc, bases,
                        c->d_div, status, st);
        break;
      case TC_KERNEL_EVAL:
        e = launch_eval(L.lpt, L.neg_pass != 0, reinterpret_cast<const EvalDesc*>(d), w0, L.nd,
                        L.units, L.per_desc, bases, status, st);
        break;
      case TC_KERNEL_RECOMP:
        e = launch_recomp(L.lpt, reinterpret_cast<const RecompDesc*>(d), w0, L.nd, L.units,
                          L.per_desc, bases, status, st);
        break;
      case kFaultKind:
        e = launch_flip(reinterpret_cast<const DPtr*>(d), L.nd, bases, st);
        break;
      case kRStepKind:
        e = launch_rstep(L.lpt, reinterpret_cast<const RStepDesc*>(d), w0, L.nd, L.units,
                         L.per_desc, bases, c->d_div, status, st);
        break;
      default:
        if (L.mleaf_n > 0)
          e = launch_mleaf(L.mleaf_n, reinterpret_cast<const LeafDesc*>(d), w0, L.nd, L.units,
                           bases, st);
        else
          e = launch_leaf(L.leaf, reinterpret_cast<const LeafDesc*>(d), w0, L.nd, L.units,
                          bases, st);
        break;
    }
    if (e != hipSuccess) return hip_fail(e);
    if (tl) {
      HIPCHK(hipEventRecord(eb, st));
      c->timed.push_back({L.kind == kRStepKind ? TC_KERNEL_STEP : L.kind, ea, eb});
    }
  }
  return TC_OK;
}

bool overlaps(const void* a, size_t an, const void* b, size_t bn) {
  const uint8_t* x = static_cast<const uint8_t*>(a);
  const uint8_t* y = static_cast<const uint8_t*>(b);
  return x < y + bn && y < x + an;
}

std::string plan_key(size_t nu, size_t nv, const tc_plan& p) {
  std::string k = std::to_string(nu) + "x" + std::to_string(nv) + ":";
  for (int i = 0; i < p.levels; i++)
    k += std::to_string(p.B[i]) +
         (p.variant[i] == TC_VAR_INF ? "i" : p.variant[i] == TC_VAR_HALF ? "h" : "e") + ",";
  if (p.leaf == TC_LEAF_NTT) k += "N";
  if (p.chunk) k += "c" + std::to_string(p.chunk);
  return k;
}

// Drops least-recently-used idle plans until the cached plans' device memory
// plus `incoming` fits the limit (caller holds c->mu).  Plans with work in
// flight are kept; a plan still referenced by a caller lives until released.
void evict_plans(Ctx* c, size_t incoming) {
  size_t total = incoming;
  std::vector<std::pair<uint64_t, std::string>> idle;  // (last use, key) of evictable plans
  for (auto& kv : c->cache) {
    const size_t b = kv.second->device_bytes();
    total += b;
    if (b > 0 && kv.second->idle()) idle.push_back({kv.second->last_use, kv.first});
  }
  (void)hipGetLastError();
  if (total <= c->cache_limit) return;
  std::sort(idle.begin(), idle.end());
  for (auto& v : idle) {
    if (total <= c->cache_limit) return;
    auto it = c->cache.find(v.second);
    total -= it->second->device_bytes();
    c->cache.erase(it);
  }
}

// Cache key of tc_mul's own choice for nu x nv: the plan of a balanced
// product, or the pieces' plans of an unbalanced one.
std::string default_key(int64_t nu, int64_t nv) {
  if (!cut(nu, nv)) return plan_key(nu, nv, default_plan(std::max(nu, nv)));
  const int64_t a = std::max(nu, nv), s = std::min(nu, nv);
  const int64_t r = a - (a + s - 1) / s * s + s;
  std::string k = "c" + std::to_string(nu) + "x" + std::to_string(nv) + "[" +
                  plan_key(s, s, default_plan(s));
  if (r < s) k += default_key(r, s);
  return k + "]";
}

// Plans compiled with the fault-injection hook, or in strict mode, are
// cached apart.
std::string fault_prefix(const Ctx* c) {
  std::string k = c->strict ? "X:" : "";
  if (c->fault_item >= 0) k += "F" + std::to_string(c->fault_item) + ":";
  return k;
}

// p == nullptr: tc_mul's own choice (chunked when unbalanced).  sq: u and v
// are the same operand (the plan reads it through u only).
int compile_single(Ctx* c, size_t nu, size_t nv, const tc_plan* p, bool sq,
                   std::shared_ptr<Compiled>* out) {
  const std::string key = fault_prefix(c) + std::string("s") + (sq ? "q" : "") +
                          (p ? plan_key(nu, nv, *p) : "d" + default_key(nu, nv));
  {
    std::lock_guard<std::mutex> lk(c->mu);
    auto it = c->cache.find(key);
    if (it != c->cache.end()) {
      *out = it->second;
      return TC_OK;
    }
  }
  Builder b;
  b.ctx = c;
  b.fault_item = c->fault_item;
  b.fuse_recomp = !c->strict;
  const int vb = sq ? BUF_U : BUF_V;
  const bool ok = p ? gen_product(b, nu, nv, *p, BUF_U, vb, BUF_W)
                    : gen_mul_default(b, dptr(BUF_U, 0), (int64_t)nu, dptr(vb, 0), (int64_t)nv,
                                      dptr(BUF_W, 0), 0);
  if (!ok) return TC_ERR_UNSUPPORTED;
  std::shared_ptr<Compiled> cp;
  const int rc = finish(b, &cp);
  if (rc != TC_OK) return rc;
  std::lock_guard<std::mutex> lk(c->mu);
  c->cache[key] = cp;
  *out = cp;
  return TC_OK;
}

int new_instance(const Compiled& cp, std::unique_ptr<Instance>* out) {
  auto I = std::make_unique<Instance>();
  HIPCHK(hipMalloc(&I->d_bases, sizeof(Bases)));
  HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&I->h_bases), sizeof(Bases), hipHostMallocDefault));
  if (cp.scratch_bytes) HIPCHK(hipMalloc(&I->scratch, cp.scratch_bytes));
  if (cp.table_n) {
    HIPCHK(hipMalloc(&I->d_table, cp.table_n * sizeof(void*)));
    HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&I->h_table), cp.table_n * sizeof(void*),
                         hipHostMallocDefault));
  }
  HIPCHK(hipEventCreateWithFlags(&I->done, hipEventDisableTiming));
  *out = std::move(I);
  return TC_OK;
}

// A free instance of cp (caller holds c->mu).
int acquire_instance(Ctx* c, Compiled& cp, Instance** out) {
  for (auto& i : cp.inst) {
    if (hipEventQuery(i->done) == hipSuccess) {
      *out = i.get();
      return TC_OK;
    }
  }
  (void)hipGetLastError();
  if (cp.inst.size() < kMaxInstances) {
    evict_plans(c, cp.scratch_bytes);
    std::unique_ptr<Instance> I;
    const int rc = new_instance(cp, &I);
    if (rc != TC_OK) return rc;
    cp.inst.push_back(std::move(I));
    *out = cp.inst.back().get();
    return TC_OK;
  }
  // all busy: wait for the one that was used first
  Instance* I = cp.inst.front().get();
  HIPCHK(hipEventSynchronize(I->done));
  std::rotate(cp.inst.begin(), cp.inst.begin() + 1, cp.inst.end());
  *out = I;
  return TC_OK;
}

int capture_graph(Ctx* c, const Compiled& cp, Instance& I) {
  if (!c->capture_stream) HIPCHK(hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking));
  HIPCHK(hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeThreadLocal));
  const int rc = launch_all(c, cp, cp.d_blob, I.d_bases, I.scratch, false, c->capture_stream);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(c->capture_stream, &g);
  if (rc != TC_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return hip_fail(e);
  const hipError_t e2 = hipGraphInstantiate(&I.exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e2 != hipSuccess) return hip_fail(e2);
  return TC_OK;
}

// Runs a compiled plan on `st` with the given operand/result addresses
// (p[0..2]) and, for batches, the per-item pointer table.  status == nullptr:
// exactness failures go to the device's sticky word; else each item's go to
// its own word, and status[i] (device or host memory) receives TC_OK or
// TC_ERR_INEXACT per item in stream order.
int execute(Ctx* c, Compiled& cp, const Bases& hb, void* const* table, hipStream_t st,
            int32_t* status = nullptr) {
  std::lock_guard<std::mutex> lk(c->mu);
  cp.last_use = ++c->use_clock;
  Instance* I = nullptr;
  int rc = acquire_instance(c, cp, &I);
  if (rc != TC_OK) return rc;
  *I->h_bases = hb;
  I->h_bases->scratch = I->scratch;
  I->h_bases->table = reinterpret_cast<uint8_t* const*>(I->d_table);
  if (status) {
    I->h_bases->err = reinterpret_cast<uint32_t*>(I->scratch + cp.item_err_off);
    I->h_bases->err_stride = 1;
  } else {
    I->h_bases->err = c->d_err;
    I->h_bases->err_stride = 0;
  }
  HIPCHK(hipMemcpyAsync(I->d_bases, I->h_bases, sizeof(Bases), hipMemcpyHostToDevice, st));
  if (cp.table_n) {
    std::memcpy(I->h_table, table, cp.table_n * sizeof(void*));
    HIPCHK(hipMemcpyAsync(I->d_table, I->h_table, cp.table_n * sizeof(void*),
                          hipMemcpyHostToDevice, st));
  }
  if (c->timing || !c->graphs) {
    rc = launch_all(c, cp, cp.d_blob, I->d_bases, I->scratch, c->timing, st);
  } else {
    if (!I->exec) rc = capture_graph(c, cp, *I);
    if (rc == TC_OK) {
      const hipError_t e = hipGraphLaunch(I->exec, st);
      if (e != hipSuccess) rc = hip_fail(e);
    }
  }
  if (rc == TC_OK && status) {
    // device memory and pinned host memory take the statuses straight from
    // the kernel; pageable host memory through a staged copy
    hipPointerAttribute_t pa;
    bool direct = false;
    int32_t* dp = nullptr;
    if (hipPointerGetAttributes(&pa, status) == hipSuccess) {
      // a kernel may write it only through a device address the runtime gave
      if (pa.type == hipMemoryTypeDevice || pa.type == hipMemoryTypeManaged) dp = status;
      else if (pa.type == hipMemoryTypeHost && pa.devicePointer)
        dp = static_cast<int32_t*>(pa.devicePointer);
      direct = dp != nullptr;
    }
    (void)hipGetLastError();
    const uint32_t* ie = reinterpret_cast<const uint32_t*>(I->scratch + cp.item_err_off);
    hipError_t e;
    if (direct) {
      e = launch_item_status(ie, dp, cp.items, TC_ERR_INEXACT, st);
    } else {
      int32_t* staged = reinterpret_cast<int32_t*>(I->scratch + cp.item_stat_off);
      e = launch_item_status(ie, staged, cp.items, TC_ERR_INEXACT, st);
      if (e == hipSuccess)
        e = hipMemcpyAsync(status, staged, (size_t)cp.items * 4, hipMemcpyDefault, st);
    }
    if (e != hipSuccess) rc = hip_fail(e);
  }
  const hipError_t e = hipEventRecord(I->done, st);
  if (rc == TC_OK && e != hipSuccess) rc = hip_fail(e);
  return rc;
}

// Single-phase entry points: compile, run once without a graph, wait.
int run_phase_blob(Ctx* c, Builder& b, const Bases& base_in, hipStream_t st) {
  std::shared_ptr<Compiled> cp;
  int rc = finish(b, &cp);
  if (rc != TC_OK) return rc;
  const bool g = c->graphs;
  c->graphs = false;
  rc = execute(c, *cp, base_in, nullptr, st);
  c->graphs = g;
  if (rc != TC_OK) return rc;
  HIPCHK(hipStreamSynchronize(st));
  return TC_OK;
}

}  // namespace

// ===================================================================== C ABI

extern "C" {

int tc_init(void) {
  Ctx* c;
  return get_ctx(&c);
}

const char* tc_hip_error_string(void) { return g_hip_err.c_str(); }

const char* tc_strerror(int code) {
  switch (code) {
    case TC_OK: return "ok";
    case TC_ERR_INVALID: return "invalid argument";
    case TC_ERR_NOMEM: return "out of memory";
    case TC_ERR_HIP: return "HIP runtime error";
    case TC_ERR_AGAIN: return "queue full, try again";
    case TC_ERR_NOT_READY: return "not ready";
    case TC_ERR_INEXACT: return "device exactness check failed";
    case TC_ERR_UNSUPPORTED: return "unsupported";
    case TC_ERR_WORKSPACE: return "product exceeds the fixed workspace";
    default: return "unknown error";
  }
}

int tc_plan_default(size_t nu, size_t nv, tc_plan* out) {
  if (!out || nu == 0 || nv == 0) return TC_ERR_INVALID;
  *out = default_plan((int64_t)std::max(nu, nv));
  return TC_OK;
}

namespace {
// plan == nullptr: tc_mul's own choice.
size_t workspace_bytes(size_t nu, size_t nv, const tc_plan* plan) {
  if (nu == 0 || nv == 0 || (plan && !plan_ok(*plan))) return 0;
  Ctx* c;
  if (get_plan_ctx(&c) != TC_OK) return 0;
  Builder b;
  b.ctx = c;
  const bool ok = plan ? gen_product(b, nu, nv, *plan, BUF_U, BUF_V, BUF_W)
                       : gen_mul_default(b, dptr(BUF_U, 0), (int64_t)nu, dptr(BUF_V, 0),
                                         (int64_t)nv, dptr(BUF_W, 0), 0);
  if (!ok) return 0;
  std::shared_ptr<Compiled> cp;
  if (finish(b, &cp, /*to_device=*/false) != TC_OK) return 0;
  return cp->scratch_bytes;
}

int mul_single(tc_limb* w, const tc_limb* u, size_t nu, const tc_limb* v, size_t nv,
               const tc_plan* plan, hipStream_t stream) {
  if (!w || !u || !v || nu == 0 || nv == 0 || (plan && !plan_ok(*plan))) return TC_ERR_INVALID;
  if (nu > ((size_t)1 << 31) || nv > ((size_t)1 << 31)) return TC_ERR_UNSUPPORTED;
  if (overlaps(w, (nu + nv) * 4, u, nu * 4) || overlaps(w, (nu + nv) * 4, v, nv * 4))
    return TC_ERR_INVALID;
  if (plan && !leaves_fit((int64_t)std::max(nu, nv), *plan)) return TC_ERR_UNSUPPORTED;
  Ctx* c;
  int rc = get_ctx(&c);
  if (rc != TC_OK) return rc;
  std::shared_ptr<Compiled> cp;
  rc = compile_single(c, nu, nv, plan, u == v && nu == nv, &cp);
  if (rc != TC_OK) return rc;
  Bases bases;
  bases.scratch = nullptr;
  bases.p[0] = (uint8_t*)u;
  bases.p[1] = (uint8_t*)v;
  bases.p[2] = (uint8_t*)w;
  bases.table = nullptr;
  return execute(c, *cp, bases, nullptr, stream);
}
}  // namespace

size_t tc_workspace_bytes_plan(size_t nu, size_t nv, const tc_plan* plan) {
  return plan ? workspace_bytes(nu, nv, plan) : 0;
}

size_t tc_workspace_bytes(size_t nu, size_t nv) { return workspace_bytes(nu, nv, nullptr); }

int tc_mul_plan(tc_limb* w, const tc_limb* u, size_t nu, const tc_limb* v, size_t nv,
                const tc_plan* plan, hipStream_t stream) {
  if (!plan) return TC_ERR_INVALID;
  return mul_single(w, u, nu, v, nv, plan, stream);
}

int tc_mul(tc_limb* w, const tc_limb* u, size_t nu, const tc_limb* v, size_t nv,
           hipStream_t stream) {
  return mul_single(w, u, nu, v, nv, nullptr, stream);
}

namespace {
// Item outputs must not overlap each other or any item's input: the output
// ranges, sorted by address, are checked pairwise in order, and every input
// range against the output ranges that start below its end.
bool batch_aliasing(const tc_mul_desc* d, size_t count) {
  std::vector<std::pair<uintptr_t, uintptr_t>> outs(count);  // [begin, end)
  for (size_t i = 0; i < count; i++) {
    const uintptr_t w = (uintptr_t)d[i].w;
    outs[i] = {w, w + (d[i].nu + d[i].nv) * 4};
  }
  std::sort(outs.begin(), outs.end());
  for (size_t i = 1; i < count; i++)
    if (outs[i].first < outs[i - 1].second) return true;
  auto hits = [&](uintptr_t lo, uintptr_t hi) {
    // the last output starting below hi is the only one that may reach lo:
    // outputs are disjoint and sorted, so their ends increase too
    auto it = std::lower_bound(outs.begin(), outs.end(), std::make_pair(hi, (uintptr_t)0));
    if (it == outs.begin()) return false;
    --it;
    return it->second > lo;
  };
  for (size_t i = 0; i < count; i++) {
    const uintptr_t u = (uintptr_t)d[i].u, v = (uintptr_t)d[i].v;
    if (hits(u, u + d[i].nu * 4) || hits(v, v + d[i].nv * 4)) return true;
  }
  return false;
}

int mul_batch(const tc_mul_desc* d, size_t count, const tc_plan* plans, int32_t* status,
              hipStream_t stream) {
  if (!d || count == 0 || count > ((size_t)1 << 24)) return TC_ERR_INVALID;
  std::vector<tc_plan> ps(count);
  std::string key = "b";
  for (size_t i = 0; i < count; i++) {
    const tc_mul_desc& x = d[i];
    if (!x.w || !x.u || !x.v || x.nu == 0 || x.nv == 0) return TC_ERR_INVALID;
    if (x.nu > ((size_t)1 << 31) || x.nv > ((size_t)1 << 31)) return TC_ERR_UNSUPPORTED;
    if (x.u == x.v && x.nu == x.nv) key += "q";
    if (!plans) {
      key += default_key((int64_t)x.nu, (int64_t)x.nv) + ";";
      continue;
    }
    ps[i] = plans[i];
    if (!plan_ok(ps[i])) return TC_ERR_INVALID;
    if (!leaves_fit((int64_t)std::max(x.nu, x.nv), ps[i])) return TC_ERR_UNSUPPORTED;
    key += plan_key(x.nu, x.nv, ps[i]) + ";";
  }
  if (batch_aliasing(d, count)) return TC_ERR_INVALID;
  Ctx* c;
  int rc = get_ctx(&c);
  if (rc != TC_OK) return rc;
  key = fault_prefix(c) + key;
  std::shared_ptr<Compiled> cp;
  {
    std::lock_guard<std::mutex> lk(c->mu);
    auto it = c->cache.find(key);
    if (it != c->cache.end()) cp = it->second;
  }
  if (!cp) {
    Builder b;
    b.ctx = c;
    b.single = false;
    b.items = (int64_t)count;
    b.fault_item = c->fault_item;
    b.fuse_recomp = !c->strict;
    for (size_t i = 0; i < count; i++) {
      const int base = BUF_TABLE0 + 3 * (int)i;
      b.item = (int32_t)i;
      // a square reads its operand through the u entry only
      const int vb = d[i].u == d[i].v && d[i].nu == d[i].nv ? base : base + 1;
      const bool ok = plans ? gen_product(b, d[i].nu, d[i].nv, ps[i], base, vb, base + 2)
                            : gen_mul_default(b, dptr(base, 0), (int64_t)d[i].nu, dptr(vb, 0),
                                              (int64_t)d[i].nv, dptr(base + 2, 0), 0);
      if (!ok) return TC_ERR_UNSUPPORTED;
    }
    rc = finish(b, &cp);
    if (rc != TC_OK) return rc;
    cp->table_n = 3 * count;
    std::lock_guard<std::mutex> lk(c->mu);
    c->cache[key] = cp;
  }
  // per-call pointer table, copied to the instance before the run
  std::vector<void*> table(count * 3);
  for (size_t i = 0; i < count; i++) {
    table[3 * i] = (void*)d[i].u;
    table[3 * i + 1] = (void*)d[i].v;
    table[3 * i + 2] = (void*)d[i].w;
  }
  Bases bases;
  std::memset(&bases, 0, sizeof bases);
  return execute(c, *cp, bases, table.data(), stream, status);
}
}  // namespace

int tc_mul_batch(const tc_mul_desc* d, size_t count, int32_t* status_or_null, hipStream_t stream) {
  return mul_batch(d, count, nullptr, status_or_null, stream);
}

int tc_mul_batch_plan(const tc_mul_desc* d, size_t count, const tc_plan* plans,
                      int32_t* status_or_null, hipStream_t stream) {
  if (!plans) return TC_ERR_INVALID;
  return mul_batch(d, count, plans, status_or_null, stream);
}

int tc_get_error(void) {
  Ctx* c;
  int rc = get_ctx(&c);
  if (rc != TC_OK) return rc;
  // one atomic exchange on the device takes the word and clears it, so no
  // error set meanwhile by work on other streams is lost
  std::lock_guard<std::mutex> lk(c->err_mu);
  *c->h_err = 0;
  const hipError_t e = launch_take_error(c->d_err, c->h_err, c->err_stream);
  if (e != hipSuccess) return hip_fail(e);
  HIPCHK(hipStreamSynchronize(c->err_stream));
  return *c->h_err ? TC_ERR_INEXACT : TC_OK;
}

int tc_sync(hipStream_t stream) {
  HIPCHK(hipStreamSynchronize(stream));
  return tc_get_error();
}

int tc_eval(tc_limb* out, uint8_t* sign, const tc_limb* u, size_t nu, int B, int variant,
            size_t bl, size_t nout, hipStream_t stream) {
  tc_plan p;
  std::memset(&p, 0, sizeof p);
  p.levels = 1;
  p.B[0] = B;
  p.variant[0] = variant;
  if (!out || !sign || !u || nu == 0 || bl == 0 || nout == 0 || !plan_ok(p)) return TC_ERR_INVALID;
  Ctx* c;
  int rc = get_ctx(&c);
  if (rc != TC_OK) return rc;
  Builder b;
  b.ctx = c;
  const int npts = 2 * B - 1;
  const int lpt = lpt_for((int64_t)nout + 1);
  PhaseDescs& ph = b.phase(key_eval(0, lpt), TC_KERNEL_EVAL, lpt);
  for (int k = 0; k < npts; k++)
    ph.evals.push_back(eval_desc(dptr(BUF_U, 0), 0, (int64_t)nu, (int64_t)bl,
                                 dptr(BUF_V, (int64_t)k * nout * 4), 0, dptr(BUF_W, k), 0, 1,
                                 (int64_t)nout, B, variant, k));
  Bases bases;
  bases.scratch = nullptr;
  bases.p[0] = (uint8_t*)u;
  bases.p[1] = (uint8_t*)out;
  bases.p[2] = sign;
  bases.table = nullptr;
  return run_phase_blob(c, b, bases, stream);
}

int tc_interp(tc_limb* w, size_t nw, const tc_limb* y, const uint8_t* sign, size_t ny, int B,
              int variant, hipStream_t stream) {
  tc_plan p;
  std::memset(&p, 0, sizeof p);
  p.levels = 1;
  p.B[0] = B;
  p.variant[0] = variant;
  if (!w || !y || !sign || nw == 0 || ny == 0 || !plan_ok(p)) return TC_ERR_INVALID;
  Ctx* c;
  int rc = get_ctx(&c);
  if (rc != TC_OK) return rc;
  Builder b;
  b.ctx = c;
  const int npts = 2 * B - 1;
  InterpLayout IL;
  IL.npoly = variant == TC_VAR_EVENODD ? 2 : 1;
  IL.nvals = variant == TC_VAR_EVENODD ? B : 2 * B - 1;
  IL.Y = (int64_t)ny + kInterpHeadroom;
  IL.node_stride = (int64_t)IL.npoly * IL.nvals * 2 * IL.Y;
  IL.base = dptr(BUF_SCRATCH, b.alloc((size_t)IL.node_stride * 4));
  auto prod = [&](int k, bool neg, int shl) {
    TermDesc t = term_sm(dptr(BUF_U, (int64_t)k * ny * 4), 0, (int64_t)ny, dptr(BUF_V, k),
                         none_ptr(), 0, neg, shl);
    t.sidx = (int16_t)k;
    return t;
  };
  std::vector<DPtr> ws;
  const int ilpt = lpt_for_step(IL.Y, wide_from(1, true));
  auto emit = [&](int sub, const StepDesc& st) {
    b.phase(key_up(0, sub, ilpt), TC_KERNEL_STEP, ilpt).steps.push_back(st);
  };
  if (!gen_interp(b, B, variant, 1, IL, prod, emit, &ws)) return TC_ERR_UNSUPPORTED;
  // copy the coefficients out (nw limbs each)
  const int lpt = lpt_for((int64_t)nw);
  PhaseDescs& ph = b.phase(key_up(0, SUB_RECOMP, lpt), TC_KERNEL_STEP, lpt);
  for (int k = 0; k < npts; k++) {
    StepDesc s;
    std::memset(&s, 0, sizeof s);
    s.out = dptr(BUF_W, (int64_t)k * nw * 4);
    s.count = 1;
    s.Y = (int32_t)nw;
    s.div[0] = s.div[1] = -1;
    s.nterms = 1;
    s.t[0] = term_tc(ws[k], 0, IL.Y, false, 0);
    for (int i = 1; i < kStepTerms; i++) s.t[i] = term_none();
    ph.steps.push_back(s);
  }
  Bases bases;
  bases.scratch = nullptr;
  bases.p[0] = (uint8_t*)y;
  bases.p[1] = (uint8_t*)sign;
  bases.p[2] = (uint8_t*)w;
  bases.table = nullptr;
  return run_phase_blob(c, b, bases, stream);
}

int tc_recompose(tc_limb* out, size_t nout, const tc_limb* w, size_t nw, int B, size_t bl,
                 hipStream_t stream) {
  if (!out || !w || nout == 0 || nw == 0 || bl == 0 || B < 2 || B > kMaxB) return TC_ERR_INVALID;
  Ctx* c;
  int rc = get_ctx(&c);
  if (rc != TC_OK) return rc;
  Builder b;
  b.ctx = c;
  std::vector<DPtr> ws;
  for (int k = 0; k < 2 * B - 1; k++) ws.push_back(dptr(BUF_U, (int64_t)k * nw * 4));
  RecompDesc r = recomp_desc(ws, 0, (int64_t)bl, (int64_t)nw, dptr(BUF_W, 0), 0, 1, (int64_t)nout);
  const int lpt = lpt_for_recomp(r.ncompute, wide_from(1, true));
  b.phase(key_up(0, SUB_RECOMP, lpt), TC_KERNEL_RECOMP, lpt).recomps.push_back(r);
  Bases bases;
  bases.scratch = nullptr;
  bases.p[0] = (uint8_t*)w;
  bases.p[1] = nullptr;
  bases.p[2] = (uint8_t*)out;
  bases.table = nullptr;
  return run_phase_blob(c, b, bases, stream);
}

int tc_school(tc_limb* p, const tc_limb* u, const tc_limb* v, size_t n, size_t count,
              hipStream_t stream) {
  if (!p || !u || !v || n == 0 || count == 0) return TC_ERR_INVALID;
  if (n > (size_t)kLeafMax) return TC_ERR_UNSUPPORTED;
  Ctx* c;
  int rc = get_ctx(&c);
  if (rc != TC_OK) return rc;
  Builder b;
  b.ctx = c;
  LeafDesc d;
  std::memset(&d, 0, sizeof d);
  d.U = dptr(BUF_U, 0);
  d.V = dptr(BUF_V, 0);
  d.P = dptr(BUF_W, 0);
  d.u_stride = d.v_stride = (int64_t)n;
  d.p_stride = 2 * (int64_t)n;
  d.count = (int64_t)count;
  d.n = d.u_width = d.v_width = (int32_t)n;
  d.p_width = 2 * (int32_t)n;
  add_leaf_desc(b, d);
  Bases bases;
  bases.scratch = nullptr;
  bases.p[0] = (uint8_t*)u;
  bases.p[1] = (uint8_t*)v;
  bases.p[2] = (uint8_t*)p;
  bases.table = nullptr;
  return run_phase_blob(c, b, bases, stream);
}

int tc_measure_mad_rate(double* per_s) {
  if (!per_s) return TC_ERR_INVALID;
  Ctx* c;
  int rc = get_ctx(&c);
  if (rc != TC_OK) return rc;
  const hipError_t e = measure_mad_rate(per_s);
  return e == hipSuccess ? TC_OK : hip_fail(e);
}

int tc_ntt_params(size_t na, size_t nb, int* bits, size_t* N, size_t* C) {
  if (na == 0 || nb == 0) return TC_ERR_INVALID;
  if (na > ((size_t)1 << 31) || nb > ((size_t)1 << 31)) return TC_ERR_UNSUPPORTED;
  int w = 0, logN = 0;
  if (!ntt_choose((int64_t)na, (int64_t)nb, &w, &logN)) return TC_ERR_UNSUPPORTED;
  if (bits) *bits = w;
  if (N) *N = (size_t)1 << logN;
  if (C) *C = (size_t)1 << std::min(logN, kNttLogRowMax);
  return TC_OK;
}

int tc_ntt_forward(uint64_t* X, const tc_limb* u, size_t nu, int bits, size_t N,
                   hipStream_t stream) {
  if (!X || !u || nu == 0 || bits < 16 || bits > 30 || N < 64 || N > ((size_t)1 << 24) ||
      (N & (N - 1)) || nu > ((size_t)1 << 31) || (size_t)ntt_pieces((int64_t)nu, bits) > N)
    return TC_ERR_INVALID;
  Ctx* c;
  int rc = get_ctx(&c);
  if (rc != TC_OK) return rc;
  Builder b;
  b.ctx = c;
  int logN = 0;
  while (((size_t)1 << logN) < N) logN++;
  NttDesc d;
  std::memset(&d, 0, sizeof d);
  d.U = d.V = dptr(BUF_U, 0);
  d.P = dptr(BUF_W, 0);
  d.count = 1;
  d.u_width = d.v_width = (int32_t)nu;
  d.bits = bits;
  d.logC = std::min(logN, kNttLogRowMax);
  d.logR = logN - d.logC;
  d.square = 1;  // one array: the U transform, in the caller's X
  d.X = dptr(BUF_W, 0);
  if (d.logR > 0)
    b.phase({ST_LEAF * 1000000000LL + 800000 + kNttColFwd, 0}, kNttKind0 + kNttColFwd, 0).ntts.push_back(d);
  b.phase({ST_LEAF * 1000000000LL + 800000 + kNttRowFwd, 0}, kNttKind0 + kNttRowFwd, 0).ntts.push_back(d);
  Bases bases;
  std::memset(&bases, 0, sizeof bases);
  bases.p[0] = (uint8_t*)u;
  bases.p[2] = (uint8_t*)X;
  return run_phase_blob(c, b, bases, stream);
}

int tc_plan_cost_get(size_t nu, size_t nv, const tc_plan* plan, tc_plan_cost* out) {
  if (!out || (plan && !plan_ok(*plan)) || nu == 0 || nv == 0) return TC_ERR_INVALID;
  if (plan && !leaves_fit((int64_t)std::max(nu, nv), *plan)) return TC_ERR_UNSUPPORTED;
  Ctx* c;
  int rc = get_plan_ctx(&c);
  if (rc != TC_OK) return rc;
  Builder b;
  b.ctx = c;
  const bool ok = plan ? gen_product(b, nu, nv, *plan, BUF_U, BUF_V, BUF_W)
                       : gen_mul_default(b, dptr(BUF_U, 0), (int64_t)nu, dptr(BUF_V, 0),
                                         (int64_t)nv, dptr(BUF_W, 0), 0);
  if (!ok) return TC_ERR_UNSUPPORTED;
  std::shared_ptr<Compiled> cp;
  rc = finish(b, &cp, /*to_device=*/false);
  if (rc != TC_OK) return rc;
  *out = cp->cost;
  return TC_OK;
}

int tc_autotune(size_t nu, size_t nv, int flags, tc_plan* best, double* best_ms) {
  if (nu == 0 || nv == 0 || flags != 0) return TC_ERR_INVALID;
  if (nu > ((size_t)1 << 31) || nv > ((size_t)1 << 31)) return TC_ERR_UNSUPPORTED;
  const int64_t n = (int64_t)std::max(nu, nv);
  // candidates: no level (one leaf), or a first split B1 followed by 3- or
  // 16-way levels down to a vector-ALU (512) or matrix-core (2048) leaf
  std::vector<tc_plan> cands;
  auto same = [](const tc_plan& a, const tc_plan& b) {
    if (a.levels != b.levels) return false;
    for (int i = 0; i < a.levels; i++)
      if (a.B[i] != b.B[i] || a.variant[i] != b.variant[i]) return false;
    return true;
  };
  auto add = [&](const tc_plan& p) {
    for (auto& q : cands)
      if (same(p, q)) return;
    cands.push_back(p);
  };
  for (const int64_t leafmax : {kLeafVmax, kLeafMax}) {
    if (n <= leafmax) {
      tc_plan p;
      std::memset(&p, 0, sizeof p);
      add(p);
      continue;
    }
    for (const int B1 : {2, 3, 4, -4, 8, 16, 32}) {
      // -4: Toom-4 on 0, +-1, +-2, 1/2, infinity
      const int var1 = B1 < 0 ? TC_VAR_HALF : TC_VAR_EVENODD;
      const int b1 = B1 < 0 ? -B1 : B1;
      if (!split_ok(n, b1, var1)) continue;
      for (const int lower : {3, 16}) {
        tc_plan p;
        std::memset(&p, 0, sizeof p);
        p.B[0] = b1;
        p.variant[0] = var1;
        p.levels = 1;
        int64_t w = (n + b1 - 1) / b1 + growth_limbs(b1, var1);
        bool ok = true;
        while (w > leafmax) {
          int B = lower;
          if (!split_ok(w, B, TC_VAR_EVENODD)) B = 3;
          if (p.levels >= TC_MAX_LEVELS || !split_ok(w, B, TC_VAR_EVENODD)) {
            ok = false;
            break;
          }
          p.B[p.levels++] = B;
          w = (w + B - 1) / B + growth_limbs(B, TC_VAR_EVENODD);
        }
        if (ok) add(p);
      }
    }
  }
  Ctx* c;
  int rc = get_ctx(&c);
  if (rc != TC_OK) return rc;
  size_t fr = 0, tot = 0;
  HIPCHK(hipMemGetInfo(&fr, &tot));
  // operands: a fixed pseudo-random pattern (the timing does not depend on it)
  tc_limb *du = nullptr, *dv = nullptr, *dw = nullptr;
  hipStream_t st = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto cleanup = [&]() {
    if (st) (void)hipStreamSynchronize(st);
    if (du) (void)hipFree(du);
    if (dv) (void)hipFree(dv);
    if (dw) (void)hipFree(dw);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st) (void)hipStreamDestroy(st);
  };
  {
    std::vector<tc_limb> h(std::max(nu, nv));
    uint64_t x = 0x9e3779b97f4a7c15ull;
    for (auto& l : h) {
      x = x * 6364136223846793005ull + 1442695040888963407ull;
      l = (tc_limb)(x >> 32);
    }
    if (hipMalloc(&du, nu * 4) != hipSuccess || hipMalloc(&dv, nv * 4) != hipSuccess ||
        hipMalloc(&dw, (nu + nv) * 4) != hipSuccess ||
        hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess ||
        hipMemcpyAsync(du, h.data(), nu * 4, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(dv, h.data(), nv * 4, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
      cleanup();
      return TC_ERR_NOMEM;
    }
  }
  double best_t = 1e300;
  tc_plan best_p{};
  // each candidate runs as a batch of one: tuned plans serve batches (and
  // the serving loop) as much as single products, and batches take the
  // wider chunks
  auto run = [&](const tc_plan& p) {
    const tc_mul_desc d{dw, du, nu, dv, nv};
    return tc_mul_batch_plan(&d, 1, &p, nullptr, st);
  };
  auto time_plan = [&](const tc_plan& p) {
    if (tc_workspace_bytes_plan(nu, nv, &p) > fr / 2) return;
    if (run(p) != TC_OK) return;  // compiles, warms up
    if (hipStreamSynchronize(st) != hipSuccess) return;
    // time at least 3 runs, more while the total stays short
    double ms = 1e300;
    for (int rep = 0; rep < 16; rep++) {
      (void)hipEventRecord(e0, st);
      if (run(p) != TC_OK) break;
      (void)hipEventRecord(e1, st);
      if (hipEventSynchronize(e1) != hipSuccess) break;
      float t = 0.f;
      (void)hipEventElapsedTime(&t, e0, e1);
      ms = std::min(ms, (double)t);
      if (rep >= 2 && ms * (rep + 1) > 200.0) break;
    }
    if (ms < best_t) {
      best_t = ms;
      best_p = p;
    }
  };
  for (const tc_plan& p : cands) time_plan(p);
  // the tile shape of the linear passes: the winner with half and double
  // the chunk width (a plan without a Toom level has no such pass)
  if (best_t < 1e299 && best_p.levels > 0) {
    const tc_plan w = best_p;
    for (const int ch : {-1, 1}) {
      tc_plan p = w;
      p.chunk = ch;
      time_plan(p);
    }
  }
  cleanup();
  rc = tc_get_error();
  if (rc != TC_OK) return rc;
  if (best_t >= 1e299) return TC_ERR_UNSUPPORTED;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned[size_class(n)] = best_p;
    g_tuned_ms[size_class(n)] = best_t;
  }
  if (best) *best = best_p;
  if (best_ms) *best_ms = best_t;
  return TC_OK;
}

int tc_autotune_clear(void) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tuned.clear();
  g_tuned_ms.clear();
  return TC_OK;
}

}  // extern "C"

namespace {
// The device a tuning table belongs to: architecture and compute units.
std::string device_key() {
  int dev = 0;
  hipDeviceProp_t pr;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&pr, dev) != hipSuccess) {
    (void)hipGetLastError();
    return "";
  }
  std::string arch = pr.gcnArchName;
  arch = arch.substr(0, arch.find(':'));
  return arch + "/" + std::to_string(pr.multiProcessorCount) + "cu";
}

// A minimal reader for the table format tc_autotune_save writes.
struct Scan {
  const std::string& t;
  size_t i = 0;
  explicit Scan(const std::string& s) : t(s) {}
  void ws() {
    while (i < t.size() && (t[i] == ' ' || t[i] == '\n' || t[i] == '\t' || t[i] == '\r')) i++;
  }
  bool lit(char c) {
    ws();
    if (i < t.size() && t[i] == c) {
      i++;
      return true;
    }
    return false;
  }
  bool str(std::string* out) {
    if (!lit('"')) return false;
    const size_t j = t.find('"', i);
    if (j == std::string::npos) return false;
    *out = t.substr(i, j - i);
    i = j + 1;
    return true;
  }
  bool num(double* out) {
    ws();
    const char* b = t.c_str() + i;
    char* e = nullptr;
    *out = std::strtod(b, &e);
    if (e == b) return false;
    i += (size_t)(e - b);
    return true;
  }
};
}  // namespace

extern "C" {

int tc_autotune_save(const char* path) {
  if (!path) return TC_ERR_INVALID;
  const std::string dk = device_key();
  if (dk.empty()) return TC_ERR_HIP;
  std::string out = "{\n  \"device\": \"" + dk + "\",\n  \"classes\": [";
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    bool first = true;
    for (const auto& kv : g_tuned) {
      out += first ? "\n" : ",\n";
      first = false;
      char ms[64];
      std::snprintf(ms, sizeof ms, "%.6g", g_tuned_ms.count(kv.first) ? g_tuned_ms[kv.first] : 0.0);
      out += "    {\"class\": " + std::to_string(kv.first) + ", \"plan\": [";
      for (int l = 0; l < kv.second.levels; l++)
        out += std::string(l ? ", " : "") + "[" + std::to_string(kv.second.B[l]) + ", " +
               std::to_string(kv.second.variant[l]) + "]";
      out += "]";
      if (kv.second.chunk) out += ", \"chunk\": " + std::to_string(kv.second.chunk);
      out += std::string(", \"ms\": ") + ms + "}";
    }
  }
  out += "\n  ]\n}\n";
  FILE* f = std::fopen(path, "w");
  if (!f) return TC_ERR_INVALID;
  const bool ok = std::fwrite(out.data(), 1, out.size(), f) == out.size();
  return (std::fclose(f) == 0 && ok) ? TC_OK : TC_ERR_INVALID;
}

int tc_autotune_load(const char* path) {
  if (!path) return TC_ERR_INVALID;
  FILE* f = std::fopen(path, "r");
  if (!f) return TC_ERR_INVALID;
  std::string text;
  char buf[4096];
  size_t k;
  while ((k = std::fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, k);
  std::fclose(f);
  const std::string dk = device_key();
  if (dk.empty()) return TC_ERR_HIP;
  Scan sc(text);
  std::string key, dev;
  std::map<int, tc_plan> plans;
  std::map<int, double> times;
  if (!sc.lit('{') || !sc.str(&key) || key != "device" || !sc.lit(':') || !sc.str(&dev) ||
      !sc.lit(',') || !sc.str(&key) || key != "classes" || !sc.lit(':') || !sc.lit('['))
    return TC_ERR_INVALID;
  if (dev != dk) return TC_ERR_UNSUPPORTED;  // tuned on another device
  bool more = !sc.lit(']');
  while (more) {
    double cls = 0, ms = 0;
    tc_plan p;
    std::memset(&p, 0, sizeof p);
    if (!sc.lit('{') || !sc.str(&key) || key != "class" || !sc.lit(':') || !sc.num(&cls) ||
        !sc.lit(',') || !sc.str(&key) || key != "plan" || !sc.lit(':') || !sc.lit('['))
      return TC_ERR_INVALID;
    bool lv = !sc.lit(']');
    while (lv) {
      double B = 0, var = 0;
      if (p.levels >= TC_MAX_LEVELS || !sc.lit('[') || !sc.num(&B) || !sc.lit(',') ||
          !sc.num(&var) || !sc.lit(']'))
        return TC_ERR_INVALID;
      p.B[p.levels] = (int)B;
      p.variant[p.levels] = (int)var;
      p.levels++;
      lv = sc.lit(',');
      if (!lv && !sc.lit(']')) return TC_ERR_INVALID;
    }
    if (!sc.lit(',') || !sc.str(&key)) return TC_ERR_INVALID;
    if (key == "chunk") {  // optional: the tuned chunk scale
      double ch = 0;
      if (!sc.lit(':') || !sc.num(&ch) || !sc.lit(',') || !sc.str(&key)) return TC_ERR_INVALID;
      p.chunk = (int)ch;
    }
    if (!plan_ok(p) || key != "ms" || !sc.lit(':') || !sc.num(&ms) || !sc.lit('}'))
      return TC_ERR_INVALID;
    plans[(int)cls] = p;
    times[(int)cls] = ms;
    more = sc.lit(',');
    if (!more && !sc.lit(']')) return TC_ERR_INVALID;
  }
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (const auto& kv : plans) {
    g_tuned[kv.first] = kv.second;
    g_tuned_ms[kv.first] = times[kv.first];
  }
  return TC_OK;
}

int tc_autotune_count(void) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  return (int)g_tuned.size();
}

int tc_set_cache_limit(size_t bytes) {
  Ctx* c;
  const int rc = get_ctx(&c);
  if (rc != TC_OK) return rc;
  std::lock_guard<std::mutex> lk(c->mu);
  c->cache_limit = bytes;
  evict_plans(c, 0);
  return TC_OK;
}

int tc_mul_noalloc(tc_limb* w, const tc_limb* u, size_t nu, const tc_limb* v, size_t nv,
                   hipStream_t stream) {
  if (!w || !u || !v || nu == 0 || nv == 0) return TC_ERR_INVALID;
  if (nu > ((size_t)1 << 31) || nv > ((size_t)1 << 31)) return TC_ERR_UNSUPPORTED;
  if (overlaps(w, (nu + nv) * 4, u, nu * 4) || overlaps(w, (nu + nv) * 4, v, nv * 4))
    return TC_ERR_INVALID;
  Ctx* c;
  int rc = find_ctx(&c);  // set up by tc_init: nothing is created here
  if (rc != TC_OK) return rc;
  if (!c->na_ptr) return TC_ERR_HIP;
  const bool sq = u == v && nu == nv;
  std::shared_ptr<Compiled> cp;
  {
    // host-side plan of tc_mul's own choice, kept per shape (host memory only)
    const std::string key = fault_prefix(c) + (sq ? "q" : "") + default_key((int64_t)nu, (int64_t)nv);
    std::lock_guard<std::mutex> lk(c->mu);
    auto it = c->na_cache.find(key);
    if (it != c->na_cache.end()) {
      cp = it->second;
    } else {
      Builder b;
      b.ctx = c;
      b.fault_item = c->fault_item;
      b.fuse_recomp = !c->strict;
      if (!gen_mul_default(b, dptr(BUF_U, 0), (int64_t)nu, dptr(sq ? BUF_U : BUF_V, 0), (int64_t)nv,
                           dptr(BUF_W, 0), 0))
        return TC_ERR_UNSUPPORTED;
      rc = finish(b, &cp, /*to_device=*/false);
      if (rc != TC_OK) return rc;
      c->na_cache[key] = cp;
    }
  }
  // workspace: [Bases | descriptors | scratch], each 256-byte aligned
  const size_t off_blob = 256;
  const size_t off_scr = align_up(off_blob + cp->h_blob.size(), 256);
  if (off_scr + cp->scratch_bytes > kNoAllocBytes) return TC_ERR_WORKSPACE;
  std::lock_guard<std::mutex> lk(c->na_mu);
  uint8_t* base = c->na_ptr;
  Bases& hb = c->na_bases;
  hb.scratch = base + off_scr;
  hb.p[0] = (uint8_t*)u;
  hb.p[1] = (uint8_t*)v;
  hb.p[2] = (uint8_t*)w;
  hb.table = nullptr;
  hb.err = c->d_err;
  hb.err_stride = 0;
  // stream-ordered copies from host memory: the previous call's kernels on
  // this stream have finished with the workspace before these land
  HIPCHK(hipMemcpyAsync(base, &hb, sizeof(Bases), hipMemcpyHostToDevice, stream));
  if (!cp->h_blob.empty())
    HIPCHK(hipMemcpyAsync(base + off_blob, cp->h_blob.data(), cp->h_blob.size(),
                          hipMemcpyHostToDevice, stream));
  return launch_all(c, *cp, base + off_blob, reinterpret_cast<const Bases*>(base), base + off_scr,
                    false, stream);
}

size_t tc_noalloc_capacity(void) { return kNoAllocBytes; }

int tc_set_strict(int on) {
  Ctx* c;
  int rc = get_ctx(&c);
  if (rc != TC_OK) return rc;
  std::lock_guard<std::mutex> lk(c->mu);
  c->strict = on != 0;
  return TC_OK;
}

int tc_debug_fault(int item) {
  if (item < -1) return TC_ERR_INVALID;
  Ctx* c;
  int rc = get_ctx(&c);
  if (rc != TC_OK) return rc;
  std::lock_guard<std::mutex> lk(c->mu);
  c->fault_item = item;
  return TC_OK;
}

int tc_timing_enable(int on) {
  Ctx* c;
  int rc = get_ctx(&c);
  if (rc != TC_OK) return rc;
  std::lock_guard<std::mutex> lk(c->mu);
  c->timing = on != 0;
  return TC_OK;
}

int tc_timing_read(int64_t* launches, double* ms) {
  if (!launches || !ms) return TC_ERR_INVALID;
  Ctx* c;
  int rc = get_ctx(&c);
  if (rc != TC_OK) return rc;
  std::lock_guard<std::mutex> lk(c->mu);
  for (int i = 0; i < TC_KERNEL_CLASSES; i++) {
    launches[i] = 0;
    ms[i] = 0.0;
  }
  for (auto& t : c->timed) {
    HIPCHK(hipEventSynchronize(t.b));
    float f = 0.f;
    HIPCHK(hipEventElapsedTime(&f, t.a, t.b));
    launches[t.kind] += 1;
    ms[t.kind] += f;
    c->event_pool.push_back(t.a);
    c->event_pool.push_back(t.b);
  }
  c->timed.clear();
  return TC_OK;
}

}  // extern "C"
