// tc_internal.hpp -- declarations shared by the host runtime and the kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>

#include "tc_types.hpp"

namespace tc {

struct LeafShape {
  int R;            // columns per group
  int tpl;          // lanes per leaf
  size_t lds_bytes; // dynamic LDS of a 256-thread workgroup
};

// Leaves up to kLeafVmax limbs run on the vector ALUs (64 lanes x 8
// columns); wider ones, up to kLeafMax, on the matrix cores (measured: the
// matrix-core leaf wins from a few dozen limbs up).
constexpr int kLeafVmax = 32;
constexpr int kLeafMax = 2048;

LeafShape leaf_shape(int n);

// per_desc > 0: every descriptor holds per_desc waves (direct indexing).
// Kernels report exactness failures in the error word of each descriptor's
// item (Bases::err, Bases::err_stride).
hipError_t launch_step(int lpt, const StepDesc* d, const int64_t* wave0, int nd, int64_t waves,
                       int64_t per_desc, const Bases* b, const DivEntry* divtab, uint64_t* status,
                       hipStream_t st);
// Recomposing steps (a single-round level's interpolation and recomposition).
hipError_t launch_rstep(int lpt, const RStepDesc* d, const int64_t* w0, int nd, int64_t waves,
                        int64_t per_desc, const Bases* b, const DivEntry* divtab, uint64_t* status,
                        hipStream_t st);
// neg_pass: the sign fix-up of multi-chunk evaluations (after the evaluation).
hipError_t launch_eval(int lpt, bool neg_pass, const EvalDesc* d, const int64_t* wave0, int nd,
                       int64_t waves, int64_t per_desc, const Bases* b, uint64_t* status,
                       hipStream_t st);
hipError_t launch_recomp(int lpt, const RecompDesc* d, const int64_t* wave0, int nd,
                         int64_t waves, int64_t per_desc, const Bases* b, uint64_t* status,
                         hipStream_t st);
// status[i] = item_err[i] ? code : 0 for i < n.
hipError_t launch_item_status(const uint32_t* item_err, int32_t* status, int64_t n, int32_t code,
                              hipStream_t st);
// Flips bit 0 of the limb at each of the n (<= 256) targets (test hook).
hipError_t launch_flip(const DPtr* targets, int n, const Bases* b, hipStream_t st);
// *out = the word at err, which is cleared in the same atomic step.
hipError_t launch_take_error(uint32_t* err, uint32_t* out, hipStream_t st);
// Clears nr ranges (device array of (byte offset from base, 64-bit words)
// pairs, the longest max_words) in one launch.
hipError_t launch_fill_ranges(uint8_t* base, const int64_t* ranges, int nr, int64_t max_words,
                              hipStream_t st);
// Matrix-core schoolbook leaves (one workgroup per leaf of width n, all
// descriptors of the launch with the same n).
int mleaf_lds_bytes(int n);
hipError_t launch_mleaf(int n, const LeafDesc* d, const int64_t* wg0, int nd, int64_t wgs,
                        const Bases* b, hipStream_t st);
hipError_t set_mleaf_lds_limit(size_t bytes);
// One launch covers leaves of one shape; descriptor i owns workgroups
// [wg0[i], wg0[i+1]).
hipError_t launch_leaf(const LeafShape& s, const LeafDesc* d, const int64_t* wg0, int nd,
                       int64_t wgs, const Bases* b, hipStream_t st);

// Transform leaves (tc_ntt.hip): the launches of one leaf phase, in order.
// Units are workgroups, or waves for the carry pass (engine chunks of 64 lpt
// limbs); lds is the dynamic LDS of the transform kernels.  roots: the table
// laid out as kNttRoot* in tc_types.hpp.
enum : int { kNttColFwd = 0, kNttRowFwd = 1, kNttRowMul = 2, kNttColInv = 3, kNttCarry = 4 };
hipError_t launch_ntt(int which, const NttDesc* d, const int64_t* u0, int nd, int64_t units,
                      int lpt, size_t lds, const Bases* b, const uint64_t* roots,
                      uint64_t* status, hipStream_t st);

// Multiply-adds (v_mad_u64_u32) per second on the current device, from a
// throughput probe of about 2 ms on the null stream (synchronous).
hipError_t measure_mad_rate(double* per_s);

}  // namespace tc
