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

// Largest leaf the schoolbook kernel takes (64 lanes x 8 columns).
constexpr int kLeafMax = 512;

LeafShape leaf_shape(int n);

hipError_t launch_step(int lpt, const StepDesc* d, const int64_t* wave0, int nd, int64_t waves,
                       const Bases& b, const DivEntry* divtab, uint32_t* err, hipStream_t st);
hipError_t launch_eval(int lpt, const EvalDesc* d, const int64_t* wave0, int nd, int64_t waves,
                       const Bases& b, uint32_t* err, hipStream_t st);
hipError_t launch_recomp(int lpt, const RecompDesc* d, const int64_t* wave0, int nd,
                         int64_t waves, const Bases& b, uint32_t* err, hipStream_t st);
// One launch covers leaves of one shape; descriptor i owns workgroups
// [wg0[i], wg0[i+1]).
hipError_t launch_leaf(const LeafShape& s, const LeafDesc* d, const int64_t* wg0, int nd,
                       int64_t wgs, const Bases& b, uint32_t* err, hipStream_t st);

}  // namespace tc
