// FP64 plan generation on the GPU (internal header).  Produces the same
// row-major tile blocks M_J[r][q] as build_ftb_blocks (plan_host.h).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <vector>

#include "plan_host.h"

namespace dsbt {

// Doubles of device scratch that build_ftb_blocks_device needs for (l, B, NT).
size_t device_plan_scratch_doubles(int ell, int B, int NT);

// Blocks of (l, B) over NT tiles computed on the current device in FP64 and
// copied to `blocks` (NT * R * R doubles, R = B + ceil(l/2)); `scratch` holds at
// least device_plan_scratch_doubles(ell, B, NT) doubles.  Synchronises
// `stream`; throws std::runtime_error on a HIP failure.
void build_ftb_blocks_device(int ell, int B, int NT, double* scratch, std::vector<double>& blocks,
                             hipStream_t stream);

}  // namespace dsbt
