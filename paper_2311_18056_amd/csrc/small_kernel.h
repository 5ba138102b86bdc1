// Online-stage kernel for small problems: the whole loop of Algorithm 1 on one workgroup with
// the layer matrix of the active penalty held in registers.
#pragma once
#include <hip/hip_runtime.h>

#include "layer_kernel.h"

namespace rqp {

// Problems with n + m <= kSmallRows rows run on one workgroup of kSmallBlock threads; the
// layer matrix of the active penalty (at most 128 x 128 entries) sits in registers, at most 16
// entries per thread.
constexpr int kSmallRows = 128;
constexpr int kSmallBlock = 1024;

// Sets the kernel's LDS limit for L = n + m rows on the current device (once per handle, at
// setup, before the first launch_small).
template <typename T>
hipError_t prepare_small(int L);

// Runs the solves described by `a` (plain solves and sequences, Ruiz-scaled or not; no closed
// loop: a.Ad must be null) as one workgroup.
template <typename T>
hipError_t launch_small(const LayerArgs& a, hipStream_t st);

}  // namespace rqp
