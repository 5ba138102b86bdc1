// Online-stage kernel for small problems: the whole loop of Algorithm 1 on one workgroup with
// the layer matrix of the active penalty held in LDS.
#pragma once
#include <hip/hip_runtime.h>

#include "layer_kernel.h"

namespace rqp {

// Problems with n + m <= kSmallRows rows run on one workgroup of kSmallBlock threads; the
// layer matrix of the active penalty (at most 128 x 128 entries, 128 KB in FP64) sits in LDS.
constexpr int kSmallRows = 128;
constexpr int kSmallBlock = 1024;

// Dynamic LDS bytes of the single-workgroup kernel for L = n + m rows.
template <typename T>
size_t small_lds_bytes(int L);

// Runs the solves described by `a` (plain solves and sequences; no closed loop, no scaling:
// a.Ad and a.sc_dual must be null) as one workgroup. Sets the kernel's LDS limit on first use.
template <typename T>
hipError_t launch_small(const LayerArgs& a, hipStream_t st);

}  // namespace rqp
