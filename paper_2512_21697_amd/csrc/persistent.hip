// One variant of the persistent solver kernel per object file (the build compiles this source four
// times with TDDE_VARIANT = 2 * mixed + preconditioned), so the variants compile in parallel.
#include "solver.hpp"

#ifndef TDDE_VARIANT
#error "TDDE_VARIANT (0..3) must be defined"
#endif

namespace tdde {

#define TDDE_CAT2(a, b) a##b
#define TDDE_CAT(a, b) TDDE_CAT2(a, b)

// Host-side handle of the kernel (for hipLaunchCooperativeKernel and the occupancy query).
const void* TDDE_CAT(persistent_variant_, TDDE_VARIANT)() {
  return reinterpret_cast<const void*>(&persistent_kernel<(TDDE_VARIANT & 1) != 0, (TDDE_VARIANT & 2) != 0>);
}

}  // namespace tdde
