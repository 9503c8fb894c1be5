// fpm_c64s.hip -- instantiation of the principal-minor kernels for one element type.
#include "fpm_impl.h"

namespace apm {

// the ranges that mixed_k0_range (fpm.hip) reports for this type
static_assert(RaggedK0<FC64S>::lo == 3 && RaggedK0<FC64S>::hi == 3 && BigK0<FC64S>::lo == 3 && BigK0<FC64S>::hi == 4,
              "mixed-order lane-subtree ranges");

template <>
int default_k0<FC64S>(int n)
{
    return 4;
}

hipError_t fpm_launch_c64s(const LaunchMinors& L, hipStream_t st) { return fpm_launch_field<FC64S>(L, st); }

}  // namespace apm
