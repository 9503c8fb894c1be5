// fpm_c128.hip -- instantiation of the principal-minor kernels for one element type.
#include "fpm_impl.h"

namespace apm {

// the ranges that mixed_k0_range (fpm.hip) reports for this type
static_assert(RaggedK0<FC128>::lo == 2 && RaggedK0<FC128>::hi == 2 && BigK0<FC128>::lo == 2 && BigK0<FC128>::hi == 3,
              "mixed-order lane-subtree ranges");

template <>
int default_k0<FC128>(int n)
{
    return 3;
}

hipError_t fpm_launch_c128(const LaunchMinors& L, hipStream_t st) { return fpm_launch_field<FC128>(L, st); }

}  // namespace apm
