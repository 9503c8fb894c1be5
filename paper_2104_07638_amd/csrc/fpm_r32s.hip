// fpm_r32s.hip -- instantiation of the principal-minor kernels for one element type.
#include "fpm_impl.h"

namespace apm {

// the ranges that mixed_k0_range (fpm.hip) reports for this type
static_assert(RaggedK0<FR32S>::lo == 3 && RaggedK0<FR32S>::hi == 4 && BigK0<FR32S>::lo == 4 && BigK0<FR32S>::hi == 5,
              "mixed-order lane-subtree ranges");

template <>
int default_k0<FR32S>(int n)
{
    return 5;
}

hipError_t fpm_launch_r32s(const LaunchMinors& L, hipStream_t st) { return fpm_launch_field<FR32S>(L, st); }

}  // namespace apm
