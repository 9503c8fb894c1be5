// fpm_r32s.hip -- instantiation of the principal-minor kernels for one element type.
#include "fpm_impl.h"

namespace apm {

template <>
int default_k0<FR32S>(int n)
{
    return 5;
}

hipError_t fpm_launch_r32s(const LaunchMinors& L, hipStream_t st) { return fpm_launch_field<FR32S>(L, st); }

}  // namespace apm
