// fpm_c128.hip -- instantiation of the principal-minor kernels for one element type.
#include "fpm_impl.h"

namespace apm {

template <>
int default_k0<FC128>(int n)
{
    return 3;
}

hipError_t fpm_launch_c128(const LaunchMinors& L, hipStream_t st) { return fpm_launch_field<FC128>(L, st); }

}  // namespace apm
