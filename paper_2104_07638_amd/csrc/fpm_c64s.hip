// fpm_c64s.hip -- instantiation of the principal-minor kernels for one element type.
#include "fpm_impl.h"

namespace apm {

template <>
int default_k0<FC64S>(int n)
{
    return 4;
}

hipError_t fpm_launch_c64s(const LaunchMinors& L, hipStream_t st) { return fpm_launch_field<FC64S>(L, st); }

}  // namespace apm
