// fpm.hip -- dispatch of apm_all_minors to the per-type kernel instantiations.
#include "apm_kernels.h"

namespace apm {

hipError_t fpm_launch_r64(const LaunchMinors& L, hipStream_t st);
hipError_t fpm_launch_r32s(const LaunchMinors& L, hipStream_t st);
hipError_t fpm_launch_c128(const LaunchMinors& L, hipStream_t st);
hipError_t fpm_launch_c64s(const LaunchMinors& L, hipStream_t st);

hipError_t fpm_launch(const LaunchMinors& L, hipStream_t st)
{
    switch (L.dtype) {
    case 0: return fpm_launch_r64(L, st);
    case 1: return fpm_launch_r32s(L, st);
    case 2: return fpm_launch_c128(L, st);
    case 3: return fpm_launch_c64s(L, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace apm
