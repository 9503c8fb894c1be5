// fpm_r64.hip -- instantiation of the principal-minor kernels for one element type.
#include "fpm_impl.h"

namespace apm {

template <>
int default_k0<FR64>(int n)
{
    return 5;
}

hipError_t fpm_launch_r64(const LaunchMinors& L, hipStream_t st) { return fpm_launch_field<FR64>(L, st); }

int64_t fpm_topq_bytes(int64_t batch) { return 4 * ((int64_t)kTopHead + batch * (kTopEntryInts + 1 + kSplit)); }

int64_t fpm_topq_bytes_unsplit(int64_t batch) { return 4 * ((int64_t)kTopHead + batch * (kTopEntryInts + 1)); }

}  // namespace apm
