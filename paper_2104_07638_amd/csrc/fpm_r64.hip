// fpm_r64.hip -- instantiation of the principal-minor kernels for one element type.
#include "fpm_impl.h"

namespace apm {

// the ranges that mixed_k0_range (fpm.hip) reports for this type
static_assert(RaggedK0<FR64>::lo == 3 && RaggedK0<FR64>::hi == 4 && BigK0<FR64>::lo == 4 && BigK0<FR64>::hi == 5,
              "mixed-order lane-subtree ranges");

template <>
int default_k0<FR64>(int n)
{
    return 5;
}

hipError_t fpm_launch_r64(const LaunchMinors& L, hipStream_t st) { return fpm_launch_field<FR64>(L, st); }

int64_t fpm_topq_bytes(int64_t batch) { return 4 * ((int64_t)kTopHead + batch * (kTopEntryInts + 1 + kSplit)); }

int64_t fpm_topq_bytes_unsplit(int64_t batch) { return 4 * ((int64_t)kTopHead + batch * (kTopEntryInts + 1)); }

}  // namespace apm
