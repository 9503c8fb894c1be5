// stubs.hip -- temporary: entry points whose kernels are not built yet.
#include "apm_kernels.h"
namespace apm {

hipError_t perm_launch(const LaunchPerm&, hipStream_t) { return hipErrorNotSupported; }
}  // namespace apm
