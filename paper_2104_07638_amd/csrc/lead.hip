// lead.hip -- leading principal minors by successive Schur complements (Sec. III) on gfx950.
//
// det A[:k, :k] for k = 1..n: elimination without row exchanges on the leading block, the
// k-th pivot being the ratio of consecutive leading minors (the ratio rule of Sec. II
// along the tree's rightmost path).  As the paper notes, no pivot correction is possible
// here (it would need minors that are never formed), so a zero pivot makes the later
// minors non-finite (info = -3).
//
// Mapping: one wavefront per matrix, the matrix in LDS with rows of n + 1 entries (lanes
// updating different rows of one column fall on different banks); at step k lane i
// updates row k + 1 + i of the trailing block with the pivot row scaled by 1/pivot.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "apm_device.h"
#include "apm_kernels.h"

namespace apm {
namespace {

constexpr int kLeadMax = 32;

template <class F>
__global__ __launch_bounds__(64) void lead_kernel(const typename F::E* __restrict__ A, typename F::E* __restrict__ out,
                                                  int32_t* __restrict__ info, int32_t batch, int n)
{
    using E = typename F::E;
    __shared__ E M[kLeadMax * (kLeadMax + 1)];
    __shared__ E wv[kLeadMax];
    const int b = blockIdx.x;
    if (b >= batch) return;
    const int lane = threadIdx.x;
    const int ld = n + 1;
    const E* A0 = A + (int64_t)b * n * n;
    E* ob = out + (int64_t)b * n;
    bool fin = true;
    for (int e = lane; e < n * n; e += 64) {
        const E v = A0[e];
        fin = fin && F::in_finite(v);
        M[(e / n) * ld + e % n] = v;
    }
    if (!__all(fin ? 1 : 0)) {
        for (int k = lane; k < n; k += 64) F::store_nan(ob, nullptr, k, false);
        if (info && lane == 0) info[b] = -2;
        return;
    }
    wave_sync();
    E mk = F::one();
    double chk = 0.0;
    for (int k = 0; k < n; ++k) {
        const E pv = M[k * ld + k];
        mk = F::bmul(mk, pv, 0);
        if (lane == 0) {
            ob[k] = mk;
            chk += F::fincheck(mk);
        }
        const int t = n - k - 1;   // order of the trailing block
        if (t == 0) break;
        if (lane < t) wv[lane] = F::rowscale(M[k * ld + k + 1 + lane], F::recip(pv));
        wave_sync();
        if (lane < t) {
            E* row = &M[(k + 1 + lane) * ld];
            const E c = row[k];
            for (int j = 0; j < t; ++j) row[k + 1 + j] = F::upd(row[k + 1 + j], c, wv[j]);
        }
        wave_sync();
    }
    const bool bad = __any(chk == 0.0 ? 0 : 1);
    if (info && lane == 0) info[b] = bad ? -3 : 0;
}

}  // namespace

hipError_t lead_launch(int dtype, const void* A, void* out, int32_t* info, int32_t batch, int n, hipStream_t st)
{
    if (n < 1 || n > kLeadMax) return hipErrorInvalidValue;
    if (dtype == 0) {
        hipLaunchKernelGGL(lead_kernel<FR64>, dim3((unsigned)batch), dim3(64), 0, st, static_cast<const double*>(A),
                           static_cast<double*>(out), info, batch, n);
    } else if (dtype == 2) {
        hipLaunchKernelGGL(lead_kernel<FC128>, dim3((unsigned)batch), dim3(64), 0, st, static_cast<const cd*>(A),
                           static_cast<cd*>(out), info, batch, n);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace apm
