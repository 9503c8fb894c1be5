// mc.hip -- Metropolis-Hastings step over vertex configurations on gfx950.
//
// The weight of a configuration is |c[V]|, the connected sum over all its vertices
// (Sec. V.A, Eq. (recursion)) of a[S] = det(M[S])^2 with M_ij = G0(X_i - X_j), computed by
// the minors and connected-sum kernels of this library.  The kernels here do the rest
// of a step: the moved vertex and its context features, the proposal (uniform, or drawn
// from the network's site and time-bin logits) with its log proposal ratio, the
// gather of the proposal's propagator matrix from the G0 table, the acceptance test
// and the regression loss that trains the network.
//
// Random numbers: Philox4x64-10 (Salmon, Moraes, Dror & Shaw, SC'11) keyed by
// (seed, 0) at counter (walker, step, call, 0).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "apm_device.h"
#include "apm_kernels.h"

namespace apm {
namespace {

struct U4 {
    uint64_t x, y, z, w;
};

__device__ __forceinline__ U4 philox(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0, uint64_t k1)
{
    constexpr uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    constexpr uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
        const uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
        const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += W0;
        k1 += W1;
    }
    return {c0, c1, c2, c3};
}

__device__ __forceinline__ U4 draws(const McArgs& a, int w, int call)
{
    return philox((uint64_t)w, (uint64_t)(uint32_t)a.step, (uint64_t)call, 0ull, a.seed, 0ull);
}

__device__ __forceinline__ U4 load_draw(const uint64_t* p)
{
    const ulonglong2 lo = reinterpret_cast<const ulonglong2*>(p)[0], hi = reinterpret_cast<const ulonglong2*>(p)[1];
    return {lo.x, lo.y, hi.x, hi.y};
}

// Walkers per workgroup (256 threads) of the per-walker kernels: one wavefront per walker
// (kWgWalkers), or a group of 16 lanes per walker (kGrpWalkers) where a walker's work is
// small.
constexpr int kWgWalkers = 4;
constexpr int kGrpWalkers = 16;
static_assert(64 * kWgWalkers == 256, "the per-walker kernels are launched with 256 threads");

// Draws 0 and 1 of the calling thread's walker w = w0 + threadIdx.x / (256 / WPG) (WPG walkers
// per workgroup), in every lane.  Read from the step's table when it is filled.  Otherwise
// lanes 0 .. 2 WPG - 1 of wavefront 0 compute the workgroup's 2 WPG Philox chains at once
// (lane 2 i + c: walker w0 + i, call c), so the workgroup pays for one chain instead of WPG;
// with a table they also store them there.  Called by every thread of the workgroup (it holds
// a barrier); walkers past a.W get nothing.
template <int WPG>
__device__ __forceinline__ void wg_draws(const McArgs& a, int w0, U4& d0, U4& d1)
{
    static_assert(2 * WPG <= 64, "the chains fit one wavefront");
    const int wi = threadIdx.x / (256 / WPG);
    if (a.draws && a.draws_ready) {
        const int w = w0 + wi;
        if (w < a.W) {
            d0 = load_draw(a.draws + (size_t)w * 8);
            d1 = load_draw(a.draws + (size_t)w * 8 + 4);
        }
        return;
    }
    __shared__ ulonglong2 sh[WPG * 2][2];
    const int t = threadIdx.x;
    if (t < 2 * WPG && w0 + (t >> 1) < a.W) {
        const U4 d = draws(a, w0 + (t >> 1), t & 1);
        sh[t][0] = make_ulonglong2(d.x, d.y);
        sh[t][1] = make_ulonglong2(d.z, d.w);
        if (a.draws) {
            ulonglong2* p = reinterpret_cast<ulonglong2*>(a.draws + ((size_t)w0 * 2 + t) * 4);
            p[0] = sh[t][0];
            p[1] = sh[t][1];
        }
    }
    __syncthreads();
    const ulonglong2 a0 = sh[2 * wi][0], a1 = sh[2 * wi][1], b0 = sh[2 * wi + 1][0], b1 = sh[2 * wi + 1][1];
    d0 = {a0.x, a0.y, a1.x, a1.y};
    d1 = {b0.x, b0.y, b1.x, b1.y};
}

__device__ __forceinline__ int below(uint64_t r, int m) { return (int)__umul64hi(r, (uint64_t)m); }

__device__ __forceinline__ double unif(uint64_t r) { return ((double)(r >> 12) + 0.5) * 0x1p-52; }

__device__ __forceinline__ uint16_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// Cross-lane reductions and scans by DPP: within rows of 16 lanes (row_shr:1, 2, 4, 8), then
// across rows (row_bcast:15 into rows 1 and 3, row_bcast:31 into rows 2 and 3), which leaves
// a scan's total in lane 63; reductions read it from there.  All 64 lanes must be active.
// dpp_d: lane i gets v of its DPP source lane, or `old` where there is none (bc: 0 instead).
template <int CTRL, int RM = 0xF, bool BC = false>
__device__ __forceinline__ double dpp_d(double old, double v)
{
    const int lo = __builtin_amdgcn_update_dpp(__double2loint(old), __double2loint(v), CTRL, RM, 0xF, BC);
    const int hi = __builtin_amdgcn_update_dpp(__double2hiint(old), __double2hiint(v), CTRL, RM, 0xF, BC);
    return __hiloint2double(hi, lo);
}

template <int CTRL, int RM = 0xF>
__device__ __forceinline__ int dpp_i(int old, int v)
{
    return __builtin_amdgcn_update_dpp(old, v, CTRL, RM, 0xF, false);
}

__device__ __forceinline__ double lane63_d(double v)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
    return __hiloint2double(hi, lo);
}

// largest value over the wavefront (any doubles; -inf allowed)
__device__ __forceinline__ double wave_max_d(double v)
{
    v = fmax(v, dpp_d<0x111>(v, v));
    v = fmax(v, dpp_d<0x112>(v, v));
    v = fmax(v, dpp_d<0x114>(v, v));
    v = fmax(v, dpp_d<0x118>(v, v));
    v = fmax(v, dpp_d<0x142, 0xA>(v, v));
    v = fmax(v, dpp_d<0x143, 0xC>(v, v));
    return lane63_d(v);
}

__device__ __forceinline__ int wave_min_i(int v)
{
    v = min(v, dpp_i<0x111>(v, v));
    v = min(v, dpp_i<0x112>(v, v));
    v = min(v, dpp_i<0x114>(v, v));
    v = min(v, dpp_i<0x118>(v, v));
    v = min(v, dpp_i<0x142, 0xA>(v, v));
    v = min(v, dpp_i<0x143, 0xC>(v, v));
    return __builtin_amdgcn_readlane(v, 63);
}

__device__ __forceinline__ int wave_max_i(int v)
{
    v = max(v, dpp_i<0x111>(v, v));
    v = max(v, dpp_i<0x112>(v, v));
    v = max(v, dpp_i<0x114>(v, v));
    v = max(v, dpp_i<0x118>(v, v));
    v = max(v, dpp_i<0x142, 0xA>(v, v));
    v = max(v, dpp_i<0x143, 0xC>(v, v));
    return __builtin_amdgcn_readlane(v, 63);
}

// inclusive prefix sum over the 64 lanes
__device__ __forceinline__ double wave_scan(double v)
{
    v += dpp_d<0x111, 0xF, true>(0.0, v);
    v += dpp_d<0x112, 0xF, true>(0.0, v);
    v += dpp_d<0x114, 0xF, true>(0.0, v);
    v += dpp_d<0x118, 0xF, true>(0.0, v);
    v += dpp_d<0x142, 0xA>(0.0, v);
    v += dpp_d<0x143, 0xC>(0.0, v);
    return v;
}

// v of lane i - 1 (0 in lane 0): wave_shr:1
__device__ __forceinline__ double wave_shr1(double v) { return dpp_d<0x138, 0xF, true>(0.0, v); }

// Propagator matrix of walker w with vertex k replaced by vnew (k < 0: no replacement),
// by a group of G lanes (G divides 64, all of them active).  Vertices outside the grid give
// NaN entries (no table read).  Lane i < n of the group first unpacks vertex i into
// (x, y, t), packed x | y << 8 | t << 16 (L <= 256, t < 2^15), or ~0 outside the grid; each
// entry then takes the periodic differences of two such words.
template <int G>
__device__ void gather_grp(const McArgs& a, int w, int k, uint32_t vnew, double* __restrict__ mats)
{
    const int r = threadIdx.x & (G - 1), gbase = (int)(threadIdx.x & 63) & ~(G - 1);
    const int n = a.n, L = a.L, L2 = L * L, nn = n * n;
    uint32_t xyt = 0xFFFFFFFFu;
    if (r < n) {
        const uint32_t v = (r == k) ? vnew : a.state[(size_t)w * n + r];
        const int s = (int)(v & 0xFFFFu), t = (int)(v >> 16);
        if (s < L2 && t < a.n_tau) xyt = (uint32_t)(s % L) | ((uint32_t)(s / L) << 8) | ((uint32_t)t << 16);
    }
    double* M = mats + (size_t)w * nn;
    for (int base = 0; base < nn; base += G) {
        const int e = base + r;
        const int i = e < nn ? e / n : 0, j = e < nn ? e - i * n : 0;
        const uint32_t pi = (uint32_t)__shfl((int)xyt, gbase + i, 64), pj = (uint32_t)__shfl((int)xyt, gbase + j, 64);
        if (e < nn) {
            double val = __builtin_nan("");
            if (((pi | pj) >> 31) == 0) {
                int dx = (int)(pi & 0xFFu) - (int)(pj & 0xFFu);
                int dy = (int)((pi >> 8) & 0xFFu) - (int)((pj >> 8) & 0xFFu);
                dx += dx < 0 ? L : 0;
                dy += dy < 0 ? L : 0;
                const int d = (int)(pi >> 16) - (int)(pj >> 16) + a.n_tau - 1;
                val = a.g0[(size_t)d * L2 + dy * L + dx];
            }
            M[e] = val;
        }
    }
}

// moved vertex and (optionally) BF16 context features; 16 lanes per walker (n <= 16)
__global__ __launch_bounds__(256) void mc_context_kernel(McArgs a, int32_t* __restrict__ moved,
                                                         uint16_t* __restrict__ feat, int dp)
{
    constexpr int G = 256 / kGrpWalkers;
    const int r = threadIdx.x & (G - 1), gbase = (int)(threadIdx.x & 63) & ~(G - 1);
    const int w = blockIdx.x * kGrpWalkers + threadIdx.x / G;
    U4 d0, d1;
    wg_draws<kGrpWalkers>(a, blockIdx.x * kGrpWalkers, d0, d1);
    if (w >= a.W) return;   // whole groups
    const int n = a.n;
    const int k = below(d0.x, n);
    if (r == 0) moved[w] = k;
    if (!feat) return;
    const uint32_t v = r < n ? a.state[(size_t)w * n + r] : 0xFFFFFFFFu;
    int rank = 0;
    for (int j = 0; j < n; ++j) {
        const uint32_t vj = (uint32_t)__shfl((int)v, gbase + j, 64);
        if (j != k && j != r && (vj < v || (vj == v && j < r))) ++rank;
    }
    uint16_t* f = feat + (size_t)w * dp;
    if (r < n && r != k) {
        const int s = (int)(v & 0xFFFFu), t = (int)(v >> 16);
        f[3 * rank + 0] = f2bf((float)(s % a.L) / (float)a.L);
        f[3 * rank + 1] = f2bf((float)(s / a.L) / (float)a.L);
        f[3 * rank + 2] = f2bf(((float)t + 0.5f) / (float)a.n_tau);
    }
    for (int q = 3 * (n - 1) + r; q < dp; q += G) f[q] = 0;
}

struct Dist {
    double mx, tot;   // max logit, sum of exp(logit - mx)
};

// log q~(old) - log q~(new) of the mixed learned proposal
//   q~(v) = (1 - eps) (es / tot_s) (eb / tot_b) / per_bin + eps / (L^2 n_tau),
// with es, eb the site and bin terms exp(logit - max) of v and tot_s, tot_b their sums.
// Both are proportional to es eb + C with C = eps per_bin tot_s tot_b / ((1 - eps) L^2 n_tau),
// so the ratio takes one logarithm; eps = 1 is the uniform proposal (ratio 1).
__device__ __forceinline__ double log_q_ratio(const McArgs& a, double eso, double ebo, double esn, double ebn, Dist ds,
                                              Dist db, int per_bin)
{
    if (!(a.eps < 1.0)) return 0.0;
    const double C = a.eps * (double)per_bin * ds.tot * db.tot / ((1.0 - a.eps) * ((double)(a.L * a.L) * a.n_tau));
    return log((eso * ebo + C) / (esn * ebn + C));
}

// The uniform proposal (site and time point uniform, log q ratio 0) and its matrices, one
// wavefront per walker (groups of 16 lanes measured no faster: the gather dominates).
// moved_out != NULL: the moved vertex is drawn here (as the context kernel draws it) and
// written to moved_out; otherwise it is read from moved.
__global__ __launch_bounds__(256) void mc_propose_uniform_kernel(McArgs a, const int32_t* __restrict__ moved,
                                                                 int32_t* __restrict__ moved_out,
                                                                 uint32_t* __restrict__ prop,
                                                                 double* __restrict__ logq, double* __restrict__ mats)
{
    constexpr int G = 256 / kWgWalkers;
    const int r = threadIdx.x & (G - 1);
    const int w = blockIdx.x * kWgWalkers + threadIdx.x / G;
    U4 d0, d1;
    wg_draws<kWgWalkers>(a, blockIdx.x * kWgWalkers, d0, d1);
    if (w >= a.W) return;   // whole groups
    const int n = a.n;
    int k;
    if (moved_out) {
        k = below(d0.x, n);
        if (r == 0) moved_out[w] = k;
    } else {
        k = moved[w];
        if (k < 0 || k >= n) k = 0;
    }
    const uint32_t vnew = (uint32_t)below(d0.z, a.L * a.L) | ((uint32_t)below(d0.w, a.n_tau) << 16);
    if (r == 0) {
        prop[w] = vnew;
        logq[w] = 0.0;
    }
    gather_grp<G>(a, w, k, vnew, mats);
}

// The learned proposal (site and time bin from the network's logits, mixed with the uniform
// proposal at weight eps) with its log q ratio, and its matrices; one wavefront per walker.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) void mc_propose_kernel(McArgs a, const int32_t* __restrict__ moved,
                                                         const float* __restrict__ logits, int stride,
                                                         uint32_t* __restrict__ prop, double* __restrict__ logq,
                                                         double* __restrict__ mats)
{
    const int lane = threadIdx.x & 63;
    const int w = blockIdx.x * kWgWalkers + (threadIdx.x >> 6);
    U4 d0, d1;
    wg_draws<kWgWalkers>(a, blockIdx.x * kWgWalkers, d0, d1);
    if (w >= a.W) return;
    const int n = a.n, L2 = a.L * a.L;
    int k = moved[w];
    if (k < 0 || k >= n) k = 0;
    int site = below(d0.z, L2), t = below(d0.w, a.n_tau);
    double lq = 0.0;
    {
        const float* lg = logits + (size_t)w * stride;
        const int per_bin = a.n_tau / a.n_bin;
        // site distribution: lane owns the contiguous block [j0, j1); up to kPc of its terms
        // exp(logit - max) are kept in registers for the draw and for q~
        const int P = (L2 + kWave - 1) / kWave;
        const int j0 = min(L2, lane * P), j1 = min(L2, j0 + P);
        double mx = -INFINITY;
        for (int j = j0; j < j1; ++j) mx = fmax(mx, (double)lg[j]);
        mx = wave_max_d(mx);
        constexpr int kPc = 4;   // P at L = 16; a lane evaluates only the terms it owns
        double pc[kPc];
        double part = 0.0;
#pragma unroll
        for (int u = 0; u < kPc; ++u) {
            pc[u] = 0.0;
            if (j0 + u < j1) pc[u] = exp((double)lg[j0 + u] - mx);
            part += pc[u];
        }
        for (int j = j0 + kPc; j < j1; ++j) part += exp((double)lg[j] - mx);
        const double incl = wave_scan(part);
        const double excl = wave_shr1(incl);
        const Dist ds{mx, lane63_d(incl)};
        // bin distribution: one bin per lane
        const double bl = lane < a.n_bin ? (double)lg[L2 + lane] : -INFINITY;
        const double mxb = wave_max_d(bl);
        const double pbl = lane < a.n_bin ? exp(bl - mxb) : 0.0;
        const double inclb = wave_scan(pbl);
        const Dist db{mxb, lane63_d(inclb)};
        if (!(unif(d0.y) < a.eps)) {
            const double tg = unif(d1.x) * ds.tot;
            int cand = 0x7FFFFFFF, lastpos = -1;
            double run = excl;
            auto visit = [&](int j, double p) {
                run += p;
                if (p > 0.0) {
                    lastpos = j;
                    if (run > tg && cand == 0x7FFFFFFF) cand = j;
                }
            };
#pragma unroll
            for (int u = 0; u < kPc; ++u)
                if (j0 + u < j1) visit(j0 + u, pc[u]);
            for (int j = j0 + kPc; j < j1; ++j) visit(j, exp((double)lg[j] - mx));
            site = wave_min_i(cand);
            if (site == 0x7FFFFFFF) site = wave_max_i(lastpos);
            const double tgb = unif(d1.y) * db.tot;
            const int cb = (lane < a.n_bin && pbl > 0.0 && inclb > tgb) ? lane : 0x7FFFFFFF;
            int b = wave_min_i(cb);
            if (b == 0x7FFFFFFF) b = wave_max_i((lane < a.n_bin && pbl > 0.0) ? lane : -1);
            t = b * per_bin + below(d1.z, per_bin);
        }
        const uint32_t vk = a.state[(size_t)w * n + k];
        // the exp terms of the old and the new site (recomputed: the same values the owning
        // lanes hold) and bin (taken from the lane that holds it)
        auto site_term = [&](int sj) { return exp((double)lg[sj] - ds.mx); };
        auto bin_term = [&](int bj) {
            return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(pbl), bj),
                                    __builtin_amdgcn_readlane(__double2loint(pbl), bj));
        };
        const int so = (int)(vk & 0xFFFFu) < L2 ? (int)(vk & 0xFFFFu) : 0;
        const int to = (int)(vk >> 16) < a.n_tau ? (int)(vk >> 16) : 0;
        lq = log_q_ratio(a, site_term(so), bin_term(to / per_bin), site_term(site), bin_term(t / per_bin), ds, db,
                         per_bin);
    }
    const uint32_t vnew = (uint32_t)site | ((uint32_t)t << 16);
    if (lane == 0) {
        prop[w] = vnew;
        logq[w] = lq;
    }
    gather_grp<64>(a, w, k, vnew, mats);
}

__global__ __launch_bounds__(256) void mc_gather_kernel(McArgs a, double* __restrict__ mats)
{
    const int w = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (w >= a.W) return;
    gather_grp<64>(a, w, -1, 0u, mats);
}

struct Wt {
    double lc;
    int8_t sg;
};

// full_weight (below) from the (c[V], d[V]) pair of walker w that the connected-sum kernel
// wrote; one lane.
__device__ __forceinline__ Wt summ_weight(const McArgs& a, int w, const double* __restrict__ summ)
{
    const double cv = summ[2 * w], dv = summ[2 * w + 1];
    const bool ok = isfinite(cv) && cv != 0.0 && !(a.resolve > 0.0 && !(fabs(cv) >= a.resolve * dv));
    return ok ? Wt{log(fabs(cv)), cv > 0.0 ? (int8_t)1 : (int8_t)-1} : Wt{-INFINITY, (int8_t)0};
}

// log|c[V]| and the sign of c[V] for walker w, or (-inf, 0) when c[V] is zero, not
// finite, or (resolve > 0) below resolve * d[V] with
//     d[V] = |a[V]| + sum_{T containing vertex 0, T != V} |c[T]| |a[V \ T]|,  a = m^2,
// the rounding scale of the recursion at V.  Called by a whole wavefront.
__device__ Wt full_weight(const McArgs& a, int w, const double* __restrict__ c, const double* __restrict__ m,
                         const double* __restrict__ summ)
{
    const int lane = lane_id();
    if (summ) return summ_weight(a, w, summ);
    const uint32_t nm = 1u << a.n, V = nm - 1u;
    const double* cw = c + (size_t)w * nm;
    const double* mw = m + (size_t)w * nm;
    const double cv = cw[V];
    bool ok = isfinite(cv) && cv != 0.0;
    if (ok && a.resolve > 0.0) {
        double part = 0.0;
        for (uint32_t i = lane; i < nm / 2; i += kWave) {
            const uint32_t T = 2u * i + 1u;                 // sets containing vertex 0
            if (T == V) {
                part += mw[V] * mw[V];                     // |a[V]|
            } else {
                const double mr = mw[V & ~T];
                part += fabs(cw[T]) * (mr * mr);
            }
        }
        for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o);
        ok = fabs(cv) >= a.resolve * part;
    }
    return ok ? Wt{log(fabs(cv)), cv > 0.0 ? (int8_t)1 : (int8_t)-1} : Wt{-INFINITY, (int8_t)0};
}

// Acceptance test and state update of walker w, given the weight of its proposal.
__device__ __forceinline__ void accept_one(const McArgs& a, int w, Wt wt, const int32_t* __restrict__ moved,
                                           const uint32_t* __restrict__ prop, const double* __restrict__ logq,
                                           double* logc_out, uint8_t* acc_out, float* obs_logw, int8_t* obs_sign)
{
    double lw = a.logw[w];
    int8_t sg = a.sign[w];
    const int k = moved[w];
    const U4 d1 = (a.draws && a.draws_ready) ? load_draw(a.draws + (size_t)w * 8 + 4) : draws(a, w, 1);
    const double logR = wt.lc - lw + logq[w];
    const bool acc = (k >= 0 && k < a.n) && wt.lc > -INFINITY && (!(lw > -INFINITY) || log(unif(d1.w)) < logR);
    if (acc) {
        a.state[(size_t)w * a.n + k] = prop[w];
        lw = wt.lc;
        sg = wt.sg;
        a.logw[w] = lw;
        a.sign[w] = sg;
    }
    if (logc_out) logc_out[w] = wt.lc;
    if (acc_out) acc_out[w] = acc ? 1 : 0;
    if (obs_logw) obs_logw[w] = (float)lw;
    if (obs_sign) obs_sign[w] = sg;
}

// one wavefront per walker (the weight reduced over c[] and the minors)
__global__ __launch_bounds__(256) void mc_accept_kernel(McArgs a, const int32_t* __restrict__ moved,
                                                        const uint32_t* __restrict__ prop,
                                                        const double* __restrict__ logq,
                                                        const double* __restrict__ c,
                                                        const double* __restrict__ minors, double* logc_out,
                                                        uint8_t* acc_out, float* obs_logw, int8_t* obs_sign)
{
    const int w = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (w >= a.W) return;
    const Wt wt = full_weight(a, w, c, minors, nullptr);
    if (lane_id() != 0) return;
    accept_one(a, w, wt, moved, prop, logq, logc_out, acc_out, obs_logw, obs_sign);
}

// one lane per walker, with (c[V], d[V]) per walker from the connected-sum kernel
__global__ __launch_bounds__(256) void mc_accept_summ_kernel(McArgs a, const int32_t* __restrict__ moved,
                                                             const uint32_t* __restrict__ prop,
                                                             const double* __restrict__ logq,
                                                             const double* __restrict__ summ, double* logc_out,
                                                             uint8_t* acc_out, float* obs_logw, int8_t* obs_sign)
{
    const int w = blockIdx.x * 256 + threadIdx.x;
    if (w >= a.W) return;
    accept_one(a, w, summ_weight(a, w, summ), moved, prop, logq, logc_out, acc_out, obs_logw, obs_sign);
}

__global__ __launch_bounds__(256) void mc_set_kernel(McArgs a, const double* __restrict__ c,
                                                     const double* __restrict__ minors,
                                                     const double* __restrict__ summ)
{
    const int w = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (w >= a.W) return;
    const Wt wt = full_weight(a, w, c, minors, summ);
    if (lane_id() == 0) {
        a.logw[w] = wt.lc;
        a.sign[w] = wt.sg;
    }
}

// Regression targets: y = log|c'| clipped below at (max - clip); g[r] = 2 (pred - y) / W.
__global__ __launch_bounds__(1024) void mc_loss_kernel(McArgs a, const float* __restrict__ logits, int Op,
                                                       const uint32_t* __restrict__ prop,
                                                       const double* __restrict__ logc, float* __restrict__ gbuf,
                                                       float* loss, double clip)
{
    __shared__ double red[1024 / 64];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int L2 = a.L * a.L, per_bin = a.n_tau / a.n_bin;
    double mx = -INFINITY;
    for (int r = tid; r < a.W; r += 1024) {
        const double y = logc[r];
        if (isfinite(y)) mx = fmax(mx, y);
    }
    mx = wave_max(mx);
    if (lane == 0) red[wv] = mx;
    __syncthreads();
    mx = -INFINITY;
    for (int i = 0; i < 16; ++i) mx = fmax(mx, red[i]);
    __syncthreads();
    const bool any = mx > -INFINITY;
    const double floor_y = mx - clip;
    double sum = 0.0;
    for (int r = tid; r < a.W; r += 1024) {
        float gr = 0.0f;
        if (any) {
            double y = logc[r];
            y = isfinite(y) ? fmax(y, floor_y) : floor_y;
            const uint32_t v = prop[r];
            const int s = (int)(v & 0xFFFFu), b = (int)(v >> 16) / per_bin;
            const double pred = (double)logits[(size_t)r * Op + s] + (double)logits[(size_t)r * Op + L2 + b];
            const double diff = pred - y;
            gr = (float)(2.0 * diff / a.W);
            sum += diff * diff;
        }
        gbuf[r] = gr;
    }
    for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o);
    if (lane == 0) red[wv] = sum;
    __syncthreads();
    if (tid == 0 && loss) {
        double s = 0.0;
        for (int i = 0; i < 16; ++i) s += red[i];
        loss[0] = (float)(s / (a.W > 0 ? a.W : 1));
    }
}

__global__ __launch_bounds__(256) void mc_dout_kernel(McArgs a, int Op, const uint32_t* __restrict__ prop,
                                                      const float* __restrict__ gbuf, float* __restrict__ dout)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)a.W * Op) return;
    const int r = (int)(i / Op), f = (int)(i % Op);
    const uint32_t v = prop[r];
    const int L2 = a.L * a.L;
    const int s = (int)(v & 0xFFFFu), b = (int)(v >> 16) / (a.n_tau / a.n_bin);
    dout[i] = (f == s || f == L2 + b) ? gbuf[r] : 0.0f;
}

unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

hipError_t mc_context_launch(const McArgs& a, int32_t* moved, uint16_t* feat, int dp, hipStream_t st)
{
    if (a.W == 0) return hipSuccess;
    hipLaunchKernelGGL(mc_context_kernel, dim3(blocks_for(a.W, kGrpWalkers)), dim3(256), 0, st, a, moved, feat, dp);
    return hipGetLastError();
}

hipError_t mc_propose_launch(const McArgs& a, const int32_t* moved, int32_t* moved_out, const float* logits,
                             int stride, uint32_t* prop, double* logq, double* mats, hipStream_t st)
{
    if (a.W == 0) return hipSuccess;
    if (logits) {
        if (moved_out) return hipErrorInvalidValue;   // the learned proposal takes the context's moved vertex
        hipLaunchKernelGGL(mc_propose_kernel, dim3(blocks_for(a.W, kWgWalkers)), dim3(64 * kWgWalkers), 0, st, a,
                           moved, logits, stride, prop, logq, mats);
    } else {
        hipLaunchKernelGGL(mc_propose_uniform_kernel, dim3(blocks_for(a.W, kWgWalkers)), dim3(256), 0, st, a, moved,
                           moved_out, prop, logq, mats);
    }
    return hipGetLastError();
}

hipError_t mc_gather_launch(const McArgs& a, double* mats, hipStream_t st)
{
    if (a.W == 0) return hipSuccess;
    hipLaunchKernelGGL(mc_gather_kernel, dim3(blocks_for(a.W, 4)), dim3(256), 0, st, a, mats);
    return hipGetLastError();
}

hipError_t mc_accept_launch(const McArgs& a, const int32_t* moved, const uint32_t* prop, const double* logq,
                            const double* c, const double* minors, const double* summ, double* logc_out,
                            uint8_t* acc_out, float* obs_logw, int8_t* obs_sign, hipStream_t st)
{
    if (a.W == 0) return hipSuccess;
    if (summ)
        hipLaunchKernelGGL(mc_accept_summ_kernel, dim3(blocks_for(a.W, 256)), dim3(256), 0, st, a, moved, prop, logq,
                           summ, logc_out, acc_out, obs_logw, obs_sign);
    else
        hipLaunchKernelGGL(mc_accept_kernel, dim3(blocks_for(a.W, 4)), dim3(256), 0, st, a, moved, prop, logq, c,
                           minors, logc_out, acc_out, obs_logw, obs_sign);
    return hipGetLastError();
}

hipError_t mc_set_launch(const McArgs& a, const double* c, const double* minors, const double* summ, hipStream_t st)
{
    if (a.W == 0) return hipSuccess;
    hipLaunchKernelGGL(mc_set_kernel, dim3(blocks_for(a.W, 4)), dim3(256), 0, st, a, c, minors, summ);
    return hipGetLastError();
}

hipError_t mc_loss_launch(const McArgs& a, const float* logits, int Op, const uint32_t* prop, const double* logc,
                          float* gbuf, float* dout, float* loss, double clip, hipStream_t st)
{
    if (a.W == 0) return hipSuccess;
    hipLaunchKernelGGL(mc_loss_kernel, dim3(1), dim3(1024), 0, st, a, logits, Op, prop, logc, gbuf, loss, clip);
    hipLaunchKernelGGL(mc_dout_kernel, dim3(blocks_for((int64_t)a.W * Op, 256)), dim3(256), 0, st, a, Op, prop, gbuf,
                       dout);
    return hipGetLastError();
}

}  // namespace apm
