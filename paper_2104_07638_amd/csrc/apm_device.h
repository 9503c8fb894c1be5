// apm_device.h -- scalar "fields" and wave-level helpers shared by the gfx950 kernels.
//
// A field bundles the arithmetic one variant of the principal-minor tree needs:
//   E   matrix element type held in LDS and registers (the Schur updates run in E)
//   R   type of the pivot reciprocal (fp64 in every variant: the pivot division,
//       the near-zero test and the shift stay in fp64, also on the fp32 paths)
//   Bs  running product of pivots ("base" of a tree node: the minor of its kept set)
//   V   value type in true units used by the post-order pivot corrections
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace apm {

constexpr int kWave = 64;

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Order this wavefront's own global stores before its later loads of the same addresses.
// Each block is a single wavefront, so workgroup scope suffices: it waits for the
// outstanding memory operations without the L2 write-back that an agent-scope fence costs.
__device__ __forceinline__ void wave_mem_fence() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup"); }

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p ? 1 : 0); }

__device__ __forceinline__ double wave_max(double v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}

// Largest of a non-negative double over the wavefront, by DPP within and across rows of 16
// lanes (a max-scan that leaves the total in lane 63; lanes with no source read 0), then
// read from lane 63.  All 64 lanes must be active.
template <int CTRL, int ROWMASK = 0xF>
__device__ __forceinline__ double dpp_max_nonneg(double v)
{
    const int lo = __double2loint(v), hi = __double2hiint(v);
    const int slo = __builtin_amdgcn_update_dpp(0, lo, CTRL, ROWMASK, 0xF, true);
    const int shi = __builtin_amdgcn_update_dpp(0, hi, CTRL, ROWMASK, 0xF, true);
    return fmax(v, __hiloint2double(shi, slo));
}

__device__ __forceinline__ double wave_max_nonneg(double v)
{
    v = dpp_max_nonneg<0x111>(v);        // row_shr:1
    v = dpp_max_nonneg<0x112>(v);        // row_shr:2
    v = dpp_max_nonneg<0x114>(v);        // row_shr:4
    v = dpp_max_nonneg<0x118>(v);        // row_shr:8
    v = dpp_max_nonneg<0x142, 0xA>(v);   // row_bcast:15
    v = dpp_max_nonneg<0x143, 0xC>(v);   // row_bcast:31
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ int wave_sum(int v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// 1/x in fp64: hardware reciprocal estimate refined by two Newton steps.
__device__ __forceinline__ double rcp64(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

// ---- pivot shift (Sec. II, pivot correction), shared by the Schur-complement trees ----------
constexpr int8_t kNoEv = 0;      // "no shifted pivot" marker in the one-byte shift-code tables

// Magnitude of the pivot shift: the power of two 2^(floor(log2(rmax * min(rmax, cmax)) / 2)
// + kShiftLog2), about min(sqrt(rmax cmax), rmax) / 16.  The correction
// det A[S] = det A~[S] - C det A[S \ {l}] loses about eps C / |row l| of the Hadamard bound
// of A[S] to cancellation, so C stays at or below the pivot row's scale; the sign alignment
// below keeps |p + C| >= |C|, so the right child's elements change by at most
// rmax cmax / |C| (at most 16 times the larger of the column scale and sqrt(rmax cmax)).
constexpr int kShiftLog2 = -4;

// A shift is recorded as one byte: code = 2 (de + kShiftBias) + (C < 0), with
// C = +-2^(es + de) in stored units (es: exponent of s = max |A_ij|) and de clamped to
// [1 - kShiftBias, 127 - kShiftBias] = [-119, 7]: shifts far below the matrix's largest
// entry (rows of a near-singular or strongly graded part) are more common than shifts
// above it, which need growth of the Schur complements beyond 2^11 s.  kNoEv (0) marks
// "no shift".
constexpr int kShiftBias = 120;

__device__ __forceinline__ double shift_value(int es, int code)
{
    const int u = code & 0xFF;
    const double C = ldexp(1.0, es + (u >> 1) - kShiftBias);
    return (u & 1) ? -C : C;
}

// Code of the shift of a pivot whose row / column (within the node's matrix, the pivot left
// out) have largest magnitudes rmax / cmax; neg: Re p < 0.
__device__ __forceinline__ int8_t shift_code(double rmax, double cmax, int es, bool neg)
{
    int de = kShiftLog2;
    const double pr = rmax * fmin(rmax, cmax);
    if (pr > 0.0) {
        int ep;
        (void)frexp(pr, &ep);
        de = (ep >> 1) + kShiftLog2 - es;
    }
    de = de < 1 - kShiftBias ? 1 - kShiftBias : (de > 127 - kShiftBias ? 127 - kShiftBias : de);
    return (int8_t)(uint8_t)(2 * (de + kShiftBias) + (neg ? 1 : 0));
}

// Complex values aligned to their size, so that one 16-byte (8-byte) LDS or global access
// moves a whole value: paired half-size LDS accesses of a padded row fall on the same
// banks every eight rows.
struct alignas(16) cd { double x, y; };
struct alignas(8) cf { float x, y; };

__device__ __forceinline__ cd operator*(cd a, cd b) { return {fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x)}; }
__device__ __forceinline__ cd operator-(cd a, cd b) { return {a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ cd operator*(double s, cd a) { return {s * a.x, s * a.y}; }

// running product with a separate binary exponent: value = m * 2^e, |m| in [0.5, 1) or m == 0
struct SBr { float m; int e; };
struct SBc { cf m; int e; };

// ------------------------------------------------------------------------------- R64
struct FR64 {
    static constexpr int kId = 0;   // apm_dtype
    using In = double;
    using E = double;
    using R = double;
    using Bs = double;
    using V = double;
    static constexpr bool kScaled = false;
    static constexpr bool kComplex = false;
    __device__ static double in_mag(In v) { return fabs(v); }
    __device__ static bool in_finite(In v) { return isfinite(v); }
    __device__ static E conv(In v, double sc) { return v; }
    __device__ static double mag(E p) { return fabs(p); }
    __device__ static double re(E p) { return p; }
    __device__ static E shift(E p, double C) { return p + C; }
    __device__ static R recip(E p) { return rcp64(p); }
    __device__ static E rowscale(E v, R r) { return v * r; }
    __device__ static E det2(E p, E r, E c, E d) { return fma(p, d, -c * r); }   // p d - c r
    __device__ static E zero() { return 0.0; }
    __device__ static E upd(E a, E c, E w) { return fma(-c, w, a); }
    __device__ static Bs one() { return 1.0; }
    __device__ static Bs bmul(Bs b, E p, int) { return b * p; }
    __device__ static void store(void* out, int16_t*, int64_t i, Bs v, bool)
    {
        static_cast<double*>(out)[i] = v;
    }
    __device__ static void* optr(void* out, int64_t i, bool) { return static_cast<double*>(out) + i; }
    __device__ static void store_rel(void* p, int16_t*, int r, Bs v, bool) { static_cast<double*>(p)[r] = v; }
    __device__ static double fincheck(Bs v) { return v * 0.0; }
    __device__ static V load_v(const void* out, const int16_t*, int64_t i, bool)
    {
        return static_cast<const double*>(out)[i];
    }
    __device__ static void store_v(void* out, int16_t*, int64_t i, V v, bool)
    {
        static_cast<double*>(out)[i] = v;
    }
    __device__ static V sub_scaled(V a, double C, V b) { return fma(-C, b, a); }
    __device__ static void store_nan(void* out, int16_t*, int64_t i, bool)
    {
        static_cast<double*>(out)[i] = __builtin_nan("");
    }
};

// ------------------------------------------------------------------------------- R32S
// fp32 Schur updates, fp64 pivot reciprocal/test/shift, float mantissa + int exponent product.
struct FR32S {
    static constexpr int kId = 1;   // apm_dtype
    using In = double;
    using E = float;
    using R = double;
    using Bs = SBr;
    using V = double;
    static constexpr bool kScaled = true;
    static constexpr bool kComplex = false;
    __device__ static double in_mag(In v) { return fabs(v); }
    __device__ static bool in_finite(In v) { return isfinite(v); }
    __device__ static E conv(In v, double sc) { return (float)(v * sc); }
    __device__ static double mag(E p) { return fabs((double)p); }
    __device__ static double re(E p) { return (double)p; }
    __device__ static E shift(E p, double C) { return (float)((double)p + C); }
    __device__ static R recip(E p) { return rcp64((double)p); }
    __device__ static E rowscale(E v, R r) { return (float)((double)v * r); }
    // p d - c r with exact fp64 products of the fp32 operands, one rounding to fp32
    __device__ static E det2(E p, E r, E c, E d) { return (float)fma((double)p, (double)d, -((double)c * (double)r)); }
    __device__ static E zero() { return 0.0f; }
    __device__ static E upd(E a, E c, E w) { return fmaf(-c, w, a); }
    __device__ static Bs one() { return {0.5f, 1}; }
    __device__ static Bs bmul(Bs b, E p, int e0)
    {
        float m = b.m * p;
        int ee;
        m = frexpf(m, &ee);
        return {m, b.e + ee + e0};
    }
    __device__ static void store(void* out, int16_t* ex, int64_t i, Bs v, bool f64)
    {
        if (f64) {
            static_cast<double*>(out)[i] = ldexp((double)v.m, v.e);
        } else {
            static_cast<float*>(out)[i] = v.m;
            ex[i] = (int16_t)v.e;
        }
    }
    __device__ static void* optr(void* out, int64_t i, bool f64)
    {
        return f64 ? (void*)(static_cast<double*>(out) + i) : (void*)(static_cast<float*>(out) + i);
    }
    __device__ static void store_rel(void* p, int16_t* e, int r, Bs v, bool f64)
    {
        if (f64) {
            static_cast<double*>(p)[r] = ldexp((double)v.m, v.e);
        } else {
            static_cast<float*>(p)[r] = v.m;
            e[r] = (int16_t)v.e;
        }
    }
    __device__ static double fincheck(Bs v) { return (double)(v.m * 0.0f); }
    __device__ static V load_v(const void* out, const int16_t* ex, int64_t i, bool f64)
    {
        if (f64) return static_cast<const double*>(out)[i];
        float m = static_cast<const float*>(out)[i];
        int16_t e = ex[i];
        return ldexp((double)m, (int)e);
    }
    __device__ static void store_v(void* out, int16_t* ex, int64_t i, V v, bool f64)
    {
        if (f64) {
            static_cast<double*>(out)[i] = v;
        } else {
            int ee;
            double m = frexp(v, &ee);
            float mf = (float)m;
            if (fabsf(mf) == 1.0f) { mf *= 0.5f; ++ee; }
            static_cast<float*>(out)[i] = mf;
            ex[i] = (int16_t)(mf == 0.0f ? 0 : ee);
        }
    }
    __device__ static V sub_scaled(V a, double C, V b) { return fma(-C, b, a); }
    __device__ static void store_nan(void* out, int16_t* ex, int64_t i, bool f64)
    {
        if (f64) {
            static_cast<double*>(out)[i] = __builtin_nan("");
        } else {
            static_cast<float*>(out)[i] = __builtin_nanf("");
            ex[i] = 0;
        }
    }
};

// ------------------------------------------------------------------------------- C128
struct FC128 {
    static constexpr int kId = 2;   // apm_dtype
    using In = cd;
    using E = cd;
    using R = cd;
    using Bs = cd;
    using V = cd;
    static constexpr bool kScaled = false;
    static constexpr bool kComplex = true;
    __device__ static double in_mag(In v) { return fmax(fabs(v.x), fabs(v.y)); }
    __device__ static bool in_finite(In v) { return isfinite(v.x) && isfinite(v.y); }
    __device__ static E conv(In v, double) { return v; }
    __device__ static double mag(E p) { return fmax(fabs(p.x), fabs(p.y)); }
    __device__ static double re(E p) { return p.x; }
    __device__ static E shift(E p, double C) { return {p.x + C, p.y}; }
    // 1/p = conj(p) / |p|^2, with p scaled by the power of two 2^-k nearest its larger
    // component before squaring, so that |p|^2 neither overflows nor underflows for any
    // representable pivot: 1/p = 2^-k conj(q) / |q|^2, q = 2^-k p.
    __device__ static R recip(E p)
    {
        int k = 0;
        (void)frexp(fmax(fabs(p.x), fabs(p.y)), &k);
        const double qx = ldexp(p.x, -k), qy = ldexp(p.y, -k);
        const double d = ldexp(rcp64(fma(qx, qx, qy * qy)), -k);
        return {qx * d, -qy * d};
    }
    __device__ static E rowscale(E v, R r) { return v * r; }
    __device__ static E det2(E p, E r, E c, E d)
    {
        return {fma(p.x, d.x, fma(-p.y, d.y, fma(-c.x, r.x, c.y * r.y))),
                fma(p.x, d.y, fma(p.y, d.x, fma(-c.x, r.y, -c.y * r.x)))};
    }
    __device__ static E zero() { return {0.0, 0.0}; }
    __device__ static E upd(E a, E c, E w)
    {
        // a - c * w
        return {fma(-c.x, w.x, fma(c.y, w.y, a.x)), fma(-c.x, w.y, fma(-c.y, w.x, a.y))};
    }
    __device__ static Bs one() { return {1.0, 0.0}; }
    __device__ static Bs bmul(Bs b, E p, int) { return b * p; }
    __device__ static void store(void* out, int16_t*, int64_t i, Bs v, bool)
    {
        static_cast<cd*>(out)[i] = v;
    }
    __device__ static void* optr(void* out, int64_t i, bool) { return static_cast<cd*>(out) + i; }
    __device__ static void store_rel(void* p, int16_t*, int r, Bs v, bool) { static_cast<cd*>(p)[r] = v; }
    __device__ static double fincheck(Bs v) { return v.x * 0.0 + v.y * 0.0; }
    __device__ static V load_v(const void* out, const int16_t*, int64_t i, bool)
    {
        const double* p = static_cast<const double*>(out) + 2 * i;
        return {p[0], p[1]};
    }
    __device__ static void store_v(void* out, int16_t*, int64_t i, V v, bool)
    {
        static_cast<cd*>(out)[i] = v;
    }
    __device__ static V sub_scaled(V a, double C, V b) { return {fma(-C, b.x, a.x), fma(-C, b.y, a.y)}; }
    __device__ static void store_nan(void* out, int16_t*, int64_t i, bool)
    {
        static_cast<cd*>(out)[i] = {__builtin_nan(""), __builtin_nan("")};
    }
};

// ------------------------------------------------------------------------------- C64S
// complex64 Schur updates; fp64 pivot reciprocal/test/shift; complex mantissa + exponent.
struct FC64S {
    static constexpr int kId = 3;   // apm_dtype
    using In = cd;
    using E = cf;
    using R = cd;
    using Bs = SBc;
    using V = cd;
    static constexpr bool kScaled = true;
    static constexpr bool kComplex = true;
    __device__ static double in_mag(In v) { return fmax(fabs(v.x), fabs(v.y)); }
    __device__ static bool in_finite(In v) { return isfinite(v.x) && isfinite(v.y); }
    __device__ static E conv(In v, double sc) { return {(float)(v.x * sc), (float)(v.y * sc)}; }
    __device__ static double mag(E p) { return (double)fmaxf(fabsf(p.x), fabsf(p.y)); }
    __device__ static double re(E p) { return (double)p.x; }
    __device__ static E shift(E p, double C) { return {(float)((double)p.x + C), p.y}; }
    __device__ static R recip(E p)
    {
        double px = p.x, py = p.y;
        double d = rcp64(fma(px, px, py * py));
        return {px * d, -py * d};
    }
    __device__ static E rowscale(E v, R r)
    {
        double vx = v.x, vy = v.y;
        return {(float)fma(vx, r.x, -vy * r.y), (float)fma(vx, r.y, vy * r.x)};
    }
    __device__ static E det2(E p, E r, E c, E d)
    {
        const double px = p.x, py = p.y, dx = d.x, dy = d.y, cx = c.x, cy = c.y, rx = r.x, ry = r.y;
        return {(float)fma(px, dx, fma(-py, dy, fma(-cx, rx, cy * ry))),
                (float)fma(px, dy, fma(py, dx, fma(-cx, ry, -cy * rx)))};
    }
    __device__ static E zero() { return {0.0f, 0.0f}; }
    __device__ static E upd(E a, E c, E w)
    {
        return {fmaf(-c.x, w.x, fmaf(c.y, w.y, a.x)), fmaf(-c.x, w.y, fmaf(-c.y, w.x, a.y))};
    }
    __device__ static Bs one() { return {{0.5f, 0.0f}, 1}; }
    __device__ static Bs bmul(Bs b, E p, int e0)
    {
        cf m = {fmaf(b.m.x, p.x, -b.m.y * p.y), fmaf(b.m.x, p.y, b.m.y * p.x)};
        float big = fmaxf(fabsf(m.x), fabsf(m.y));
        int ee;
        (void)frexpf(big, &ee);
        m.x = ldexpf(m.x, -ee);
        m.y = ldexpf(m.y, -ee);
        return {m, b.e + ee + e0};
    }
    __device__ static void store(void* out, int16_t* ex, int64_t i, Bs v, bool f64)
    {
        if (f64) {
            static_cast<cd*>(out)[i] = {ldexp((double)v.m.x, v.e), ldexp((double)v.m.y, v.e)};
        } else {
            static_cast<cf*>(out)[i] = v.m;
            ex[i] = (int16_t)v.e;
        }
    }
    __device__ static void* optr(void* out, int64_t i, bool f64)
    {
        return f64 ? (void*)(static_cast<cd*>(out) + i) : (void*)(static_cast<cf*>(out) + i);
    }
    __device__ static void store_rel(void* p, int16_t* e, int r, Bs v, bool f64)
    {
        if (f64) {
            static_cast<cd*>(p)[r] = {ldexp((double)v.m.x, v.e), ldexp((double)v.m.y, v.e)};
        } else {
            static_cast<cf*>(p)[r] = v.m;
            e[r] = (int16_t)v.e;
        }
    }
    __device__ static double fincheck(Bs v) { return (double)(v.m.x * 0.0f + v.m.y * 0.0f); }
    __device__ static V load_v(const void* out, const int16_t* ex, int64_t i, bool f64)
    {
        if (f64) {
            const double* p = static_cast<const double*>(out) + 2 * i;
            return {p[0], p[1]};
        }
        const float* p = static_cast<const float*>(out) + 2 * i;
        int e = ex[i];
        return {ldexp((double)p[0], e), ldexp((double)p[1], e)};
    }
    __device__ static void store_v(void* out, int16_t* ex, int64_t i, V v, bool f64)
    {
        if (f64) {
            static_cast<cd*>(out)[i] = v;
        } else {
            double big = fmax(fabs(v.x), fabs(v.y));
            int ee = 0;
            if (big != 0.0) (void)frexp(big, &ee);
            cf m = {(float)ldexp(v.x, -ee), (float)ldexp(v.y, -ee)};
            if (fmaxf(fabsf(m.x), fabsf(m.y)) >= 1.0f) { m.x *= 0.5f; m.y *= 0.5f; ++ee; }
            static_cast<cf*>(out)[i] = m;
            ex[i] = (int16_t)ee;
        }
    }
    __device__ static V sub_scaled(V a, double C, V b) { return {fma(-C, b.x, a.x), fma(-C, b.y, a.y)}; }
    __device__ static void store_nan(void* out, int16_t* ex, int64_t i, bool f64)
    {
        if (f64) {
            static_cast<cd*>(out)[i] = {__builtin_nan(""), __builtin_nan("")};
        } else {
            static_cast<cf*>(out)[i] = {__builtin_nanf(""), __builtin_nanf("")};
            ex[i] = 0;
        }
    }
};

}  // namespace apm
