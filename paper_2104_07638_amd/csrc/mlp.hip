// mlp.hip -- the proposal network on the gfx950 matrix cores: BF16 operands, fp32 sums.
//
// Network: h1 = tanh(W1 x + b1), h2 = tanh(W2 h1 + b2), out = W3 h2 + b3, hidden width
// 128.  Every product is computed transposed, Z^T = W H^T, with v_mfma_f32_16x16x16_bf16:
//   A operand (16 x 16, M x K): lane l holds A[l % 16][4 (l / 16) + 0..3]
//   B operand (16 x 16, K x N): lane l holds B[4 (l / 16) + 0..3][l % 16]
//   D result  (16 x 16, M x N): lane l holds D[4 (l / 16) + 0..3][l % 16]
// With the weights as A and the activations (features x batch) as B, the D tile of 16
// output features is exactly the B operand of the next layer's k-step over those
// features.  The forward pass runs one workgroup per 32 batch rows (two N tiles sharing
// every weight load); its wavefronts split each layer's output features and pass the
// activations on through LDS.
//
// The forward pass reads its BF16 weights (net.w) in that A-operand order: for a layer of
// M x K weights, tile (mt, ks) (rows 16 mt.., columns 16 ks..) is 64 lanes x 4 values stored
// contiguously from ((mt (K / 16) + ks) 64 + lane) 4, so that one load instruction of a
// wavefront reads 512 consecutive bytes (from row-major rows it would touch 16 cache lines).
//
// Backward: the hidden gradients are chained the same way through the transposed
// weights (W^T kept as a second BF16 copy); the weight gradients dW = dZ^T H sum over
// the batch, one wavefront per 16 x 16 tile of dW with the batch as the K dimension,
// from BF16 copies of dZ and H stored feature-major ([feature][batch]).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "apm_kernels.h"

namespace apm {
namespace {

constexpr int H = 128;

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);   // round to nearest, ties to even
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ v4s pack_bf(v4f v)
{
    v4s r;
    r[0] = (short)f2bf(v[0]);
    r[1] = (short)f2bf(v[1]);
    r[2] = (short)f2bf(v[2]);
    r[3] = (short)f2bf(v[3]);
    return r;
}

__device__ __forceinline__ float bf2f(short b) { return __uint_as_float(((uint32_t)(uint16_t)b) << 16); }

__device__ __forceinline__ float tanh_f(float z)
{
    const float e = __expf(2.0f * z);   // inf for large z gives 1, 0 for very negative z gives -1
    return 1.0f - 2.0f / (e + 1.0f);
}

__device__ __forceinline__ v4f mfma(v4s a, v4s b, v4f c)
{
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ v4s ld4(const uint16_t* p) { return *reinterpret_cast<const v4s*>(p); }

// store the 4 values a lane holds for (features f0..f0+3, batch row r) feature-major
__device__ __forceinline__ void store_t(uint16_t* dst, int B, int f0, int r, v4s v)
{
#pragma unroll
    for (int j = 0; j < 4; ++j) dst[(size_t)(f0 + j) * B + r] = (uint16_t)v[j];
}

// Forward pass: one workgroup of kFwdWaves wavefronts per 32 batch rows.  The wavefronts
// split the output features of every layer (wave v computes hidden tiles kMtPerWave v.. and
// output tiles v, v + kFwdWaves, ...) and exchange the BF16 activations through LDS between
// layers, already in B-operand order.  Each wavefront needs only its slice of the weights and
// loads all of it up front (straight from L2, one batch of independent loads), so the three
// layers wait for memory once.  The kernel is latency-bound (one workgroup per CU at the
// Monte Carlo batch); eight wavefronts measured faster than four (fewer output tiles each).
#ifndef APM_MLP_FWD_WAVES
#define APM_MLP_FWD_WAVES 8
#endif
#ifndef APM_MLP_W3PRE
#define APM_MLP_W3PRE 3
#endif
constexpr int kFwdWaves = APM_MLP_FWD_WAVES;   // 2, 4 or 8
constexpr int kMtPerWave = 8 / kFwdWaves;
constexpr int kW3Pre = APM_MLP_W3PRE;    // output tiles per wavefront whose weights are loaded up front
static_assert(kFwdWaves == 2 || kFwdWaves == 4 || kFwdWaves == 8, "hidden tiles split evenly over the wavefronts");

// This lane's A operands of row tile mt (k-steps 0..KS-1) of a layer, from the
// fragment-ordered weights: one address per tile, the k-steps at constant offsets of 512 B.
template <int KS>
__device__ __forceinline__ void load_tile(const uint16_t* __restrict__ W, int mt, v4s (&a)[KS])
{
    const uint16_t* p = W + (size_t)(uint32_t)mt * (KS * 256) + (threadIdx.x & 63) * 4;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) a[ks] = ld4(p + ks * 256);
}

template <int KS>
__device__ __forceinline__ void load_slice(const uint16_t* __restrict__ W, int mt0, v4s (&a)[kMtPerWave][KS])
{
#pragma unroll
    for (int m = 0; m < kMtPerWave; ++m) load_tile<KS>(W, mt0 + m, a[m]);
}

// the biases of this lane's features 16 (mt0 + m) + 4 (lane / 16) + 0..3 of the hidden tiles
// mt0 .. mt0+kMtPerWave-1
__device__ __forceinline__ void load_bias(const float* __restrict__ b, int mt0, v4f (&bb)[kMtPerWave])
{
    const int g = (threadIdx.x & 63) >> 4;
#pragma unroll
    for (int m = 0; m < kMtPerWave; ++m) bb[m] = *reinterpret_cast<const v4f*>(b + 16 * (mt0 + m) + 4 * g);
}

// tanh(W in + b) for the hidden tiles mt0 .. mt0+kMtPerWave-1 of both row tiles (bb: their
// biases, from load_bias)
template <int KS>
__device__ __forceinline__ void hidden_slice(const v4s (&a)[kMtPerWave][KS], const v4f (&bb)[kMtPerWave],
                                             const v4s (&in)[2][KS], int mt0, v4s* act_out, int row0, int B,
                                             float* save, uint16_t* save_t)
{
    const int lane = threadIdx.x & 63, r16 = lane & 15, g = lane >> 4;
#pragma unroll
    for (int m = 0; m < kMtPerWave; ++m) {
        const int mt = mt0 + m;
        v4f a0 = {0.f, 0.f, 0.f, 0.f}, a1 = a0;
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            a0 = mfma(a[m][ks], in[0][ks], a0);
            a1 = mfma(a[m][ks], in[1][ks], a1);
        }
        const int f0 = 16 * mt + 4 * g;
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
            const v4f z = (nt == 0 ? a0 : a1) + bb[m];
            v4f h;
            h[0] = tanh_f(z[0]);
            h[1] = tanh_f(z[1]);
            h[2] = tanh_f(z[2]);
            h[3] = tanh_f(z[3]);
            const v4s hb = pack_bf(h);
            act_out[(mt * 2 + nt) * 64 + lane] = hb;
            const int r = row0 + 16 * nt + r16;
            if (save) *reinterpret_cast<v4f*>(save + (size_t)r * H + f0) = h;
            if (save_t) store_t(save_t, B, f0, r, hb);
        }
    }
}

template <int KS1>
__global__ __launch_bounds__(64 * kFwdWaves) void mlp_fwd_kernel(const uint16_t* __restrict__ w,
                                                                 const float* __restrict__ bias,
                                                                 const uint16_t* __restrict__ x, int B, int Op,
                                                                 float* __restrict__ out, float* h1s, float* h2s,
                                                                 uint16_t* actT)
{
    constexpr int DP = 16 * KS1;
    __shared__ v4s act1[8 * 2 * 64], act2[8 * 2 * 64];   // [feature tile][row tile][lane]
    const int lane = threadIdx.x & 63, r16 = lane & 15, g = lane >> 4, wv = threadIdx.x >> 6;
    const int row0 = blockIdx.x * 32;
    const uint16_t* W1 = w;
    const uint16_t* W2 = W1 + H * DP;
    const uint16_t* W3 = W2 + H * H;

    const int ntile = Op / 16;
    const float* b3 = bias + 2 * H;
    // every input, weight and bias this wavefront uses (a slice of each layer) is requested up
    // front, in the order the layers need them, so that each layer waits only for its own
    // operands and the three layers wait for memory about once
    v4s xo[2][KS1];
#pragma unroll
    for (int nt = 0; nt < 2; ++nt)
#pragma unroll
        for (int ks = 0; ks < KS1; ++ks) xo[nt][ks] = ld4(x + (size_t)(row0 + 16 * nt + r16) * DP + 16 * ks + 4 * g);
    v4s w1[kMtPerWave][KS1], w2[kMtPerWave][8], w3[kW3Pre][8];
    v4f bb1[kMtPerWave], bb2[kMtPerWave], bb3[kW3Pre];
    load_slice<KS1>(W1, kMtPerWave * wv, w1);
    load_bias(bias, kMtPerWave * wv, bb1);
    __builtin_amdgcn_sched_barrier(0);   // keep this issue order (the scheduler groups loads by size)
    load_slice<8>(W2, kMtPerWave * wv, w2);
    load_bias(bias + H, kMtPerWave * wv, bb2);
    __builtin_amdgcn_sched_barrier(0);
    // (tiles past the last one load the last tile again, unused: unconditional loads keep the
    // compiler's count of loads in flight exact, so no wait covers more than it needs)
#pragma unroll
    for (int u = 0; u < kW3Pre; ++u) {
        const int t = min(wv + u * kFwdWaves, ntile - 1);
        load_tile<8>(W3, t, w3[u]);
        bb3[u] = *reinterpret_cast<const v4f*>(b3 + 16 * t + 4 * g);
    }
    if (actT && wv == 0) {   // training: feature-major BF16 copy of the input
#pragma unroll
        for (int nt = 0; nt < 2; ++nt)
#pragma unroll
            for (int ks = 0; ks < KS1; ++ks) store_t(actT, B, 16 * ks + 4 * g, row0 + 16 * nt + r16, xo[nt][ks]);
    }
    hidden_slice<KS1>(w1, bb1, xo, kMtPerWave * wv, act1, row0, B, h1s, actT ? actT + (size_t)DP * B : nullptr);
    __syncthreads();

    v4s h1o[2][8];
#pragma unroll
    for (int kt = 0; kt < 8; ++kt)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) h1o[nt][kt] = act1[(kt * 2 + nt) * 64 + lane];
    hidden_slice<8>(w2, bb2, h1o, kMtPerWave * wv, act2, row0, B, h2s, actT ? actT + (size_t)(DP + H) * B : nullptr);
    __syncthreads();

    v4s h2o[2][8];
#pragma unroll
    for (int kt = 0; kt < 8; ++kt)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) h2o[nt][kt] = act2[(kt * 2 + nt) * 64 + lane];
    auto out_tile = [&](int t, const v4s (&a)[8], v4f bb) {
        v4f a0 = {0.f, 0.f, 0.f, 0.f}, a1 = a0;
#pragma unroll
        for (int ks = 0; ks < 8; ++ks) {
            a0 = mfma(a[ks], h2o[0][ks], a0);
            a1 = mfma(a[ks], h2o[1][ks], a1);
        }
        const int f0 = 16 * t + 4 * g;
        *reinterpret_cast<v4f*>(out + (size_t)(row0 + r16) * Op + f0) = a0 + bb;
        *reinterpret_cast<v4f*>(out + (size_t)(row0 + 16 + r16) * Op + f0) = a1 + bb;
    };
#pragma unroll
    for (int u = 0; u < kW3Pre; ++u) {
        const int t = wv + u * kFwdWaves;
        if (t < ntile) out_tile(t, w3[u], bb3[u]);
    }
    // tiles beyond the preloaded ones (wide output layers)
    for (int t = wv + kW3Pre * kFwdWaves; t < ntile; t += kFwdWaves) {
        v4s a[8];
        load_tile<8>(W3, t, a);
        out_tile(t, a, *reinterpret_cast<const v4f*>(b3 + 16 * t + 4 * g));
    }
}

// dz2 = (W3^T dout^T) * (1 - h2^2), dz1 = (W2^T dz2^T) * (1 - h1^2); BF16 feature-major
// copies of dout, dz2 and dz1 go to gT = [Op | H | H][B].
__global__ __launch_bounds__(64) void mlp_bwd_act_kernel(const uint16_t* __restrict__ wt, int DP, int Op,
                                                         const float* __restrict__ dout, int B,
                                                         const float* __restrict__ h1s,
                                                         const float* __restrict__ h2s, uint16_t* __restrict__ gT)
{
    const int lane = threadIdx.x & 63, r16 = lane & 15, g = lane >> 4;
    const int row0 = blockIdx.x * 32;
    const uint16_t* W2T = wt + (size_t)H * DP;        // [H][H]
    const uint16_t* W3T = W2T + H * H;                // [H][Op]
    uint16_t* doT = gT;
    uint16_t* dz2T = gT + (size_t)Op * B;
    uint16_t* dz1T = dz2T + (size_t)H * B;

    v4f acc[8][2];
#pragma unroll
    for (int mt = 0; mt < 8; ++mt) acc[mt][0] = acc[mt][1] = v4f{0.f, 0.f, 0.f, 0.f};
    for (int ks = 0; ks < Op / 16; ++ks) {
        v4s bo[2];
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
            const int r = row0 + 16 * nt + r16;
            bo[nt] = pack_bf(*reinterpret_cast<const v4f*>(dout + (size_t)r * Op + 16 * ks + 4 * g));
            store_t(doT, B, 16 * ks + 4 * g, r, bo[nt]);
        }
#pragma unroll
        for (int mt = 0; mt < 8; ++mt) {
            const v4s a = ld4(W3T + (size_t)(16 * mt + r16) * Op + 16 * ks + 4 * g);
            acc[mt][0] = mfma(a, bo[0], acc[mt][0]);
            acc[mt][1] = mfma(a, bo[1], acc[mt][1]);
        }
    }
    v4s dz2o[2][8];
#pragma unroll
    for (int mt = 0; mt < 8; ++mt)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
            const int r = row0 + 16 * nt + r16;
            const int f0 = 16 * mt + 4 * g;
            const v4f h = *reinterpret_cast<const v4f*>(h2s + (size_t)r * H + f0);
            const v4f dz = acc[mt][nt] * (1.0f - h * h);
            dz2o[nt][mt] = pack_bf(dz);
            store_t(dz2T, B, f0, r, dz2o[nt][mt]);
        }
#pragma unroll
    for (int mt = 0; mt < 8; ++mt) {
        v4f a0 = {0.f, 0.f, 0.f, 0.f}, a1 = a0;
#pragma unroll
        for (int ks = 0; ks < 8; ++ks) {
            const v4s a = ld4(W2T + (size_t)(16 * mt + r16) * H + 16 * ks + 4 * g);
            a0 = mfma(a, dz2o[0][ks], a0);
            a1 = mfma(a, dz2o[1][ks], a1);
        }
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
            const int r = row0 + 16 * nt + r16;
            const int f0 = 16 * mt + 4 * g;
            const v4f h = *reinterpret_cast<const v4f*>(h1s + (size_t)r * H + f0);
            const v4f dz = (nt == 0 ? a0 : a1) * (1.0f - h * h);
            store_t(dz1T, B, f0, r, pack_bf(dz));
        }
    }
}

// dW[f][k] = sum_r dZ[r][f] act[r][k] and db[f] = sum_r dZ[r][f], one 16 x 16 tile of dW per
// wavefront.  Tiles: layer 3 (Op/16 x 8), then layer 2 (8 x 8), then layer 1 (8 x DP/16).
__global__ __launch_bounds__(64) void mlp_wgrad_kernel(const uint16_t* __restrict__ gT,
                                                       const uint16_t* __restrict__ actT, int B, int DP, int Op,
                                                       float* __restrict__ grad)
{
    const int lane = threadIdx.x & 63, r16 = lane & 15, g = lane >> 4;
    const int T3 = (Op / 16) * 8;
    int t = blockIdx.x;
    const uint16_t* A;     // dZ^T [f][B]
    const uint16_t* Bm;    // act^T [k][B]
    float* dW;
    float* db;
    int ld, it, kt;
    float* bias = grad + (size_t)H * DP + H * H + (size_t)Op * H;
    if (t < T3) {
        it = t / 8;
        kt = t % 8;
        A = gT;
        Bm = actT + (size_t)(DP + H) * B;
        dW = grad + (size_t)H * DP + H * H;
        ld = H;
        db = bias + 2 * H;
    } else if (t < T3 + 64) {
        t -= T3;
        it = t / 8;
        kt = t % 8;
        A = gT + (size_t)Op * B;
        Bm = actT + (size_t)DP * B;
        dW = grad + (size_t)H * DP;
        ld = H;
        db = bias + H;
    } else {
        t -= T3 + 64;
        const int kt1 = DP / 16;
        it = t / kt1;
        kt = t % kt1;
        A = gT + (size_t)(Op + H) * B;
        Bm = actT;
        dW = grad;
        ld = DP;
        db = bias;
    }
    const uint16_t* pa = A + (size_t)(16 * it + r16) * B + 4 * g;
    const uint16_t* pb = Bm + (size_t)(16 * kt + r16) * B + 4 * g;
    v4f c0 = {0.f, 0.f, 0.f, 0.f}, c1 = c0;
    float bs = 0.f;
    for (int r0 = 0; r0 < B; r0 += 32) {
        const v4s a0 = ld4(pa + r0), b0 = ld4(pb + r0);
        const v4s a1 = ld4(pa + r0 + 16), b1 = ld4(pb + r0 + 16);
        c0 = mfma(a0, b0, c0);
        c1 = mfma(a1, b1, c1);
        if (kt == 0)
            bs += (bf2f(a0[0]) + bf2f(a0[1])) + (bf2f(a0[2]) + bf2f(a0[3])) + (bf2f(a1[0]) + bf2f(a1[1])) +
                  (bf2f(a1[2]) + bf2f(a1[3]));
    }
    const v4f c = c0 + c1;
#pragma unroll
    for (int j = 0; j < 4; ++j) dW[(size_t)(16 * it + 4 * g + j) * ld + 16 * kt + r16] = c[j];
    if (kt == 0) {
        bs += __shfl_xor(bs, 16);
        bs += __shfl_xor(bs, 32);
        if (g == 0) db[16 * it + r16] = bs;
    }
}

// Adam step (update != 0) and/or refresh of the BF16 copies w and wt from param.
__global__ __launch_bounds__(256) void mlp_adam_kernel(float* __restrict__ p, const float* __restrict__ gr,
                                                       float* __restrict__ m, float* __restrict__ v,
                                                       uint16_t* __restrict__ w, uint16_t* __restrict__ wt,
                                                       int64_t P, int DP, int Op, int update, float lr, float b1,
                                                       float b2, float eps, float c1, float c2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P) return;
    float x = p[i];
    if (update) {
        const float gi = gr[i];
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        x -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
        p[i] = x;
    }
    const int64_t s2 = (int64_t)H * DP, s3 = s2 + H * H, nw = s3 + (int64_t)Op * H;
    if (i < nw) {
        const uint16_t bits = f2bf(x);
        // element (row, col) of the M x K layer at `base`: fragment copy at
        // ((row/16 (K/16) + col/16) 64 + lane) 4 + col % 4, lane = 16 ((col % 16) / 4) + row % 16;
        // transposed copy at col M + row
        int64_t base, K, M;
        if (i < s2) {
            base = 0, K = DP, M = H;
        } else if (i < s3) {
            base = s2, K = H, M = H;
        } else {
            base = s3, K = H, M = Op;
        }
        const int64_t row = (i - base) / K, col = (i - base) % K;
        const int64_t lane = 16 * ((col & 15) >> 2) + (row & 15);
        w[base + (((row >> 4) * (K >> 4) + (col >> 4)) * 64 + lane) * 4 + (col & 3)] = bits;
        wt[base + col * M + row] = bits;
    }
}

}  // namespace

int64_t mlp_param_count(int dp, int op) { return (int64_t)H * dp + H * H + (int64_t)op * H + H + H + op; }
int64_t mlp_weight_count(int dp, int op) { return (int64_t)H * dp + H * H + (int64_t)op * H; }

int64_t mlp_work_bytes(int dp, int op, int B)
{
    const int64_t f32 = 2 * (int64_t)B * H * 4;                       // h1, h2 fp32 [B][H]
    const int64_t act = (int64_t)(dp + 2 * H) * B * 2;                // x^T, h1^T, h2^T bf16
    const int64_t gra = (int64_t)(op + 2 * H) * B * 2;                // dout^T, dz2^T, dz1^T bf16
    auto al = [](int64_t v) { return (v + 255) & ~(int64_t)255; };
    return al(f32) + al(act) + al(gra);
}

MlpWork mlp_work_carve(void* work, int dp, int op, int B)
{
    auto al = [](int64_t v) { return (v + 255) & ~(int64_t)255; };
    char* p = static_cast<char*>(work);
    MlpWork wk;
    wk.h1 = reinterpret_cast<float*>(p);
    wk.h2 = wk.h1 + (size_t)B * H;
    p += al(2 * (int64_t)B * H * 4);
    wk.actT = reinterpret_cast<uint16_t*>(p);
    p += al((int64_t)(dp + 2 * H) * B * 2);
    wk.gT = reinterpret_cast<uint16_t*>(p);
    return wk;
}

hipError_t mlp_forward_launch(const MlpNet& net, const uint16_t* x, int B, float* out, const MlpWork* wk,
                              hipStream_t st)
{
    if (B == 0) return hipSuccess;
    const float* bias = net.param + mlp_weight_count(net.dp, net.op);
    float* h1 = wk ? wk->h1 : nullptr;
    float* h2 = wk ? wk->h2 : nullptr;
    uint16_t* actT = wk ? wk->actT : nullptr;
    const dim3 grid((unsigned)(B / 32)), block(64 * kFwdWaves);
    switch (net.dp / 16) {
    case 1: hipLaunchKernelGGL(mlp_fwd_kernel<1>, grid, block, 0, st, net.w, bias, x, B, net.op, out, h1, h2, actT); break;
    case 2: hipLaunchKernelGGL(mlp_fwd_kernel<2>, grid, block, 0, st, net.w, bias, x, B, net.op, out, h1, h2, actT); break;
    case 3: hipLaunchKernelGGL(mlp_fwd_kernel<3>, grid, block, 0, st, net.w, bias, x, B, net.op, out, h1, h2, actT); break;
    case 4: hipLaunchKernelGGL(mlp_fwd_kernel<4>, grid, block, 0, st, net.w, bias, x, B, net.op, out, h1, h2, actT); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t mlp_backward_launch(const MlpNet& net, const float* dout, int B, const MlpWork& wk, hipStream_t st)
{
    if (B == 0) return hipSuccess;
    hipLaunchKernelGGL(mlp_bwd_act_kernel, dim3((unsigned)(B / 32)), dim3(64), 0, st, net.wt, net.dp, net.op, dout, B,
                       wk.h1, wk.h2, wk.gT);
    const int tiles = (net.op / 16) * 8 + 64 + 8 * (net.dp / 16);
    hipLaunchKernelGGL(mlp_wgrad_kernel, dim3((unsigned)tiles), dim3(64), 0, st, wk.gT, wk.actT, B, net.dp, net.op,
                       net.grad);
    return hipGetLastError();
}

hipError_t mlp_adam_launch(const MlpNet& net, bool update, float lr, float b1, float b2, float eps, int t,
                           hipStream_t st)
{
    const int64_t P = mlp_param_count(net.dp, net.op);
    const float c1 = update ? (float)(1.0 / (1.0 - pow((double)b1, (double)t))) : 1.0f;
    const float c2 = update ? (float)(1.0 / (1.0 - pow((double)b2, (double)t))) : 1.0f;
    hipLaunchKernelGGL(mlp_adam_kernel, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, st, net.param, net.grad,
                       net.m, net.v, net.w, net.wt, P, net.dp, net.op, update ? 1 : 0, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

}  // namespace apm
