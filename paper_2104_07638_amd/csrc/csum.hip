// csum.hip -- CDet connected sums (Sec. V.A, Eq. (recursion)) on gfx950.
//
//   c[S] = a[S] - sum_{T subsetneq S, j in T} c[T] a[S \ T],   a[S] = m_up[S] m_dn[S].
//
// For a distinguished vertex j write S = {j} + X and T = {j} + Y with X, Y subsets of the
// vertices above j (m = n-1-j bits).  Then, with c'[X] = c[{j}+X], a0[X] = a[{j}+X] and
// b[U] = a[U] (U above j, nonempty),
//
//   c'[X] = a0[X] - sum_{Y subsetneq X} c'[Y] b[X \ Y]                          (*)
//
// a triangular subset convolution of 3^m multiply-adds.  Rooted mode solves (*) for j = 0;
// "all" mode solves it for every j (independent problems, one workgroup each).
//
// Blocking (one workgroup per problem: one wavefront up to 10 bits, four above):
//   * X = (X2, X1): X1 = the low P = min(m, 11) bits, X2 = the rest.  Blocks of 2^P values
//     are staged in LDS (c' block, b block and the right-hand side).  Block X2 needs every
//     block Y2 subsetneq X2 (a full subset convolution of two blocks, "conv") and then the
//     triangular solve (*) restricted to the block ("tri") with the b block of X2 = 0.
//   * inside a block, X1 = (Xh, Xl) with Xl the low LB bits held in registers (LB = 4, or
//     3 for problems of at most 9 bits): one (Xh, Yh) pair is an LB-bit subset convolution
//     of two rows of 2^LB values (81 FMAs for 32 loaded values at LB = 4).  The 2^|Xh|
//     pairs of a row are split over G lanes of one wavefront and summed with DPP row
//     shifts.  tri takes the rows rank by rank (|Xh|); conv rows are independent and
//     follow a fixed balanced schedule over the four wavefronts.
//   * the c' and b blocks have padded rows (see the layouts below), so that lanes reading
//     different rows at the same column spread over the LDS banks.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "apm_device.h"
#include "apm_kernels.h"

namespace apm {
namespace {

#ifndef APM_CS_PMAX
#define APM_CS_PMAX 11
#endif
constexpr int kPmax = APM_CS_PMAX;

// threads per problem: one wavefront for small problems, four for large ones
#ifndef APM_CS_NT_LARGE
#define APM_CS_NT_LARGE 256
#endif
template <int M>
constexpr int cs_threads() { return M <= 10 ? 64 : APM_CS_NT_LARGE; }

// LDS block layouts.  The c' and b blocks, read row by row by many lanes at once, have rows
// padded to 2^LB + 2 values: row r starts 16 bytes further round the banks than row r-1, and
// each 16-byte pair of a row sits at a fixed offset from the row start (an immediate of the
// load).  The right-hand-side block (one reader per row) keeps unpadded rows with the pairs
// swizzled by row (pair slot p XOR (row mod W/2)).
#ifndef APM_CS_PAD
#define APM_CS_PAD 1
#endif
constexpr bool kPad = APM_CS_PAD != 0;

// doubles of a block of 2^P values with rows of 2^LB values
template <int P, int LB, bool PAD>
constexpr int block_len() { return (PAD && LB >= 2) ? (1 << P) + (2 << (P - LB)) : (1 << P); }

// Element X1 of an LDS block.
template <int LB, bool PAD>
__device__ __forceinline__ int sw(int x1)
{
    if constexpr (LB <= 1) {
        return x1;
    } else if constexpr (PAD) {
        constexpr int W = 1 << LB;
        return (x1 >> LB) * (W + 2) + (x1 & (W - 1));
    } else {
        constexpr int W = 1 << LB;
        constexpr int pm = (W >> 1) - 1;
        const int row = x1 >> LB, col = x1 & (W - 1);
        return row * W + ((((col >> 1) ^ (row & pm)) << 1) | (col & 1));
    }
}

// Byte address of a row.  Swizzled rows start at row * 8W bytes, a multiple of the 16-byte
// pair slots they span, so the slot (p ^ (row & pm)) of pair p is the row's address with
// bits 4.. XORed by p: one XOR per load.
template <int LB, bool PAD>
__device__ __forceinline__ uint32_t row_addr(int row)
{
    constexpr int W = 1 << LB;
    constexpr int pm = (W >> 1) - 1;
    // rows have at most 7 bits: with the mask the product is a full-rate 24-bit multiply
    // (an unbounded row index becomes a quarter-rate 32-bit one)
    if constexpr (PAD) return ((uint32_t)row & 0x7Fu) * (8u * (W + 2));
    return (uint32_t)row * (8u * W) + ((uint32_t)(row & pm) << 4);
}

template <int LB, bool PAD>
__device__ __forceinline__ double2 ld_pair(const double* buf, uint32_t a, int p)
{
    if constexpr (PAD) return *reinterpret_cast<const double2*>(reinterpret_cast<const char*>(buf) + a + (p << 4));
    return *reinterpret_cast<const double2*>(reinterpret_cast<const char*>(buf) + (a ^ ((uint32_t)p << 4)));
}

template <int LB, bool PAD>
__device__ __forceinline__ void load_row(const double* buf, int row, double (&v)[1 << LB])
{
    constexpr int W = 1 << LB;
    if constexpr (LB <= 1) {
#pragma unroll
        for (int i = 0; i < W; ++i) v[i] = buf[row * W + i];
    } else {
        const uint32_t a = row_addr<LB, PAD>(row);
#pragma unroll
        for (int p = 0; p < W / 2; ++p) {
            const double2 t = ld_pair<LB, PAD>(buf, a, p);
            v[2 * p] = t.x;
            v[2 * p + 1] = t.y;
        }
    }
}

// acc[x] -= sum_{y subset of x} f[y] g[x \ y]   (LB-bit subset convolution, unrolled)
template <int LB>
__device__ __forceinline__ void conv_tile(const double (&f)[1 << LB], const double (&g)[1 << LB],
                                          double (&acc)[1 << LB])
{
    constexpr int W = 1 << LB;
#pragma unroll
    for (int x = 0; x < W; ++x)
#pragma unroll
        for (int y = 0; y < W; ++y)
            if ((y & ~x) == 0) acc[x] = fma(-f[y], g[x ^ y], acc[x]);
}

// c[x] = r[x] - sum_{y subsetneq x} c[y] g0[x \ y], x in increasing order (in place on r).
template <int LB>
__device__ __forceinline__ void tri_tile(double (&r)[1 << LB], const double (&g0)[1 << LB])
{
    constexpr int W = 1 << LB;
#pragma unroll
    for (int x = 1; x < W; ++x)
#pragma unroll
        for (int y = 0; y < W; ++y)
            if ((y & ~x) == 0 && y != x) r[x] = fma(-r[y], g0[x ^ y], r[x]);
}

// The same product for 5-bit tiles with the operands loaded in halves (split on the top
// tile bit), so that only 48 operand values are live at a time:
//   acc_lo -= f_lo * g_lo;  acc_hi -= f_lo * g_hi + f_hi * g_lo.
template <int LB>
__device__ __forceinline__ void load_half(const double* buf, int row, int half, double (&v)[1 << (LB - 1)])
{
    constexpr int W = 1 << LB;
    const uint32_t a = row_addr<LB, kPad>(row);
#pragma unroll
    for (int p = 0; p < W / 4; ++p) {
        const double2 t = ld_pair<LB, kPad>(buf, a, p + half * (W / 4));
        v[2 * p] = t.x;
        v[2 * p + 1] = t.y;
    }
}

template <int HB>
__device__ __forceinline__ void conv_half(const double (&f)[1 << HB], const double (&g)[1 << HB], double* acc)
{
    constexpr int W = 1 << HB;
#pragma unroll
    for (int x = 0; x < W; ++x)
#pragma unroll
        for (int y = 0; y < W; ++y)
            if ((y & ~x) == 0) acc[x] = fma(-f[y], g[x ^ y], acc[x]);
}

template <int LB>
__device__ __forceinline__ void conv_rows_split(const double* cb, int yrow, const double* bb, int drow,
                                                double (&acc)[1 << LB])
{
    constexpr int HW = 1 << (LB - 1);
    double f[HW], g0[HW], g1[HW];
    load_half<LB>(cb, yrow, 0, f);
    load_half<LB>(bb, drow, 0, g0);
    load_half<LB>(bb, drow, 1, g1);
    conv_half<LB - 1>(f, g0, acc);
    conv_half<LB - 1>(f, g1, acc + HW);
    load_half<LB>(cb, yrow, 1, f);
    conv_half<LB - 1>(f, g0, acc + HW);
}

// v += v of the lane DELTA below (0 if outside the row of 16 / the group), for doubles.
template <int CTRL, int ROWMASK = 0xF>
__device__ __forceinline__ double dpp_add(double v)
{
    const int lo = __double2loint(v), hi = __double2hiint(v);
    const int slo = __builtin_amdgcn_update_dpp(0, lo, CTRL, ROWMASK, 0xF, true);
    const int shi = __builtin_amdgcn_update_dpp(0, hi, CTRL, ROWMASK, 0xF, true);
    return v + __hiloint2double(shi, slo);
}

// Sum over aligned groups of G consecutive lanes; the total lands in the LAST lane of
// each group.  row_shr:k (0x110 + k) shifts within rows of 16 lanes; row_bcast:15 (0x142)
// and row_bcast:31 (0x143) carry row ends across rows.
template <int W>
__device__ __forceinline__ void group_sum(double (&acc)[W], int G)
{
    if (G >= 2) {
#pragma unroll
        for (int i = 0; i < W; ++i) acc[i] = dpp_add<0x111>(acc[i]);
    }
    if (G >= 4) {
#pragma unroll
        for (int i = 0; i < W; ++i) acc[i] = dpp_add<0x112>(acc[i]);
    }
    if (G >= 8) {
#pragma unroll
        for (int i = 0; i < W; ++i) acc[i] = dpp_add<0x114>(acc[i]);
    }
    if (G >= 16) {
#pragma unroll
        for (int i = 0; i < W; ++i) acc[i] = dpp_add<0x118>(acc[i]);
    }
    if (G >= 32) {
#pragma unroll
        for (int i = 0; i < W; ++i) acc[i] = dpp_add<0x142, 0xA>(acc[i]);
    }
    if (G >= 64) {
#pragma unroll
        for (int i = 0; i < W; ++i) acc[i] = dpp_add<0x143, 0xC>(acc[i]);
    }
}

struct CsArgs {
    const double* up;
    const double* dn;
    double* c;
    int weights;       // m_up already holds a[]
    double* summ;      // rooted problems of at most one block: (c[V], d[V]) per matrix instead of c[]
};

// a[S] from the inputs
__device__ __forceinline__ double weight(const CsArgs& g, int64_t base, int64_t S)
{
    const double u = g.up[base + S];
    if (g.weights) return u;
    return u * (g.dn ? g.dn[base + S] : u);
}

#ifndef APM_CS_LB_SMALL
#define APM_CS_LB_SMALL 3     // problems of at most 9 bits
#endif
#ifndef APM_CS_LB_LARGE
#define APM_CS_LB_LARGE 4
#endif
#ifndef APM_CS_GMUL_SMALL
#define APM_CS_GMUL_SMALL 2   // one-wavefront problems (m <= 10)
#endif
#ifndef APM_CS_GMUL
#define APM_CS_GMUL 2
#endif
#ifndef APM_CS_GMUL_TRI
#define APM_CS_GMUL_TRI 2
#endif
#ifndef APM_CS_SCHED
#define APM_CS_SCHED 1
#endif

template <int M>
struct CsPlan {
    static constexpr int P = M < kPmax ? M : kPmax;     // block bits
    static constexpr int TB = M - P;                    // block-index bits
    static constexpr int LBW = M <= 9 ? APM_CS_LB_SMALL : APM_CS_LB_LARGE;
    static constexpr int LB = P < LBW ? P : LBW;        // register tile bits
    static constexpr int H = P - LB;                    // row bits inside a block
    static constexpr int ROWS = 1 << H;
};

// One rank pass over the rows of a block: TRI (rows of rank r of block X2, pairs
// Yh subsetneq Xh, then the in-row triangular solve) or CONV (pairs Yh subset of Xh,
// result subtracted from the right-hand side in the output).
template <int LB, bool PAD>
__device__ __forceinline__ void store_row(double* buf, int row, const double (&v)[1 << LB])
{
    constexpr int W = 1 << LB;
    if constexpr (LB <= 1) {
#pragma unroll
        for (int i = 0; i < W; ++i) buf[row * W + i] = v[i];
    } else {
        const uint32_t a = row_addr<LB, PAD>(row);
#pragma unroll
        for (int p = 0; p < W / 2; ++p)
            *reinterpret_cast<double2*>(reinterpret_cast<char*>(buf) + (PAD ? a + (p << 4) : (a ^ ((uint32_t)p << 4)))) =
                make_double2(v[2 * p], v[2 * p + 1]);
    }
}

// One rank pass over the rows Xh of rank r of a block: TRI (pairs Yh subsetneq Xh, then
// the in-row triangular solve; the finished row goes to cb_out) or CONV (pairs Yh subset
// of Xh).  Either way the result updates the right-hand-side row in rb.
// One row group: lane s of the G lanes of row Xh takes the pairs s, s + G, ... of the row
// (Yh subsetneq Xh for TRI, Yh subset of Xh for CONV); the partial rows are summed over the
// group and the last lane updates the right-hand-side row in rb (TRI: then solves the row
// in place and writes it to cb_out).  Every lane of the wavefront calls it with the same G.
template <int M, bool TRI, int GC = 0, bool RPAD = false>
__device__ __forceinline__ void row_group(bool valid, uint32_t xh, int items, int G, int s, const double* cb,
                                          const double* bb, double* rb, double* cb_out)
{
    using CP = CsPlan<M>;
    constexpr int LB = CP::LB, W = 1 << LB;
    if constexpr (GC > 0) G = GC;
    double acc[W];
#pragma unroll
    for (int i = 0; i < W; ++i) acc[i] = 0.0;
    if (valid) {
        // pair k = s + G t has Yh = pdep(s) | pdep(t) over the bits of Xh above its lowest
        // log2(G) ones: the second part steps through the subsets of those bits in order.
        // s < G: its bits go to the lowest log2(G) bits of Xh, and xhi keeps the rest.
        uint32_t ys = 0, xhi = xh;
        for (int gg = 1; gg < G; gg <<= 1) {
            const uint32_t low = xhi & (0u - xhi);
            if (s & gg) ys |= low;
            xhi ^= low;
        }
        uint32_t z = 0;
        for (int k = s; k < items; k += G, z = (z - xhi) & xhi) {
            const uint32_t yh = ys | z;
            if constexpr (LB >= 3) {
                conv_rows_split<LB>(cb, (int)yh, bb, (int)(xh ^ yh), acc);
            } else {
                double f[W], gg[W];
                load_row<LB, kPad>(cb, (int)yh, f);
                load_row<LB, kPad>(bb, (int)(xh ^ yh), gg);
                conv_tile<LB>(f, gg, acc);
            }
        }
    }
    // sum the G partial rows (consecutive lanes of one wavefront) into the last lane
    group_sum<W>(acc, G);
    if (valid && s == G - 1) {
        double rr[W];
        load_row<LB, RPAD>(rb, (int)xh, rr);
#pragma unroll
        for (int i = 0; i < W; ++i) rr[i] += acc[i];
        if constexpr (TRI) {
            double g0[W];
            load_row<LB, kPad>(bb, 0, g0);
            tri_tile<LB>(rr, g0);
            store_row<LB, kPad>(cb_out, (int)xh, rr);
        } else {
            store_row<LB, RPAD>(rb, (int)xh, rr);
        }
    }
}

// One rank pass over the rows Xh of rank r of a block, G lanes per row (G the largest power
// of two with nout G GMUL <= threads, G <= 64 and G <= the pairs of a row).
template <int M, int NT, bool TRI, bool RPAD = false>
__device__ __forceinline__ void rank_pass(int tid, int r, const uint16_t* rk_tab, const int* rk_off, const double* cb,
                                          const double* bb, double* rb, double* cb_out)
{
    const int nout = rk_off[r + 1] - rk_off[r];
    const int items = TRI ? (1 << r) - 1 : (1 << r);
    int G = 1;
    // lanes per problem: a whole wavefront (GMUL 2: at most half of it per pass, measured
    // faster than the whole one), or four wavefronts
    constexpr int GMUL = NT < kWave ? 1 : (NT == kWave ? APM_CS_GMUL_SMALL : (TRI ? APM_CS_GMUL_TRI : APM_CS_GMUL));
    constexpr int GMAX = NT < kWave ? NT : kWave;
    while (G * 2 <= GMAX && nout * G * GMUL <= NT && G * 2 <= (items > 0 ? items : 1)) G *= 2;
    const int lg = __builtin_ctz((unsigned)G);   // G is a power of two: shifts, not divisions
    const int per_pass = NT >> lg;
    for (int ob = 0; ob < nout; ob += per_pass) {
        const int o = ob + (tid >> lg);
        const bool valid = o < nout;
        row_group<M, TRI, 0, RPAD>(valid, valid ? rk_tab[rk_off[r] + o] : 0u, items, G, tid & (G - 1), cb, bb, rb,
                                   cb_out);
    }
}

// CONV of a block with 7 row bits on four wavefronts: the rows are independent, so the
// ranks need no order and each wavefront takes a fixed share of them.  A wave task is G
// lanes per row over one or two rank segments (rank, first row, rows); the shares below
// minimise the largest per-wavefront cost over every choice of G per rank (cost per task:
// 120 per pair step of a lane, 48 per summation level, 120 for the row update and set-up):
//   wave 0: rank 5, G = 2 (42 lanes, 16 steps)
//   wave 1: rank 4, G = 1 (35 lanes, 16 steps)
//   wave 2: rank 6, G = 8 (56 lanes, 8 steps); ranks 2 and 0, G = 1 (22 lanes, 4 steps)
//   wave 3: ranks 3 and 1, G = 1 (42 lanes, 8 steps); rank 7, G = 64 (2 steps)
template <int M, int G>
__device__ __forceinline__ void conv_task(int lane, int r1, int k1, int r2, int k2, const uint16_t* rk_tab,
                                          const int* rk_off, const double* cb, const double* bb, double* rb)
{
    const int q = lane / G;
    const bool in1 = q < k1, in2 = !in1 && q < k1 + k2;
    const int r = in1 ? r1 : r2;
    const int o = in1 ? q : q - k1;
    const bool valid = in1 || in2;
    const uint32_t xh = valid ? rk_tab[rk_off[r] + o] : 0u;
    row_group<M, false, G>(valid, xh, 1 << r, G, lane % G, cb, bb, rb, nullptr);
}

template <int M, int NT>
__device__ __forceinline__ void conv_block(int tid, const uint16_t* rk_tab, const int* rk_off, const double* cb,
                                           const double* bb, double* rb)
{
    constexpr int H = CsPlan<M>::H;
    if constexpr (H == 7 && NT == 4 * kWave && APM_CS_SCHED) {
        const int wave = __builtin_amdgcn_readfirstlane(tid / kWave);
        const int lane = tid % kWave;
        if (wave == 0) {
            conv_task<M, 2>(lane, 5, 21, 0, 0, rk_tab, rk_off, cb, bb, rb);
        } else if (wave == 1) {
            conv_task<M, 1>(lane, 4, 35, 0, 0, rk_tab, rk_off, cb, bb, rb);
        } else if (wave == 2) {
            conv_task<M, 8>(lane, 6, 7, 0, 0, rk_tab, rk_off, cb, bb, rb);
            conv_task<M, 1>(lane, 2, 21, 0, 1, rk_tab, rk_off, cb, bb, rb);
        } else {
            conv_task<M, 1>(lane, 3, 35, 1, 7, rk_tab, rk_off, cb, bb, rb);
            conv_task<M, 64>(lane, 7, 1, 0, 0, rk_tab, rk_off, cb, bb, rb);
        }
    } else {
        for (int r = 0; r <= H; ++r) rank_pass<M, NT, false>(tid, r, rk_tab, rk_off, cb, bb, rb, nullptr);
    }
}

// Rows of a block (H bits) sorted by rank: tab[H] lists the masks of popcount 0, 1, ...,
// off[H][r] is where rank r starts.
struct RankTables {
    uint16_t tab[8][128];
    int off[8][9];
};

constexpr RankTables make_rank_tables()
{
    RankTables t{};
    for (int h = 0; h < 8; ++h) {
        int pos = 0;
        for (int r = 0; r <= h; ++r) {
            t.off[h][r] = pos;
            for (int x = 0; x < (1 << h); ++x) {
                int c = 0;
                for (int y = x; y; y &= y - 1) ++c;
                if (c == r) t.tab[h][pos++] = (uint16_t)x;
            }
        }
        t.off[h][h + 1] = pos;
    }
    return t;
}

__constant__ RankTables kRank = make_rank_tables();


// Problem (matrix b, root j): solve (*) for the m = n-1-j vertices above j, with NT lanes
// (tid in [0, NT)).  act = false runs the same passes and barriers without touching memory.
template <int M, int NT>
__device__ void cs_problem(const CsArgs& g, int64_t base, int j, bool zero_even, int tid, bool act, double* lds_c,
                           double* lds_b, double* lds_r, uint16_t* rk_tab, int* rk_off)
{
    using CP = CsPlan<M>;
    constexpr int P = CP::P, LB = CP::LB, H = CP::H;
    const int jsh = j + 1;                          // X -> S = (1 << j) | (X << (j+1))
    const int64_t sroot = base + (int64_t(1) << j);  // element index of S = {j}
    double* c = g.c;
    // right-hand side: its own block when there are cross-block terms; otherwise the c'
    // block itself (row Xh is read as right-hand side and overwritten by its solution in
    // the pass of its rank, after every row it depends on)
    constexpr bool kInPlace = CP::TB == 0;
    constexpr bool kRPad = kInPlace ? kPad : false;
    double* rhs = kInPlace ? lds_c : lds_r;

    static_assert(H < 8, "rank tables cover rows of up to 7 bits");
    for (int i = tid; i < (1 << H); i += NT) rk_tab[i] = kRank.tab[H][i];
    if (tid <= H + 1) rk_off[tid] = kRank.off[H][tid];
    // rooted problem in one block: a0[x] = a[2x + 1] and b[x] = a[2x] are neighbours, so
    // one 16-byte load per x stages both (the block's own b is staged later otherwise)
    constexpr bool kOneBlock = CP::TB == 0;
    const bool pair_stage = kOneBlock && j == 0 && !(base & 1);
    if (pair_stage && act) {
        // the loads of CH entries are issued before their stores (one memory round trip per
        // CH entries instead of per entry)
        constexpr int N = 1 << P, IT = (N + NT - 1) / NT, CH = IT < 4 ? IT : 4;
        const bool two = !g.weights && g.dn;
#pragma unroll
        for (int i0 = 0; i0 < IT; i0 += CH) {
            double2 u[CH], d[CH];
#pragma unroll
            for (int i = 0; i < CH; ++i) {
                const int x1 = tid + (i0 + i) * NT;
                if (x1 < N) {
                    u[i] = *reinterpret_cast<const double2*>(g.up + base + 2 * x1);
                    if (two) d[i] = *reinterpret_cast<const double2*>(g.dn + base + 2 * x1);
                }
            }
#pragma unroll
            for (int i = 0; i < CH; ++i) {
                const int x1 = tid + (i0 + i) * NT;
                if (x1 < N) {
                    double w0, w1;
                    if (g.weights) {
                        w0 = u[i].x;
                        w1 = u[i].y;
                    } else if (two) {
                        w0 = u[i].x * d[i].x;
                        w1 = u[i].y * d[i].y;
                    } else {
                        w0 = u[i].x * u[i].x;
                        w1 = u[i].y * u[i].y;
                    }
                    lds_b[sw<LB, kPad>(x1)] = x1 ? w0 : 0.0;
                    rhs[sw<LB, kRPad>(x1)] = w1;
                }
            }
        }
    }
    for (int x2 = 0; x2 < (1 << CP::TB); ++x2) {
        // right-hand side a0 of the block
        if (!pair_stage) {
            for (int x1 = act ? tid : (1 << P); x1 < (1 << P); x1 += NT) {
                const int64_t x = ((int64_t)x2 << P) | x1;
                rhs[sw<LB, kRPad>(x1)] = weight(g, base, (int64_t(1) << j) | (x << jsh));
            }
        }
        // cross-block contributions: every Y2 subsetneq X2
        for (uint32_t y2 = 0; y2 < (uint32_t)x2; ++y2) {
            if (y2 & ~(uint32_t)x2) continue;
            const uint32_t d2 = (uint32_t)x2 ^ y2;
            __syncthreads();
            for (int x1 = act ? tid : (1 << P); x1 < (1 << P); x1 += NT) {
                lds_c[sw<LB, kPad>(x1)] = c[sroot + ((((int64_t)y2 << P) | x1) << jsh)];
                lds_b[sw<LB, kPad>(x1)] = weight(g, base, (((int64_t)d2 << P) | x1) << jsh);
            }
            __syncthreads();
            conv_block<M, NT>(tid, rk_tab, rk_off, lds_c, lds_b, rhs);
        }
        // the block's own triangular solve, with b of block 0
        __syncthreads();
        if (!pair_stage) {
            for (int x1 = act ? tid : (1 << P); x1 < (1 << P); x1 += NT)
                lds_b[sw<LB, kPad>(x1)] = x1 ? weight(g, base, (int64_t)x1 << jsh) : 0.0;
            __syncthreads();
        }
        // a[V] for the summary (the in-place solve overwrites it)
        const double a_full = (CP::TB == 0 && g.summ) ? rhs[sw<LB, kRPad>((1 << P) - 1)] : 0.0;
        for (int r = 0; r <= H; ++r) {
            rank_pass<M, NT, true, kRPad>(tid, r, rk_tab, rk_off, lds_c, lds_b, rhs, lds_c);
            __syncthreads();
        }
        if constexpr (CP::TB == 0) {
            if (g.summ) {
                // only the full-set value and the recursion's rounding scale at it:
                // d[V] = |a[V]| + sum_{X full-exclusive} |c'[X]| |b[full \ X]|, with a[V] = a0[full]
                constexpr int full = (1 << P) - 1;
                double part = 0.0;
                for (int x1 = tid; x1 < full; x1 += NT) part += fabs(lds_c[sw<LB, kPad>(x1)]) * fabs(lds_b[sw<LB, kPad>(full ^ x1)]);
                for (int o = (NT < kWave ? NT : kWave) / 2; o > 0; o >>= 1) part += __shfl_xor(part, o);
                if constexpr (NT > kWave) {
                    __syncthreads();
                    if ((tid & (kWave - 1)) == 0) lds_b[tid / kWave] = part;   // b block no longer needed
                    __syncthreads();
                    part = 0.0;
                    for (int w = 0; w < NT / kWave; ++w) part += lds_b[w];
                }
                if (tid == 0 && act) {
                    g.summ[0] = lds_c[sw<LB, kPad>(full)];
                    g.summ[1] = fabs(a_full) + part;
                }
                return;
            }
        }
        if (zero_even && !(base & 1)) {
            // rooted problem: write (c[2x] = 0, c[2x+1] = c'[x]) as one 16-byte store
            for (int x1 = act ? tid : (1 << P); x1 < (1 << P); x1 += NT) {
                const int64_t x = ((int64_t)x2 << P) | x1;
                *reinterpret_cast<double2*>(c + base + 2 * x) = make_double2(0.0,
                                                                             lds_c[sw<LB, kPad>(x1)]);
            }
        } else {
            for (int x1 = act ? tid : (1 << P); x1 < (1 << P); x1 += NT) {
                const int64_t x = ((int64_t)x2 << P) | x1;
                c[sroot + (x << jsh)] = lds_c[sw<LB, kPad>(x1)];
                if (zero_even) c[base + 2 * x] = 0.0;
            }
        }
    }
    if (j == 0 && tid == 0 && act) c[base] = 0.0;   // c[empty] = 0
}

// Problem p of a launch: matrix b (through the size-sorted queue order when given) and root j.
struct CsMap {
    int32_t batch;
    int n_uniform;
    const int32_t* nv;
    const int64_t* off;
    const int32_t* order;   // mixed-order rooted batches: matrix indices by decreasing order, else NULL
    int roots;
};

__device__ __forceinline__ bool cs_locate(const CsMap& mp, int64_t p, int m_want, int* b_out, int* j_out,
                                          int64_t* base_out)
{
    if (p >= (int64_t)mp.batch * mp.roots) return false;
    int b = (int)(p / mp.roots);
    const int j = (int)(p % mp.roots);
    if (mp.order) b = mp.order[b];
    const int n = mp.n_uniform > 0 ? mp.n_uniform : mp.nv[b];
    if (n - 1 - j != m_want) return false;   // problems with exactly m_want bits
    *b_out = b;
    *j_out = j;
    *base_out = mp.off ? mp.off[b] : ((int64_t)b << n);
    return true;
}

// One problem per workgroup (cs_threads<M>() threads).
template <int M>
__global__ __launch_bounds__(cs_threads<M>()) void cs_kernel(CsArgs g, CsMap mp)
{
    using CP = CsPlan<M>;
    __shared__ __align__(16) double lds_c[block_len<CP::P, CP::LB, kPad>()];
    __shared__ __align__(16) double lds_b[block_len<CP::P, CP::LB, kPad>()];
    // problems of one block solve in place in the c' block: no separate right-hand side
    __shared__ __align__(16) double lds_r[CP::TB == 0 ? 2 : block_len<CP::P, CP::LB, false>()];
    __shared__ uint16_t rk_tab[1 << CsPlan<M>::H];
    __shared__ int rk_off[CsPlan<M>::H + 2];
    int b = 0, j = 0;
    int64_t base = 0;
    if (!cs_locate(mp, blockIdx.x, M, &b, &j, &base)) return;
    // the rooted problem also writes c[S] = 0 for the sets without vertex 0
    CsArgs gb = g;
    if (gb.summ) gb.summ += 2 * (int64_t)b;
    cs_problem<M, cs_threads<M>()>(gb, base, j, mp.roots == 1, (int)threadIdx.x, true, lds_c, lds_b, lds_r, rk_tab,
                                   rk_off);
}

// Mixed-order rooted batches: every problem of 11 bits or more in one launch, taken from the
// queue order (largest first, so that the shorter problems fill the end of the launch); each
// workgroup runs the code for its problem's size.  All these sizes share the 11-bit blocks.
constexpr int kLargeMin = 11;

template <int M>
__device__ __forceinline__ void cs_large_dispatch(int m, const CsArgs& g, int64_t base, double* lds_c, double* lds_b,
                                                  double* lds_r, uint16_t* rk_tab, int* rk_off)
{
    if constexpr (M >= kLargeMin) {
        if (m == M) {
            cs_problem<M, cs_threads<M>()>(g, base, 0, true, (int)threadIdx.x, true, lds_c, lds_b, lds_r, rk_tab,
                                           rk_off);
            return;
        }
        cs_large_dispatch<M - 1>(m, g, base, lds_c, lds_b, lds_r, rk_tab, rk_off);
    }
}

__global__ __launch_bounds__(APM_CS_NT_LARGE) __attribute__((amdgpu_waves_per_eu(3))) void cs_kernel_large(CsArgs g, CsMap mp,
                                                                                                  int m_max)
{
    using CP = CsPlan<kLargeMin + 1>;   // the block layout of every size from 11 bits up
    static_assert(CsPlan<19>::P == CP::P && CsPlan<kLargeMin>::P == CP::P && CsPlan<19>::H == CP::H, "one layout");
    __shared__ __align__(16) double lds_c[block_len<CP::P, CP::LB, kPad>()];
    __shared__ __align__(16) double lds_b[block_len<CP::P, CP::LB, kPad>()];
    __shared__ __align__(16) double lds_r[block_len<CP::P, CP::LB, false>()];
    __shared__ uint16_t rk_tab[1 << CP::H];
    __shared__ int rk_off[CP::H + 2];
    if (blockIdx.x >= (unsigned)mp.batch) return;
    const int b = mp.order[blockIdx.x];
    const int n = mp.nv[b];
    const int m = n - 1;
    if (m < kLargeMin || m > m_max) return;
    const int64_t base = mp.off ? mp.off[b] : ((int64_t)b << n);
    cs_large_dispatch<19>(m, g, base, lds_c, lds_b, lds_r, rk_tab, rk_off);
}

template <int M>
hipError_t launch_m(CsArgs g, const CsMap& mp, hipStream_t st)
{
    const int64_t problems = (int64_t)mp.batch * mp.roots;
    hipLaunchKernelGGL(cs_kernel<M>, dim3((unsigned)problems), dim3(cs_threads<M>()), 0, st, g, mp);
    return hipGetLastError();
}

template <int M>
hipError_t launch_all_m(int mlo, int mhi, CsArgs g, const CsMap& mp, hipStream_t st)
{
    if constexpr (M < 0) {
        return hipSuccess;
    } else {
        if (M >= mlo && M <= mhi) {
            hipError_t e = launch_m<M>(g, mp, st);
            if (e != hipSuccess) return e;
        }
        return launch_all_m<M - 1>(mlo, mhi, g, mp, st);
    }
}

}  // namespace

hipError_t cs_launch(const LaunchCS& L, hipStream_t st)
{
    CsArgs g{L.m_up, L.m_dn, L.c, (L.mode & 2u) ? 1 : 0, L.summ};
    const bool all = (L.mode & 1u) != 0;
    const int nmax = L.n_uniform > 0 ? L.n_uniform : L.n_max;
    const int nmin = L.n_uniform > 0 ? L.n_uniform : 1;
    const int roots = all ? nmax : 1;
    CsMap mp{L.batch, L.n_uniform, L.n, L.off, nullptr, roots};
    // one launch per problem size m = n-1-j (largest first); each workgroup exits unless its
    // problem has exactly that size
    int mhi = nmax - 1;
    const int mlo = all ? 0 : nmin - 1;
    if (!all && L.n_uniform <= 0 && L.order) {
        // mixed orders, rooted: the large problems in one size-sorted launch, then the rest
        mp.order = L.order;
        if (mhi >= kLargeMin) {
            hipLaunchKernelGGL(cs_kernel_large, dim3((unsigned)L.batch), dim3(APM_CS_NT_LARGE), 0, st, g, mp, mhi);
            const hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
            mhi = kLargeMin - 1;
        }
    }
    return launch_all_m<19>(mlo, mhi, g, mp, st);
}

}  // namespace apm
