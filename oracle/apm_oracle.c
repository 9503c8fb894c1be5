/*
 * apm_oracle.c -- CPU oracle for the principal-minor library (TEST INFRASTRUCTURE).
 *
 * This file is test infrastructure.  It is a plain, slow, obviously correct
 * reference for the quantities computed in Simkovic & Ferrero, "Fast Principal
 * Minor Algorithms for Quantum Many Body Systems" (arXiv:2104.07638).  Only the
 * test suite, the smoke check and the CPU-baseline leg of the benchmark may load
 * it.  The product path (the HIP library) shares no code with it and never
 * calls it.
 *
 * Conventions (Sec. II, problem statement and bit-mask example S_13 = {1,3,4}):
 *   - a subset of the rows/columns {0..n-1} is the integer mask m; bit k of m
 *     set  <=>  row/column k is kept (0-based: the paper's 1-based row k+1).
 *   - out[m] = det(A[S_m]); the empty minor out[0] = 1.
 *   - matrices are dense row-major; complex values are interleaved (re, im).
 *
 * Every function computes the plain definition, with no reuse between subsets:
 *   - principal minors: Gaussian elimination with partial pivoting on each
 *     gathered submatrix (the "trivial way" of Sec. II, O(n^3 2^n));
 *   - connected sums: the recursion of Sec. V.A, Eq. (recursion), summed
 *     directly over subsets (O(3^n));
 *   - permanent principal minors: Ryser's inclusion-exclusion formula of
 *     Sec. IV applied separately to every subset, with the (-1)^|S| factor
 *     that the printed Eq. (ryser) omits (see the note at apm_oracle_perm).
 *
 * Accuracy: fp64 / complex128 throughout.  Partial pivoting makes the minors
 * backward stable; they are not exact for near-singular submatrices (tests use
 * a high-precision reference there).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_MAX_N 24
#define ORACLE_MAX_W 32   /* widest 2n x 2n matrix of the XOR minors */

/* ORACLE_PLANT selects a deliberate mistake, used only by the test that checks
 * that the pins catch plausible errors.  The shipped library is built with 0. */
#ifndef ORACLE_PLANT
#define ORACLE_PLANT 0
#endif

static int popcount32(uint32_t x) { return __builtin_popcount(x); }

/* Determinant of a dense k x k real matrix (row-major, overwritten) by
 * Gaussian elimination with partial pivoting.  det of the 0 x 0 matrix is 1. */
static double det_real_inplace(int k, double *M)
{
    double det = 1.0;
    for (int c = 0; c < k; ++c) {
        int piv = c;
        double best = fabs(M[c * k + c]);
        for (int r = c + 1; r < k; ++r) {
            double v = fabs(M[r * k + c]);
            if (v > best) { best = v; piv = r; }
        }
        if (best == 0.0) return 0.0;
        if (piv != c) {
            for (int j = 0; j < k; ++j) {
                double t = M[c * k + j]; M[c * k + j] = M[piv * k + j]; M[piv * k + j] = t;
            }
#if ORACLE_PLANT != 1
            det = -det;
#endif
        }
        double p = M[c * k + c];
        det *= p;
        for (int r = c + 1; r < k; ++r) {
            double f = M[r * k + c] / p;
            if (f == 0.0) continue;
#if ORACLE_PLANT == 2
            for (int j = c + 1; j < k; ++j) M[r * k + j] -= f * M[j * k + c];
#else
            for (int j = c + 1; j < k; ++j) M[r * k + j] -= f * M[c * k + j];
#endif
        }
    }
    return det;
}

/* Complex version; M holds k*k interleaved (re, im) pairs.  Result in d[0..1]. */
static void det_cplx_inplace(int k, double *M, double *d)
{
    double dr = 1.0, di = 0.0;
    for (int c = 0; c < k; ++c) {
        int piv = c;
        double best = hypot(M[2 * (c * k + c)], M[2 * (c * k + c) + 1]);
        for (int r = c + 1; r < k; ++r) {
            double v = hypot(M[2 * (r * k + c)], M[2 * (r * k + c) + 1]);
            if (v > best) { best = v; piv = r; }
        }
        if (best == 0.0) { d[0] = 0.0; d[1] = 0.0; return; }
        if (piv != c) {
            for (int j = 0; j < 2 * k; ++j) {
                double t = M[2 * c * k + j]; M[2 * c * k + j] = M[2 * piv * k + j]; M[2 * piv * k + j] = t;
            }
            dr = -dr; di = -di;
        }
        double pr = M[2 * (c * k + c)], pi = M[2 * (c * k + c) + 1];
        double nr = dr * pr - di * pi, ni = dr * pi + di * pr;
        dr = nr; di = ni;
        double den = pr * pr + pi * pi;
        for (int r = c + 1; r < k; ++r) {
            double ar = M[2 * (r * k + c)], ai = M[2 * (r * k + c) + 1];
            /* f = a / p */
#if ORACLE_PLANT == 6
            double fr = (ar * pr + ai * pi) / den, fi = (ar * pi - ai * pr) / den;
#else
            double fr = (ar * pr + ai * pi) / den, fi = (ai * pr - ar * pi) / den;
#endif
            for (int j = c + 1; j < k; ++j) {
                double br = M[2 * (c * k + j)], bi = M[2 * (c * k + j) + 1];
                M[2 * (r * k + j)]     -= fr * br - fi * bi;
                M[2 * (r * k + j) + 1] -= fr * bi + fi * br;
            }
        }
    }
    d[0] = dr; d[1] = di;
}

/* All 2^n principal minors of a real n x n matrix, one LU per subset
 * (Sec. II: det(A[S_m]) for every mask m, det(A[empty]) = 1). */
int apm_oracle_minors_r64(int n, const double *A, double *out)
{
    if (n < 0 || n > ORACLE_MAX_N) return -1;
    double sub[ORACLE_MAX_N * ORACLE_MAX_N];
    int idx[ORACLE_MAX_N];
    const uint32_t nm = 1u << n;
    for (uint32_t m = 0; m < nm; ++m) {
        int k = 0;
        for (int i = 0; i < n; ++i) if (m >> i & 1u) idx[k++] = i;
        for (int a = 0; a < k; ++a)
            for (int b = 0; b < k; ++b) sub[a * k + b] = A[idx[a] * n + idx[b]];
        out[m] = det_real_inplace(k, sub);
    }
    return 0;
}

/* The same definition evaluated only at the listed masks (for parity checks of
 * large orders, where all 2^n LU factorisations would take too long). */
int apm_oracle_minors_r64_masks(int n, const double *A, int count, const uint32_t *masks, double *out)
{
    if (n < 0 || n > ORACLE_MAX_N) return -1;
    double sub[ORACLE_MAX_N * ORACLE_MAX_N];
    int idx[ORACLE_MAX_N];
    for (int t = 0; t < count; ++t) {
        uint32_t m = masks[t];
        int k = 0;
#if ORACLE_PLANT == 12
        for (int i = 0; i < n; ++i) if (m >> (n - 1 - i) & 1u) idx[k++] = i;
#else
        for (int i = 0; i < n; ++i) if (m >> i & 1u) idx[k++] = i;
#endif
        for (int a = 0; a < k; ++a)
            for (int b = 0; b < k; ++b) {
#if ORACLE_PLANT == 13
                const int ra = (a == k - 1 && k > 1) ? a - 1 : a;
#else
                const int ra = a;
#endif
                sub[a * k + b] = A[idx[ra] * n + idx[b]];
            }
        out[t] = det_real_inplace(k, sub);
    }
    return 0;
}

/* Complex128 version (Sec. V.C: Keldysh matrices have complex entries). */
int apm_oracle_minors_c128(int n, const double *A, double *out)
{
    if (n < 0 || n > ORACLE_MAX_N) return -1;
    double sub[2 * ORACLE_MAX_N * ORACLE_MAX_N];
    int idx[ORACLE_MAX_N];
    const uint32_t nm = 1u << n;
    for (uint32_t m = 0; m < nm; ++m) {
        int k = 0;
        for (int i = 0; i < n; ++i) if (m >> i & 1u) idx[k++] = i;
        for (int a = 0; a < k; ++a)
            for (int b = 0; b < k; ++b) {
                sub[2 * (a * k + b)]     = A[2 * (idx[a] * n + idx[b])];
                sub[2 * (a * k + b) + 1] = A[2 * (idx[a] * n + idx[b]) + 1];
            }
        det_cplx_inplace(k, sub, &out[2 * m]);
    }
    return 0;
}

/* Connected sums, Sec. V.A, Eq. (recursion):
 *     c[S] = a[S] - sum_{T subsetneq S, j in T} c[T] a[S \ T],
 * with the distinguished vertex j fixed per S.
 *   mode 0 (rooted): j = vertex 0; c[S] is produced for every S containing
 *                    vertex 0 and c[S] = 0 is written for every other S;
 *   mode 1 (all):    j = the lowest vertex of S; c[S] for every nonempty S.
 * c[empty] = 0 and a[empty] is never read.  Subsets are visited in increasing
 * numeric order, which visits every proper subset T of S before S. */
int apm_oracle_connected_sums(int n, const double *a, double *c, int mode)
{
    if (n < 0 || n > ORACLE_MAX_N || (mode != 0 && mode != 1)) return -1;
    const uint32_t nm = 1u << n;
    c[0] = 0.0;
    for (uint32_t S = 1; S < nm; ++S) {
        uint32_t jbit = (mode == 0) ? 1u : (S & (0u - S));
        if (!(S & jbit)) { c[S] = 0.0; continue; }
        double acc = a[S];
        /* proper subsets T of S that contain j: T = jbit | U, U a subset of S \ jbit, T != S */
        uint32_t rest = S & ~jbit;
        uint32_t U = rest;
        for (;;) {
            uint32_t T = jbit | U;
#if ORACLE_PLANT == 3
            if (T != S) acc -= c[T] * a[T];
#elif ORACLE_PLANT == 4
            if (T != S) acc -= c[T] * a[S & ~T];
            else if (U != 0) acc -= c[jbit] * a[S & ~jbit];
#else
            if (T != S) acc -= c[T] * a[S & ~T];
#endif
            if (U == 0) break;
            U = (U - 1) & rest;
        }
        c[S] = acc;
    }
    return 0;
}

/* Error scale of the recursion (test metric, not part of the method):
 *     d[S] = |a[S]| + sum_{T subsetneq S, j in T} |c[T]| |a[S \ T]|
 * with the same choice of j as apm_oracle_connected_sums; every rounding error of the
 * recursion at S is a small multiple of eps * d[S]. */
int apm_oracle_cs_scale(int n, const double *a, const double *c, double *d, int mode)
{
    if (n < 0 || n > ORACLE_MAX_N || (mode != 0 && mode != 1)) return -1;
    const uint32_t nm = 1u << n;
    d[0] = 0.0;
    for (uint32_t S = 1; S < nm; ++S) {
        uint32_t jbit = (mode == 0) ? 1u : (S & (0u - S));
        if (!(S & jbit)) { d[S] = 0.0; continue; }
        double acc = fabs(a[S]);
        uint32_t rest = S & ~jbit;
        uint32_t U = rest;
        for (;;) {
            uint32_t T = jbit | U;
            if (T != S) acc += fabs(c[T]) * fabs(a[S & ~T]);
            if (U == 0) break;
            U = (U - 1) & rest;
        }
        d[S] = acc;
    }
    return 0;
}

/* First-order bound on the change of the connected sums when the weights a[] carry
 * errors of at most da[] (metric helper for parity tests whose weights come from
 * independently rounded minors): from Eq. (recursion),
 *     e[S] = da[S] + sum_{T: j in T, T != S} ( e[T] |a[S \ T]| + |c[T]| da[S \ T] ). */
int apm_oracle_cs_input_bound(int n, const double *a, const double *c, const double *da, double *e, int mode)
{
    if (n < 0 || n > ORACLE_MAX_N || (mode != 0 && mode != 1)) return -1;
    const uint32_t nm = 1u << n;
    e[0] = 0.0;
    for (uint32_t S = 1; S < nm; ++S) {
        uint32_t jbit = (mode == 0) ? 1u : (S & (0u - S));
        if (!(S & jbit)) { e[S] = 0.0; continue; }
        double acc = da[S];
        uint32_t rest = S & ~jbit;
        uint32_t U = rest;
        for (;;) {
            uint32_t T = jbit | U;
            if (T != S) acc += e[T] * fabs(a[S & ~T]) + fabs(c[T]) * da[S & ~T];
            if (U == 0) break;
            U = (U - 1) & rest;
        }
        e[S] = acc;
    }
    return 0;
}

/* Permanent principal minors by Ryser's formula applied to each subset S
 * separately (Sec. IV, the "naive successive application", O(n 3^n)):
 *     per(A[S]) = (-1)^|S| sum_{T subset of S} (-1)^|T| prod_{i in S} sum_{j in T} A_ij.
 * Reading: the printed Eq. (ryser) lacks the overall (-1)^n; with it the
 * formula gives per = 1 for the 1x1 matrix [1] and k! for the all-ones k x k
 * matrix, as it must.  out[0] = 1 (empty product, T = S = empty). */
static double ryser_subset(int n, const double *A, uint32_t S)
{
    double total = 0.0;
    uint32_t T = S;
    for (;;) {
        double prod = 1.0;
        for (int i = 0; i < n; ++i) {
            if (!(S >> i & 1u)) continue;
            double rs = 0.0;
            for (int j = 0; j < n; ++j) if (T >> j & 1u) rs += A[i * n + j];
            prod *= rs;
        }
#if ORACLE_PLANT == 5
        int sgn = (popcount32(T) & 1) ? -1 : 1;
#else
        int sgn = ((popcount32(S) - popcount32(T)) & 1) ? -1 : 1;
#endif
        total += sgn * prod;
        if (T == 0) break;
        T = (T - 1) & S;
    }
    return total;
}

int apm_oracle_perm_minors(int n, const double *A, double *out)
{
    if (n < 0 || n > ORACLE_MAX_N) return -1;
    const uint32_t nm = 1u << n;
    for (uint32_t S = 0; S < nm; ++S) out[S] = ryser_subset(n, A, S);
    return 0;
}

/* per(A[S]) for the listed masks only (same formula, same code as above). */
int apm_oracle_perm_minors_masks(int n, const double *A, int count, const uint32_t *masks, double *out)
{
    if (n < 0 || n > ORACLE_MAX_N || count < 0) return -1;
    for (int m = 0; m < count; ++m) {
        if (n < 32 && (masks[m] >> n) != 0u) return -1;
        out[m] = ryser_subset(n, A, masks[m]);
    }
    return 0;
}

/* ---- batched drivers (OpenMP over matrices; the per-matrix work is above) ---- */

/* Matrix b has order n[b]; its input starts at element in_off[b] of A (for the
 * complex kernels: complex element, i.e. 2 doubles each) and its 2^n[b]
 * outputs start at element out_off[b] of out.  Returns 0, or -1 on a bad n. */
/* XOR principal minors of a 2n x 2n matrix read as n x n blocks of 2 x 2 (Sec. III, the
 * XOR case): the principal minors that keep exactly one of the rows/columns 2i, 2i+1 of
 * every block i.  The tree that computes them may take the blocks in any order; the
 * paper fixes none for the lower-order minors it yields on the way.  Here the last block
 * is taken first, so depth k lists the minors of the k trailing blocks: for k = 1..n and
 * every k-bit choice word beta (bit i: row 2(n-k+i) + beta_i of block n-k+i is kept),
 *     out[2^k - 2 + beta] = det A[R, R],   R = {2(n-k+i) + beta_i : i < k},
 * and the 2^n full-order minors (bit i <-> block i) are the last 2^n of the 2^(n+1) - 2
 * entries.  With the Keldysh block matrix of Sec. V.C these are the determinants of the
 * branch assignments.  Each determinant is a separate partial-pivoting LU of the
 * gathered k x k matrix. */
static void xor_rows(int n, int k, uint32_t beta, int *idx)
{
    for (int i = 0; i < k; ++i) {
#if ORACLE_PLANT == 7
        idx[i] = 2 * (n - k + i) + 1 - (int)(beta >> i & 1u);
#else
        idx[i] = 2 * (n - k + i) + (int)(beta >> i & 1u);
#endif
    }
}

static int64_t xor_index(int k, uint32_t alpha) { return ((int64_t)1 << k) - 2 + alpha; }

/* column of the gathered matrix for kept row index r of block i */
static int xor_col(int r)
{
#if ORACLE_PLANT == 8
    return r ^ 1;
#else
    return r;
#endif
}

int apm_oracle_xor_minors_r64(int n, const double *A, double *out)
{
    if (n < 1 || 2 * n > ORACLE_MAX_W) return -1;
    const int w = 2 * n;
    double sub[ORACLE_MAX_W * ORACLE_MAX_W];
    int idx[ORACLE_MAX_W];
    for (int k = 1; k <= n; ++k)
        for (uint32_t alpha = 0; alpha < (1u << k); ++alpha) {
            xor_rows(n, k, alpha, idx);
            for (int a = 0; a < k; ++a)
                for (int b = 0; b < k; ++b) sub[a * k + b] = A[idx[a] * w + xor_col(idx[b])];
            out[xor_index(k, alpha)] = det_real_inplace(k, sub);
        }
    return 0;
}

int apm_oracle_xor_minors_c128(int n, const double *A, double *out)
{
    if (n < 1 || 2 * n > ORACLE_MAX_W) return -1;
    const int w = 2 * n;
    double sub[2 * ORACLE_MAX_W * ORACLE_MAX_W];
    int idx[ORACLE_MAX_W];
    for (int k = 1; k <= n; ++k)
        for (uint32_t alpha = 0; alpha < (1u << k); ++alpha) {
            xor_rows(n, k, alpha, idx);
            for (int a = 0; a < k; ++a)
                for (int b = 0; b < k; ++b) {
                    sub[2 * (a * k + b)]     = A[2 * (idx[a] * w + xor_col(idx[b]))];
                    sub[2 * (a * k + b) + 1] = A[2 * (idx[a] * w + xor_col(idx[b])) + 1];
                }
            det_cplx_inplace(k, sub, &out[2 * xor_index(k, alpha)]);
        }
    return 0;
}

/* XNOR principal minors of a 2n x 2n matrix read as n x n blocks of 2 x 2 (Sec. III, the
 * XNOR case): the principal minors that keep both or neither of the rows/columns 2i, 2i+1
 * of every block i.  out[mask] = det A[R, R] with R = {2i, 2i+1 : bit i of mask set},
 * out[0] = 1 (2^n entries).  Each determinant is a separate partial-pivoting LU of the
 * gathered 2k x 2k matrix. */
static int xnor_rows(int n, uint32_t mask, int *idx)
{
    int k = 0;
    for (int i = 0; i < n; ++i)
        if (mask >> i & 1u) {
#if ORACLE_PLANT == 9
            idx[k++] = 2 * i;
            idx[k++] = 2 * i;
#else
            idx[k++] = 2 * i;
            idx[k++] = 2 * i + 1;
#endif
        }
    return k;
}

int apm_oracle_xnor_minors_r64(int n, const double *A, double *out)
{
    if (n < 1 || 2 * n > ORACLE_MAX_W) return -1;
    const int w = 2 * n;
    double sub[ORACLE_MAX_W * ORACLE_MAX_W];
    int idx[ORACLE_MAX_W];
    for (uint32_t mask = 0; mask < (1u << n); ++mask) {
        const int k = xnor_rows(n, mask, idx);
        for (int a = 0; a < k; ++a)
            for (int b = 0; b < k; ++b) sub[a * k + b] = A[idx[a] * w + idx[b]];
        out[mask] = det_real_inplace(k, sub);
    }
    return 0;
}

int apm_oracle_xnor_minors_c128(int n, const double *A, double *out)
{
    if (n < 1 || 2 * n > ORACLE_MAX_W) return -1;
    const int w = 2 * n;
    double sub[2 * ORACLE_MAX_W * ORACLE_MAX_W];
    int idx[ORACLE_MAX_W];
    for (uint32_t mask = 0; mask < (1u << n); ++mask) {
        const int k = xnor_rows(n, mask, idx);
        for (int a = 0; a < k; ++a)
            for (int b = 0; b < k; ++b) {
                sub[2 * (a * k + b)]     = A[2 * (idx[a] * w + idx[b])];
                sub[2 * (a * k + b) + 1] = A[2 * (idx[a] * w + idx[b]) + 1];
            }
        det_cplx_inplace(k, sub, &out[2 * mask]);
    }
    return 0;
}

/* Leading principal minors (Sec. III, "Leading principal minors"): out[k-1] = det of the
 * leading k x k submatrix, k = 1..n (the subsets with masks 2^k - 1).  Each is a separate
 * partial-pivoting LU of the gathered matrix. */
static int lead_order(int k)
{
#if ORACLE_PLANT == 10
    return k > 1 ? k - 1 : k;
#else
    return k;
#endif
}

int apm_oracle_leading_minors_r64(int n, const double *A, double *out)
{
    if (n < 1 || n > ORACLE_MAX_W) return -1;
    double sub[ORACLE_MAX_W * ORACLE_MAX_W];
    for (int k = 1; k <= n; ++k) {
        const int q = lead_order(k);
        for (int a = 0; a < q; ++a)
            for (int b = 0; b < q; ++b) sub[a * q + b] = A[a * n + b];
        out[k - 1] = det_real_inplace(q, sub);
    }
    return 0;
}

int apm_oracle_leading_minors_c128(int n, const double *A, double *out)
{
    if (n < 1 || n > ORACLE_MAX_W) return -1;
    double sub[2 * ORACLE_MAX_W * ORACLE_MAX_W];
    for (int k = 1; k <= n; ++k) {
        const int q = lead_order(k);
        for (int a = 0; a < q; ++a)
            for (int b = 0; b < q; ++b) {
                sub[2 * (a * q + b)]     = A[2 * (a * n + b)];
                sub[2 * (a * q + b) + 1] = A[2 * (a * n + b) + 1];
            }
        det_cplx_inplace(q, sub, &out[2 * (k - 1)]);
    }
    return 0;
}

/* NAND principal minors of a 2n x 2n matrix of 2 x 2 blocks (Sec. III, the NAND case): the
 * principal minors that keep at most one of the rows/columns 2i, 2i+1 of every block i.
 * The choice of block i is the ternary digit t_i (0: neither row, 1: row 2i, 2: row
 * 2i+1); out[sum_i t_i 3^i] = det A[R, R] over the kept rows, out[0] = 1 (3^n entries).
 * Each determinant is a separate partial-pivoting LU of the gathered matrix. */
static int nand_rows(int n, uint32_t code, int *idx)
{
    int k = 0;
    for (int i = 0; i < n; ++i, code /= 3u) {
        const uint32_t t = code % 3u;
#if ORACLE_PLANT == 11
        if (t) idx[k++] = 2 * i + (int)(2u - t);
#else
        if (t) idx[k++] = 2 * i + (int)(t - 1u);
#endif
    }
    return k;
}

static uint32_t pow3u(int n)
{
    uint32_t p = 1;
    for (int i = 0; i < n; ++i) p *= 3u;
    return p;
}

int apm_oracle_nand_minors_r64(int n, const double *A, double *out)
{
    if (n < 1 || 2 * n > ORACLE_MAX_W || n > 16) return -1;
    const int w = 2 * n;
    double sub[ORACLE_MAX_W * ORACLE_MAX_W];
    int idx[ORACLE_MAX_W];
    for (uint32_t code = 0; code < pow3u(n); ++code) {
        const int k = nand_rows(n, code, idx);
        for (int a = 0; a < k; ++a)
            for (int b = 0; b < k; ++b) sub[a * k + b] = A[idx[a] * w + idx[b]];
        out[code] = det_real_inplace(k, sub);
    }
    return 0;
}

int apm_oracle_nand_minors_c128(int n, const double *A, double *out)
{
    if (n < 1 || 2 * n > ORACLE_MAX_W || n > 16) return -1;
    const int w = 2 * n;
    double sub[2 * ORACLE_MAX_W * ORACLE_MAX_W];
    int idx[ORACLE_MAX_W];
    for (uint32_t code = 0; code < pow3u(n); ++code) {
        const int k = nand_rows(n, code, idx);
        for (int a = 0; a < k; ++a)
            for (int b = 0; b < k; ++b) {
                sub[2 * (a * k + b)]     = A[2 * (idx[a] * w + idx[b])];
                sub[2 * (a * k + b) + 1] = A[2 * (idx[a] * w + idx[b]) + 1];
            }
        det_cplx_inplace(k, sub, &out[2 * code]);
    }
    return 0;
}

typedef int (*oracle_fn)(int, const double *, double *);

static int run_batch(oracle_fn fn, int width, int B, const int32_t *n, const int64_t *in_off,
                     const int64_t *out_off, const double *A, double *out, int nthreads)
{
    int bad = 0;
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads) reduction(| : bad)
#endif
    for (int b = 0; b < B; ++b) {
        if (fn(n[b], A + (size_t)width * in_off[b], out + (size_t)width * out_off[b]) != 0) bad |= 1;
    }
    (void)nthreads;
    return bad ? -1 : 0;
}

int apm_oracle_minors_r64_batch(int B, const int32_t *n, const int64_t *in_off, const int64_t *out_off,
                                const double *A, double *out, int nthreads)
{
    return run_batch(apm_oracle_minors_r64, 1, B, n, in_off, out_off, A, out, nthreads);
}

int apm_oracle_minors_c128_batch(int B, const int32_t *n, const int64_t *in_off, const int64_t *out_off,
                                 const double *A, double *out, int nthreads)
{
    return run_batch(apm_oracle_minors_c128, 2, B, n, in_off, out_off, A, out, nthreads);
}

int apm_oracle_perm_minors_batch(int B, const int32_t *n, const int64_t *in_off, const int64_t *out_off,
                                 const double *A, double *out, int nthreads)
{
    return run_batch(apm_oracle_perm_minors, 1, B, n, in_off, out_off, A, out, nthreads);
}

int apm_oracle_connected_sums_batch(int B, const int32_t *n, const int64_t *off, const double *a,
                                    double *c, int mode, int nthreads)
{
    int bad = 0;
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads) reduction(| : bad)
#endif
    for (int b = 0; b < B; ++b) {
        if (apm_oracle_connected_sums(n[b], a + off[b], c + off[b], mode) != 0) bad |= 1;
    }
    (void)nthreads;
    return bad ? -1 : 0;
}

int apm_oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
