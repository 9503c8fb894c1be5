/*
 * apm.h -- C ABI of libapm.so: all principal minors, CDet connected sums and
 * permanent principal minors of batches of small matrices on AMD MI355X (gfx950).
 *
 * Source of the operations: Simkovic & Ferrero, "Fast Principal Minor
 * Algorithms for Quantum Many Body Systems", arXiv:2104.07638.
 *
 * Common conventions
 *   - Subsets of {0..n-1} are integer masks; bit k set <=> row/column k kept
 *     (the paper's Sec. II convention S_13 = {1,3,4}, shifted to 0-based rows).
 *     Every output array of a matrix of order n has 2^n entries in mask order.
 *   - Matrices are dense row-major; complex values are interleaved (re, im) pairs
 *     (the layout of torch.complex128 / complex64 and C99 _Complex double), each value
 *     aligned to its size (16 bytes for complex128, 8 for complex64), as every
 *     allocation of those types is: the kernels move a whole value per access.
 *   - Pointers inside apm_batch and every data pointer are DEVICE pointers unless
 *     stated otherwise; the caller owns all of them.  The library owns only its
 *     small internal workspace (queue counters and packed offsets of mixed-order
 *     batches), allocated on first use per device and grown when a larger mixed-order
 *     batch arrives.  Mixed-order calls (n_uniform == 0) share that workspace: they
 *     must not overlap in time on one device (order them on one stream).  A call that
 *     would grow it must not be the first such call inside a graph capture.  A grown
 *     workspace replaces the old one, which is kept (not freed) until the process ends,
 *     so a graph captured earlier stays valid; its replays keep using the old buffer.
 *     Uniform-order calls of apm_all_minors keep one more small buffer per (device,
 *     stream): the queue of matrices whose pivot corrections in the top tree levels are
 *     applied by a follow-up launch.  Calls on one stream are ordered by the stream.
 *     The queue is allocated and grown only outside stream capture; a captured call
 *     whose stream has no queue of the batch's size applies those corrections inside
 *     the minors kernel (same results, bit for bit).  A graph that did capture a queue
 *     uses the capturing stream's buffer: its replays must not overlap direct calls on
 *     that stream.  Like the workspace, a queue (and the XOR minors' per-stream node
 *     workspace) is never freed when a larger one replaces it.
 *   - Calls are asynchronous: arguments are validated on the host, work is
 *     enqueued on `stream`, and the call returns.  Results are valid once the
 *     stream has been synchronised.  Argument errors return before anything is
 *     enqueued.  No call aborts, prints, or throws across the ABI.
 *   - Calls are reentrant; calls that write the same buffers must be ordered by
 *     the caller (same stream or events).
 */
#ifndef APM_H
#define APM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    APM_OK = 0,
    APM_EINVAL = 1,          /* bad argument (null pointer, bad size, bad enum)        */
    APM_EUNSUPPORTED = 2,    /* valid request outside what this build implements       */
    APM_EDEVICE = 3,         /* a HIP call failed (launch error, no device)           */
    APM_ENOMEM = 4           /* internal workspace allocation failed                  */
} apm_status;

typedef enum {
    APM_R64 = 0,    /* real fp64 in, fp64 Schur updates, fp64 out                              */
    APM_R32S = 1,   /* real fp64 in, fp32 Schur updates with fp64 pivot division/test/shift,
                       output float mantissa + int16 exponent (or fp64 with APM_OUT_F64)       */
    APM_C128 = 2,   /* complex128 in/out (Sec. V.C matrices are complex)                       */
    APM_C64S = 3    /* complex128 in, complex64 updates, fp64 pivot handling, output complex64
                       mantissa + int16 exponent (or complex128 with APM_OUT_F64)              */
} apm_dtype;

#define APM_MAX_N 20          /* largest matrix order accepted by apm_all_minors          */
#define APM_MAX_N_CS 20       /* largest order accepted by apm_connected_sums             */
#define APM_MAX_N_PERM 16     /* largest order accepted by apm_all_perm_minors            */
#define APM_MAX_N_XOR 16      /* most 2 x 2 blocks accepted by apm_xor_minors             */
#define APM_MAX_N_LEAD 32     /* largest order accepted by apm_leading_minors             */
#define APM_MAX_N_NAND 13     /* most 2 x 2 blocks accepted by apm_nand_minors (3^n out)  */

/* opaque HIP stream (binary compatible with hipStream_t); NULL = the default stream */
typedef struct ihipStream_t *apm_stream;

/* Batch descriptor (host struct; the arrays it points to are device arrays). */
typedef struct {
    int32_t batch;            /* number of matrices B >= 0; B == 0 is a no-op              */
    int32_t n_uniform;        /* > 0: every matrix has this order; 0: orders in n[]       */
    const int32_t *n;         /* [B] per-matrix orders in [1, max] (only if n_uniform==0) */
    int32_t n_max;            /* with n[]: an upper bound of n[] (0 = the maximum)        */
    const int64_t *in_off;    /* [B] element offset of matrix b; NULL = packed b*n*n
                                 (ragged batches: NULL = packed prefix sums of n_b^2)      */
    const int64_t *out_off;   /* [B] element offset of the 2^n_b outputs of b; NULL =
                                 packed b*2^n (ragged: prefix sums of 2^n_b)              */
} apm_batch;

/* Options (NULL = defaults).
 * Pivot shift (Sec. II, pivot correction; the paper leaves the test and C open):
 * at a tree node with pivot p, largest row entry r = max_j |M_0j| and largest column
 * entry c = max_i |M_i0| of the node's matrix (|z| = max(|Re z|, |Im z|) for complex),
 * p is shifted to p + C when |p|^2 < piv_tol^2 * r * c or p == 0.  C is the power of
 * two 2^(floor(log2(r min(r, c)) / 2) - 4), about min(sqrt(r c), r) / 16 (s / 16 when
 * r c == 0, with s = max_ij |A_ij|), with the sign of Re p, so that |p + C| >= |C|.  The test is
 * invariant under diagonal similarity, as the minors are.  The minors are corrected
 * exactly for every shift (det A[S] = det A~[S] - C det A[S \ {l}]), so piv_tol trades
 * the number of corrections against the growth of the unshifted Schur complements. */
typedef struct {
    double piv_tol;           /* <= 0: default 1e-3 (every element type)                  */
    uint32_t flags;           /* APM_OUT_F64 | APM_NO_PERTURB                             */
} apm_opts;

#define APM_OUT_F64 1u        /* R32S/C64S: write fp64/complex128 values, no exponents     */
#define APM_NO_PERTURB 2u     /* never shift pivots (a zero pivot then yields non-finite
                                 minors in its right subtree, reported as info = -3)       */

/*
 * apm_all_minors -- all 2^n principal minors det(A[S]) of every matrix of the batch.
 *
 * Passage: Sec. II (problem statement; det of the empty matrix = 1; the Schur-
 * complement binary tree, Eqs. (dets_schur), (eq:schur), (lemma1), (lemma2),
 * (eq:minor), Algorithm 1, its depth-first traversal, and the pivot correction
 * det A[S] = det A~[S] - C det A[S \ {l}]).
 *
 *   dt      element type / precision variant (apm_dtype).
 *   A       input matrices: double (R64, R32S) or complex128 (C128, C64S).
 *   bd      batch descriptor (host pointer, must not be NULL).
 *   minors  output: B x 2^n values in mask order, minors[0] = 1:
 *             R64: double;  C128: complex128;
 *             R32S: float mantissa m (|m| in [0.5,1) or 0) with value m * 2^exp;
 *             C64S: complex64 mantissa (max(|re|,|im|) in [0.5,1) or 0), same exp;
 *             with APM_OUT_F64 the two scaled variants write double / complex128.
 *   exp     int16 exponents, same indexing as minors; required for R32S/C64S without
 *           APM_OUT_F64, must be NULL otherwise.
 *   info    [B] int32 or NULL: >= 0 number of shifted pivots of matrix b;
 *           -2 non-finite input (outputs set to NaN); -3 a non-finite output.
 *   opt     options or NULL.
 * A uniform batch whose tree has between one and five top levels (n - 6 minus the
 * lane-subtree order; fp64 at n = 12..16) enqueues the minors launch and then one
 * launch per top level for the deferred pivot corrections (ownership notes above).
 * Returns APM_OK, APM_EINVAL (bad argument), APM_EUNSUPPORTED (n > APM_MAX_N), or
 * APM_EDEVICE (launch failure).
 */
apm_status apm_all_minors(apm_dtype dt, const void *A, const apm_batch *bd, void *minors, int16_t *exp,
                          int32_t *info, const apm_opts *opt, apm_stream stream);

#define APM_CS_ROOTED 0u      /* distinguished vertex j = 0; c[S] = 0 for S not containing 0 */
#define APM_CS_ALL 1u         /* j = lowest vertex of S; c[S] for every nonempty S           */

/*
 * apm_all_minors_noalloc -- apm_all_minors that allocates nothing.
 *
 * For callers that cannot allocate device memory: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  Same arguments, results (bit for bit)
 * and errors as apm_all_minors, with these differences:
 *   - batch must be at most APM_NOALLOC_MAX_BATCH; a larger batch returns
 *     APM_EUNSUPPORTED before anything is enqueued;
 *   - the call's scratch (the deferred pivot-correction queue of a uniform batch; the
 *     queue head, queue order and packed offsets of a mixed-order batch) is one static
 *     device array of 1 MiB + 4.25 KiB per GPU, loaded with the library and held until the
 *     process ends; its device address is looked up on the first call on each GPU.  No
 *     call allocates or frees device memory;
 *   - every call on a GPU uses that GPU's array and leaves its contents to the next
 *     call: calls that overlap in time on one GPU (other streams, concurrent graph
 *     replays) race, and the caller must order them.  Each call clears what must start
 *     at zero with a small kernel on `stream` (no memset), so it can be captured.
 */
#define APM_NOALLOC_MAX_BATCH 16384
apm_status apm_all_minors_noalloc(apm_dtype dt, const void *A, const apm_batch *bd, void *minors,
                                  int16_t *exp, int32_t *info, const apm_opts *opt, apm_stream stream);

/*
 * apm_connected_sums -- CDet connected sums from subset weights.
 *
 * Passage: Sec. V.A, the weights a[S] = det M_up[S] det M_dn[S] and Eq. (recursion)
 *     c[S] = a[S] - sum_{T subsetneq S, j in T} c[T] a[S \ T].
 *
 *   m_up    [B x 2^n] fp64 minors of M_up (mask order), e.g. apm_all_minors output.
 *   m_dn    [B x 2^n] fp64 minors of M_dn, or NULL for m_dn = m_up (a = m_up^2).
 *           With APM_CS_WEIGHTS in mode, m_up already holds a[] and m_dn must be NULL.
 *   bd      batch descriptor; in_off/out_off (if given) index both m_* and c.
 *   c       [B x 2^n] fp64 output; c[empty] = 0.
 *   mode    APM_CS_ROOTED or APM_CS_ALL, optionally | APM_CS_WEIGHTS.
 * Returns APM_OK, APM_EINVAL, APM_EUNSUPPORTED (n > APM_MAX_N_CS) or APM_EDEVICE.
 */
#define APM_CS_WEIGHTS 2u
apm_status apm_connected_sums(const double *m_up, const double *m_dn, const apm_batch *bd, double *c,
                              uint32_t mode, apm_stream stream);

/*
 * apm_all_perm_minors -- all 2^n permanent principal minors per(A[S]).
 *
 * Passage: Sec. IV (Ryser's formula, its per-subset form and the division-free
 * product recursion over subsets, O(3^n)).  Real fp64 only.
 *
 *   A       [B x n x n] fp64 input;  perm  [B x 2^n] fp64 output, perm[0] = 1.
 * Returns APM_OK, APM_EINVAL, APM_EUNSUPPORTED (n > APM_MAX_N_PERM) or APM_EDEVICE.
 */
apm_status apm_all_perm_minors(const double *A, const apm_batch *bd, double *perm, apm_stream stream);

/*
 * apm_xor_minors -- XOR principal minors of 2n x 2n matrices of 2 x 2 blocks.
 *
 * Passage: Sec. III, the XOR case (the principal minors that keep exactly one of the
 * rows/columns 2i, 2i+1 of every block i, computed by the binary tree of Schur
 * complements whose two branches keep one row of the next block each), and Sec. V.C
 * (with the Keldysh block matrix [[G++, G+-], [G-+, G--]] these are the determinants of
 * all 2^n Keldysh index assignments; the lower-order ones come as side products).
 *
 *   dt      APM_R64 (double) or APM_C128 (complex128); others APM_EUNSUPPORTED.
 *   A       [B x 2n x 2n] row-major input (device).
 *   bd      uniform batch: n_uniform = n, the number of blocks (1 <= n <= APM_MAX_N_XOR);
 *           per-matrix orders and offset arrays are not supported (APM_EUNSUPPORTED).
 *   out     [B x (2^(n+1) - 2)] output (device).  The tree takes the last block first,
 *           so depth k = 1..n lists the minors of the k trailing blocks: entry
 *           2^k - 2 + beta is det A[R, R] with R = {2(n-k+i) + beta_i : i < k} (bit i of
 *           beta chooses the row of block n-k+i).  The 2^n order-n minors (bit i <->
 *           block i) are the last 2^n entries.
 *   info    [B] int32 or NULL: 0, -2 non-finite input (outputs NaN), or -3 a non-finite
 *           output (a zero pivot: this tree admits no pivot shift, Sec. III).
 * Matrices with more than six blocks use a workspace of the library per (device,
 * stream), 3 KB per matrix at n = 8 and 47 KB at n = 14 (complex128; half for double),
 * grown outside stream capture only (a captured call that would grow it returns
 * APM_EUNSUPPORTED).
 * Returns APM_OK, APM_EINVAL, APM_EUNSUPPORTED, APM_ENOMEM or APM_EDEVICE.
 */
apm_status apm_xor_minors(apm_dtype dt, const void *A, const apm_batch *bd, void *out, int32_t *info,
                          apm_stream stream);

/*
 * apm_xnor_minors -- XNOR principal minors of 2n x 2n matrices of 2 x 2 blocks.
 *
 * Passage: Sec. III, the XNOR case (the principal minors that keep both or neither of the
 * rows/columns 2i, 2i+1 of every block i, computed by the binary tree whose branches drop
 * a block or take the Schur complement over it as a 2 x 2 pivot; no pivot corrections).
 *
 *   dt, A, bd, info, stream   as for apm_xor_minors (info -3: a singular pivot block).
 *   out     [B x 2^n] output: entry mask is det A[R, R], R = the two rows of every block i
 *           with bit i of mask set; entry 0 = 1.
 * Uses the same per-(device, stream) workspace as apm_xor_minors.
 * Returns APM_OK, APM_EINVAL, APM_EUNSUPPORTED, APM_ENOMEM or APM_EDEVICE.
 */
apm_status apm_xnor_minors(apm_dtype dt, const void *A, const apm_batch *bd, void *out, int32_t *info,
                           apm_stream stream);

/*
 * apm_nand_minors -- NAND principal minors of 2n x 2n matrices of 2 x 2 blocks.
 *
 * Passage: Sec. III, the NAND case (the principal minors that keep at most one of the
 * rows/columns 2i, 2i+1 of every block i: the ternary tree whose branches leave the block
 * out or take the Schur complement over one of its two diagonal entries, O(3^n)).
 *
 *   dt, A, stream   as for apm_xor_minors.
 *   info    [B] int32 or NULL: the number of pivot shifts made (>= 0), -2 non-finite
 *           input (outputs NaN), -3 a non-finite output.  Pivot shift: the test and C of
 *           apm_opts at the default piv_tol, on each kept row's pivot with the row and
 *           column entries that enter the child's Schur complement (the other row of the
 *           block left out); the child's subtree is corrected once it is complete,
 *           deepest node first (det A[S] = det A~[S] - C det A[S \ {l}], S \ {l} being the
 *           entry with block l left out), and its own entry is the parent's minor times
 *           the true pivot.
 *   bd      uniform batch, n_uniform = n blocks, 1 <= n <= APM_MAX_N_NAND, no offsets.
 *   out     [B x 3^n]: entry sum_i t_i 3^i is the determinant over the kept rows, with
 *           t_i = 0 (block i left out), 1 (row 2i kept) or 2 (row 2i+1 kept); entry 0 = 1.
 * Uses the same per-(device, stream) workspace as apm_xor_minors.
 * Returns APM_OK, APM_EINVAL, APM_EUNSUPPORTED, APM_ENOMEM or APM_EDEVICE.
 */
apm_status apm_nand_minors(apm_dtype dt, const void *A, const apm_batch *bd, void *out, int32_t *info,
                           apm_stream stream);

/*
 * apm_leading_minors -- the n leading principal minors det A[:k, :k], k = 1..n.
 *
 * Passage: Sec. III, "Leading principal minors" (successive Schur complements give the
 * minors of the subsets 2^k - 1 in O(n^3); no pivot correction is possible).
 *
 *   dt      APM_R64 or APM_C128 (others APM_EUNSUPPORTED).
 *   A       [B x n x n] row-major input; bd uniform, 1 <= n <= APM_MAX_N_LEAD, no offsets.
 *   out     [B x n]: out[b][k-1] = det A_b[:k, :k].
 *   info    [B] int32 or NULL: 0, -2 non-finite input (outputs NaN), -3 non-finite output
 *           (a zero pivot: elimination runs without row exchanges).
 * Returns APM_OK, APM_EINVAL, APM_EUNSUPPORTED or APM_EDEVICE.
 */
apm_status apm_leading_minors(apm_dtype dt, const void *A, const apm_batch *bd, void *out, int32_t *info,
                              apm_stream stream);

/*
 * apm_autotune_minors -- pick the per-order layout of apm_all_minors by measurement.
 *
 * The layout parameter is the order K0 of the per-lane register subtrees (the mid
 * levels are expanded breadth-first down to nodes of order K0, one per lane).  Every
 * instantiated K0 for (dt, n) is timed on a synthetic batch of `batch` diagonally
 * dominant matrices on `stream`; the fastest is installed for all later uniform-order
 * calls with that dtype and order in this process (an APM_K0 environment value still
 * takes precedence).  Allocates and frees device memory and synchronises `stream`: call
 * it outside timed regions and graph captures.
 *   k0      if not NULL, receives the chosen value (host pointer).
 * Returns APM_OK, APM_EINVAL (bad dt, n outside [1, APM_MAX_N], batch < 1),
 * APM_ENOMEM or APM_EDEVICE.
 */
apm_status apm_autotune_minors(apm_dtype dt, int32_t n, int32_t batch, int32_t *k0, apm_stream stream);

/* The lane-subtree order apm_all_minors uses for (dt, n) now (APM_K0, tuned or default);
 * -1 for bad arguments.  Host-only. */
int32_t apm_minors_k0(apm_dtype dt, int32_t n);

/*
 * Tuning cache.  apm_autotune_minors also records its choice in a JSON file,
 *   {"version": 1, "k0": {"<gfx>/<dtype>/<n>": K0, ...}}
 * keyed by the current device's architecture name (e.g. gfx950), the dtype (r64, r32s,
 * c128, c64s) and the order (or "mixed" / "mixed-large" for the mixed-order kernels,
 * apm_autotune_minors_mixed); apm_plan_create with APM_PLAN_AUTOTUNE reads it before timing
 * anything, so that tuned layouts carry over between processes.  The file is the value of
 * the environment variable APM_TUNE_CACHE, else $HOME/.cache/apm_tune.json (an empty
 * APM_TUNE_CACHE disables it); missing or malformed files are ignored.
 *
 * apm_tune_cache_load installs the entries of the file `path` (NULL: the default path)
 * for the current device's architecture into this process's table, as if tuned here
 * (values outside the instantiated range are skipped).  Returns the number installed, or
 * -1 if the file cannot be read or no device is current.  Host-only, synchronous.
 */
int32_t apm_tune_cache_load(const char *path);

/*
 * apm_autotune_minors_mixed -- the same choice for the two kernels of a mixed-order launch of
 * apm_all_minors (orders 14..16 in one persistent kernel, the other orders in another;
 * each instantiated at two lane-subtree orders).
 *
 * Times each choice of each kernel on a synthetic batch of `batch` matrices (>= 1) of orders
 * 10..16 in turn (diagonally dominant, no pivot shifts), with the other kernel at its
 * current choice, installs the fastest for dt (later mixed-order calls, and plans created
 * with APM_PLAN_AUTOTUNE, use them) and records them in the tuning cache under
 * "<gfx>/<dtype>/mixed" and "<gfx>/<dtype>/mixed-large".  *k0_small / *k0_large (either may
 * be NULL) receive the choices.  Allocates its buffers, uses the library's mixed-order
 * workspace and synchronizes `stream`; not for use under stream capture.
 * Returns APM_OK, APM_EINVAL, APM_ENOMEM or APM_EDEVICE.
 *
 * apm_minors_k0_mixed -- the lane-subtree orders a mixed-order launch of dt uses now (the
 * tuned ones, else the defaults); -1 for an invalid dt.  Either pointer may be NULL.
 */
apm_status apm_autotune_minors_mixed(apm_dtype dt, int32_t batch, int32_t *k0_small, int32_t *k0_large,
                                     apm_stream stream);
void apm_minors_k0_mixed(apm_dtype dt, int32_t *k0_small, int32_t *k0_large);

/*
 * Plans -- one of the operations above, or the CDet pipeline, bound to fixed buffers and
 * shapes, prepared once and enqueued many times (the Monte Carlo use: the same batch
 * shapes every step, new matrix values in the same buffers).
 *
 * apm_plan_create validates the description as the direct call would, allocates the
 * plan's own workspace (queue head and order, packed offsets, deferred-correction queue;
 * never shared with direct calls or other plans), pins the lane-subtree order of uniform
 * minors, or those of the two mixed-order kernels (timing every instantiated order first
 * with APM_PLAN_AUTOTUNE, as apm_autotune_minors / apm_autotune_minors_mixed do, when
 * neither the process nor the tuning cache has a value for that dtype and order yet), and
 * records the whole launch sequence once into a HIP graph on a private stream.
 * apm_plan_launch then enqueues that graph on the caller's stream: one launch call for the
 * whole sequence, with results bit-identical to the direct calls.  With APM_PLAN_EAGER the
 * plan records nothing and each launch enqueues the kernels one by one (same results).
 *
 * The caller keeps every buffer named in the description (and the device arrays of its
 * apm_batch) alive and at the same addresses until apm_plan_destroy; their contents may
 * change between launches.  create allocates, zeroes the workspace and (autotuning)
 * times kernels on buffers of its own, synchronising its private stream: call it outside
 * timed regions and outside stream capture.  It enqueues nothing on the caller's buffers.
 * The plan belongs to the device current at create; launch it with that device current.
 * Launches of one plan must be ordered (one stream, or events): two launches in flight
 * at once share its workspace.  Launches of different plans are independent.
 * apm_plan_destroy waits for the device to finish its work before freeing the plan (it
 * frees device memory).
 */
typedef enum {
    APM_PLAN_MINORS = 0,          /* apm_all_minors(dtype, A, &batch, minors, exp, info, &opts)     */
    APM_PLAN_CONNECTED_SUMS = 1,  /* apm_connected_sums(m_up, m_dn, &batch, c, cs_mode)            */
    APM_PLAN_PERM_MINORS = 2,     /* apm_all_perm_minors(A, &batch, perm)                          */
    APM_PLAN_CDET = 3             /* Sec. V.A: minors of A (and of A_dn), then the connected sums
                                     c of the weights a[S] = det A[S] det A_dn[S] (A_dn == NULL:
                                     a = det A[S]^2); the three launches in one graph            */
} apm_plan_kind;

#define APM_PLAN_AUTOTUNE 1u      /* tune the lane-subtree orders of the minors before recording  */
#define APM_PLAN_EAGER 2u         /* record no graph; launch enqueues the kernels directly           */

typedef struct {
    apm_plan_kind kind;
    apm_dtype dtype;              /* MINORS: any; CDET: APM_R64, or APM_R32S with APM_OUT_F64 in
                                     opts.flags (the sums take fp64 minors); others: ignored       */
    apm_batch batch;              /* copied at create; the device arrays it names are not          */
    const void *A;                /* MINORS, CDET: matrices as for apm_all_minors; PERM: fp64      */
    const void *A_dn;             /* CDET: second matrix set of the same shapes, or NULL           */
    void *minors;                 /* MINORS: output as for apm_all_minors; CDET: fp64 minors of A  */
    void *minors_dn;              /* CDET with A_dn: fp64 minors of A_dn; else NULL                */
    int16_t *exp;                 /* MINORS: as for apm_all_minors; else NULL                      */
    int32_t *info;                /* MINORS, CDET: [B] info of A, or NULL                          */
    int32_t *info_dn;             /* CDET with A_dn: [B] info of A_dn, or NULL                     */
    const double *m_up;           /* CONNECTED_SUMS: inputs as for apm_connected_sums              */
    const double *m_dn;
    double *c;                    /* CONNECTED_SUMS, CDET: output connected sums                   */
    double *perm;                 /* PERM_MINORS: output                                           */
    uint32_t cs_mode;             /* CONNECTED_SUMS: as for apm_connected_sums; CDET: APM_CS_ROOTED
                                     or APM_CS_ALL                                                 */
    apm_opts opts;                /* MINORS, CDET: options by value ({0, 0} = defaults)            */
    uint32_t flags;               /* APM_PLAN_AUTOTUNE | APM_PLAN_EAGER                            */
} apm_plan_desc;

typedef struct apm_plan apm_plan;

/* Create a plan from *d (host pointer).  On success *out receives it (NULL on failure).
 * Fields a kind does not use must be NULL / 0.  In CDET, batch.in_off indexes A and A_dn
 * and batch.out_off indexes minors, minors_dn and c.
 * Must not be called while a stream capture is in progress on this thread (it allocates
 * and synchronises).
 * Returns APM_OK, APM_EINVAL (bad or inconsistent description, NULL d or out),
 * APM_EUNSUPPORTED, APM_ENOMEM or APM_EDEVICE. */
apm_status apm_plan_create(const apm_plan_desc *d, apm_plan **out);

/* Enqueue the plan's work on `stream`.  Returns APM_OK, APM_EINVAL (NULL plan, another
 * device current) or APM_EDEVICE. */
apm_status apm_plan_launch(apm_plan *p, apm_stream stream);

/* Lane-subtree order pinned in a minors or CDET plan (for a mixed-order batch: that of the
 * orders other than 14..16; 0 for other plans), and whether the plan holds a graph (1) or launches
 * eagerly (0).  Host-only; -1 for a NULL plan. */
int32_t apm_plan_k0(const apm_plan *p);
int32_t apm_plan_graphed(const apm_plan *p);

/* Free the plan, its graph, stream and workspace (NULL is a no-op). */
void apm_plan_destroy(apm_plan *p);

/* Human-readable name of a status code (static string). */
const char *apm_status_str(apm_status s);

/* The last HIP error seen by the library on this thread, as a HIP error code (0 = none). */
int apm_last_hip_error(void);

/* Status form of the same record: APM_OK if the library has seen no HIP failure on this
 * thread since the previous call of this function, else APM_ENOMEM (an allocation failed)
 * or APM_EDEVICE; each call clears the record (apm_last_hip_error keeps its value). */
apm_status apm_last_device_error(void);

/* Library version, major * 10000 + minor * 100 + patch. */
int apm_version(void);

/*
 * apm_probe_fma64 -- measurement probe (not part of the method): `blocks` workgroups of
 * 256 threads each run 8 independent fp64 FMA chains of `iters` steps, so that the
 * achieved fp64 vector FMA rate of the device can be timed by the caller around the
 * launch.  sink: device array of blocks * 256 doubles (written); *fmas (host, may be
 * NULL) receives the number of FMAs launched.  Asynchronous on `stream`.
 */
apm_status apm_probe_fma64(double *sink, int32_t blocks, int32_t iters, int64_t *fmas, apm_stream stream);

/*
 * apm_probe_copy -- measurement probe (not part of the method): copies `bytes` (a multiple
 * of 16; both pointers 16-byte aligned, device memory, not overlapping) with `blocks`
 * workgroups of 256 threads moving 16 bytes per access, so that the achievable HBM
 * bandwidth can be timed by the caller.  APM_EINVAL for a bad size or alignment.
 */
apm_status apm_probe_copy(void *dst, const void *src, int64_t bytes, int32_t blocks, apm_stream stream);

#ifdef __cplusplus
}
#endif

#endif /* APM_H */
