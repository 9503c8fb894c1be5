/*
 * apm_mc.h -- C ABI of libapm.so, part 2: Monte Carlo over vertex configurations with
 * an exact Metropolis-Hastings step and a learned proposal network.
 *
 * The weight of a configuration X of n vertices is |c[V](X)|, the connected sum over
 * the full vertex set (Simkovic & Ferrero, arXiv:2104.07638, Sec. V.A, Eq. (recursion))
 * of the CDet weights a[S] = det(M[S])^2 with M_ij = G0(X_i - X_j) (both spins share M),
 * set to zero where it is not resolved above the recursion's rounding level (see
 * apm_mc_model.resolve): c[V] cancels the disconnected products, and for spread-out
 * vertices what remains is below fp64 resolution.
 * A step evaluates it with the same kernels as apm_all_minors and apm_connected_sums.
 * The paper defines the weight and the series, not the sampler: proposal, acceptance
 * and network below are this library's design.
 *
 * Conventions are those of apm.h: device pointers unless stated otherwise, caller-owned
 * buffers, asynchronous calls on `stream`, argument errors returned before anything is
 * enqueued.  Work buffers are caller-owned device memory of the size the matching
 * *_work_bytes function returns; they carry no state between calls unless stated.
 *
 * Vertices are packed uint32: site s = y*L + x in bits 0..15, time point j in bits
 * 16..31 (imaginary time (j + 1/2) beta / n_tau).
 *
 * Random numbers: Philox4x64-10 (Salmon et al., SC'11), key (seed, 0), counter
 * (walker, step, call, 0); an integer in [0, m) is floor(r m / 2^64), a uniform in (0,1)
 * is ((r >> 12) + 1/2) 2^-52.  Call 0 draws: moved vertex k, the eps test, a uniform
 * site, a uniform time point.  Call 1: site draw, bin draw, time point inside the bin,
 * the acceptance uniform.
 */
#ifndef APM_MC_H
#define APM_MC_H

#include "apm.h"

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ proposal network */
#define APM_MLP_HIDDEN 128      /* width of both hidden layers                           */
#define APM_MLP_MAX_IN 64       /* largest logical input size                            */
#define APM_MLP_MAX_OUT 4096    /* largest logical output size                           */

/*
 * Network: h1 = tanh(W1 x + b1), h2 = tanh(W2 h1 + b2), out = W3 h2 + b3 with hidden
 * width 128.  Weights are BF16 (copies of fp32 master parameters), biases fp32;
 * products accumulate in fp32 on the matrix cores; the inputs x and the hidden
 * activations enter each product as BF16.
 * Sizes: Dp = max(16, d_in rounded up to 16), Op = d_out rounded up to 16.  The fp32
 * parameter vector is packed W1 (128 x Dp) | W2 (128 x 128) | W3 (Op x 128) | b1 (128)
 * | b2 (128) | b3 (Op), matrices row-major [out][in]; padding rows/columns are zero and
 * stay zero under apm_mlp_adam.
 * The BF16 copy w (read by the forward pass) holds each M x K matrix in matrix-core operand
 * order: element (r, c) at ((r/16 (K/16) + c/16) 64 + 16 ((c % 16)/4) + r % 16) 4 + c % 4
 * from the matrix's start (the same start as in param).  wt holds each transpose row-major.
 */
typedef struct {
    int32_t d_in;             /* logical input size, 1..APM_MLP_MAX_IN                     */
    int32_t d_out;            /* logical output size, 1..APM_MLP_MAX_OUT                   */
    float *param;             /* [apm_mlp_param_count] fp32 master parameters              */
    float *grad;              /* same packing: written by apm_mlp_backward                 */
    float *adam_m;            /* same packing: Adam first moment (caller zeroes it once)   */
    float *adam_v;            /* same packing: Adam second moment (caller zeroes it once)  */
    uint16_t *w;              /* [apm_mlp_weight_count] BF16 W1|W2|W3, operand order above */
    uint16_t *wt;             /* [apm_mlp_weight_count] BF16 W1^T|W2^T|W3^T                */
} apm_mlp;

typedef struct {
    float lr, beta1, beta2, eps;   /* Adam hyper-parameters (Kingma & Ba, Algorithm 1)     */
    int32_t t;                     /* step number >= 1 (bias correction)                    */
} apm_adam;

/* Host-side size queries; -1 for sizes outside the limits above. */
int64_t apm_mlp_param_count(int32_t d_in, int32_t d_out);
int64_t apm_mlp_weight_count(int32_t d_in, int32_t d_out);
/* Bytes of the work buffer that carries activations from apm_mlp_forward to
 * apm_mlp_backward for `batch` rows (a multiple of 32). */
int64_t apm_mlp_work_bytes(int32_t d_in, int32_t d_out, int32_t batch);

/* Write the BF16 copies w and wt from param (call after writing param). */
apm_status apm_mlp_sync(const apm_mlp *net, apm_stream stream);

/*
 * apm_mlp_forward -- out = network(x) for `batch` rows.
 *   x      [batch x Dp] BF16 inputs (padding columns zero).
 *   out    [batch x Op] fp32.
 *   work   NULL for inference; else a buffer of apm_mlp_work_bytes that keeps what
 *          apm_mlp_backward needs (overwritten by the next forward with a work buffer).
 * batch must be a multiple of 32.  Returns APM_OK, APM_EINVAL or APM_EDEVICE.
 */
apm_status apm_mlp_forward(const apm_mlp *net, const uint16_t *x, int32_t batch, float *out, void *work,
                           apm_stream stream);

/*
 * apm_mlp_backward -- grad = d/dparam of sum(out * dout), for the rows of the last
 * forward that used `work`.  The BF16 rounding of inputs and activations is taken as
 * the identity in the derivative; the operands of the products (dout and the hidden
 * gradients) enter as BF16.  Overwrites net->grad.
 */
apm_status apm_mlp_backward(const apm_mlp *net, const float *dout, int32_t batch, void *work,
                            apm_stream stream);

/* One Adam step on param with grad; updates adam_m, adam_v and the BF16 copies. */
apm_status apm_mlp_adam(const apm_mlp *net, const apm_adam *h, apm_stream stream);

/* ------------------------------------------------------------------ Monte Carlo */
#define APM_MC_MAX_N 16

typedef struct {
    int32_t n;                /* vertices per configuration, 2..APM_MC_MAX_N               */
    int32_t L;                /* lattice side, 1..256                                     */
    int32_t n_tau;            /* time points, 1..32768                                    */
    int32_t n_bin;            /* time bins of the learned proposal, 1..64, divides n_tau  */
    double eps;               /* uniform fraction of the learned proposal, in [0, 1]      */
    double resolve;           /* >= 0: a configuration whose |c[V]| is below resolve * d[V]
                                 has weight 0, with d[V] = |a[V]| + sum over T containing
                                 vertex 0, T != V, of |c[T]| |a[V \ T]| (the rounding
                                 scale of the recursion at V); 0 keeps every nonzero c[V] */
    const double *g0;         /* [(2 n_tau - 1) x L^2] fp64: row d + n_tau - 1 holds the
                                 time difference d beta / n_tau (d = 0 is 0^-), column
                                 dy*L + dx the site difference mod L                     */
} apm_mc_model;

typedef struct {
    int32_t walkers;          /* W >= 0                                                   */
    uint32_t *state;          /* [W x n] packed vertices, updated in place                */
    double *logw;             /* [W] log|c[V]| of the current configuration (-inf: 0)     */
    int8_t *sign;             /* [W] sign of c[V] (0 when it is zero or not finite)       */
} apm_mc_chain;

/* Optional per-step outputs: each a [W] device array, or NULL. */
typedef struct {
    int32_t *moved;           /* moved vertex k                                           */
    uint32_t *proposed;       /* proposed vertex v'                                       */
    double *logq;             /* log q~(v_k | ctx) - log q~(v' | ctx) (0 for uniform)     */
    double *logc_prop;        /* log|c[V](X')| of the proposal (-inf for 0 / non-finite)  */
    uint8_t *accepted;        /* 1 if the move was accepted                               */
    float *obs_logw;          /* log|c[V]| after the step                                 */
    int8_t *obs_sign;         /* sign of c[V] after the step                              */
    float *loss;              /* [1] mean squared error of the training step (if trained) */
} apm_mc_record;

/* Bytes of the work buffer of apm_mc_evaluate / apm_mc_step for W walkers; with_net != 0
 * adds what the learned proposal and its training need. */
int64_t apm_mc_work_bytes(const apm_mc_model *m, int32_t walkers, int32_t with_net);

/* logw and sign of the current configurations (initialisation).  Invalid vertices
 * (site >= L^2 or time point >= n_tau) and unresolved weights give logw = -inf,
 * sign = 0. */
apm_status apm_mc_evaluate(const apm_mc_model *m, const apm_mc_chain *ch, void *work, apm_stream stream);

/*
 * apm_mc_step -- one Metropolis-Hastings step of every walker.
 *   1. k uniform; context = the other n-1 vertices sorted by packed value (time point,
 *      then site); features (x/L, y/L, (j+1/2)/n_tau) per context vertex, BF16.
 *   2. net == NULL: v' uniform over sites x time points.  Otherwise, out = net(features)
 *      (d_in = 3(n-1), d_out = L^2 + n_bin: site logits then bin logits); with
 *      probability eps v' is uniform, else site ~ softmax(site logits), bin ~
 *      softmax(bin logits), time point uniform in the bin;
 *      q~(v) = (1-eps) p_site p_bin / (n_tau/n_bin) + eps / (L^2 n_tau).
 *      Categorical draws take the first index whose running sum exceeds u * total.
 *   3. c[V](X') via the minors and the rooted connected-sum recursion.
 *   4. accept iff log u < log|c'| - log|c| + log q~(v_k) - log q~(v'); a zero,
 *      unresolved or non-finite c' is rejected; a walker at weight 0 moves to any
 *      proposal of nonzero weight.
 *   5. train != NULL (requires net): regression of site logit + bin logit of v' on
 *      log|c'| clipped below at (batch maximum - 30), mean squared error over the
 *      walkers, then apm_mlp_backward and one Adam step with *train.
 * walkers must be a multiple of 32 when net != NULL.
 * Returns APM_OK, APM_EINVAL, APM_EUNSUPPORTED (n > APM_MC_MAX_N) or APM_EDEVICE.
 */
apm_status apm_mc_step(const apm_mc_model *m, const apm_mc_chain *ch, const apm_mlp *net,
                       const apm_adam *train, uint64_t seed, int32_t step, const apm_mc_record *rec,
                       void *work, apm_stream stream);

/*
 * The parts of apm_mc_step, for callers that supply their own proposal logits.
 *   apm_mc_context: moved [W] and, if feat != NULL, features [W x Dp] BF16 (step 1).
 *   apm_mc_propose: proposed [W], logq [W] and the proposal's matrices [W x n x n]
 *                   from logits [W x logit_stride] fp32 (NULL: uniform) (step 2).
 *   apm_mc_accept:  c[V] of `mats`, then the decision and state update (steps 3-4);
 *                   work as for apm_mc_step without a network.
 */
apm_status apm_mc_context(const apm_mc_model *m, const apm_mc_chain *ch, uint64_t seed, int32_t step,
                          int32_t *moved, uint16_t *feat, apm_stream stream);
apm_status apm_mc_propose(const apm_mc_model *m, const apm_mc_chain *ch, uint64_t seed, int32_t step,
                          const int32_t *moved, const float *logits, int32_t logit_stride, uint32_t *proposed,
                          double *logq, double *mats, apm_stream stream);
apm_status apm_mc_accept(const apm_mc_model *m, const apm_mc_chain *ch, uint64_t seed, int32_t step,
                         const int32_t *moved, const uint32_t *proposed, const double *logq, const double *mats,
                         const apm_mc_record *rec, void *work, apm_stream stream);

#ifdef __cplusplus
}
#endif

#endif /* APM_MC_H */
