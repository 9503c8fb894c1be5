// apm_kernels.h -- host-side entry points of the kernel translation units (internal).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace apm {

// Default relative pivot-shift threshold of the minors tree, every element type.
constexpr double kDefaultPivTol = 1e-3;

// Queue-preparation workspace: int32 counter[0] is the mixed-order queue head, counter[1] the
// head of the large-order queue, counter[kBucketBase + k] (k = 0..22) the start in the queue
// order of the matrices of order 20 - k (k = 21: invalid orders; k = 22: the end); ints 32..63
// hold the persistent kernels' per-stream queue heads (256 bytes in all).
constexpr int kBucketBase = 8;

struct LaunchMinors {
    int dtype;                 // apm_dtype
    const void* A;
    void* out;
    int16_t* ex;
    int32_t* info;
    int32_t batch;
    int32_t n_uniform;         // > 0 uniform order; 0 ragged (n, order, counter used)
    const int32_t* n;          // ragged: per-matrix orders
    int32_t n_max;             // ragged: bound on n[]
    const int64_t* in_off;
    const int64_t* out_off;
    double tau;
    bool perturb, out_f64;
    int32_t* order;            // ragged: workspace [batch] (matrix indices, descending n)
    int32_t* counter;          // ragged: workspace, queue head
    int64_t* ioff_ws;          // ragged: workspace [batch] packed input offsets (if in_off == NULL)
    int64_t* ooff_ws;          // ragged: workspace [batch] packed output offsets (if out_off == NULL)
    int n_workers;             // ragged: number of compute units (persistent grid sizing)
    int force_k0;              // > 0: lane-subtree order to use (autotuning, plans); 0: the table
                               // (mixed orders: that of the orders other than 14..16)
    int force_k0_big;          // mixed orders: > 0: that of the orders 14..16; 0: the table
    int32_t* topq;             // uniform batches: deferred top-level correction queue (NULL: none)
    int32_t topq_cap;          // its capacity in matrices (fpm_topq_bytes of that many)
    bool no_split;             // one work item per matrix (bit-identical results either way)
};

// Leading ints of a deferred-correction queue that hold its counters (the listed matrices and
// the completion counts of the correction launch): zero before a launch that uses it.
constexpr int kTopCounterInts = 10;

// Bytes of a deferred-correction queue for `batch` matrices: a slot and a list entry per
// matrix and one info code per work item of a split launch (zeroed once at allocation; each
// use leaves it zeroed).
int64_t fpm_topq_bytes(int64_t batch);
// The part of it that a launch with one work item per matrix (no_split) uses.
int64_t fpm_topq_bytes_unsplit(int64_t batch);

hipError_t fpm_launch(const LaunchMinors& L, hipStream_t st);

// Lane-subtree order per (dtype, order): tuned values installed by the autotuner
// (0 = none), the instantiated range of a dtype, and the synthetic tuning input.
int tuned_k0(int dtype, int n);
void set_tuned_k0(int dtype, int n, int k0);
void k0_range(int dtype, int* lo, int* hi);
// The same for the two kernels of a mixed-order launch (which 0: orders other than 14..16,
// 1: orders 14..16): tuned value (0 = none), instantiated range, default.
int tuned_mixed_k0(int dtype, int which);
void set_tuned_mixed_k0(int dtype, int which, int k0);
void mixed_k0_range(int dtype, int which, int* lo, int* hi, int* def);
// Synthetic mixed-order tuning input: orders nv (device, [batch]) at packed offsets ioff.
hipError_t fill_tune_input_mixed(void* A, int dtype, const int32_t* nv, const int64_t* ioff, int batch,
                                 hipStream_t st);
hipError_t fill_tune_input(void* A, int dtype, int n, int batch, hipStream_t st);
hipError_t fpm_prep_launch(const LaunchMinors& L, hipStream_t st);   // ragged-batch queue preparation

struct LaunchCS {
    const double* m_up;
    const double* m_dn;
    double* c;
    int32_t batch;
    int32_t n_uniform;
    const int32_t* n;
    int32_t n_max;
    const int64_t* off;        // element offsets (shared by inputs and output), may be NULL
    uint32_t mode;
    double* summ;              // rooted, orders <= 12 only: (c[V], d[V]) per matrix instead of c[]
    const int32_t* order;      // mixed orders: matrix indices by decreasing order (queue preparation), or NULL
};

hipError_t cs_launch(const LaunchCS& L, hipStream_t st);

struct LaunchPerm {
    const double* A;
    double* out;
    int32_t batch;
    int32_t n_uniform;
    const int32_t* n;
    int32_t n_max;
    const int64_t* in_off;
    const int64_t* out_off;
};

hipError_t perm_launch(const LaunchPerm& L, hipStream_t st);

struct LaunchXor {
    int dtype;                 // apm_dtype: R64 or C128
    const void* A;             // [batch][2n][2n]
    void* out;                 // [batch][2^(n+1) - 2]
    int32_t* info;
    int32_t batch;
    int n;                     // blocks per matrix
    void* ws;                  // top-level node matrices, ws_stride elements per matrix
    int64_t ws_stride;
    int mode;                  // 0: XOR minors [batch][2^(n+1) - 2]; 1: XNOR [batch][2^n];
                               // 2: NAND [batch][3^n]
};

// Elements of top-level workspace per matrix with n blocks (0: none needed).
int64_t xor_ws_elems(int n, int mode);
hipError_t xor_launch(const LaunchXor& L, hipStream_t st);

// Leading principal minors: [batch][n] of [batch][n][n] (dtype R64 or C128, n <= 32).
hipError_t lead_launch(int dtype, const void* A, void* out, int32_t* info, int32_t batch, int n, hipStream_t st);

// ---------------------------------------------------------------- proposal network
struct MlpNet {
    int dp, op;                // padded input / output sizes
    float* param;
    float* grad;
    float* m;
    float* v;
    uint16_t* w;
    uint16_t* wt;
};

struct MlpWork {
    float* h1;                 // [B][128] fp32 activations
    float* h2;
    uint16_t* actT;            // [Dp + 256][B] bf16: x^T | h1^T | h2^T
    uint16_t* gT;              // [Op + 256][B] bf16: dout^T | dz2^T | dz1^T
};

int64_t mlp_param_count(int dp, int op);
int64_t mlp_weight_count(int dp, int op);
int64_t mlp_work_bytes(int dp, int op, int B);
MlpWork mlp_work_carve(void* work, int dp, int op, int B);
hipError_t mlp_forward_launch(const MlpNet& net, const uint16_t* x, int B, float* out, const MlpWork* wk,
                              hipStream_t st);
hipError_t mlp_backward_launch(const MlpNet& net, const float* dout, int B, const MlpWork& wk, hipStream_t st);
hipError_t mlp_adam_launch(const MlpNet& net, bool update, float lr, float b1, float b2, float eps, int t,
                           hipStream_t st);

// ---------------------------------------------------------------- Monte Carlo step
struct McArgs {
    int n, L, n_tau, n_bin;
    double eps;
    double resolve;
    const double* g0;
    int W;
    uint32_t* state;
    double* logw;
    int8_t* sign;
    uint64_t seed;
    int step;
    // the step's draw table: draws 0 and 1 of walker w at entries 2 w and 2 w + 1, 4 x uint64
    // each.  NULL: every kernel computes the draws it needs.  Otherwise the first kernel of
    // the step that needs them computes and stores them (draws_ready = 0), the later ones
    // read them (draws_ready = 1).
    uint64_t* draws;
    int draws_ready;
};

hipError_t mc_context_launch(const McArgs& a, int32_t* moved, uint16_t* feat, int dp, hipStream_t st);
// moved_out != NULL: draw the moved vertex (as mc_context_launch does) into moved_out
// instead of reading it from moved.
hipError_t mc_propose_launch(const McArgs& a, const int32_t* moved, int32_t* moved_out, const float* logits,
                             int stride, uint32_t* prop, double* logq, double* mats, hipStream_t st);
hipError_t mc_gather_launch(const McArgs& a, double* mats, hipStream_t st);
// summ (if not NULL): per-walker (c[V], d[V]) written by the connected-sum kernel; else
// c[V] and d[V] are formed from the full c[] and minors arrays.
hipError_t mc_accept_launch(const McArgs& a, const int32_t* moved, const uint32_t* prop, const double* logq,
                            const double* c, const double* minors, const double* summ, double* logc_out,
                            uint8_t* acc_out, float* obs_logw, int8_t* obs_sign, hipStream_t st);
hipError_t mc_set_launch(const McArgs& a, const double* c, const double* minors, const double* summ,
                         hipStream_t st);
hipError_t mc_loss_launch(const McArgs& a, const float* logits, int Op, const uint32_t* prop, const double* logc,
                          float* gbuf, float* dout, float* loss, double clip, hipStream_t st);

}  // namespace apm
