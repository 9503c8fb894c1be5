// apm_kernels.h -- host-side entry points of the kernel translation units (internal).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace apm {

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
};

hipError_t fpm_launch(const LaunchMinors& L, hipStream_t st);
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

}  // namespace apm
