// api.hip -- the C ABI of libapm.so: argument validation, workspaces, launches.
#include <math.h>
#include <stdlib.h>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "../../include/apm.h"
#include "apm_kernels.h"

namespace {

thread_local int g_last_hip_error = 0;

apm_status from_hip(hipError_t e)
{
    if (e == hipSuccess) return APM_OK;
    g_last_hip_error = (int)e;
    if (e == hipErrorOutOfMemory) return APM_ENOMEM;
    return APM_EDEVICE;
}

// Per-device workspace for ragged batches: queue head, queue order, packed offsets.
struct Workspace {
    void* buf = nullptr;        // counter (256 B) | order [cap] int32 | ioff [cap] int64 | ooff [cap] int64
    int64_t cap = 0;
    int cus = 0;
};

std::mutex g_ws_mu;
std::vector<Workspace> g_ws;

apm_status get_workspace(int64_t batch, int32_t** counter, int32_t** order, int64_t** ioff, int64_t** ooff,
                         int* cus)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return from_hip(e);
    std::lock_guard<std::mutex> lk(g_ws_mu);
    if ((int)g_ws.size() <= dev) g_ws.resize(dev + 1);
    Workspace& w = g_ws[dev];
    if (w.cus == 0) {
        int v = 0;
        e = hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return from_hip(e);
        w.cus = v;
    }
    if (w.cap < batch) {
        if (w.buf) (void)hipFree(w.buf);
        w.buf = nullptr;
        int64_t cap = batch < 4096 ? 4096 : batch;
        e = hipMalloc(&w.buf, 256 + (size_t)cap * (4 + 8 + 8));
        if (e != hipSuccess) { w.cap = 0; return from_hip(e); }
        w.cap = cap;
    }
    char* p = static_cast<char*>(w.buf);
    *counter = reinterpret_cast<int32_t*>(p);
    *order = reinterpret_cast<int32_t*>(p + 256);
    *ioff = reinterpret_cast<int64_t*>(p + 256 + (size_t)w.cap * 4);
    *ooff = reinterpret_cast<int64_t*>(p + 256 + (size_t)w.cap * 12);
    *cus = w.cus;
    return APM_OK;
}

// Per-(device, stream) queue of deferred top-level corrections for uniform batches.  Each
// use leaves it zeroed; a call that failed after using it marks it for re-zeroing.  It is
// only (re)allocated or re-zeroed outside stream capture: a captured call that would need
// that runs the corrections inside the minors kernel instead.
struct TopQueue {
    void* buf = nullptr;
    int64_t cap = 0;
    bool dirty = false;
};
std::map<std::pair<int, hipStream_t>, TopQueue> g_topq;

int32_t* get_topq(hipStream_t st, int64_t batch, int32_t* cap_out, TopQueue** q_out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    std::lock_guard<std::mutex> lk(g_ws_mu);
    TopQueue& q = g_topq[std::make_pair(dev, st)];
    if (q.cap < batch || q.dirty) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return nullptr;
        if (q.cap < batch) {
            if (q.buf) (void)hipFree(q.buf);
            q.buf = nullptr;
            q.cap = 0;
            const int64_t cap = batch < 4096 ? 4096 : batch;
            if (hipMalloc(&q.buf, (size_t)apm::fpm_topq_bytes(cap)) != hipSuccess) {
                q.buf = nullptr;
                return nullptr;
            }
            q.cap = cap;
        }
        if (hipMemsetAsync(q.buf, 0, (size_t)apm::fpm_topq_bytes(q.cap), st) != hipSuccess) return nullptr;
        q.dirty = false;
    }
    *cap_out = (int32_t)q.cap;
    *q_out = &q;
    return static_cast<int32_t*>(q.buf);
}

bool bad_batch(const apm_batch* bd, int nmax)
{
    if (!bd || bd->batch < 0) return true;
    if (bd->n_uniform < 0) return true;
    if (bd->n_uniform == 0 && bd->batch > 0 && !bd->n) return true;
    if (bd->n_uniform == 0 && (bd->n_max < 0)) return true;
    (void)nmax;
    return false;
}

// Packed default offsets of a ragged batch given without offset arrays: the queue
// preparation kernel writes the prefix sums of n_b^2 and 2^n_b into the workspace.
apm_status packed_offsets(const apm_batch* bd, hipStream_t st, const int64_t** ioff, const int64_t** ooff)
{
    apm::LaunchMinors L{};
    L.batch = bd->batch;
    L.n = bd->n;
    apm_status s = get_workspace(bd->batch, &L.counter, &L.order, &L.ioff_ws, &L.ooff_ws, &L.n_workers);
    if (s != APM_OK) return s;
    hipError_t e = apm::fpm_prep_launch(L, st);
    if (e != hipSuccess) return from_hip(e);
    *ioff = L.ioff_ws;
    *ooff = L.ooff_ws;
    return APM_OK;
}

}  // namespace

extern "C" {

const char* apm_status_str(apm_status s)
{
    switch (s) {
    case APM_OK: return "APM_OK";
    case APM_EINVAL: return "APM_EINVAL: invalid argument";
    case APM_EUNSUPPORTED: return "APM_EUNSUPPORTED: unsupported size or variant";
    case APM_EDEVICE: return "APM_EDEVICE: HIP error";
    case APM_ENOMEM: return "APM_ENOMEM: device allocation failed";
    default: return "APM_?: unknown status";
    }
}

int apm_last_hip_error(void) { return g_last_hip_error; }

int apm_version(void) { return 100; }

apm_status apm_all_minors(apm_dtype dt, const void* A, const apm_batch* bd, void* minors, int16_t* exp,
                          int32_t* info, const apm_opts* opt, apm_stream stream)
{
    if ((int)dt < 0 || (int)dt > 3) return APM_EINVAL;
    if (bad_batch(bd, APM_MAX_N)) return APM_EINVAL;
    const bool scaled = (dt == APM_R32S || dt == APM_C64S);
    const uint32_t flags = opt ? opt->flags : 0u;
    if (flags & ~(APM_OUT_F64 | APM_NO_PERTURB)) return APM_EINVAL;
    const bool out_f64 = (flags & APM_OUT_F64) != 0;
    if (opt && !isfinite(opt->piv_tol)) return APM_EINVAL;
    if (bd->n_uniform > APM_MAX_N || bd->n_max > APM_MAX_N) return APM_EUNSUPPORTED;
    if (bd->batch == 0) return APM_OK;
    if (!A || !minors) return APM_EINVAL;
    if (scaled && !out_f64 && !exp) return APM_EINVAL;
    if ((!scaled || out_f64) && exp) return APM_EINVAL;

    apm::LaunchMinors L{};
    L.dtype = (int)dt;
    L.A = A;
    L.out = minors;
    L.ex = exp;
    L.info = info;
    L.batch = bd->batch;
    L.n_uniform = bd->n_uniform;
    L.n = bd->n;
    L.n_max = bd->n_max > 0 ? bd->n_max : APM_MAX_N;
    L.in_off = bd->in_off;
    L.out_off = bd->out_off;
    const double tau_def = scaled ? 1e-3 : 1e-4;
    L.tau = (opt && opt->piv_tol > 0) ? opt->piv_tol : tau_def;
    L.perturb = !(flags & APM_NO_PERTURB);
    L.out_f64 = out_f64;
    TopQueue* tq = nullptr;
    if (bd->n_uniform == 0) {
        apm_status s = get_workspace(bd->batch, &L.counter, &L.order, &L.ioff_ws, &L.ooff_ws, &L.n_workers);
        if (s != APM_OK) return s;
    } else if (bd->batch <= INT32_MAX / 2) {
        L.topq = get_topq((hipStream_t)stream, bd->batch, &L.topq_cap, &tq);
    }
    const hipError_t e = apm::fpm_launch(L, (hipStream_t)stream);
    if (e != hipSuccess && tq) {
        std::lock_guard<std::mutex> lk(g_ws_mu);
        tq->dirty = true;
    }
    return from_hip(e);
}

int32_t apm_minors_k0(apm_dtype dt, int32_t n)
{
    if ((int)dt < 0 || (int)dt > 3 || n < 1 || n > APM_MAX_N) return -1;
    const char* e = getenv("APM_K0");
    int k = e ? atoi(e) : 0;
    if (k <= 0) k = apm::tuned_k0((int)dt, n);
    if (k <= 0) {
        static const int def[4] = {5, 5, 3, 4};   // the per-type defaults of the kernels
        k = def[(int)dt];
    }
    int lo, hi;
    apm::k0_range((int)dt, &lo, &hi);
    return k < lo ? lo : (k > hi ? hi : k);
}

apm_status apm_autotune_minors(apm_dtype dt, int32_t n, int32_t batch, int32_t* k0_out, apm_stream stream)
{
    if ((int)dt < 0 || (int)dt > 3 || n < 1 || n > APM_MAX_N || batch < 1) return APM_EINVAL;
    const hipStream_t st = (hipStream_t)stream;
    const bool cplx = (dt == APM_C128 || dt == APM_C64S), scaled = (dt == APM_R32S || dt == APM_C64S);
    const size_t in_b = (size_t)batch * n * n * (cplx ? 16 : 8);
    const size_t out_b = ((size_t)batch << n) * (scaled ? (cplx ? 8 : 4) : (cplx ? 16 : 8));
    const size_t ex_b = scaled ? ((size_t)batch << n) * 2 : 0;
    void *A = nullptr, *out = nullptr, *ex = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int lo, hi;
    apm::k0_range((int)dt, &lo, &hi);
    int best = apm_minors_k0(dt, n);
    hipError_t e = hipMalloc(&A, in_b);
    if (e == hipSuccess) e = hipMalloc(&out, out_b);
    if (e == hipSuccess && ex_b) e = hipMalloc(&ex, ex_b);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = apm::fill_tune_input(A, (int)dt, n, batch, st);
    if (e == hipSuccess && n > 6) {
        float best_ms = 3.4e38f;
        int prev_eff = -1;
        for (int k = lo; k <= hi && e == hipSuccess; ++k) {
            const int eff = (n - 6) < k ? (n - 6) : k;     // the order actually used
            if (eff == prev_eff) continue;
            prev_eff = eff;
            apm::LaunchMinors L{};
            L.dtype = (int)dt;
            L.A = A;
            L.out = out;
            L.ex = static_cast<int16_t*>(ex);
            L.batch = batch;
            L.n_uniform = n;
            L.n_max = n;
            L.tau = scaled ? 1e-3 : 1e-4;
            L.perturb = true;
            L.force_k0 = k;
            e = apm::fpm_launch(L, st);                       // warm-up
            if (e == hipSuccess) e = hipEventRecord(e0, st);
            for (int r = 0; r < 3 && e == hipSuccess; ++r) e = apm::fpm_launch(L, st);
            if (e == hipSuccess) e = hipEventRecord(e1, st);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e == hipSuccess && ms < best_ms) {
                best_ms = ms;
                best = k;
            }
        }
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (ex) (void)hipFree(ex);
    if (out) (void)hipFree(out);
    if (A) (void)hipFree(A);
    if (e != hipSuccess) return from_hip(e);
    apm::set_tuned_k0((int)dt, n, best);
    if (k0_out) *k0_out = best;
    return APM_OK;
}

apm_status apm_connected_sums(const double* m_up, const double* m_dn, const apm_batch* bd, double* c,
                              uint32_t mode, apm_stream stream)
{
    if (bad_batch(bd, APM_MAX_N_CS)) return APM_EINVAL;
    if (mode & ~(APM_CS_ALL | APM_CS_WEIGHTS)) return APM_EINVAL;
    if ((mode & APM_CS_WEIGHTS) && m_dn) return APM_EINVAL;
    if (bd->n_uniform > APM_MAX_N_CS || bd->n_max > APM_MAX_N_CS) return APM_EUNSUPPORTED;
    if (bd->in_off != bd->out_off) return APM_EINVAL;   // one offset array indexes inputs and output
    if (bd->batch == 0) return APM_OK;
    if (!m_up || !c) return APM_EINVAL;
    if (c == m_up || c == m_dn) return APM_EINVAL;      // the output must not alias the inputs
    apm::LaunchCS L{};
    L.m_up = m_up;
    L.m_dn = m_dn;
    L.c = c;
    L.batch = bd->batch;
    L.n_uniform = bd->n_uniform;
    L.n = bd->n;
    L.n_max = bd->n_max > 0 ? bd->n_max : APM_MAX_N_CS;
    L.off = bd->out_off;
    L.mode = mode;
    if (bd->n_uniform == 0 && !L.off) {
        const int64_t* ioff = nullptr;
        apm_status s = packed_offsets(bd, (hipStream_t)stream, &ioff, &L.off);
        if (s != APM_OK) return s;
    }
    return from_hip(apm::cs_launch(L, (hipStream_t)stream));
}

apm_status apm_all_perm_minors(const double* A, const apm_batch* bd, double* perm, apm_stream stream)
{
    if (bad_batch(bd, APM_MAX_N_PERM)) return APM_EINVAL;
    if (bd->n_uniform > APM_MAX_N_PERM || bd->n_max > APM_MAX_N_PERM) return APM_EUNSUPPORTED;
    if (bd->batch == 0) return APM_OK;
    if (!A || !perm) return APM_EINVAL;
    apm::LaunchPerm L{};
    L.A = A;
    L.out = perm;
    L.batch = bd->batch;
    L.n_uniform = bd->n_uniform;
    L.n = bd->n;
    L.n_max = bd->n_max > 0 ? bd->n_max : APM_MAX_N_PERM;
    L.in_off = bd->in_off;
    L.out_off = bd->out_off;
    if (bd->n_uniform == 0 && (!L.in_off || !L.out_off)) {
        const int64_t *ioff = nullptr, *ooff = nullptr;
        apm_status s = packed_offsets(bd, (hipStream_t)stream, &ioff, &ooff);
        if (s != APM_OK) return s;
        if (!L.in_off) L.in_off = ioff;
        if (!L.out_off) L.out_off = ooff;
    }
    return from_hip(apm::perm_launch(L, (hipStream_t)stream));
}

}  // extern "C"
