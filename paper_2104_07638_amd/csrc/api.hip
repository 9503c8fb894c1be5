// api.hip -- the C ABI of libapm.so: argument validation, workspaces, launches.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <map>
#include <string>
#include <mutex>
#include <new>
#include <utility>
#include <vector>

#include <sys/stat.h>

#include "../../include/apm.h"
#include "apm_kernels.h"

namespace {

thread_local int g_last_hip_error = 0;
thread_local int g_unreported_hip_error = 0;   // cleared by apm_last_device_error

apm_status from_hip(hipError_t e)
{
    if (e == hipSuccess) return APM_OK;
    g_last_hip_error = (int)e;
    g_unreported_hip_error = (int)e;
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

// Buffers replaced by larger ones.  A graph captured from an earlier call may still hold
// their addresses, so they are kept (never freed) until the process ends; capacities grow
// at least geometrically, so the retired ones together never exceed the live one.
std::vector<void*> g_retired;

void retire(void* p)
{
    if (p) g_retired.push_back(p);
}

int64_t grown(int64_t cur, int64_t need, int64_t floor_cap)
{
    int64_t cap = cur * 2;
    if (cap < need) cap = need;
    return cap < floor_cap ? floor_cap : cap;
}

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
        const int64_t cap = grown(w.cap, batch, 4096);
        void* nb = nullptr;
        e = hipMalloc(&nb, 256 + (size_t)cap * (4 + 8 + 8));
        if (e != hipSuccess) return from_hip(e);
        retire(w.buf);
        w.buf = nb;
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
            const int64_t cap = grown(q.cap, batch, 4096);
            void* nb = nullptr;
            if (hipMalloc(&nb, (size_t)apm::fpm_topq_bytes(cap)) != hipSuccess) return nullptr;
            retire(q.buf);
            q.buf = nb;
            q.cap = cap;
        }
        if (hipMemsetAsync(q.buf, 0, (size_t)apm::fpm_topq_bytes(q.cap), st) != hipSuccess) return nullptr;
        q.dirty = false;
    }
    *cap_out = (int32_t)q.cap;
    *q_out = &q;
    return static_cast<int32_t*>(q.buf);
}

// Per-(device, stream) workspace of the XOR minors' top levels (node matrices), grown on
// demand outside stream capture; calls on one stream are ordered by the stream.
struct XorWs {
    void* buf = nullptr;
    size_t cap = 0;
};
std::map<std::pair<int, hipStream_t>, XorWs> g_xws;

apm_status get_xor_ws(hipStream_t st, size_t bytes, void** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return from_hip(e);
    std::lock_guard<std::mutex> lk(g_ws_mu);
    XorWs& w = g_xws[std::make_pair(dev, st)];
    if (w.cap < bytes) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        e = hipStreamIsCapturing(st, &cs);
        if (e != hipSuccess) return from_hip(e);
        if (cs != hipStreamCaptureStatusNone) return APM_EUNSUPPORTED;
        const size_t cap = bytes > 2 * w.cap ? bytes : 2 * w.cap;
        void* nb = nullptr;
        e = hipMalloc(&nb, cap);
        if (e != hipSuccess) return from_hip(e);
        retire(w.buf);
        w.buf = nb;
        w.cap = cap;
    }
    *out = w.buf;
    return APM_OK;
}

// ---- persistent cache of autotuned lane-subtree orders -------------------------------------
// A JSON file {"version": 1, "k0": {"<gfx>/<dtype>/<n>": K0, ...}} (gfx: the device's
// architecture name up to its first ':'; <n> an order, or "mixed" / "mixed-large" for the
// two kernels of a mixed-order launch), written by apm_autotune_minors and
// apm_autotune_minors_mixed and read by plan creation with APM_PLAN_AUTOTUNE.  Path:
// APM_TUNE_CACHE, else $HOME/.cache/apm_tune.json; an empty APM_TUNE_CACHE disables the
// cache.  Unreadable or malformed files are ignored.
const char* kDtypeName[4] = {"r64", "r32s", "c128", "c64s"};
const char* kMixedKey[2] = {"mixed", "mixed-large"};

std::string tune_cache_path()
{
    const char* e = getenv("APM_TUNE_CACHE");
    if (e) return std::string(e);
    const char* h = getenv("HOME");
    if (!h || !*h) return std::string();
    return std::string(h) + "/.cache/apm_tune.json";
}

bool device_arch(std::string* out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return false;
    std::string a(prop.gcnArchName);
    const size_t c = a.find(':');
    *out = c == std::string::npos ? a : a.substr(0, c);
    return !out->empty();
}

// Reads "key": value pairs of the "k0" object.  Returns false if the file is missing or malformed.
bool tune_cache_read(const std::string& path, std::map<std::string, int>* kv)
{
    FILE* f = path.empty() ? nullptr : fopen(path.c_str(), "rb");
    if (!f) return false;
    std::string txt;
    char buf[4096];
    size_t r;
    while ((r = fread(buf, 1, sizeof buf, f)) > 0 && txt.size() < (1u << 20)) txt.append(buf, r);
    fclose(f);
    const size_t k = txt.find("\"k0\"");
    if (k == std::string::npos) return false;
    size_t i = txt.find('{', k);
    if (i == std::string::npos) return false;
    for (++i; i < txt.size();) {
        const size_t q0 = txt.find_first_of("\"}", i);
        if (q0 == std::string::npos) return false;
        if (txt[q0] == '}') return true;
        const size_t q1 = txt.find('"', q0 + 1);
        if (q1 == std::string::npos) return false;
        const std::string key = txt.substr(q0 + 1, q1 - q0 - 1);
        const size_t colon = txt.find(':', q1);
        if (colon == std::string::npos) return false;
        char* end = nullptr;
        const long v = strtol(txt.c_str() + colon + 1, &end, 10);
        if (end == txt.c_str() + colon + 1) return false;
        (*kv)[key] = (int)v;
        i = (size_t)(end - txt.c_str());
    }
    return false;
}

bool tune_cache_write(const std::string& path, const std::map<std::string, int>& kv)
{
    if (path.empty()) return false;
    const size_t slash = path.rfind('/');
    if (slash != std::string::npos && slash > 0) {
        const std::string dir = path.substr(0, slash);
        (void)mkdir(dir.c_str(), 0755);
    }
    const std::string tmp = path + ".tmp";
    FILE* f = fopen(tmp.c_str(), "wb");
    if (!f) return false;
    fprintf(f, "{\n  \"version\": 1,\n  \"k0\": {");
    bool first = true;
    for (const auto& e : kv) {
        fprintf(f, "%s\n    \"%s\": %d", first ? "" : ",", e.first.c_str(), e.second);
        first = false;
    }
    fprintf(f, "\n  }\n}\n");
    const bool ok = fclose(f) == 0;
    return ok && rename(tmp.c_str(), path.c_str()) == 0;
}

std::mutex g_tune_mu;

// Installs the cached values of this device's architecture; returns how many.
int tune_cache_install(const std::string& path)
{
    std::string arch;
    if (!device_arch(&arch)) return -1;
    std::map<std::string, int> kv;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (!tune_cache_read(path, &kv)) return -1;
    int count = 0;
    for (int dt = 0; dt < 4; ++dt) {
        for (int n = 1; n <= APM_MAX_N; ++n) {
            const auto it = kv.find(arch + "/" + kDtypeName[dt] + "/" + std::to_string(n));
            if (it == kv.end()) continue;
            int lo, hi;
            apm::k0_range(dt, &lo, &hi);
            if (it->second < lo || it->second > hi) continue;
            apm::set_tuned_k0(dt, n, it->second);
            ++count;
        }
        for (int w = 0; w < 2; ++w) {
            const auto it = kv.find(arch + "/" + kDtypeName[dt] + "/" + kMixedKey[w]);
            if (it == kv.end()) continue;
            int lo, hi, def;
            apm::mixed_k0_range(dt, w, &lo, &hi, &def);
            if (it->second < lo || it->second > hi) continue;
            apm::set_tuned_mixed_k0(dt, w, it->second);
            ++count;
        }
    }
    return count;
}

// Records (key suffix -> K0) entries of dtype dt in the cache file.
void tune_cache_record_keys(int dt, const std::pair<std::string, int>* e, int count)
{
    std::string arch;
    if (!device_arch(&arch)) return;
    const std::string path = tune_cache_path();
    if (path.empty()) return;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    std::map<std::string, int> kv;
    (void)tune_cache_read(path, &kv);
    for (int i = 0; i < count; ++i) kv[arch + "/" + kDtypeName[dt] + "/" + e[i].first] = e[i].second;
    (void)tune_cache_write(path, kv);
}

void tune_cache_record(int dt, int n, int k0)
{
    const std::pair<std::string, int> e(std::to_string(n), k0);
    tune_cache_record_keys(dt, &e, 1);
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

// Argument checks and launch descriptions shared by the direct calls and the plans.  On
// APM_OK with *noop set the batch is empty and nothing is to be enqueued.
apm_status minors_args(apm_dtype dt, const void* A, const apm_batch* bd, void* minors, int16_t* exp,
                       int32_t* info, const apm_opts* opt, apm::LaunchMinors* L, bool* noop)
{
    *noop = false;
    if ((int)dt < 0 || (int)dt > 3) return APM_EINVAL;
    if (bad_batch(bd, APM_MAX_N)) return APM_EINVAL;
    const bool scaled = (dt == APM_R32S || dt == APM_C64S);
    const uint32_t flags = opt ? opt->flags : 0u;
    if (flags & ~(APM_OUT_F64 | APM_NO_PERTURB)) return APM_EINVAL;
    const bool out_f64 = (flags & APM_OUT_F64) != 0;
    if (opt && !isfinite(opt->piv_tol)) return APM_EINVAL;
    if (bd->n_uniform > APM_MAX_N || bd->n_max > APM_MAX_N) return APM_EUNSUPPORTED;
    if (bd->batch == 0) {
        *noop = true;
        return APM_OK;
    }
    if (!A || !minors) return APM_EINVAL;
    if (scaled && !out_f64 && !exp) return APM_EINVAL;
    if ((!scaled || out_f64) && exp) return APM_EINVAL;
    *L = apm::LaunchMinors{};
    L->dtype = (int)dt;
    L->A = A;
    L->out = minors;
    L->ex = exp;
    L->info = info;
    L->batch = bd->batch;
    L->n_uniform = bd->n_uniform;
    L->n = bd->n;
    L->n_max = bd->n_max > 0 ? bd->n_max : APM_MAX_N;
    L->in_off = bd->in_off;
    L->out_off = bd->out_off;
    L->tau = (opt && opt->piv_tol > 0) ? opt->piv_tol : apm::kDefaultPivTol;
    L->perturb = !(flags & APM_NO_PERTURB);
    L->out_f64 = out_f64;
    return APM_OK;
}

apm_status cs_args(const double* m_up, const double* m_dn, const apm_batch* bd, double* c, uint32_t mode,
                   apm::LaunchCS* L, bool* noop)
{
    *noop = false;
    if (bad_batch(bd, APM_MAX_N_CS)) return APM_EINVAL;
    if (mode & ~(APM_CS_ALL | APM_CS_WEIGHTS)) return APM_EINVAL;
    if ((mode & APM_CS_WEIGHTS) && m_dn) return APM_EINVAL;
    if (bd->n_uniform > APM_MAX_N_CS || bd->n_max > APM_MAX_N_CS) return APM_EUNSUPPORTED;
    if (bd->in_off != bd->out_off) return APM_EINVAL;   // one offset array indexes inputs and output
    if (bd->batch == 0) {
        *noop = true;
        return APM_OK;
    }
    if (!m_up || !c) return APM_EINVAL;
    if (c == m_up || c == m_dn) return APM_EINVAL;      // the output must not alias the inputs
    *L = apm::LaunchCS{};
    L->m_up = m_up;
    L->m_dn = m_dn;
    L->c = c;
    L->batch = bd->batch;
    L->n_uniform = bd->n_uniform;
    L->n = bd->n;
    L->n_max = bd->n_max > 0 ? bd->n_max : APM_MAX_N_CS;
    L->off = bd->out_off;
    L->mode = mode;
    return APM_OK;
}

apm_status perm_args(const double* A, const apm_batch* bd, double* perm, apm::LaunchPerm* L, bool* noop)
{
    *noop = false;
    if (bad_batch(bd, APM_MAX_N_PERM)) return APM_EINVAL;
    if (bd->n_uniform > APM_MAX_N_PERM || bd->n_max > APM_MAX_N_PERM) return APM_EUNSUPPORTED;
    if (bd->batch == 0) {
        *noop = true;
        return APM_OK;
    }
    if (!A || !perm) return APM_EINVAL;
    *L = apm::LaunchPerm{};
    L->A = A;
    L->out = perm;
    L->batch = bd->batch;
    L->n_uniform = bd->n_uniform;
    L->n = bd->n;
    L->n_max = bd->n_max > 0 ? bd->n_max : APM_MAX_N_PERM;
    L->in_off = bd->in_off;
    L->out_off = bd->out_off;
    return APM_OK;
}

// Packed default offsets of a ragged batch given without offset arrays: the queue
// preparation kernel writes the prefix sums of n_b^2 and 2^n_b into the workspace.
apm_status packed_offsets(const apm_batch* bd, hipStream_t st, const int64_t** ioff, const int64_t** ooff,
                          const int32_t** order = nullptr)
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
    if (order) *order = L.order;
    return APM_OK;
}

// ---- scratch of apm_all_minors_noalloc ------------------------------------------------------
// One static device array per GPU (loaded with the code object, held until the process ends):
// the deferred pivot-correction queue of a uniform batch, or the queue head, queue order and
// packed offsets of a mixed-order batch, of at most APM_NOALLOC_MAX_BATCH matrices.
constexpr int64_t kScratchBytes = 256 + 64 * (int64_t)APM_NOALLOC_MAX_BATCH + 4096;
constexpr int64_t kScrOrder = 256;                                             // int32 [max]
constexpr int64_t kScrIoff = kScrOrder + 4 * (int64_t)APM_NOALLOC_MAX_BATCH;    // int64 [max]
constexpr int64_t kScrOoff = kScrIoff + 8 * (int64_t)APM_NOALLOC_MAX_BATCH;     // int64 [max]
static_assert(kScrOoff + 8 * (int64_t)APM_NOALLOC_MAX_BATCH <= kScratchBytes, "mixed-order layout fits");

__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
void* g_scratch_ptr[kMaxDevices];   // device address of `scratch` per device, looked up once
int g_scratch_cus[kMaxDevices];

// The device address of this device's copy of `scratch` (its host-side name is only a
// stand-in) and the device's compute-unit count, looked up on the first call per device.
apm_status scratch_address(char** base, int* cus)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return from_hip(e);
    if (dev < 0 || dev >= kMaxDevices) return APM_EUNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_ws_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return from_hip(e);
        if (!p) return APM_EDEVICE;
        int v = 0;
        e = hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return from_hip(e);
        g_scratch_cus[dev] = v;
        g_scratch_ptr[dev] = p;
    }
    *base = static_cast<char*>(g_scratch_ptr[dev]);
    *cus = g_scratch_cus[dev];
    return APM_OK;
}

// Clears the deferred-correction queue's counters (matrices listed, completion counts of the
// correction launch); a listed matrix's slot is written in full (one work item per matrix)
// before it is read.  A kernel, not a memset, so that the call can be captured into a graph.
__global__ void scratch_head_clear_kernel(int32_t* q)
{
    if (threadIdx.x < apm::kTopCounterInts) q[threadIdx.x] = 0;
}

}  // namespace

// A plan: the launch descriptions of one operation (or of the CDet pipeline) bound to the
// caller's buffers and to a workspace of its own, recorded once into a graph.
struct apm_plan {
    apm_plan_kind kind = APM_PLAN_MINORS;
    bool noop = false;            // empty batch: launches enqueue nothing
    bool has_dn = false;          // CDET with a second matrix set
    bool prep = false;            // CS / PERM on a mixed-order batch without offsets
    int dev = 0;
    int k0 = 0;                   // pinned lane-subtree order (uniform minors), else 0
    apm::LaunchMinors Lm{}, Lm_dn{}, Lprep{};
    apm::LaunchCS Lc{};
    apm::LaunchPerm Lp{};
    void* ws = nullptr;           // counter | order | ioff | ooff | deferred-correction queue
    size_t ws_bytes = 0;
    bool dirty = false;           // an eager launch failed after the queue was used
    hipStream_t ps = nullptr;     // private stream the graph is recorded on
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
};

namespace {

size_t round256(size_t x) { return (x + 255) & ~(size_t)255; }

hipError_t plan_enqueue(const apm_plan* p, hipStream_t st)
{
    hipError_t e = hipSuccess;
    switch (p->kind) {
    case APM_PLAN_MINORS:
        return apm::fpm_launch(p->Lm, st);
    case APM_PLAN_CONNECTED_SUMS:
        if (p->prep) e = apm::fpm_prep_launch(p->Lprep, st);
        if (e == hipSuccess) e = apm::cs_launch(p->Lc, st);
        return e;
    case APM_PLAN_PERM_MINORS:
        if (p->prep) e = apm::fpm_prep_launch(p->Lprep, st);
        if (e == hipSuccess) e = apm::perm_launch(p->Lp, st);
        return e;
    case APM_PLAN_CDET:
        e = apm::fpm_launch(p->Lm, st);
        if (e == hipSuccess && p->has_dn) e = apm::fpm_launch(p->Lm_dn, st);
        if (e == hipSuccess) e = apm::cs_launch(p->Lc, st);
        return e;
    }
    return hipErrorInvalidValue;
}

// Checks of a plan description; fills the launch descriptions (without workspace).
apm_status plan_args(const apm_plan_desc* d, apm_plan* p)
{
    const apm_batch* bd = &d->batch;
    p->kind = d->kind;
    if (d->flags & ~(APM_PLAN_AUTOTUNE | APM_PLAN_EAGER)) return APM_EINVAL;
    bool noop = false, noop2 = false;
    apm_status s = APM_OK;
    switch (d->kind) {
    case APM_PLAN_MINORS:
        if (d->A_dn || d->minors_dn || d->info_dn || d->m_up || d->m_dn || d->c || d->perm || d->cs_mode)
            return APM_EINVAL;
        s = minors_args(d->dtype, d->A, bd, d->minors, d->exp, d->info, &d->opts, &p->Lm, &noop);
        break;
    case APM_PLAN_CONNECTED_SUMS:
        if (d->A || d->A_dn || d->minors || d->minors_dn || d->exp || d->info || d->info_dn || d->perm)
            return APM_EINVAL;
        s = cs_args(d->m_up, d->m_dn, bd, d->c, d->cs_mode, &p->Lc, &noop);
        break;
    case APM_PLAN_PERM_MINORS:
        if (d->A_dn || d->minors || d->minors_dn || d->exp || d->info || d->info_dn || d->m_up || d->m_dn ||
            d->c || d->cs_mode)
            return APM_EINVAL;
        s = perm_args(static_cast<const double*>(d->A), bd, d->perm, &p->Lp, &noop);
        break;
    case APM_PLAN_CDET: {
        if (d->exp || d->m_up || d->m_dn || d->perm) return APM_EINVAL;
        const bool f64 = (d->opts.flags & APM_OUT_F64) != 0;
        if (!(d->dtype == APM_R64 || (d->dtype == APM_R32S && f64))) return APM_EINVAL;
        if (d->cs_mode & ~APM_CS_ALL) return APM_EINVAL;
        if ((d->A_dn == nullptr) != (d->minors_dn == nullptr)) return APM_EINVAL;
        if (!d->A_dn && d->info_dn) return APM_EINVAL;
        if (d->minors && (d->minors == d->minors_dn || d->minors == (void*)d->c || d->minors_dn == (void*)d->c))
            return APM_EINVAL;
        s = minors_args(d->dtype, d->A, bd, d->minors, nullptr, d->info, &d->opts, &p->Lm, &noop);
        if (s == APM_OK && d->A_dn)
            s = minors_args(d->dtype, d->A_dn, bd, d->minors_dn, nullptr, d->info_dn, &d->opts, &p->Lm_dn, &noop2);
        apm_batch cb = *bd;
        cb.in_off = bd->out_off;
        if (s == APM_OK)
            s = cs_args(static_cast<const double*>(d->minors), static_cast<const double*>(d->minors_dn), &cb, d->c,
                        d->cs_mode, &p->Lc, &noop2);
        p->has_dn = d->A_dn != nullptr;
        break;
    }
    default:
        return APM_EINVAL;
    }
    if (s != APM_OK) return s;
    p->noop = noop;
    return APM_OK;
}

// Allocates and zeroes the plan's workspace and points the launch descriptions at it.
apm_status plan_workspace(const apm_plan_desc* d, apm_plan* p)
{
    const apm_batch* bd = &d->batch;
    const int64_t B = bd->batch;
    const bool ragged = bd->n_uniform == 0;
    const bool minors = d->kind == APM_PLAN_MINORS || d->kind == APM_PLAN_CDET;
    p->prep = ragged && (d->kind == APM_PLAN_CONNECTED_SUMS ||
                         (d->kind == APM_PLAN_PERM_MINORS && (!bd->in_off || !bd->out_off)));
    const bool need_ragged = ragged && (minors || p->prep);
    const bool need_topq = !ragged && minors && B <= INT32_MAX / 2;
    const size_t o_order = 256, o_ioff = o_order + round256((size_t)B * 4), o_ooff = o_ioff + round256((size_t)B * 8),
                 o_topq = need_ragged ? o_ooff + round256((size_t)B * 8) : 0;
    p->ws_bytes = need_topq ? o_topq + (size_t)apm::fpm_topq_bytes(B) : o_topq;
    if (p->ws_bytes == 0) return APM_OK;
    hipError_t e = hipMalloc(&p->ws, p->ws_bytes);
    if (e != hipSuccess) {
        p->ws = nullptr;
        return from_hip(e);
    }
    e = hipMemsetAsync(p->ws, 0, p->ws_bytes, p->ps);
    if (e == hipSuccess) e = hipStreamSynchronize(p->ps);
    if (e != hipSuccess) return from_hip(e);
    char* w = static_cast<char*>(p->ws);
    int cus = 0;
    if (need_ragged) {
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->dev);
        if (e != hipSuccess) return from_hip(e);
    }
    auto bind = [&](apm::LaunchMinors& L) {
        if (need_ragged) {
            L.counter = reinterpret_cast<int32_t*>(w);
            L.order = reinterpret_cast<int32_t*>(w + o_order);
            L.ioff_ws = reinterpret_cast<int64_t*>(w + o_ioff);
            L.ooff_ws = reinterpret_cast<int64_t*>(w + o_ooff);
            L.n_workers = cus;
        }
        if (need_topq) {
            L.topq = reinterpret_cast<int32_t*>(w + o_topq);
            L.topq_cap = (int32_t)B;
        }
    };
    if (minors) {
        bind(p->Lm);
        if (p->has_dn) bind(p->Lm_dn);
        if (d->kind == APM_PLAN_CDET && ragged && !bd->out_off) p->Lc.off = p->Lm.ooff_ws;
        if (d->kind == APM_PLAN_CDET && ragged) p->Lc.order = p->Lm.order;
    }
    if (p->prep) {
        p->Lprep.batch = bd->batch;
        p->Lprep.n = bd->n;
        bind(p->Lprep);
        if (d->kind == APM_PLAN_CONNECTED_SUMS) {
            if (!bd->out_off) p->Lc.off = p->Lprep.ooff_ws;
            p->Lc.order = p->Lprep.order;
        } else {
            if (!p->Lp.in_off) p->Lp.in_off = p->Lprep.ioff_ws;
            if (!p->Lp.out_off) p->Lp.out_off = p->Lprep.ooff_ws;
        }
    }
    return APM_OK;
}

void plan_free(apm_plan* p)
{
    if (!p) return;
    if (p->ge) (void)hipGraphExecDestroy(p->ge);
    if (p->g) (void)hipGraphDestroy(p->g);
    if (p->ps) {
        (void)hipStreamSynchronize(p->ps);
        (void)hipStreamDestroy(p->ps);
    }
    if (p->ws) (void)hipFree(p->ws);
    delete p;
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

apm_status apm_last_device_error(void)
{
    const int e = g_unreported_hip_error;
    g_unreported_hip_error = 0;
    if (e == 0) return APM_OK;
    return e == (int)hipErrorOutOfMemory ? APM_ENOMEM : APM_EDEVICE;
}

int apm_version(void) { return 100; }

apm_status apm_all_minors(apm_dtype dt, const void* A, const apm_batch* bd, void* minors, int16_t* exp,
                          int32_t* info, const apm_opts* opt, apm_stream stream)
{
    apm::LaunchMinors L{};
    bool noop = false;
    apm_status s = minors_args(dt, A, bd, minors, exp, info, opt, &L, &noop);
    if (s != APM_OK || noop) return s;
    TopQueue* tq = nullptr;
    if (bd->n_uniform == 0) {
        s = get_workspace(bd->batch, &L.counter, &L.order, &L.ioff_ws, &L.ooff_ws, &L.n_workers);
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

apm_status apm_all_minors_noalloc(apm_dtype dt, const void* A, const apm_batch* bd, void* minors, int16_t* exp,
                                  int32_t* info, const apm_opts* opt, apm_stream stream)
{
    apm::LaunchMinors L{};
    bool noop = false;
    apm_status s = minors_args(dt, A, bd, minors, exp, info, opt, &L, &noop);
    if (s != APM_OK || noop) return s;
    if (bd->batch > APM_NOALLOC_MAX_BATCH) return APM_EUNSUPPORTED;
    char* base = nullptr;
    int cus = 0;
    s = scratch_address(&base, &cus);
    if (s != APM_OK) return s;
    const hipStream_t st = (hipStream_t)stream;
    if (bd->n_uniform == 0) {
        // the queue-preparation kernel of the launch resets the queue head itself
        L.counter = reinterpret_cast<int32_t*>(base);
        L.order = reinterpret_cast<int32_t*>(base + kScrOrder);
        L.ioff_ws = reinterpret_cast<int64_t*>(base + kScrIoff);
        L.ooff_ws = reinterpret_cast<int64_t*>(base + kScrOoff);
        L.n_workers = cus;
    } else {
        if (apm::fpm_topq_bytes_unsplit(bd->batch) > kScratchBytes) return APM_EUNSUPPORTED;
        L.topq = reinterpret_cast<int32_t*>(base);
        L.topq_cap = bd->batch;
        L.no_split = true;   // one work item per matrix: no per-item info codes to hold
        hipLaunchKernelGGL(scratch_head_clear_kernel, dim3(1), dim3(64), 0, st, L.topq);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return from_hip(e);
    }
    return from_hip(apm::fpm_launch(L, st));
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
            L.tau = apm::kDefaultPivTol;
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
    tune_cache_record((int)dt, n, best);
    if (k0_out) *k0_out = best;
    return APM_OK;
}

void apm_minors_k0_mixed(apm_dtype dt, int32_t* k0_small, int32_t* k0_large)
{
    int32_t* out[2] = {k0_small, k0_large};
    for (int w = 0; w < 2; ++w) {
        if (!out[w]) continue;
        if ((int)dt < 0 || (int)dt > 3) {
            *out[w] = -1;
            continue;
        }
        int lo, hi, def;
        apm::mixed_k0_range((int)dt, w, &lo, &hi, &def);
        const int t = apm::tuned_mixed_k0((int)dt, w);
        const int k = t > 0 ? t : def;
        *out[w] = k < lo ? lo : (k > hi ? hi : k);
    }
}

apm_status apm_autotune_minors_mixed(apm_dtype dt, int32_t batch, int32_t* k0_small, int32_t* k0_large,
                                     apm_stream stream)
{
    if ((int)dt < 0 || (int)dt > 3 || batch < 1) return APM_EINVAL;
    const hipStream_t st = (hipStream_t)stream;
    const bool cplx = (dt == APM_C128 || dt == APM_C64S), scaled = (dt == APM_R32S || dt == APM_C64S);
    // synthetic batch: orders 10..16 in turn (the large-order kernel takes 14..16)
    std::vector<int32_t> nh((size_t)batch);
    std::vector<int64_t> ih((size_t)batch), oh((size_t)batch);
    int64_t in_e = 0, out_e = 0;
    for (int32_t b = 0; b < batch; ++b) {
        const int n = 10 + b % 7;
        nh[b] = n;
        ih[b] = in_e;
        oh[b] = out_e;
        in_e += (int64_t)n * n;
        out_e += int64_t(1) << n;
    }
    const size_t in_b = (size_t)in_e * (cplx ? 16 : 8);
    const size_t out_b = (size_t)out_e * (scaled ? (cplx ? 8 : 4) : (cplx ? 16 : 8));
    const size_t ex_b = scaled ? (size_t)out_e * 2 : 0;
    void *A = nullptr, *out = nullptr, *ex = nullptr, *nv = nullptr, *io = nullptr, *oo = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int best[2], lo[2], hi[2];
    for (int w = 0; w < 2; ++w) {
        apm::mixed_k0_range((int)dt, w, &lo[w], &hi[w], &best[w]);
        const int t = apm::tuned_mixed_k0((int)dt, w);
        if (t > 0) best[w] = t;
    }
    int32_t *counter = nullptr, *order = nullptr;
    int64_t *ioff_ws = nullptr, *ooff_ws = nullptr;
    int cus = 0;
    apm_status s = get_workspace(batch, &counter, &order, &ioff_ws, &ooff_ws, &cus);
    if (s != APM_OK) return s;
    hipError_t e = hipMalloc(&A, in_b);
    if (e == hipSuccess) e = hipMalloc(&out, out_b);
    if (e == hipSuccess && ex_b) e = hipMalloc(&ex, ex_b);
    if (e == hipSuccess) e = hipMalloc(&nv, (size_t)batch * 4);
    if (e == hipSuccess) e = hipMalloc(&io, (size_t)batch * 8);
    if (e == hipSuccess) e = hipMalloc(&oo, (size_t)batch * 8);
    if (e == hipSuccess) e = hipMemcpyAsync(nv, nh.data(), (size_t)batch * 4, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(io, ih.data(), (size_t)batch * 8, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(oo, oh.data(), (size_t)batch * 8, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess)
        e = apm::fill_tune_input_mixed(A, (int)dt, static_cast<const int32_t*>(nv), static_cast<const int64_t*>(io),
                                       batch, st);
    // each kernel's choices timed with the other kernel at its current choice (the two
    // kernels take disjoint orders; their times add)
    for (int w = 0; w < 2 && e == hipSuccess; ++w) {
        float best_ms = 3.4e38f;
        const int keep = best[w];
        for (int k = lo[w]; k <= hi[w] && e == hipSuccess; ++k) {
            apm::LaunchMinors L{};
            L.dtype = (int)dt;
            L.A = A;
            L.out = out;
            L.ex = static_cast<int16_t*>(ex);
            L.batch = batch;
            L.n_uniform = 0;
            L.n = static_cast<const int32_t*>(nv);
            L.n_max = 16;
            L.in_off = static_cast<const int64_t*>(io);
            L.out_off = static_cast<const int64_t*>(oo);
            L.tau = apm::kDefaultPivTol;
            L.perturb = true;
            L.order = order;
            L.counter = counter;
            L.ioff_ws = ioff_ws;
            L.ooff_ws = ooff_ws;
            L.n_workers = cus;
            L.force_k0 = w == 0 ? k : best[0];
            L.force_k0_big = w == 1 ? k : best[1];
            e = apm::fpm_launch(L, st);                       // warm-up
            if (e == hipSuccess) e = hipEventRecord(e0, st);
            for (int r = 0; r < 3 && e == hipSuccess; ++r) e = apm::fpm_launch(L, st);
            if (e == hipSuccess) e = hipEventRecord(e1, st);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e == hipSuccess && ms < best_ms) {
                best_ms = ms;
                best[w] = k;
            }
        }
        if (e != hipSuccess) best[w] = keep;
    }
    const hipError_t es = hipStreamSynchronize(st);   // before the host arrays and buffers go
    if (e == hipSuccess) e = es;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    for (void* q : {ex, out, A, nv, io, oo})
        if (q) (void)hipFree(q);
    if (e != hipSuccess) return from_hip(e);
    for (int w = 0; w < 2; ++w) apm::set_tuned_mixed_k0((int)dt, w, best[w]);
    const std::pair<std::string, int> rec[2] = {{kMixedKey[0], best[0]}, {kMixedKey[1], best[1]}};
    tune_cache_record_keys((int)dt, rec, 2);
    if (k0_small) *k0_small = best[0];
    if (k0_large) *k0_large = best[1];
    return APM_OK;
}

int32_t apm_tune_cache_load(const char* path)
{
    return tune_cache_install(path ? std::string(path) : tune_cache_path());
}

apm_status apm_connected_sums(const double* m_up, const double* m_dn, const apm_batch* bd, double* c,
                              uint32_t mode, apm_stream stream)
{
    apm::LaunchCS L{};
    bool noop = false;
    apm_status s = cs_args(m_up, m_dn, bd, c, mode, &L, &noop);
    if (s != APM_OK || noop) return s;
    if (bd->n_uniform == 0) {
        // the queue preparation sorts the matrices by order (and packs default offsets)
        const int64_t *ioff = nullptr, *ooff = nullptr;
        s = packed_offsets(bd, (hipStream_t)stream, &ioff, &ooff, &L.order);
        if (s != APM_OK) return s;
        if (!L.off) L.off = ooff;
    }
    return from_hip(apm::cs_launch(L, (hipStream_t)stream));
}

apm_status apm_all_perm_minors(const double* A, const apm_batch* bd, double* perm, apm_stream stream)
{
    apm::LaunchPerm L{};
    bool noop = false;
    apm_status s = perm_args(A, bd, perm, &L, &noop);
    if (s != APM_OK || noop) return s;
    if (bd->n_uniform == 0 && (!L.in_off || !L.out_off)) {
        const int64_t *ioff = nullptr, *ooff = nullptr;
        s = packed_offsets(bd, (hipStream_t)stream, &ioff, &ooff);
        if (s != APM_OK) return s;
        if (!L.in_off) L.in_off = ioff;
        if (!L.out_off) L.out_off = ooff;
    }
    return from_hip(apm::perm_launch(L, (hipStream_t)stream));
}

namespace {

apm_status block_minors(int mode, apm_dtype dt, const void* A, const apm_batch* bd, void* out, int32_t* info,
                        apm_stream stream)
{
    if ((int)dt < 0 || (int)dt > 3) return APM_EINVAL;
    if (bad_batch(bd, APM_MAX_N_XOR)) return APM_EINVAL;
    if (dt != APM_R64 && dt != APM_C128) return APM_EUNSUPPORTED;
    if (bd->n_uniform == 0 || bd->in_off || bd->out_off) return APM_EUNSUPPORTED;
    if (bd->n_uniform > (mode == 2 ? APM_MAX_N_NAND : APM_MAX_N_XOR)) return APM_EUNSUPPORTED;
    if (bd->batch == 0) return APM_OK;
    if (!A || !out) return APM_EINVAL;
    apm::LaunchXor L{};
    L.dtype = (int)dt;
    L.A = A;
    L.out = out;
    L.info = info;
    L.batch = bd->batch;
    L.n = bd->n_uniform;
    L.mode = mode;
    L.ws_stride = apm::xor_ws_elems(L.n, mode);
    if (L.ws_stride > 0) {
        const size_t bytes = (size_t)L.ws_stride * (size_t)bd->batch * (dt == APM_C128 ? 16 : 8);
        apm_status s = get_xor_ws((hipStream_t)stream, bytes, &L.ws);
        if (s != APM_OK) return s;
    }
    return from_hip(apm::xor_launch(L, (hipStream_t)stream));
}

}  // namespace

apm_status apm_xor_minors(apm_dtype dt, const void* A, const apm_batch* bd, void* out, int32_t* info,
                          apm_stream stream)
{
    return block_minors(0, dt, A, bd, out, info, stream);
}

apm_status apm_xnor_minors(apm_dtype dt, const void* A, const apm_batch* bd, void* out, int32_t* info,
                           apm_stream stream)
{
    return block_minors(1, dt, A, bd, out, info, stream);
}

apm_status apm_nand_minors(apm_dtype dt, const void* A, const apm_batch* bd, void* out, int32_t* info,
                           apm_stream stream)
{
    return block_minors(2, dt, A, bd, out, info, stream);
}

apm_status apm_leading_minors(apm_dtype dt, const void* A, const apm_batch* bd, void* out, int32_t* info,
                              apm_stream stream)
{
    if ((int)dt < 0 || (int)dt > 3) return APM_EINVAL;
    if (bad_batch(bd, APM_MAX_N_LEAD)) return APM_EINVAL;
    if (dt != APM_R64 && dt != APM_C128) return APM_EUNSUPPORTED;
    if (bd->n_uniform == 0 || bd->in_off || bd->out_off) return APM_EUNSUPPORTED;
    if (bd->n_uniform > APM_MAX_N_LEAD) return APM_EUNSUPPORTED;
    if (bd->batch == 0) return APM_OK;
    if (!A || !out) return APM_EINVAL;
    return from_hip(apm::lead_launch((int)dt, A, out, info, bd->batch, bd->n_uniform, (hipStream_t)stream));
}

apm_status apm_plan_create(const apm_plan_desc* d, apm_plan** out)
{
    if (!out) return APM_EINVAL;
    *out = nullptr;
    if (!d) return APM_EINVAL;
    apm_plan* p = new (std::nothrow) apm_plan();
    if (!p) return APM_ENOMEM;
    apm_status s = plan_args(d, p);
    hipError_t e = hipSuccess;
    if (s == APM_OK && !p->noop) {
        e = hipGetDevice(&p->dev);
        if (e != hipSuccess) s = from_hip(e);
    }
    if (s == APM_OK && !p->noop) {
        e = hipStreamCreateWithFlags(&p->ps, hipStreamNonBlocking);
        if (e != hipSuccess) {
            p->ps = nullptr;
            s = from_hip(e);
        }
    }
    if (s == APM_OK && !p->noop) s = plan_workspace(d, p);
    const bool uniform_minors = (d->kind == APM_PLAN_MINORS || d->kind == APM_PLAN_CDET) && d->batch.n_uniform > 0;
    if (s == APM_OK && !p->noop && uniform_minors) {
        const int n = d->batch.n_uniform;
        if ((d->flags & APM_PLAN_AUTOTUNE) && apm::tuned_k0((int)d->dtype, n) <= 0 && !getenv("APM_K0"))
            (void)tune_cache_install(tune_cache_path());
        if ((d->flags & APM_PLAN_AUTOTUNE) && apm::tuned_k0((int)d->dtype, n) <= 0 && !getenv("APM_K0")) {
            // the synthetic tuning batch: the plan's size, at most 8192 matrices and 2 GiB of output
            int32_t tb = d->batch.batch < 8192 ? d->batch.batch : 8192;
            while (tb > 256 && ((int64_t)tb << n) * 16 > ((int64_t)1 << 31)) tb /= 2;
            s = apm_autotune_minors(d->dtype, n, tb, nullptr, p->ps);
        }
        if (s == APM_OK) {
            p->k0 = apm_minors_k0(d->dtype, n);
            p->Lm.force_k0 = p->k0;
            p->Lm_dn.force_k0 = p->k0;
        }
    }
    const bool mixed_minors = (d->kind == APM_PLAN_MINORS || d->kind == APM_PLAN_CDET) && d->batch.n_uniform == 0;
    if (s == APM_OK && !p->noop && mixed_minors) {
        if ((d->flags & APM_PLAN_AUTOTUNE) &&
            (apm::tuned_mixed_k0((int)d->dtype, 0) <= 0 || apm::tuned_mixed_k0((int)d->dtype, 1) <= 0)) {
            (void)tune_cache_install(tune_cache_path());
            if (apm::tuned_mixed_k0((int)d->dtype, 0) <= 0 || apm::tuned_mixed_k0((int)d->dtype, 1) <= 0) {
                const int32_t tb = d->batch.batch < 8192 ? d->batch.batch : 8192;
                s = apm_autotune_minors_mixed(d->dtype, tb < 7 ? 7 : tb, nullptr, nullptr, p->ps);
            }
        }
        if (s == APM_OK) {
            int32_t ks = 0, kl = 0;
            apm_minors_k0_mixed(d->dtype, &ks, &kl);
            p->k0 = ks;
            p->Lm.force_k0 = p->Lm_dn.force_k0 = ks;
            p->Lm.force_k0_big = p->Lm_dn.force_k0_big = kl;
        }
    }
    if (s == APM_OK && !p->noop && !(d->flags & APM_PLAN_EAGER)) {
        e = hipStreamBeginCapture(p->ps, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            const hipError_t e_rec = plan_enqueue(p, p->ps);
            hipGraph_t g = nullptr;
            e = hipStreamEndCapture(p->ps, &g);
            p->g = g;
            if (e == hipSuccess) e = e_rec;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&p->ge, p->g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            p->ge = nullptr;
            s = from_hip(e);
        }
    }
    if (s != APM_OK) {
        plan_free(p);
        return s;
    }
    *out = p;
    return APM_OK;
}

apm_status apm_plan_launch(apm_plan* p, apm_stream stream)
{
    if (!p) return APM_EINVAL;
    if (p->noop) return APM_OK;
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return from_hip(e);
    if (dev != p->dev) return APM_EINVAL;
    const hipStream_t st = (hipStream_t)stream;
    if (p->ge) return from_hip(hipGraphLaunch(p->ge, st));
    if (p->dirty) {
        // a failed eager launch may have left deferred corrections queued: clear them
        // (outside capture only; an eager plan is not recorded while in this state)
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        e = hipStreamIsCapturing(st, &cs);
        if (e != hipSuccess) return from_hip(e);
        if (cs != hipStreamCaptureStatusNone) return APM_EINVAL;
        e = hipMemsetAsync(p->ws, 0, p->ws_bytes, st);
        if (e != hipSuccess) return from_hip(e);
        p->dirty = false;
    }
    e = plan_enqueue(p, st);
    if (e != hipSuccess) p->dirty = true;
    return from_hip(e);
}

int32_t apm_plan_k0(const apm_plan* p) { return p ? p->k0 : -1; }

int32_t apm_plan_graphed(const apm_plan* p) { return p ? (p->ge != nullptr ? 1 : 0) : -1; }

void apm_plan_destroy(apm_plan* p) { plan_free(p); }

}  // extern "C"
