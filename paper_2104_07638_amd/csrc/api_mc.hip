// api_mc.hip -- C ABI of the Monte Carlo step and the proposal network: validation,
// work-buffer layout and the launch sequence of one step.
#include <math.h>

#include "../../include/apm_mc.h"
#include "apm_kernels.h"

namespace {

constexpr double kClip = 30.0;      // regression targets clipped below at (max - 30)

apm_status from_hip(hipError_t e)
{
    if (e == hipSuccess) return APM_OK;
    if (e == hipErrorOutOfMemory) return APM_ENOMEM;
    return APM_EDEVICE;
}

int pad_in(int d) { return d <= 16 ? 16 : (d + 15) / 16 * 16; }
int pad_out(int d) { return (d + 15) / 16 * 16; }
bool bad_dims(int d_in, int d_out) { return d_in < 1 || d_in > APM_MLP_MAX_IN || d_out < 1 || d_out > APM_MLP_MAX_OUT; }
int64_t al(int64_t v) { return (v + 255) & ~(int64_t)255; }

bool bad_net(const apm_mlp* net)
{
    return !net || bad_dims(net->d_in, net->d_out) || !net->param || !net->w || !net->wt;
}

apm::MlpNet net_of(const apm_mlp* net)
{
    return apm::MlpNet{pad_in(net->d_in), pad_out(net->d_out), net->param, net->grad, net->adam_m, net->adam_v,
                       net->w, net->wt};
}

apm_status check_model(const apm_mc_model* m, bool need_table = true)
{
    if (!m || (need_table && !m->g0)) return APM_EINVAL;
    if (m->n < 2) return APM_EINVAL;
    if (m->n > APM_MC_MAX_N) return APM_EUNSUPPORTED;
    if (m->L < 1 || m->L > 256 || m->n_tau < 1 || m->n_tau > 32768) return APM_EINVAL;
    if (m->n_bin < 1 || m->n_bin > 64 || m->n_tau % m->n_bin != 0) return APM_EINVAL;
    if (!(m->eps >= 0.0 && m->eps <= 1.0)) return APM_EINVAL;
    if (!(m->resolve >= 0.0) || !isfinite(m->resolve)) return APM_EINVAL;
    return APM_OK;
}

apm_status check_chain(const apm_mc_chain* ch)
{
    if (!ch || ch->walkers < 0) return APM_EINVAL;
    if (ch->walkers > 0 && (!ch->state || !ch->logw || !ch->sign)) return APM_EINVAL;
    return APM_OK;
}

apm_status check_net_for(const apm_mc_model* m, const apm_mc_chain* ch, const apm_mlp* net)
{
    if (bad_net(net)) return APM_EINVAL;
    if (net->d_in != 3 * (m->n - 1) || net->d_out != m->L * m->L + m->n_bin) return APM_EINVAL;
    if (ch->walkers % 32 != 0) return APM_EINVAL;
    return APM_OK;
}

struct McWork {
    double* mats;
    double* minors;
    double* csum;
    int32_t* info;
    int32_t* moved;
    uint32_t* prop;
    double* logq;
    double* logc;
    double* summ;      // (c[V], d[V]) per walker, orders <= 12
    uint64_t* draws;   // the step's Philox draws: calls 0 and 1 of every walker, 4 x uint64 each
    uint16_t* feat;
    float* logits;
    float* dout;
    float* gbuf;
    void* mlp;
};

// Layout of the step's work buffer; returns its size.  base == NULL only sizes it.
int64_t mc_layout(const apm_mc_model* m, int64_t W, bool with_net, char* base, McWork* wk)
{
    const int64_t nn = (int64_t)m->n * m->n, nm = (int64_t)1 << m->n;
    const int dp = pad_in(3 * (m->n - 1)), op = pad_out(m->L * m->L + m->n_bin);
    int64_t off = 0;
    auto take = [&](int64_t bytes) {
        char* p = base ? base + off : nullptr;
        off += al(bytes);
        return p;
    };
    McWork w{};
    w.mats = reinterpret_cast<double*>(take(W * nn * 8));
    w.minors = reinterpret_cast<double*>(take(W * nm * 8));
    w.csum = reinterpret_cast<double*>(take(W * nm * 8));
    w.info = reinterpret_cast<int32_t*>(take(W * 4));
    w.moved = reinterpret_cast<int32_t*>(take(W * 4));
    w.prop = reinterpret_cast<uint32_t*>(take(W * 4));
    w.logq = reinterpret_cast<double*>(take(W * 8));
    w.logc = reinterpret_cast<double*>(take(W * 8));
    w.summ = reinterpret_cast<double*>(take(W * 16));
    w.draws = reinterpret_cast<uint64_t*>(take(W * 64));
    if (with_net) {
        w.feat = reinterpret_cast<uint16_t*>(take(W * dp * 2));
        w.logits = reinterpret_cast<float*>(take(W * op * 4));
        w.dout = reinterpret_cast<float*>(take(W * op * 4));
        w.gbuf = reinterpret_cast<float*>(take(W * 4));
        w.mlp = take(apm::mlp_work_bytes(dp, op, (int)W));
    }
    if (wk) *wk = w;
    return off;
}

apm::McArgs args_of(const apm_mc_model* m, const apm_mc_chain* ch, uint64_t seed, int32_t step)
{
    apm::McArgs a{};
    a.n = m->n;
    a.L = m->L;
    a.n_tau = m->n_tau;
    a.n_bin = m->n_bin;
    a.eps = m->eps;
    a.resolve = m->resolve;
    a.g0 = m->g0;
    a.W = ch->walkers;
    a.state = ch->state;
    a.logw = ch->logw;
    a.sign = ch->sign;
    a.seed = seed;
    a.step = step;
    return a;
}

double* summ_of(const apm::McArgs& a, const McWork& wk) { return a.n <= 12 ? wk.summ : nullptr; }

// c[V] of the configurations whose matrices are in wk.mats: minors, then the rooted recursion.
hipError_t weights(const apm::McArgs& a, const McWork& wk, hipStream_t st)
{
    apm::LaunchMinors L{};
    L.dtype = APM_R64;
    L.A = wk.mats;
    L.out = wk.minors;
    L.info = wk.info;
    L.batch = a.W;
    L.n_uniform = a.n;
    L.n_max = a.n;
    L.tau = apm::kDefaultPivTol;
    L.perturb = true;
    hipError_t e = apm::fpm_launch(L, st);
    if (e != hipSuccess) return e;
    apm::LaunchCS C{};
    C.m_up = wk.minors;
    C.c = wk.csum;
    C.batch = a.W;
    C.n_uniform = a.n;
    C.n_max = a.n;
    C.mode = APM_CS_ROOTED;
    // up to 12 vertices the rooted recursion fits one LDS block: the kernel then writes only
    // c[V] and its rounding scale d[V] per walker instead of the whole c[] array
    C.summ = summ_of(a, wk);
    return apm::cs_launch(C, st);
}

}  // namespace

extern "C" {

int64_t apm_mlp_param_count(int32_t d_in, int32_t d_out)
{
    return bad_dims(d_in, d_out) ? -1 : apm::mlp_param_count(pad_in(d_in), pad_out(d_out));
}

int64_t apm_mlp_weight_count(int32_t d_in, int32_t d_out)
{
    return bad_dims(d_in, d_out) ? -1 : apm::mlp_weight_count(pad_in(d_in), pad_out(d_out));
}

int64_t apm_mlp_work_bytes(int32_t d_in, int32_t d_out, int32_t batch)
{
    if (bad_dims(d_in, d_out) || batch < 0 || batch % 32) return -1;
    return apm::mlp_work_bytes(pad_in(d_in), pad_out(d_out), batch);
}

apm_status apm_mlp_sync(const apm_mlp* net, apm_stream stream)
{
    if (bad_net(net)) return APM_EINVAL;
    return from_hip(apm::mlp_adam_launch(net_of(net), false, 0.f, 0.f, 0.f, 0.f, 1, (hipStream_t)stream));
}

apm_status apm_mlp_forward(const apm_mlp* net, const uint16_t* x, int32_t batch, float* out, void* work,
                           apm_stream stream)
{
    if (bad_net(net) || batch < 0 || batch % 32) return APM_EINVAL;
    if (batch == 0) return APM_OK;
    if (!x || !out) return APM_EINVAL;
    const apm::MlpNet nt = net_of(net);
    apm::MlpWork wk{};
    if (work) wk = apm::mlp_work_carve(work, nt.dp, nt.op, batch);
    return from_hip(apm::mlp_forward_launch(nt, x, batch, out, work ? &wk : nullptr, (hipStream_t)stream));
}

apm_status apm_mlp_backward(const apm_mlp* net, const float* dout, int32_t batch, void* work, apm_stream stream)
{
    if (bad_net(net) || !net->grad || batch < 0 || batch % 32) return APM_EINVAL;
    if (batch == 0) return APM_OK;
    if (!dout || !work) return APM_EINVAL;
    const apm::MlpNet nt = net_of(net);
    const apm::MlpWork wk = apm::mlp_work_carve(work, nt.dp, nt.op, batch);
    return from_hip(apm::mlp_backward_launch(nt, dout, batch, wk, (hipStream_t)stream));
}

apm_status apm_mlp_adam(const apm_mlp* net, const apm_adam* h, apm_stream stream)
{
    if (bad_net(net) || !net->grad || !net->adam_m || !net->adam_v || !h) return APM_EINVAL;
    if (h->t < 1 || !(h->lr >= 0.f) || !(h->beta1 >= 0.f && h->beta1 < 1.f) || !(h->beta2 >= 0.f && h->beta2 < 1.f) ||
        !(h->eps > 0.f) || !isfinite(h->lr))
        return APM_EINVAL;
    return from_hip(apm::mlp_adam_launch(net_of(net), true, h->lr, h->beta1, h->beta2, h->eps, h->t,
                                         (hipStream_t)stream));
}

int64_t apm_mc_work_bytes(const apm_mc_model* m, int32_t walkers, int32_t with_net)
{
    if (check_model(m, false) != APM_OK || walkers < 0) return -1;
    if (with_net && walkers % 32) return -1;
    return mc_layout(m, walkers, with_net != 0, nullptr, nullptr);
}

apm_status apm_mc_evaluate(const apm_mc_model* m, const apm_mc_chain* ch, void* work, apm_stream stream)
{
    apm_status s = check_model(m);
    if (s != APM_OK) return s;
    if ((s = check_chain(ch)) != APM_OK) return s;
    if (ch->walkers == 0) return APM_OK;
    if (!work) return APM_EINVAL;
    McWork wk;
    mc_layout(m, ch->walkers, false, static_cast<char*>(work), &wk);
    const apm::McArgs a = args_of(m, ch, 0, 0);
    const hipStream_t st = (hipStream_t)stream;
    hipError_t e = apm::mc_gather_launch(a, wk.mats, st);
    if (e == hipSuccess) e = weights(a, wk, st);
    if (e == hipSuccess) e = apm::mc_set_launch(a, wk.csum, wk.minors, summ_of(a, wk), st);
    return from_hip(e);
}

apm_status apm_mc_context(const apm_mc_model* m, const apm_mc_chain* ch, uint64_t seed, int32_t step, int32_t* moved,
                          uint16_t* feat, apm_stream stream)
{
    apm_status s = check_model(m);
    if (s != APM_OK) return s;
    if ((s = check_chain(ch)) != APM_OK) return s;
    if (ch->walkers == 0) return APM_OK;
    if (!moved) return APM_EINVAL;
    const int dp = pad_in(3 * (m->n - 1));
    return from_hip(apm::mc_context_launch(args_of(m, ch, seed, step), moved, feat, dp, (hipStream_t)stream));
}

apm_status apm_mc_propose(const apm_mc_model* m, const apm_mc_chain* ch, uint64_t seed, int32_t step,
                          const int32_t* moved, const float* logits, int32_t logit_stride, uint32_t* proposed,
                          double* logq, double* mats, apm_stream stream)
{
    apm_status s = check_model(m);
    if (s != APM_OK) return s;
    if ((s = check_chain(ch)) != APM_OK) return s;
    if (logits && logit_stride < m->L * m->L + m->n_bin) return APM_EINVAL;
    if (ch->walkers == 0) return APM_OK;
    if (!moved || !proposed || !logq || !mats) return APM_EINVAL;
    return from_hip(apm::mc_propose_launch(args_of(m, ch, seed, step), moved, nullptr, logits, logit_stride, proposed,
                                           logq, mats, (hipStream_t)stream));
}

apm_status apm_mc_accept(const apm_mc_model* m, const apm_mc_chain* ch, uint64_t seed, int32_t step,
                         const int32_t* moved, const uint32_t* proposed, const double* logq, const double* mats,
                         const apm_mc_record* rec, void* work, apm_stream stream)
{
    apm_status s = check_model(m);
    if (s != APM_OK) return s;
    if ((s = check_chain(ch)) != APM_OK) return s;
    if (ch->walkers == 0) return APM_OK;
    if (!moved || !proposed || !logq || !mats || !work) return APM_EINVAL;
    McWork wk;
    mc_layout(m, ch->walkers, false, static_cast<char*>(work), &wk);
    wk.mats = const_cast<double*>(mats);
    const apm::McArgs a = args_of(m, ch, seed, step);
    const hipStream_t st = (hipStream_t)stream;
    hipError_t e = weights(a, wk, st);
    if (e == hipSuccess)
        e = apm::mc_accept_launch(a, moved, proposed, logq, wk.csum, wk.minors, summ_of(a, wk),
                                  rec ? rec->logc_prop : nullptr,
                                  rec ? rec->accepted : nullptr, rec ? rec->obs_logw : nullptr,
                                  rec ? rec->obs_sign : nullptr, st);
    return from_hip(e);
}

apm_status apm_mc_step(const apm_mc_model* m, const apm_mc_chain* ch, const apm_mlp* net, const apm_adam* train,
                       uint64_t seed, int32_t step, const apm_mc_record* rec, void* work, apm_stream stream)
{
    apm_status s = check_model(m);
    if (s != APM_OK) return s;
    if ((s = check_chain(ch)) != APM_OK) return s;
    if (net && (s = check_net_for(m, ch, net)) != APM_OK) return s;
    if (train && (!net || !net->grad || !net->adam_m || !net->adam_v || train->t < 1)) return APM_EINVAL;
    if (ch->walkers == 0) return APM_OK;
    if (!work) return APM_EINVAL;
    const int W = ch->walkers;
    McWork wk;
    mc_layout(m, W, net != nullptr, static_cast<char*>(work), &wk);
    int32_t* moved = rec && rec->moved ? rec->moved : wk.moved;
    uint32_t* prop = rec && rec->proposed ? rec->proposed : wk.prop;
    double* logq = rec && rec->logq ? rec->logq : wk.logq;
    double* logc = rec && rec->logc_prop ? rec->logc_prop : wk.logc;
    apm::McArgs a = args_of(m, ch, seed, step);
    const hipStream_t st = (hipStream_t)stream;
    const int dp = pad_in(3 * (m->n - 1)), op = pad_out(m->L * m->L + m->n_bin);

    // the first kernel that needs the step's draws (context with a network, else the
    // proposal) computes both per walker and stores them; the later kernels read them
    a.draws = wk.draws;
    a.draws_ready = 0;
    hipError_t e = hipSuccess;
    if (net) {
        e = apm::mc_context_launch(a, moved, wk.feat, dp, st);
        a.draws_ready = 1;
    }
    apm::MlpNet nt{};
    apm::MlpWork mw{};
    if (net) {
        nt = net_of(net);
        if (train) mw = apm::mlp_work_carve(wk.mlp, dp, op, W);
        if (e == hipSuccess) e = apm::mlp_forward_launch(nt, wk.feat, W, wk.logits, train ? &mw : nullptr, st);
    }
    // without a network the proposal kernel also draws the moved vertex
    if (e == hipSuccess)
        e = apm::mc_propose_launch(a, net ? moved : nullptr, net ? nullptr : moved, net ? wk.logits : nullptr, op, prop,
                                   logq, wk.mats, st);
    a.draws_ready = 1;
    if (e == hipSuccess) e = weights(a, wk, st);
    if (e == hipSuccess)
        e = apm::mc_accept_launch(a, moved, prop, logq, wk.csum, wk.minors, summ_of(a, wk), logc,
                                  rec ? rec->accepted : nullptr,
                                  rec ? rec->obs_logw : nullptr, rec ? rec->obs_sign : nullptr, st);
    if (train) {
        if (e == hipSuccess)
            e = apm::mc_loss_launch(a, wk.logits, op, prop, logc, wk.gbuf, wk.dout, rec ? rec->loss : nullptr, kClip,
                                    st);
        if (e == hipSuccess) e = apm::mlp_backward_launch(nt, wk.dout, W, mw, st);
        if (e == hipSuccess)
            e = apm::mlp_adam_launch(nt, true, train->lr, train->beta1, train->beta2, train->eps, train->t, st);
    }
    return from_hip(e);
}

}  // extern "C"
