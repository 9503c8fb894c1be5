"""Pins of the Monte Carlo / proposal-network oracle against facts fixed outside it:
numpy's Philox bit generator, torch's bfloat16 rounding and autograd, finite
differences, closed forms, and exact enumeration of a tiny configuration space."""
import numpy as np
import pytest
import torch

import workloads as wl
from oracle import mc, mlp, philox

TINY = wl.McModel(n=3, L=2, n_tau=4, n_bin=2, beta=4.0, mu=0.3, eps=0.1)


# ------------------------------------------------------------------ Philox4x64-10
@pytest.mark.parametrize("key,ctr", [((0, 0), (0, 0, 0, 0)), ((123456789, 987654321), (5, 6, 7, 8)),
                                     ((2**64 - 1, 2**63 + 5), (2**64 - 2, 2**64 - 1, 17, 2**40)),
                                     ((20210415, 0), (8191, 3, 1, 0))])
def test_philox_matches_numpy(key, ctr):
    # numpy's Philox advances its counter by one before each block of four outputs
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=np.array(ctr, dtype=np.uint64))
    ref = bg.random_raw(8)
    c = [int(v) for v in ctr]
    got = []
    for _ in range(2):
        for i in range(4):                      # 256-bit counter increment with carry
            c[i] = (c[i] + 1) % 2**64
            if c[i]:
                break
        got.extend(philox.philox4x64(np.array(c, dtype=np.uint64), np.array(key, dtype=np.uint64)).tolist())
    assert [int(v) for v in ref] == got


def test_philox_mulhilo_against_python_ints():
    rng = np.random.default_rng(1)
    a = rng.integers(0, 2**63, size=1000, dtype=np.uint64) * np.uint64(2) + np.uint64(1)
    b = rng.integers(0, 2**63, size=1000, dtype=np.uint64) * np.uint64(2)
    hi, lo = philox.mulhilo(a, b)
    for x, y, h, l in zip(a.tolist(), b.tolist(), hi.tolist(), lo.tolist()):
        assert (x * y) >> 64 == h and (x * y) & (2**64 - 1) == l


def test_draw_mappings():
    r = np.array([0, 2**63, 2**64 - 1], dtype=np.uint64)
    assert philox.below(r, 10).tolist() == [0, 5, 9]
    u = philox.uniform(r)
    assert u[0] == 2.0**-53 and u[1] == 0.5 + 2.0**-53 and u[2] == 1.0 - 2.0**-53
    d = philox.mc_draws(7, np.arange(20000), 3, 0)
    k = philox.below(d[:, 0], 10)
    assert set(np.unique(k).tolist()) == set(range(10))
    assert abs(np.bincount(k).min() - 2000) < 200


# ------------------------------------------------------------------ bfloat16 rounding
def test_bf16_matches_torch():
    rng = np.random.default_rng(2)
    x = np.concatenate([rng.standard_normal(20000).astype(np.float32),
                        (1.0 + np.arange(256, dtype=np.float32) * 2.0**-15),      # ties and near-ties
                        np.array([0.0, -0.0, 1e-30, 3.0e38, -5.5], dtype=np.float32)])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(mlp.bf16(x), ref)


def test_bf16_ties_to_even():
    assert mlp.bf16(1.0 + 2.0**-8) == 1.0
    assert mlp.bf16(1.0 + 3 * 2.0**-8) == 1.0 + 2.0**-6


# ------------------------------------------------------------------ network
def _net(d_in=27, d_out=40, B=7, seed=3):
    rng = np.random.default_rng(seed)
    p = wl.mlp_init(d_in, d_out, seed=seed, gain=1.5).astype(np.float64)
    W1, W2, W3, b1, b2, b3 = mlp.unpack(p, d_in, d_out)
    b1[:] = rng.standard_normal(b1.shape) * 0.1
    b2[:] = rng.standard_normal(b2.shape) * 0.1
    b3[:d_out] = rng.standard_normal(d_out) * 0.1
    dp, op = mlp.dims(d_in, d_out)
    x = np.zeros((B, dp))
    x[:, :d_in] = rng.random((B, d_in))
    dout = np.zeros((B, op))
    dout[:, :d_out] = rng.standard_normal((B, d_out))
    return p, x, dout


def test_mlp_gradient_central_differences():
    d_in, d_out = 27, 40
    p, x, dout = _net(d_in, d_out)
    out, cache = mlp.forward(p, x, d_in, d_out, rounding=False)
    g = mlp.backward(cache, dout)
    rng = np.random.default_rng(4)
    idx = np.concatenate([rng.integers(0, p.size, 60), np.arange(p.size - 50, p.size)])
    h = 1e-6
    for i in idx:
        pp = p.copy()
        pp[i] += h
        fp = np.sum(mlp.forward(pp, x, d_in, d_out, rounding=False)[0] * dout)
        pp[i] -= 2 * h
        fm = np.sum(mlp.forward(pp, x, d_in, d_out, rounding=False)[0] * dout)
        fd = (fp - fm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_mlp_matches_torch_autograd():
    d_in, d_out = 27, 40
    p, x, dout = _net(d_in, d_out)
    out, cache = mlp.forward(p, x, d_in, d_out, rounding=False)
    g = mlp.backward(cache, dout)
    pt = torch.tensor(p, dtype=torch.float64, requires_grad=True)
    dp, op = mlp.dims(d_in, d_out)
    H = mlp.HIDDEN
    o = 0
    parts = []
    for shp in [(H, dp), (H, H), (op, H), (H,), (H,), (op,)]:
        cnt = int(np.prod(shp))
        parts.append(pt[o:o + cnt].reshape(shp))
        o += cnt
    W1, W2, W3, b1, b2, b3 = parts
    xt = torch.tensor(x)
    h1 = torch.tanh(xt @ W1.T + b1)
    h2 = torch.tanh(h1 @ W2.T + b2)
    ot = h2 @ W3.T + b3
    (ot * torch.tensor(dout)).sum().backward()
    np.testing.assert_allclose(out, ot.detach().numpy(), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(g, pt.grad.numpy(), rtol=1e-10, atol=1e-12)


def test_mlp_rounding_points():
    # with rounding, the network equals the unrounded one evaluated on bf16 weights and
    # bf16 activations; check one layer by hand
    d_in, d_out = 5, 16
    p, x, _ = _net(d_in, d_out, B=3)
    out, cache = mlp.forward(p, x, d_in, d_out, rounding=True)
    W1 = mlp.unpack(p, d_in, d_out)[0]
    b1 = mlp.unpack(p, d_in, d_out)[3]
    np.testing.assert_array_equal(cache["h1"], np.tanh(mlp.bf16(x) @ mlp.bf16(W1).T + b1))
    assert np.all(mlp.bf16(cache["h2b"]) == cache["h2b"])


def test_adam_matches_torch_and_first_step_closed_form():
    rng = np.random.default_rng(5)
    p0 = rng.standard_normal(50)
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    pt = torch.tensor(p0, requires_grad=True)
    opt = torch.optim.Adam([pt], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    for t in range(1, 6):
        g = rng.standard_normal(50)
        if t == 1:
            p1, _, _ = mlp.adam(p, m, v, g, 1, lr=1e-2)
            np.testing.assert_allclose(p - p1, 1e-2 * g / (np.abs(g) + 1e-8), rtol=1e-12)
        p, m, v = mlp.adam(p, m, v, g, t, lr=1e-2)
        opt.zero_grad()
        pt.grad = torch.tensor(g)
        opt.step()
    np.testing.assert_allclose(p, pt.detach().numpy(), rtol=1e-12, atol=1e-14)


# ------------------------------------------------------------------ Monte Carlo pieces
def test_g0_table_closed_forms():
    m = wl.McModel(n=4, L=8, n_tau=16, n_bin=4, beta=2.0, mu=0.0)
    g0 = wl.mc_g0_table(m)
    # half filling: G0(0, 0^-) = density = 1/2; jump G0(0,0^+) - G0(0,0^-) = -1 as dtau -> 0
    assert abs(g0[m.n_tau - 1, 0] - 0.5) < 1e-14
    # antiperiodicity: G0(r, tau - beta) = -G0(r, tau) on the grid (d and d - n_tau)
    for d in range(1, m.n_tau):
        np.testing.assert_allclose(g0[d + m.n_tau - 1 - m.n_tau], -g0[d + m.n_tau - 1], atol=1e-14)


def test_matrices_and_features_by_hand():
    m = TINY
    g0 = wl.mc_g0_table(m)
    v = mc.pack([3, 0, 1], [2, 2, 0])            # sites (x,y): (1,1), (0,0), (1,0)
    M = mc.matrices(m, g0, v[None])[0]
    # M_01: dx = 1, dy = 1, dtau = 0 (equal times: 0^-) ; M_20: dx = 0, dy = 1, d = -2
    assert M[0, 1] == g0[m.n_tau - 1, 1 * 2 + 1]
    assert M[2, 0] == g0[-2 + m.n_tau - 1, 1 * 2 + 0]
    assert np.all(np.diag(M) == g0[m.n_tau - 1, 0])
    ctx = mc.context(m, v[None], np.array([1]))
    assert ctx.tolist() == [[int(mc.pack(1, 0)), int(mc.pack(3, 2))]]
    f = mc.features(m, ctx)
    assert f.shape == (1, 16)
    np.testing.assert_array_equal(f[0, :6], [0.5, 0.0, 0.125, 0.5, 0.5, 0.625])
    assert np.all(f[0, 6:] == 0)


def test_two_vertex_connected_sum_closed_form():
    m = wl.McModel(n=2, L=4, n_tau=8, n_bin=2, beta=3.0, mu=0.2)
    g0 = wl.mc_g0_table(m)
    st = wl.mc_initial_states(64, m, seed=9)
    M = mc.matrices(m, g0, st)
    det = M[:, 0, 0] * M[:, 1, 1] - M[:, 0, 1] * M[:, 1, 0]
    # c[{0,1}] = a[{0,1}] - a[{0}] a[{1}] with a = det^2
    np.testing.assert_allclose(mc.full_connected_sum(m, g0, st), det**2 - (M[:, 0, 0] * M[:, 1, 1]) ** 2,
                               rtol=1e-12, atol=1e-15)


def test_proposal_distribution_normalised_and_sampled():
    m = wl.McModel(n=3, L=4, n_tau=8, n_bin=4, eps=0.2)
    rng = np.random.default_rng(6)
    logits = np.zeros((1, 16 + 4))
    logits[0] = rng.standard_normal(20) * 2
    sites, ts = np.meshgrid(np.arange(16), np.arange(8), indexing="ij")
    lq = mc.log_q(m, np.repeat(logits, sites.size, axis=0), sites.ravel(), ts.ravel())
    assert abs(np.exp(lq).sum() - 1.0) < 1e-12
    # the sampler draws from exactly this distribution
    W = 200000
    states = np.zeros((W, 3), dtype=np.uint32)
    d0, d1 = mc.draws(11, W, 0)
    prop, _ = mc.propose(m, states, np.zeros(W, dtype=np.int64), d0, d1, np.repeat(logits, W, axis=0))
    s, t = mc.unpack(prop)
    h = np.bincount(s * 8 + t, minlength=128)
    e = np.exp(lq) * W
    chi2 = ((h - e) ** 2 / e).sum()
    assert chi2 < 127 + 6 * np.sqrt(2 * 127)


def test_categorical_first_crossing():
    p = np.array([[0.0, 1.0, 0.0, 2.0, 1.0]])
    assert mc.categorical(p, np.array([0.0]))[0] == 1
    assert mc.categorical(p, np.array([0.2499]))[0] == 1
    assert mc.categorical(p, np.array([0.25]))[0] == 3
    assert mc.categorical(p, np.array([0.7499]))[0] == 3
    assert mc.categorical(p, np.array([0.75]))[0] == 4
    assert mc.categorical(p, np.array([1.0]))[0] == 4


def _detailed_balance_residual(model, params, accept_prob=mc.accept_probability):
    g0 = wl.mc_g0_table(model)
    S = mc.enumerate_states(model)
    c = mc.full_connected_sum(model, g0, S)
    lw = mc.log_abs(c)
    pi = np.abs(c) / np.abs(c).sum()
    V = model.L * model.L * model.n_tau
    L2 = model.L * model.L
    site, t = mc.unpack(S)
    vidx = site + L2 * t
    index = (vidx * (V ** np.arange(model.n))).sum(1)
    assert np.all(index == np.arange(S.shape[0]))
    cand_s, cand_t = np.arange(V) % L2, np.arange(V) // L2
    worst = 0.0
    for k in range(model.n):
        kk = np.full(S.shape[0], k)
        ctx = mc.context(model, S, kk)
        if params is None:
            lq_all = np.full((S.shape[0], V), -np.log(V))
        else:
            logits, _ = mlp.forward(params, mc.features(model, ctx), model.d_in, model.d_out)
            lq_all = np.stack([mc.log_q(model, logits, np.full(S.shape[0], cs), np.full(S.shape[0], ct))
                               for cs, ct in zip(cand_s, cand_t)], axis=1)
        for vp in range(V):
            X2 = index + (vp - vidx[:, k]) * V**k
            same = X2 == index
            lq_ratio = lq_all[np.arange(S.shape[0]), vidx[:, k]] - lq_all[:, vp]
            fwd = np.array([accept_prob(a, b, q) for a, b, q in zip(lw, lw[X2], lq_ratio)])
            flow = pi * np.exp(lq_all[:, vp]) * fwd
            rev = np.array([accept_prob(a, b, -q) for a, b, q in zip(lw[X2], lw, lq_ratio)])
            flow_back = pi[X2] * np.exp(lq_all[np.arange(S.shape[0]), vidx[:, k]]) * rev
            r = np.abs(flow - flow_back)[~same] / np.maximum(flow, flow_back)[~same].clip(1e-300)
            worst = max(worst, float(r.max(initial=0.0)))
    return worst


def test_detailed_balance_uniform_and_learned():
    assert _detailed_balance_residual(TINY, None) <= 1e-12
    params = wl.mlp_init(TINY.d_in, TINY.d_out, seed=4, gain=4.0)
    assert _detailed_balance_residual(TINY, params) <= 1e-12


def test_detailed_balance_catches_a_wrong_proposal_ratio():
    # a planted mistake in the acceptance (proposal ratio dropped) must break the pin
    params = wl.mlp_init(TINY.d_in, TINY.d_out, seed=4, gain=4.0)
    wrong = lambda lw, lc, lq: mc.accept_probability(lw, lc, 0.0)   # noqa: E731
    assert _detailed_balance_residual(TINY, params, wrong) > 1e-3


def _chi2_states(model, states, pi):
    from scipy.stats import chi2 as C
    V = model.L * model.L * model.n_tau
    site, t = mc.unpack(states)
    idx = ((site + model.L * model.L * t) * (V ** np.arange(model.n))).sum(1)
    h = np.bincount(idx, minlength=V ** model.n)
    e = pi * states.shape[0]
    gh, ge, ch, ce = [], [], 0, 0.0
    for i in np.argsort(e):
        ch += h[i]
        ce += e[i]
        if ce >= 10:
            gh.append(ch)
            ge.append(ce)
            ch, ce = 0, 0.0
    gh[-1] += ch
    ge[-1] += ce
    gh, ge = np.array(gh), np.array(ge)
    x = ((gh - ge) ** 2 / ge).sum()
    return C.sf(x, len(ge) - 1)


@pytest.mark.parametrize("learned", [False, True])
def test_oracle_sampler_reaches_pi(learned):
    model = TINY
    g0 = wl.mc_g0_table(model)
    S = mc.enumerate_states(model)
    c = mc.full_connected_sum(model, g0, S)
    pi = np.abs(c) / np.abs(c).sum()
    params = wl.mlp_init(model.d_in, model.d_out, seed=4, gain=2.0) if learned else None
    W = 4096
    st = wl.mc_initial_states(W, model, seed=12)
    cc = mc.full_connected_sum(model, g0, st)
    lw, sg = mc.log_abs(cc), np.sign(cc)
    for s in range(200 if learned else 80):
        r = mc.step(model, g0, st, lw, sg, 77, s, params=params)
        st, lw, sg = r["states"], r["logw"], r["sign"]
    assert _chi2_states(model, st, pi) > 1e-4


def test_loss_gradient_finite_differences():
    m = wl.McModel(n=3, L=4, n_tau=8, n_bin=4)
    rng = np.random.default_rng(8)
    W = 64
    logits = rng.standard_normal((W, 32))
    prop = mc.pack(rng.integers(0, 16, W), rng.integers(0, 8, W))
    y = rng.standard_normal(W) * 5
    y[3] = -np.inf
    y[5] = -80.0
    loss, dout = mc.loss_grad(m, logits, prop, y)
    for r, f in [(0, int(prop[0] & 0xFFFF)), (3, 16 + int(prop[3] >> 16) // 2), (5, 7)]:
        lp = logits.copy()
        lp[r, f] += 1e-6
        lm = logits.copy()
        lm[r, f] -= 1e-6
        fd = (mc.loss_grad(m, lp, prop, y)[0] - mc.loss_grad(m, lm, prop, y)[0]) / 2e-6
        assert abs(fd - dout[r, f]) < 1e-7


def test_resolution_cutoff_two_vertices():
    # n = 2: d[V] = |a[V]| + |c[{0}]| |a[{1}]| = det^2 + (M00 M11)^2 and c[V] = det^2 - (M00 M11)^2
    m = wl.McModel(n=2, L=4, n_tau=8, n_bin=2, beta=3.0, mu=0.2, resolve=0.5)
    g0 = wl.mc_g0_table(m)
    st = wl.mc_initial_states(256, m, seed=10)
    M = mc.matrices(m, g0, st)
    det2 = (M[:, 0, 0] * M[:, 1, 1] - M[:, 0, 1] * M[:, 1, 0]) ** 2
    dd = (M[:, 0, 0] * M[:, 1, 1]) ** 2
    keep = np.abs(det2 - dd) >= 0.5 * (det2 + dd)
    lw, sg = mc.weight(m, g0, st)
    assert 0 < keep.sum() < 256
    np.testing.assert_array_equal(np.isfinite(lw), keep)
    np.testing.assert_allclose(lw[keep], np.log(np.abs(det2 - dd))[keep], rtol=1e-12)
    assert np.all(sg[~keep] == 0)
