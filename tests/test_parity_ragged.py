"""Mixed-order batches: one persistent launch over matrices of different orders
(apm_all_minors with per-matrix n[]), and the CDet pipeline on such a batch."""
import numpy as np
import pytest

from oracle import metrics
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def apm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2104_07638_amd as m
    return m


def pack(mats):
    ns = np.array([m.shape[0] for m in mats], dtype=np.int32)
    flat = np.concatenate([m.ravel() for m in mats])
    ooff = np.concatenate([[0], np.cumsum(np.left_shift(1, ns.astype(np.int64)))[:-1]]).astype(np.int64)
    return ns, flat, ooff, int(np.sum(np.left_shift(1, ns.astype(np.int64))))


def test_ragged_all_orders(apm, oracle_mod):
    import torch
    rng = np.random.default_rng(3)
    orders = [5, 1, 20, 9, 14, 2, 16, 11, 6, 18, 3, 12, 8, 17, 10, 13, 4, 7, 15, 19] * 2
    mats = [W.lattice_batch(1, k, W.Lattice(32, 1.0, -0.5, 5.0), seed=300 + i)[0] for i, k in enumerate(orders)]
    ns, flat, ooff, tot = pack(mats)
    out = torch.full((tot,), 3.0, dtype=torch.float64, device="cuda")
    n_t = torch.from_numpy(ns).cuda()
    A_t = torch.from_numpy(flat).cuda()
    _, _, info = apm.all_minors_ragged(A_t, n_t, 20, "r64", out=out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    info = info.cpu().numpy()
    assert np.all(info >= 0), info
    for k, M in enumerate(mats):
        n = M.shape[0]
        seg = got[ooff[k]:ooff[k] + (1 << n)]
        if n <= 14:
            ref = oracle_mod.minors(M)
            assert metrics.mixed_err(seg, ref, metrics.hadamard_bounds(M)).max() <= 1e-10, n
        else:
            masks = np.unique(np.concatenate([rng.integers(0, 1 << n, 800), [0, (1 << n) - 1]]))
            ref = oracle_mod.minors_at(M, masks)
            assert metrics.mixed_err(seg[masks], ref, metrics.hadamard_at(M, masks)).max() <= 1e-10, n


@pytest.mark.parametrize("orders", [[12], [15], [9, 16], [3, 14, 11], [16, 15, 14] * 3 + [10],
                                    [2, 5, 8, 11, 14] * 20, [13, 7] * 300])
def test_ragged_queue_streams(apm, oracle_mod, orders):
    """Batches smaller than the persistent grids and batches whose orders leave some of the
    interleaved queue streams without work: every matrix is taken exactly once (each output
    written, the sentinel gone) and agrees with LU per subset."""
    import torch
    mats = [W.lattice_batch(1, k, W.Lattice(32, 1.0, -0.5, 5.0), seed=900 + i)[0] for i, k in enumerate(orders)]
    ns, flat, ooff, tot = pack(mats)
    out = torch.full((tot,), 3.0, dtype=torch.float64, device="cuda")
    _, _, info = apm.all_minors_ragged(torch.from_numpy(flat).cuda(), torch.from_numpy(ns).cuda(), int(ns.max()), "r64",
                                       out=out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    assert np.all(info.cpu().numpy() >= 0)
    done = set()
    for k, M in enumerate(mats):
        n = M.shape[0]
        if n in done and len(mats) > 40:
            continue   # long batches: one matrix of each order against the oracle
        done.add(n)
        seg = got[ooff[k]:ooff[k] + (1 << n)]
        ref = oracle_mod.minors(M)
        assert metrics.mixed_err(seg, ref, metrics.hadamard_bounds(M)).max() <= 1e-10, (k, n)
    # every matrix was written: the sentinel survives nowhere (a minor equal to it is vanishingly rare)
    assert not np.any(got == 3.0)


def test_ragged_bad_order_reported(apm):
    import torch
    ns = np.array([3, 25, 0, 4], dtype=np.int32)
    flat = np.concatenate([np.eye(3).ravel(), np.zeros(0), np.zeros(0), 2 * np.eye(4).ravel()])
    ioff = np.array([0, 9, 9, 9], dtype=np.int64)
    ooff = np.array([0, 8, 8, 8], dtype=np.int64)
    out = torch.zeros(8 + 16, dtype=torch.float64, device="cuda")
    _, _, info = apm.all_minors_ragged(torch.from_numpy(flat).cuda(), torch.from_numpy(ns).cuda(), 20, "r64",
                                       in_off=torch.from_numpy(ioff).cuda(), out_off=torch.from_numpy(ooff).cuda(),
                                       out=out)
    torch.cuda.synchronize()
    assert info.cpu().numpy().tolist() == [0, -1, -1, 0]
    o = out.cpu().numpy()
    assert np.all(o[:8] == 1.0)
    assert np.allclose(o[8:], [2.0 ** bin(m).count("1") for m in range(16)])


@pytest.mark.parametrize("dtype", ["r32s", "c128"])
def test_ragged_other_types(apm, oracle_mod, dtype):
    import torch
    orders = [6, 12, 3, 10, 14, 8]
    if dtype == "c128":
        mats = [W.keldysh_batch(1, k, seed=50 + k)[0] for k in orders]
        ref = [oracle_mod.minors_complex(M) for M in mats]
    else:
        mats = [W.lattice_batch(1, k, W.Lattice(32, 1.0, -0.5, 5.0), seed=50 + k)[0] for k in orders]
        ref = [oracle_mod.minors(M) for M in mats]
    ns, flat, ooff, tot = pack(mats)
    if dtype == "c128":
        out = torch.empty(tot, dtype=torch.complex128, device="cuda")
        _, _, info = apm.all_minors_ragged(torch.from_numpy(flat).cuda(), torch.from_numpy(ns).cuda(), 14, dtype,
                                           out=out)
        got = out.cpu().numpy()
        tol = 1e-10
    else:
        out = torch.empty(tot, dtype=torch.float32, device="cuda")
        ex = torch.empty(tot, dtype=torch.int16, device="cuda")
        _, _, info = apm.all_minors_ragged(torch.from_numpy(flat).cuda(), torch.from_numpy(ns).cuda(), 14, dtype,
                                           out=out, exp=ex)
        got = apm.decode_scaled(out, ex).cpu().numpy()
        tol = 1e-4
    torch.cuda.synchronize()
    for k, M in enumerate(mats):
        seg = got[ooff[k]:ooff[k] + (1 << M.shape[0])]
        assert metrics.mixed_err(seg, ref[k], metrics.hadamard_bounds(M)).max() <= tol


def test_cdet_pipeline_ragged(apm, oracle_mod):
    """Minors -> weights a = det^2 -> rooted connected sums, mixed orders, vs the oracle."""
    import torch
    orders = [10, 13, 11, 12, 10, 14]
    mats = [W.lattice_batch(1, k, W.Lattice(32, 1.0, -0.5, 5.0), seed=70 + i)[0] for i, k in enumerate(orders)]
    ns, flat, ooff, tot = pack(mats)
    m = torch.empty(tot, dtype=torch.float64, device="cuda")
    n_t = torch.from_numpy(ns).cuda()
    apm.all_minors_ragged(torch.from_numpy(flat).cuda(), n_t, 14, "r64", out=m)
    c = torch.empty_like(m)
    off = torch.from_numpy(ooff).cuda()
    bd = apm.make_batch(len(ns), 0, n_t, 14, off, off)
    assert apm.apm_connected_sums(apm._ptr(m), None, bd, apm._ptr(c), apm.APM_CS_ROOTED, apm._stream(None)) == 0
    torch.cuda.synchronize()
    got = c.cpu().numpy()
    for k, M in enumerate(mats):
        a = oracle_mod.minors(M) ** 2
        ref = oracle_mod.connected_sums(a, 0)
        d = oracle_mod.cs_scale(a, ref, 0)
        seg = got[ooff[k]:ooff[k] + (1 << M.shape[0])]
        assert np.all(np.abs(seg - ref) <= 1e-10 * d + 1e-300)


def test_mixed_pipeline_graph_replay(apm, oracle_mod):
    """The mixed-order pipeline (queue preparation, persistent minors launch, connected
    sums) captured in a HIP graph and replayed several times, with eager work between the
    replays (clearing the outputs and an unrelated ragged launch that reuses the library's
    queue workspace): every replay reproduces the eager result bit for bit."""
    import torch
    mats, ns = W.lattice_ragged(600, 8, 14, W.Lattice(32, 1.0, -0.5, 5.0), seed=91)
    nsz, flat, ooff, tot = pack(mats)
    A = torch.from_numpy(flat).cuda()
    n_t = torch.from_numpy(nsz).cuda()
    m = torch.empty(tot, dtype=torch.float64, device="cuda")
    c = torch.empty_like(m)
    bd = apm.make_batch(len(nsz), 0, n_t, 14, None, None)

    def pipeline():
        apm.all_minors_ragged(A, n_t, 14, "r64", out=m)
        rc = apm.apm_connected_sums(apm._ptr(m), None, bd, apm._ptr(c), apm.APM_CS_ROOTED, apm._stream(None))
        assert rc == 0

    pipeline()
    torch.cuda.synchronize()
    m_ref, c_ref = m.clone(), c.clone()
    # the eager result is right
    got = m_ref.cpu().numpy()
    for k in range(0, len(mats), 37):
        M = mats[k]
        seg = got[ooff[k]:ooff[k] + (1 << M.shape[0])]
        assert metrics.mixed_err(seg, oracle_mod.minors(M), metrics.hadamard_bounds(M)).max() <= 1e-10
    other_mats, other_ns = W.lattice_ragged(100, 10, 12, W.Lattice(32, 1.0, -0.5, 5.0), seed=92)
    o_ns, o_flat, _, o_tot = pack(other_mats)
    oA = torch.from_numpy(o_flat).cuda()
    on_t = torch.from_numpy(o_ns).cuda()
    om = torch.empty(o_tot, dtype=torch.float64, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        pipeline()
    torch.cuda.current_stream().wait_stream(side)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        pipeline()
    for i in range(4):
        m.zero_()
        c.zero_()
        apm.all_minors_ragged(oA, on_t, 12, "r64", out=om)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(m, m_ref), i
        assert torch.equal(c, c_ref), i


def test_ragged_default_offsets_csum_perm(apm, oracle_mod):
    """Mixed-order batches given without offset arrays use the packed prefix sums of
    n_b^2 and 2^n_b, for the connected sums and the permanents as for the minors."""
    import torch
    mats, ns = W.lattice_ragged(64, 3, 12, W.Lattice(16, 1.0, 0.0, 4.0), seed=93)
    nsz, flat, ooff, tot = pack(mats)
    n_t = torch.from_numpy(nsz).cuda()
    A = torch.from_numpy(flat).cuda()
    m = torch.empty(tot, dtype=torch.float64, device="cuda")
    apm.all_minors_ragged(A, n_t, 12, "r64", out=m)
    c_def = torch.empty_like(m)
    c_exp = torch.empty_like(m)
    st = apm._stream(None)
    assert apm.apm_connected_sums(apm._ptr(m), None, apm.make_batch(len(nsz), 0, n_t, 12, None, None),
                                  apm._ptr(c_def), apm.APM_CS_ROOTED, st) == 0
    oo = torch.from_numpy(ooff).cuda()
    assert apm.apm_connected_sums(apm._ptr(m), None, apm.make_batch(len(nsz), 0, n_t, 12, oo, oo),
                                  apm._ptr(c_exp), apm.APM_CS_ROOTED, st) == 0
    p_def = torch.empty_like(m)
    assert apm.apm_all_perm_minors(apm._ptr(A), apm.make_batch(len(nsz), 0, n_t, 12, None, None),
                                   apm._ptr(p_def), st) == 0
    torch.cuda.synchronize()
    assert torch.equal(c_def, c_exp)
    got = p_def.cpu().numpy()
    for k in range(0, len(mats), 5):
        M = mats[k]
        seg = got[ooff[k]:ooff[k] + (1 << M.shape[0])]
        ref = oracle_mod.perm_minors(M)
        assert np.allclose(seg, ref, rtol=1e-9, atol=1e-12 * np.abs(ref).max())


def test_capture_survives_workspace_growth(apm, oracle_mod):
    """A graph captured from a direct mixed-order call keeps the library workspace it
    recorded: a later direct call that needs a larger workspace replaces it without
    freeing it, so the next replay reads and writes live memory and gives the same bits."""
    import torch
    mats, _ = W.lattice_ragged(48, 6, 11, W.Lattice(16, 1.0, 0.0, 4.0), seed=95)
    ns, flat, ooff, tot = pack(mats)
    A = torch.from_numpy(flat).cuda()
    n_t = torch.from_numpy(ns).cuda()
    m = torch.empty(tot, dtype=torch.float64, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        apm.all_minors_ragged(A, n_t, 11, "r64", out=m)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    m_ref = m.clone()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        apm.all_minors_ragged(A, n_t, 11, "r64", out=m)
    # more matrices than any earlier call of this process used: the workspace must grow
    big = 1 << 17
    rng = np.random.default_rng(96)
    bns = rng.integers(2, 5, big).astype(np.int32)
    bflat = np.concatenate([np.eye(k).ravel() * 2.0 for k in bns])
    btot = int(np.sum(np.left_shift(1, bns.astype(np.int64))))
    bm = torch.empty(btot, dtype=torch.float64, device="cuda")
    _, _, binfo = apm.all_minors_ragged(torch.from_numpy(bflat).cuda(), torch.from_numpy(bns).cuda(), 4, "r64",
                                        out=bm)
    torch.cuda.synchronize()
    assert int(binfo.min()) == 0
    # minors of 2 I: 2^|S|
    bo = np.concatenate([[0], np.cumsum(np.left_shift(1, bns.astype(np.int64)))[:-1]])
    got = bm.cpu().numpy()
    for k in range(0, big, 4099):
        seg = got[bo[k]:bo[k] + (1 << bns[k])]
        assert np.array_equal(seg, 2.0 ** np.array([bin(s).count("1") for s in range(1 << bns[k])]))
    for i in range(2):
        m.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(m, m_ref), i


def test_mixed_kernel_variants_and_autotune(apm, oracle_mod, tmp_path, monkeypatch):
    """Every instantiated lane-subtree order of the two mixed-order kernels (installed through
    the tuning cache) against the oracle on a batch of orders 1..20; then the mixed-order
    autotuner records its choices in the cache and a plan created with autotuning pins them."""
    import json
    import torch
    path = tmp_path / "tune.json"
    monkeypatch.setenv("APM_TUNE_CACHE", str(path))
    rng = np.random.default_rng(11)
    orders = [14, 3, 16, 9, 15, 12, 1, 13, 20, 10, 7, 16, 11, 14, 5, 18]
    mats = [W.lattice_batch(1, k, W.Lattice(32, 1.0, -0.5, 5.0), seed=900 + i)[0] for i, k in enumerate(orders)]
    ns, flat, ooff, tot = pack(mats)
    n_t = torch.from_numpy(ns).cuda()
    A_t = torch.from_numpy(flat).cuda()
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    default = apm.minors_k0_mixed("r64")
    assert default == (4, 5)
    try:
        for ks in (3, 4):
            for kl in (4, 5):
                json.dump({"version": 1, "k0": {f"{arch}/r64/mixed": ks, f"{arch}/r64/mixed-large": kl}},
                          open(path, "w"))
                assert apm.tune_cache_load(str(path)) == 2
                assert apm.minors_k0_mixed("r64") == (ks, kl)
                out = torch.full((tot,), 3.0, dtype=torch.float64, device="cuda")
                _, _, info = apm.all_minors_ragged(A_t, n_t, 20, "r64", out=out)
                torch.cuda.synchronize()
                got = out.cpu().numpy()
                assert np.all(info.cpu().numpy() >= 0)
                for k, M in enumerate(mats):
                    n = M.shape[0]
                    seg = got[ooff[k]:ooff[k] + (1 << n)]
                    if n <= 12:
                        e = metrics.mixed_err(seg, oracle_mod.minors(M), metrics.hadamard_bounds(M))
                    else:
                        masks = np.unique(np.concatenate([rng.integers(0, 1 << n, 600), [0, (1 << n) - 1]]))
                        e = metrics.mixed_err(seg[masks], oracle_mod.minors_at(M, masks), metrics.hadamard_at(M, masks))
                    assert e.max() <= 1e-10, (ks, kl, n, float(e.max()))
        # the autotuner: choices in range, installed, and recorded under the mixed keys
        path.unlink()
        ks, kl = apm.autotune_minors_mixed("r64", batch=700)
        assert ks in (3, 4) and kl in (4, 5)
        assert apm.minors_k0_mixed("r64") == (ks, kl)
        doc = json.load(open(path))
        assert doc["k0"][f"{arch}/r64/mixed"] == ks and doc["k0"][f"{arch}/r64/mixed-large"] == kl
        # a plan with autotuning takes the installed values
        out = torch.empty((tot,), dtype=torch.float64, device="cuda")
        p = apm.plan_minors(A_t, out, n=n_t, n_max=20, autotune=True)
        assert p.k0 == ks
        p.launch()
        torch.cuda.synchronize()
        ref = torch.empty_like(out)
        apm.all_minors_ragged(A_t, n_t, 20, "r64", out=ref)
        torch.cuda.synchronize()
        assert torch.equal(out, ref)
        p.close()
    finally:
        json.dump({"version": 1, "k0": {f"{arch}/r64/mixed": default[0], f"{arch}/r64/mixed-large": default[1]}},
                  open(path, "w"))
        apm.tune_cache_load(str(path))
    assert apm.minors_k0_mixed("r64") == default


@pytest.mark.parametrize("dtype", ["r32s", "c128", "c64s"])
def test_mixed_kernel_variants_other_types(apm, oracle_mod, dtype, tmp_path):
    """The other element types' mixed-order kernel variants (every instantiated lane-subtree
    order of both kernels, installed through a cache file) against the oracle: orders below,
    inside and above the large-order kernel's range."""
    import json
    import torch
    ranges = {"r32s": ((3, 4), (4, 5)), "c128": ((2,), (2, 3)), "c64s": ((3,), (3, 4))}[dtype]
    cplx = dtype in ("c128", "c64s")
    orders = [9, 14, 15, 3, 16, 12] if cplx else [9, 14, 15, 3, 16, 12, 17]
    if cplx:
        mats = [W.keldysh_batch(1, k, seed=70 + k)[0] for k in orders]
    else:
        mats = [W.lattice_batch(1, k, W.Lattice(32, 1.0, -0.5, 5.0), seed=70 + k)[0] for k in orders]
    ns, flat, ooff, tot = pack(mats)
    rng = np.random.default_rng(5)
    refs = []   # (masks or None, reference values, bounds)
    for M in mats:
        n = M.shape[0]
        if cplx or n <= 12:
            full = oracle_mod.minors_complex(M) if cplx else oracle_mod.minors(M)
            refs.append((None, full, metrics.hadamard_bounds(M)))
        else:
            masks = np.unique(np.concatenate([rng.integers(0, 1 << n, 400), [0, (1 << n) - 1]]))
            refs.append((masks, oracle_mod.minors_at(M, masks), metrics.hadamard_at(M, masks)))
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    path = tmp_path / "tune.json"
    default = apm.minors_k0_mixed(dtype)
    tol = 1e-10 if dtype == "c128" else 1e-4
    A = torch.from_numpy(flat).cuda()
    n_t = torch.from_numpy(ns).cuda()
    try:
        for ks in ranges[0]:
            for kl in ranges[1]:
                json.dump({"version": 1, "k0": {f"{arch}/{dtype}/mixed": ks, f"{arch}/{dtype}/mixed-large": kl}},
                          open(path, "w"))
                assert apm.tune_cache_load(str(path)) == 2 and apm.minors_k0_mixed(dtype) == (ks, kl)
                if dtype == "c128":
                    out = torch.empty(tot, dtype=torch.complex128, device="cuda")
                    _, _, info = apm.all_minors_ragged(A, n_t, max(orders), dtype, out=out)
                    got = out.cpu().numpy()
                else:
                    out = torch.empty(tot, dtype=torch.complex64 if cplx else torch.float32, device="cuda")
                    ex = torch.empty(tot, dtype=torch.int16, device="cuda")
                    _, _, info = apm.all_minors_ragged(A, n_t, max(orders), dtype, out=out, exp=ex)
                    got = apm.decode_scaled(out, ex).cpu().numpy()
                torch.cuda.synchronize()
                assert np.all(info.cpu().numpy() >= 0)
                for k, M in enumerate(mats):
                    seg = got[ooff[k]:ooff[k] + (1 << M.shape[0])]
                    masks, ref, H = refs[k]
                    e = metrics.mixed_err(seg if masks is None else seg[masks], ref, H)
                    assert e.max() <= tol, (dtype, ks, kl, M.shape[0], float(e.max()))
    finally:
        json.dump({"version": 1, "k0": {f"{arch}/{dtype}/mixed": default[0],
                                        f"{arch}/{dtype}/mixed-large": default[1]}}, open(path, "w"))
        apm.tune_cache_load(str(path))
    assert apm.minors_k0_mixed(dtype) == default
