"""Plans (apm_plan_create / apm_plan_launch): each kind recorded once into a HIP graph by
the library and launched several times, with new input values written into the same
buffers and eager work in between, must give bit-for-bit the results of the direct calls
on the same inputs.  The direct calls are themselves checked against the oracle by the
other parity tests; here one small case per kind is also checked against the oracle."""
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


def same(a, b):
    """Bitwise equality of two tensors (NaNs included)."""
    import torch
    if a.dtype.is_complex:
        a, b = torch.view_as_real(a), torch.view_as_real(b)
    return torch.equal(a.contiguous().view(torch.uint8), b.contiguous().view(torch.uint8))


LAT = W.Lattice(32, 1.0, -0.5, 5.0)


def lattice_t(B, n, seed):
    import torch
    return torch.from_numpy(W.lattice_batch(B, n, LAT, seed=seed)).cuda()


def ragged(B, lo, hi, seed):
    import torch
    mats, ns = W.lattice_ragged(B, lo, hi, LAT, seed=seed)
    flat = torch.from_numpy(np.concatenate([m.ravel() for m in mats])).cuda()
    tot = int(np.sum(np.left_shift(1, ns.astype(np.int64))))
    return mats, ns, flat, torch.from_numpy(ns).cuda(), tot


@pytest.mark.parametrize("dtype,n,B", [("r64", 16, 300), ("r64", 9, 257), ("r32s", 14, 200), ("c128", 12, 130),
                                       ("c64s", 13, 100)])
def test_plan_minors_uniform(apm, dtype, n, B):
    import torch
    cplx = dtype in ("c128", "c64s")
    src = [torch.from_numpy(W.keldysh_batch(B, n, seed=70 + r)).cuda() if cplx else lattice_t(B, n, 70 + r)
           for r in range(3)]
    if not cplx:      # near-singular pivots: shifted pivots and deferred corrections
        src[1] = torch.from_numpy(W.inject_stress(src[1].cpu().numpy(), every=16)[0]).cuda()
    A = torch.empty_like(src[0])
    ref, ex_ref, info_ref = apm.all_minors(src[0], dtype)
    out = torch.empty_like(ref)
    ex = None if ex_ref is None else torch.empty_like(ex_ref)
    info = torch.empty_like(info_ref)
    plan = apm.plan_minors(A, out, dtype, exp=ex, info=info)
    assert plan.graphed and plan.k0 == apm.apm_minors_k0(apm.DTYPES[dtype], n)
    side = torch.cuda.Stream()
    for r in range(6):
        A.copy_(src[r % 3])
        if r % 2:         # odd launches on another stream
            side.wait_stream(torch.cuda.current_stream())
            plan.launch(side)
            torch.cuda.current_stream().wait_stream(side)
        else:
            plan.launch()
        ref, ex_ref, info_ref = apm.all_minors(src[r % 3], dtype)      # eager work between launches
        torch.cuda.synchronize()
        assert same(out, ref), (dtype, n, r)
        assert ex is None or same(ex, ex_ref)
        assert same(info, info_ref)


def test_plan_minors_oracle(apm, oracle_mod):
    import torch
    A = lattice_t(40, 10, 91)
    out = torch.empty((40, 1 << 10), dtype=torch.float64, device="cuda")
    plan = apm.plan_minors(A, out, "r64")
    plan.launch()
    plan.launch()
    torch.cuda.synchronize()
    An = A.cpu().numpy()
    got = out.cpu().numpy()
    for b in range(40):
        ref = oracle_mod.minors(An[b])
        assert metrics.mixed_err(got[b], ref, metrics.hadamard_bounds(An[b])).max() <= 1e-10, b


def test_plan_autotune_and_eager(apm):
    import torch
    A = lattice_t(512, 15, 92)
    out = torch.empty((512, 1 << 15), dtype=torch.float64, device="cuda")
    tuned = apm.plan_minors(A, out, "r64", autotune=True)
    k = tuned.k0
    assert k == apm.apm_minors_k0(apm.APM_R64, 15)    # installed for the process, pinned in the plan
    tuned.launch()
    torch.cuda.synchronize()
    got = out.clone()
    ref, _, _ = apm.all_minors(A, "r64")
    eager = apm.plan_minors(A, out, "r64", eager=True)
    assert not eager.graphed and eager.k0 == k
    out.fill_(7.0)
    eager.launch()
    eager.launch()
    torch.cuda.synchronize()
    assert same(got, ref) and same(out, ref)
    tuned.close()
    eager.close()


def test_plan_minors_ragged(apm, oracle_mod):
    import torch
    mats, ns, flat, n_t, tot = ragged(700, 8, 16, 93)
    A = torch.empty_like(flat)
    out = torch.empty(tot, dtype=torch.float64, device="cuda")
    info = torch.empty(700, dtype=torch.int32, device="cuda")
    plan = apm.plan_minors(A, out, "r64", info=info, n=n_t, n_max=16)
    ref = torch.empty_like(out)
    for r in range(3):
        A.copy_(flat * (1.0 + r))
        plan.launch()
        _, _, info_ref = apm.all_minors_ragged(flat * (1.0 + r), n_t, 16, "r64", out=ref)
        torch.cuda.synchronize()
        assert same(out, ref), r
        assert same(info, info_ref)
    # one matrix of each order against the oracle (last launch: A = 3 * lattice)
    ooff = np.concatenate([[0], np.cumsum(np.left_shift(1, ns.astype(np.int64)))[:-1]])
    got = out.cpu().numpy()
    for n in range(8, 13):
        b = int(np.flatnonzero(ns == n)[0])
        M = 3.0 * mats[b]
        seg = got[ooff[b]:ooff[b] + (1 << n)]
        assert metrics.mixed_err(seg, oracle_mod.minors(M), metrics.hadamard_bounds(M)).max() <= 1e-10, n


def test_plan_connected_sums(apm, oracle_mod):
    import torch
    m, _, _ = apm.all_minors(lattice_t(64, 11, 94), "r64")
    m_dn, _, _ = apm.all_minors(lattice_t(64, 11, 95), "r64")
    for mode, dn in ((apm.APM_CS_ROOTED, None), (apm.APM_CS_ALL, m_dn)):
        c = torch.empty_like(m)
        plan = apm.plan_connected_sums(m, c, m_dn=dn, mode=mode)
        plan.launch()
        plan.launch()
        ref = apm.connected_sums(m, dn, mode=mode)
        torch.cuda.synchronize()
        assert same(c, ref), mode
    a = (m * m_dn)[:3].cpu().numpy()
    got = c[:3].cpu().numpy()
    for b in range(3):
        cref = oracle_mod.connected_sums(a[b], 1)
        d = oracle_mod.cs_scale(a[b], cref, 1)
        assert np.all(np.abs(got[b] - cref) <= 1e-10 * d + 1e-300), b


def test_plan_connected_sums_ragged_packed(apm):
    """Mixed orders without offset arrays: the plan runs its own queue preparation."""
    import torch
    mats, ns, flat, n_t, tot = ragged(300, 6, 14, 96)
    m = torch.empty(tot, dtype=torch.float64, device="cuda")
    apm.all_minors_ragged(flat, n_t, 14, "r64", out=m)
    c = torch.empty_like(m)
    bd = apm.make_batch(300, 0, n_t, 14)
    plan = apm.plan_connected_sums(m, c, n=n_t, n_max=14)
    plan.launch()
    ref = torch.empty_like(m)
    assert apm.apm_connected_sums(apm._ptr(m), None, bd, apm._ptr(ref), apm.APM_CS_ROOTED, apm._stream(None)) == 0
    torch.cuda.synchronize()
    assert same(c, ref)


def test_plan_perm_minors(apm, oracle_mod):
    import torch
    P = torch.from_numpy(W.gauss_batch(96, 12, seed=97)).cuda()
    out = torch.empty((96, 1 << 12), dtype=torch.float64, device="cuda")
    plan = apm.plan_perm_minors(P, out)
    plan.launch()
    ref = apm.all_perm_minors(P)
    torch.cuda.synchronize()
    assert same(out, ref)
    Pn = P[:2].cpu().numpy()
    masks = np.arange(1 << 12, dtype=np.uint32)[::37]
    for b in range(2):
        rs = np.abs(Pn[b]).sum(axis=1)
        bound = np.array([np.prod(rs[[i for i in range(12) if m >> i & 1]]) * 2.0 ** bin(int(m)).count("1")
                          for m in masks])
        ref = oracle_mod.perm_minors_at(Pn[b], masks)
        assert np.all(np.abs(out[b].cpu().numpy()[masks] - ref) <= 1e-10 * bound), b
    # mixed orders without offsets
    rng = np.random.default_rng(98)
    ns = rng.integers(1, 14, 200).astype(np.int32)
    flat = torch.from_numpy(rng.standard_normal(int(np.sum(ns.astype(np.int64) ** 2))) / 3).cuda()
    tot = int(np.sum(np.left_shift(1, ns.astype(np.int64))))
    n_t = torch.from_numpy(ns).cuda()
    bd = apm.make_batch(200, 0, n_t, 13)
    o2 = torch.empty(tot, dtype=torch.float64, device="cuda")
    r2 = torch.empty_like(o2)
    plan2 = apm.plan_perm_minors(flat, o2, n=n_t, n_max=13)
    plan2.launch()
    assert apm.apm_all_perm_minors(apm._ptr(flat), bd, apm._ptr(r2), apm._stream(None)) == 0
    torch.cuda.synchronize()
    assert same(o2, r2)


@pytest.mark.parametrize("two_sets", [False, True])
def test_plan_cdet_uniform(apm, two_sets):
    import torch
    B, n = 256, 14
    src = [lattice_t(B, n, 100 + r) for r in range(4)]
    A = torch.empty_like(src[0])
    A_dn = torch.empty_like(src[0]) if two_sets else None
    mm = torch.empty((B, 1 << n), dtype=torch.float64, device="cuda")
    md = torch.empty_like(mm) if two_sets else None
    c = torch.empty_like(mm)
    info = torch.empty(B, dtype=torch.int32, device="cuda")
    plan = apm.plan_cdet(A, mm, c, A_dn=A_dn, minors_dn=md, info=info)
    for r in range(3):
        A.copy_(src[r])
        if two_sets:
            A_dn.copy_(src[r + 1])
        plan.launch()
        m_ref, _, info_ref = apm.all_minors(src[r], "r64")
        d_ref = apm.all_minors(src[r + 1], "r64")[0] if two_sets else None
        c_ref = apm.connected_sums(m_ref, d_ref)
        torch.cuda.synchronize()
        assert same(mm, m_ref) and same(c, c_ref) and same(info, info_ref), r
        assert not two_sets or same(md, d_ref)


def test_plan_cdet_ragged_and_r32s(apm):
    import torch
    mats, ns, flat, n_t, tot = ragged(500, 10, 16, 101)
    mm = torch.empty(tot, dtype=torch.float64, device="cuda")
    c = torch.empty_like(mm)
    bd = apm.make_batch(500, 0, n_t, 16)
    plan = apm.plan_cdet(flat, mm, c, n=n_t, n_max=16)
    plan.launch()
    plan.launch()
    m_ref = torch.empty_like(mm)
    c_ref = torch.empty_like(mm)
    apm.all_minors_ragged(flat, n_t, 16, "r64", out=m_ref)
    assert apm.apm_connected_sums(apm._ptr(m_ref), None, bd, apm._ptr(c_ref), apm.APM_CS_ROOTED,
                                  apm._stream(None)) == 0
    torch.cuda.synchronize()
    assert same(mm, m_ref) and same(c, c_ref)
    # explicit output offsets with gaps between the matrices (matrices still packed)
    sizes = np.left_shift(1, ns.astype(np.int64))
    oo_np = np.concatenate([[0], np.cumsum(sizes + 8)[:-1]]).astype(np.int64)
    oo = torch.from_numpy(oo_np).cuda()
    tot2 = int(oo_np[-1] + sizes[-1])
    m2 = torch.full((tot2,), 5.0, dtype=torch.float64, device="cuda")
    c2 = torch.full_like(m2, 5.0)
    plan2 = apm.plan_cdet(flat, m2, c2, n=n_t, n_max=16, out_off=oo)
    plan2.launch()
    torch.cuda.synchronize()
    for b in range(0, 500, 37):
        seg2 = slice(int(oo_np[b]), int(oo_np[b] + sizes[b]))
        seg = slice(int(sizes[:b].sum()), int(sizes[:b + 1].sum()))
        assert same(m2[seg2], m_ref[seg]) and same(c2[seg2], c_ref[seg]), b
    assert torch.all(m2[int(oo_np[1]) - 8:int(oo_np[1])] == 5.0)        # gaps untouched
    # fp32-scaled minors with fp64 output feeding the sums
    A = lattice_t(128, 13, 102)
    m32 = torch.empty((128, 1 << 13), dtype=torch.float64, device="cuda")
    c32 = torch.empty_like(m32)
    p32 = apm.plan_cdet(A, m32, c32, dtype="r32s")
    p32.launch()
    r32, _, _ = apm.all_minors(A, "r32s", out_f64=True)
    cr = apm.connected_sums(r32)
    torch.cuda.synchronize()
    assert same(m32, r32) and same(c32, cr)


def test_tune_cache_roundtrip(apm, tmp_path, monkeypatch):
    """The autotuner records its choice in the JSON tuning cache keyed by (architecture,
    dtype, order), and a cache file is installed as if tuned in this process."""
    import json
    path = tmp_path / "tune.json"
    monkeypatch.setenv("APM_TUNE_CACHE", str(path))
    k = apm.autotune_minors("r64", 11, batch=256)
    doc = json.load(open(path))
    keys = [key for key in doc["k0"] if key.endswith("/r64/11")]
    assert len(keys) == 1 and keys[0].startswith("gfx") and doc["k0"][keys[0]] == k
    other = 3 if k != 3 else 4
    doc["k0"][keys[0]] = other
    json.dump(doc, open(path, "w"))
    try:
        assert apm.tune_cache_load(str(path)) == 1
        assert apm.apm_minors_k0(apm.APM_R64, 11) == other
        # a plan created with autotuning now takes the installed value without timing
        import torch
        A = torch.from_numpy(W.lattice_batch(64, 11, W.Lattice(32, 1.0, -0.5, 5.0), seed=3)).cuda()
        out = torch.empty((64, 1 << 11), dtype=torch.float64, device="cuda")
        p = apm.plan_minors(A, out, autotune=True)
        assert p.k0 == other
        p.close()
    finally:
        doc["k0"][keys[0]] = k
        json.dump(doc, open(path, "w"))
        apm.tune_cache_load(str(path))
    assert apm.apm_minors_k0(apm.APM_R64, 11) == k
    assert apm.tune_cache_load(str(tmp_path / "missing.json")) == -1
