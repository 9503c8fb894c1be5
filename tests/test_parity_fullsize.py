"""GPU parity at the full sizes of the secondary workloads, with the inputs and launch
configuration the benchmark times, on sampled outputs the oracle computes one by one:

* 8192 lattice matrices of mixed order n in {10..16} (one persistent launch) and their
  rooted connected sums (a = det^2);
* 4096 complex Keldysh matrices of order 14, complex128 and complex64-scaled;
* all permanent principal minors of 2048 real order-12 matrices.
"""
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


def test_mixed_orders_8192_sampled(apm, oracle_mod):
    import torch
    mats, ns = W.lattice_ragged(8192, 10, 16, W.Lattice(32, 1.0, -0.5, 5.0), seed=W.BASE_SEED + 1)
    flat = torch.from_numpy(np.concatenate([m.ravel() for m in mats])).cuda()
    n_t = torch.from_numpy(ns).cuda()
    sizes = np.left_shift(1, ns.astype(np.int64))
    ooff_np = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    ooff = torch.from_numpy(ooff_np).cuda()
    mm = torch.empty(int(sizes.sum()), dtype=torch.float64, device="cuda")
    cc = torch.empty_like(mm)
    _, _, info = apm.all_minors_ragged(flat, n_t, 16, "r64", out=mm, out_off=ooff)
    bd = apm.make_batch(8192, 0, n_t, 16, ooff, ooff)
    assert apm.apm_connected_sums(apm._ptr(mm), None, bd, apm._ptr(cc), apm.APM_CS_ROOTED, apm._stream(None)) == 0
    torch.cuda.synchronize()
    assert np.all(info.cpu().numpy() >= 0)
    rng = np.random.default_rng(8192)
    sel = rng.choice(8192, 48, replace=False)
    for b in sel:
        n = int(ns[b])
        masks = np.unique(np.concatenate([rng.integers(0, 1 << n, 256, dtype=np.uint32),
                                          np.array([0, (1 << n) - 1], dtype=np.uint32)]))
        got = mm[int(ooff_np[b]) + torch.from_numpy(masks.astype(np.int64)).cuda()].cpu().numpy()
        ref = oracle_mod.minors_at(mats[b], masks)
        H = metrics.hadamard_bounds(mats[b])[masks]
        assert np.max(metrics.mixed_err(got, ref, H)) <= 1e-10, (b, n)
    # connected sums of sampled matrices of each order, from the GPU's own minors
    for n in range(10, 17):
        b = int(np.flatnonzero(ns == n)[0])
        seg = slice(int(ooff_np[b]), int(ooff_np[b]) + (1 << n))
        m = mm[seg].cpu().numpy()
        c = cc[seg].cpu().numpy()
        cref = oracle_mod.connected_sums(m * m, 0)
        d = oracle_mod.cs_scale(m * m, cref, 0)
        assert np.all(np.abs(c - cref) <= 1e-10 * d + 1e-300), n


def test_keldysh_4096_sampled(apm, oracle_mod):
    import torch
    K = torch.from_numpy(W.keldysh_batch(4096, 14)).cuda()
    oc = torch.empty((4096, 1 << 14), dtype=torch.complex128, device="cuda")
    apm.all_minors(K, "c128", out=oc)
    o64, ex, _ = apm.all_minors(K, "c64s")
    torch.cuda.synchronize()
    rng = np.random.default_rng(4096)
    sel = np.sort(rng.choice(4096, 12, replace=False))
    A = K[torch.from_numpy(sel).cuda()].cpu().numpy()
    ref = oracle_mod.minors_complex(A)
    idx = torch.from_numpy(sel).cuda()
    assert metrics.max_mixed_err(oc[idx].cpu().numpy(), ref, A) <= 1e-10
    val = apm.decode_scaled(o64[idx], ex[idx]).cpu().numpy()
    assert metrics.max_mixed_err(val, ref, A) <= 1e-4


def test_perm_2048_sampled(apm, oracle_mod):
    import torch
    P = W.gauss_batch(2048, 12)
    got_t = apm.all_perm_minors(torch.from_numpy(P).cuda())
    torch.cuda.synchronize()
    rng = np.random.default_rng(2048)
    sel = rng.choice(2048, 16, replace=False)
    for b in sel:
        masks = np.unique(np.concatenate([rng.integers(0, 1 << 12, 128, dtype=np.uint32),
                                          np.array([0, (1 << 12) - 1], dtype=np.uint32)]))
        got = got_t[int(b)][torch.from_numpy(masks.astype(np.int64)).cuda()].cpu().numpy()
        ref = oracle_mod.perm_minors_at(P[b], masks)
        rs = np.abs(P[b]).sum(axis=1)
        bound = np.array([np.prod(rs[[i for i in range(12) if m >> i & 1]]) * 2.0 ** bin(int(m)).count("1")
                          for m in masks])
        assert np.all(np.abs(got - ref) <= 1e-10 * bound), b
