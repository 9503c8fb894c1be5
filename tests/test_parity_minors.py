"""GPU parity of apm_all_minors against the CPU oracle (mixed-metric tolerances:
1e-10 for fp64 / complex128, 1e-4 for the fp32-scaled variants)."""
import numpy as np
import pytest

from oracle import metrics
import workloads as W

pytestmark = pytest.mark.gpu

TOL64 = 1e-10
TOL32 = 1e-4


@pytest.fixture(scope="module")
def apm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2104_07638_amd as m
    return m


def run(apm, A, dtype="r64", **kw):
    import torch
    At = torch.from_numpy(np.ascontiguousarray(A)).cuda()
    out, ex, info = apm.all_minors(At, dtype, **kw)
    torch.cuda.synchronize()
    if ex is not None:
        out = apm.decode_scaled(out, ex)
    return out.cpu().numpy(), info.cpu().numpy()


def test_lattice_n8_full_batch(apm, oracle_mod):
    """1024 real 8x8 lattice propagator matrices (L=16, t=1, mu=0, beta=4), every minor."""
    A = W.lattice_batch(1024, 8, W.Lattice(16, 1.0, 0.0, 4.0))
    out, info = run(apm, A)
    ref = oracle_mod.minors(A)
    assert np.all(info == 0)
    assert out[:, 0].tolist() == [1.0] * 1024
    assert metrics.max_mixed_err(out, ref, A) <= TOL64


@pytest.mark.parametrize("n", list(range(1, 15)))
def test_all_orders_gauss(apm, oracle_mod, n):
    rng = np.random.default_rng(100 + n)
    A = rng.standard_normal((5, n, n)) / np.sqrt(n) + np.eye(n)
    out, info = run(apm, A)
    ref = oracle_mod.minors(A)
    assert metrics.max_mixed_err(out, ref, A) <= TOL64
    assert np.all(info >= 0)


@pytest.mark.parametrize("n", [15, 16, 17, 18, 20])
def test_large_orders_sampled(apm, oracle_mod, n):
    A = W.lattice_batch(3, n, W.Lattice(32, 1.0, -0.5, 5.0), seed=7 + n)
    out, info = run(apm, A)
    rng = np.random.default_rng(n)
    masks = np.unique(np.concatenate([rng.integers(0, 1 << n, 3000), [0, 1, (1 << n) - 1, 1 << (n - 1)],
                                      (1 << np.arange(n))]))
    for b in range(3):
        ref = oracle_mod.minors_at(A[b], masks)
        e = metrics.mixed_err(out[b, masks], ref, metrics.hadamard_at(A[b], masks))
        assert e.max() <= TOL64, (b, e.max())
    # sum of all minors = det(I + A), checked on the whole output
    for b in range(3):
        ref = np.linalg.det(np.eye(n) + A[b])
        assert abs(out[b].sum() - ref) <= 1e-9 * np.abs(out[b]).sum()


def spine_shifts(n):
    """Shifts a zero diagonal needs: every left-spine node of order >= 2 has a zero pivot
    (Sec. II: n-1 of them).  Here 2 x 2 nodes inside the per-lane subtrees (orders n >= 8,
    whose lane subtrees have order >= 2) are finished by their explicit determinant
    without a division, so the last spine node needs no shift there."""
    return n - 1 if n < 8 else n - 2


@pytest.mark.parametrize("n", [2, 3, 6, 7, 8, 10, 11, 12, 16])
def test_zero_diagonal_shifts(apm, oracle_mod, n):
    """Sec. II: a matrix with zero diagonal needs one pivot correction per left-spine
    node that divides, and generically exactly that many when only (near-)exact zeros are
    shifted (tiny tau).  With the default threshold a few relatively small Schur pivots
    may be shifted too."""
    G = W.zero_diagonal(W.gauss_batch(4, n, seed=n))
    out, info = run(apm, G, tau=1e-12)
    assert np.all(info == spine_shifts(n)), info
    assert metrics.max_mixed_err(out, oracle_mod.minors(G), G) <= TOL64
    out, info = run(apm, G)
    assert np.all(info >= spine_shifts(n)), info
    assert metrics.max_mixed_err(out, oracle_mod.minors(G), G) <= TOL64
    # lattice propagators with zero diagonal, at the library's default threshold
    for lat in (W.Lattice(16, 1.0, 0.0, 4.0), W.Lattice(32, 1.0, -0.5, 5.0)):
        A = W.zero_diagonal(W.lattice_batch(4, n, lat, seed=n))
        out, info = run(apm, A)
        assert np.all(info >= spine_shifts(n)), info
        assert metrics.max_mixed_err(out, oracle_mod.minors(A), A) <= TOL64


@pytest.mark.parametrize("mu,L,beta", [(0.0, 16, 4.0), (-0.5, 32, 5.0)])
@pytest.mark.parametrize("n", [8, 12, 16])
def test_zero_diagonal_lattice_default_threshold(apm, oracle_mod, mu, L, beta, n):
    """The DiagMC case that motivates the pivot correction (Sec. II): propagator matrices
    with their diagonal set to zero, half-filled (mu = 0, every odd-order minor vanishes
    structurally) and at the mixed-order workload's filling, every minor within 1e-10 at the
    library's default threshold, and a complex128 copy of the same matrices."""
    A = W.zero_diagonal(W.lattice_batch(16, n, W.Lattice(L, 1.0, mu, beta), seed=1000 + n))
    ref = oracle_mod.minors(A)
    out, info = run(apm, A)
    assert np.all(info >= spine_shifts(n)), info
    assert metrics.max_mixed_err(out, ref, A) <= TOL64
    out, info = run(apm, A.astype(np.complex128), "c128")
    assert metrics.max_mixed_err(out, ref, A) <= TOL64


def test_zero_diagonal_lattice_fp32_scaled(apm, oracle_mod):
    """fp32-scaled minors of zero-diagonal propagators: with the shift threshold raised to
    0.03 (the default 1e-3 leaves Schur complements whose fp32 rounding exceeds the gate on
    these matrices) every minor is within the fp32 gate."""
    for lat in (W.Lattice(16, 1.0, 0.0, 4.0), W.Lattice(32, 1.0, -0.5, 5.0)):
        for n in (8, 12, 16):
            A = W.zero_diagonal(W.lattice_batch(4, n, lat, seed=n))
            out, info = run(apm, A, "r32s", tau=0.03)
            assert metrics.max_mixed_err(out, oracle_mod.minors(A), A) <= TOL32, (lat, n)


def test_stress_injections_n16(apm, oracle_mod):
    A = W.lattice_batch(256, 16, W.Lattice(32, 1.0, -0.5, 5.0), seed=3)
    A, log = W.inject_stress(A, every=64)
    out, info = run(apm, A)
    stressed = [b for b, _, _ in log]
    ref = oracle_mod.minors(A[stressed])
    assert metrics.max_mixed_err(out[stressed], ref, A[stressed]) <= TOL64
    assert np.all(info >= 0)
    normal = [1, 2, 100, 255]
    ref = oracle_mod.minors(A[normal])
    assert metrics.max_mixed_err(out[normal], ref, A[normal]) <= TOL64


def test_exact_zero_pivots_and_singular(apm, oracle_mod):
    rng = np.random.default_rng(5)
    n = 12
    A = rng.standard_normal((4, n, n))
    A[0] = 0.0                                 # all-zero matrix
    A[1, 3, :] = A[1, 5, :]                    # singular: two equal rows
    A[2, :, 7] = 0.0                           # zero column
    A[3, 0, 0] = 0.0
    A[3, 11, 11] = 0.0
    out, info = run(apm, A)
    ref = oracle_mod.minors(A)
    assert metrics.max_mixed_err(out, ref, A) <= TOL64
    assert np.all(out[0, 1:] == 0.0) and out[0, 0] == 1.0


def test_nonfinite_input_reported(apm):
    A = np.eye(8)[None].repeat(3, 0).copy()
    A[1, 2, 3] = np.nan
    A[2, 0, 0] = np.inf
    out, info = run(apm, A)
    assert info.tolist() == [0, -2, -2]
    assert np.all(np.isnan(out[1])) and np.all(np.isnan(out[2]))
    assert np.all(out[0] == 1.0)


def test_offsets_and_determinism(apm, oracle_mod):
    import torch
    rng = np.random.default_rng(9)
    n, B = 10, 6
    A = rng.standard_normal((B, n, n)) + 2 * np.eye(n)
    # scatter the matrices with gaps, outputs in reverse order
    buf = np.zeros(B * n * n + 1000)
    ioff = np.array([37 + b * (n * n + 50) for b in range(B)], dtype=np.int64)
    for b in range(B):
        buf[ioff[b]:ioff[b] + n * n] = A[b].ravel()
    ooff = np.array([(B - 1 - b) * (1 << n) for b in range(B)], dtype=np.int64)
    dA = torch.from_numpy(buf).cuda()
    out = torch.full((B << n,), 7.0, dtype=torch.float64, device="cuda")
    info = torch.empty(B, dtype=torch.int32, device="cuda")
    bd = apm.make_batch(B, n, None, 0, torch.from_numpy(ioff).cuda(), torch.from_numpy(ooff).cuda())
    for rep in range(2):
        rc = apm.apm_all_minors(apm.APM_R64, apm._ptr(dA), bd, apm._ptr(out), None, apm._ptr(info), None,
                                apm._stream(None))
        assert rc == 0
        torch.cuda.synchronize()
        got = out.cpu().numpy().reshape(B, 1 << n)[::-1]
        if rep == 0:
            first = got.copy()
        else:
            assert np.array_equal(first, got)
    ref = oracle_mod.minors(A)
    assert metrics.max_mixed_err(got, ref, A) <= TOL64


@pytest.mark.parametrize("n", [8, 12, 16])
def test_fp32_scaled(apm, oracle_mod, n):
    A = W.lattice_batch(16, n, W.Lattice(32, 1.0, -0.5, 5.0), seed=11)
    A, _ = W.inject_stress(A, every=8)
    ref = oracle_mod.minors(A)
    out, info = run(apm, A, "r32s")
    assert metrics.max_mixed_err(out, ref, A) <= TOL32
    out2, _ = run(apm, A, "r32s", out_f64=True)
    assert metrics.max_mixed_err(out2, ref, A) <= TOL32


def test_fp32_scaled_large_range(apm, oracle_mod):
    """Entries of size 1e30 and 1e-30: the exponent carries what fp32 cannot."""
    rng = np.random.default_rng(12)
    A = rng.standard_normal((4, 10, 10)) + 3 * np.eye(10)
    A[0] *= 1e30
    A[1] *= 1e-30
    ref = oracle_mod.minors(A)
    out, info = run(apm, A, "r32s")
    assert metrics.max_mixed_err(out, ref, A) <= TOL32


@pytest.mark.parametrize("n", [4, 9, 14])
def test_complex_keldysh(apm, oracle_mod, n):
    A = W.keldysh_batch(8, n, seed=21 + n)
    ref = oracle_mod.minors_complex(A)
    out, info = run(apm, A, "c128")
    assert metrics.max_mixed_err(out, ref, A) <= TOL64
    out, info = run(apm, A, "c64s")
    assert metrics.max_mixed_err(out, ref, A) <= TOL32
    out, info = run(apm, A, "c64s", out_f64=True)
    assert metrics.max_mixed_err(out, ref, A) <= TOL32


def test_complex_zero_diagonal(apm, oracle_mod):
    rng = np.random.default_rng(3)
    n = 11
    A = rng.standard_normal((3, n, n)) + 1j * rng.standard_normal((3, n, n))
    A[:, np.arange(n), np.arange(n)] = 0
    out, info = run(apm, A, "c128")
    assert np.all(info == spine_shifts(n))
    ref = oracle_mod.minors_complex(A)
    assert metrics.max_mixed_err(out, ref, A) <= TOL64


@pytest.mark.parametrize("dtype,n", [("r64", 12), ("c128", 11), ("r32s", 9)])
def test_autotuned_layout(apm, oracle_mod, dtype, n):
    """apm_autotune_minors installs one of the instantiated lane-subtree orders for
    (dtype, n); results stay correct with it."""
    k = apm.autotune_minors(dtype, n, batch=512)
    dt = apm.DTYPES[dtype]
    assert apm.apm_minors_k0(dt, n) == k
    lo, hi = {"r64": (3, 5), "r32s": (3, 5), "c128": (2, 3)}[dtype]
    assert lo <= k <= hi
    if dtype == "c128":
        A = W.keldysh_batch(64, n, seed=n)
        out, info = run(apm, A, "c128")
        ref = oracle_mod.minors_complex(A)
        assert metrics.max_mixed_err(out, ref, A) <= TOL64
    else:
        A = W.lattice_batch(64, n, W.Lattice(32, 1.0, -0.5, 5.0), seed=n)
        out, info = run(apm, A, dtype)
        ref = oracle_mod.minors(A)
        assert metrics.max_mixed_err(out, ref, A) <= (TOL64 if dtype == "r64" else 1e-4)


def test_deferred_top_corrections_match_in_wave(apm, oracle_mod):
    """Uniform batches queue their top-level pivot corrections for a follow-up launch; a
    captured call on a stream without a queue of that size applies them inside the minors
    kernel.  Both orders of work give the same bits, and both match the oracle."""
    import torch
    n, B = 12, 4104                                    # more matrices than a fresh queue holds
    A = W.lattice_batch(B, n, W.Lattice(16, 1.0, 0.2, 4.0), seed=77)
    A[::8] = W.zero_diagonal(A[::8])                   # spine shifts, the top level included
    At = torch.from_numpy(A).cuda()
    out = torch.empty((B, 1 << n), dtype=torch.float64, device="cuda")
    info = torch.empty(B, dtype=torch.int32, device="cuda")
    apm.all_minors(At, "r64", out=out, info=info)   # queued corrections
    apm.all_minors(At, "r64", out=out, info=info)   # the queue was left ready for reuse
    torch.cuda.synchronize()
    eager, eager_info = out.clone(), info.clone()
    g = torch.cuda.CUDAGraph()
    out2 = torch.empty_like(out)
    info2 = torch.empty_like(info)
    with torch.cuda.graph(g):
        apm.all_minors(At, "r64", out=out2, info=info2)
    for _ in range(2):
        out2.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out2, eager)
        assert torch.equal(info2, eager_info)
    assert int((eager_info > 0).sum()) >= B // 8
    sel = np.arange(0, B, 97)
    ref = oracle_mod.minors(A[sel])
    assert metrics.max_mixed_err(eager[sel].cpu().numpy(), ref, A[sel]) <= TOL64


def test_full_bench_batch_sampled(apm, oracle_mod):
    """The timed workload at its full size and in its launch configuration: 8192 order-16
    lattice matrices (L=32, t=1, mu=-0.5, beta=5), every 64th made near-singular, one
    uniform fp64 call with the default threshold (the deferred top-level corrections
    included).  Sampled matrices (all stressed ones among them) and sampled masks against
    LU per subset; the rooted connected sums of some of them against the direct recursion
    on the GPU's own minors."""
    import torch
    n, B = 16, 8192
    A = W.lattice_batch(B, n, W.Lattice(32, 1.0, -0.5, 5.0), seed=W.BASE_SEED)
    A, log = W.inject_stress(A, every=64)
    At = torch.from_numpy(A).cuda()
    out, _, info = apm.all_minors(At, "r64")
    torch.cuda.synchronize()
    rng = np.random.default_rng(16)
    stressed = [b for b, _, _ in log]
    sel = sorted(set(stressed) | set(rng.choice(B, 96, replace=False).tolist()))
    masks = np.unique(np.concatenate([rng.integers(0, 1 << n, 384, dtype=np.uint32),
                                      np.array([0, 1, (1 << n) - 1, 0x8000, 0x7FFF], dtype=np.uint32)]))
    got = out[sel][:, torch.from_numpy(masks.astype(np.int64)).cuda()].cpu().numpy()
    assert np.all(info.cpu().numpy() >= 0)
    for k, b in enumerate(sel):
        ref = oracle_mod.minors_at(A[b], masks)
        H = metrics.hadamard_bounds(A[b])[masks]
        assert np.max(metrics.mixed_err(got[k], ref, H)) <= TOL64, b
    cs = apm.connected_sums(out[sel[:4]].contiguous())
    torch.cuda.synchronize()
    m = out[sel[:4]].cpu().numpy()
    cref = oracle_mod.connected_sums(m * m, 0)
    tol = 1e-10 * oracle_mod.cs_scale(m * m, cref, 0) + 1e-300
    assert np.all(np.abs(cs.cpu().numpy() - cref) <= tol)


def test_full_bench_batch_fp32_scaled_sampled(apm, oracle_mod):
    """The fp32-scaled variant on the full timed batch: all 128 injected near-singular
    matrices and 64 sampled others, on sampled masks, within the 1e-4 gate."""
    import torch
    n, B = 16, 8192
    A = W.lattice_batch(B, n, W.Lattice(32, 1.0, -0.5, 5.0), seed=W.BASE_SEED)
    A, log = W.inject_stress(A, every=64)
    out, ex, info = apm.all_minors(torch.from_numpy(A).cuda(), "r32s")
    torch.cuda.synchronize()
    rng = np.random.default_rng(32)
    stressed = sorted(b for b, _, _ in log)
    normal = sorted(set(rng.choice(B, 64, replace=False).tolist()) - set(stressed))
    masks = np.unique(np.concatenate([rng.integers(0, 1 << n, 256, dtype=np.uint32),
                                      np.array([0, (1 << n) - 1], dtype=np.uint32)]))
    idx = torch.from_numpy(masks.astype(np.int64)).cuda()
    for group, gate in ((normal, TOL32), (stressed, TOL32)):
        val = apm.decode_scaled(out[group][:, idx], ex[group][:, idx]).cpu().numpy()
        for k, b in enumerate(group):
            ref = oracle_mod.minors_at(A[b], masks)
            H = metrics.hadamard_bounds(A[b])[masks]
            assert np.max(metrics.mixed_err(val[k], ref, H)) <= gate, b
    assert np.all(info.cpu().numpy() >= 0)


def test_complex_extreme_pivots(apm, oracle_mod):
    """Complex pivots of magnitude about 1e+160, whose squared modulus overflows fp64: the
    row and the column of index 0 (pivoted first at this order) of diagonally dominant
    complex matrices are scaled by 2^265, so every minor containing index 0 is exactly
    2^530 times that of the unscaled matrix (the reference from the oracle), and the root
    pivot is that large.  Also leading minors, whose first pivot is the same entry."""
    rng = np.random.default_rng(61)
    n = 9
    B0 = (rng.standard_normal((6, n, n)) + 1j * rng.standard_normal((6, n, n))) / 3 + 3 * np.eye(n)
    ref0 = oracle_mod.minors_complex(B0)
    A = B0.copy()
    A[:, 0, :] *= 2.0 ** 265
    A[:, :, 0] *= 2.0 ** 265
    masks = np.arange(1 << n)
    ref = ref0 * np.where(masks & 1, 2.0 ** 530, 1.0)[None, :]
    out, info = run(apm, A, "c128")
    assert np.all(info == 0), info
    assert np.all(np.isfinite(out))
    # the Hadamard bound of A itself overflows here (every row holds a 2^265 entry), and
    # the minors of a diagonally dominant matrix are well conditioned: plain relative error
    assert np.max(np.abs(out - ref) / np.abs(ref)) <= 1e-12
    import torch
    lo, li = apm.leading_minors(torch.from_numpy(A).cuda())
    torch.cuda.synchronize()
    lref = ref[:, (1 << np.arange(1, n + 1)) - 1]
    lo = lo.cpu().numpy()
    assert np.all(np.isfinite(lo))
    assert np.max(np.abs(lo - lref) / np.abs(lref)) <= 1e-12
