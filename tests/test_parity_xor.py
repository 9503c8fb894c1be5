"""GPU parity of the XOR minors (Sec. III XOR case; Sec. V.C Keldysh block matrices) with
the oracle: element by element for every depth at small sizes (spanning the orders where
the top levels run from the workspace), on sampled matrices at the full size of the
benchmark, and the branch-signed sum that the largest-time identity sends to zero.  The
XNOR minors (Sec. III XNOR case) use the same kernel and are checked the same way."""
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


def xor_hadamard(A):
    """Hadamard bound prod_{i in R} ||A[i, R]||_2 of every entry's kept rows R, in output
    order (depth k: R = {2(n-k+i) + beta_i})."""
    n = A.shape[0] // 2
    out = []
    for k in range(1, n + 1):
        beta = np.arange(1 << k)[:, None]
        R = 2 * (n - k + np.arange(k))[None, :] + ((beta >> np.arange(k)[None, :]) & 1)
        sub = A[R[:, :, None], R[:, None, :]]
        out.append(np.prod(np.linalg.norm(sub, axis=2), axis=1))
    return np.concatenate(out)


def check(A, got, ref, tol=1e-10):
    """Mixed error per entry against max(|ref|, Hadamard bound of the kept rows)."""
    n = A.shape[0] // 2
    e = metrics.mixed_err(got, ref, xor_hadamard(A))
    assert e.max() <= tol, (n, float(e.max()), int(np.argmax(e)))


@pytest.mark.parametrize("n", list(range(1, 10)))
def test_keldysh_all_depths(apm, oracle_mod, n):
    import torch
    A = W.keldysh_block(6, n, seed=400 + n)
    out, info = apm.xor_minors(torch.from_numpy(A).cuda())
    torch.cuda.synchronize()
    assert np.all(info.cpu().numpy() == 0)
    got = out.cpu().numpy()
    ref = oracle_mod.xor_minors(A)
    for b in range(A.shape[0]):
        check(A[b], got[b], ref[b])


@pytest.mark.parametrize("n", [1, 3, 6, 7, 9])
def test_random_real_and_complex(apm, oracle_mod, n):
    import torch
    rng = np.random.default_rng(410 + n)
    for cplx in (False, True):
        A = rng.standard_normal((5, 2 * n, 2 * n)) + 2.0 * np.eye(2 * n)
        if cplx:
            A = A + 1j * rng.standard_normal((5, 2 * n, 2 * n))
        out, info = apm.xor_minors(torch.from_numpy(A).cuda())
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        ref = oracle_mod.xor_minors(A)
        for b in range(5):
            check(A[b], got[b], ref[b])


def test_largest_time_on_gpu(apm):
    """Branch-signed sums of the GPU's own minors vanish at every depth."""
    import torch
    n = 10
    A = W.keldysh_block(64, n, seed=420)
    out, _ = apm.xor_minors(torch.from_numpy(A).cuda())
    got = out.cpu().numpy()
    for k in range(1, n + 1):
        seg = got[:, (1 << k) - 2:(1 << (k + 1)) - 2]
        sgn = np.array([(-1) ** bin(a).count("1") for a in range(1 << k)])
        assert np.all(np.abs(seg @ sgn) <= 1e-12 * np.abs(seg).sum(axis=1)), k


def test_full_size_sampled(apm, oracle_mod):
    """4096 Keldysh block matrices with 14 blocks (the benchmark's batch): sampled matrices
    against the oracle at every depth, the largest-time identity on all of them."""
    import torch
    n = 14
    A = W.keldysh_block(4096, n, seed=W.BASE_SEED + 4)
    dA = torch.from_numpy(A).cuda()
    out, info = apm.xor_minors(dA)
    torch.cuda.synchronize()
    assert np.all(info.cpu().numpy() == 0)
    sel = np.random.default_rng(4096).choice(4096, 6, replace=False)
    got = out[torch.from_numpy(sel).cuda()].cpu().numpy()
    ref = oracle_mod.xor_minors(A[sel])
    for i in range(len(sel)):
        check(A[sel[i]], got[i], ref[i])
    full = out[:, (1 << n) - 2:]
    sgn = torch.tensor([(-1.0) ** bin(a).count("1") for a in range(1 << n)], dtype=torch.float64, device="cuda")
    s = (full * sgn).sum(dim=1).abs()
    assert bool(torch.all(s <= 1e-12 * full.abs().sum(dim=1)))


def test_error_codes(apm):
    import torch
    n = 7
    A = W.keldysh_block(4, n, seed=430)
    A[1, 3, 5] = np.nan                        # non-finite input
    A[2, 2 * n - 1, 2 * n - 1] = 0.0           # zero pivot in the first decided block
    out, info = apm.xor_minors(torch.from_numpy(A).cuda())
    torch.cuda.synchronize()
    info = info.cpu().numpy()
    assert info[0] == 0 and info[1] == -2 and info[2] == -3 and info[3] == 0
    assert bool(torch.all(torch.isnan(out[1].real)))
    assert bool(torch.all(torch.isfinite(out[0].real)))
    # an empty batch is a no-op
    rc = apm.apm_xor_minors(apm.APM_C128, None, apm.make_batch(0, n), None, None, apm._stream(None))
    assert rc == apm.APM_OK


def xnor_hadamard(A):
    """Hadamard bound of the kept rows of every XNOR entry (block-mask order)."""
    n = A.shape[0] // 2
    out = np.ones(1 << n)
    for mask in range(1, 1 << n):
        r = [x for i in range(n) if mask >> i & 1 for x in (2 * i, 2 * i + 1)]
        sub = A[np.ix_(r, r)]
        out[mask] = np.prod(np.linalg.norm(sub, axis=1))
    return out


@pytest.mark.parametrize("n", [1, 2, 4, 6, 7, 8, 10])
def test_xnor_parity(apm, oracle_mod, n):
    import torch
    rng = np.random.default_rng(500 + n)
    for cplx in (False, True):
        A = rng.standard_normal((4, 2 * n, 2 * n)) + 3.0 * np.eye(2 * n)
        if cplx:
            A = A + 1j * rng.standard_normal((4, 2 * n, 2 * n))
        out, info = apm.xnor_minors(torch.from_numpy(A).cuda())
        torch.cuda.synchronize()
        assert np.all(info.cpu().numpy() == 0)
        got = out.cpu().numpy()
        ref = oracle_mod.xnor_minors(A)
        for b in range(4):
            e = metrics.mixed_err(got[b], ref[b], xnor_hadamard(A[b]))
            assert e.max() <= 1e-10, (n, cplx, b, float(e.max()))


def test_xnor_keldysh_full_size_sampled(apm, oracle_mod):
    """4096 Keldysh block matrices of 14 blocks, sampled matrices against the oracle."""
    import torch
    n = 14
    A = W.keldysh_block(4096, n, seed=W.BASE_SEED + 4)
    out, info = apm.xnor_minors(torch.from_numpy(A).cuda())
    torch.cuda.synchronize()
    assert np.all(info.cpu().numpy() == 0)
    sel = np.random.default_rng(4097).choice(4096, 3, replace=False)
    got = out[torch.from_numpy(sel).cuda()].cpu().numpy()
    ref = oracle_mod.xnor_minors(A[sel])
    masks = np.unique(np.concatenate([np.random.default_rng(1).integers(0, 1 << n, 400), [0, (1 << n) - 1]]))
    for i in range(len(sel)):
        H = np.ones(len(masks))
        for t, mask in enumerate(masks):
            r = [x for k in range(n) if mask >> k & 1 for x in (2 * k, 2 * k + 1)]
            if r:
                H[t] = np.prod(np.linalg.norm(A[sel[i]][np.ix_(r, r)], axis=1))
        e = metrics.mixed_err(got[i][masks], ref[i][masks], H)
        assert e.max() <= 1e-10, (int(sel[i]), float(e.max()))


def nand_rows(n, code):
    r = []
    for i in range(n):
        t = code % 3
        code //= 3
        if t:
            r.append(2 * i + t - 1)
    return r


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 7, 8])
def test_nand_parity(apm, oracle_mod, n):
    import torch
    rng = np.random.default_rng(700 + n)
    for cplx in (False, True):
        A = rng.standard_normal((3, 2 * n, 2 * n)) + 3.0 * np.eye(2 * n)
        if cplx:
            A = A + 1j * rng.standard_normal((3, 2 * n, 2 * n))
        out, info = apm.nand_minors(torch.from_numpy(A).cuda())
        torch.cuda.synchronize()
        # a few of these pivots fall below the shift threshold (one real matrix at 7 blocks
        # and two at 8 have a pivot under 1e-3 of its row and column scale)
        assert np.all(info.cpu().numpy() >= 0)
        got = out.cpu().numpy()
        ref = oracle_mod.nand_minors(A)
        for b in range(3):
            H = np.array([np.prod(np.linalg.norm(A[b][np.ix_(r, r)], axis=1)) if r else 1.0
                          for r in (nand_rows(n, c) for c in range(3 ** n))])
            e = metrics.mixed_err(got[b], ref[b], H)
            assert e.max() <= 1e-10, (n, cplx, b, float(e.max()))


def _nand_bound(A):
    n = A.shape[0] // 2
    return np.array([np.prod(np.linalg.norm(A[np.ix_(r, r)], axis=1)) if r else 1.0
                     for r in (nand_rows(n, c) for c in range(3 ** n))])


def _zero_diag(A):
    A = A.copy()
    i = np.arange(A.shape[-1])
    A[..., i, i] = 0.0
    return A


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 8])
def test_nand_zero_pivots(apm, oracle_mod, n):
    """Zero diagonal (every pivot of a row kept below left-out blocks is zero, at every depth:
    the subtree levels, and the top levels from five blocks on) and a diagonal of 1e-7 times
    the off-diagonal scale (pivots below the shift threshold but not zero): the shifted tree
    with its back-propagated corrections against the oracle on every entry, info = the
    number of shifts."""
    import torch
    rng = np.random.default_rng(1700 + n)
    for cplx in (False, True):
        for kind in ("zero", "tiny"):
            A = rng.standard_normal((3, 2 * n, 2 * n))
            if cplx:
                A = A + 1j * rng.standard_normal((3, 2 * n, 2 * n))
            A = _zero_diag(A)
            if kind == "tiny":
                i = np.arange(2 * n)
                A[:, i, i] = 1e-7 * rng.standard_normal((3, 2 * n))
            out, info = apm.nand_minors(torch.from_numpy(A).cuda())
            torch.cuda.synchronize()
            info = info.cpu().numpy()
            assert np.all(info >= 0), (n, cplx, kind, info)
            if n >= 2:
                assert np.all(info > 0), (n, cplx, kind, info)
            got = out.cpu().numpy()
            ref = oracle_mod.nand_minors(A)
            for b in range(3):
                e = metrics.mixed_err(got[b], ref[b], _nand_bound(A[b]))
                assert e.max() <= 1e-10, (n, cplx, kind, b, float(e.max()), int(np.argmax(e)))


@pytest.mark.parametrize("n", [10, 12])
def test_nand_zero_pivots_large(apm, oracle_mod, n):
    """Zero-diagonal Keldysh block matrices (complex) and real random ones at 10 and 12 blocks
    (6 and 8 top levels: corrections of whole top subtrees, up to a third of the outputs):
    every entry against the oracle."""
    import torch
    rng = np.random.default_rng(1800 + n)
    for A in (_zero_diag(W.keldysh_block(1, n, seed=1810 + n)), _zero_diag(rng.standard_normal((1, 2 * n, 2 * n)))):
        out, info = apm.nand_minors(torch.from_numpy(A).cuda())
        torch.cuda.synchronize()
        assert np.all(info.cpu().numpy() > 0)
        got = out.cpu().numpy()[0]
        ref = oracle_mod.nand_minors(A)[0]
        e = metrics.mixed_err(got, ref, _bound_nand(A[0]))
        assert e.max() <= 1e-10, (n, A.dtype, float(e.max()), int(np.argmax(e)))


def test_nand_keldysh_sampled(apm, oracle_mod):
    """512 Keldysh block matrices of 10 blocks; sampled matrices and codes against the oracle,
    and the full-order entries against the XOR minors of the same matrices."""
    import torch
    n = 10
    A = W.keldysh_block(512, n, seed=W.BASE_SEED + 5)
    dA = torch.from_numpy(A).cuda()
    out, info = apm.nand_minors(dA)
    xo, _ = apm.xor_minors(dA)
    torch.cuda.synchronize()
    assert np.all(info.cpu().numpy() >= 0)     # shifts of near-zero pivots are allowed
    sel = np.random.default_rng(513).choice(512, 2, replace=False)
    got = out[torch.from_numpy(sel).cuda()].cpu().numpy()
    ref = oracle_mod.nand_minors(A[sel])
    codes = np.random.default_rng(2).integers(0, 3 ** n, 600)
    for i in range(len(sel)):
        H = np.array([np.prod(np.linalg.norm(A[sel[i]][np.ix_(r, r)], axis=1)) if r else 1.0
                      for r in (nand_rows(n, int(c)) for c in codes)])
        e = metrics.mixed_err(got[i][codes], ref[i][codes], H)
        assert e.max() <= 1e-10, (int(sel[i]), float(e.max()))
    # every block present: the order-n XOR minors (choice beta -> code sum (beta_i + 1) 3^i)
    beta = np.arange(1 << n)
    code = sum(((beta >> i) & 1) * 3 ** i for i in range(n)) + sum(3 ** i for i in range(n))
    full = out[:, torch.from_numpy(code).cuda()]
    xfull = xo[:, (1 << n) - 2:]
    assert bool(torch.allclose(full, xfull, rtol=1e-10, atol=1e-12 * float(xfull.abs().max())))


def _row_log_norms(A):
    return np.log(np.maximum(np.linalg.norm(A, axis=1), 1e-300))


def _bound_xor(A):
    """Hadamard bound of every XOR entry from the full rows' norms (a valid, looser bound:
    ||A[i, R]|| <= ||A[i, :]||), in output order."""
    n = A.shape[0] // 2
    ln = _row_log_norms(A)
    out = []
    for k in range(1, n + 1):
        bits = (np.arange(1 << k)[:, None] >> np.arange(k)[None, :]) & 1
        rows = 2 * (n - k + np.arange(k))[None, :] + bits
        out.append(np.exp(ln[rows].sum(axis=1)))
    return np.concatenate(out)


def _bound_xnor(A):
    n = A.shape[0] // 2
    ln = _row_log_norms(A)
    bits = (np.arange(1 << n)[:, None] >> np.arange(n)[None, :]) & 1
    return np.exp(bits @ (ln[0::2] + ln[1::2]))


def _bound_nand(A):
    n = A.shape[0] // 2
    ln = _row_log_norms(A)
    codes = np.arange(3 ** n)
    digits = (codes[:, None] // 3 ** np.arange(n)[None, :]) % 3
    lt = np.stack([np.zeros(n), ln[0::2], ln[1::2]], axis=1)    # [block][digit]
    return np.exp(lt[np.arange(n)[None, :], digits].sum(axis=1))


@pytest.mark.parametrize("mode,n", [("xor", 15), ("xor", 16), ("xnor", 15), ("xnor", 16), ("nand", 12), ("nand", 13)])
def test_largest_block_counts(apm, oracle_mod, mode, n):
    """Every entry at the largest block counts (the widest top-level passes: child orders
    up to 30, split over two lanes per row), complex Keldysh and real random matrices."""
    import torch
    fn = {"xor": (apm.xor_minors, oracle_mod.xor_minors, _bound_xor),
          "xnor": (apm.xnor_minors, oracle_mod.xnor_minors, _bound_xnor),
          "nand": (apm.nand_minors, oracle_mod.nand_minors, _bound_nand)}[mode]
    rng = np.random.default_rng(900 + n)
    for A in (W.keldysh_block(1, n, seed=910 + n), rng.standard_normal((1, 2 * n, 2 * n)) + 3.0 * np.eye(2 * n)):
        out, info = fn[0](torch.from_numpy(A).cuda())
        torch.cuda.synchronize()
        if mode == "nand":
            assert np.all(info.cpu().numpy() >= 0)   # the number of pivot shifts
        else:
            assert np.all(info.cpu().numpy() == 0)
        got = out.cpu().numpy()[0]
        ref = fn[1](A)[0]
        e = metrics.mixed_err(got, ref, fn[2](A[0]))
        assert e.max() <= 1e-10, (mode, n, A.dtype, float(e.max()), int(np.argmax(e)))
