"""GPU parity of the leading principal minors (Sec. III) with the oracle: every order up to
32, real and complex, the 8192 x n=16 lattice batch on sampled matrices, and the error
codes (non-finite input, a zero pivot of the elimination without row exchanges)."""
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


def lead_hadamard(A):
    n = A.shape[0]
    return np.array([np.prod(np.linalg.norm(A[:k, :k], axis=1)) for k in range(1, n + 1)])


@pytest.mark.parametrize("n", [1, 2, 3, 7, 16, 20, 31, 32])
def test_orders(apm, oracle_mod, n):
    import torch
    rng = np.random.default_rng(600 + n)
    for cplx in (False, True):
        A = rng.standard_normal((8, n, n)) + 2.0 * np.eye(n)
        if cplx:
            A = A + 1j * rng.standard_normal((8, n, n))
        out, info = apm.leading_minors(torch.from_numpy(A).cuda())
        torch.cuda.synchronize()
        assert np.all(info.cpu().numpy() == 0)
        got = out.cpu().numpy()
        ref = oracle_mod.leading_minors(A)
        for b in range(8):
            e = metrics.mixed_err(got[b], ref[b], lead_hadamard(A[b]))
            assert e.max() <= 1e-10, (n, cplx, b, float(e.max()))


def test_lattice_batch_sampled(apm, oracle_mod):
    import torch
    A = W.lattice_batch(8192, 16, W.Lattice(32, 1.0, -0.5, 5.0), seed=W.BASE_SEED + 2)
    out, info = apm.leading_minors(torch.from_numpy(A).cuda())
    torch.cuda.synchronize()
    assert np.all(info.cpu().numpy() == 0)
    sel = np.random.default_rng(8193).choice(8192, 64, replace=False)
    got = out.cpu().numpy()[sel]
    ref = oracle_mod.leading_minors(A[sel])
    for i, b in enumerate(sel):
        e = metrics.mixed_err(got[i], ref[i], lead_hadamard(A[b]))
        assert e.max() <= 1e-10, (int(b), float(e.max()))


def test_error_codes(apm):
    import torch
    A = np.tile(np.eye(6) * 2.0, (3, 1, 1))
    A[1, 2, 4] = np.inf
    A[2, 0, 0] = 0.0                 # zero first pivot
    out, info = apm.leading_minors(torch.from_numpy(A).cuda())
    torch.cuda.synchronize()
    assert list(info.cpu().numpy()) == [0, -2, -3]
    np.testing.assert_array_equal(out[0].cpu().numpy(), 2.0 ** np.arange(1, 7))
    assert bool(torch.all(torch.isnan(out[1])))
