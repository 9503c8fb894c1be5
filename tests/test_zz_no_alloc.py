"""apm_all_minors_noalloc (the all-minors entry point whose scratch is a static device
array) against apm_all_minors through the C ABI: the same bits on two calls in a row, the
second with a smaller input, for a uniform batch with deferred top-level corrections and
for a mixed-order batch; and the batch limit."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def apm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2104_07638_amd as m
    return m


def _call(apm, fn, dt, A, bd, out, exp, info, tau=0.0):
    rc = fn(dt, apm._ptr(A), bd, apm._ptr(out), apm._ptr(exp), apm._ptr(info), apm.apm_opts(tau, 0),
            apm._stream(None))
    assert rc == 0, apm.status_name(rc) if hasattr(apm, "status_name") else rc


@pytest.mark.parametrize("dtype", ["r64", "r32s"])
def test_noalloc_uniform_matches(apm, dtype):
    import torch
    dt = apm.DTYPES[dtype]
    n = 16
    A = W.lattice_batch(640, n, W.Lattice(32, 1.0, -0.5, 5.0), seed=501)
    A, _ = W.inject_stress(A, every=16)                 # top-level shifts: the deferred queue is used
    A[::5] = W.zero_diagonal(A[::5])
    for B in (640, 200):                                # two calls in a row, the second smaller
        dA = torch.from_numpy(A[:B].copy()).cuda()
        ot = torch.float32 if dtype == "r32s" else torch.float64
        outs, exps, infos = [], [], []
        for fn in (apm.apm_all_minors, apm.apm_all_minors_noalloc):
            out = torch.full((B, 1 << n), 7.0, dtype=ot, device="cuda")
            exp = torch.zeros((B, 1 << n), dtype=torch.int16, device="cuda") if dtype == "r32s" else None
            info = torch.full((B,), -9, dtype=torch.int32, device="cuda")
            _call(apm, fn, dt, dA, apm.make_batch(B, n), out, exp, info)
            outs.append(out)
            exps.append(exp)
            infos.append(info)
        torch.cuda.synchronize()
        assert torch.equal(outs[0], outs[1])
        if dtype == "r32s":
            assert torch.equal(exps[0], exps[1])
        assert torch.equal(infos[0], infos[1])
        assert int((infos[1] > 0).sum()) > 0 and int(infos[1].min()) >= 0


def test_noalloc_ragged_matches(apm):
    import torch
    for B, seed in ((1500, 511), (300, 512)):           # the second call smaller
        mats, ns = W.lattice_ragged(B, 6, 16, W.Lattice(32, 1.0, -0.5, 5.0), seed=seed)
        flat = torch.from_numpy(np.concatenate([m.ravel() for m in mats])).cuda()
        n_t = torch.from_numpy(ns).cuda()
        tot = int(np.sum(np.left_shift(1, ns.astype(np.int64))))
        outs, infos = [], []
        for fn in (apm.apm_all_minors, apm.apm_all_minors_noalloc):
            out = torch.full((tot,), 7.0, dtype=torch.float64, device="cuda")
            info = torch.full((B,), -9, dtype=torch.int32, device="cuda")
            _call(apm, fn, apm.APM_R64, flat, apm.make_batch(B, 0, n_t, 16, None, None), out, None, info)
            outs.append(out)
            infos.append(info)
        torch.cuda.synchronize()
        assert torch.equal(outs[0], outs[1])
        assert torch.equal(infos[0], infos[1])
        assert int(infos[1].min()) >= 0


def test_noalloc_batch_limit(apm):
    import torch
    B = apm.APM_NOALLOC_MAX_BATCH + 1
    A = torch.zeros((B, 2, 2), dtype=torch.float64, device="cuda")
    out = torch.zeros((B, 4), dtype=torch.float64, device="cuda")
    rc = apm.apm_all_minors_noalloc(apm.APM_R64, apm._ptr(A), apm.make_batch(B, 2), apm._ptr(out), None, None,
                                    None, apm._stream(None))
    assert rc == apm.APM_EUNSUPPORTED
