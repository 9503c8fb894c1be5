"""The C ABI library loads, exports every symbol include/*.h declares, and rejects bad
arguments on the host before any device work (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def apm():
    import paper_2104_07638_amd as m
    return m


def _declared():
    names = set()
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            src = open(os.path.join(ROOT, "include", h)).read()
            names |= set(re.findall(r"^\s*(?:apm_status|const char|int|int32_t|int64_t|void)\s*\*?\s*(apm_\w+)\s*\(", src,
                                    re.M))
    return sorted(names)


def test_header_declarations_are_exported(apm):
    decl = _declared()
    assert set(decl) == set(apm.EXPORTS), decl
    lib = ctypes.CDLL(apm.LIB_PATH)
    for name in decl:
        assert hasattr(lib, name), name


def test_status_strings(apm):
    for s in range(5):
        assert apm.apm_status_str(s).startswith("APM_")
    assert apm.apm_version() >= 100


def _bd(apm, batch=4, n=8, **kw):
    return apm.apm_batch(batch, n, kw.get("nptr"), kw.get("n_max", 0), kw.get("ioff"), kw.get("ooff"))


P = ctypes.c_void_p(16)   # a non-null pointer that is never dereferenced by validation


def test_minors_validation(apm):
    f = apm.apm_all_minors
    assert f(0, None, _bd(apm, batch=0), None, None, None, None, None) == apm.APM_OK
    assert f(0, P, None, P, None, None, None, None) == apm.APM_EINVAL
    assert f(9, P, _bd(apm), P, None, None, None, None) == apm.APM_EINVAL
    assert f(-1, P, _bd(apm), P, None, None, None, None) == apm.APM_EINVAL
    assert f(0, None, _bd(apm), P, None, None, None, None) == apm.APM_EINVAL
    assert f(0, P, _bd(apm), None, None, None, None, None) == apm.APM_EINVAL
    assert f(0, P, _bd(apm, batch=-1), P, None, None, None, None) == apm.APM_EINVAL
    assert f(0, P, _bd(apm, n=21), P, None, None, None, None) == apm.APM_EUNSUPPORTED
    assert f(0, P, _bd(apm, n=0), P, None, None, None, None) == apm.APM_EINVAL   # ragged without n[]
    # scaled variants need exponents unless fp64 output is requested, others must not get them
    assert f(1, P, _bd(apm), P, None, None, None, None) == apm.APM_EINVAL
    assert f(0, P, _bd(apm), P, P, None, None, None) == apm.APM_EINVAL
    bad = apm.apm_opts(0.0, 1 << 7)
    assert f(0, P, _bd(apm), P, None, None, bad, None) == apm.APM_EINVAL
    nan = apm.apm_opts(float("nan"), 0)
    assert f(0, P, _bd(apm), P, None, None, nan, None) == apm.APM_EINVAL


def test_cs_and_perm_validation(apm):
    assert apm.apm_connected_sums(P, None, _bd(apm, batch=0), P, 0, None) == apm.APM_OK
    assert apm.apm_connected_sums(P, None, _bd(apm), P, 8, None) == apm.APM_EINVAL
    assert apm.apm_connected_sums(P, P, _bd(apm), P, apm.APM_CS_WEIGHTS, None) == apm.APM_EINVAL
    assert apm.apm_connected_sums(None, None, _bd(apm), P, 0, None) == apm.APM_EINVAL
    assert apm.apm_connected_sums(P, None, _bd(apm, n=21), P, 0, None) == apm.APM_EUNSUPPORTED
    assert apm.apm_all_perm_minors(P, _bd(apm, n=17), P, None) == apm.APM_EUNSUPPORTED
    assert apm.apm_all_perm_minors(None, _bd(apm), P, None) == apm.APM_EINVAL
    assert apm.apm_all_perm_minors(P, _bd(apm, batch=0), P, None) == apm.APM_OK


def _model(apm, n=10, L=16, n_tau=128, n_bin=16, eps=0.1, g0=16, resolve=0.0):
    return apm.apm_mc_model(n, L, n_tau, n_bin, eps, resolve, g0)


def test_mlp_sizes_and_validation(apm):
    assert apm.apm_mlp_param_count(27, 272) == 128 * 32 + 128 * 128 + 272 * 128 + 128 + 128 + 272
    assert apm.apm_mlp_weight_count(6, 8) == 128 * 16 + 128 * 128 + 16 * 128
    assert apm.apm_mlp_param_count(0, 8) == -1 and apm.apm_mlp_param_count(65, 8) == -1
    assert apm.apm_mlp_param_count(8, 4097) == -1
    assert apm.apm_mlp_work_bytes(27, 272, 33) == -1 and apm.apm_mlp_work_bytes(27, 272, 64) > 0
    net = apm.apm_mlp(27, 272, 16, 16, 16, 16, 16, 16)
    assert apm.apm_mlp_forward(net, P, 48, P, None, None) == apm.APM_EINVAL        # batch % 32
    assert apm.apm_mlp_forward(net, None, 32, P, None, None) == apm.APM_EINVAL
    assert apm.apm_mlp_forward(net, P, 0, P, None, None) == apm.APM_OK
    assert apm.apm_mlp_forward(None, P, 32, P, None, None) == apm.APM_EINVAL
    assert apm.apm_mlp_backward(net, P, 32, None, None) == apm.APM_EINVAL          # needs the forward work
    bad = apm.apm_mlp(0, 272, 16, 16, 16, 16, 16, 16)
    assert apm.apm_mlp_sync(bad, None) == apm.APM_EINVAL
    assert apm.apm_mlp_adam(net, apm.apm_adam(1e-3, 0.9, 0.999, 1e-8, 0), None) == apm.APM_EINVAL
    assert apm.apm_mlp_adam(net, apm.apm_adam(1e-3, 1.0, 0.999, 1e-8, 1), None) == apm.APM_EINVAL
    assert apm.apm_mlp_adam(net, None, None) == apm.APM_EINVAL


def test_mc_validation(apm):
    ch = apm.apm_mc_chain(64, 16, 16, 16)
    assert apm.apm_mc_work_bytes(_model(apm, g0=0), 64, 1) > 0                      # sizing needs no table
    assert apm.apm_mc_work_bytes(_model(apm), 33, 1) == -1
    assert apm.apm_mc_work_bytes(_model(apm, n=1), 64, 0) == -1
    f = apm.apm_mc_step
    assert f(_model(apm, n=17), ch, None, None, 1, 0, None, P, None) == apm.APM_EUNSUPPORTED
    assert f(_model(apm, n=1), ch, None, None, 1, 0, None, P, None) == apm.APM_EINVAL
    assert f(_model(apm, n_tau=100, n_bin=16), ch, None, None, 1, 0, None, P, None) == apm.APM_EINVAL
    assert f(_model(apm, n_bin=65, n_tau=130), ch, None, None, 1, 0, None, P, None) == apm.APM_EINVAL
    assert f(_model(apm, eps=1.5), ch, None, None, 1, 0, None, P, None) == apm.APM_EINVAL
    assert f(_model(apm, L=257), ch, None, None, 1, 0, None, P, None) == apm.APM_EINVAL
    assert f(_model(apm, g0=0), ch, None, None, 1, 0, None, P, None) == apm.APM_EINVAL
    assert f(_model(apm, resolve=-1.0), ch, None, None, 1, 0, None, P, None) == apm.APM_EINVAL
    assert f(_model(apm, resolve=float("nan")), ch, None, None, 1, 0, None, P, None) == apm.APM_EINVAL
    assert f(_model(apm), ch, None, None, 1, 0, None, None, None) == apm.APM_EINVAL    # no work buffer
    assert f(_model(apm), apm.apm_mc_chain(64, None, 16, 16), None, None, 1, 0, None, P, None) == apm.APM_EINVAL
    net = apm.apm_mlp(27, 272, 16, 16, 16, 16, 16, 16)
    wrong = apm.apm_mlp(26, 272, 16, 16, 16, 16, 16, 16)
    assert f(_model(apm), ch, wrong, None, 1, 0, None, P, None) == apm.APM_EINVAL     # sizes do not match n, L
    assert f(_model(apm), apm.apm_mc_chain(48, 16, 16, 16), net, None, 1, 0, None, P, None) == apm.APM_EINVAL
    adam = apm.apm_adam(1e-3, 0.9, 0.999, 1e-8, 1)
    assert f(_model(apm), ch, None, adam, 1, 0, None, P, None) == apm.APM_EINVAL      # training needs a net
    assert f(_model(apm), apm.apm_mc_chain(0, None, None, None), None, None, 1, 0, None, None, None) == apm.APM_OK
    assert apm.apm_mc_propose(_model(apm), ch, 1, 0, P, P, 100, P, P, P, None) == apm.APM_EINVAL  # short stride
    assert apm.apm_mc_context(_model(apm), ch, 1, 0, None, None, None) == apm.APM_EINVAL
    assert apm.apm_mc_accept(_model(apm), ch, 1, 0, P, P, P, P, None, None, None) == apm.APM_EINVAL
    assert apm.apm_mc_evaluate(_model(apm), ch, None, None) == apm.APM_EINVAL


def test_autotune_validation(apm):
    assert apm.apm_autotune_minors(0, 0, 16, None, None) == apm.APM_EINVAL
    assert apm.apm_autotune_minors(0, 21, 16, None, None) == apm.APM_EINVAL
    assert apm.apm_autotune_minors(4, 10, 16, None, None) == apm.APM_EINVAL
    assert apm.apm_autotune_minors(0, 10, 0, None, None) == apm.APM_EINVAL
    assert apm.apm_minors_k0(0, 16) in (3, 4, 5) and apm.apm_minors_k0(2, 14) in (2, 3)
    assert apm.apm_minors_k0(0, 0) == -1 and apm.apm_minors_k0(5, 8) == -1


def _plan(apm, **kw):
    d = apm.apm_plan_desc(**kw)
    h = ctypes.c_void_p()
    rc = apm.apm_plan_create(d, ctypes.byref(h))
    if rc != apm.APM_OK:
        assert not h.value       # no plan handed out on failure
    return rc, h


def test_plan_validation(apm):
    K = apm
    h = ctypes.c_void_p()
    assert apm.apm_plan_create(None, ctypes.byref(h)) == apm.APM_EINVAL
    assert apm._lib.apm_plan_create(ctypes.byref(apm.apm_plan_desc()), None) == apm.APM_EINVAL
    assert apm.apm_plan_launch(None, None) == apm.APM_EINVAL
    assert apm.apm_plan_k0(None) == -1 and apm.apm_plan_graphed(None) == -1
    apm.apm_plan_destroy(None)
    bd = _bd(apm)
    assert _plan(apm, kind=9, batch=bd, A=P, minors=P)[0] == K.APM_EINVAL
    assert _plan(apm, kind=K.APM_PLAN_MINORS, batch=bd, A=P, minors=P, flags=8)[0] == K.APM_EINVAL
    # the checks of the direct call apply
    assert _plan(apm, kind=K.APM_PLAN_MINORS, batch=bd, A=None, minors=P)[0] == K.APM_EINVAL
    assert _plan(apm, kind=K.APM_PLAN_MINORS, batch=_bd(apm, n=21), A=P, minors=P)[0] == K.APM_EUNSUPPORTED
    assert _plan(apm, kind=K.APM_PLAN_MINORS, dtype=1, batch=bd, A=P, minors=P)[0] == K.APM_EINVAL
    assert _plan(apm, kind=K.APM_PLAN_PERM_MINORS, batch=_bd(apm, n=17), A=P, perm=P)[0] == K.APM_EUNSUPPORTED
    assert _plan(apm, kind=K.APM_PLAN_CONNECTED_SUMS, batch=bd, m_up=P, c=P)[0] == K.APM_EINVAL   # aliasing
    assert _plan(apm, kind=K.APM_PLAN_CONNECTED_SUMS, batch=_bd(apm, ioff=P), m_up=P,
                 c=ctypes.c_void_p(32))[0] == K.APM_EINVAL                                      # two offsets
    # fields another kind uses must be empty
    assert _plan(apm, kind=K.APM_PLAN_MINORS, batch=bd, A=P, minors=P, c=P)[0] == K.APM_EINVAL
    assert _plan(apm, kind=K.APM_PLAN_PERM_MINORS, batch=bd, A=P, perm=P, minors=P)[0] == K.APM_EINVAL
    assert _plan(apm, kind=K.APM_PLAN_CONNECTED_SUMS, batch=bd, m_up=P, c=ctypes.c_void_p(32),
                 A=P)[0] == K.APM_EINVAL
    # CDet: fp64 minors only (r64, or r32s with fp64 output), consistent second set, no aliasing
    q, r, t = ctypes.c_void_p(32), ctypes.c_void_p(48), ctypes.c_void_p(64)
    assert _plan(apm, kind=K.APM_PLAN_CDET, dtype=2, batch=bd, A=P, minors=q, c=r)[0] == K.APM_EINVAL
    assert _plan(apm, kind=K.APM_PLAN_CDET, dtype=1, batch=bd, A=P, minors=q, c=r)[0] == K.APM_EINVAL
    assert _plan(apm, kind=K.APM_PLAN_CDET, batch=bd, A=P, A_dn=P, minors=q, c=r)[0] == K.APM_EINVAL
    assert _plan(apm, kind=K.APM_PLAN_CDET, batch=bd, A=P, minors=q, minors_dn=t, c=r)[0] == K.APM_EINVAL
    assert _plan(apm, kind=K.APM_PLAN_CDET, batch=bd, A=P, minors=q, c=q)[0] == K.APM_EINVAL
    assert _plan(apm, kind=K.APM_PLAN_CDET, batch=bd, A=P, A_dn=P, minors=q, minors_dn=q, c=r)[0] == K.APM_EINVAL
    assert _plan(apm, kind=K.APM_PLAN_CDET, batch=bd, A=P, minors=q, c=r, cs_mode=2)[0] == K.APM_EINVAL
    assert _plan(apm, kind=K.APM_PLAN_CDET, batch=bd, A=P, minors=q, c=r, info_dn=t)[0] == K.APM_EINVAL
    # an empty batch gives a plan whose launches enqueue nothing (no device needed)
    rc, h = _plan(apm, kind=K.APM_PLAN_CDET, batch=_bd(apm, batch=0), A=P, minors=q, c=r)
    assert rc == K.APM_OK and h.value
    assert apm.apm_plan_launch(h, None) == K.APM_OK
    assert apm.apm_plan_k0(h) == 0 and apm.apm_plan_graphed(h) == 0
    apm.apm_plan_destroy(h)


def test_device_error_record(apm):
    import torch
    if torch.cuda.is_available():
        pytest.skip("needs a host without a GPU to force a HIP failure")
    apm.apm_last_device_error()                       # clear
    assert apm.apm_last_device_error() == apm.APM_OK
    rc, h = _plan(apm, kind=apm.APM_PLAN_MINORS, batch=_bd(apm), A=P, minors=ctypes.c_void_p(32))
    assert rc == apm.APM_EDEVICE                      # no device: the plan cannot be made
    assert apm.apm_last_device_error() == apm.APM_EDEVICE
    assert apm.apm_last_device_error() == apm.APM_OK  # cleared by the read
    assert apm.apm_last_hip_error() != 0              # the HIP code stays


def test_xor_validation(apm):
    f = apm.apm_xor_minors
    assert f(2, P, _bd(apm, batch=0), P, None, None) == apm.APM_OK
    assert f(9, P, _bd(apm), P, None, None) == apm.APM_EINVAL
    assert f(1, P, _bd(apm), P, None, None) == apm.APM_EUNSUPPORTED          # r32s: not built
    assert f(3, P, _bd(apm), P, None, None) == apm.APM_EUNSUPPORTED          # c64s: not built
    assert f(2, P, _bd(apm, n=17), P, None, None) == apm.APM_EUNSUPPORTED
    assert f(2, P, _bd(apm, n=0, nptr=P), P, None, None) == apm.APM_EUNSUPPORTED   # mixed orders
    assert f(2, P, _bd(apm, ioff=P), P, None, None) == apm.APM_EUNSUPPORTED
    assert f(2, None, _bd(apm), P, None, None) == apm.APM_EINVAL
    assert f(2, P, _bd(apm), None, None, None) == apm.APM_EINVAL
    assert f(2, P, None, P, None, None) == apm.APM_EINVAL


def test_xnor_validation(apm):
    f = apm.apm_xnor_minors
    assert f(0, P, _bd(apm, batch=0), P, None, None) == apm.APM_OK
    assert f(7, P, _bd(apm), P, None, None) == apm.APM_EINVAL
    assert f(1, P, _bd(apm), P, None, None) == apm.APM_EUNSUPPORTED
    assert f(0, P, _bd(apm, n=17), P, None, None) == apm.APM_EUNSUPPORTED
    assert f(0, P, _bd(apm, ooff=P), P, None, None) == apm.APM_EUNSUPPORTED
    assert f(0, P, _bd(apm), None, None, None) == apm.APM_EINVAL


def test_leading_validation(apm):
    f = apm.apm_leading_minors
    assert f(0, P, _bd(apm, batch=0), P, None, None) == apm.APM_OK
    assert f(5, P, _bd(apm), P, None, None) == apm.APM_EINVAL
    assert f(3, P, _bd(apm), P, None, None) == apm.APM_EUNSUPPORTED
    assert f(0, P, _bd(apm, n=33), P, None, None) == apm.APM_EUNSUPPORTED
    assert f(0, None, _bd(apm), P, None, None) == apm.APM_EINVAL


def test_nand_validation(apm):
    f = apm.apm_nand_minors
    assert f(2, P, _bd(apm, batch=0), P, None, None) == apm.APM_OK
    assert f(2, P, _bd(apm, n=14), P, None, None) == apm.APM_EUNSUPPORTED
    assert f(1, P, _bd(apm), P, None, None) == apm.APM_EUNSUPPORTED
    assert f(2, None, _bd(apm), P, None, None) == apm.APM_EINVAL
