"""The C ABI library loads, exports every symbol include/apm.h declares, and rejects bad
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
    src = open(os.path.join(ROOT, "include", "apm.h")).read()
    return sorted(set(re.findall(r"^\s*(?:apm_status|const char|int)\s*\*?\s*(apm_\w+)\s*\(", src, re.M)))


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
