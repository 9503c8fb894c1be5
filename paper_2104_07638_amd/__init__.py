"""Python binding of libapm.so: all principal minors, CDet connected sums and permanent
principal minors of batches of small matrices on AMD MI355X (gfx950).

Operations (Simkovic & Ferrero, arXiv:2104.07638):

* ``apm_all_minors`` / ``all_minors``         -- Sec. II: det(A[S]) for all 2^n subsets S
  by the Schur-complement binary tree with pivot shifts and their back-propagation.
* ``apm_connected_sums`` / ``connected_sums`` -- Sec. V.A, Eq. (recursion).
* ``apm_all_perm_minors`` / ``all_perm_minors`` -- Sec. IV, O(3^n) permanent minors.

The ``apm_*`` functions mirror the C ABI of ``include/apm.h`` one to one and take raw
device pointers; the lower-case wrappers marshal torch tensors (device memory and the
current HIP stream).  Every step runs in the HIP kernels of libapm.so; there is no
CPU path.  Importing this module without the built library raises ImportError.
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (loads the HIP runtime that libapm.so binds to)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libapm.so")

APM_OK, APM_EINVAL, APM_EUNSUPPORTED, APM_EDEVICE, APM_ENOMEM = 0, 1, 2, 3, 4
APM_R64, APM_R32S, APM_C128, APM_C64S = 0, 1, 2, 3
APM_MAX_N, APM_MAX_N_CS, APM_MAX_N_PERM = 20, 20, 16
APM_OUT_F64, APM_NO_PERTURB = 1, 2
APM_CS_ROOTED, APM_CS_ALL, APM_CS_WEIGHTS = 0, 1, 2

DTYPES = {"r64": APM_R64, "r32s": APM_R32S, "c128": APM_C128, "c64s": APM_C64S}

#: names exported by include/apm.h (checked by the tests)
EXPORTS = ("apm_all_minors", "apm_connected_sums", "apm_all_perm_minors", "apm_status_str",
           "apm_last_hip_error", "apm_version")


class apm_batch(ctypes.Structure):
    _fields_ = [("batch", ctypes.c_int32), ("n_uniform", ctypes.c_int32), ("n", ctypes.c_void_p),
                ("n_max", ctypes.c_int32), ("in_off", ctypes.c_void_p), ("out_off", ctypes.c_void_p)]


class apm_opts(ctypes.Structure):
    _fields_ = [("piv_tol", ctypes.c_double), ("flags", ctypes.c_uint32)]


class ApmError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = _lib.apm_status_str(status).decode() if _lib is not None else str(status)
        super().__init__(f"{where}: {msg}")


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libapm.so is not built ({LIB_PATH}); run __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    lib.apm_all_minors.argtypes = [ctypes.c_int, vp, ctypes.POINTER(apm_batch), vp, vp, vp,
                                   ctypes.POINTER(apm_opts), vp]
    lib.apm_all_minors.restype = ctypes.c_int
    lib.apm_connected_sums.argtypes = [vp, vp, ctypes.POINTER(apm_batch), vp, ctypes.c_uint32, vp]
    lib.apm_connected_sums.restype = ctypes.c_int
    lib.apm_all_perm_minors.argtypes = [vp, ctypes.POINTER(apm_batch), vp, vp]
    lib.apm_all_perm_minors.restype = ctypes.c_int
    lib.apm_status_str.argtypes = [ctypes.c_int]
    lib.apm_status_str.restype = ctypes.c_char_p
    lib.apm_last_hip_error.restype = ctypes.c_int
    lib.apm_version.restype = ctypes.c_int
    return lib


_lib = _load()


# ----------------------------------------------------------------- raw C-ABI mirrors
def apm_all_minors(dt, A, bd, minors, exp, info, opt, stream):
    return _lib.apm_all_minors(int(dt), A, ctypes.byref(bd) if bd is not None else None, minors, exp, info,
                               ctypes.byref(opt) if opt is not None else None, stream)


def apm_connected_sums(m_up, m_dn, bd, c, mode, stream):
    return _lib.apm_connected_sums(m_up, m_dn, ctypes.byref(bd) if bd is not None else None, c, int(mode),
                                   stream)


def apm_all_perm_minors(A, bd, perm, stream):
    return _lib.apm_all_perm_minors(A, ctypes.byref(bd) if bd is not None else None, perm, stream)


def apm_status_str(s):
    return _lib.apm_status_str(int(s)).decode()


def apm_last_hip_error():
    return _lib.apm_last_hip_error()


def apm_version():
    return _lib.apm_version()


# ----------------------------------------------------------------- torch wrappers
def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _check(rc, where):
    if rc != APM_OK:
        raise ApmError(rc, where)


def make_batch(batch, n_uniform=0, n=None, n_max=0, in_off=None, out_off=None):
    """Build an apm_batch from sizes and optional device tensors (int32 n, int64 offsets)."""
    return apm_batch(int(batch), int(n_uniform), _ptr(n), int(n_max), _ptr(in_off), _ptr(out_off))


def all_minors(A, dtype="r64", *, out=None, exp=None, info=None, out_f64=False, tau=0.0, perturb=True,
               stream=None):
    """All principal minors of a (B, n, n) device tensor.

    Returns (minors, exp, info).  ``minors`` is (B, 2**n): float64 (r64), complex128
    (c128), or for r32s / c64s float32 / complex64 mantissas with int16 exponents in
    ``exp`` (value = m * 2**exp); with ``out_f64`` the scaled variants return
    float64 / complex128 values and ``exp`` is None."""
    dt = DTYPES[dtype]
    if A.dim() != 3 or A.shape[1] != A.shape[2]:
        raise ValueError("A must be (B, n, n)")
    B, n = A.shape[0], A.shape[1]
    cplx = dt in (APM_C128, APM_C64S)
    want = torch.complex128 if cplx else torch.float64
    if A.dtype != want or not A.is_cuda or not A.is_contiguous():
        raise TypeError(f"A must be a contiguous {want} CUDA tensor")
    scaled = dt in (APM_R32S, APM_C64S)
    dev = A.device
    if out is None:
        if scaled and not out_f64:
            otype = torch.complex64 if cplx else torch.float32
        else:
            otype = torch.complex128 if cplx else torch.float64
        out = torch.empty((B, 1 << n), dtype=otype, device=dev)
    if scaled and not out_f64 and exp is None:
        exp = torch.empty((B, 1 << n), dtype=torch.int16, device=dev)
    if not (scaled and not out_f64):
        exp = None
    if info is None:
        info = torch.empty(B, dtype=torch.int32, device=dev)
    bd = make_batch(B, n)
    flags = (APM_OUT_F64 if out_f64 else 0) | (0 if perturb else APM_NO_PERTURB)
    opt = apm_opts(float(tau), flags)
    _check(apm_all_minors(dt, _ptr(A), bd, _ptr(out), _ptr(exp), _ptr(info), opt, _stream(stream)),
           "apm_all_minors")
    return out, exp, info


def all_minors_ragged(A_flat, n, n_max=0, dtype="r64", *, in_off=None, out_off=None, out=None, exp=None,
                      info=None, out_f64=False, tau=0.0, perturb=True, stream=None):
    """Ragged batch: matrices of orders n[b] (device int32) packed in ``A_flat``
    (default offsets: prefix sums of n_b^2 and 2^n_b, computed on the device)."""
    dt = DTYPES[dtype]
    B = n.numel()
    if in_off is None:
        sz = n.to(torch.int64) ** 2
        in_off = torch.cumsum(sz, 0) - sz
    if out_off is None:
        sz = torch.ones_like(n, dtype=torch.int64) << n.to(torch.int64)
        out_off = torch.cumsum(sz, 0) - sz
    if out is None:
        raise ValueError("ragged batches need a preallocated output")
    if info is None:
        info = torch.empty(B, dtype=torch.int32, device=A_flat.device)
    bd = make_batch(B, 0, n, n_max, in_off, out_off)
    flags = (APM_OUT_F64 if out_f64 else 0) | (0 if perturb else APM_NO_PERTURB)
    opt = apm_opts(float(tau), flags)
    _check(apm_all_minors(dt, _ptr(A_flat), bd, _ptr(out), _ptr(exp), _ptr(info), opt, _stream(stream)),
           "apm_all_minors")
    return out, exp, info


def connected_sums(m_up, m_dn=None, *, mode=APM_CS_ROOTED, weights=False, out=None, stream=None):
    """CDet connected sums of a (B, 2**n) float64 tensor of minors (or weights)."""
    B, nm = m_up.shape
    n = nm.bit_length() - 1
    if out is None:
        out = torch.empty_like(m_up)
    bd = make_batch(B, n)
    md = mode | (APM_CS_WEIGHTS if weights else 0)
    _check(apm_connected_sums(_ptr(m_up), _ptr(m_dn), bd, _ptr(out), md, _stream(stream)),
           "apm_connected_sums")
    return out


def all_perm_minors(A, *, out=None, stream=None):
    """All permanent principal minors of a (B, n, n) float64 tensor."""
    B, n = A.shape[0], A.shape[1]
    if out is None:
        out = torch.empty((B, 1 << n), dtype=torch.float64, device=A.device)
    bd = make_batch(B, n)
    _check(apm_all_perm_minors(_ptr(A), bd, _ptr(out), _stream(stream)), "apm_all_perm_minors")
    return out


def decode_scaled(m, e):
    """value = m * 2**e for the scaled outputs (host-side helper for callers)."""
    if torch.is_complex(m):
        s = torch.ldexp(torch.ones_like(e, dtype=torch.float64), e.to(torch.float64))
        return m.to(torch.complex128) * s
    return torch.ldexp(m.to(torch.float64), e.to(torch.float64))
