"""Python binding of libapm.so: all principal minors, CDet connected sums and permanent
principal minors of batches of small matrices on AMD MI355X (gfx950).

Operations (Simkovic & Ferrero, arXiv:2104.07638):

* ``apm_all_minors`` / ``all_minors``         -- Sec. II: det(A[S]) for all 2^n subsets S
  by the Schur-complement binary tree with pivot shifts and their back-propagation.
* ``apm_connected_sums`` / ``connected_sums`` -- Sec. V.A, Eq. (recursion).
* ``apm_all_perm_minors`` / ``all_perm_minors`` -- Sec. IV, O(3^n) permanent minors.
* ``apm_xor_minors`` / ``xor_minors``         -- Sec. III (XOR case), Sec. V.C: the
  determinants of every Keldysh index assignment of a 2n x 2n block matrix.
* ``apm_xnor_minors`` / ``xnor_minors``       -- Sec. III (XNOR case): whole-block minors.
* ``apm_leading_minors`` / ``leading_minors`` -- Sec. III: the n leading principal minors.
* ``apm_nand_minors`` / ``nand_minors``       -- Sec. III (NAND case): at most one row per block.
* ``apm_mc_*`` / ``apm_mlp_*`` (``include/apm_mc.h``) -- Metropolis-Hastings steps over
  vertex configurations weighted by |c[V]| (Sec. V.A), with a learned proposal network
  trained by the library's own forward/backward/Adam kernels (``Mlp``, ``mc_step``).

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
APM_MAX_N, APM_MAX_N_CS, APM_MAX_N_PERM, APM_MAX_N_XOR, APM_MAX_N_LEAD, APM_MAX_N_NAND = 20, 20, 16, 16, 32, 13
APM_OUT_F64, APM_NO_PERTURB = 1, 2
APM_CS_ROOTED, APM_CS_ALL, APM_CS_WEIGHTS = 0, 1, 2
APM_PLAN_MINORS, APM_PLAN_CONNECTED_SUMS, APM_PLAN_PERM_MINORS, APM_PLAN_CDET = 0, 1, 2, 3
APM_PLAN_AUTOTUNE, APM_PLAN_EAGER = 1, 2
APM_NOALLOC_MAX_BATCH = 16384

DTYPES = {"r64": APM_R64, "r32s": APM_R32S, "c128": APM_C128, "c64s": APM_C64S}

#: names exported by include/apm.h (checked by the tests)
EXPORTS = ("apm_all_minors", "apm_connected_sums", "apm_all_perm_minors", "apm_status_str",
           "apm_last_hip_error", "apm_version",
           "apm_mlp_param_count", "apm_mlp_weight_count", "apm_mlp_work_bytes", "apm_mlp_sync",
           "apm_mlp_forward", "apm_mlp_backward", "apm_mlp_adam", "apm_mc_work_bytes", "apm_mc_evaluate",
           "apm_mc_step", "apm_mc_context", "apm_mc_propose", "apm_mc_accept", "apm_autotune_minors",
           "apm_minors_k0", "apm_plan_create", "apm_plan_launch", "apm_plan_k0", "apm_plan_graphed",
           "apm_plan_destroy", "apm_last_device_error", "apm_xor_minors", "apm_xnor_minors",
           "apm_leading_minors", "apm_nand_minors", "apm_all_minors_noalloc", "apm_probe_fma64", "apm_probe_copy", "apm_tune_cache_load",
           "apm_autotune_minors_mixed", "apm_minors_k0_mixed")

APM_MLP_HIDDEN, APM_MLP_MAX_IN, APM_MLP_MAX_OUT, APM_MC_MAX_N = 128, 64, 4096, 16


class apm_batch(ctypes.Structure):
    _fields_ = [("batch", ctypes.c_int32), ("n_uniform", ctypes.c_int32), ("n", ctypes.c_void_p),
                ("n_max", ctypes.c_int32), ("in_off", ctypes.c_void_p), ("out_off", ctypes.c_void_p)]


class apm_opts(ctypes.Structure):
    _fields_ = [("piv_tol", ctypes.c_double), ("flags", ctypes.c_uint32)]


class apm_plan_desc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("dtype", ctypes.c_int), ("batch", apm_batch), ("A", ctypes.c_void_p),
                ("A_dn", ctypes.c_void_p), ("minors", ctypes.c_void_p), ("minors_dn", ctypes.c_void_p),
                ("exp", ctypes.c_void_p), ("info", ctypes.c_void_p), ("info_dn", ctypes.c_void_p),
                ("m_up", ctypes.c_void_p), ("m_dn", ctypes.c_void_p), ("c", ctypes.c_void_p),
                ("perm", ctypes.c_void_p), ("cs_mode", ctypes.c_uint32), ("opts", apm_opts),
                ("flags", ctypes.c_uint32)]


class apm_mlp(ctypes.Structure):
    _fields_ = [("d_in", ctypes.c_int32), ("d_out", ctypes.c_int32), ("param", ctypes.c_void_p),
                ("grad", ctypes.c_void_p), ("adam_m", ctypes.c_void_p), ("adam_v", ctypes.c_void_p),
                ("w", ctypes.c_void_p), ("wt", ctypes.c_void_p)]


class apm_adam(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float), ("t", ctypes.c_int32)]


class apm_mc_model(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("L", ctypes.c_int32), ("n_tau", ctypes.c_int32), ("n_bin", ctypes.c_int32),
                ("eps", ctypes.c_double), ("resolve", ctypes.c_double), ("g0", ctypes.c_void_p)]


class apm_mc_chain(ctypes.Structure):
    _fields_ = [("walkers", ctypes.c_int32), ("state", ctypes.c_void_p), ("logw", ctypes.c_void_p),
                ("sign", ctypes.c_void_p)]


class apm_mc_record(ctypes.Structure):
    _fields_ = [("moved", ctypes.c_void_p), ("proposed", ctypes.c_void_p), ("logq", ctypes.c_void_p),
                ("logc_prop", ctypes.c_void_p), ("accepted", ctypes.c_void_p), ("obs_logw", ctypes.c_void_p),
                ("obs_sign", ctypes.c_void_p), ("loss", ctypes.c_void_p)]


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
    lib.apm_probe_fma64.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64), vp]
    lib.apm_probe_fma64.restype = ctypes.c_int
    lib.apm_tune_cache_load.argtypes = [ctypes.c_char_p]
    lib.apm_tune_cache_load.restype = ctypes.c_int32
    lib.apm_probe_copy.argtypes = [vp, vp, ctypes.c_int64, ctypes.c_int32, vp]
    lib.apm_probe_copy.restype = ctypes.c_int
    lib.apm_all_minors_noalloc.argtypes = lib.apm_all_minors.argtypes
    lib.apm_all_minors_noalloc.restype = ctypes.c_int
    for name in ("apm_xor_minors", "apm_xnor_minors", "apm_leading_minors", "apm_nand_minors"):
        getattr(lib, name).argtypes = [ctypes.c_int, vp, ctypes.POINTER(apm_batch), vp, vp, vp]
        getattr(lib, name).restype = ctypes.c_int
    lib.apm_status_str.argtypes = [ctypes.c_int]
    lib.apm_status_str.restype = ctypes.c_char_p
    lib.apm_last_hip_error.restype = ctypes.c_int
    lib.apm_version.restype = ctypes.c_int
    i32, i64, u64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
    lib.apm_autotune_minors.argtypes = [ctypes.c_int, i32, i32, ctypes.POINTER(i32), vp]
    lib.apm_autotune_minors.restype = ctypes.c_int
    lib.apm_minors_k0.argtypes = [ctypes.c_int, i32]
    lib.apm_minors_k0.restype = i32
    lib.apm_autotune_minors_mixed.argtypes = [ctypes.c_int, i32, ctypes.POINTER(i32), ctypes.POINTER(i32), vp]
    lib.apm_autotune_minors_mixed.restype = ctypes.c_int
    lib.apm_minors_k0_mixed.argtypes = [ctypes.c_int, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    lib.apm_minors_k0_mixed.restype = None
    lib.apm_plan_create.argtypes = [ctypes.POINTER(apm_plan_desc), ctypes.POINTER(vp)]
    lib.apm_plan_create.restype = ctypes.c_int
    lib.apm_plan_launch.argtypes = [vp, vp]
    lib.apm_plan_launch.restype = ctypes.c_int
    lib.apm_plan_k0.argtypes = [vp]
    lib.apm_plan_k0.restype = i32
    lib.apm_plan_graphed.argtypes = [vp]
    lib.apm_plan_graphed.restype = i32
    lib.apm_plan_destroy.argtypes = [vp]
    lib.apm_plan_destroy.restype = None
    lib.apm_last_device_error.restype = ctypes.c_int
    P = ctypes.POINTER
    for name in ("apm_mlp_param_count", "apm_mlp_weight_count"):
        getattr(lib, name).argtypes = [i32, i32]
        getattr(lib, name).restype = i64
    lib.apm_mlp_work_bytes.argtypes = [i32, i32, i32]
    lib.apm_mlp_work_bytes.restype = i64
    lib.apm_mlp_sync.argtypes = [P(apm_mlp), vp]
    lib.apm_mlp_forward.argtypes = [P(apm_mlp), vp, i32, vp, vp, vp]
    lib.apm_mlp_backward.argtypes = [P(apm_mlp), vp, i32, vp, vp]
    lib.apm_mlp_adam.argtypes = [P(apm_mlp), P(apm_adam), vp]
    lib.apm_mc_work_bytes.argtypes = [P(apm_mc_model), i32, i32]
    lib.apm_mc_work_bytes.restype = i64
    lib.apm_mc_evaluate.argtypes = [P(apm_mc_model), P(apm_mc_chain), vp, vp]
    lib.apm_mc_step.argtypes = [P(apm_mc_model), P(apm_mc_chain), P(apm_mlp), P(apm_adam), u64, i32,
                                P(apm_mc_record), vp, vp]
    lib.apm_mc_context.argtypes = [P(apm_mc_model), P(apm_mc_chain), u64, i32, vp, vp, vp]
    lib.apm_mc_propose.argtypes = [P(apm_mc_model), P(apm_mc_chain), u64, i32, vp, vp, i32, vp, vp, vp, vp]
    lib.apm_mc_accept.argtypes = [P(apm_mc_model), P(apm_mc_chain), u64, i32, vp, vp, vp, vp, P(apm_mc_record),
                                  vp, vp]
    for name in ("apm_mlp_sync", "apm_mlp_forward", "apm_mlp_backward", "apm_mlp_adam", "apm_mc_evaluate",
                 "apm_mc_step", "apm_mc_context", "apm_mc_propose", "apm_mc_accept", "apm_autotune_minors",
           "apm_minors_k0"):
        getattr(lib, name).restype = ctypes.c_int
    return lib


_lib = _load()


# ----------------------------------------------------------------- raw C-ABI mirrors
def apm_all_minors(dt, A, bd, minors, exp, info, opt, stream):
    return _lib.apm_all_minors(int(dt), A, ctypes.byref(bd) if bd is not None else None, minors, exp, info,
                               ctypes.byref(opt) if opt is not None else None, stream)


def apm_all_minors_noalloc(dt, A, bd, minors, exp, info, opt, stream):
    return _lib.apm_all_minors_noalloc(int(dt), A, ctypes.byref(bd) if bd is not None else None, minors, exp,
                                       info, ctypes.byref(opt) if opt is not None else None, stream)


def probe_fma64(blocks, iters, stream=None):
    """Launch the fp64 FMA-rate probe; returns (sink tensor, FMAs launched)."""
    sink = torch.empty(blocks * 256, dtype=torch.float64, device="cuda")
    f = ctypes.c_int64(0)
    _check(_lib.apm_probe_fma64(_ptr(sink), int(blocks), int(iters), ctypes.byref(f), _stream(stream)),
           "apm_probe_fma64")
    return sink, f.value


def tune_cache_load(path=None):
    """Install the tuned lane-subtree orders of a cache file (None: the default path) for the
    current device; returns how many, or -1."""
    return int(_lib.apm_tune_cache_load(None if path is None else str(path).encode()))


def probe_copy(dst, src, blocks, stream=None):
    """Launch the copy probe from tensor src to tensor dst (same byte size)."""
    nb = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nb:
        raise ValueError("probe_copy: sizes differ")
    _check(_lib.apm_probe_copy(_ptr(dst), _ptr(src), int(nb), int(blocks), _stream(stream)), "apm_probe_copy")


def apm_connected_sums(m_up, m_dn, bd, c, mode, stream):
    return _lib.apm_connected_sums(m_up, m_dn, ctypes.byref(bd) if bd is not None else None, c, int(mode),
                                   stream)


def apm_all_perm_minors(A, bd, perm, stream):
    return _lib.apm_all_perm_minors(A, ctypes.byref(bd) if bd is not None else None, perm, stream)


def apm_xor_minors(dt, A, bd, out, info, stream):
    return _lib.apm_xor_minors(int(dt), A, ctypes.byref(bd) if bd is not None else None, out, info, stream)


def apm_xnor_minors(dt, A, bd, out, info, stream):
    return _lib.apm_xnor_minors(int(dt), A, ctypes.byref(bd) if bd is not None else None, out, info, stream)


def apm_nand_minors(dt, A, bd, out, info, stream):
    return _lib.apm_nand_minors(int(dt), A, ctypes.byref(bd) if bd is not None else None, out, info, stream)


def apm_leading_minors(dt, A, bd, out, info, stream):
    return _lib.apm_leading_minors(int(dt), A, ctypes.byref(bd) if bd is not None else None, out, info, stream)


def apm_status_str(s):
    return _lib.apm_status_str(int(s)).decode()


def apm_last_hip_error():
    return _lib.apm_last_hip_error()


def apm_version():
    return _lib.apm_version()


def apm_last_device_error():
    return _lib.apm_last_device_error()


def apm_plan_create(desc, out):
    return _lib.apm_plan_create(ctypes.byref(desc) if desc is not None else None, out)


def apm_plan_launch(plan, stream):
    return _lib.apm_plan_launch(plan, stream)


def apm_plan_k0(plan):
    return _lib.apm_plan_k0(plan)


def apm_plan_graphed(plan):
    return _lib.apm_plan_graphed(plan)


def apm_plan_destroy(plan):
    _lib.apm_plan_destroy(plan)


def apm_autotune_minors(dt, n, batch, k0, stream):
    return _lib.apm_autotune_minors(int(dt), int(n), int(batch), k0, stream)


def apm_minors_k0(dt, n):
    return _lib.apm_minors_k0(int(dt), int(n))


def apm_autotune_minors_mixed(dt, batch, k0_small, k0_large, stream):
    return _lib.apm_autotune_minors_mixed(int(dt), int(batch), k0_small, k0_large, stream)


def apm_minors_k0_mixed(dt, k0_small, k0_large):
    _lib.apm_minors_k0_mixed(int(dt), k0_small, k0_large)


def autotune_minors_mixed(dtype, batch=4096, stream=None):
    """Time the lane-subtree orders of the two mixed-order kernels (orders other than 14..16, and
    14..16) on a synthetic batch of orders 10..16 and install the fastest; returns them."""
    ks, kl = ctypes.c_int32(0), ctypes.c_int32(0)
    _check(apm_autotune_minors_mixed(DTYPES[dtype], batch, ctypes.byref(ks), ctypes.byref(kl), _stream(stream)),
           "apm_autotune_minors_mixed")
    return ks.value, kl.value


def minors_k0_mixed(dtype):
    """The lane-subtree orders a mixed-order launch of dtype uses now: (orders other than 14..16,
    orders 14..16)."""
    ks, kl = ctypes.c_int32(0), ctypes.c_int32(0)
    apm_minors_k0_mixed(DTYPES[dtype], ctypes.byref(ks), ctypes.byref(kl))
    return ks.value, kl.value


def autotune_minors(dtype, n, batch=4096, stream=None):
    """Time every instantiated lane-subtree order for (dtype, n) and install the fastest;
    returns it."""
    k = ctypes.c_int32(0)
    _check(apm_autotune_minors(DTYPES[dtype], n, batch, ctypes.byref(k), _stream(stream)), "apm_autotune_minors")
    return k.value


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
    (offsets None: packed prefix sums of n_b^2 and 2^n_b, formed by the library's own
    queue-preparation kernel on the device)."""
    dt = DTYPES[dtype]
    B = n.numel()
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


def xor_minors(A, *, out=None, info=None, stream=None):
    """XOR principal minors of a (B, 2n, 2n) float64 or complex128 tensor of 2 x 2 blocks.

    Returns (out, info): out is (B, 2**(n+1) - 2); depth k = 1..n occupies entries
    2**k - 2 ... 2**(k+1) - 3 and lists the minors of the k trailing blocks (bit i of the
    entry's offset chooses the row of block n-k+i); the order-n minors are the last 2**n."""
    if A.dim() != 3 or A.shape[1] != A.shape[2] or A.shape[1] % 2:
        raise ValueError("A must be (B, 2n, 2n)")
    if not A.is_cuda or not A.is_contiguous() or A.dtype not in (torch.float64, torch.complex128):
        raise TypeError("A must be a contiguous float64 or complex128 CUDA tensor")
    B, n = A.shape[0], A.shape[1] // 2
    dt = APM_C128 if A.dtype == torch.complex128 else APM_R64
    if out is None:
        out = torch.empty((B, (2 << n) - 2), dtype=A.dtype, device=A.device)
    if info is None:
        info = torch.empty(B, dtype=torch.int32, device=A.device)
    _check(apm_xor_minors(dt, _ptr(A), make_batch(B, n), _ptr(out), _ptr(info), _stream(stream)),
           "apm_xor_minors")
    return out, info


def xnor_minors(A, *, out=None, info=None, stream=None):
    """XNOR principal minors of a (B, 2n, 2n) float64 or complex128 tensor of 2 x 2 blocks:
    (B, 2**n), entry mask = det of the rows/columns of the blocks in mask (entry 0 = 1)."""
    if A.dim() != 3 or A.shape[1] != A.shape[2] or A.shape[1] % 2:
        raise ValueError("A must be (B, 2n, 2n)")
    if not A.is_cuda or not A.is_contiguous() or A.dtype not in (torch.float64, torch.complex128):
        raise TypeError("A must be a contiguous float64 or complex128 CUDA tensor")
    B, n = A.shape[0], A.shape[1] // 2
    dt = APM_C128 if A.dtype == torch.complex128 else APM_R64
    if out is None:
        out = torch.empty((B, 1 << n), dtype=A.dtype, device=A.device)
    if info is None:
        info = torch.empty(B, dtype=torch.int32, device=A.device)
    _check(apm_xnor_minors(dt, _ptr(A), make_batch(B, n), _ptr(out), _ptr(info), _stream(stream)),
           "apm_xnor_minors")
    return out, info


def nand_minors(A, *, out=None, info=None, stream=None):
    """NAND principal minors of a (B, 2n, 2n) float64 or complex128 tensor of 2 x 2 blocks:
    (B, 3**n), entry sum_i t_i 3**i with t_i = 0 (block i out), 1 (row 2i), 2 (row 2i+1)."""
    if A.dim() != 3 or A.shape[1] != A.shape[2] or A.shape[1] % 2:
        raise ValueError("A must be (B, 2n, 2n)")
    if not A.is_cuda or not A.is_contiguous() or A.dtype not in (torch.float64, torch.complex128):
        raise TypeError("A must be a contiguous float64 or complex128 CUDA tensor")
    B, n = A.shape[0], A.shape[1] // 2
    dt = APM_C128 if A.dtype == torch.complex128 else APM_R64
    if out is None:
        out = torch.empty((B, 3 ** n), dtype=A.dtype, device=A.device)
    if info is None:
        info = torch.empty(B, dtype=torch.int32, device=A.device)
    _check(apm_nand_minors(dt, _ptr(A), make_batch(B, n), _ptr(out), _ptr(info), _stream(stream)),
           "apm_nand_minors")
    return out, info


def leading_minors(A, *, out=None, info=None, stream=None):
    """Leading principal minors det A[:k, :k] (k = 1..n) of a (B, n, n) float64 or
    complex128 tensor: (B, n)."""
    if A.dim() != 3 or A.shape[1] != A.shape[2]:
        raise ValueError("A must be (B, n, n)")
    if not A.is_cuda or not A.is_contiguous() or A.dtype not in (torch.float64, torch.complex128):
        raise TypeError("A must be a contiguous float64 or complex128 CUDA tensor")
    B, n = A.shape[0], A.shape[1]
    dt = APM_C128 if A.dtype == torch.complex128 else APM_R64
    if out is None:
        out = torch.empty((B, n), dtype=A.dtype, device=A.device)
    if info is None:
        info = torch.empty(B, dtype=torch.int32, device=A.device)
    _check(apm_leading_minors(dt, _ptr(A), make_batch(B, n), _ptr(out), _ptr(info), _stream(stream)),
           "apm_leading_minors")
    return out, info


def decode_scaled(m, e):
    """value = m * 2**e for the scaled outputs (host-side helper for callers)."""
    if torch.is_complex(m):
        s = torch.ldexp(torch.ones_like(e, dtype=torch.float64), e.to(torch.float64))
        return m.to(torch.complex128) * s
    return torch.ldexp(m.to(torch.float64), e.to(torch.float64))


class Plan:
    """An ``apm_plan``: one operation (or the CDet pipeline) bound to fixed device tensors,
    recorded once into a HIP graph by the library and enqueued by ``launch()``.

    Build one with the ``plan_*`` helpers below; the plan keeps references to every tensor
    it names, so they stay allocated (their values may change between launches)."""

    def __init__(self, desc, keep, where):
        self._keep = keep
        self._h = ctypes.c_void_p()
        _check(apm_plan_create(desc, ctypes.byref(self._h)), where)

    def launch(self, stream=None):
        _check(apm_plan_launch(self._h, _stream(stream)), "apm_plan_launch")

    @property
    def k0(self):
        return apm_plan_k0(self._h)

    @property
    def graphed(self):
        return bool(apm_plan_graphed(self._h))

    def close(self):
        if self._h:
            apm_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        if _lib is not None and getattr(self, "_h", None):
            self.close()


def _plan_flags(autotune, eager):
    return (APM_PLAN_AUTOTUNE if autotune else 0) | (APM_PLAN_EAGER if eager else 0)


def _plan_batch(A, n, n_max, in_off, out_off):
    """Uniform batch from the (B, n, n) shape of A, or a mixed-order one from device int32
    orders ``n`` (matrices packed by default, ``in_off`` / ``out_off`` int64 offsets)."""
    if n is None:
        if in_off is not None or out_off is not None:
            raise ValueError("offsets are taken with per-matrix orders n only")
        return make_batch(A.shape[0], A.shape[1])
    return make_batch(n.numel(), 0, n, n_max, in_off, out_off)


def plan_minors(A, out, dtype="r64", *, exp=None, info=None, out_f64=False, tau=0.0, perturb=True,
                n=None, n_max=0, in_off=None, out_off=None, autotune=False, eager=False):
    """Plan of ``all_minors`` (uniform (B, n, n) ``A``) or of a mixed-order batch (orders
    ``n``, matrices in the flat ``A``)."""
    bd = _plan_batch(A, n, n_max, in_off, out_off)
    flags = (APM_OUT_F64 if out_f64 else 0) | (0 if perturb else APM_NO_PERTURB)
    d = apm_plan_desc(kind=APM_PLAN_MINORS, dtype=DTYPES[dtype], batch=bd, A=A.data_ptr(),
                      minors=out.data_ptr(), exp=None if exp is None else exp.data_ptr(),
                      info=None if info is None else info.data_ptr(), opts=apm_opts(float(tau), flags),
                      flags=_plan_flags(autotune, eager))
    return Plan(d, (A, out, exp, info, n, in_off, out_off), "apm_plan_create(minors)")


def plan_connected_sums(m_up, c, *, m_dn=None, mode=APM_CS_ROOTED, weights=False, n=None, n_max=0, off=None,
                        eager=False):
    """Plan of ``connected_sums`` on (B, 2**n) tensors, or on a mixed-order batch (orders
    ``n``; ``off`` indexes the inputs and the output, packed by default)."""
    if n is None:
        B, nm = m_up.shape
        bd = make_batch(B, nm.bit_length() - 1)
    else:
        bd = make_batch(n.numel(), 0, n, n_max, off, off)
    d = apm_plan_desc(kind=APM_PLAN_CONNECTED_SUMS, batch=bd, m_up=m_up.data_ptr(),
                      m_dn=None if m_dn is None else m_dn.data_ptr(), c=c.data_ptr(),
                      cs_mode=mode | (APM_CS_WEIGHTS if weights else 0), flags=_plan_flags(False, eager))
    return Plan(d, (m_up, m_dn, c, n, off), "apm_plan_create(connected sums)")


def plan_perm_minors(A, out, *, n=None, n_max=0, in_off=None, out_off=None, eager=False):
    """Plan of ``all_perm_minors`` (uniform (B, n, n) ``A``, or a mixed-order batch)."""
    bd = _plan_batch(A, n, n_max, in_off, out_off)
    d = apm_plan_desc(kind=APM_PLAN_PERM_MINORS, batch=bd, A=A.data_ptr(), perm=out.data_ptr(),
                      flags=_plan_flags(False, eager))
    return Plan(d, (A, out, n, in_off, out_off), "apm_plan_create(perm minors)")


def plan_cdet(A, minors, c, *, A_dn=None, minors_dn=None, info=None, info_dn=None, dtype="r64",
              mode=APM_CS_ROOTED, tau=0.0, perturb=True, n=None, n_max=0, in_off=None, out_off=None,
              autotune=False, eager=False):
    """Plan of the CDet pipeline of Sec. V.A: the fp64 minors of ``A`` (and ``A_dn``) and the
    connected sums ``c`` of a = det A[S] det A_dn[S] (a = det A[S]^2 without ``A_dn``).
    Mixed orders: ``in_off`` indexes the matrices, ``out_off`` the minors and the sums."""
    bd = _plan_batch(A, n, n_max, in_off, out_off)
    flags = (APM_OUT_F64 if dtype == "r32s" else 0) | (0 if perturb else APM_NO_PERTURB)
    p = (lambda t: None if t is None else t.data_ptr())
    d = apm_plan_desc(kind=APM_PLAN_CDET, dtype=DTYPES[dtype], batch=bd, A=A.data_ptr(), A_dn=p(A_dn),
                      minors=minors.data_ptr(), minors_dn=p(minors_dn), info=p(info), info_dn=p(info_dn),
                      c=c.data_ptr(), cs_mode=mode, opts=apm_opts(float(tau), flags),
                      flags=_plan_flags(autotune, eager))
    return Plan(d, (A, A_dn, minors, minors_dn, info, info_dn, c, n, in_off, out_off), "apm_plan_create(cdet)")


# ----------------------------------------------------------------- Monte Carlo + proposal network
def _ref(x):
    return None if x is None else ctypes.byref(x)


def apm_mlp_param_count(d_in, d_out):
    return _lib.apm_mlp_param_count(int(d_in), int(d_out))


def apm_mlp_weight_count(d_in, d_out):
    return _lib.apm_mlp_weight_count(int(d_in), int(d_out))


def apm_mlp_work_bytes(d_in, d_out, batch):
    return _lib.apm_mlp_work_bytes(int(d_in), int(d_out), int(batch))


def apm_mlp_sync(net, stream):
    return _lib.apm_mlp_sync(_ref(net), stream)


def apm_mlp_forward(net, x, batch, out, work, stream):
    return _lib.apm_mlp_forward(_ref(net), x, int(batch), out, work, stream)


def apm_mlp_backward(net, dout, batch, work, stream):
    return _lib.apm_mlp_backward(_ref(net), dout, int(batch), work, stream)


def apm_mlp_adam(net, h, stream):
    return _lib.apm_mlp_adam(_ref(net), _ref(h), stream)


def apm_mc_work_bytes(m, walkers, with_net):
    return _lib.apm_mc_work_bytes(_ref(m), int(walkers), int(with_net))


def apm_mc_evaluate(m, ch, work, stream):
    return _lib.apm_mc_evaluate(_ref(m), _ref(ch), work, stream)


def apm_mc_step(m, ch, net, train, seed, step, rec, work, stream):
    return _lib.apm_mc_step(_ref(m), _ref(ch), _ref(net), _ref(train), int(seed), int(step), _ref(rec), work, stream)


def apm_mc_context(m, ch, seed, step, moved, feat, stream):
    return _lib.apm_mc_context(_ref(m), _ref(ch), int(seed), int(step), moved, feat, stream)


def apm_mc_propose(m, ch, seed, step, moved, logits, stride, proposed, logq, mats, stream):
    return _lib.apm_mc_propose(_ref(m), _ref(ch), int(seed), int(step), moved, logits, int(stride), proposed, logq,
                               mats, stream)


def apm_mc_accept(m, ch, seed, step, moved, proposed, logq, mats, rec, work, stream):
    return _lib.apm_mc_accept(_ref(m), _ref(ch), int(seed), int(step), moved, proposed, logq, mats, _ref(rec), work,
                              stream)


def mlp_dims(d_in, d_out):
    """Padded (Dp, Op) of the proposal network."""
    return max(16, -(-d_in // 16) * 16), -(-d_out // 16) * 16


class Mlp:
    """Device buffers of one proposal network (fp32 master parameters, gradient, Adam
    moments, BF16 weight copies) and its C descriptor."""

    def __init__(self, d_in, d_out, params=None, device="cuda"):
        P = apm_mlp_param_count(d_in, d_out)
        NW = apm_mlp_weight_count(d_in, d_out)
        if P < 0:
            raise ValueError("network sizes out of range")
        self.d_in, self.d_out = int(d_in), int(d_out)
        self.dp, self.op = mlp_dims(d_in, d_out)
        f32 = dict(dtype=torch.float32, device=device)
        self.param = torch.zeros(P, **f32)
        if params is not None:
            self.param.copy_(torch.as_tensor(params, dtype=torch.float32))
        self.grad = torch.zeros(P, **f32)
        self.adam_m = torch.zeros(P, **f32)
        self.adam_v = torch.zeros(P, **f32)
        self.w = torch.zeros(NW, dtype=torch.bfloat16, device=device)
        self.wt = torch.zeros(NW, dtype=torch.bfloat16, device=device)
        self.c = apm_mlp(self.d_in, self.d_out, self.param.data_ptr(), self.grad.data_ptr(),
                         self.adam_m.data_ptr(), self.adam_v.data_ptr(), self.w.data_ptr(), self.wt.data_ptr())
        self.t = 0
        self.sync()

    def sync(self, stream=None):
        _check(apm_mlp_sync(self.c, _stream(stream)), "apm_mlp_sync")

    def work(self, batch):
        return torch.empty(apm_mlp_work_bytes(self.d_in, self.d_out, batch), dtype=torch.uint8,
                           device=self.param.device)

    def forward(self, x, out=None, work=None, stream=None):
        """x: (B, Dp) bfloat16 device tensor -> (B, Op) float32 logits."""
        B = x.shape[0]
        if x.dtype != torch.bfloat16 or x.shape[1] != self.dp or not x.is_contiguous():
            raise TypeError("x must be a contiguous (B, Dp) bfloat16 tensor")
        if out is None:
            out = torch.empty((B, self.op), dtype=torch.float32, device=x.device)
        _check(apm_mlp_forward(self.c, _ptr(x), B, _ptr(out), _ptr(work), _stream(stream)), "apm_mlp_forward")
        return out

    def backward(self, dout, work, stream=None):
        _check(apm_mlp_backward(self.c, _ptr(dout), dout.shape[0], _ptr(work), _stream(stream)),
               "apm_mlp_backward")
        return self.grad

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, t=None, stream=None):
        self.t = self.t + 1 if t is None else int(t)
        h = apm_adam(lr, beta1, beta2, eps, self.t)
        _check(apm_mlp_adam(self.c, h, _stream(stream)), "apm_mlp_adam")


class McChain:
    """Walker state on the device: packed vertices (int32 storage of the uint32 words),
    log|c[V]| and the sign of c[V]."""

    def __init__(self, states, device="cuda"):
        if isinstance(states, torch.Tensor):
            if states.dtype != torch.int32:
                raise TypeError("device states must be int32 storage of the packed uint32 vertices")
            st = states
        else:
            import numpy as np
            st = torch.from_numpy(np.ascontiguousarray(np.asarray(states, dtype=np.uint32)).view(np.int32))
        self.state = st.to(device).contiguous()
        W = self.state.shape[0]
        self.logw = torch.full((W,), float("-inf"), dtype=torch.float64, device=device)
        self.sign = torch.zeros(W, dtype=torch.int8, device=device)
        self.c = apm_mc_chain(W, self.state.data_ptr(), self.logw.data_ptr(), self.sign.data_ptr())

    @property
    def walkers(self):
        return self.state.shape[0]


def mc_model(n, L, n_tau, n_bin, eps, g0, resolve=0.0):
    """C descriptor of the model; ``g0`` is the device fp64 table (kept alive by the caller)."""
    return apm_mc_model(int(n), int(L), int(n_tau), int(n_bin), float(eps), float(resolve), g0.data_ptr())


def mc_work(model, walkers, with_net, device="cuda"):
    nb = apm_mc_work_bytes(model, walkers, 1 if with_net else 0)
    if nb < 0:
        raise ValueError("bad model or walker count")
    return torch.empty(max(nb, 1), dtype=torch.uint8, device=device)


class McRecord:
    """Per-step outputs of ``mc_step`` (device tensors)."""

    def __init__(self, walkers, device="cuda", loss=True):
        W = walkers
        self.moved = torch.empty(W, dtype=torch.int32, device=device)
        self.proposed = torch.empty(W, dtype=torch.int32, device=device)
        self.logq = torch.empty(W, dtype=torch.float64, device=device)
        self.logc_prop = torch.empty(W, dtype=torch.float64, device=device)
        self.accepted = torch.empty(W, dtype=torch.uint8, device=device)
        self.obs_logw = torch.empty(W, dtype=torch.float32, device=device)
        self.obs_sign = torch.empty(W, dtype=torch.int8, device=device)
        self.loss = torch.zeros(1, dtype=torch.float32, device=device) if loss else None
        self.c = self._c()

    def _c(self, obs_logw=None, obs_sign=None):
        return apm_mc_record(self.moved.data_ptr(), self.proposed.data_ptr(), self.logq.data_ptr(),
                             self.logc_prop.data_ptr(), self.accepted.data_ptr(),
                             (self.obs_logw if obs_logw is None else obs_logw).data_ptr(),
                             (self.obs_sign if obs_sign is None else obs_sign).data_ptr(),
                             self.loss.data_ptr() if self.loss is not None else None)


def mc_evaluate(model, chain, work, stream=None):
    _check(apm_mc_evaluate(model, chain.c, _ptr(work), _stream(stream)), "apm_mc_evaluate")


def mc_step(model, chain, work, seed, step, net=None, train=None, record=None, stream=None):
    """One Metropolis-Hastings step of every walker; ``train`` = dict(lr, beta1, beta2,
    eps, t) trains ``net`` on the step's proposals."""
    h = None
    if train is not None:
        h = apm_adam(train.get("lr", 1e-3), train.get("beta1", 0.9), train.get("beta2", 0.999),
                     train.get("eps", 1e-8), int(train["t"]))
    rec = record.c if isinstance(record, McRecord) else record
    _check(apm_mc_step(model, chain.c, net.c if net is not None else None, h, seed, step, rec, _ptr(work),
                       _stream(stream)), "apm_mc_step")
