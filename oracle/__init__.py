"""CPU oracle for the principal-minor library -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously correct reference implementations of what the GPU path
computes (Simkovic & Ferrero, arXiv:2104.07638).  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import this package.  It shares no code with the HIP library and never imports
it; the two meet only through the seeded generators in ``workloads``.

Functions (all fp64 / complex128, row-major inputs, outputs in bit-mask order,
bit k <-> row/column k, out[0] = det of the empty matrix = 1):

* ``minors(A)``            -- Sec. II: det(A[S]) for every subset S, one
                              partial-pivoting LU per subset (C, ``apm_oracle.c``).
* ``connected_sums(a, mode)`` -- Sec. V.A, Eq. (recursion), direct O(3^n) loop.
* ``perm_minors(A)``       -- Sec. IV: Ryser's formula per subset, with the
                              (-1)^|S| factor the printed Eq. (ryser) drops.
* ``xnor_minors(A)``       -- Sec. III, XNOR case: det of every whole-block subset.
* ``leading_minors(A)``    -- Sec. III: det of every leading k x k submatrix.
* ``nand_minors(A)``       -- Sec. III, NAND case: det of every at-most-one-row-per-block
                              subset.
* ``xor_minors(A)``        -- Sec. III, XOR case: det of every one-row-per-block
                              choice of a 2n x 2n block matrix, and of the trailing
                              k blocks for every depth k < n.
* ``g0``-independent: the oracle consumes host matrices built by ``workloads``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "apm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True, path: str = _LIB, plant: int = 0) -> str:
    """Compile ``apm_oracle.c`` (gcc -O2, OpenMP) into ``path``.

    ``plant`` != 0 builds a deliberately broken variant; only the test that
    checks the pins' power uses it."""
    if force or not os.path.exists(path):
        tmp = path + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               "-Wall", f"-DORACLE_PLANT={int(plant)}", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, path)
    return path


def load_library(path: str):
    """Load an oracle shared library and declare its C signatures."""
    lib = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int32)
    lp = ctypes.POINTER(ctypes.c_int64)
    for name in ("apm_oracle_minors_r64", "apm_oracle_minors_c128", "apm_oracle_perm_minors"):
        fn = getattr(lib, name)
        fn.argtypes = [ctypes.c_int, dp, dp]
        fn.restype = ctypes.c_int
    lib.apm_oracle_connected_sums.argtypes = [ctypes.c_int, dp, dp, ctypes.c_int]
    lib.apm_oracle_cs_input_bound.argtypes = [ctypes.c_int, dp, dp, dp, dp, ctypes.c_int]
    lib.apm_oracle_cs_input_bound.restype = ctypes.c_int
    lib.apm_oracle_connected_sums.restype = ctypes.c_int
    for name in ("apm_oracle_minors_r64_batch", "apm_oracle_minors_c128_batch",
                 "apm_oracle_perm_minors_batch"):
        fn = getattr(lib, name)
        fn.argtypes = [ctypes.c_int, ip, lp, lp, dp, dp, ctypes.c_int]
        fn.restype = ctypes.c_int
    lib.apm_oracle_connected_sums_batch.argtypes = [ctypes.c_int, ip, lp, dp, dp, ctypes.c_int,
                                                    ctypes.c_int]
    lib.apm_oracle_connected_sums_batch.restype = ctypes.c_int
    lib.apm_oracle_max_threads.restype = ctypes.c_int
    lib.apm_oracle_minors_r64_masks.argtypes = [ctypes.c_int, dp, ctypes.c_int,
                                                ctypes.POINTER(ctypes.c_uint32), dp]
    lib.apm_oracle_minors_r64_masks.restype = ctypes.c_int
    lib.apm_oracle_perm_minors_masks.argtypes = [ctypes.c_int, dp, ctypes.c_int,
                                                 ctypes.POINTER(ctypes.c_uint32), dp]
    lib.apm_oracle_perm_minors_masks.restype = ctypes.c_int
    lib.apm_oracle_cs_scale.argtypes = [ctypes.c_int, dp, dp, dp, ctypes.c_int]
    lib.apm_oracle_cs_scale.restype = ctypes.c_int
    for name in ("apm_oracle_xor_minors_r64", "apm_oracle_xor_minors_c128", "apm_oracle_xnor_minors_r64",
                 "apm_oracle_xnor_minors_c128", "apm_oracle_leading_minors_r64",
                 "apm_oracle_leading_minors_c128", "apm_oracle_nand_minors_r64", "apm_oracle_nand_minors_c128"):
        fn = getattr(lib, name)
        fn.argtypes = [ctypes.c_int, dp, dp]
        fn.restype = ctypes.c_int
    return lib


def _load(lib=None):
    global _lib
    if lib is not None:
        return lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        _lib = load_library(_LIB)
    return _lib


def _dp(x):
    return x.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def max_threads() -> int:
    return int(_load().apm_oracle_max_threads())


def _as_batch(A, complex_=False):
    A = np.asarray(A)
    single = A.ndim == 2
    if single:
        A = A[None]
    if complex_:
        A = np.ascontiguousarray(A, dtype=np.complex128)
    else:
        if np.iscomplexobj(A):
            raise TypeError("real oracle called with complex input")
        A = np.ascontiguousarray(A, dtype=np.float64)
    return A, single


def minors(A, nthreads: int = 0, lib=None) -> np.ndarray:
    """All principal minors of a real (B, n, n) or (n, n) matrix batch (Sec. II).

    Returns (B, 2**n) (or (2**n,) for a single matrix), fp64."""
    A, single = _as_batch(A)
    B, n, _ = A.shape
    out = np.empty((B, 1 << n), dtype=np.float64)
    nv = np.full(B, n, dtype=np.int32)
    ioff = (np.arange(B, dtype=np.int64) * n * n)
    ooff = (np.arange(B, dtype=np.int64) << n)
    rc = _load(lib).apm_oracle_minors_r64_batch(B, nv.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                            ioff.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                            ooff.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                            _dp(A), _dp(out), int(nthreads))
    if rc != 0:
        raise ValueError("oracle: bad matrix order")
    return out[0] if single else out


def minors_at(A, masks, lib=None) -> np.ndarray:
    """det(A[S_m]) for the listed masks only (same definition as ``minors``)."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    n = A.shape[0]
    masks = np.ascontiguousarray(masks, dtype=np.uint32)
    out = np.empty(masks.shape[0], dtype=np.float64)
    rc = _load(lib).apm_oracle_minors_r64_masks(n, _dp(A), int(masks.shape[0]),
                                                masks.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                                                _dp(out))
    if rc != 0:
        raise ValueError("oracle: bad matrix order")
    return out


def minors_complex(A, nthreads: int = 0, lib=None) -> np.ndarray:
    """All principal minors of a complex128 batch (Sec. V.C matrices are complex)."""
    A, single = _as_batch(A, complex_=True)
    B, n, _ = A.shape
    out = np.empty((B, 1 << n), dtype=np.complex128)
    nv = np.full(B, n, dtype=np.int32)
    ioff = (np.arange(B, dtype=np.int64) * n * n)
    ooff = (np.arange(B, dtype=np.int64) << n)
    rc = _load(lib).apm_oracle_minors_c128_batch(B, nv.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                             ioff.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                             ooff.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                             _dp(A.view(np.float64)), _dp(out.view(np.float64)),
                                             int(nthreads))
    if rc != 0:
        raise ValueError("oracle: bad matrix order")
    return out[0] if single else out


def xor_minors(A, lib=None) -> np.ndarray:
    """XOR principal minors of 2n x 2n matrices of 2 x 2 blocks (Sec. III, XOR case).

    For depth k = 1..n and every k-bit choice word beta over the k trailing blocks (bit i:
    row/column 2(n-k+i) + beta_i of block n-k+i kept), entry 2^k - 2 + beta is
    det A[R, R], R = {2(n-k+i) + beta_i : i < k}; the order-n minors (bit i <-> block i)
    are the last 2^n entries.  Real or complex input of shape (B, 2n, 2n) or (2n, 2n);
    returns (B, 2^(n+1) - 2) (or one row)."""
    A = np.asarray(A)
    single = A.ndim == 2
    if single:
        A = A[None]
    cplx = np.iscomplexobj(A)
    A = np.ascontiguousarray(A, dtype=np.complex128 if cplx else np.float64)
    B, w, _ = A.shape
    if w % 2:
        raise ValueError("xor_minors: the order must be even (2 x 2 blocks)")
    n = w // 2
    out = np.empty((B, (1 << (n + 1)) - 2), dtype=A.dtype)
    L = _load(lib)
    fn = L.apm_oracle_xor_minors_c128 if cplx else L.apm_oracle_xor_minors_r64
    for b in range(B):
        src = A[b].view(np.float64) if cplx else A[b]
        dst = out[b].view(np.float64) if cplx else out[b]
        if fn(n, _dp(src), _dp(dst)) != 0:
            raise ValueError("oracle: bad matrix order")
    return out[0] if single else out


def xnor_minors(A, lib=None) -> np.ndarray:
    """XNOR principal minors of 2n x 2n matrices of 2 x 2 blocks (Sec. III, XNOR case):
    entry mask is det A[R, R], R = the two rows of every block i with bit i of mask set
    (entry 0 = 1).  Real or complex input (B, 2n, 2n) or (2n, 2n); returns (B, 2^n)."""
    A = np.asarray(A)
    single = A.ndim == 2
    if single:
        A = A[None]
    cplx = np.iscomplexobj(A)
    A = np.ascontiguousarray(A, dtype=np.complex128 if cplx else np.float64)
    B, w, _ = A.shape
    if w % 2:
        raise ValueError("xnor_minors: the order must be even (2 x 2 blocks)")
    n = w // 2
    out = np.empty((B, 1 << n), dtype=A.dtype)
    L = _load(lib)
    fn = L.apm_oracle_xnor_minors_c128 if cplx else L.apm_oracle_xnor_minors_r64
    for b in range(B):
        src = A[b].view(np.float64) if cplx else A[b]
        dst = out[b].view(np.float64) if cplx else out[b]
        if fn(n, _dp(src), _dp(dst)) != 0:
            raise ValueError("oracle: bad matrix order")
    return out[0] if single else out


def nand_minors(A, lib=None) -> np.ndarray:
    """NAND principal minors of 2n x 2n matrices of 2 x 2 blocks (Sec. III, NAND case):
    entry sum_i t_i 3^i (t_i = 0: block i left out, 1: row 2i kept, 2: row 2i+1 kept) is the
    determinant over the kept rows (entry 0 = 1).  Real or complex (B, 2n, 2n) or (2n, 2n);
    returns (B, 3^n)."""
    A = np.asarray(A)
    single = A.ndim == 2
    if single:
        A = A[None]
    cplx = np.iscomplexobj(A)
    A = np.ascontiguousarray(A, dtype=np.complex128 if cplx else np.float64)
    B, w, _ = A.shape
    if w % 2:
        raise ValueError("nand_minors: the order must be even (2 x 2 blocks)")
    n = w // 2
    out = np.empty((B, 3 ** n), dtype=A.dtype)
    L = _load(lib)
    fn = L.apm_oracle_nand_minors_c128 if cplx else L.apm_oracle_nand_minors_r64
    for b in range(B):
        src = A[b].view(np.float64) if cplx else A[b]
        dst = out[b].view(np.float64) if cplx else out[b]
        if fn(n, _dp(src), _dp(dst)) != 0:
            raise ValueError("oracle: bad matrix order")
    return out[0] if single else out


def leading_minors(A, lib=None) -> np.ndarray:
    """Leading principal minors (Sec. III): entry k-1 is det A[:k, :k], k = 1..n.  Real or
    complex (B, n, n) or (n, n); returns (B, n) (or one row)."""
    A = np.asarray(A)
    single = A.ndim == 2
    if single:
        A = A[None]
    cplx = np.iscomplexobj(A)
    A = np.ascontiguousarray(A, dtype=np.complex128 if cplx else np.float64)
    B, n, _ = A.shape
    out = np.empty((B, n), dtype=A.dtype)
    L = _load(lib)
    fn = L.apm_oracle_leading_minors_c128 if cplx else L.apm_oracle_leading_minors_r64
    for b in range(B):
        src = A[b].view(np.float64) if cplx else A[b]
        dst = out[b].view(np.float64) if cplx else out[b]
        if fn(n, _dp(src), _dp(dst)) != 0:
            raise ValueError("oracle: bad matrix order")
    return out[0] if single else out


def minors_ragged(mats, nthreads: int = 0, lib=None):
    """Principal minors of a list of real matrices of different orders."""
    B = len(mats)
    ns = np.array([m.shape[0] for m in mats], dtype=np.int32)
    ioff = np.zeros(B, dtype=np.int64)
    ooff = np.zeros(B, dtype=np.int64)
    if B:
        ioff[1:] = np.cumsum(ns[:-1].astype(np.int64) ** 2)
        ooff[1:] = np.cumsum(np.left_shift(1, ns[:-1].astype(np.int64)))
    flat = np.ascontiguousarray(np.concatenate([np.asarray(m, dtype=np.float64).ravel() for m in mats])
                                if B else np.zeros(0))
    total = int(ooff[-1] + (1 << int(ns[-1]))) if B else 0
    out = np.empty(total, dtype=np.float64)
    rc = _load(lib).apm_oracle_minors_r64_batch(B, ns.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                            ioff.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                            ooff.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                            _dp(flat), _dp(out), int(nthreads))
    if rc != 0:
        raise ValueError("oracle: bad matrix order")
    return [out[int(o):int(o) + (1 << int(k))] for o, k in zip(ooff, ns)]


def connected_sums(a, mode: int = 0, nthreads: int = 0, lib=None) -> np.ndarray:
    """Connected sums c[S] from subset weights a[S] (Sec. V.A, Eq. (recursion)).

    ``a`` is (B, 2**n) or (2**n,).  mode 0: rooted at vertex 0 (c = 0 on sets
    without vertex 0); mode 1: every nonempty set, rooted at its lowest vertex."""
    a = np.asarray(a, dtype=np.float64)
    single = a.ndim == 1
    if single:
        a = a[None]
    a = np.ascontiguousarray(a)
    B, nm = a.shape
    n = nm.bit_length() - 1
    if (1 << n) != nm:
        raise ValueError("length must be a power of two")
    c = np.empty_like(a)
    nv = np.full(B, n, dtype=np.int32)
    off = np.arange(B, dtype=np.int64) * nm
    rc = _load(lib).apm_oracle_connected_sums_batch(B, nv.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                                off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                                _dp(a), _dp(c), int(mode), int(nthreads))
    if rc != 0:
        raise ValueError("oracle: bad arguments")
    return c[0] if single else c


def cs_scale(a, c, mode: int = 0, lib=None) -> np.ndarray:
    """Error scale of the recursion at every S (metric helper for parity tests):
    d[S] = |a[S]| + sum_T |c[T]| |a[S \\ T]| over the recursion's terms."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    c = np.ascontiguousarray(c, dtype=np.float64)
    n = a.shape[-1].bit_length() - 1
    d = np.empty_like(a)
    for idx in np.ndindex(a.shape[:-1]):
        rc = _load(lib).apm_oracle_cs_scale(n, _dp(np.ascontiguousarray(a[idx])), _dp(np.ascontiguousarray(c[idx])),
                                            _dp(d[idx]), int(mode))
        if rc != 0:
            raise ValueError("oracle: bad arguments")
    return d


def cs_input_bound(a, c, da, mode: int = 0, lib=None) -> np.ndarray:
    """First-order bound on |c' - c| when the weights carry errors of at most ``da``
    (metric helper for parity tests; Eq. (recursion) differentiated term by term)."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    c = np.ascontiguousarray(c, dtype=np.float64)
    da = np.ascontiguousarray(da, dtype=np.float64)
    n = a.shape[-1].bit_length() - 1
    e = np.empty_like(a)
    for idx in np.ndindex(a.shape[:-1]):
        rc = _load(lib).apm_oracle_cs_input_bound(n, _dp(np.ascontiguousarray(a[idx])),
                                                  _dp(np.ascontiguousarray(c[idx])),
                                                  _dp(np.ascontiguousarray(da[idx])), _dp(e[idx]), int(mode))
        if rc != 0:
            raise ValueError("oracle: bad arguments")
    return e


def perm_minors(A, nthreads: int = 0, lib=None) -> np.ndarray:
    """All permanent principal minors (Sec. IV), Ryser per subset."""
    A, single = _as_batch(A)
    B, n, _ = A.shape
    out = np.empty((B, 1 << n), dtype=np.float64)
    nv = np.full(B, n, dtype=np.int32)
    ioff = (np.arange(B, dtype=np.int64) * n * n)
    ooff = (np.arange(B, dtype=np.int64) << n)
    rc = _load(lib).apm_oracle_perm_minors_batch(B, nv.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                             ioff.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                             ooff.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                             _dp(A), _dp(out), int(nthreads))
    if rc != 0:
        raise ValueError("oracle: bad matrix order")
    return out[0] if single else out


def perm_minors_at(A, masks, lib=None) -> np.ndarray:
    """per(A[S_m]) for the listed masks only (same definition as ``perm_minors``)."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    n = A.shape[0]
    masks = np.ascontiguousarray(masks, dtype=np.uint32)
    out = np.empty(masks.shape[0], dtype=np.float64)
    rc = _load(lib).apm_oracle_perm_minors_masks(n, _dp(A), int(masks.shape[0]),
                                                 masks.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                                                 _dp(out))
    if rc != 0:
        raise ValueError("oracle: bad matrix order or mask")
    return out


def cdet_weights(m_up, m_dn=None) -> np.ndarray:
    """Sec. V.A: a[S] = det(M_up[S]) det(M_dn[S]) from two minors arrays
    (a single array stands for both spins)."""
    m_up = np.asarray(m_up, dtype=np.float64)
    return m_up * (m_up if m_dn is None else np.asarray(m_dn, dtype=np.float64))
