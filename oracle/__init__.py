"""ORACLE -- test infrastructure only.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path in
``paper_1809_10786_amd`` never imports it, and the two share no code: no
kernels, tables, helpers or constants.

Two independent references for the NFSGLFT of Wuelker, "Fast SGL Fourier
transforms for scattered data":

* ``direct`` (C, ``sgl_direct.c``): the exact NDSGLFT matrix Lambda of
  Def. 1.3 and its adjoint, by direct O(B^3 M) summation with three-term
  recurrences.  This is the judge of every GPU result.
* ``stepwise`` (numpy, ``stepwise.py``): the paper's fast algorithm taken in
  the paper's own order and notation (radial subtransform, spherical
  subtransform, trigonometric coefficients eta, then the NDFT or the Gaussian
  NFFT of Section 2), used to pin individual stages.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_lib = None


def lib():
    """Load (building it first if absent) the C oracle library."""
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        for suffix in ("", "_ld"):
            f = getattr(L, "oracle_forward" + suffix)
            f.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                          ctypes.c_void_p, ctypes.c_int32]
            f.restype = ctypes.c_int
            a = getattr(L, "oracle_adjoint" + suffix)
            a.argtypes = f.argtypes
            a.restype = ctypes.c_int
            b = getattr(L, "oracle_basis" + suffix)
            b.argtypes = [ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]
            b.restype = None
        L.oracle_num_coeffs.argtypes = [ctypes.c_int32]
        L.oracle_num_coeffs.restype = ctypes.c_int64
        L.oracle_mu.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
        L.oracle_mu.restype = ctypes.c_int64
        L.oracle_max_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def num_coeffs(B: int) -> int:
    return B * (B + 1) * (2 * B + 1) // 6


def _c128(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


def _pts(p):
    p = np.ascontiguousarray(p, dtype=np.float64)
    assert p.ndim == 2 and p.shape[1] == 3
    return p


def direct_forward(B, points, fhat, nthreads=0, long_double=False):
    """Exact f = Lambda fhat (Def. 1.3, eq. (1.2)); complex128 of length M."""
    p = _pts(points)
    fh = _c128(fhat)
    assert fh.shape == (num_coeffs(B),)
    out = np.empty(p.shape[0], dtype=np.complex128)
    fn = lib().oracle_forward_ld if long_double else lib().oracle_forward
    rc = fn(B, p.shape[0], p.ctypes.data, fh.ctypes.data, out.ctypes.data, nthreads)
    assert rc == 0
    return out


def direct_adjoint(B, points, y, nthreads=0, long_double=False):
    """Exact fhat = Lambda^H y; complex128 of length Nc."""
    p = _pts(points)
    yy = _c128(y)
    assert yy.shape == (p.shape[0],)
    out = np.empty(num_coeffs(B), dtype=np.complex128)
    fn = lib().oracle_adjoint_ld if long_double else lib().oracle_adjoint
    rc = fn(B, p.shape[0], p.ctypes.data, yy.ctypes.data, out.ctypes.data, nthreads)
    assert rc == 0
    return out


def basis(B, point, long_double=False):
    """All Nc values H_mu(x) at one point."""
    p = np.ascontiguousarray(point, dtype=np.float64).reshape(3)
    out = np.empty(num_coeffs(B), dtype=np.complex128)
    fn = lib().oracle_basis_ld if long_double else lib().oracle_basis
    fn(B, p.ctypes.data, out.ctypes.data)
    return out


def max_threads() -> int:
    return int(lib().oracle_max_threads())
