"""FP64 CPU oracle for the 3D real DFT -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never uses it and
shares no code with it (the C source is ``oracle/oracle.c``).

What it computes: the paper's forward r2c transform of an n0 x n1 x n2 real
array to n0 x n1 x (n2/2+1) complex and the c2r inverse (Sec. 2, problem
statement), forward sign minus, no normalisation, natural-order spectrum
(Sec. 2.2, Fig. 4).  See the header of ``oracle.c`` for every reading taken
where the paper is silent.

Every function here takes and returns numpy float64 / complex128 arrays in C
order.  ``threads`` <= 0 means "all OpenMP threads".
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_i64 = ctypes.c_int64
_dp = ctypes.POINTER(ctypes.c_double)


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (plain C11, OpenMP, -O2) into liboracle.so."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra",
               _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        L.oracle_dft1d.argtypes = [_i64, ctypes.c_int, _dp, _dp]
        L.oracle_fft1d.argtypes = [_i64, ctypes.c_int, _dp, _dp]
        L.oracle_r2c.argtypes = [_i64, _i64, _i64, _dp, _dp, ctypes.c_int]
        L.oracle_c2r.argtypes = [_i64, _i64, _i64, _dp, _dp, ctypes.c_int]
        L.oracle_c2r_ex.argtypes = [_i64, _i64, _i64, _dp, _dp, ctypes.c_int, _dp]
        L.oracle_r2c_direct.argtypes = [_i64, _i64, _i64, _dp, _dp]
        L.oracle_c2r_direct.argtypes = [_i64, _i64, _i64, _dp, _dp]
        L.oracle_r2c_point.argtypes = [_i64, _i64, _i64, _dp, _i64, _i64, _i64, _dp]
        L.oracle_c2r_point.argtypes = [_i64, _i64, _i64, _dp, _i64, _i64, _i64, _dp]
        for name in ("oracle_dft1d", "oracle_fft1d", "oracle_r2c", "oracle_c2r", "oracle_c2r_ex",
                     "oracle_r2c_direct", "oracle_c2r_direct", "oracle_r2c_point",
                     "oracle_c2r_point", "oracle_max_threads"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def _real(x) -> np.ndarray:
    return np.ascontiguousarray(x, dtype=np.float64)


def _cplx(X) -> np.ndarray:
    return np.ascontiguousarray(X, dtype=np.complex128)


def _check(rc: int, what: str) -> None:
    if rc != 0:
        raise RuntimeError("%s failed with code %d" % (what, rc))


def half(n2: int) -> int:
    """Number of kept k2 bins: n2/2+1 (integer division)."""
    return n2 // 2 + 1


def max_threads() -> int:
    return lib().oracle_max_threads()


def dft1d(x, sign: int = -1) -> np.ndarray:
    """Naive O(n^2) DFT, the definition (long double accumulation)."""
    x = _cplx(x).ravel()
    out = np.empty_like(x)
    _check(lib().oracle_dft1d(x.size, sign, _ptr(x.view(np.float64)), _ptr(out.view(np.float64))),
           "oracle_dft1d")
    return out


def fft1d(x, sign: int = -1) -> np.ndarray:
    """Plain recursive mixed-radix FFT (naive DFT on prime lengths)."""
    x = _cplx(x).ravel()
    out = np.empty_like(x)
    _check(lib().oracle_fft1d(x.size, sign, _ptr(x.view(np.float64)), _ptr(out.view(np.float64))),
           "oracle_fft1d")
    return out


def r2c(x, threads: int = 0) -> np.ndarray:
    """Forward 3D r2c in the paper's step order; returns n0 x n1 x (n2/2+1)."""
    x = _real(x)
    n0, n1, n2 = x.shape
    X = np.empty((n0, n1, half(n2)), dtype=np.complex128)
    _check(lib().oracle_r2c(n0, n1, n2, _ptr(x), _ptr(X.view(np.float64)), threads), "oracle_r2c")
    return X


def c2r(X, n2: int, threads: int = 0, return_max_imag: bool = False):
    """Inverse 3D c2r (steps of r2c in reverse order); X is not modified."""
    X = _cplx(X)
    n0, n1, h = X.shape
    if h != half(n2):
        raise ValueError("last axis %d does not match n2=%d" % (h, n2))
    y = np.empty((n0, n1, n2), dtype=np.float64)
    mi = ctypes.c_double(0.0)
    _check(lib().oracle_c2r_ex(n0, n1, n2, _ptr(X.view(np.float64)), _ptr(y), threads,
                               ctypes.byref(mi)), "oracle_c2r")
    return (y, mi.value) if return_max_imag else y


def r2c_direct(x) -> np.ndarray:
    """Forward transform by the literal triple sum (tiny sizes only)."""
    x = _real(x)
    n0, n1, n2 = x.shape
    X = np.empty((n0, n1, half(n2)), dtype=np.complex128)
    _check(lib().oracle_r2c_direct(n0, n1, n2, _ptr(x), _ptr(X.view(np.float64))),
           "oracle_r2c_direct")
    return X


def c2r_direct(X, n2: int) -> np.ndarray:
    """Inverse by the definition Re(IDFT3(E(X))) on the full grid (tiny sizes)."""
    X = _cplx(X)
    n0, n1, h = X.shape
    if h != half(n2):
        raise ValueError("last axis %d does not match n2=%d" % (h, n2))
    y = np.empty((n0, n1, n2), dtype=np.float64)
    _check(lib().oracle_c2r_direct(n0, n1, n2, _ptr(X.view(np.float64)), _ptr(y)),
           "oracle_c2r_direct")
    return y


def r2c_point(x, k) -> complex:
    """One forward output X[k0,k1,k2] from the definition, O(N) work."""
    x = _real(x)
    n0, n1, n2 = x.shape
    out = np.zeros(2)
    _check(lib().oracle_r2c_point(n0, n1, n2, _ptr(x), int(k[0]), int(k[1]), int(k[2]), _ptr(out)),
           "oracle_r2c_point")
    return complex(out[0], out[1])


def c2r_point(X, n2: int, j) -> float:
    """One inverse output y[j0,j1,j2] from the definition, O(M) work."""
    X = _cplx(X)
    n0, n1, h = X.shape
    if h != half(n2):
        raise ValueError("last axis %d does not match n2=%d" % (h, n2))
    out = np.zeros(1)
    _check(lib().oracle_c2r_point(n0, n1, n2, _ptr(X.view(np.float64)), int(j[0]), int(j[1]),
                                  int(j[2]), _ptr(out)), "oracle_c2r_point")
    return float(out[0])


# ---- pruned transforms (the dealiased solver's view of the transform) ----
#
# The pseudo-spectral solver the transform serves (Sec. 1) keeps only the
# modes inside a box and treats the rest as zero (with the two-thirds rule,
# |k| <= n/3 per axis).  A pruned forward transform is the forward transform
# restricted to the box; a pruned inverse is the inverse of the spectrum
# zeroed outside it.  Both are plain definitions on top of r2c / c2r.

def box_mask(shape, kmax) -> np.ndarray:
    """Boolean n0 x n1 x (n2/2+1) mask of the kept modes: |k0| <= K0,
    |k1| <= K1 (signed index k or k - n), 0 <= k2 <= K2.  A negative K keeps
    the whole axis."""
    n0, n1, n2 = shape
    K0, K1, K2 = (int(v) for v in kmax)

    def keep(n, K):
        i = np.arange(n)
        s = np.where(i <= n // 2, i, i - n)  # signed index
        return np.ones(n, bool) if K < 0 else np.abs(s) <= K

    k2 = np.arange(half(n2))
    m2 = np.ones(half(n2), bool) if K2 < 0 else k2 <= K2
    return keep(n0, K0)[:, None, None] & keep(n1, K1)[None, :, None] & m2[None, None, :]


def r2c_pruned(x, kmax, threads: int = 0) -> np.ndarray:
    """Forward transform with every mode outside the box set to zero."""
    X = r2c(x, threads)
    X[~box_mask(np.shape(x), kmax)] = 0
    return X


def c2r_pruned(X, n2: int, kmax, threads: int = 0) -> np.ndarray:
    """Inverse transform of X with every mode outside the box set to zero
    (X is not modified)."""
    X = np.array(_cplx(X), copy=True)
    n0, n1, _ = X.shape
    X[~box_mask((n0, n1, n2), kmax)] = 0
    return c2r(X, n2, threads)
