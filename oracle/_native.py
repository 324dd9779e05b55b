"""Loader for the oracle's C core (``af_direct.c``).

Test infrastructure only.  Builds ``liboracle_af.so`` next to the source with
gcc when it is missing or older than the source.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "af_direct.c")
_LIB = os.path.join(_HERE, "liboracle_af.so")
_handle = None


def build(force=False):
    """Compile the oracle's C core with gcc (-O2, OpenMP, IEEE semantics)."""
    if (not force and os.path.exists(_LIB)
            and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC)):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared",
                           "-std=gnu11", "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _handle
    if _handle is None:
        build()
        h = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        h.oracle_chi.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp]
        h.oracle_chi.restype = ctypes.c_int
        h.oracle_adjoint.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp, dp]
        h.oracle_adjoint.restype = ctypes.c_int
        ip = ctypes.POINTER(ctypes.c_int)
        h.oracle_chi_rows.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ip, dp, dp]
        h.oracle_chi_rows.restype = ctypes.c_int
        h.oracle_chi_circ.argtypes = [ctypes.c_int, dp, dp]
        h.oracle_chi_circ.restype = ctypes.c_int
        h.oracle_adjoint_circ.argtypes = [ctypes.c_int, dp, dp, dp]
        h.oracle_adjoint_circ.restype = ctypes.c_int
        h.oracle_threads.argtypes = []
        h.oracle_threads.restype = ctypes.c_int
        _handle = h
    return _handle


def threads():
    """OpenMP threads the C core runs on."""
    return int(lib().oracle_threads())


def _ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def chi(s, m, max_lag):
    """Direct-sum complex AF rows tau in [-T, T], bins k in [0, M)."""
    s = np.ascontiguousarray(np.asarray(s, dtype=np.complex128))
    n = s.shape[0]
    out = np.empty((2 * max_lag + 1, m), dtype=np.complex128)
    rc = lib().oracle_chi(n, m, max_lag, _ptr(s.view(np.float64)), _ptr(out.view(np.float64)))
    if rc != 0:
        raise ValueError("oracle_chi rejected n=%d m=%d max_lag=%d" % (n, m, max_lag))
    return out


def chi_rows(s, m, taus):
    """Direct-sum chi rows for the given lags only."""
    s = np.ascontiguousarray(np.asarray(s, dtype=np.complex128))
    taus = np.ascontiguousarray(np.asarray(taus, dtype=np.int32))
    out = np.empty((len(taus), m), dtype=np.complex128)
    rc = lib().oracle_chi_rows(s.shape[0], m, len(taus), taus.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                               _ptr(s.view(np.float64)), _ptr(out.view(np.float64)))
    if rc != 0:
        raise ValueError("oracle_chi_rows rejected its arguments")
    return out


def adjoint(s, m, max_lag, G):
    """sum over lags of the adjoint of chi applied to G = dL/d conj(chi)."""
    s = np.ascontiguousarray(np.asarray(s, dtype=np.complex128))
    G = np.ascontiguousarray(np.asarray(G, dtype=np.complex128))
    n = s.shape[0]
    assert G.shape == (2 * max_lag + 1, m)
    g = np.empty(n, dtype=np.complex128)
    rc = lib().oracle_adjoint(n, m, max_lag, _ptr(s.view(np.float64)),
                              _ptr(G.view(np.float64)), _ptr(g.view(np.float64)))
    if rc != 0:
        raise ValueError("oracle_adjoint rejected n=%d m=%d max_lag=%d" % (n, m, max_lag))
    return g


def chi_circ(s):
    """Direct-sum periodic AF, rows tau in [0, N), bins k in [0, N)."""
    s = np.ascontiguousarray(np.asarray(s, dtype=np.complex128))
    n = s.shape[0]
    out = np.empty((n, n), dtype=np.complex128)
    if lib().oracle_chi_circ(n, _ptr(s.view(np.float64)), _ptr(out.view(np.float64))) != 0:
        raise ValueError("oracle_chi_circ rejected n=%d" % n)
    return out


def adjoint_circ(s, G):
    """Adjoint of the periodic AF applied to G = dL/d conj(chi_c), [N][N]."""
    s = np.ascontiguousarray(np.asarray(s, dtype=np.complex128))
    G = np.ascontiguousarray(np.asarray(G, dtype=np.complex128))
    n = s.shape[0]
    assert G.shape == (n, n)
    g = np.empty(n, dtype=np.complex128)
    if lib().oracle_adjoint_circ(n, _ptr(s.view(np.float64)), _ptr(G.view(np.float64)),
                                 _ptr(g.view(np.float64))) != 0:
        raise ValueError("oracle_adjoint_circ rejected n=%d" % n)
    return g
