"""Build and load the oracle's plain-C Legendre loops (test infrastructure).

ORACLE -- test infrastructure only; see oracle/__init__.py.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "legendre.c")
_BUILD = os.path.join(_HERE, "_build")
_LIB = os.path.join(_BUILD, "liboracle_legendre.so")

_lib = None


def build(force=False):
    """Compile legendre.c with gcc (OpenMP, no fast-math)."""
    os.makedirs(_BUILD, exist_ok=True)
    if (not force and os.path.exists(_LIB)
            and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC)):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
           "-D_DEFAULT_SOURCE", _SRC, "-o", tmp, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        path = build()
        L = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        L.oracle_lambda.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                    dp, dp, dp]
        L.oracle_lambda.restype = None
        for name in ("oracle_legendre_analysis", "oracle_legendre_synthesis"):
            f = getattr(L, name)
            f.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp,
                          dp, dp, ctypes.c_int]
            f.restype = None
        _lib = L
    return _lib


def threads():
    v = os.environ.get("SHTX_ORACLE_THREADS")
    if v:
        return max(1, int(v))
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1


def ptr(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
