"""Builds and loads the oracle's C part with gcc: the binary128 Newell
evaluator (newell_q.c) and the compensated direct demag sum (direct_sum.c).

Test infrastructure only (see the package docstring)."""
import ctypes
import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, "newell_q.c"), os.path.join(_HERE, "direct_sum.c")]
_LIB = os.path.join(_HERE, "liboracle_newell.so")
_lib = None


def build(force=False):
    """Compile the C sources -> liboracle_newell.so (IEEE, no fast-math)."""
    newest = max(os.path.getmtime(s) for s in _SRCS)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < newest:
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-fno-fast-math"] + _SRCS +
                              ["-o", tmp, "-lquadmath", "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        i64, dbl, pd, pi64 = ctypes.c_int64, ctypes.c_double, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)
        L.oracle_newell.argtypes = [i64, i64, i64, dbl, dbl, dbl, pd, pd]
        L.oracle_far.argtypes = [i64, i64, i64, dbl, dbl, dbl, pd]
        L.oracle_tensor_at.argtypes = [i64, i64, i64, dbl, dbl, dbl, dbl, pd]
        L.oracle_tensor_many.argtypes = [i64, pi64, dbl, dbl, dbl, dbl, pd]
        L.oracle_tensor_octant.argtypes = [i64, i64, i64, dbl, dbl, dbl, dbl, pd]
        L.oracle_demag_direct_at.argtypes = [i64, i64, i64, pd, pd, pd, dbl, i64, pi64, pd]
        for f in (L.oracle_newell, L.oracle_far, L.oracle_tensor_at, L.oracle_tensor_many, L.oracle_tensor_octant,
                  L.oracle_demag_direct_at):
            f.restype = None
        _lib = L
    return _lib
