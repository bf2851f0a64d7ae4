"""ctypes loader for oracle/ax_ref.c (the plain C loop nest, used to time the
CPU baseline).  Test infrastructure only.  ``build()`` compiles it with gcc."""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ax_ref.c")
LIB = os.path.join(HERE, "liboracle_ax.so")


def build():
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", SRC, "-o", LIB])
    return LIB


def _lib():
    if not os.path.exists(LIB):
        build()
    lib = ctypes.CDLL(LIB)
    dp = ctypes.POINTER(ctypes.c_double)
    lib.oracle_ax_ref.argtypes = [dp] * 15 + [ctypes.c_int64, ctypes.c_int]
    lib.oracle_ax_ref.restype = None
    lib.oracle_num_threads.restype = ctypes.c_int
    return lib


def _p(a):
    if a is None:
        return ctypes.cast(None, ctypes.POINTER(ctypes.c_double))
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def ax_ref(u, dx, dy, dz, dxt, dyt, dzt, h1, g11, g22, g33, g12, g13, g23):
    lib = _lib()
    w = np.empty_like(u)
    lib.oracle_ax_ref(_p(w), _p(u), _p(dx), _p(dy), _p(dz), _p(dxt), _p(dyt), _p(dzt),
                      _p(h1), _p(g11), _p(g22), _p(g33), _p(g12), _p(g13), _p(g23),
                      u.shape[0], u.shape[1])
    return w


def num_threads():
    return _lib().oracle_num_threads()
