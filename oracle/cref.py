"""ctypes loader for oracle/sem_ref.c: the plain-C statement of the path (box
coordinates, geometry, element operator, diagonal, Fourier source, gather,
Jacobi-PCG).  Test infrastructure only: it times the CPU baseline and gives
reference solutions on boxes the numpy oracle is too slow for.  ``build()``
compiles it with gcc; every function is pinned against the numpy oracle in
tests/test_oracle_cref.py.
"""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sem_ref.c")
LIB = os.path.join(HERE, "liboracle_sem.so")

_dp = ctypes.POINTER(ctypes.c_double)
_lp = ctypes.POINTER(ctypes.c_int64)
_i64 = ctypes.c_int64
_int = ctypes.c_int
_dbl = ctypes.c_double
_handle = None


def build():
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", SRC, "-o", LIB, "-lm"])
    return LIB


def _lib():
    global _handle
    if _handle is not None:
        return _handle
    if not os.path.exists(LIB):
        build()
    lib = ctypes.CDLL(LIB)
    lib.oracle_box_coords.argtypes = [_int, _int, _dbl, _dp, _dp, _dp, _dp]
    lib.oracle_box_coords.restype = None
    lib.oracle_geometry.argtypes = [_dp, _dp, _dp, _i64, _int, _dp, _dp] + [_dp] * 7
    lib.oracle_geometry.restype = _dbl
    lib.oracle_ax.argtypes = [_dp, _dp, _dp, _dp] + [_dp] * 7 + [_i64, _int]
    lib.oracle_ax.restype = None
    lib.oracle_diag.argtypes = [_dp, _dp, _dp] + [_dp] * 7 + [_i64, _int]
    lib.oracle_diag.restype = None
    lib.oracle_fourier.argtypes = [_dp, _dp, _dp, _dp, _i64, _lp, _dp, _dp, _int]
    lib.oracle_fourier.restype = None
    lib.oracle_gather.argtypes = [_dp, _dp, _lp, _i64, _i64]
    lib.oracle_gather.restype = None
    lib.oracle_pcg.argtypes = ([_dp, _dp, _lp, _i64, _int, _i64, _dp, _dp] + [_dp] * 7
                               + [_dbl, _int, _int, _dp])
    lib.oracle_pcg.restype = _int
    lib.oracle_apply_assembled.argtypes = [_dp, _dp, _lp, _i64, _int, _i64, _dp, _dp] + [_dp] * 7
    lib.oracle_apply_assembled.restype = _int
    lib.oracle_num_threads.restype = _int
    lib.oracle_set_threads.argtypes = [_int]
    lib.oracle_set_threads.restype = None
    _handle = lib
    return lib


def _p(a):
    if a is None:
        return ctypes.cast(None, _dp)
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def _pl(a):
    assert a.dtype == np.int64 and a.flags.c_contiguous
    return a.ctypes.data_as(_lp)


def _c(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def box_coords(n, lx, amp, xi):
    """x, y, z (each (n^3, lx, lx, lx)) of the deformed periodic box."""
    xi = _c(xi)
    out = [np.empty((n ** 3, lx, lx, lx)) for _ in range(3)]
    _lib().oracle_box_coords(n, lx, float(amp), _p(xi), *(_p(a) for a in out))
    return tuple(out)


def geometry(x, y, z, lx, Dh, w):
    """(G, B, min det J): G = (g11, g22, g33, g12, g13, g23)."""
    x, y, z, Dh, w = (_c(a) for a in (x, y, z, Dh, w))
    G = [np.empty_like(x) for _ in range(6)]
    B = np.empty_like(x)
    dmin = _lib().oracle_geometry(_p(x), _p(y), _p(z), x.shape[0], lx, _p(Dh), _p(w),
                                  *(_p(g) for g in G), _p(B))
    return tuple(G), B, dmin


def ax(u, Dh, h1, G, h2b=None):
    """w_e = A_e u_e (+ h2b u_e) on every element (u: (E, lx, lx, lx))."""
    u, Dh, h1, h2b = _c(u), _c(Dh), _c(h1), _c(h2b)
    G = [_c(g) for g in G]
    w = np.empty_like(u)
    _lib().oracle_ax(_p(w), _p(u), _p(Dh), _p(h1), *(_p(g) for g in G), _p(h2b),
                     u.shape[0], u.shape[1])
    return w


def diag(Dh, h1, G, h2b=None):
    Dh, h1, h2b = _c(Dh), _c(h1), _c(h2b)
    G = [_c(g) for g in G]
    d = np.empty_like(G[0])
    _lib().oracle_diag(_p(d), _p(Dh), _p(h1), *(_p(g) for g in G), _p(h2b),
                       G[0].shape[0], G[0].shape[1])
    return d


def fourier(x, y, z, k, amp, phase):
    x, y, z = _c(x), _c(y), _c(z)
    k = np.ascontiguousarray(k, dtype=np.int64)
    amp, phase = _c(amp), _c(phase)
    f = np.empty_like(x)
    _lib().oracle_fourier(_p(f), _p(x), _p(y), _p(z), x.size, _pl(k), _p(amp), _p(phase), len(amp))
    return f


def gather(u_local, ids, n_unique):
    u_local = _c(u_local)
    ids = np.ascontiguousarray(ids, dtype=np.int64)
    out = np.empty(n_unique)
    _lib().oracle_gather(_p(out), _p(u_local), _pl(ids), u_local.size, n_unique)
    return out


def pcg(b, ids, n_unique, Dh, h1, G, tol=1e-10, maxit=100000, project=True, h2b=None):
    """Jacobi-PCG on the assembled operator; returns (x, iterations, relres)."""
    b, Dh, h1, h2b = _c(b), _c(Dh), _c(h1), _c(h2b)
    G = [_c(g) for g in G]
    ids = np.ascontiguousarray(ids, dtype=np.int64)
    x = np.empty(n_unique)
    rel = ctypes.c_double(0.0)
    it = _lib().oracle_pcg(_p(x), _p(b), _pl(ids), G[0].shape[0], G[0].shape[1], n_unique,
                           _p(Dh), _p(h1), *(_p(g) for g in G), _p(h2b), float(tol), int(maxit),
                           int(bool(project)), ctypes.byref(rel))
    if it < 0:
        raise MemoryError("oracle_pcg: out of memory")
    return x, it, rel.value


def apply_assembled(x, ids, n_unique, Dh, h1, G, h2b=None):
    """A_G x (+ h2 B x) on unique vectors."""
    x, Dh, h1, h2b = _c(x), _c(Dh), _c(h1), _c(h2b)
    G = [_c(g) for g in G]
    ids = np.ascontiguousarray(ids, dtype=np.int64)
    y = np.empty(n_unique)
    if _lib().oracle_apply_assembled(_p(y), _p(x), _pl(ids), G[0].shape[0], G[0].shape[1],
                                     n_unique, _p(Dh), _p(h1), *(_p(g) for g in G), _p(h2b)) < 0:
        raise MemoryError("oracle_apply_assembled: out of memory")
    return y


def num_threads():
    return _lib().oracle_num_threads()


def set_threads(n):
    _lib().oracle_set_threads(int(n))


class BigBox:
    """The n^3 box (amplitude a, lx) of oracle.solve.BoxProblem assembled by
    the C statement, for sizes where the numpy oracle is too slow: periodic,
    or with u = 0 on the boundary (``dirichlet``); Poisson, or Helmholtz with
    the constant h2 (A + h2 B).  GLL data and ids come from the numpy oracle,
    everything else from sem_ref.c.  Only the periodic Poisson operator is
    singular: its right-hand sides and solutions are mean-free."""

    def __init__(self, n, lx, a, h1_unique=None, dirichlet=False, h2=None):
        from .gll import gll_nodes_weights, deriv_matrix
        from .mesh import global_ids, n_unique, global_ids_dirichlet, n_unique_dirichlet
        xi, w = gll_nodes_weights(lx - 1)
        self.n, self.lx, self.a = n, lx, a
        self.project = not dirichlet and h2 is None
        self.Dh = deriv_matrix(xi)
        self.coords = box_coords(n, lx, a, xi)
        self.G, self.B, self.min_detj = geometry(*self.coords, lx, self.Dh, w)
        ids = global_ids_dirichlet(n, lx) if dirichlet else global_ids(n, lx)
        self.ids = np.ascontiguousarray(ids, dtype=np.int64)
        self.nu = n_unique_dirichlet(n, lx) if dirichlet else n_unique(n, lx)
        self.h1 = None
        if h1_unique is not None:
            # scattered like any unique field: 0 on Dirichlet nodes
            self.h1 = np.where(self.ids >= 0, h1_unique[np.maximum(self.ids, 0)], 0.0)
        self.h2b = None if h2 is None else h2 * self.B

    def fourier_rhs(self, k, amp, phase, const=0.0):
        """b_G = Q^T (B (const + f)), mean removed on the singular operator."""
        f = fourier(*self.coords, k, amp, phase) + const
        b = gather(self.B * f, self.ids, self.nu)
        return b - b.mean() if self.project else b

    def pcg(self, b, tol=1e-10, maxit=100000):
        return pcg(b, self.ids, self.nu, self.Dh, self.h1, self.G, tol, maxit,
                   project=self.project, h2b=self.h2b)

    def apply(self, x):
        return apply_assembled(x, self.ids, self.nu, self.Dh, self.h1, self.G, h2b=self.h2b)
