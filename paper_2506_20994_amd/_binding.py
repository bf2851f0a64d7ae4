"""ctypes binding of libsem.so.  Argument marshalling only."""
import ctypes
import os
import weakref

import torch

__all__ = ["SemError", "SEM_F64", "SEM_F32", "SEM_BF16", "SEM_OK", "SEM_NOT_CONVERGED",
           "SEM_FELL_BACK", "SEM_EINVAL", "SEM_EUNSUPPORTED_LX", "SEM_EHIP", "SEM_EBREAKDOWN",
           "SEM_ENOMEM", "SEM_EGEOMETRY", "lib", "lib_path", "sem_create", "sem_destroy",
           "sem_sync", "sem_gll", "sem_box_mesh", "sem_box_mesh_dirichlet", "sem_geometry", "sem_scatter",
           "sem_ax_diag", "sem_fourier", "sem_convert", "sem_ax", "sem_ax_helmholtz", "sem_gs_setup",
           "sem_gs_destroy", "sem_gs_info", "sem_gs_dirichlet_count", "sem_gs", "sem_gs_mult", "Context", "GsPlan",
           "dtype_code", "EXPORTS", "sem_gs_owner", "sem_remove_mean", "sem_remove_mean_static", "sem_cg_setup",
           "sem_cg_destroy", "sem_cg_solve", "SemOperator", "SemSolveOpts", "SemSolveStats",
           "CgSolver", "SEM_SOLVE_F64", "SEM_SOLVE_F32_IR", "SEM_SOLVE_BF16_IR",
           "LearnedPrecond", "sem_lp_create", "sem_lp_destroy", "sem_lp_set", "sem_lp_get",
           "sem_lp_set_step", "sem_lp_get_step", "sem_lp_bind", "sem_lp_samples", "sem_lp_forward",
           "sem_lp_gradients", "sem_lp_adam", "sem_lp_set_metric", "sem_lp_set_jacobi_base", "sem_lp_set_linear", "sem_lp_train_step", "sem_lp_apply", "sem_lp_apply_unique", "sem_lp_save", "sem_lp_load", "sem_lp_set_block", "LP_SLOTS", "lp_slots", "lp_sizes", "sem_lp_lx", "sem_lp_set_product",
           "SEM_LP_IN", "SEM_LP_IN_PAD", "SEM_LP_HIDDEN", "SEM_LP_OUT", "SemMgOpts", "Multigrid",
           "sem_mg_create", "sem_mg_destroy", "sem_mg_levels", "sem_mg_level_info", "sem_mg_set_lmax",
           "sem_mg_apply", "sem_mg_set_graphs", "sem_ax_set_variant", "sem_ax_get_variant", "sem_ax_tune", "sem_ax_tune_on",
           "SEM_AX_DEFAULT", "SEM_AX_COLUMN", "SEM_AX_COLUMN_PF", "SEM_AX_SLICE", "SEM_AX_3D", "SEM_AX_WAVE", "SEM_AX_VARIANTS", "sem_lp_snapshot", "sem_lp_reference_block"]

SEM_LP_IN, SEM_LP_IN_PAD, SEM_LP_HIDDEN, SEM_LP_OUT = 518, 528, 256, 512      # lx = 8


def lp_sizes(lx):
    """(outputs n = lx^3, inputs n + 6, padded feature width) of a network for lx"""
    n = lx ** 3
    return n, n + 6, (n + 6 + 15) // 16 * 16


def lp_slots(lx=8, hidden=256):
    """slot -> shape of the float32 array it holds (parameters; +6 m, +12 v, +18 grads)"""
    n, ni, _ = lp_sizes(lx)
    h = hidden
    return [(h, ni), (h,), (h, h), (h,), (n, h), (n,)]


LP_SLOTS = lp_slots(8)

SEM_SOLVE_F64, SEM_SOLVE_F32_IR, SEM_SOLVE_BF16_IR = 0, 1, 2
SEM_AX_DEFAULT, SEM_AX_COLUMN, SEM_AX_COLUMN_PF, SEM_AX_SLICE, SEM_AX_3D, SEM_AX_WAVE = -1, 0, 1, 2, 3, 4
SEM_AX_VARIANTS = 5


class SemOperator(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in
                ("dx", "dy", "dz", "dxt", "dyt", "dzt", "h1", "g11", "g22", "g33", "g12", "g13",
                 "g23")] + [("nel", ctypes.c_int64), ("lx", ctypes.c_int), ("h2b", ctypes.c_void_p)]


class SemSolveOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("maxit", ctypes.c_int), ("precision", ctypes.c_int),
                ("inner_tol", ctypes.c_double), ("inner_maxit", ctypes.c_int),
                ("max_outer", ctypes.c_int), ("check_every", ctypes.c_int),
                ("learned", ctypes.c_void_p), ("ir_mode", ctypes.c_int), ("delta", ctypes.c_double),
                ("mg", ctypes.c_void_p)]


class SemMgOpts(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("amp", ctypes.c_double), ("dirichlet", ctypes.c_int),
                ("h2", ctypes.c_double), ("degree", ctypes.c_int), ("lo", ctypes.c_double),
                ("hi", ctypes.c_double), ("n_coarse", ctypes.c_int), ("lanczos_steps", ctypes.c_int),
                ("fine_bf16", ctypes.c_int), ("galerkin", ctypes.c_int)]


class SemSolveStats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("outer", ctypes.c_int), ("relres", ctypes.c_double),
                ("relres_hist", ctypes.c_double * 64), ("converged", ctypes.c_int),
                ("breakdown", ctypes.c_int), ("jacobi_steps", ctypes.c_int),
                ("fell_back", ctypes.c_int)]

    def as_dict(self):
        return {"iterations": self.iterations, "outer": self.outer, "relres": self.relres,
                "relres_hist": list(self.relres_hist[:self.outer]),
                "converged": bool(self.converged), "breakdown": bool(self.breakdown),
                "jacobi_steps": self.jacobi_steps, "fell_back": bool(self.fell_back)}

SEM_F64, SEM_F32, SEM_BF16 = 0, 1, 2
SEM_OK, SEM_NOT_CONVERGED, SEM_FELL_BACK = 0, 1, 2
SEM_EINVAL, SEM_EUNSUPPORTED_LX, SEM_EHIP = -1, -2, -3
SEM_EBREAKDOWN, SEM_ENOMEM, SEM_EGEOMETRY = -4, -5, -6

_HERE = os.path.dirname(os.path.abspath(__file__))
lib_path = os.path.join(_HERE, "libsem.so")

_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_int = ctypes.c_int
_dbl = ctypes.c_double
_pdbl = ctypes.POINTER(ctypes.c_double)
_pi64 = ctypes.POINTER(ctypes.c_int64)

# name -> (restype, argtypes); the exported C ABI
EXPORTS = {
    "sem_create": (_int, [ctypes.POINTER(_vp), _vp]),
    "sem_destroy": (_int, [_vp]),
    "sem_set_stream": (_int, [_vp, _vp]),
    "sem_last_error": (ctypes.c_char_p, [_vp]),
    "sem_sync": (_int, [_vp]),
    "sem_gll": (_int, [_int, _pdbl, _pdbl, _pdbl, _pdbl]),
    "sem_box_mesh": (_int, [_vp, _int, _int, _dbl, _vp, _vp, _vp, _vp]),
    "sem_box_mesh_dirichlet": (_int, [_vp, _int, _int, _dbl, _vp, _vp, _vp, _vp]),
    "sem_geometry": (_int, [_vp, _vp, _vp, _vp, _i64, _int] + [_vp] * 7 + [_pdbl]),
    "sem_scatter": (_int, [_vp, _vp, _vp, _vp, _i64, _int]),
    "sem_ax_diag": (_int, [_vp, _vp, _vp, _vp] + [_vp] * 6 + [_i64, _int]),
    "sem_fourier": (_int, [_vp, _vp, _vp, _vp, _vp, _vp, _i64, _pi64, _pdbl, _pdbl, _int]),
    "sem_convert": (_int, [_vp, _vp, _int, _vp, _int, _i64]),
    "sem_ax": (_int, [_vp, _vp, _vp] + [_vp] * 6 + [_vp] * 7 + [_i64, _int, _int, _int]),
    "sem_ax_helmholtz": (_int, [_vp, _vp, _vp] + [_vp] * 6 + [_vp] * 7 + [_vp, _i64, _int, _int, _int]),
    "sem_gs_setup": (_int, [_vp, _pi64, _i64, ctypes.POINTER(_vp)]),
    "sem_gs_destroy": (_int, [_vp]),
    "sem_gs_info": (_int, [_vp, _pi64, _pi64]),
    "sem_gs_dirichlet_count": (_int, [_vp, _pi64]),
    "sem_gs": (_int, [_vp, _vp, _int]),
    "sem_gs_mult": (_int, [_vp, _vp]),
    "sem_gs_owner": (_int, [_vp, _vp]),
    "sem_remove_mean": (_int, [_vp, _vp]),
    "sem_remove_mean_static": (_int, [_vp, _vp]),
    "sem_cg_setup": (_int, [_vp, _vp, _vp, _vp, ctypes.POINTER(_vp)]),
    "sem_cg_destroy": (_int, [_vp]),
    "sem_cg_solve": (_int, [_vp, _vp, _vp, _vp, _vp]),
    "sem_lp_create": (_int, [_vp, _i64, ctypes.POINTER(_vp)]),
    "sem_lp_create_lx": (_int, [_vp, _int, _int, _i64, ctypes.POINTER(_vp)]),
    "sem_lp_lx": (_int, [_vp, ctypes.POINTER(_int), ctypes.POINTER(_int)]),
    "sem_lp_set_product": (_int, [_vp, _int]),
    "sem_lp_destroy": (_int, [_vp]),
    "sem_lp_set": (_int, [_vp, _int, ctypes.POINTER(ctypes.c_float), _i64]),
    "sem_lp_get": (_int, [_vp, _int, ctypes.POINTER(ctypes.c_float), _i64]),
    "sem_lp_set_step": (_int, [_vp, _i64]),
    "sem_lp_get_step": (_int, [_vp, _pi64]),
    "sem_lp_bind": (_int, [_vp, _vp, _vp]),
    "sem_lp_samples": (_int, [_vp, _vp, _vp, _vp, _i64, _vp, _vp, _i64]),
    "sem_lp_forward": (_int, [_vp, _vp, _i64, _vp]),
    "sem_lp_gradients": (_int, [_vp, _vp, _vp, _i64, ctypes.POINTER(ctypes.c_float)]),
    "sem_lp_adam": (_int, [_vp, _dbl, _dbl, _dbl, _dbl]),
    "sem_lp_train_step": (_int, [_vp, _vp, _vp, _vp, _i64, _dbl, _vp]),
    "sem_lp_apply": (_int, [_vp, _vp, _vp, _int]),
    "sem_lp_apply_unique": (_int, [_vp, _vp, _vp, _int]),
    "sem_lp_save": (_int, [_vp, ctypes.c_char_p]),
    "sem_lp_set_block": (_int, [_vp, _vp, _i64]),
    "sem_lp_load": (_int, [_vp, ctypes.c_char_p]),
    "sem_lp_set_metric": (_int, [_vp, _dbl]),
    "sem_lp_set_jacobi_base": (_int, [_vp, _int]),
    "sem_lp_set_linear": (_int, [_vp, _int]),
    "sem_lp_snapshot": (_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _i64, _vp, _vp, _i64]),
    "sem_lp_reference_block": (_int, [_vp, _int, _pdbl]),
    "sem_ax_set_variant": (_int, [_vp, _int, _int]),
    "sem_ax_get_variant": (_int, [_vp, _int, ctypes.POINTER(_int)]),
    "sem_ax_tune": (_int, [_vp, _int, _i64, _int, _pdbl, ctypes.POINTER(_int)]),
    "sem_ax_tune_on": (_int, [_vp, _vp, _vp] + [_vp] * 6 + [_vp] * 7 + [_i64, _int, _int, _pdbl, ctypes.POINTER(_int)]),
    "sem_mg_create": (_int, [_vp, _vp, _vp, _vp, ctypes.POINTER(_vp)]),
    "sem_mg_destroy": (_int, [_vp]),
    "sem_mg_levels": (_int, [_vp, ctypes.POINTER(_int)]),
    "sem_mg_level_info": (_int, [_vp, _int, ctypes.POINTER(_int), ctypes.POINTER(_int), _pi64, _pdbl, _pdbl]),
    "sem_mg_set_lmax": (_int, [_vp, _int, _dbl]),
    "sem_mg_apply": (_int, [_vp, _vp, _vp, _int]),
    "sem_mg_set_graphs": (_int, [_vp, _int]),
}

_LIB = None


def lib():
    """The loaded libsem.so; raises if it is not built."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(lib_path):
            raise ImportError(f"{lib_path} is not built; run python -m paper_2506_20994_amd.build")
        L = ctypes.CDLL(lib_path)
        for name, (res, args) in EXPORTS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _LIB = L
    return _LIB


class SemError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"[{code}] {msg}")
        self.code = code


def _check(rc, ctx_handle=None):
    if rc < 0:
        msg = lib().sem_last_error(ctx_handle)
        raise SemError(rc, msg.decode() if msg else "")
    return rc


_TORCH_CODES = {torch.float64: SEM_F64, torch.float32: SEM_F32, torch.bfloat16: SEM_BF16}


def dtype_code(t):
    return _TORCH_CODES[t.dtype]


def _ptr(t):
    """Device pointer of a contiguous GPU tensor (None -> NULL)."""
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if not t.is_cuda:
        raise ValueError("expected a GPU tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return t.data_ptr()


class Context:
    """Owns a sem_ctx_t; launches on torch's current stream at each call.
    Closing it first closes every plan, solver and network made from it."""

    def __init__(self):
        h = _vp()
        _check(lib().sem_create(ctypes.byref(h), _vp(torch.cuda.current_stream().cuda_stream)))
        self.handle = h
        self._children = weakref.WeakSet()

    def bind(self):
        if not self.handle:
            raise SemError(SEM_EINVAL, "context is closed")
        lib().sem_set_stream(self.handle, _vp(torch.cuda.current_stream().cuda_stream))
        return self.handle

    def adopt(self, child):
        self._children.add(child)
        return child

    def close(self):
        if self.handle:
            for c in list(self._children):
                c.close()
            lib().sem_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class GsPlan:
    def __init__(self, ctx, handle):
        self.ctx, self.handle = ctx, handle
        ctx.adopt(self)

    def close(self):
        if self.handle:
            lib().sem_gs_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sem_create():
    return Context()


def sem_destroy(ctx):
    ctx.close()


def sem_sync(ctx):
    _check(lib().sem_sync(ctx.bind()), ctx.handle)


def sem_gll(lx):
    """(xi, w, dx, dxt) as float64 numpy arrays (host)."""
    import numpy as np
    xi, w = np.empty(lx), np.empty(lx)
    dx, dxt = np.empty((lx, lx)), np.empty((lx, lx))
    c = lambda a: a.ctypes.data_as(_pdbl)  # noqa: E731
    _check(lib().sem_gll(lx, c(xi), c(w), c(dx), c(dxt)))
    return xi, w, dx, dxt


def sem_box_mesh(ctx, n, lx, amp, x=None, y=None, z=None, ids=None):
    h = ctx.bind()
    _check(lib().sem_box_mesh(h, n, lx, float(amp), _ptr(x), _ptr(y), _ptr(z), _ptr(ids)), h)


def sem_box_mesh_dirichlet(ctx, n, lx, amp, x=None, y=None, z=None, ids=None):
    h = ctx.bind()
    _check(lib().sem_box_mesh_dirichlet(h, n, lx, float(amp), _ptr(x), _ptr(y), _ptr(z), _ptr(ids)), h)


def sem_geometry(ctx, x, y, z, nel, lx, g11, g22, g33, g12, g13, g23, bm=None):
    """Returns min det J."""
    h = ctx.bind()
    dmin = _dbl(0.0)
    _check(lib().sem_geometry(h, _ptr(x), _ptr(y), _ptr(z), nel, lx, _ptr(g11), _ptr(g22),
                              _ptr(g33), _ptr(g12), _ptr(g13), _ptr(g23), _ptr(bm),
                              ctypes.byref(dmin)), h)
    return dmin.value


def sem_scatter(ctx, out_local, in_unique, ids, n_local=None):
    h = ctx.bind()
    n = out_local.numel() if n_local is None else n_local
    _check(lib().sem_scatter(h, _ptr(out_local), _ptr(in_unique), _ptr(ids), n,
                             dtype_code(out_local)), h)


def sem_ax_diag(ctx, d, dx, h1, g11, g22, g33, g12, g13, g23, nel, lx):
    h = ctx.bind()
    _check(lib().sem_ax_diag(h, _ptr(d), _ptr(dx), _ptr(h1), _ptr(g11), _ptr(g22), _ptr(g33),
                             _ptr(g12), _ptr(g13), _ptr(g23), nel, lx), h)


def sem_fourier(ctx, f, x, y, z, scale, k, amp, phase):
    """k: int64 numpy (m, 3); amp, phase: float64 numpy (m,)."""
    import numpy as np
    h = ctx.bind()
    k = np.ascontiguousarray(k, dtype=np.int64)
    amp = np.ascontiguousarray(amp, dtype=np.float64)
    phase = np.ascontiguousarray(phase, dtype=np.float64)
    _check(lib().sem_fourier(h, _ptr(f), _ptr(x), _ptr(y), _ptr(z), _ptr(scale), f.numel(),
                             k.ctypes.data_as(_pi64), amp.ctypes.data_as(_pdbl),
                             phase.ctypes.data_as(_pdbl), len(amp)), h)


def sem_convert(ctx, dst, src):
    h = ctx.bind()
    if dst.numel() != src.numel():
        raise ValueError("size mismatch")
    _check(lib().sem_convert(h, _ptr(dst), dtype_code(dst), _ptr(src), dtype_code(src),
                             dst.numel()), h)


def sem_ax(ctx, w, u, dx, dy, dz, dxt, dyt, dzt, h1, g11, g22, g33, g12, g13, g23, nel, lx,
           field_dtype=None, out_dtype=None):
    h = ctx.bind()
    fd = dtype_code(u) if field_dtype is None else field_dtype
    od = dtype_code(w) if out_dtype is None else out_dtype
    _check(lib().sem_ax(h, _ptr(w), _ptr(u), _ptr(dx), _ptr(dy), _ptr(dz), _ptr(dxt), _ptr(dyt),
                        _ptr(dzt), _ptr(h1), _ptr(g11), _ptr(g22), _ptr(g33), _ptr(g12),
                        _ptr(g13), _ptr(g23), nel, lx, fd, od), h)


def sem_ax_helmholtz(ctx, w, u, dx, dy, dz, dxt, dyt, dzt, h1, g11, g22, g33, g12, g13, g23, h2b, nel,
                     lx, field_dtype=None, out_dtype=None):
    h = ctx.bind()
    fd = dtype_code(u) if field_dtype is None else field_dtype
    od = dtype_code(w) if out_dtype is None else out_dtype
    _check(lib().sem_ax_helmholtz(h, _ptr(w), _ptr(u), _ptr(dx), _ptr(dy), _ptr(dz), _ptr(dxt), _ptr(dyt),
                                  _ptr(dzt), _ptr(h1), _ptr(g11), _ptr(g22), _ptr(g33), _ptr(g12),
                                  _ptr(g13), _ptr(g23), _ptr(h2b), nel, lx, fd, od), h)


def sem_gs_setup(ctx, ids_host):
    """ids_host: int64 numpy array (host) of global ids."""
    import numpy as np
    ids_host = np.ascontiguousarray(ids_host, dtype=np.int64).ravel()
    h = ctx.bind()
    out = _vp()
    _check(lib().sem_gs_setup(h, ids_host.ctypes.data_as(_pi64), ids_host.size,
                              ctypes.byref(out)), h)
    return GsPlan(ctx, out)


def sem_gs_destroy(gs):
    gs.close()


def sem_gs_info(gs):
    nu, ns = ctypes.c_int64(0), ctypes.c_int64(0)
    _check(lib().sem_gs_info(gs.handle, ctypes.byref(nu), ctypes.byref(ns)), gs.ctx.handle)
    return nu.value, ns.value


def sem_gs_dirichlet_count(gs):
    nd = ctypes.c_int64(0)
    _check(lib().sem_gs_dirichlet_count(gs.handle, ctypes.byref(nd)), gs.ctx.handle)
    return nd.value


def sem_gs(gs, u):
    gs.ctx.bind()
    _check(lib().sem_gs(gs.handle, _ptr(u), dtype_code(u)), gs.ctx.handle)


def sem_gs_mult(gs, mult):
    gs.ctx.bind()
    _check(lib().sem_gs_mult(gs.handle, _ptr(mult)), gs.ctx.handle)


def sem_gs_owner(gs, wgt):
    gs.ctx.bind()
    _check(lib().sem_gs_owner(gs.handle, _ptr(wgt)), gs.ctx.handle)


def sem_remove_mean(gs, x):
    gs.ctx.bind()
    _check(lib().sem_remove_mean(gs.handle, _ptr(x)), gs.ctx.handle)


def sem_remove_mean_static(gs, x):
    gs.ctx.bind()
    _check(lib().sem_remove_mean_static(gs.handle, _ptr(x)), gs.ctx.handle)


class CgSolver:
    def __init__(self, ctx, handle, keep):
        self.ctx, self.handle, self._keep = ctx, handle, keep
        ctx.adopt(self)

    def close(self):
        if self.handle:
            lib().sem_cg_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _opts(tol=1e-10, maxit=0, precision=SEM_SOLVE_F64, inner_tol=0.0, inner_maxit=0,
          max_outer=0, check_every=0, learned=None, ir_mode=0, delta=0.0, mg=None):
    return SemSolveOpts(tol, maxit, precision, inner_tol, inner_maxit, max_outer, check_every,
                        learned.handle if learned is not None else None, ir_mode, delta,
                        mg.handle if mg is not None else None)


def sem_cg_setup(ctx, gs, D, h1, G, nel, lx, h2b=None, **opts):
    """D = (dx, dy, dz, dxt, dyt, dzt), G = (g11, g22, g33, g12, g13, g23): float64
    device tensors; h2b (optional) the Helmholtz mass term h2 * bm.  opts: see
    SemSolveOpts (precision fixed here)."""
    A = SemOperator(*[_ptr(t) for t in D], _ptr(h1), *[_ptr(t) for t in G], nel, lx, _ptr(h2b))
    o = _opts(**opts)
    h = ctx.bind()
    out = _vp()
    _check(lib().sem_cg_setup(h, gs.handle, ctypes.byref(A), ctypes.byref(o), ctypes.byref(out)), h)
    return CgSolver(ctx, out, (D, h1, G, gs, h2b))


def sem_cg_destroy(cg):
    cg.close()


def sem_cg_solve(cg, x, b, **opts):
    """Returns (status, stats dict).  Raises on negative status."""
    o = _opts(**opts)
    st = SemSolveStats()
    cg.ctx.bind()
    rc = lib().sem_cg_solve(cg.handle, _ptr(x), _ptr(b), ctypes.byref(o), ctypes.byref(st))
    _check(rc, cg.ctx.handle)
    return rc, st.as_dict()


class LearnedPrecond:
    def __init__(self, ctx, handle, max_rows, lx=8, hidden=256):
        self.ctx, self.handle, self.max_rows, self.lx, self.hidden = ctx, handle, max_rows, lx, hidden
        self.n_out, self.n_in, self.n_in_pad = lp_sizes(lx)
        self._bound = None
        ctx.adopt(self)

    def close(self):
        if self.handle:
            lib().sem_lp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sem_lp_create(ctx, max_rows, lx=8, hidden=256):
    """A network for elements of lx^3 nodes with hidden layers of width
    `hidden` (sem_lp_create_lx)."""
    out = _vp()
    h = ctx.bind()
    _check(lib().sem_lp_create_lx(h, int(lx), int(hidden), int(max_rows), ctypes.byref(out)), h)
    return LearnedPrecond(ctx, out, max_rows, lx, hidden)


def sem_lp_set_product(lp, kind):
    """0 automatic, 1 weight-stationary (lx = 8), 2 general MFMA product"""
    _check(lib().sem_lp_set_product(lp.handle, int(kind)), lp.ctx.handle)


def sem_lp_lx(lp):
    """(lx, hidden width) of the network"""
    v, hd = _int(0), _int(0)
    _check(lib().sem_lp_lx(lp.handle, ctypes.byref(v), ctypes.byref(hd)), lp.ctx.handle)
    return v.value, hd.value


def sem_lp_destroy(lp):
    lp.close()


def sem_lp_set(lp, which, values):
    import numpy as np
    a = np.ascontiguousarray(values, dtype=np.float32).ravel()
    _check(lib().sem_lp_set(lp.handle, which, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                            a.size), lp.ctx.handle)


def sem_lp_get(lp, which):
    import numpy as np
    shape = lp_slots(lp.lx, lp.hidden)[which % 6]
    a = np.empty(shape, dtype=np.float32)
    _check(lib().sem_lp_get(lp.handle, which, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                            a.size), lp.ctx.handle)
    return a


def sem_lp_set_step(lp, step):
    _check(lib().sem_lp_set_step(lp.handle, int(step)), lp.ctx.handle)


def sem_lp_get_step(lp):
    s = ctypes.c_int64(0)
    _check(lib().sem_lp_get_step(lp.handle, ctypes.byref(s)), lp.ctx.handle)
    return s.value


def sem_lp_bind(lp, D, h1, G, nel, lx, gs):
    A = SemOperator(*[_ptr(t) for t in D], _ptr(h1), *[_ptr(t) for t in G], nel, lx)
    lp.ctx.bind()
    _check(lib().sem_lp_bind(lp.handle, ctypes.byref(A), gs.handle), lp.ctx.handle)
    lp._bound = (D, h1, G, gs)


def sem_lp_samples(lp, r, err, elems, X, T, row0):
    lp.ctx.bind()
    _check(lib().sem_lp_samples(lp.handle, _ptr(r), _ptr(err), _ptr(elems), elems.numel(),
                                _ptr(X), _ptr(T), int(row0)), lp.ctx.handle)


def sem_lp_forward(lp, X, Y):
    lp.ctx.bind()
    _check(lib().sem_lp_forward(lp.handle, _ptr(X), X.shape[0], _ptr(Y)), lp.ctx.handle)


def sem_lp_gradients(lp, X, T):
    loss = ctypes.c_float(0.0)
    lp.ctx.bind()
    _check(lib().sem_lp_gradients(lp.handle, _ptr(X), _ptr(T), X.shape[0], ctypes.byref(loss)),
           lp.ctx.handle)
    return loss.value


def sem_lp_adam(lp, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    lp.ctx.bind()
    _check(lib().sem_lp_adam(lp.handle, lr, beta1, beta2, eps), lp.ctx.handle)


def sem_lp_train_step(lp, X, T, rows, lr, loss_dev):
    lp.ctx.bind()
    _check(lib().sem_lp_train_step(lp.handle, _ptr(X), _ptr(T), _ptr(rows), rows.numel(), lr,
                                   _ptr(loss_dev)), lp.ctx.handle)


def sem_lp_apply(lp, z, r):
    lp.ctx.bind()
    _check(lib().sem_lp_apply(lp.handle, _ptr(z), _ptr(r), dtype_code(r)), lp.ctx.handle)


def sem_lp_set_block(lp, W):
    import numpy as np
    a = np.ascontiguousarray(W, dtype=np.float32).ravel()
    lp.ctx.bind()
    _check(lib().sem_lp_set_block(lp.handle, a.ctypes.data, a.size), lp.ctx.handle)


def sem_lp_save(lp, path):
    lp.ctx.bind()
    _check(lib().sem_lp_save(lp.handle, os.fsencode(path)), lp.ctx.handle)


def sem_lp_load(lp, path):
    lp.ctx.bind()
    _check(lib().sem_lp_load(lp.handle, os.fsencode(path)), lp.ctx.handle)


def sem_lp_apply_unique(lp, z, r):
    lp.ctx.bind()
    _check(lib().sem_lp_apply_unique(lp.handle, _ptr(z), _ptr(r), dtype_code(r)), lp.ctx.handle)


def sem_lp_set_metric(lp, mu):
    _check(lib().sem_lp_set_metric(lp.handle, float(mu)), lp.ctx.handle)


def sem_lp_set_jacobi_base(lp, on):
    _check(lib().sem_lp_set_jacobi_base(lp.handle, int(bool(on))), lp.ctx.handle)


def sem_lp_set_linear(lp, on):
    _check(lib().sem_lp_set_linear(lp.handle, int(bool(on))), lp.ctx.handle)


class Multigrid:
    def __init__(self, ctx, handle, keep):
        self.ctx, self.handle, self._keep = ctx, handle, keep
        ctx.adopt(self)

    def close(self):
        if self.handle:
            self.ctx.bind()
            lib().sem_mg_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sem_mg_create(ctx, gs, D, G, nel, lx, n, amp, dirichlet=False, h2=0.0, h2b=None, degree=0, lo=0.0,
                  hi=0.0, n_coarse=0, lanczos_steps=0, fine_bf16=False, galerkin=False):
    """The multigrid hierarchy of the n^3 box operator (D, G float64 device
    tensors as for sem_cg_setup, h1 = 1; h2b = h2 * bm for a Helmholtz operator)."""
    A = SemOperator(*[_ptr(t) for t in D], None, *[_ptr(t) for t in G], nel, lx, _ptr(h2b))
    o = SemMgOpts(n, amp, int(bool(dirichlet)), h2, degree, lo, hi, n_coarse, lanczos_steps, int(bool(fine_bf16)),
                  int(bool(galerkin)))
    h = ctx.bind()
    out = _vp()
    _check(lib().sem_mg_create(h, gs.handle, ctypes.byref(A), ctypes.byref(o), ctypes.byref(out)), h)
    return Multigrid(ctx, out, (D, G, gs, h2b))


def sem_mg_destroy(mg):
    mg.close()


def sem_mg_levels(mg):
    c = _int(0)
    _check(lib().sem_mg_levels(mg.handle, ctypes.byref(c)), mg.ctx.handle)
    return c.value


def sem_mg_level_info(mg, level):
    """(n, lx, n_unique, lmax, amplitude) of a level"""
    n, lx, nu, lm, am = _int(0), _int(0), _i64(0), _dbl(0.0), _dbl(0.0)
    _check(lib().sem_mg_level_info(mg.handle, level, ctypes.byref(n), ctypes.byref(lx), ctypes.byref(nu),
                                   ctypes.byref(lm), ctypes.byref(am)), mg.ctx.handle)
    return n.value, lx.value, nu.value, lm.value, am.value


def sem_mg_set_lmax(mg, level, lmax):
    _check(lib().sem_mg_set_lmax(mg.handle, level, float(lmax)), mg.ctx.handle)


def sem_mg_set_graphs(mg, on):
    _check(lib().sem_mg_set_graphs(mg.handle, int(bool(on))), mg.ctx.handle)


def sem_mg_apply(mg, z, r):
    mg.ctx.bind()
    _check(lib().sem_mg_apply(mg.handle, _ptr(z), _ptr(r), dtype_code(r)), mg.ctx.handle)


def sem_lp_snapshot(lp, x, xstar, b, r_out, err_out, elems, X, T, row0):
    lp.ctx.bind()
    _check(lib().sem_lp_snapshot(lp.handle, _ptr(x), _ptr(xstar), _ptr(b), _ptr(r_out), _ptr(err_out),
                                 _ptr(elems), elems.numel(), _ptr(X), _ptr(T), row0), lp.ctx.handle)


def sem_lp_reference_block(ctx, lx=8):
    """kappa A_ee^-1 of the undeformed element (host float64, (lx^3, lx^3))"""
    import numpy as np
    W = np.empty((lx ** 3, lx ** 3))
    h = ctx.bind()
    _check(lib().sem_lp_reference_block(h, lx, W.ctypes.data_as(_pdbl)), h)
    return W


def sem_ax_set_variant(ctx, lx, variant):
    h = ctx.bind()
    _check(lib().sem_ax_set_variant(h, lx, variant), h)


def sem_ax_get_variant(ctx, lx):
    v = _int(0)
    h = ctx.bind()
    _check(lib().sem_ax_get_variant(h, lx, ctypes.byref(v)), h)
    return v.value


def sem_ax_tune(ctx, lx, nel, reps=20):
    """Times the float64 operator's variants at lx on nel elements and selects
    the fastest; returns (best, [us per variant, -1 where none])."""
    us = (ctypes.c_double * SEM_AX_VARIANTS)()
    best = _int(0)
    h = ctx.bind()
    _check(lib().sem_ax_tune(h, lx, nel, reps, us, ctypes.byref(best)), h)
    return best.value, list(us)


def sem_ax_tune_on(ctx, w, u, dx, dy, dz, dxt, dyt, dzt, h1, g11, g22, g33, g12, g13, g23, nel, lx, reps=20):
    """Times the float64 operator's variants on these operands (w is
    overwritten) and selects the fastest; returns (best, [us per variant])."""
    us = (ctypes.c_double * SEM_AX_VARIANTS)()
    best = _int(0)
    h = ctx.bind()
    _check(lib().sem_ax_tune_on(h, _ptr(w), _ptr(u), _ptr(dx), _ptr(dy), _ptr(dz), _ptr(dxt), _ptr(dyt),
                                _ptr(dzt), _ptr(h1), _ptr(g11), _ptr(g22), _ptr(g33), _ptr(g12), _ptr(g13),
                                _ptr(g23), nel, lx, reps, us, ctypes.byref(best)), h)
    return best.value, list(us)
