"""Python binding of libpd, the gfx950 pressure solver for the staggered spectral semi-implicit DG
scheme of arXiv:1602.05806 (Section 2).

Argument marshalling only: every function forwards device pointers of torch tensors and the
current HIP stream to the C ABI declared in ``include/pd.h``; all arithmetic runs in the HIP
kernels of ``libpd.so``. There is no CPU fallback: importing this package fails if the library
has not been built (``python -c "import __graft_entry__ as g; g.build()"``).
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpd.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"libpd.so not found at {LIB_PATH}: build the HIP library first "
        "(make -C paper_1602_05806_amd/csrc, or __graft_entry__.build())")

# torch is loaded first so that libpd binds to the HIP runtime torch already uses (both carry the
# soname libamdhip64.so.7; loading libpd first would bring a second runtime into the process).
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)

# status codes, precisions, operators, configuration keys (mirrors include/pd.h)
PD_OK, PD_EINVAL, PD_ENOMEM, PD_EDEVICE, PD_ENOCONV, PD_EBREAKDOWN = 0, -1, -2, -3, -4, -5
PD_FP64, PD_FP32, PD_FP32_REFINE64 = 0, 1, 2
PD_OP_PRESSURE, PD_OP_VISCOUS = 0, 1
(PD_CFG_STEP_PREC, PD_CFG_P_RTOL, PD_CFG_V_RTOL, PD_CFG_MAXIT, PD_CFG_CONVECTION,
 PD_CFG_RU_FACTOR, PD_CFG_TIMING, PD_CFG_CHECK_EVERY, PD_CFG_KZ, PD_CFG_TILES_PER_WG,
 PD_CFG_PREFETCH, PD_CFG_TILE_VARIANT, PD_CFG_DEFER_X, PD_CFG_ONE_KERNEL,
 PD_CFG_EXPLICIT_VISC, PD_CFG_PRECOND) = range(16)
PD_BATCH_AUTOTUNE, PD_BATCH_RETUNE = 1, 2
PD_BCFG_CHUNK, PD_BCFG_GRAPH, PD_BCFG_RU_FACTOR, PD_BCFG_PRECOND = 0, 1, 2, 3
(PD_TAB_NODES, PD_TAB_WEIGHTS, PD_TAB_L, PD_TAB_C, PD_TAB_R, PD_TAB_PNULL, PD_TAB_PNULL_ODD,
 PD_TAB_PV, PD_TAB_PLAM) = range(9)
PD_TTAB_NODES, PD_TTAB_WEIGHTS, PD_TTAB_PSI0, PD_TTAB_PSI1, PD_TTAB_MV, PD_TTAB_AINV = range(6)

EXPORTED = ["pd_setup", "pd_destroy", "pd_last_error", "pd_sizes", "pd_nodes", "pd_table_1d", "pd_apply",
            "pd_cg_solve", "pd_rhs_div", "pd_project_velocity", "pd_project_null",
            "pd_l2_project", "pd_convect", "pd_step", "pd_configure", "pd_timing",
            "pd_l2_project_adjoint", "pd_rhs_div_adjoint", "pd_project_velocity_adjoint",
            "pd_convect_adjoint", "pd_step_adjoint", "pd_kinetic_energy", "pd_project_null_noalloc", "pd_step_st",
            "pd_time_table",
            "pd_batch_setup", "pd_batch_destroy", "pd_batch_last_error", "pd_batch_layout",
            "pd_batch_variants", "pd_batch_configure", "pd_batch_cg_solve"]


class pd_solve_info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("outer_iters", ctypes.c_int), ("status", ctypes.c_int),
                ("restarts", ctypes.c_int), ("fallback_iter", ctypes.c_int), ("reserved", ctypes.c_int),
                ("rel_res_recur", ctypes.c_double), ("rel_res_true", ctypes.c_double),
                ("ms", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_vp = ctypes.c_void_p
_lib.pd_setup.argtypes = [ctypes.POINTER(_vp), ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                          ctypes.POINTER(ctypes.c_double), ctypes.c_int, ctypes.c_double,
                          ctypes.c_double, ctypes.c_double, ctypes.c_uint, _vp]
_lib.pd_destroy.argtypes = [_vp]
_lib.pd_destroy.restype = None
_lib.pd_last_error.argtypes = [_vp]
_lib.pd_last_error.restype = ctypes.c_char_p
_lib.pd_sizes.argtypes = [_vp, ctypes.POINTER(ctypes.c_longlong),
                          ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(ctypes.c_int)]
_lib.pd_nodes.argtypes = [_vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
_lib.pd_table_1d.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
_lib.pd_apply.argtypes = [_vp, ctypes.c_int, ctypes.c_int, _vp, _vp, _vp]
_lib.pd_cg_solve.argtypes = [_vp, ctypes.c_int, ctypes.c_int, _vp, _vp, ctypes.c_double,
                             ctypes.c_int, ctypes.POINTER(pd_solve_info), _vp]
_lib.pd_rhs_div.argtypes = [_vp, ctypes.POINTER(_vp), _vp, _vp]
_lib.pd_project_velocity.argtypes = [_vp, _vp, ctypes.POINTER(_vp), _vp]
_lib.pd_project_null.argtypes = [_vp, ctypes.c_int, _vp, _vp]
_lib.pd_project_null_noalloc.argtypes = [_vp, ctypes.c_int, _vp, _vp]
_lib.pd_l2_project.argtypes = [_vp, ctypes.c_int, ctypes.c_int, _vp, _vp, _vp]
_lib.pd_convect.argtypes = [_vp, ctypes.POINTER(_vp), _vp]
_lib.pd_step.argtypes = [_vp, ctypes.POINTER(_vp), _vp, ctypes.POINTER(pd_solve_info), _vp]
_lib.pd_configure.argtypes = [_vp, ctypes.c_int, ctypes.c_double]
_lib.pd_timing.argtypes = [_vp, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                           ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(ctypes.c_double),
                           ctypes.c_int]
_lib.pd_l2_project_adjoint.argtypes = [_vp, ctypes.c_int, ctypes.c_int, _vp, _vp, _vp]
_lib.pd_rhs_div_adjoint.argtypes = [_vp, _vp, ctypes.POINTER(_vp), _vp]
_lib.pd_project_velocity_adjoint.argtypes = [_vp, ctypes.POINTER(_vp), _vp, _vp]
_lib.pd_convect_adjoint.argtypes = [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), _vp]
_lib.pd_step_adjoint.argtypes = [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                                 ctypes.POINTER(pd_solve_info), _vp]
_lib.pd_kinetic_energy.argtypes = [_vp, ctypes.POINTER(_vp), ctypes.c_double, ctypes.POINTER(_vp),
                                   ctypes.POINTER(ctypes.c_double), _vp]
_lib.pd_step_st.argtypes = [_vp, ctypes.c_int, ctypes.POINTER(_vp), _vp, ctypes.POINTER(pd_solve_info),
                            _vp]
_lib.pd_time_table.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
_lib.pd_batch_setup.argtypes = [ctypes.POINTER(_vp), ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int),
                                ctypes.c_double, ctypes.c_uint, _vp]
_lib.pd_batch_destroy.argtypes = [_vp]
_lib.pd_batch_destroy.restype = None
_lib.pd_batch_last_error.argtypes = [_vp]
_lib.pd_batch_last_error.restype = ctypes.c_char_p
_lib.pd_batch_layout.argtypes = [_vp, ctypes.POINTER(ctypes.c_longlong)]
_lib.pd_batch_variants.argtypes = [_vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
_lib.pd_batch_configure.argtypes = [_vp, ctypes.c_int, ctypes.c_double]
_lib.pd_batch_cg_solve.argtypes = [_vp, ctypes.c_int, _vp, _vp, ctypes.c_double, ctypes.c_int,
                                   ctypes.POINTER(pd_solve_info), _vp]


class PdError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libpd error {code}: {msg}")
        self.code = code


def _stream(stream):
    if stream is not None:
        return stream
    import torch
    return torch.cuda.current_stream().cuda_stream


def _ptr(t, ndof=None, dtype=None):
    """Device pointer of a contiguous CUDA tensor (validated against the expected size/dtype)."""
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a CUDA (HIP) torch tensor")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"expected dtype {dtype}, got {t.dtype}")
    if ndof is not None and t.numel() != ndof:
        raise ValueError(f"expected {ndof} elements, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


class Context:
    """Owns one pd_ctx. Sizes: .ncells, .ndof, .dim; .N; nodes via pd_nodes()."""

    def __init__(self, handle, dim, N):
        self._h = handle
        self.dim = dim
        self.N = N
        nc, nd, d = ctypes.c_longlong(), ctypes.c_longlong(), ctypes.c_int()
        _check(self, _lib.pd_sizes(self._h, ctypes.byref(nc), ctypes.byref(nd), ctypes.byref(d)))
        self.ncells, self.ndof = nc.value, nd.value

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("context destroyed")
        return self._h

    def close(self):
        if self._h is not None:
            _lib.pd_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _check(ctx, rc, allow=()):
    if rc == PD_OK or rc in allow:
        return rc
    h = None if ctx is None else ctx._h
    msg = _lib.pd_last_error(h)
    raise PdError(rc, msg.decode() if msg else "")


def pd_setup(dim, ncell, length, N, dt, theta, nu, periodic_mask=None, stream=None):
    nc = (ctypes.c_int * 3)(*(list(ncell) + [1] * (3 - len(ncell))))
    ln = (ctypes.c_double * 3)(*(list(length) + [1.0] * (3 - len(length))))
    mask = (1 << dim) - 1 if periodic_mask is None else periodic_mask
    h = ctypes.c_void_p()
    rc = _lib.pd_setup(ctypes.byref(h), dim, nc, ln, int(N), float(dt), float(theta), float(nu),
                       mask, ctypes.c_void_p(_stream(stream)))
    if rc != PD_OK:
        raise PdError(rc, _lib.pd_last_error(None).decode())
    return Context(h, dim, int(N))


def pd_destroy(ctx):
    ctx.close()


def pd_nodes(ctx):
    n = ctx.N + 1
    xi = (ctypes.c_double * n)()
    w = (ctypes.c_double * n)()
    _check(ctx, _lib.pd_nodes(ctx.handle, xi, w))
    return list(xi), list(w)


def pd_table_1d(N, which):
    """Host-only: the library's FP64 1D table `which` (PD_TAB_*) for degree N, as a list."""
    out = (ctypes.c_double * 81)()
    cnt = _lib.pd_table_1d(int(N), int(which), out)
    if cnt < 0:
        raise PdError(cnt, f"pd_table_1d: bad degree {N} or table {which}")
    return list(out)[:cnt]


def _dtype(prec):
    import torch
    return torch.float32 if prec == PD_FP32 else torch.float64


def pd_apply(ctx, op, prec, x, y, stream=None):
    dt = _dtype(prec)
    _check(ctx, _lib.pd_apply(ctx.handle, op, prec, _ptr(x, ctx.ndof, dt), _ptr(y, ctx.ndof, dt),
                              ctypes.c_void_p(_stream(stream))))


def pd_cg_solve(ctx, op, prec, b, x, rtol, maxit, stream=None):
    """Returns the pd_solve_info as a dict; raises on invalid use or device errors.
    Non-convergence / breakdown are reported through info['status']."""
    import torch
    info = pd_solve_info()
    rc = _lib.pd_cg_solve(ctx.handle, op, prec, _ptr(b, ctx.ndof, torch.float64),
                          _ptr(x, ctx.ndof, torch.float64), float(rtol), int(maxit),
                          ctypes.byref(info), ctypes.c_void_p(_stream(stream)))
    _check(ctx, rc, allow=(PD_ENOCONV, PD_EBREAKDOWN))
    return info.as_dict()


def _vec3(ctx, u):
    import torch
    arr = (ctypes.c_void_p * 3)()
    for d in range(ctx.dim):
        arr[d] = _ptr(u[d], ctx.ndof, torch.float64).value
    return arr


def pd_rhs_div(ctx, u, b, stream=None):
    import torch
    _check(ctx, _lib.pd_rhs_div(ctx.handle, _vec3(ctx, u), _ptr(b, ctx.ndof, torch.float64),
                                ctypes.c_void_p(_stream(stream))))


def pd_project_velocity(ctx, q, u, stream=None):
    import torch
    _check(ctx, _lib.pd_project_velocity(ctx.handle, _ptr(q, ctx.ndof, torch.float64),
                                         _vec3(ctx, u), ctypes.c_void_p(_stream(stream))))


def pd_project_null(ctx, prec, v, stream=None):
    _check(ctx, _lib.pd_project_null(ctx.handle, prec, _ptr(v, ctx.ndof, _dtype(prec)),
                                     ctypes.c_void_p(_stream(stream))))


def pd_project_null_noalloc(ctx, prec, v, stream=None):
    _check(ctx, _lib.pd_project_null_noalloc(ctx.handle, prec, _ptr(v, ctx.ndof, _dtype(prec)),
                                             ctypes.c_void_p(_stream(stream))))


def pd_l2_project(ctx, d, direction, src, dst, stream=None):
    import torch
    _check(ctx, _lib.pd_l2_project(ctx.handle, d, direction, _ptr(src, ctx.ndof, torch.float64),
                                   _ptr(dst, ctx.ndof, torch.float64),
                                   ctypes.c_void_p(_stream(stream))))


def pd_convect(ctx, um, stream=None):
    _check(ctx, _lib.pd_convect(ctx.handle, _vec3(ctx, um), ctypes.c_void_p(_stream(stream))))


def pd_step(ctx, u, p, stream=None):
    """One fractional step in place on u (dual components) and p. Returns 4 solve-info dicts
    (viscous x, y, z; pressure)."""
    import torch
    info = (pd_solve_info * 4)()
    rc = _lib.pd_step(ctx.handle, _vec3(ctx, u), _ptr(p, ctx.ndof, torch.float64), info,
                      ctypes.c_void_p(_stream(stream)))
    _check(ctx, rc, allow=(PD_ENOCONV, PD_EBREAKDOWN))
    return [i.as_dict() for i in info]


def pd_step_st(ctx, M, u, p_nodes, stream=None):
    """One space-time step of degree M in time (Picard pressure correction) in place on u (dual
    components, U^n in, end value out); p_nodes ((M+1) * ndof FP64) receives the pressure at the
    time nodes. Returns the 3 + (M+1)^2 solve-info dicts (viscous x, y, z; pressure solves)."""
    import torch
    m = int(M) + 1
    info = (pd_solve_info * (3 + m * m))()
    rc = _lib.pd_step_st(ctx.handle, int(M), _vec3(ctx, u), _ptr(p_nodes, m * ctx.ndof, torch.float64),
                         info, ctypes.c_void_p(_stream(stream)))
    _check(ctx, rc, allow=(PD_ENOCONV, PD_EBREAKDOWN))
    return [i.as_dict() for i in info]


def pd_time_table(M, which):
    """Host-only: the library's time table `which` (PD_TTAB_*) for degree M, as a list."""
    out = (ctypes.c_double * 25)()
    cnt = _lib.pd_time_table(int(M), int(which), out)
    if cnt < 0:
        raise PdError(cnt, f"pd_time_table: bad degree {M} or table {which}")
    return list(out)[:cnt]


def pd_l2_project_adjoint(ctx, d, direction, src, dst, stream=None):
    import torch
    _check(ctx, _lib.pd_l2_project_adjoint(ctx.handle, d, direction,
                                           _ptr(src, ctx.ndof, torch.float64),
                                           _ptr(dst, ctx.ndof, torch.float64),
                                           ctypes.c_void_p(_stream(stream))))


def pd_rhs_div_adjoint(ctx, bbar, ubar, stream=None):
    import torch
    _check(ctx, _lib.pd_rhs_div_adjoint(ctx.handle, _ptr(bbar, ctx.ndof, torch.float64),
                                        _vec3(ctx, ubar), ctypes.c_void_p(_stream(stream))))


def pd_project_velocity_adjoint(ctx, ubar, qbar, stream=None):
    import torch
    _check(ctx, _lib.pd_project_velocity_adjoint(ctx.handle, _vec3(ctx, ubar),
                                                 _ptr(qbar, ctx.ndof, torch.float64),
                                                 ctypes.c_void_p(_stream(stream))))


def pd_convect_adjoint(ctx, um, ubar, stream=None):
    _check(ctx, _lib.pd_convect_adjoint(ctx.handle, _vec3(ctx, um), _vec3(ctx, ubar),
                                        ctypes.c_void_p(_stream(stream))))


def pd_step_adjoint(ctx, u, ubar, stream=None):
    """Adjoint of pd_step at U^n = u (unchanged): ubar in = cotangent of U^{n+1}, out = that of
    U^n. Returns 4 solve-info dicts (adjoint viscous x, y, z; adjoint pressure)."""
    info = (pd_solve_info * 4)()
    rc = _lib.pd_step_adjoint(ctx.handle, _vec3(ctx, u), _vec3(ctx, ubar), info,
                              ctypes.c_void_p(_stream(stream)))
    _check(ctx, rc, allow=(PD_ENOCONV, PD_EBREAKDOWN))
    return [i.as_dict() for i in info]


def pd_kinetic_energy(ctx, u, grad=None, gscale=1.0, stream=None):
    """Mean kinetic energy of the dual velocity u (returned as a float); with grad (dim FP64
    tensors) also grad[d] = gscale * dK/du_d."""
    e = ctypes.c_double()
    g = _vec3(ctx, grad) if grad is not None else None
    _check(ctx, _lib.pd_kinetic_energy(ctx.handle, _vec3(ctx, u), float(gscale), g,
                                       ctypes.byref(e), ctypes.c_void_p(_stream(stream))))
    return e.value


def pd_configure(ctx, key, value):
    _check(ctx, _lib.pd_configure(ctx.handle, int(key), float(value)))


def pd_timing(ctx, prec, reset=True):
    ms, cnt, by = ctypes.c_double(), ctypes.c_longlong(), ctypes.c_double()
    _check(ctx, _lib.pd_timing(ctx.handle, prec, ctypes.byref(ms), ctypes.byref(cnt),
                               ctypes.byref(by), 1 if reset else 0))
    return dict(total_ms=ms.value, launches=cnt.value, bytes_per_launch=by.value)


class Batch:
    """Owns one pd_batch: .count problems, packed layout .offsets (count + 1), .total DoFs."""

    def __init__(self, handle, count):
        self._h = handle
        self.count = count
        off = (ctypes.c_longlong * (count + 1))()
        _bcheck(self, _lib.pd_batch_layout(self._h, off))
        self.offsets = list(off)
        self.total = self.offsets[-1]

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("batch destroyed")
        return self._h

    def close(self):
        if self._h is not None:
            _lib.pd_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _bcheck(batch, rc, allow=()):
    if rc == PD_OK or rc in allow:
        return rc
    h = None if batch is None else batch._h
    msg = _lib.pd_batch_last_error(h)
    raise PdError(rc, msg.decode() if msg else "")


def pd_batch_setup(ncell, length, N, dt, flags=0, stream=None):
    """ncell, length: sequences of (nx, ny) / (Lx, Ly) pairs; N: degrees."""
    count = len(N)
    if len(ncell) != count or len(length) != count:
        raise ValueError("ncell, length and N must have one entry per problem")
    nc = (ctypes.c_int * (2 * count))(*[int(v) for p in ncell for v in p])
    ln = (ctypes.c_double * (2 * count))(*[float(v) for p in length for v in p])
    nn = (ctypes.c_int * count)(*[int(v) for v in N])
    h = ctypes.c_void_p()
    rc = _lib.pd_batch_setup(ctypes.byref(h), count, nc, ln, nn, float(dt), int(flags),
                             ctypes.c_void_p(_stream(stream)))
    if rc != PD_OK:
        raise PdError(rc, _lib.pd_batch_last_error(None).decode())
    return Batch(h, count)


def pd_batch_destroy(batch):
    batch.close()


def pd_batch_variants(batch, prec):
    v = (ctypes.c_int * batch.count)()
    _bcheck(batch, _lib.pd_batch_variants(batch.handle, prec, v))
    return list(v)


def pd_batch_configure(batch, key, value):
    _bcheck(batch, _lib.pd_batch_configure(batch.handle, int(key), float(value)))


def pd_batch_cg_solve(batch, prec, b, x, rtol, maxit, stream=None):
    """Solves every problem; returns (rc, list of per-problem solve-info dicts). Non-convergence
    and breakdown are reported through rc and the infos, other failures raise."""
    import torch
    info = (pd_solve_info * batch.count)()
    rc = _lib.pd_batch_cg_solve(batch.handle, prec, _ptr(b, batch.total, torch.float64),
                                _ptr(x, batch.total, torch.float64), float(rtol), int(maxit),
                                info, ctypes.c_void_p(_stream(stream)))
    _bcheck(batch, rc, allow=(PD_ENOCONV, PD_EBREAKDOWN))
    return rc, [i.as_dict() for i in info]
