"""Python binding of libtmsap.so, the MI355X twisted-mass operator / SAP / FGMRES library.

Argument marshalling only: every step runs in the HIP kernels behind the C ABI
declared in include/tm.h.  PyTorch supplies device memory and the stream.  The
binding raises if the compiled library is missing; there is no CPU fallback.

Tensors are complex128 on the current GPU in the canonical layout:
  U    [V, 4, 3, 3]       (or any shape with that many elements)
  psi  [nsys, V, 4, 3]
Sites are lexicographic over dims = (T, Z, Y, X), t slowest; direction mu: 0 = t, 1 = x, 2 = y, 3 = z.
"""
from __future__ import annotations

import ctypes
import os
from typing import Sequence

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("TMSAP_LIB") or os.path.join(_HERE, "libtmsap.so")

TM_OK, TM_NOT_CONVERGED = 0, 1
ERRORS = {-1: "TM_ERR_ARG", -2: "TM_ERR_DIMS", -3: "TM_ERR_BLOCKS", -4: "TM_ERR_PREC", -5: "TM_ERR_HIP",
          -6: "TM_ERR_NOMEM", -7: "TM_ERR_NONFINITE", -8: "TM_ERR_NOT_SU3"}
PREC = {"f64": 0, "f32": 1, "f16": 2, "bf16": 3}
IO = {"canonical": 0, "internal": 1}
FORMS = {"flexible": 0, "defect_correction": 1}
MAX_SYS = 64

# Every entry point declared in include/tm.h.
EXPORTS = (
    "tm_opts_default", "tm_init", "tm_finalize", "tm_last_error", "tm_gauge_release", "tm_dirac_apply",
    "tm_sap_smooth", "tm_solver_opts_default", "tm_fgmres_solve", "tm_spinor_bytes", "tm_spinor_import",
    "tm_spinor_export", "tm_spinor_import_range", "tm_spinor_export_range", "tm_autotune_sap", "tm_cg_solve",
    "tm_mg_params_default", "tm_mg_setup", "tm_mg_destroy", "tm_mg_get_info", "tm_mg_export", "tm_mg_restrict",
    "tm_mg_prolong", "tm_mg_coarse_apply", "tm_mg_coarse_solve", "tm_mg_precond", "tm_probe_fp32_fma",
    "tm_sap_smooth_noalloc",
)


class TMError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class Geom(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int * 4), ("antiperiodic_t", ctypes.c_int), ("nsys", ctypes.c_int),
                ("mu", ctypes.POINTER(ctypes.c_double)), ("theta", ctypes.c_double * 4),
                ("mu_shift", ctypes.c_double * 2)]


class Opts(ctypes.Structure):
    _fields_ = [("storage", ctypes.c_int), ("compute", ctypes.c_int), ("stream", ctypes.c_void_p),
                ("io", ctypes.c_int), ("layout_block", ctypes.c_int * 4), ("gauge_tag", ctypes.c_ulonglong),
                ("sys_tile", ctypes.c_int), ("sap_eo", ctypes.c_int)]


class SolverOpts(ctypes.Structure):
    _fields_ = [("form", ctypes.c_int), ("restart", ctypes.c_int), ("max_iters", ctypes.c_int),
                ("n_cycles", ctypes.c_int), ("mr_iters", ctypes.c_int), ("block_dims", ctypes.c_int * 4),
                ("inner_tol", ctypes.c_double), ("max_outer", ctypes.c_int), ("group", ctypes.c_int),
                ("mg", ctypes.c_void_p), ("x_in", ctypes.c_int)]


class MgParams(ctypes.Structure):
    _fields_ = [("block_dims", ctypes.c_int * 4), ("n_vec", ctypes.c_int), ("setup_iters", ctypes.c_int),
                ("setup_cycles", ctypes.c_int), ("delta", ctypes.c_double), ("coarse_tol", ctypes.c_double),
                ("coarse_restart", ctypes.c_int), ("coarse_max_restarts", ctypes.c_int),
                ("post_cycles", ctypes.c_int), ("mr_iters", ctypes.c_int), ("coarse_eo", ctypes.c_int)]


class MgInfo(ctypes.Structure):
    _fields_ = [("cdims", ctypes.c_int * 4), ("n_vec", ctypes.c_int), ("t_setup", ctypes.c_double),
                ("applications", ctypes.c_longlong), ("coarse_iters", ctypes.c_longlong),
                ("t_coarse", ctypes.c_double)]


class Report(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("outer", ctypes.c_int), ("converged", ctypes.c_int),
                ("true_rel_res", ctypes.c_double * MAX_SYS), ("t_total", ctypes.c_double),
                ("t_sap", ctypes.c_double), ("sap_cycles", ctypes.c_longlong),
                ("sap_sys_cycles", ctypes.c_longlong), ("group", ctypes.c_int), ("block_dims", ctypes.c_int * 4),
                ("sys_tile", ctypes.c_int)]


_lib = None


def lib():
    """The loaded library; raises when it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(the library has no CPU fallback)")
        # torch's HIP runtime goes in first: the library then binds to the same runtime (same
        # soname) as the tensors and streams it is handed, instead of loading a second one
        import torch  # noqa: F401

        L = ctypes.CDLL(LIB_PATH)
        vp, P = ctypes.c_void_p, ctypes.POINTER
        L.tm_opts_default.argtypes = [P(Opts)]
        L.tm_opts_default.restype = None
        L.tm_solver_opts_default.argtypes = [P(SolverOpts)]
        L.tm_solver_opts_default.restype = None
        L.tm_init.restype = ctypes.c_int
        L.tm_finalize.restype = ctypes.c_int
        L.tm_last_error.restype = ctypes.c_char_p
        L.tm_gauge_release.argtypes = [vp]
        L.tm_dirac_apply.argtypes = [P(Geom), vp, vp, vp, ctypes.c_double, ctypes.c_double, P(Opts)]
        L.tm_sap_smooth.argtypes = [P(Geom), vp, vp, vp, ctypes.c_double, ctypes.c_double, P(ctypes.c_int),
                                    ctypes.c_int, ctypes.c_int, P(Opts)]
        L.tm_sap_smooth_noalloc.argtypes = L.tm_sap_smooth.argtypes
        L.tm_fgmres_solve.argtypes = [P(Geom), vp, vp, vp, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                      P(SolverOpts), P(Opts), P(Report)]
        L.tm_spinor_bytes.argtypes = [P(Geom), P(Opts)]
        L.tm_spinor_bytes.restype = ctypes.c_size_t
        L.tm_spinor_import.argtypes = [P(Geom), vp, vp, P(Opts)]
        L.tm_spinor_export.argtypes = [P(Geom), vp, vp, P(Opts)]
        L.tm_cg_solve.argtypes = [P(Geom), vp, vp, vp, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                  P(Opts), P(Report)]
        L.tm_spinor_import_range.argtypes = [P(Geom), vp, vp, ctypes.c_int, ctypes.c_int, P(Opts)]
        L.tm_spinor_export_range.argtypes = [P(Geom), vp, vp, ctypes.c_int, ctypes.c_int, P(Opts)]
        L.tm_mg_params_default.argtypes = [P(MgParams)]
        L.tm_mg_params_default.restype = None
        L.tm_mg_setup.argtypes = [P(Geom), vp, ctypes.c_double, ctypes.c_double, P(MgParams), vp,
                                  P(ctypes.c_void_p), P(Opts)]
        L.tm_mg_destroy.argtypes = [vp]
        L.tm_mg_get_info.argtypes = [vp, P(MgInfo)]
        L.tm_mg_export.argtypes = [vp, vp, vp, P(Opts)]
        L.tm_mg_restrict.argtypes = [vp, ctypes.c_int, vp, vp, P(Opts)]
        L.tm_mg_prolong.argtypes = [vp, ctypes.c_int, vp, vp, P(Opts)]
        L.tm_mg_coarse_apply.argtypes = [vp, ctypes.c_int, P(ctypes.c_double), vp, vp, P(Opts)]
        L.tm_mg_coarse_solve.argtypes = [vp, ctypes.c_int, P(ctypes.c_double), vp, vp, ctypes.c_double, ctypes.c_int,
                                         ctypes.c_int, P(ctypes.c_int), P(Opts)]
        L.tm_mg_precond.argtypes = [P(Geom), vp, vp, vp, P(Opts)]
        L.tm_autotune_sap.argtypes = [P(Geom), vp, ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                      P(Opts), P(ctypes.c_int), P(ctypes.c_int)]
        L.tm_probe_fp32_fma.argtypes = [P(ctypes.c_double), P(Opts)]
        _lib = L
    return _lib


def _check(rc: int, allow_not_converged: bool = False) -> int:
    if rc == TM_OK or (allow_not_converged and rc == TM_NOT_CONVERGED):
        return rc
    raise TMError(rc, lib().tm_last_error().decode())


def _stream_handle(stream):
    """None: torch's current stream; False: the null stream (no torch call)."""
    if stream is False:
        return ctypes.c_void_p(None)
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def make_geom(dims: Sequence[int], mu, antiperiodic_t: bool = False, theta=None, mu_shift=None):
    """theta: twisted boundary phases (radians) for t, x, y, z; mu_shift: added to mu on even / odd sites."""
    mus = [float(mu)] if isinstance(mu, (int, float)) else [float(m) for m in mu]
    arr = (ctypes.c_double * len(mus))(*mus)
    th = [float(t) for t in (theta or (0.0, 0.0, 0.0, 0.0))]
    ms = [float(t) for t in (mu_shift or (0.0, 0.0))]
    g = Geom((ctypes.c_int * 4)(*[int(d) for d in dims]), int(bool(antiperiodic_t)), len(mus),
             ctypes.cast(arr, ctypes.POINTER(ctypes.c_double)), (ctypes.c_double * 4)(*th),
             (ctypes.c_double * 2)(*ms))
    g._keep = arr
    return g


def make_opts(storage: str = "f64", compute: str | None = None, stream=None, io: str = "canonical",
              layout_block=None, gauge_tag: int = 0):
    o = Opts()
    lib().tm_opts_default(ctypes.byref(o))
    o.storage = PREC[storage]
    o.compute = PREC[compute] if compute else (PREC["f64"] if storage == "f64" else PREC["f32"])
    o.stream = _stream_handle(stream)
    o.io = IO[io]
    if layout_block is not None:
        o.layout_block = (ctypes.c_int * 4)(*[int(v) for v in layout_block])
    o.gauge_tag = int(gauge_tag)
    return o


def _ptr(t) -> ctypes.c_void_p:
    if not t.is_cuda:
        raise ValueError("tensor must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _expect(t, what: str, numel: int | None = None) -> None:
    """A canonical complex128 tensor; numel, when given, is the element count the call implies."""
    import torch

    if t.dtype != torch.complex128:
        raise TypeError(f"{what} must be complex128 in the canonical layout")
    if numel is not None and numel > 0 and t.numel() != numel:
        raise ValueError(f"{what} has {t.numel()} complex elements; the call's dims and systems imply {numel}")


def _expect_bytes(t, nbytes: int, what: str) -> None:
    """An internal-layout buffer holding at least nbytes."""
    have = t.numel() * t.element_size()
    if nbytes > 0 and have < nbytes:
        raise ValueError(f"{what} holds {have} bytes; the internal layout of the call needs {nbytes}")


def _canon(t, what: str, numel: int | None = None):
    _expect(t, what, numel)
    return _ptr(t)


def _internal(t, nbytes: int, what: str) -> ctypes.c_void_p:
    _expect_bytes(t, nbytes, what)
    return _ptr(t)


def _volume(dims) -> int:
    """Sites of dims, or 0 when a dimension is not positive (the library reports that error itself)."""
    V = 1
    for d in dims:
        if int(d) <= 0:
            return 0
        V *= int(d)
    return V


def _spinor_numel(dims, nsys: int) -> int:
    return nsys * _volume(dims) * 12


def _link_numel(dims) -> int:
    return _volume(dims) * 36


def tm_init() -> None:
    _check(lib().tm_init())


def tm_finalize() -> None:
    _check(lib().tm_finalize())


def tm_gauge_release(U) -> None:
    _check(lib().tm_gauge_release(ctypes.c_void_p(U.data_ptr())))


def tm_dirac_apply(dims, U, psi, kappa: float, mu, c_sw: float, out=None, *, storage: str = "f64",
                   antiperiodic_t: bool = False, stream=None, io: str = "canonical", layout_block=None,
                   theta=None, mu_shift=None,
                   gauge_tag: int = 0):
    """out_k = D(mu_k) psi_k for every system k (psi: [nsys, V, 4, 3] complex128, or internal buffers)."""
    import torch

    g = make_geom(dims, mu, antiperiodic_t, theta, mu_shift)
    o = make_opts(storage, stream=stream, io=io, layout_block=layout_block, gauge_tag=gauge_tag)
    if out is None:
        out = torch.empty_like(psi)
    _expect(U, "U", _link_numel(dims))
    if io == "canonical":
        n = _spinor_numel(dims, g.nsys)
        _expect(psi, "psi", n)
        _expect(out, "out", n)
        pin, pout = _ptr(psi), _ptr(out)
    else:
        n = _spinor_bytes(g, o)
        _expect_bytes(psi, n, "psi")
        _expect_bytes(out, n, "out")
        pin, pout = _ptr(psi), _ptr(out)
    _check(lib().tm_dirac_apply(ctypes.byref(g), _ptr(U), pin, pout, float(kappa), float(c_sw), ctypes.byref(o)))
    return out


def tm_sap_smooth(dims, U, b, x, kappa: float, mu, c_sw: float, block_dims, n_cycles: int, mr_iters: int, *,
                  storage: str = "f64", antiperiodic_t: bool = False, stream=None, io: str = "canonical",
                  theta=None, mu_shift=None,
                  gauge_tag: int = 0, sys_tile: int = 0, eo: bool = False):
    """x <- SAP(b, x): n_cycles red-black cycles, mr_iters MR steps per block (x is in/out).

    eo: even-odd preconditioned block solves (MR on the odd-site Schur complement)."""
    return _sap(lib().tm_sap_smooth, dims, U, b, x, kappa, mu, c_sw, block_dims, n_cycles, mr_iters, storage,
                antiperiodic_t, stream, io, theta, mu_shift, gauge_tag, sys_tile, eo)


def tm_sap_smooth_noalloc(dims, U, b, x, kappa: float, mu, c_sw: float, block_dims, n_cycles: int, mr_iters: int,
                          *, storage: str = "f64", antiperiodic_t: bool = False, stream=None, io: str = "canonical",
                          theta=None, mu_shift=None, sys_tile: int = 0):
    """tm_sap_smooth without device allocation: the library's fixed per-GPU scratch array holds the
    gauge copy, clover and internal b / x (TMError TM_ERR_ARG when the problem does not fit)."""
    return _sap(lib().tm_sap_smooth_noalloc, dims, U, b, x, kappa, mu, c_sw, block_dims, n_cycles, mr_iters,
                storage, antiperiodic_t, stream, io, theta, mu_shift, 0, sys_tile, False)


def _sap(fn, dims, U, b, x, kappa, mu, c_sw, block_dims, n_cycles, mr_iters, storage, antiperiodic_t, stream, io,
         theta, mu_shift, gauge_tag, sys_tile, eo):
    g = make_geom(dims, mu, antiperiodic_t, theta, mu_shift)
    o = make_opts(storage, stream=stream, io=io, layout_block=block_dims, gauge_tag=gauge_tag)
    o.sys_tile = int(sys_tile)
    o.sap_eo = int(bool(eo))
    bd = (ctypes.c_int * 4)(*[int(v) for v in block_dims])
    _expect(U, "U", _link_numel(dims))
    if io == "canonical":
        n = _spinor_numel(dims, g.nsys)
        _expect(b, "b", n)
        _expect(x, "x", n)
    else:
        n = _spinor_bytes(g, o)
        _expect_bytes(b, n, "b")
        _expect_bytes(x, n, "x")
    _check(fn(ctypes.byref(g), _ptr(U), _ptr(b), _ptr(x), float(kappa), float(c_sw), bd, int(n_cycles),
              int(mr_iters), ctypes.byref(o)))
    return x


def solver_opts(form: str = "flexible", restart: int = 20, max_iters: int = 2000, n_cycles: int = 4,
                mr_iters: int = 4, block_dims=(4, 4, 4, 4), inner_tol: float = 1e-6, max_outer: int = 50,
                group: int = 0, x_in: bool = True) -> SolverOpts:
    s = SolverOpts()
    lib().tm_solver_opts_default(ctypes.byref(s))
    s.form = FORMS[form]
    s.restart, s.max_iters, s.n_cycles, s.mr_iters = int(restart), int(max_iters), int(n_cycles), int(mr_iters)
    s.block_dims = (ctypes.c_int * 4)(*[int(v) for v in (block_dims or (0, 0, 0, 0))])
    s.inner_tol, s.max_outer, s.group = float(inner_tol), int(max_outer), int(group)
    s.x_in = int(bool(x_in))
    return s


def tm_fgmres_solve(dims, U, b, x, kappa: float, mu, c_sw: float, tol: float, *, storage: str = "f32",
                    antiperiodic_t: bool = False, stream=None, gauge_tag: int = 0, sys_tile: int = 0,
                    theta=None, mu_shift=None,
                    eo: bool = False, mg: "MG | None" = None, **solver_kw):
    """Solve D(mu_k) x_k = b_k to a true relative residual tol; returns (status, report dict).

    mg: a two-level handle (MG) whose method preconditions FGMRES instead of SAP.
    x_in=False (a solver option): the solve starts from zero and x is output only."""
    g = make_geom(dims, mu, antiperiodic_t, theta, mu_shift)
    o = make_opts(storage, stream=stream, gauge_tag=gauge_tag)
    o.sys_tile = int(sys_tile)
    o.sap_eo = int(bool(eo))
    s = solver_opts(**solver_kw)
    if mg is not None:
        s.mg = mg.handle
    rep = Report()
    n = _spinor_numel(dims, g.nsys)
    _expect(U, "U", _link_numel(dims))
    _expect(b, "b", n)
    _expect(x, "x", n)
    rc = _check(lib().tm_fgmres_solve(ctypes.byref(g), _ptr(U), _ptr(b), _ptr(x), float(kappa), float(c_sw),
                                      float(tol), ctypes.byref(s), ctypes.byref(o), ctypes.byref(rep)),
                allow_not_converged=True)
    n = g.nsys
    return rc, {"iters": rep.iters, "outer": rep.outer, "converged": rep.converged,
                "true_rel_res": [rep.true_rel_res[k] for k in range(n)], "t_total": rep.t_total,
                "t_sap": rep.t_sap, "sap_cycles": rep.sap_cycles, "sap_sys_cycles": rep.sap_sys_cycles,
                "group": rep.group, "block_dims": tuple(rep.block_dims), "sys_tile": rep.sys_tile}


def tm_cg_solve(dims, U, b, x, kappa: float, mu, c_sw: float, tol: float, *, max_iters: int = 100000,
                antiperiodic_t: bool = False, theta=None, mu_shift=None, stream=None, gauge_tag: int = 0):
    """CG on the squared even-odd reduced system (FP64 baseline); returns (status, report dict)."""
    g = make_geom(dims, mu, antiperiodic_t, theta, mu_shift)
    o = make_opts("f64", stream=stream, gauge_tag=gauge_tag)
    rep = Report()
    n = _spinor_numel(dims, g.nsys)
    _expect(U, "U", _link_numel(dims))
    _expect(b, "b", n)
    _expect(x, "x", n)
    rc = _check(lib().tm_cg_solve(ctypes.byref(g), _ptr(U), _ptr(b), _ptr(x), float(kappa), float(c_sw), float(tol),
                                  int(max_iters), ctypes.byref(o), ctypes.byref(rep)),
                allow_not_converged=True)
    n = len(list(mu))
    return rc, {"iters": rep.iters, "converged": rep.converged,
                "true_rel_res": [rep.true_rel_res[k] for k in range(n)], "t_total": rep.t_total, "group": rep.group}


def _spinor_bytes(g: Geom, o: Opts) -> int:
    return int(lib().tm_spinor_bytes(ctypes.byref(g), ctypes.byref(o)))


def tm_spinor_bytes(dims, nsys: int, storage: str, layout_block=None) -> int:
    """Bytes of an internal buffer (host-side arithmetic, no GPU call)."""
    g = make_geom(dims, [0.0] * nsys)
    o = make_opts(storage, stream=False, io="internal", layout_block=layout_block)
    return _spinor_bytes(g, o)


def tm_spinor_import(dims, canon, internal, *, storage: str, layout_block=None, stream=None):
    nsys = canon.shape[0]
    g = make_geom(dims, [0.0] * nsys)
    o = make_opts(storage, stream=stream, io="internal", layout_block=layout_block)
    _expect(canon, "canon", _spinor_numel(dims, nsys))
    _expect_bytes(internal, _spinor_bytes(g, o), "internal")
    _check(lib().tm_spinor_import(ctypes.byref(g), _ptr(canon), _ptr(internal), ctypes.byref(o)))
    return internal


def tm_spinor_export(dims, internal, canon, *, storage: str, layout_block=None, stream=None):
    nsys = canon.shape[0]
    g = make_geom(dims, [0.0] * nsys)
    o = make_opts(storage, stream=stream, io="internal", layout_block=layout_block)
    _expect(canon, "canon", _spinor_numel(dims, nsys))
    _expect_bytes(internal, _spinor_bytes(g, o), "internal")
    _check(lib().tm_spinor_export(ctypes.byref(g), _ptr(internal), _ptr(canon), ctypes.byref(o)))
    return canon


def tm_spinor_import_range(dims, canon, internal, nsys: int, first: int, *, storage: str, layout_block=None,
                           stream=None):
    """canon ([count][V][4][3]) -> systems first..first+count-1 of an internal buffer of nsys systems."""
    g = make_geom(dims, [0.0] * nsys)
    o = make_opts(storage, stream=stream, io="internal", layout_block=layout_block)
    count = int(canon.shape[0])
    _expect(canon, "canon", _spinor_numel(dims, count))
    _expect_bytes(internal, _spinor_bytes(g, o), "internal")
    _check(lib().tm_spinor_import_range(ctypes.byref(g), _ptr(canon), _ptr(internal), int(first), count,
                                        ctypes.byref(o)))
    return internal


def tm_spinor_export_range(dims, internal, canon, nsys: int, first: int, *, storage: str, layout_block=None,
                           stream=None):
    """Systems first..first+count-1 of an internal buffer of nsys systems -> canon ([count][V][4][3])."""
    g = make_geom(dims, [0.0] * nsys)
    o = make_opts(storage, stream=stream, io="internal", layout_block=layout_block)
    count = int(canon.shape[0])
    _expect(canon, "canon", _spinor_numel(dims, count))
    _expect_bytes(internal, _spinor_bytes(g, o), "internal")
    _check(lib().tm_spinor_export_range(ctypes.byref(g), _ptr(internal), _ptr(canon), int(first), count,
                                        ctypes.byref(o)))
    return canon


def tm_autotune_sap(dims, U, kappa: float, mu, c_sw: float, n_cycles: int, mr_iters: int, *, storage: str = "f32",
                    stream=None, gauge_tag: int = 0, eo: bool = False):
    """Fastest (block_dims, sys_tile) for SAP applications on this lattice; cached on disk."""
    g = make_geom(dims, mu)
    o = make_opts(storage, stream=stream, gauge_tag=gauge_tag)
    o.sap_eo = int(bool(eo))
    best = (ctypes.c_int * 4)()
    tile = ctypes.c_int()
    _check(lib().tm_autotune_sap(ctypes.byref(g), _canon(U, "U", _link_numel(dims)), float(kappa), float(c_sw),
                                 int(n_cycles),
                                 int(mr_iters), ctypes.byref(o), best, ctypes.byref(tile)))
    return tuple(best), tile.value


def tm_probe_fp32_fma(*, stream=None) -> float:
    """Measured FP32 vector FMA ceiling of the current device in TFLOP/s (no packed FP32)."""
    o = make_opts("f32", stream=stream)
    out = ctypes.c_double()
    _check(lib().tm_probe_fp32_fma(ctypes.byref(out), ctypes.byref(o)))
    return out.value


def mg_params(**kw) -> MgParams:
    """Two-level parameters: the library defaults (Table 1) overridden by keyword."""
    p = MgParams()
    lib().tm_mg_params_default(ctypes.byref(p))
    for k, v in kw.items():
        if k == "block_dims":
            p.block_dims = (ctypes.c_int * 4)(*[int(a) for a in v])
        elif k in ("delta", "coarse_tol"):
            setattr(p, k, float(v))
        else:
            setattr(p, k, int(v))
    return p


class MG:
    """Two-level method (tm_mg_setup); `close()` (or garbage collection) frees it.

    Coarse vectors are complex128 tensors [nsys, nc, 2 n_vec]; fine vectors [nsys, V, 4, 3].
    `params` override the library defaults (Table 1) by field name of tm_mg_params, e.g.
    n_vec, setup_iters, delta, coarse_tol, coarse_eo (1: even-odd reduced coarse GMRES, the default;
    0: GMRES on the full coarse operator)."""

    def __init__(self, dims, U, kappa: float, mu: float, c_sw: float, v0, *, antiperiodic_t: bool = False,
                 theta=None, mu_shift=None, stream=None, gauge_tag: int = 0, **params):
        self.dims = tuple(int(d) for d in dims)
        self.antiperiodic_t, self.theta, self.mu_shift = antiperiodic_t, theta, mu_shift
        self.params = mg_params(**params)
        self.gauge_tag = gauge_tag
        g = make_geom(dims, [float(mu)], antiperiodic_t, theta, mu_shift)
        o = make_opts("f32", stream=stream, gauge_tag=gauge_tag)
        h = ctypes.c_void_p()
        _expect(U, "U", _link_numel(dims))
        _expect(v0, "v0", _spinor_numel(dims, self.params.n_vec))
        _check(lib().tm_mg_setup(ctypes.byref(g), _ptr(U), float(kappa), float(c_sw), ctypes.byref(self.params),
                                 _ptr(v0), ctypes.byref(h), ctypes.byref(o)))
        self.handle = h
        self.n_vec = self.params.n_vec
        self.cdims = tuple(d // b for d, b in zip(self.dims, self.params.block_dims))
        self.nc = 1
        for c in self.cdims:
            self.nc *= c

    def close(self) -> None:
        if getattr(self, "handle", None) is not None and self.handle.value:
            lib().tm_mg_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> dict:
        i = MgInfo()
        _check(lib().tm_mg_get_info(self.handle, ctypes.byref(i)))
        return {"cdims": tuple(i.cdims), "n_vec": i.n_vec, "t_setup": i.t_setup, "applications": i.applications,
                "coarse_iters": i.coarse_iters, "t_coarse": i.t_coarse}

    def _opts(self, stream=None):
        return make_opts("f32", stream=stream, gauge_tag=self.gauge_tag)

    def export(self, stream=None):
        """(P [n_vec, V, 4, 3], Dc [nc, 9, 2 n_vec, 2 n_vec]) as complex128 tensors."""
        import torch

        V = 1
        for d in self.dims:
            V *= d
        n2 = 2 * self.n_vec
        P = torch.empty((self.n_vec, V, 4, 3), dtype=torch.complex128, device="cuda")
        Dc = torch.empty((self.nc, 9, n2, n2), dtype=torch.complex128, device="cuda")
        _check(lib().tm_mg_export(self.handle, _ptr(P), _ptr(Dc), ctypes.byref(self._opts(stream))))
        torch.cuda.synchronize()
        return P, Dc

    def restrict(self, r, stream=None):
        import torch

        ns = r.shape[0]
        c = torch.empty((ns, self.nc, 2 * self.n_vec), dtype=torch.complex128, device=r.device)
        _check(lib().tm_mg_restrict(self.handle, ns, _canon(r, "r", _spinor_numel(self.dims, ns)), _ptr(c),
                                    ctypes.byref(self._opts(stream))))
        return c

    def prolong(self, c, stream=None):
        import torch

        ns = c.shape[0]
        V = 1
        for d in self.dims:
            V *= d
        e = torch.empty((ns, V, 4, 3), dtype=torch.complex128, device=c.device)
        _check(lib().tm_mg_prolong(self.handle, ns, _canon(c, "c", ns * self.nc * 2 * self.n_vec), _ptr(e),
                                   ctypes.byref(self._opts(stream))))
        return e

    def coarse_apply(self, x, mu_c, stream=None):
        import torch

        ns = x.shape[0]
        mus = (ctypes.c_double * ns)(*[float(m) for m in mu_c])
        y = torch.empty_like(x)
        _check(lib().tm_mg_coarse_apply(self.handle, ns, mus, _canon(x, "x", ns * self.nc * 2 * self.n_vec), _ptr(y),
                                        ctypes.byref(self._opts(stream))))
        return y

    def coarse_solve(self, b, mu_c, tol: float, restart: int, max_restarts: int, stream=None):
        import torch

        ns = b.shape[0]
        mus = (ctypes.c_double * ns)(*[float(m) for m in mu_c])
        x = torch.empty_like(b)
        it = ctypes.c_int(0)
        _check(lib().tm_mg_coarse_solve(self.handle, ns, mus, _canon(b, "b", ns * self.nc * 2 * self.n_vec), _ptr(x),
                                        float(tol), int(restart),
                                        int(max_restarts), ctypes.byref(it), ctypes.byref(self._opts(stream))))
        return x, it.value

    def precond(self, r, mu, stream=None):
        import torch

        g = make_geom(self.dims, mu, self.antiperiodic_t, self.theta, self.mu_shift)
        z = torch.empty_like(r)
        _check(lib().tm_mg_precond(ctypes.byref(g), self.handle, _canon(r, "r", _spinor_numel(self.dims, g.nsys)),
                                   _ptr(z),
                                   ctypes.byref(self._opts(stream))))
        return z
