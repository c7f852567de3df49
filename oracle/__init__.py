"""Plain FP64 CPU oracle (ctypes wrapper around tm_oracle.c).

TEST INFRASTRUCTURE ONLY.  The test suite, the smoke check and the benchmark's
CPU-baseline leg are the only code allowed to import this package.  It shares
nothing with the GPU library (no code, no headers, no tables); both sides only
receive the same seeded inputs.

Arrays are numpy complex128 in the canonical layout:
  spinor  [V][4][3]           (site lexicographic, t slowest, x fastest)
  links   [V][4][3][3]        (direction mu: 0 = t, 1 = x, 2 = y, 3 = z)
  clover  [V][12][12]
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tm_oracle.c")
_LIB = os.environ.get("TM_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no SIMD intrinsics)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-std=c11", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        )
        os.replace(tmp, _LIB)
    return _LIB


class _Op(ctypes.Structure):
    _fields_ = [
        ("dims", ctypes.c_int * 4),
        ("antiperiodic_t", ctypes.c_int),
        ("U", ctypes.c_void_p),
        ("clov", ctypes.c_void_p),
        ("m", ctypes.c_double),
        ("mu", ctypes.c_double),
        ("theta", ctypes.c_double * 4),
        ("mu_shift", ctypes.c_double * 2),
    ]


class _Report(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int),
        ("restarts", ctypes.c_int),
        ("converged", ctypes.c_int),
        ("true_rel_res", ctypes.c_double),
    ]


class _MG(ctypes.Structure):
    _fields_ = [
        ("adims", ctypes.c_int * 4),
        ("nv", ctypes.c_int),
        ("delta", ctypes.c_double),
        ("coarse_tol", ctypes.c_double),
        ("coarse_restart", ctypes.c_int),
        ("coarse_max_restarts", ctypes.c_int),
        ("post_cycles", ctypes.c_int),
        ("mr_iters", ctypes.c_int),
        ("setup_iters", ctypes.c_int),
        ("setup_cycles", ctypes.c_int),
        ("coarse_eo", ctypes.c_int),
        ("P", ctypes.c_void_p),
        ("Dc", ctypes.c_void_p),
    ]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        vp, ip = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int)
        lib.or_volume.restype = ctypes.c_long
        lib.or_volume.argtypes = [ip]
        lib.or_gamma.argtypes = [ctypes.c_int, vp]
        lib.or_clover.argtypes = [ip, vp, ctypes.c_double, vp]
        lib.or_dirac.argtypes = [ctypes.POINTER(_Op), vp, vp]
        lib.or_dirac_blockdiag.argtypes = [ctypes.POINTER(_Op), ip, vp, vp]
        lib.or_block_colour.argtypes = [ip, ip, ctypes.c_long]
        lib.or_block_colour.restype = ctypes.c_int
        lib.or_mr_block.argtypes = [ctypes.POINTER(_Op), ip, ip, vp, vp, ctypes.c_int]
        lib.or_mr_block_eo.argtypes = [ctypes.POINTER(_Op), ip, ip, vp, vp, ctypes.c_int]
        lib.or_sap.argtypes = [ctypes.POINTER(_Op), ip, ctypes.c_int, ctypes.c_int, vp, vp]
        lib.or_sap.restype = ctypes.c_int
        lib.or_sap_eo.argtypes = [ctypes.POINTER(_Op), ip, ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, vp]
        lib.or_sap_eo.restype = ctypes.c_int
        lib.or_fgmres.argtypes = [
            ctypes.POINTER(_Op), vp, vp, ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int, ip,
            ctypes.c_int, ctypes.c_int, ctypes.POINTER(_Report),
        ]
        lib.or_fgmres.restype = ctypes.c_int
        lib.or_fgmres_eo.argtypes = [
            ctypes.POINTER(_Op), vp, vp, ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int, ip,
            ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(_Report),
        ]
        lib.or_fgmres_eo.restype = ctypes.c_int
        lib.or_dhat.argtypes = [ctypes.POINTER(_Op), vp, vp]
        lib.or_dhat_dag.argtypes = [ctypes.POINTER(_Op), vp, vp]
        lib.or_cg_eo.argtypes = [ctypes.POINTER(_Op), vp, vp, ctypes.c_double, ctypes.c_int, ctypes.POINTER(_Report)]
        lib.or_cg_eo.restype = ctypes.c_int
        cp = ctypes.c_void_p
        lib.or_mg_block_orthonormalize.argtypes = [ip, ip, ctypes.c_int, vp, vp]
        lib.or_mg_restrict.argtypes = [ip, ip, ctypes.c_int, vp, vp, vp]
        lib.or_mg_prolong.argtypes = [ip, ip, ctypes.c_int, vp, vp, vp]
        lib.or_mg_coarse_build.argtypes = [ctypes.POINTER(_Op), ip, ctypes.c_int, vp, vp]
        lib.or_mg_coarse_apply.argtypes = [ip, ctypes.c_int, vp, ctypes.c_double, vp, vp]
        lib.or_mg_coarse_gmres.argtypes = [ip, ctypes.c_int, vp, ctypes.c_double, vp, vp, ctypes.c_double,
                                           ctypes.c_int, ctypes.c_int, ctypes.POINTER(_Report)]
        lib.or_mg_coarse_gmres.restype = ctypes.c_int
        lib.or_mg_precond.argtypes = [ctypes.POINTER(_Op), ctypes.POINTER(_MG), vp, vp]
        lib.or_mg_coarse_dhat.argtypes = [ip, ctypes.c_int, vp, ctypes.c_double, vp, vp]
        lib.or_mg_coarse_gmres_eo.argtypes = [ip, ctypes.c_int, vp, ctypes.c_double, vp, vp, ctypes.c_double,
                                              ctypes.c_int, ctypes.c_int, ctypes.POINTER(_Report)]
        lib.or_mg_coarse_gmres_eo.restype = ctypes.c_int
        lib.or_fgmres_mg.argtypes = [ctypes.POINTER(_Op), ctypes.POINTER(_MG), vp, vp, ctypes.c_double, ctypes.c_int,
                                     ctypes.c_int, ctypes.POINTER(_Report)]
        lib.or_fgmres_mg.restype = ctypes.c_int
        lib.or_mg_setup.argtypes = [ctypes.POINTER(_Op), ctypes.POINTER(_MG), vp, cp]
        lib.or_mg_setup.restype = ctypes.c_int
        lib.or_num_threads.restype = ctypes.c_int
        lib.or_set_num_threads.argtypes = [ctypes.c_int]
        _lib = lib
    return _lib


def _i4(v):
    return (ctypes.c_int * 4)(*[int(a) for a in v])


def _c128(a):
    a = np.ascontiguousarray(a, dtype=np.complex128)
    return a


def kappa_to_m(kappa: float) -> float:
    """Hopping-parameter relation m + 4 = 1 / (2 kappa)."""
    return 1.0 / (2.0 * kappa) - 4.0


def volume(dims) -> int:
    return int(np.prod(dims))


def gamma(mu: int) -> np.ndarray:
    g = np.zeros(16, np.complex128)
    _load().or_gamma(mu, g.ctypes.data)
    return g.reshape(4, 4)


def clover(dims, U, csw: float) -> np.ndarray:
    U = _c128(U)
    V = volume(dims)
    out = np.zeros((V, 12, 12), np.complex128)
    _load().or_clover(_i4(dims), U.ctypes.data, float(csw), out.ctypes.data)
    return out


class Operator:
    """D(mu) = (m+4) + clover - 1/2 hops + i mu Gamma5 on a periodic lattice."""

    def __init__(self, dims, U, m: float, mu: float, csw: float = 0.0, antiperiodic_t: bool = False,
                 clov: np.ndarray | None = None, theta=(0.0, 0.0, 0.0, 0.0), mu_shift=(0.0, 0.0)):
        """theta: twisted boundary phases (radians) for t, x, y, z; mu_shift: added to mu on
        even / odd sites."""
        self.theta = tuple(float(t) for t in theta)
        self.mu_shift = tuple(float(t) for t in mu_shift)
        self.dims = tuple(int(d) for d in dims)
        self.V = volume(self.dims)
        self.U = _c128(U).reshape(self.V, 4, 3, 3)
        self.m, self.mu, self.csw = float(m), float(mu), float(csw)
        self.antiperiodic_t = bool(antiperiodic_t)
        if clov is not None:
            self.clov = _c128(clov)
        elif self.csw != 0.0:
            self.clov = clover(self.dims, self.U, self.csw)
        else:
            self.clov = None
        self._op = _Op(_i4(self.dims), int(self.antiperiodic_t), self.U.ctypes.data,
                       self.clov.ctypes.data if self.clov is not None else None, self.m, self.mu,
                       (ctypes.c_double * 4)(*self.theta), (ctypes.c_double * 2)(*self.mu_shift))

    def with_mu(self, mu: float) -> "Operator":
        return Operator(self.dims, self.U, self.m, mu, self.csw, self.antiperiodic_t, self.clov, self.theta,
                        self.mu_shift)

    def _vec(self, v):
        v = _c128(v)
        assert v.size == self.V * 12, (v.shape, self.V)
        return v

    def apply(self, psi) -> np.ndarray:
        psi = self._vec(psi)
        out = np.empty_like(psi)
        _load().or_dirac(ctypes.byref(self._op), psi.ctypes.data, out.ctypes.data)
        return out

    def apply_blockdiag(self, psi, bdims) -> np.ndarray:
        psi = self._vec(psi)
        out = np.empty_like(psi)
        _load().or_dirac_blockdiag(ctypes.byref(self._op), _i4(bdims), psi.ctypes.data, out.ctypes.data)
        return out

    def block_colour(self, bdims, site: int) -> int:
        return _load().or_block_colour(_i4(self.dims), _i4(bdims), int(site))

    def mr_block(self, bdims, B, r, iters: int) -> np.ndarray:
        r = self._vec(r)
        e = np.zeros_like(r)
        _load().or_mr_block(ctypes.byref(self._op), _i4(bdims), _i4(B), r.ctypes.data, e.ctypes.data, int(iters))
        return e

    def mr_block_eo(self, bdims, B, r, iters: int) -> np.ndarray:
        """Even-odd preconditioned MR block solve (odd-site Schur complement)."""
        r = self._vec(r)
        e = np.zeros_like(r)
        _load().or_mr_block_eo(ctypes.byref(self._op), _i4(bdims), _i4(B), r.ctypes.data, e.ctypes.data,
                               int(iters))
        return e

    def sap(self, b, bdims, n_cycles: int, mr_iters: int, x0=None, eo: bool = False) -> np.ndarray:
        b = self._vec(b)
        x = np.zeros_like(b) if x0 is None else self._vec(x0).copy()
        rc = _load().or_sap_eo(ctypes.byref(self._op), _i4(bdims), int(n_cycles), int(mr_iters), int(bool(eo)),
                               b.ctypes.data, x.ctypes.data)
        if rc != 0:
            raise ValueError(f"or_sap rejected block shape {bdims} (code {rc})")
        return x

    def fgmres(self, b, tol: float, restart: int = 20, max_iters: int = 2000, precond: bool = True,
               bdims=(2, 2, 2, 2), n_cycles: int = 3, mr_iters: int = 4, x0=None, eo: bool = False):
        b = self._vec(b)
        x = np.zeros_like(b) if x0 is None else self._vec(x0).copy()
        rep = _Report()
        _load().or_fgmres_eo(ctypes.byref(self._op), b.ctypes.data, x.ctypes.data, float(tol), int(restart),
                             int(max_iters), int(bool(precond)), _i4(bdims), int(n_cycles), int(mr_iters),
                             int(bool(eo)), ctypes.byref(rep))
        return x, {"iters": rep.iters, "restarts": rep.restarts, "converged": bool(rep.converged),
                   "true_rel_res": rep.true_rel_res}

    def dhat(self, v) -> np.ndarray:
        """Even-odd reduced operator D_ee - D_eo D_oo^-1 D_oe on the even sites of v."""
        v = self._vec(v)
        out = np.empty_like(v)
        _load().or_dhat(ctypes.byref(self._op), v.ctypes.data, out.ctypes.data)
        return out

    def dhat_dag(self, v) -> np.ndarray:
        v = self._vec(v)
        out = np.empty_like(v)
        _load().or_dhat_dag(ctypes.byref(self._op), v.ctypes.data, out.ctypes.data)
        return out

    def cg_eo(self, b, tol: float, max_iters: int = 100000, x0=None):
        """CG on the squared even-odd reduced system, then the odd sites; returns (x, report)."""
        b = self._vec(b)
        x = np.zeros_like(b) if x0 is None else self._vec(x0).copy()
        rep = _Report()
        _load().or_cg_eo(ctypes.byref(self._op), b.ctypes.data, x.ctypes.data, float(tol), int(max_iters),
                         ctypes.byref(rep))
        return x, {"iters": rep.iters, "converged": bool(rep.converged), "true_rel_res": rep.true_rel_res}

    def dense(self) -> np.ndarray:
        """Dense matrix of D (12V x 12V), built column by column; tiny lattices only."""
        n = self.V * 12
        M = np.zeros((n, n), np.complex128)
        e = np.zeros(n, np.complex128)
        for j in range(n):
            e[j] = 1.0
            M[:, j] = self.apply(e)
            e[j] = 0.0
        return M

    def dense_blockdiag(self, bdims) -> np.ndarray:
        n = self.V * 12
        M = np.zeros((n, n), np.complex128)
        e = np.zeros(n, np.complex128)
        for j in range(n):
            e[j] = 1.0
            M[:, j] = self.apply_blockdiag(e, bdims)
            e[j] = 0.0
        return M


def num_threads() -> int:
    return _load().or_num_threads()


def set_num_threads(n: int) -> None:
    _load().or_set_num_threads(int(n))


class MG:
    """Two-level method of sections 2.3-2.6 on one Operator's lattice.

    Aggregates: blocks `adims` x spin halves ({0,1}, {2,3}) x colour.  P holds
    nv lattice vectors [nv][V][4][3] orthonormal on every aggregate; a coarse
    vector is [nc][2 nv] (coarse sites lexicographic in block coordinates,
    component sg*nv + i); Dc [nc][9][2nv][2nv] is the Galerkin stencil without
    the twist (term 0 = the site, 1 + mu = from one aggregate forward along mu,
    5 + mu = backward); the coarse operator is Dc + i delta mu Gamma5c.
    """

    def __init__(self, op: Operator, adims, nv: int, delta: float = 1.0, coarse_tol: float = 0.1,
                 coarse_restart: int = 100, coarse_max_restarts: int = 5, post_cycles: int = 4, mr_iters: int = 4,
                 setup_iters: int = 0, setup_cycles: int = 4, coarse_eo: bool = False):
        self.op = op
        self.adims = tuple(int(a) for a in adims)
        self.nv = int(nv)
        self.cdims = tuple(d // a for d, a in zip(op.dims, self.adims))
        self.nc = volume(self.cdims)
        self.P = np.zeros((self.nv, op.V, 4, 3), np.complex128)
        self.Dc = np.zeros((self.nc, 9, 2 * self.nv, 2 * self.nv), np.complex128)
        self._mg = _MG(_i4(self.adims), self.nv, float(delta), float(coarse_tol), int(coarse_restart),
                       int(coarse_max_restarts), int(post_cycles), int(mr_iters), int(setup_iters), int(setup_cycles),
                       int(bool(coarse_eo)), self.P.ctypes.data, self.Dc.ctypes.data)

    @property
    def delta(self) -> float:
        return self._mg.delta

    def setup(self, v0) -> np.ndarray:
        """Adaptive setup from the starting vectors v0 [nv][V][4][3]; setup_iters = 0 only orthonormalises v0
        aggregate-wise and builds the coarse stencil.  Returns the final test vectors."""
        v0 = _c128(v0).reshape(self.nv, self.op.V, 4, 3)
        out = np.zeros_like(v0)
        rc = _load().or_mg_setup(ctypes.byref(self.op._op), ctypes.byref(self._mg), v0.ctypes.data, out.ctypes.data)
        if rc != 0:
            raise ValueError(f"or_mg_setup failed (code {rc})")
        return out

    def block_orthonormalize(self, v) -> np.ndarray:
        v = _c128(v).reshape(self.nv, self.op.V, 4, 3)
        out = np.empty_like(v)
        _load().or_mg_block_orthonormalize(_i4(self.op.dims), _i4(self.adims), self.nv, v.ctypes.data,
                                           out.ctypes.data)
        return out

    def restrict(self, r) -> np.ndarray:
        r = self.op._vec(r)
        c = np.empty((self.nc, 2 * self.nv), np.complex128)
        _load().or_mg_restrict(_i4(self.op.dims), _i4(self.adims), self.nv, self.P.ctypes.data, r.ctypes.data,
                               c.ctypes.data)
        return c

    def prolong(self, c) -> np.ndarray:
        c = _c128(c).reshape(self.nc, 2 * self.nv)
        e = np.empty((self.op.V, 4, 3), np.complex128)
        _load().or_mg_prolong(_i4(self.op.dims), _i4(self.adims), self.nv, self.P.ctypes.data, c.ctypes.data,
                              e.ctypes.data)
        return e

    def coarse_build(self, op: Operator | None = None) -> None:
        _load().or_mg_coarse_build(ctypes.byref((op or self.op)._op), _i4(self.adims), self.nv, self.P.ctypes.data,
                                   self.Dc.ctypes.data)

    def coarse_apply(self, x, mu_c: float) -> np.ndarray:
        x = _c128(x).reshape(self.nc, 2 * self.nv)
        y = np.empty_like(x)
        _load().or_mg_coarse_apply(_i4(self.cdims), self.nv, self.Dc.ctypes.data, float(mu_c), x.ctypes.data,
                                   y.ctypes.data)
        return y

    def coarse_gmres(self, b, mu_c: float, tol: float, restart: int, max_restarts: int):
        b = _c128(b).reshape(self.nc, 2 * self.nv)
        x = np.empty_like(b)
        rep = _Report()
        _load().or_mg_coarse_gmres(_i4(self.cdims), self.nv, self.Dc.ctypes.data, float(mu_c), b.ctypes.data,
                                   x.ctypes.data, float(tol), int(restart), int(max_restarts), ctypes.byref(rep))
        return x, {"iters": rep.iters, "restarts": rep.restarts, "met": bool(rep.converged),
                   "rel_estimate": rep.true_rel_res}

    def coarse_dhat(self, x, mu_c: float) -> np.ndarray:
        """Even-odd reduced coarse operator on the odd coarse sites of x (even parts ignored, zero in the result)."""
        x = _c128(x).reshape(self.nc, 2 * self.nv)
        y = np.empty_like(x)
        _load().or_mg_coarse_dhat(_i4(self.cdims), self.nv, self.Dc.ctypes.data, float(mu_c), x.ctypes.data,
                                  y.ctypes.data)
        return y

    def coarse_gmres_eo(self, b, mu_c: float, tol: float, restart: int, max_restarts: int):
        b = _c128(b).reshape(self.nc, 2 * self.nv)
        x = np.empty_like(b)
        rep = _Report()
        _load().or_mg_coarse_gmres_eo(_i4(self.cdims), self.nv, self.Dc.ctypes.data, float(mu_c), b.ctypes.data,
                                      x.ctypes.data, float(tol), int(restart), int(max_restarts), ctypes.byref(rep))
        return x, {"iters": rep.iters, "restarts": rep.restarts, "met": bool(rep.converged),
                   "rel_estimate": rep.true_rel_res}

    def precond(self, r, op: Operator | None = None) -> np.ndarray:
        op = op or self.op
        r = op._vec(r)
        z = np.empty_like(r)
        _load().or_mg_precond(ctypes.byref(op._op), ctypes.byref(self._mg), r.ctypes.data, z.ctypes.data)
        return z

    def fgmres(self, b, tol: float, restart: int = 20, max_iters: int = 2000, op: Operator | None = None, x0=None):
        op = op or self.op
        b = op._vec(b)
        x = np.zeros_like(b) if x0 is None else op._vec(x0).copy()
        rep = _Report()
        _load().or_fgmres_mg(ctypes.byref(op._op), ctypes.byref(self._mg), b.ctypes.data, x.ctypes.data, float(tol),
                             int(restart), int(max_iters), ctypes.byref(rep))
        return x, {"iters": rep.iters, "restarts": rep.restarts, "converged": bool(rep.converged),
                   "true_rel_res": rep.true_rel_res}
