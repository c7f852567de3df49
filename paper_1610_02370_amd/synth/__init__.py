"""Seeded synthetic inputs shared by the GPU tests, the benchmark and the oracle tests.

Holds none of the solver's arithmetic: SU(3) links U = exp(i eps H) (H a Gaussian
combination of Gell-Mann matrices, Philox4x32-10 counters), Gaussian spinors and
point sources, all in the canonical complex128 layout:
  links  [V][4][3][3]  (direction mu: 0 = t, 1 = x, 2 = y, 3 = z)
  spinor [nsys][V][4][3]
Sites are lexicographic over dims = (T, Z, Y, X), t slowest.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synth.c")
_LIB = os.path.join(_HERE, "libtmsynth.so")
_lib = None

GAUGE_TAG = 0x67617567      # stream tag for gauge links
GAUGE_XFORM_TAG = 0x78666F72  # stream tag for gauge transformations
SPINOR_TAG = 0x73706E72     # stream tag for Gaussian spinors


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-std=c11", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        vp, u32, i64, dbl = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_int64, ctypes.c_double
        lib.synth_philox4x32_10.argtypes = [vp, vp, vp]
        lib.synth_gauge.argtypes = [u32, u32, dbl, i64, vp]
        lib.synth_gauge_sites.argtypes = [u32, u32, dbl, i64, vp, vp]
        lib.synth_su3_field.argtypes = [u32, u32, dbl, i64, vp]
        lib.synth_gaussian.argtypes = [u32, u32, i64, vp]
        _lib = lib
    return _lib


def philox4x32_10(ctr, key) -> tuple:
    c = np.array(ctr, np.uint32)
    k = np.array(key, np.uint32)
    o = np.zeros(4, np.uint32)
    _load().synth_philox4x32_10(c.ctypes.data, k.ctypes.data, o.ctypes.data)
    return tuple(int(v) for v in o)


def volume(dims) -> int:
    return int(np.prod([int(d) for d in dims]))


def gauge_field(dims, eps: float, seed: int) -> np.ndarray:
    """Links [V][4][3][3] complex128 for the whole lattice."""
    V = volume(dims)
    out = np.empty((V, 4, 3, 3), np.complex128)
    _load().synth_gauge(int(seed), GAUGE_TAG, float(eps), V, out.ctypes.data)
    return out


def gauge_links_at(sites, eps: float, seed: int) -> np.ndarray:
    """Links of selected sites only (same values as gauge_field at those sites)."""
    s = np.ascontiguousarray(np.asarray(sites, np.int64))
    out = np.empty((s.size, 4, 3, 3), np.complex128)
    _load().synth_gauge_sites(int(seed), GAUGE_TAG, float(eps), s.size, s.ctypes.data, out.ctypes.data)
    return out


def su3_field(dims, eps: float, seed: int) -> np.ndarray:
    """One SU(3) matrix per site [V][3][3] (for gauge transformations)."""
    V = volume(dims)
    out = np.empty((V, 3, 3), np.complex128)
    _load().synth_su3_field(int(seed), GAUGE_XFORM_TAG, float(eps), V, out.ctypes.data)
    return out


def gaussian_spinor(dims, nsys: int, seed: int) -> np.ndarray:
    """[nsys][V][4][3] complex128 with re, im i.i.d. N(0,1)."""
    V = volume(dims)
    out = np.empty((nsys, V, 4, 3), np.complex128)
    _load().synth_gaussian(int(seed), SPINOR_TAG, out.size, out.ctypes.data)
    return out


def point_sources(dims, components, site: int = 0) -> np.ndarray:
    """One system per (spin, colour) in `components`: 1 at `site`, that component."""
    V = volume(dims)
    out = np.zeros((len(components), V, 4, 3), np.complex128)
    for k, (s, c) in enumerate(components):
        out[k, site, s, c] = 1.0
    return out


def all_point_sources(dims, site: int = 0) -> np.ndarray:
    """The 12 sources of a point-to-all propagator (spin-major order)."""
    return point_sources(dims, [(s, c) for s in range(4) for c in range(3)], site)
