"""The C-ABI library loads on the host and exports every entry point its header declares.

No compute call is made here (no GPU in the CPU suite); tm_spinor_bytes and the
option defaults are pure host code and are checked too.
"""
import ctypes
import os
import re

import pytest

import paper_1610_02370_amd as tm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_entry_points():
    src = open(os.path.join(ROOT, "include", "tm.h")).read()
    return sorted(set(re.findall(r"TM_API\s+[\w\s\*]+?\b(tm_\w+)\s*\(", src)))


def test_header_declares_binding_exports():
    assert declared_entry_points() == sorted(tm.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = tm.lib()
    for name in declared_entry_points():
        assert hasattr(L, name), name
        assert ctypes.cast(getattr(L, name), ctypes.c_void_p).value


def test_host_only_calls():
    # 8x8x8x8 at FP64: 6 units of 32 bytes per site and system
    n = tm.tm_spinor_bytes((8, 8, 8, 8), 2, "f64")
    assert n == 2 * 6 * 4096 * 32
    # FP16 adds one FP32 scale per site and system (256-byte aligned parts)
    n16 = tm.tm_spinor_bytes((8, 8, 8, 8), 3, "f16")
    assert n16 == 3 * 6 * 4096 * 8 + 3 * 4096 * 4
    s = tm.solver_opts()
    assert (s.restart, s.n_cycles, s.mr_iters, tuple(s.block_dims)) == (20, 4, 4, (4, 4, 4, 4))


def test_table1_block_default_matches_library():
    # the library's default Schwarz block is the paper's level-1 SAP block (Table 1)
    vals = {}
    with open(os.path.join(ROOT, "tests", "golden", "table1_sap_defaults.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                k, *v = line.split()
                vals[k] = v
    s = tm.solver_opts()
    assert tuple(int(v) for v in vals["block_dims"]) == tuple(s.block_dims)


def test_bad_arguments_rejected_on_host():
    # geometry errors are detected before any device call
    g = tm.make_geom((0, 4, 4, 4), 0.1)
    o = tm.make_opts("f64", stream=False)
    rc = tm.lib().tm_dirac_apply(ctypes.byref(g), None, None, None, 0.15, 0.0, ctypes.byref(o))
    assert rc == -2
    g = tm.make_geom((4, 4, 4, 4), [0.1] * 65)
    rc = tm.lib().tm_dirac_apply(ctypes.byref(g), None, None, None, 0.15, 0.0, ctypes.byref(o))
    assert rc == -1
    o = tm.make_opts("f16", compute="f64", stream=False)
    g = tm.make_geom((4, 4, 4, 4), 0.1)
    rc = tm.lib().tm_dirac_apply(ctypes.byref(g), None, None, None, 0.15, 0.0, ctypes.byref(o))
    assert rc == -4
