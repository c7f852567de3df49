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
    # the library's own defaults, down to the last field of the struct (x is read by default)
    raw = tm.SolverOpts()
    tm.lib().tm_solver_opts_default(ctypes.byref(raw))
    assert raw.x_in == 1 and raw.mg is None and raw.inner_tol == 1e-6
    # the FMA probe rejects a missing output before it touches a device
    o = tm.make_opts("f32", stream=False)
    assert tm.lib().tm_probe_fp32_fma(None, ctypes.byref(o)) == -1


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


def read_golden(name):
    vals = {}
    with open(os.path.join(ROOT, "tests", "golden", name)) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                k, *v = line.split()
                vals[k] = v
    return vals


def test_table1_multigrid_defaults_match_library():
    # the two-level defaults are the paper's tuned set (Table 1) where a two-level method has the parameter
    vals = read_golden("table1_mg_defaults.txt")
    p = tm.mg_params()
    assert p.setup_iters == int(vals["setup_iterations"][0])
    assert p.n_vec == int(vals["test_vectors_level1"][0])
    assert tuple(p.block_dims) == tuple(int(v) for v in vals["aggregate_dims"])
    assert tuple(p.block_dims) == tuple(int(v) for v in vals["smoother_block_dims"])
    assert p.post_cycles == int(vals["post_smoothing_steps"][0])
    assert p.delta == float(vals["coarse_mu_factor"][0])
    assert p.coarse_restart == int(vals["coarse_restart"][0])
    assert p.coarse_max_restarts == int(vals["coarse_max_restarts"][0])
    assert p.coarse_tol == float(vals["coarse_relative_tolerance"][0])
    assert vals["coarse_solver"][0] == "even_odd_gmres" and p.coarse_eo == 1
    sap = read_golden("table1_sap_defaults.txt")
    assert p.mr_iters == int(sap["block_mr_iterations"][0])


def test_two_level_setup_rejects_bad_input_on_host():
    g = tm.make_geom((8, 8, 8, 8), 0.01)
    o = tm.make_opts("f32", stream=False)
    h = ctypes.c_void_p()
    dummy = ctypes.c_void_p(16)
    L = tm.lib()
    for kw, code in (({"n_vec": 0}, -1), ({"n_vec": 33}, -1), ({"coarse_restart": 129}, -1), ({"delta": 0.0}, -1),
                     ({"coarse_eo": 2}, -1), ({"block_dims": (4, 4, 4, 3)}, -2), ({"block_dims": (8, 4, 4, 4)}, -3)):
        p = tm.mg_params(**kw)
        rc = L.tm_mg_setup(ctypes.byref(g), dummy, 0.15, 1.0, ctypes.byref(p), dummy, ctypes.byref(h), ctypes.byref(o))
        assert rc == code, (kw, rc)
        assert not h.value
    # FP32 only, one setup twist
    p = tm.mg_params()
    o64 = tm.make_opts("f64", stream=False)
    assert L.tm_mg_setup(ctypes.byref(g), dummy, 0.15, 1.0, ctypes.byref(p), dummy, ctypes.byref(h),
                         ctypes.byref(o64)) == -4
    g2 = tm.make_geom((8, 8, 8, 8), [0.01, -0.01])
    assert L.tm_mg_setup(ctypes.byref(g2), dummy, 0.15, 1.0, ctypes.byref(p), dummy, ctypes.byref(h),
                         ctypes.byref(o)) == -1


def test_binding_checks_buffer_sizes_before_any_library_call():
    # a buffer smaller or larger than dims and the number of systems imply is refused on the host (a kernel
    # would otherwise read or write past it); the tensors here are host tensors, so a call whose sizes are
    # right stops at the device check instead
    import torch

    dims = (4, 4, 4, 8)
    V = 4 * 4 * 4 * 8
    U = torch.zeros((V, 4, 3, 3), dtype=torch.complex128)
    psi = torch.zeros((2, V, 4, 3), dtype=torch.complex128)
    with pytest.raises(ValueError, match="U has"):
        tm.tm_dirac_apply(dims, U[: V // 2], psi, 0.15, [0.1, -0.1], 1.0, stream=False)
    with pytest.raises(ValueError, match="psi has"):
        tm.tm_dirac_apply(dims, U, psi, 0.15, [0.1, -0.1, 0.2], 1.0, stream=False)
    with pytest.raises(ValueError, match="b has"):
        tm.tm_sap_smooth(dims, U, psi[:1], psi[1:].clone(), 0.15, [0.1, -0.1], 1.0, (2, 2, 2, 2), 1, 1, stream=False)
    with pytest.raises(ValueError, match="x has"):
        tm.tm_fgmres_solve(dims, U, psi, psi[:1].clone(), 0.15, [0.1, -0.1], 1.0, 1e-10, stream=False)
    with pytest.raises(ValueError, match="b has"):
        tm.tm_cg_solve(dims, U, psi, psi.clone(), 0.15, [0.1], 1.0, 1e-10, stream=False)
    need = tm.tm_spinor_bytes(dims, 2, "f16", layout_block=(2, 2, 2, 2))
    small = torch.zeros(need - 1, dtype=torch.uint8)
    with pytest.raises(ValueError, match="internal holds"):
        tm.tm_spinor_import(dims, psi, small, storage="f16", layout_block=(2, 2, 2, 2), stream=False)
    with pytest.raises(ValueError, match="b holds"):
        tm.tm_sap_smooth(dims, U, small, small, 0.15, [0.1, -0.1], 1.0, (2, 2, 2, 2), 1, 1, storage="f16",
                         io="internal", stream=False)
    with pytest.raises(ValueError, match="canon has"):
        tm.tm_spinor_import_range(dims, psi[:, : V // 2].contiguous(), torch.zeros(need, dtype=torch.uint8), 2, 0,
                                  storage="f16",
                                  layout_block=(2, 2, 2, 2), stream=False)
    # sizes right: only the device check is left
    with pytest.raises(ValueError, match="live on the GPU"):
        tm.tm_dirac_apply(dims, U, psi, 0.15, [0.1, -0.1], 1.0, stream=False)
    with pytest.raises(ValueError, match="live on the GPU"):
        tm.tm_spinor_import(dims, psi, torch.zeros(need, dtype=torch.uint8), storage="f16",
                            layout_block=(2, 2, 2, 2), stream=False)
