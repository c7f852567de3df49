"""GPU solve parity: tm_fgmres_solve (HIP) against the FP64 CPU oracle.

The solution of D(mu) x = b is unique, so the check is on x, not on iteration
counts: the true residual ||b - D x|| / ||b|| is recomputed with the ORACLE's
operator from the returned x and must meet the tolerance, and since every
singular value of D(mu) is >= |mu| (section 2.1), ||x - x*|| <= ||b - D x|| / |mu|
bounds the distance to the exact solution.  On 4^4 the exact solution comes
from dense LU and is compared directly.
"""
import numpy as np
import pytest

import oracle
import paper_1610_02370_amd as tm
from paper_1610_02370_amd import synth

from gpu_util import announce, dev, host, log_solve

pytestmark = pytest.mark.gpu

TOL = 1e-10
RES_SLACK = 1.05  # FP64 rounding of the oracle's recomputed residual


@pytest.fixture(scope="module")
def cfg_4444():
    dims, eps, kappa, mu, csw = (4, 4, 4, 4), 0.3, 0.16, 0.01, 0.0
    U = synth.gauge_field(dims, eps, seed=1)
    b = synth.gaussian_spinor(dims, 1, seed=101)
    op = oracle.Operator(dims, U, oracle.kappa_to_m(kappa), mu, csw)
    xs = np.linalg.solve(op.dense(), b[0].ravel())
    return dims, kappa, mu, csw, U, b, op, xs


@pytest.mark.parametrize("form,storage", [("flexible", "f64"), ("flexible", "f32"), ("flexible", "f16"),
                                          ("defect_correction", "f32"), ("defect_correction", "f16"),
                                          ("defect_correction", "bf16")])
def test_4x4x4x4_solve_against_dense_lu(cfg_4444, form, storage):
    dims, kappa, mu, csw, U, b, op, xs = cfg_4444
    announce(f"solve 4^4 form={form} storage={storage}")
    x = dev(np.zeros_like(b))
    rc, rep = tm.tm_fgmres_solve(dims, dev(U), dev(b), x, kappa, [mu], csw, TOL, storage=storage, form=form,
                                 restart=20, n_cycles=3, mr_iters=4, block_dims=(2, 2, 2, 2))
    assert rc == 0 and rep["converged"] == 1, rep
    xg = host(x)[0].ravel()
    r = b[0].ravel() - op.apply(xg)
    rel = np.linalg.norm(r) / np.linalg.norm(b)
    log_solve(f"4^4 {form}", storage, rel, TOL, rep["iters"])
    assert rel <= TOL * RES_SLACK, rel
    assert abs(rep["true_rel_res"][0] - rel) <= 0.05 * TOL
    # sigma_min >= |mu| bounds the error; the dense solution confirms it
    err = np.linalg.norm(xg - xs)
    assert err <= np.linalg.norm(r) / mu * 1.01
    assert err / np.linalg.norm(xs) < 1e-8


def test_4x4x4x4_oracle_fgmres_agrees(cfg_4444):
    dims, kappa, mu, csw, U, b, op, xs = cfg_4444
    announce("solve 4^4 oracle FGMRES vs GPU FGMRES")
    xo, rep_o = op.fgmres(b[0].ravel(), 1e-12, restart=20, precond=True, bdims=(2, 2, 2, 2), n_cycles=3, mr_iters=4)
    x = dev(np.zeros_like(b))
    tm.tm_fgmres_solve(dims, dev(U), dev(b), x, kappa, [mu], csw, 1e-12, storage="f64", restart=20, n_cycles=3,
                       mr_iters=4, block_dims=(2, 2, 2, 2))
    assert np.linalg.norm(host(x)[0].ravel() - xo) < 1e-9 * np.linalg.norm(xo)


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_long_cycles_against_dense_lu(cfg_4444, storage):
    # FGMRES(22) with one SAP cycle of one MR step: cycles run to their full length, so the
    # Gram-Schmidt sweeps see every basis size up to 22 (dots in several sweeps of at most 8
    # FP32 or 4 FP64 vectors, updates over up to 22 vectors)
    dims, kappa, mu, csw, U, b, op, xs = cfg_4444
    announce(f"solve 4^4 restart 22, weak smoother, {storage}")
    b2 = np.concatenate([b, b])
    x = dev(np.zeros_like(b2))
    rc, rep = tm.tm_fgmres_solve(dims, dev(U), dev(b2), x, kappa, [mu, -mu], csw, TOL, storage=storage,
                                 form="flexible", restart=22, n_cycles=1, mr_iters=1, block_dims=(2, 2, 2, 2),
                                 max_iters=400)
    assert rc == 0 and rep["converged"] == 2, rep
    assert rep["iters"] > 22, rep  # at least one full cycle and a restart
    xg = host(x)
    for k, m in enumerate([mu, -mu]):
        ref = np.linalg.solve(op.with_mu(m).dense(), b[0].ravel())
        r = b[0].ravel() - op.with_mu(m).apply(xg[k].ravel())
        rel = np.linalg.norm(r) / np.linalg.norm(b)
        log_solve(f"4^4 restart 22 system {k}", storage, rel, TOL, rep["iters"])
        assert rel <= TOL * RES_SLACK, (k, rel)
        assert np.linalg.norm(xg[k].ravel() - ref) / np.linalg.norm(ref) < 1e-8


def test_w_from_smoother_matches_full_operator(tmp_path):
    # FP32 storage, 4^4 blocks: the Arnoldi step takes D z from the smoother's last half-sweep on
    # one colour and runs the operator on the other.  The same solve in a process that selects the
    # general-shape FP32 kernel (TM_SAP_KERNEL=v2) forms D z with the operator everywhere.  The two
    # differ only in FP32 rounding: the same iterations up to one step where an estimate sits at a
    # tolerance, both solutions within 1e-10 by the oracle, and so within 2e-10 ||b|| / |mu| of each
    # other (sigma_min >= |mu|)
    import os
    import subprocess
    import sys

    dims, kappa, mu, csw = (8, 8, 8, 8), 0.1632, 0.003, 1.5
    U = synth.gauge_field(dims, 0.5, seed=2)
    b = synth.point_sources(dims, [(0, 0), (1, 2)])
    mus = [mu, -mu]
    kw = dict(storage="f32", form="defect_correction", restart=8, n_cycles=3, mr_iters=4, block_dims=(4, 4, 4, 4))
    announce("solve with D z from the smoother against the full operator (child process, v2 kernel)")
    x = dev(np.zeros_like(b))
    rc, rep = tm.tm_fgmres_solve(dims, dev(U), dev(b), x, kappa, mus, csw, TOL, **kw)
    assert rc == 0, rep
    np.savez(tmp_path / "in.npz", U=U, b=b)
    child = f"""
import sys, numpy as np, torch
sys.path.insert(0, {os.path.dirname(os.path.dirname(os.path.abspath(__file__)))!r})
import paper_1610_02370_amd as tm
d = np.load({str(tmp_path / "in.npz")!r})
x = torch.zeros(d["b"].shape, dtype=torch.complex128, device="cuda")
rc, rep = tm.tm_fgmres_solve({dims!r}, torch.from_numpy(d["U"]).cuda(), torch.from_numpy(d["b"]).cuda(), x,
                             {kappa!r}, {mus!r}, {csw!r}, {TOL!r}, **{kw!r})
np.savez({str(tmp_path / "out.npz")!r}, x=x.cpu().numpy(), rc=rc, iters=rep["iters"], outer=rep["outer"])
"""
    env = dict(os.environ, TM_SAP_KERNEL="v2")
    r = subprocess.run([sys.executable, "-c", child], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    o = np.load(tmp_path / "out.npz")
    assert int(o["rc"]) == 0
    assert abs(rep["iters"] - int(o["iters"])) <= 1 and abs(rep["outer"] - int(o["outer"])) <= 1, \
        (rep, o["iters"], o["outer"])
    xg = host(x)
    op = oracle.Operator(dims, U, oracle.kappa_to_m(kappa), mu, csw)
    check_solutions(op, dims, b, xg, mus, TOL, "8^4 D z from the smoother", "f32")
    check_solutions(op, dims, b, o["x"], mus, TOL, "8^4 D z from the operator", "f32")
    for k in range(2):
        assert np.linalg.norm(xg[k] - o["x"][k]) <= 2 * TOL * RES_SLACK * np.linalg.norm(b[k]) / mu


@pytest.fixture(scope="module")
def cfg_8888():
    dims, eps, kappa, mu, csw = (8, 8, 8, 8), 0.5, 0.1632, 0.003, 1.5
    U = synth.gauge_field(dims, eps, seed=2)
    op = oracle.Operator(dims, U, oracle.kappa_to_m(kappa), 0.0, csw)
    return dims, kappa, mu, csw, U, op


def check_solutions(op, dims, b, x, mus, tol, label="", prec=""):
    for k, m in enumerate(mus):
        r = b[k].ravel() - op.with_mu(m).apply(x[k].ravel())
        rel = np.linalg.norm(r) / np.linalg.norm(b[k])
        log_solve(f"{label} {dims} system {k}", prec, rel, tol)
        assert rel <= tol * RES_SLACK, (k, rel)


@pytest.mark.parametrize("form,storage", [("flexible", "f64"), ("flexible", "f32"), ("defect_correction", "f32"),
                                          ("defect_correction", "f16"), ("defect_correction", "bf16")])
def test_8x8x8x8_point_source_pm_mu(cfg_8888, form, storage):
    dims, kappa, mu, csw, U, op = cfg_8888
    announce(f"solve 8^4 +-mu form={form} storage={storage}")
    b = synth.point_sources(dims, [(0, 0), (0, 0)])
    mus = [mu, -mu]
    x = dev(np.zeros_like(b))
    rc, rep = tm.tm_fgmres_solve(dims, dev(U), dev(b), x, kappa, mus, csw, TOL, storage=storage, form=form,
                                 restart=16, n_cycles=4, mr_iters=4, block_dims=(4, 4, 4, 4))
    assert rc == 0 and rep["converged"] == 2, rep
    check_solutions(op, dims, b, host(x), mus, TOL, f"8^4 +-mu {form}", storage)


def test_8x8x8x8_twelve_sources_grouped(cfg_8888):
    # all 12 spin-colour point sources; group=5 forces groups of 5, 5 and 2
    dims, kappa, mu, csw, U, op = cfg_8888
    announce("solve 8^4 twelve sources, groups of 5")
    b = synth.all_point_sources(dims)
    mus = [mu] * 12
    x = dev(np.zeros_like(b))
    rc, rep = tm.tm_fgmres_solve(dims, dev(U), dev(b), x, kappa, mus, csw, TOL, storage="f32",
                                 form="defect_correction", restart=12, group=5)
    assert rc == 0 and rep["converged"] == 12, rep
    check_solutions(op, dims, b, host(x), mus, TOL, "8^4 twelve sources groups of 5", "f32")


def test_nonzero_initial_guess_and_antiperiodic():
    dims, kappa, mu, csw = (8, 4, 4, 8), 0.1394, 0.01, 1.5
    U = synth.gauge_field(dims, 0.6, seed=3)
    b = synth.gaussian_spinor(dims, 1, seed=103)
    x0 = synth.gaussian_spinor(dims, 1, seed=203)
    announce("solve nonzero guess, antiperiodic t")
    op = oracle.Operator(dims, U, oracle.kappa_to_m(kappa), mu, csw, antiperiodic_t=True)
    x = dev(x0)
    rc, rep = tm.tm_fgmres_solve(dims, dev(U), dev(b), x, kappa, [mu], csw, TOL, storage="f32",
                                 antiperiodic_t=True, block_dims=(2, 2, 2, 4))
    assert rc == 0
    check_solutions(op, dims, b, host(x), [mu], TOL, "nonzero guess antiperiodic", "f32")


@pytest.mark.parametrize("form", ["flexible", "defect_correction"])
def test_zero_start_without_reading_x(form):
    # x_in=False: x is output only, so NaNs in it change nothing; the result equals the solve
    # from an x of zeros bit for bit (both start from the zero vector)
    dims, kappa, mu, csw = (8, 4, 4, 8), 0.1394, 0.01, 1.5
    U = synth.gauge_field(dims, 0.6, seed=3)
    b = synth.gaussian_spinor(dims, 2, seed=104)
    announce(f"solve from zero without reading x, {form}")
    kw = dict(storage="f32", form=form, restart=8, block_dims=(2, 2, 2, 4))
    x0 = dev(np.zeros_like(b))
    rc0, rep0 = tm.tm_fgmres_solve(dims, dev(U), dev(b), x0, kappa, [mu, -mu], csw, TOL, **kw)
    xn = dev(np.full_like(b, np.nan))
    rc1, rep1 = tm.tm_fgmres_solve(dims, dev(U), dev(b), xn, kappa, [mu, -mu], csw, TOL, x_in=False, **kw)
    assert rc0 == 0 and rc1 == 0
    assert rep0["iters"] == rep1["iters"] and rep0["outer"] == rep1["outer"]
    assert np.array_equal(host(x0), host(xn))
    op = oracle.Operator(dims, U, oracle.kappa_to_m(kappa), mu, csw)
    check_solutions(op, dims, b, host(xn), [mu, -mu], TOL, f"zero start {form}", "f32")


@pytest.mark.parametrize("form", ["flexible", "defect_correction"])
def test_zero_preconditioner_ends_unconverged(cfg_4444, form):
    # no MR steps: SAP returns zero, every Arnoldi column vanishes; the solve must end unconverged
    # with x finite and untouched (no division by the zero pivot), without running to max_iters
    dims, kappa, mu, csw, U, b, op, xs = cfg_4444
    announce(f"solve with a zero preconditioner, {form}")
    x = dev(np.zeros_like(b))
    rc, rep = tm.tm_fgmres_solve(dims, dev(U), dev(b), x, kappa, [mu], csw, TOL, storage="f32", form=form,
                                 restart=8, n_cycles=2, mr_iters=0, block_dims=(2, 2, 2, 2), max_iters=400)
    assert rc == 1 and rep["converged"] == 0, rep
    assert rep["iters"] <= 2, rep
    xg = host(x)
    assert np.isfinite(xg).all() and not xg.any()
    assert abs(rep["true_rel_res"][0] - 1.0) < 1e-12


def test_solver_error_paths(cfg_4444):
    dims, kappa, mu, csw, U, b, op, xs = cfg_4444
    announce("solve error paths")
    x = dev(np.zeros_like(b))
    rc, rep = tm.tm_fgmres_solve(dims, dev(U), dev(b), x, kappa, [mu], csw, TOL, storage="f64", max_iters=2,
                                 block_dims=(2, 2, 2, 2))
    assert rc == 1 and rep["converged"] == 0 and rep["true_rel_res"][0] > TOL
    bad = b.copy()
    bad[0, 5, 1, 1] = np.inf
    with pytest.raises(tm.TMError) as e:
        tm.tm_fgmres_solve(dims, dev(U), dev(bad), x, kappa, [mu], csw, TOL, block_dims=(2, 2, 2, 2))
    assert e.value.code == -7
    with pytest.raises(tm.TMError) as e:
        tm.tm_fgmres_solve(dims, dev(U), dev(b), x, kappa, [mu], csw, TOL, restart=0, block_dims=(2, 2, 2, 2))
    assert e.value.code == -1
    with pytest.raises(tm.TMError) as e:
        tm.tm_fgmres_solve(dims, dev(U), dev(b), x, kappa, [mu], csw, TOL, storage="f64", form="defect_correction",
                           block_dims=(2, 2, 2, 2))
    assert e.value.code == -4
    # zero right-hand side: x = 0 immediately
    x = dev(np.ones_like(b))
    rc, rep = tm.tm_fgmres_solve(dims, dev(U), dev(np.zeros_like(b)), x, kappa, [mu], csw, TOL,
                                 block_dims=(2, 2, 2, 2))
    assert rc == 0


def test_16x16x16x16_twelve_sources_defect_correction():
    # the 48^3x96 workload's parameters and solver form on a lattice with
    # four blocks per axis: 12 point sources, FP32 SAP in defect correction,
    # restart 8
    dims, kappa, mu, csw = (16, 16, 16, 16), 0.1373, 0.0009, 1.5
    U = synth.gauge_field(dims, 0.6, seed=16)
    b = synth.all_point_sources(dims)
    announce("solve 16^4 twelve sources defect correction f32")
    x = dev(np.zeros_like(b))
    rc, rep = tm.tm_fgmres_solve(dims, dev(U), dev(b), x, kappa, [mu] * 12, csw, TOL, storage="f32",
                                 form="defect_correction", restart=8, n_cycles=4, mr_iters=4,
                                 block_dims=(4, 4, 4, 4), max_iters=400)
    assert rc == 0, rep
    assert rep["iters"] < 100, rep
    xg = host(x)
    op = oracle.Operator(dims, U, oracle.kappa_to_m(kappa), mu, csw)
    for k in (0, 4, 11):
        r = b[k].reshape(-1, 4, 3) - op.apply(xg[k])
        assert np.linalg.norm(r) / np.linalg.norm(b[k]) <= TOL * RES_SLACK


def test_defect_correction_tolerance_per_system(cfg_8888):
    # Each system's inner solve runs to its own tolerance: a system started from its converged
    # solution next to one started from zero leaves the first untouched and gives the second the
    # same iterations as a solve of it alone (a group-wide tolerance would let the converged system
    # relax the other's inner solves).
    dims, kappa, mu, csw, U, op = cfg_8888
    announce("defect correction: converged system next to a fresh one")
    b = synth.all_point_sources(dims)[:2]
    mus = [mu, -mu]
    kw = dict(storage="f32", form="defect_correction", restart=8, n_cycles=3, mr_iters=4, block_dims=(4, 4, 4, 4))
    x = dev(np.zeros_like(b))
    rc, rep_pair = tm.tm_fgmres_solve(dims, dev(U), dev(b), x, kappa, mus, csw, TOL, **kw)
    assert rc == 0, rep_pair
    xs = host(x)
    alone = dev(np.zeros_like(b[1:]))
    rc, rep_alone = tm.tm_fgmres_solve(dims, dev(U), dev(b[1:]), alone, kappa, mus[1:], csw, TOL, **kw)
    assert rc == 0, rep_alone
    x = dev(np.stack([xs[0], np.zeros_like(xs[1])]))
    rc, rep = tm.tm_fgmres_solve(dims, dev(U), dev(b), x, kappa, mus, csw, TOL, **kw)
    assert rc == 0, rep
    got = host(x)
    assert np.array_equal(got[0], xs[0])
    assert rep["iters"] == rep_alone["iters"] and rep["outer"] == rep_alone["outer"], (rep, rep_alone)
    assert np.abs(got[1] - host(alone)[0]).max() <= 1e-12 * np.abs(got[1]).max()
    check_solutions(op, dims, b, got, mus, TOL)
