"""GPU parity of the two-level method (sections 2.3 - 2.6) against the FP64 oracle.

Both sides build the method from the same seeded starting vectors; nothing the
GPU computes is fed to the oracle.  FP32 on the GPU against FP64:
  aggregate basis P, coarse stencil, restriction, coarse operator  1e-5
  prolongation                                                      1e-6
  coarse GMRES, a fixed number of steps (full or even-odd reduced)  1e-4
  two-level preconditioner (coarse solve + FP32 SAP post-smoothing) 5e-4
  setup with one two-level iteration                                2e-3
The even-odd coarse solver's block inverses are FP64 eliminations rounded to FP32.
The solve with the two-level preconditioner is checked on its FP64 true
residual (oracle operator) and against the oracle's solution.
"""
import numpy as np
import pytest

import oracle
import paper_1610_02370_amd as tm
from paper_1610_02370_amd import synth

from gpu_util import announce, dev, host, rel_err

pytestmark = pytest.mark.gpu

KAPPA, CSW = 0.1373, 1.5
THETA = (0.0, 0.6, -0.4, 1.1)
SHIFT = (0.003, -0.002)

CASES = {
    # dims, aggregate, n_vec, antiperiodic, theta, shift
    "4^4 aggregates": ((8, 8, 8, 8), (4, 4, 4, 4), 6, True, THETA, SHIFT),
    "2^4 aggregates, uneven coarse grid": ((16, 8, 8, 8), (2, 2, 2, 2), 5, False, (0.3, 0.0, 0.0, -0.9), (0.0, 0.0)),
    # 512-site aggregates: the kernels' large-aggregate variants and the generic smoother
    "8x4^3 aggregates": ((16, 8, 8, 8), (8, 4, 4, 4), 4, True, (0.0, 0.0, 0.5, 0.0), (0.001, 0.0)),
    # the largest number of test vectors (64 coarse components, every lane of a coarse row)
    "32 test vectors": ((8, 8, 8, 8), (4, 4, 4, 4), 32, False, (0.0, 0.0, 0.0, 0.0), (0.0, 0.0)),
    # one test vector (two coarse components per aggregate)
    "1 test vector": ((8, 8, 8, 8), (4, 4, 2, 2), 1, False, (0.2, 0.0, 0.0, 0.0), (0.0, 0.0)),
}


def build(case, mu, seed=3, **kw):
    dims, adims, nv, ap, theta, shift = CASES[case]
    U = synth.gauge_field(dims, 0.6, seed=seed)
    v0 = synth.gaussian_spinor(dims, nv, seed=100 + seed)
    params = dict(block_dims=adims, n_vec=nv, setup_iters=0, setup_cycles=2, delta=2.0, coarse_tol=0.0,
                  coarse_restart=8, coarse_max_restarts=2, post_cycles=2, mr_iters=3, coarse_eo=0)
    params.update(kw)
    announce(f"two-level setup case={case} params={params}")
    g = tm.MG(dims, dev(U), KAPPA, mu, CSW, dev(v0), antiperiodic_t=ap, theta=theta, mu_shift=shift, **params)
    op = oracle.Operator(dims, U, oracle.kappa_to_m(KAPPA), mu, CSW, antiperiodic_t=ap, theta=theta, mu_shift=shift)
    o = oracle.MG(op, adims, nv, delta=params["delta"], coarse_tol=params["coarse_tol"],
                  coarse_restart=params["coarse_restart"], coarse_max_restarts=params["coarse_max_restarts"],
                  post_cycles=params["post_cycles"], mr_iters=params["mr_iters"], setup_iters=params["setup_iters"],
                  setup_cycles=params["setup_cycles"], coarse_eo=bool(params["coarse_eo"]))
    o.setup(v0)
    return dims, U, g, o, op


@pytest.fixture(scope="module", params=sorted(CASES))
def built(request):
    return build(request.param, mu=0.01)


# the even-odd coarse solver: the smallest and largest coarse rows (block inverses of 2x2 and of
# 64x64, the latter with 128 KiB of LDS), the largest coarse grid, and 512-site aggregates
EO_CASES = ["4^4 aggregates", "2^4 aggregates, uneven coarse grid", "32 test vectors", "1 test vector",
            "8x4^3 aggregates"]


@pytest.fixture(scope="module", params=EO_CASES)
def built_eo(request):
    return build(request.param, mu=0.01, coarse_eo=1)


def test_basis_and_stencil(built):
    dims, U, g, o, op = built
    P, Dc = g.export()
    P, Dc = host(P), host(Dc)
    assert np.abs(P - o.P).max() < 1e-5 * np.abs(o.P).max()
    assert np.abs(Dc - o.Dc).max() < 1e-5 * np.abs(o.Dc).max()


def test_restrict_prolong(built):
    dims, U, g, o, op = built
    r = synth.gaussian_spinor(dims, 3, seed=41)
    c = host(g.restrict(dev(r)))
    for k in range(3):
        assert rel_err(c[k], o.restrict(r[k])) < 1e-5
    rng = np.random.default_rng(42)
    cc = rng.normal(size=(2, o.nc, 2 * o.nv)) + 1j * rng.normal(size=(2, o.nc, 2 * o.nv))
    e = host(g.prolong(dev(cc)))
    for k in range(2):
        assert rel_err(e[k], o.prolong(cc[k])) < 1e-6


def test_coarse_operator(built):
    dims, U, g, o, op = built
    rng = np.random.default_rng(43)
    mus = [0.02, -0.02, 0.0]
    x = rng.normal(size=(3, o.nc, 2 * o.nv)) + 1j * rng.normal(size=(3, o.nc, 2 * o.nv))
    y = host(g.coarse_apply(dev(x), mus))
    for k, m in enumerate(mus):
        assert rel_err(y[k], o.coarse_apply(x[k], m)) < 1e-5


def test_coarse_gmres_fixed_steps(built):
    dims, U, g, o, op = built
    rng = np.random.default_rng(44)
    mus = [0.05, -0.05]
    b = rng.normal(size=(2, o.nc, 2 * o.nv)) + 1j * rng.normal(size=(2, o.nc, 2 * o.nv))
    x, it = g.coarse_solve(dev(b), mus, 0.0, 6, 3)
    assert it == 18
    x = host(x)
    for k, m in enumerate(mus):
        ref, rep = o.coarse_gmres(b[k], m, 0.0, 6, 3)
        assert rep["iters"] == 18
        assert rel_err(x[k], ref) < 1e-4


def test_coarse_gmres_to_tolerance(built):
    dims, U, g, o, op = built
    rng = np.random.default_rng(45)
    b = rng.normal(size=(1, o.nc, 2 * o.nv)) + 1j * rng.normal(size=(1, o.nc, 2 * o.nv))
    x, it = g.coarse_solve(dev(b), [0.05], 1e-5, 64, 20)
    x = host(x)[0]
    res = np.linalg.norm(b[0] - o.coarse_apply(x, 0.05)) / np.linalg.norm(b[0])
    assert res < 2e-5
    ref, _ = o.coarse_gmres(b[0], 0.05, 1e-12, 64, 40)
    assert rel_err(x, ref) < 1e-3


def test_two_level_preconditioner(built):
    dims, U, g, o, op = built
    r = synth.gaussian_spinor(dims, 2, seed=46)
    mus = [0.01, -0.01]
    z = host(g.precond(dev(r), mus))
    for k, m in enumerate(mus):
        ref = o.precond(r[k], op.with_mu(m))
        assert rel_err(z[k], ref) < 5e-4


def test_coarse_eo_gmres_fixed_steps(built_eo):
    # three systems, two twists: the second system with the first one's twist reuses its inverses
    dims, U, g, o, op = built_eo
    rng = np.random.default_rng(54)
    mus = [0.05, -0.05, 0.05]
    b = rng.normal(size=(3, o.nc, 2 * o.nv)) + 1j * rng.normal(size=(3, o.nc, 2 * o.nv))
    x, it = g.coarse_solve(dev(b), mus, 0.0, 6, 3)
    assert it == 18
    x = host(x)
    for k, m in enumerate(mus):
        ref, rep = o.coarse_gmres_eo(b[k], m, 0.0, 6, 3)
        assert rep["iters"] == 18
        assert rel_err(x[k], ref) < 1e-4


def test_coarse_eo_gmres_more_twists_than_inverse_sets(built_eo):
    # five distinct twists: solved in runs of at most four, the cached inverse sets evicted in turn
    dims, U, g, o, op = built_eo
    rng = np.random.default_rng(55)
    mus = [0.05, -0.05, 0.02, 0.0, 0.05, -0.03]
    b = rng.normal(size=(6, o.nc, 2 * o.nv)) + 1j * rng.normal(size=(6, o.nc, 2 * o.nv))
    x, it = g.coarse_solve(dev(b), mus, 0.0, 4, 2)
    assert it == 8
    x = host(x)
    for k, m in enumerate(mus):
        ref, _ = o.coarse_gmres_eo(b[k], m, 0.0, 4, 2)
        assert rel_err(x[k], ref) < 1e-4


def test_coarse_eo_gmres_to_tolerance(built_eo):
    dims, U, g, o, op = built_eo
    rng = np.random.default_rng(56)
    b = rng.normal(size=(1, o.nc, 2 * o.nv)) + 1j * rng.normal(size=(1, o.nc, 2 * o.nv))
    x, it = g.coarse_solve(dev(b), [-0.05], 1e-5, 64, 20)
    x = host(x)[0]
    # the full coarse system's residual (even sites from the recovery)
    res = np.linalg.norm(b[0] - o.coarse_apply(x, -0.05)) / np.linalg.norm(b[0])
    assert res < 5e-5
    ref, _ = o.coarse_gmres(b[0], -0.05, 1e-12, 64, 40)
    assert rel_err(x, ref) < 1e-3


def test_two_level_preconditioner_eo(built_eo):
    dims, U, g, o, op = built_eo
    r = synth.gaussian_spinor(dims, 2, seed=57)
    mus = [0.01, -0.01]
    z = host(g.precond(dev(r), mus))
    for k, m in enumerate(mus):
        ref = o.precond(r[k], op.with_mu(m))
        assert rel_err(z[k], ref) < 5e-4


@pytest.mark.parametrize("case", ["4^4 aggregates", "32 test vectors"])
def test_setup_with_a_two_level_iteration_eo(case):
    # 6 and 32 test vectors: the global orthonormalisation runs in panels of 4 (a partial last
    # panel for 6, eight full ones for 32)
    dims, U, g, o, op = build(case, mu=0.01, seed=6, setup_iters=2, coarse_eo=1)
    P, Dc = g.export()
    P, Dc = host(P), host(Dc)
    assert np.abs(P - o.P).max() < 2e-3 * np.abs(o.P).max()
    assert np.abs(Dc - o.Dc).max() < 2e-3 * np.abs(o.Dc).max()


def test_setup_with_a_two_level_iteration():
    # iteration 1 (SAP on the starting vectors) and iteration 2 (the two-level method of iteration 1)
    dims, U, g, o, op = build("4^4 aggregates", mu=0.01, seed=5, setup_iters=2)
    P, Dc = g.export()
    P, Dc = host(P), host(Dc)
    assert np.abs(P - o.P).max() < 2e-3 * np.abs(o.P).max()
    assert np.abs(Dc - o.Dc).max() < 2e-3 * np.abs(o.Dc).max()
    # the aggregate basis is orthonormal to FP32 accuracy
    agg = (np.indices(dims).reshape(4, -1).T // 4)
    aid = np.ravel_multi_index(agg.T, (2, 2, 2, 2))
    Pm = P.reshape(o.nv, -1, 12)
    for j in (0, 7, 15):
        for sg in range(2):
            Q = Pm[:, aid == j, 6 * sg:6 * sg + 6].reshape(o.nv, -1)
            assert np.abs(Q.conj() @ Q.T - np.eye(o.nv)).max() < 1e-5


@pytest.mark.parametrize("form,eo", [("flexible", 0), ("defect_correction", 0), ("defect_correction", 1)])
def test_solve_with_two_level_preconditioner(form, eo):
    dims, U, g, o, op = build("4^4 aggregates", mu=0.01, seed=7, setup_iters=2, coarse_tol=0.1, coarse_restart=16,
                              coarse_max_restarts=2, coarse_eo=eo)
    mus = [0.01, -0.01]
    b = synth.point_sources(dims, [(0, 0), (2, 1)])
    x = dev(np.zeros_like(b))
    announce(f"two-level solve form={form} coarse_eo={eo}")
    rc, rep = tm.tm_fgmres_solve(dims, dev(U), dev(b), x, KAPPA, mus, CSW, 1e-10, storage="f32", antiperiodic_t=True,
                                 theta=THETA, mu_shift=SHIFT, mg=g, form=form, restart=16)
    assert rc == 0 and rep["converged"] == 2
    x = host(x)
    for k, m in enumerate(mus):
        opk = op.with_mu(m)
        res = np.linalg.norm(b[k].reshape(-1) - opk.apply(x[k]).reshape(-1)) / np.linalg.norm(b[k])
        assert res < 1.5e-10
        ref, rr = opk.fgmres(b[k], 1e-12, restart=20, bdims=(4, 4, 4, 4), n_cycles=3, mr_iters=4)
        assert rr["converged"]
        assert rel_err(x[k], ref) < 1e-7
    info = g.info()
    assert info["applications"] >= rep["iters"]


def test_solve_rejects_a_mismatched_handle():
    dims, U, g, o, op = build("4^4 aggregates", mu=0.01, seed=8)
    b = synth.point_sources(dims, [(0, 0)])
    x = dev(np.zeros_like(b))
    with pytest.raises(tm.TMError) as e:
        tm.tm_fgmres_solve(dims, dev(U), dev(b), x, KAPPA, [0.01], CSW, 1e-10, storage="f32", antiperiodic_t=False,
                           theta=THETA, mu_shift=SHIFT, mg=g)
    assert e.value.code == -1
    with pytest.raises(tm.TMError) as e:
        tm.tm_fgmres_solve(dims, dev(U), dev(b), x, KAPPA, [0.01], CSW, 1e-10, storage="f64", antiperiodic_t=True,
                           theta=THETA, mu_shift=SHIFT, mg=g)
    assert e.value.code == -4
