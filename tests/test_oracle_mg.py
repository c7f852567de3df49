"""Pins of the oracle's two-level method (sections 2.3-2.6).

Aggregation (section 2.3, eqs. (aggregate), (prolong)): blocks x spin halves;
the test vectors are orthonormalised on every aggregate, which makes P
Gamma5-compatible (eq. (gamma5_symmetry)).  The coarse operator is the Galerkin
product P^+ D P with the twist i delta mu Gamma5c (eq. (delta)); its
Gamma5c-symmetry and the mu^2 bound of the squared operator carry over from
the fine operator.  The two-level preconditioner is the coarse-grid correction
(eq. (multigrid_preconditioning)) followed by SAP post-smoothing, whose error
propagator is eq. (error_propagation) with no pre-smoothing.  Expected values
come from dense linear algebra (numpy / LAPACK) and closed forms, never from
the oracle's own loops.
"""
import numpy as np
import pytest

import oracle
from paper_1610_02370_amd import synth

DIMS = (4, 4, 4, 4)
ADIMS = (2, 2, 2, 2)
NV = 4


def make_op(mu=0.05, theta=(0.0, 0.0, 0.0, 0.0), shift=(0.0, 0.0), ap=False, dims=DIMS, seed=21):
    U = synth.gauge_field(dims, 0.5, seed=seed)
    return oracle.Operator(dims, U, oracle.kappa_to_m(0.15), mu, csw=1.5, antiperiodic_t=ap, theta=theta,
                           mu_shift=shift)


def random_vectors(dims, nv, seed):
    return synth.gaussian_spinor(dims, nv, seed=seed).reshape(nv, -1)


def aggregate_ids(dims, adims):
    grid = np.indices(dims).reshape(4, -1).T
    return np.ravel_multi_index((grid // np.asarray(adims)).T, np.asarray(dims) // np.asarray(adims))


def dense_P(mg):
    """Columns (j, sg, i) of P as a dense (12 V) x (2 nv nc) matrix, built from the stored test vectors."""
    V = mg.op.V
    agg = aggregate_ids(mg.op.dims, mg.adims)
    P = mg.P.reshape(mg.nv, V, 12)
    D = np.zeros((V * 12, mg.nc * 2 * mg.nv), np.complex128)
    for j in range(mg.nc):
        sites = np.nonzero(agg == j)[0]
        for sg in range(2):
            for i in range(mg.nv):
                col = np.zeros((V, 12), np.complex128)
                col[sites, 6 * sg:6 * sg + 6] = P[i, sites, 6 * sg:6 * sg + 6]
                D[:, j * 2 * mg.nv + sg * mg.nv + i] = col.reshape(-1)
    return D


def dense_coarse(mg, mu_c):
    n = mg.nc * 2 * mg.nv
    M = np.zeros((n, n), np.complex128)
    e = np.zeros(n, np.complex128)
    for k in range(n):
        e[k] = 1.0
        M[:, k] = mg.coarse_apply(e, mu_c).reshape(-1)
        e[k] = 0.0
    return M


def gamma5_coarse(mg):
    return np.tile(np.concatenate([np.ones(mg.nv), -np.ones(mg.nv)]), mg.nc)


@pytest.fixture(scope="module")
def built():
    op = make_op(theta=(0.3, -0.7, 0.0, 1.1), ap=True, shift=(0.02, -0.01))
    mg = oracle.MG(op, ADIMS, NV, delta=1.0)
    v0 = random_vectors(DIMS, NV, seed=5)
    mg.setup(v0)
    return op, mg, v0


def test_aggregate_basis_is_phase_fixed_qr(built):
    # on every aggregate A_{j,sg} the columns are the Q of a QR factorisation of the
    # test vectors there (in order), with the positive real diagonal of Gram-Schmidt
    op, mg, v0 = built
    agg = aggregate_ids(DIMS, ADIMS)
    P = mg.P.reshape(NV, op.V, 12)
    v = v0.reshape(NV, op.V, 12)
    for j in range(mg.nc):
        sites = np.nonzero(agg == j)[0]
        for sg in range(2):
            A = v[:, sites, 6 * sg:6 * sg + 6].reshape(NV, -1).T
            Q, R = np.linalg.qr(A)
            Q = Q * (np.diag(R) / np.abs(np.diag(R))).reshape(1, -1)
            got = P[:, sites, 6 * sg:6 * sg + 6].reshape(NV, -1).T
            assert np.abs(got - Q).max() < 1e-13
    Pd = dense_P(mg)
    assert np.abs(Pd.conj().T @ Pd - np.eye(Pd.shape[1])).max() < 1e-13


def test_restrict_prolong_are_P_dagger_and_P(built):
    op, mg, _ = built
    rng = np.random.default_rng(3)
    Pd = dense_P(mg)
    r = rng.normal(size=op.V * 12) + 1j * rng.normal(size=op.V * 12)
    c = rng.normal(size=Pd.shape[1]) + 1j * rng.normal(size=Pd.shape[1])
    assert np.abs(mg.restrict(r).reshape(-1) - Pd.conj().T @ r).max() < 1e-12
    assert np.abs(mg.prolong(c).reshape(-1) - Pd @ c).max() < 1e-13


def test_prolongation_commutes_with_gamma5(built):
    # eq. (gamma5_symmetry): Gamma5 P = P Gamma5c
    op, mg, _ = built
    rng = np.random.default_rng(4)
    c = rng.normal(size=(mg.nc, 2 * NV)) + 1j * rng.normal(size=(mg.nc, 2 * NV))
    g5 = np.array([1, 1, -1, -1])[None, :, None]
    lhs = g5 * mg.prolong(c)
    rhs = mg.prolong(c * gamma5_coarse(mg).reshape(mg.nc, 2 * NV))
    assert np.abs(lhs - rhs).max() < 1e-13


def test_coarse_operator_is_galerkin_product(built):
    # D_c(mu, delta = 1) = P^+ D(mu) P, dense, with twisted and antiperiodic boundaries and
    # parity-dependent twist shifts in D
    op, mg, _ = built
    Pd = dense_P(mg)
    Dd = op.dense()
    ref = Pd.conj().T @ Dd @ Pd
    got = dense_coarse(mg, op.mu)
    assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()


def test_coarse_operator_galerkin_on_uneven_coarse_grid():
    # coarse extents 4, 2, 3, 2: forward and backward neighbours differ along t and y, and every axis
    # has its own extent; matrix-free check D_c x = P^+ D P x for random coarse x
    dims = (8, 4, 6, 4)
    op = make_op(dims=dims, theta=(0.5, 0.0, -0.3, 0.2), shift=(0.03, 0.0), seed=7)
    mg = oracle.MG(op, ADIMS, 3, delta=1.0)
    mg.setup(random_vectors(dims, 3, seed=17))
    assert mg.cdims == (4, 2, 3, 2)
    rng = np.random.default_rng(18)
    for _ in range(3):
        x = rng.normal(size=(mg.nc, 6)) + 1j * rng.normal(size=(mg.nc, 6))
        ref = mg.restrict(op.apply(mg.prolong(x)))
        assert np.abs(mg.coarse_apply(x, op.mu) - ref).max() < 1e-12 * np.abs(ref).max()


def test_coarse_couples_only_neighbouring_aggregates(built):
    op, mg, _ = built
    M = dense_coarse(mg, op.mu)
    cd = np.asarray(mg.cdims)
    coords = np.array(np.unravel_index(np.arange(mg.nc), cd)).T
    n2 = 2 * NV
    for j in range(mg.nc):
        for k in range(mg.nc):
            d = np.abs(coords[j] - coords[k])
            d = np.minimum(d, cd - d)
            blk = M[j * n2:(j + 1) * n2, k * n2:(k + 1) * n2]
            if d.sum() > 1:
                assert np.abs(blk).max() == 0.0
            elif d.sum() == 1:
                assert np.abs(blk).max() > 1e-3


def test_coarse_twist_symmetries():
    # no shifts: D_c(mu)^+ = Gamma5c D_c(-mu) Gamma5c and D_c(mu)^+ D_c(mu) = D_c(0)^+ D_c(0) + (delta mu)^2
    op = make_op(mu=0.07, theta=(0.0, 0.4, 0.0, 0.0))
    mg = oracle.MG(op, ADIMS, NV, delta=3.0)
    mg.setup(random_vectors(DIMS, NV, seed=6))
    mu_c = mg.delta * op.mu
    g5 = np.diag(gamma5_coarse(mg))
    Dp, Dm, D0 = dense_coarse(mg, mu_c), dense_coarse(mg, -mu_c), dense_coarse(mg, 0.0)
    assert np.abs(Dp.conj().T - g5 @ Dm @ g5).max() < 1e-13
    lhs = Dp.conj().T @ Dp
    rhs = D0.conj().T @ D0 + mu_c ** 2 * np.eye(len(D0))
    assert np.abs(lhs - rhs).max() < 1e-12 * np.abs(lhs).max()
    # every singular value of the coarse operator is at least delta |mu|
    assert np.linalg.svd(Dp, compute_uv=False).min() >= mu_c * (1 - 1e-12)


def test_coarse_gmres_matches_dense_solve(built):
    op, mg, _ = built
    mu_c = 2.0 * op.mu
    M = dense_coarse(mg, mu_c)
    rng = np.random.default_rng(8)
    b = rng.normal(size=len(M)) + 1j * rng.normal(size=len(M))
    # restart length = dimension: GMRES terminates with the exact solution
    x, rep = mg.coarse_gmres(b, mu_c, tol=1e-13, restart=len(M), max_restarts=2)
    assert np.abs(x.reshape(-1) - np.linalg.solve(M, b)).max() < 1e-10 * np.abs(np.linalg.solve(M, b)).max()
    # low accuracy (the paper's coarse setting): the estimate is the true residual norm
    x, rep = mg.coarse_gmres(b, mu_c, tol=0.1, restart=20, max_restarts=5)
    true = np.linalg.norm(b - M @ x.reshape(-1)) / np.linalg.norm(b)
    assert rep["met"] and true <= 0.1 * (1 + 1e-10)
    assert abs(true - rep["rel_estimate"]) < 1e-10
    # tol 0: exactly restart * max_restarts steps; the residual norm never grows between restarts
    x3, rep3 = mg.coarse_gmres(b, mu_c, tol=0.0, restart=3, max_restarts=4)
    assert rep3["iters"] == 12 and rep3["restarts"] == 4
    x2, _ = mg.coarse_gmres(b, mu_c, tol=0.0, restart=3, max_restarts=3)
    assert np.linalg.norm(b - M @ x3.reshape(-1)) <= np.linalg.norm(b - M @ x2.reshape(-1)) * (1 + 1e-12)


def test_unitary_prolongation_with_exact_coarse_solve_inverts_D():
    # one-site aggregates and nv = 6: P is unitary, so P D_c^-1 P^+ = D^-1 (no smoothing, delta = 1)
    dims = (2, 2, 2, 2)
    op = make_op(dims=dims, seed=3)
    n = op.V * 12
    mg = oracle.MG(op, (1, 1, 1, 1), 6, delta=1.0, coarse_tol=1e-14, coarse_restart=n, coarse_max_restarts=2,
                   post_cycles=0)
    mg.setup(random_vectors(dims, 6, seed=9))
    rng = np.random.default_rng(10)
    r = rng.normal(size=n) + 1j * rng.normal(size=n)
    ref = np.linalg.solve(op.dense(), r)
    assert np.abs(mg.precond(r).reshape(-1) - ref).max() < 1e-10 * np.abs(ref).max()
    # a shifted coarse twist changes the correction
    mg2 = oracle.MG(op, (1, 1, 1, 1), 6, delta=4.0, coarse_tol=1e-14, coarse_restart=n, coarse_max_restarts=2,
                    post_cycles=0)
    mg2.setup(random_vectors(dims, 6, seed=9))
    assert np.abs(mg2.precond(r).reshape(-1) - ref).max() > 1e-3 * np.abs(ref).max()


def test_two_level_error_propagation():
    # eq. (error_propagation), no pre-smoothing, exact block solves and an exact coarse solve:
    # x* - z = E^k (I - P D_c^-1 P^+ D) x*, with E^k x0 = SAP(b = 0, x0) after k cycles
    op = make_op(theta=(0.2, 0.0, -0.5, 0.0), shift=(0.01, 0.03))
    n = op.V * 12
    k = 2
    mg = oracle.MG(op, ADIMS, NV, delta=1.0, coarse_tol=1e-14, coarse_restart=16 * 2 * NV, coarse_max_restarts=2,
                   post_cycles=k, mr_iters=-1)
    mg.setup(random_vectors(DIMS, NV, seed=12))
    D = op.dense()
    Pd = dense_P(mg)
    rng = np.random.default_rng(13)
    r = rng.normal(size=n) + 1j * rng.normal(size=n)
    xs = np.linalg.solve(D, r)
    cgc = xs - Pd @ np.linalg.solve(Pd.conj().T @ D @ Pd, Pd.conj().T @ r)
    rhs = op.sap(np.zeros(n, complex), ADIMS, k, -1, x0=cgc).reshape(-1)
    lhs = xs - mg.precond(r).reshape(-1)
    assert np.abs(lhs - rhs).max() < 1e-10 * np.abs(xs).max()


def test_two_level_fgmres_solves(built):
    op, mg0, v0 = built
    mg = oracle.MG(op, ADIMS, NV, delta=2.0, coarse_tol=0.1, coarse_restart=20, coarse_max_restarts=5,
                   post_cycles=2, mr_iters=4)
    mg.setup(v0)
    b = synth.point_sources(DIMS, [(0, 0)]).reshape(-1)
    x, rep = mg.fgmres(b, 1e-10, restart=20)
    assert rep["converged"] and rep["true_rel_res"] <= 1e-10
    ref = np.linalg.solve(op.dense(), b)
    assert np.abs(x.reshape(-1) - ref).max() < 1e-7 * np.abs(ref).max()


def test_setup_iterations_follow_the_paper():
    # iteration 1: v_i <- SAP(v_i) then global orthonormalisation (phase-fixed QR);
    # iteration 2: v_i <- two-level method built from iteration 1, applied to v_i, then again QR
    op = make_op(mu=0.02)
    n = op.V * 12
    v0 = random_vectors(DIMS, NV, seed=14)

    def qr(vs):
        Q, R = np.linalg.qr(np.array(vs).T)
        return (Q * (np.diag(R) / np.abs(np.diag(R))).reshape(1, -1)).T

    kw = dict(delta=2.0, coarse_tol=0.1, coarse_restart=10, coarse_max_restarts=2, post_cycles=2, mr_iters=3,
              setup_cycles=3)
    mg1 = oracle.MG(op, ADIMS, NV, setup_iters=1, **kw)
    v1 = mg1.setup(v0).reshape(NV, n)
    ref1 = qr([op.sap(v0[i], ADIMS, 3, 3).reshape(-1) for i in range(NV)])
    assert np.abs(v1 - ref1).max() < 1e-12
    mg2 = oracle.MG(op, ADIMS, NV, setup_iters=2, **kw)
    v2 = mg2.setup(v0).reshape(NV, n)
    ref2 = qr([mg1.precond(v1[i]).reshape(-1) for i in range(NV)])
    assert np.abs(v2 - ref2).max() < 1e-11
    # P and the coarse stencil are those of the final vectors
    mg3 = oracle.MG(op, ADIMS, NV, setup_iters=0, **kw)
    mg3.setup(v2)
    assert np.abs(mg3.P - mg2.P).max() < 1e-14 and np.abs(mg3.Dc - mg2.Dc).max() < 1e-14


def test_setup_exposes_low_modes():
    # inverse iteration: after setup the aggregates capture the smallest singular vectors of D(mu)
    # far better than the random starting vectors do
    op = make_op(mu=0.01)
    D = op.dense()
    _, s, Vh = np.linalg.svd(D)
    low = Vh[-6:].conj().T  # right singular vectors of the 6 smallest singular values
    v0 = random_vectors(DIMS, NV, seed=15)
    kw = dict(delta=2.0, coarse_tol=0.1, coarse_restart=10, coarse_max_restarts=2, post_cycles=2, mr_iters=3,
              setup_cycles=4)
    fracs = []
    for it in (0, 3):
        mg = oracle.MG(op, ADIMS, NV, setup_iters=it, **kw)
        mg.setup(v0)
        Pd = dense_P(mg)
        fracs.append(np.linalg.norm(Pd.conj().T @ low) ** 2 / 6)
    assert fracs[1] > 0.3 and fracs[1] > 5 * fracs[0], fracs


def even_coarse_mg():
    # coarse extents 4, 2, 2, 2 (all even: every coarse neighbour has the other parity)
    dims = (8, 4, 4, 4)
    op = make_op(dims=dims, theta=(0.4, 0.0, 0.0, -0.6), shift=(0.02, -0.01), seed=9)
    mg = oracle.MG(op, ADIMS, 3, delta=1.0)
    mg.setup(random_vectors(dims, 3, seed=19))
    cd = np.asarray(mg.cdims)
    par = np.repeat(np.indices(mg.cdims).reshape(4, -1).sum(axis=0) % 2, 2 * mg.nv)
    return op, mg, par


def test_coarse_dhat_is_the_dense_schur_complement():
    # section 2.5's reduction on the coarse grid: odd sites kept, D_oo - D_oe D_ee^-1 D_eo
    op, mg, par = even_coarse_mg()
    mu_c = 0.07
    M = dense_coarse(mg, mu_c)
    e, o = np.nonzero(par == 0)[0], np.nonzero(par == 1)[0]
    S = M[np.ix_(o, o)] - M[np.ix_(o, e)] @ np.linalg.solve(M[np.ix_(e, e)], M[np.ix_(e, o)])
    n = len(par)
    got = np.zeros((len(o), len(o)), complex)
    for k, col in enumerate(o):
        x = np.zeros(n, complex)
        x[col] = 1.0
        y = mg.coarse_dhat(x, mu_c).reshape(-1)
        assert np.abs(y[e]).max() == 0.0
        got[:, k] = y[o]
    assert np.abs(got - S).max() < 1e-12 * np.abs(S).max()


def test_coarse_gmres_eo_matches_dense_solve():
    op, mg, par = even_coarse_mg()
    mu_c = 0.05
    M = dense_coarse(mg, mu_c)
    rng = np.random.default_rng(20)
    b = rng.normal(size=len(M)) + 1j * rng.normal(size=len(M))
    ref = np.linalg.solve(M, b)
    x, rep = mg.coarse_gmres_eo(b, mu_c, 1e-13, int((par == 1).sum()), 2)
    assert np.abs(x.reshape(-1) - ref).max() < 1e-10 * np.abs(ref).max()
    # low accuracy: the estimate is the full system's true residual (its even part vanishes)
    x, rep = mg.coarse_gmres_eo(b, mu_c, 0.1, 10, 5)
    r = b - M @ x.reshape(-1)
    assert np.abs(r[par == 0]).max() < 1e-12 * np.linalg.norm(b)
    true = np.linalg.norm(r) / np.linalg.norm(b)
    assert rep["met"] and true <= 0.1 * (1 + 1e-10) and abs(true - rep["rel_estimate"]) < 1e-10


def test_two_level_with_even_odd_coarse_solve():
    # with exact coarse solves the preconditioner does not depend on how the coarse system is solved
    op, _, _ = even_coarse_mg()
    v0 = random_vectors(op.dims, 3, seed=19)
    out = []
    for eo in (False, True):
        mg = oracle.MG(op, ADIMS, 3, delta=3.0, coarse_tol=1e-14, coarse_restart=200, coarse_max_restarts=3,
                       post_cycles=1, mr_iters=3, coarse_eo=eo)
        mg.setup(v0)
        r = random_vectors(op.dims, 1, seed=21)[0]
        out.append(mg.precond(r).reshape(-1))
    assert np.abs(out[0] - out[1]).max() < 1e-10 * np.abs(out[0]).max()
