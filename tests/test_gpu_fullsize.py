"""GPU parity at the benchmark lattice sizes, on sampled outputs.

The oracle cannot run SAP on 10^7 sites in seconds, but SAP is local: after
one cycle from a given x0, the result on a block depends only on b, x0, the
links and the clover within one block (plus one site for the clover) of it.
So the oracle runs the same cycle on a 24^4 window cut out of the full
lattice (block grid aligned, colours preserved) and its central 2^4 blocks
are exact; the GPU result on those blocks must match it.  For point sources
the result vanishes beyond one block of the source, which the whole-lattice
norm checks.  Operator parity at full size uses 4^4 windows around sampled
sites; the solves are checked through the true residual recomputed by the
oracle (at every site on 32^3x64, at sampled sites on 48^3x96).

Launch configurations are the benchmark's: 4^4 blocks, FP32 storage with 6
systems per SAP launch (the solve's group size) at 48^3x96; 24 systems in
FP16 / BF16 at 64^3x128 through internal buffers, and the +-mu pair solved to
1e-10 by defect correction with FP16 / BF16 smoothing at that size; 2 systems
(+-mu) at 32^3x64.  Each result is checked norm-wise and per site against the
error model of gpu_util, as in the small-lattice parity tests.
"""
import numpy as np
import pytest

import oracle
import paper_1610_02370_amd as tm
from paper_1610_02370_amd import synth

from gpu_util import TOL as ERR_TOL
from gpu_util import announce, check_close, host, log_solve, rel_err

pytestmark = pytest.mark.gpu

BLOCK = (4, 4, 4, 4)
TOL = ERR_TOL["sap"]


def lex(dims, c):
    """Lexicographic site index (t slowest) of coordinate arrays c[..., 4]."""
    c = np.asarray(c)
    return ((c[..., 0] * dims[1] + c[..., 1]) * dims[2] + c[..., 2]) * dims[3] + c[..., 3]


def window_sites(dims, origin, size):
    """Full-lattice site indices of the periodic window [origin, origin + size), window-lexicographic."""
    axes = [(origin[a] + np.arange(size[a])) % dims[a] for a in range(4)]
    grid = np.stack(np.meshgrid(*axes, indexing="ij"), axis=-1)
    return lex(dims, grid).ravel()


def window_op(U, dims, origin, size, kappa, csw):
    Uw = U[window_sites(dims, origin, size)]
    return oracle.Operator(size, Uw, oracle.kappa_to_m(kappa), 0.0, csw)


def sap_windows(dims):
    """Two 24^4 windows (6 blocks per axis) with an even block-coordinate sum: one across the
    periodic boundary, one in the middle of the lattice."""
    nb = [d // 4 for d in dims]
    wa = [(n - 2) % n for n in nb]
    wb = [n // 2 - 3 for n in nb]
    if sum(wb) % 2:
        wb[3] += 1
    return [tuple(4 * o for o in w) for w in (wa, wb)]


def central_mask(size=(24, 24, 24, 24), lo=8, hi=16):
    axes = [(np.arange(n) >= lo) & (np.arange(n) < hi) for n in size]
    return np.logical_and.reduce(np.meshgrid(*axes, indexing="ij")).ravel()


@pytest.fixture(scope="module")
def lattice_48x96():
    import torch

    dims = (96, 48, 48, 48)
    announce("generating the 48^3x96 gauge field")
    U = synth.gauge_field(dims, 0.6, seed=4)
    yield dims, U
    tm.tm_finalize()
    torch.cuda.empty_cache()


def test_sap_48x96_f32_six_systems_sampled_blocks(lattice_48x96):
    import torch

    dims, U = lattice_48x96
    kappa, csw = 0.1373, 1.5
    mus = [0.0009 * (1 if k % 2 == 0 else -1) for k in range(6)]
    V = U.shape[0]
    announce("full-size SAP 48^3x96 f32, 6 systems, 4^4 blocks, 1 cycle")
    Ud = torch.from_numpy(U).cuda()
    b = torch.empty((6, V, 4, 3), dtype=torch.complex128, device="cuda")
    keep = {}
    for k in range(6):
        bk = synth.gaussian_spinor(dims, 1, seed=300 + k)[0]
        b[k].copy_(torch.from_numpy(bk))
        if k < 2:
            keep[k] = bk
        del bk
    x = 0.1 * b
    tm.tm_sap_smooth(dims, Ud, b, x, kappa, mus, csw, BLOCK, 1, 4, storage="f32")
    torch.cuda.synchronize()
    assert bool(torch.isfinite(torch.view_as_real(x)).all())
    mask = central_mask()
    for origin in sap_windows(dims):
        idx = window_sites(dims, origin, (24,) * 4)
        op = window_op(U, dims, origin, (24,) * 4, kappa, csw)
        got = host(x[:, torch.from_numpy(idx).cuda()])
        for k in (0, 1):
            bw = keep[k][idx]
            ref = op.with_mu(mus[k]).sap(bw, BLOCK, 1, 4, x0=0.1 * bw).reshape(-1, 4, 3)
            check_close(got[k][mask], ref[mask], "sap", "f32", f"48^3x96 window {origin} system {k}")
    del Ud, b, x
    tm.tm_finalize()
    torch.cuda.empty_cache()


def test_dirac_48x96_sampled_sites(lattice_48x96):
    import torch

    dims, U = lattice_48x96
    kappa, csw, mu = 0.1373, 1.5, 0.0009
    V = U.shape[0]
    rng = np.random.default_rng(48)
    sites = np.concatenate([[0, V - 1], rng.integers(0, V, 30)])
    psi = synth.gaussian_spinor(dims, 1, seed=348)
    announce("full-size operator 48^3x96 f64 / f32 at sampled sites")
    Ud = torch.from_numpy(U).cuda()
    pd = torch.from_numpy(psi).cuda()
    outs = {}
    for prec in ("f64", "f32"):
        out = torch.empty_like(pd)
        tm.tm_dirac_apply(dims, Ud, pd, kappa, [mu], csw, out=out, storage=prec)
        outs[prec] = host(out[0, torch.from_numpy(sites).cuda()])
        del out
    ref = np.empty((len(sites), 4, 3), np.complex128)
    for i, s in enumerate(sites):
        c = np.array(np.unravel_index(s, dims))
        origin = c - 2
        op = window_op(U, dims, origin, (4, 4, 4, 4), kappa, csw).with_mu(mu)
        w = window_sites(dims, origin, (4, 4, 4, 4))
        ref[i] = op.apply(psi[0][w]).reshape(-1, 4, 3)[lex((4, 4, 4, 4), [2, 2, 2, 2])]
    check_close(outs["f64"], ref, "dirac", "f64", "48^3x96 sampled sites")
    check_close(outs["f32"], ref, "dirac", "f32", "48^3x96 sampled sites")
    del Ud, pd
    tm.tm_finalize()
    torch.cuda.empty_cache()


def test_solve_48x96_twelve_sources_sampled_residual(lattice_48x96):
    import torch

    dims, U = lattice_48x96
    kappa, csw, mu = 0.1373, 1.5, 0.0009
    V = U.shape[0]
    announce("full-size solve 48^3x96: 12 point sources, defect correction, f32 SAP")
    Ud = torch.from_numpy(U).cuda()
    b = torch.zeros((12, V, 4, 3), dtype=torch.complex128, device="cuda")
    for k in range(12):
        b[k, 0, k // 3, k % 3] = 1.0
    x = torch.zeros_like(b)
    rc, rep = tm.tm_fgmres_solve(dims, Ud, b, x, kappa, [mu] * 12, csw, 1e-10, storage="f32",
                                 form="defect_correction", restart=8, n_cycles=4, mr_iters=4, block_dims=BLOCK)
    assert rc == 0, rep
    assert max(rep["true_rel_res"][:12]) <= 1e-10
    # oracle residual at sampled sites: |r(s)| <= ||r|| <= 1e-10 ||b|| (||b|| = 1)
    rng = np.random.default_rng(96)
    c0 = np.zeros(4, int)
    near = [c0] + [np.eye(4, dtype=int)[a] * sg for a in range(4) for sg in (1, -1)]
    sites = [lex(dims, np.mod(c, dims)) for c in near] + list(rng.integers(0, V, 15))
    for s in sites:
        c = np.array(np.unravel_index(s, dims))
        origin = c - 2
        w = window_sites(dims, origin, (4, 4, 4, 4))
        xw = host(x[:, torch.from_numpy(w).cuda()])
        op = window_op(U, dims, origin, (4, 4, 4, 4), kappa, csw).with_mu(mu)
        centre = lex((4, 4, 4, 4), [2, 2, 2, 2])
        for k in range(12):
            dx = op.apply(xw[k]).reshape(-1, 4, 3)[centre]
            bs = np.zeros((4, 3), complex)
            if s == 0:
                bs[k // 3, k % 3] = 1.0
            assert np.linalg.norm(bs - dx) <= 1.05e-10, (s, k)
    del Ud, b, x
    tm.tm_finalize()
    torch.cuda.empty_cache()


@pytest.fixture(scope="module")
def lattice_32x64():
    dims = (64, 32, 32, 32)
    announce("generating the 32^3x64 gauge field")
    return dims, synth.gauge_field(dims, 0.6, seed=3)


def test_sap_32x64_pm_mu_whole_lattice(lattice_32x64):
    import torch

    dims, U = lattice_32x64
    kappa, csw, mus = 0.1394, 1.5, [0.001, -0.001]
    announce("full-size SAP 32^3x64 f32, +-mu, 2 cycles, every site against the oracle")
    b = synth.gaussian_spinor(dims, 2, seed=303)
    x = torch.zeros((2,) + b.shape[1:], dtype=torch.complex128, device="cuda")
    tm.tm_sap_smooth(dims, torch.from_numpy(U).cuda(), torch.from_numpy(b).cuda(), x, kappa, mus, csw, BLOCK, 2, 4,
                     storage="f32")
    got = host(x)
    op = oracle.Operator(dims, U, oracle.kappa_to_m(kappa), 0.0, csw)
    for k, m in enumerate(mus):
        ref = op.with_mu(m).sap(b[k], BLOCK, 2, 4).reshape(-1, 4, 3)
        check_close(got[k], ref, "sap", "f32", f"32^3x64 whole lattice system {k}")
    del x
    tm.tm_finalize()
    torch.cuda.empty_cache()


def test_solve_32x64_pm_mu_whole_lattice_residual(lattice_32x64):
    import torch

    dims, U = lattice_32x64
    kappa, csw, mus = 0.1394, 1.5, [0.001, -0.001]
    announce("full-size solve 32^3x64, point source, +-mu, FP64 outer with FP32 SAP")
    b = synth.point_sources(dims, [(0, 0), (0, 0)])
    x = torch.zeros(b.shape, dtype=torch.complex128, device="cuda")
    rc, rep = tm.tm_fgmres_solve(dims, torch.from_numpy(U).cuda(), torch.from_numpy(b).cuda(), x, kappa, mus, csw,
                                 1e-10, storage="f32", form="flexible", restart=20, n_cycles=4, mr_iters=4,
                                 block_dims=BLOCK)
    assert rc == 0, rep
    xg = host(x)
    op = oracle.Operator(dims, U, oracle.kappa_to_m(kappa), 0.0, csw)
    for k, m in enumerate(mus):
        r = b[k].reshape(-1, 4, 3) - op.with_mu(m).apply(xg[k])
        rel = np.linalg.norm(r) / np.linalg.norm(b[k])
        log_solve(f"32^3x64 +-mu flexible system {k} (oracle, whole lattice)", "f32", rel, 1e-10, rep["iters"])
        assert rel <= 1.05e-10
    del x
    tm.tm_finalize()
    torch.cuda.empty_cache()


@pytest.fixture(scope="module")
def lattice_64x128():
    dims = (128, 64, 64, 64)
    announce("generating the 64^3x128 gauge field")
    return dims, synth.gauge_field(dims, 0.6, seed=5)


@pytest.mark.parametrize("prec", ["f16", "bf16"])
def test_sap_64x128_24_systems_internal_point_sources(lattice_64x128, prec):
    import torch

    dims, U = lattice_64x128
    kappa, csw, mu = 0.1373, 1.5, 0.0009
    V = U.shape[0]
    nsys = 24
    mus = [mu] * 12 + [-mu] * 12
    rng = np.random.default_rng(128)
    # one point source per system, each in its own block, spread over the lattice
    src = [np.array([rng.integers(0, d) for d in dims]) for _ in range(nsys)]
    src[0] = np.zeros(4, int)
    src[1] = np.array(dims) - 1
    announce(f"full-size SAP 64^3x128 {prec}: 24 systems in one launch, internal buffers")
    Ud = torch.from_numpy(U).cuda()
    nbytes = tm.tm_spinor_bytes(dims, nsys, prec, layout_block=BLOCK)
    bi = torch.zeros(nbytes, dtype=torch.uint8, device="cuda")
    xi = torch.zeros(nbytes, dtype=torch.uint8, device="cuda")
    one = torch.zeros((1, V, 4, 3), dtype=torch.complex128, device="cuda")
    for k in range(nsys):
        one.zero_()
        one[0, int(lex(dims, src[k])), (k % 12) // 3, k % 3] = 1.0
        tm.tm_spinor_import_range(dims, one, bi, nsys, k, storage=prec, layout_block=BLOCK)
    tm.tm_sap_smooth(dims, Ud, bi, xi, kappa, mus, csw, BLOCK, 1, 4, storage=prec, io="internal")
    for k in (0, 1, 5, 12, 17, 23):
        tm.tm_spinor_export_range(dims, xi, one, nsys, k, storage=prec, layout_block=BLOCK)
        total = float((one.abs() ** 2).sum())
        assert np.isfinite(total) and total > 0
        # window with the source block at window block 2: everything nonzero lies in blocks 1..3
        origin = (src[k] // 4) * 4 - 8
        if int((origin // 4).sum()) % 2:
            origin[3] -= 4
        idx = window_sites(dims, origin, (24,) * 4)
        got = host(one[0, torch.from_numpy(idx).cuda()])
        # nothing outside the window (SAP reaches one block beyond the source block per cycle)
        assert abs(float((np.abs(got) ** 2).sum()) - total) <= 1e-6 * total
        bw = np.zeros((len(idx), 4, 3), complex)
        bw[int(np.nonzero(idx == lex(dims, src[k]))[0][0]), (k % 12) // 3, k % 3] = 1.0
        ref = window_op(U, dims, origin, (24,) * 4, kappa, csw).with_mu(mus[k]).sap(bw, BLOCK, 1, 4)
        check_close(got, ref.reshape(-1, 4, 3), "sap", prec, f"64^3x128 system {k} source {tuple(src[k])}")
    del Ud, bi, xi, one
    tm.tm_finalize()
    torch.cuda.empty_cache()


def sampled_residual_check(dims, U, x, kappa, csw, mus, src_site, src_sc, sites, bound=1.05e-10):
    """|b_s - (D x)_s| <= bound at each sampled site s (so ||b|| = 1 point sources), the oracle's
    operator applied on a 4^4 window around s."""
    import torch

    centre = lex((4, 4, 4, 4), [2, 2, 2, 2])
    worst = 0.0
    for s in sites:
        c = np.array(np.unravel_index(s, dims))
        origin = c - 2
        w = window_sites(dims, origin, (4, 4, 4, 4))
        xw = host(x[:, torch.from_numpy(w).cuda()])
        op = window_op(U, dims, origin, (4, 4, 4, 4), kappa, csw)
        for k, m in enumerate(mus):
            dx = op.with_mu(m).apply(xw[k]).reshape(-1, 4, 3)[centre]
            bs = np.zeros((4, 3), complex)
            if s == src_site:
                bs[src_sc[k]] = 1.0
            r = float(np.linalg.norm(bs - dx))
            worst = max(worst, r)
            assert r <= bound, (s, k, r)
    return worst


@pytest.mark.parametrize("prec", ["f16", "bf16"])
def test_solve_64x128_pm_mu_16bit_defect_correction(lattice_64x128, prec):
    # the +-mu pair of one point source at 64^3x128 to a true 1e-10: FP64 residual loop around
    # FP32 FGMRES whose SAP runs on FP16 (with per-site scales) or BF16 links and spinors; the
    # group is what fits the device (both systems of the pair, about 147 GB of workspace)
    import torch

    dims, U = lattice_64x128
    kappa, csw, mu = 0.1373, 1.5, 0.0009
    V = U.shape[0]
    mus = [mu, -mu]
    announce(f"full-size solve 64^3x128 {prec}: point source, +-mu, defect correction")
    Ud = torch.from_numpy(U).cuda()
    b = torch.zeros((2, V, 4, 3), dtype=torch.complex128, device="cuda")
    b[:, 0, 0, 0] = 1.0
    x = torch.zeros_like(b)
    rc, rep = tm.tm_fgmres_solve(dims, Ud, b, x, kappa, mus, csw, 1e-10, storage=prec, form="defect_correction",
                                 restart=8, n_cycles=4, mr_iters=4, block_dims=BLOCK)
    announce(f"  status {rc}, {rep['iters']} inner steps, {rep['outer']} corrections, group {rep['group']}, "
             f"true residuals {rep['true_rel_res']}, {rep['t_total']:.1f} s")
    assert rc == 0, rep
    assert max(rep["true_rel_res"][:2]) <= 1e-10
    assert rep["block_dims"] == BLOCK
    rng = np.random.default_rng(128)
    c0 = np.zeros(4, int)
    near = [c0] + [np.eye(4, dtype=int)[a] * sg for a in range(4) for sg in (1, -1)]
    sites = [int(lex(dims, np.mod(c, dims))) for c in near] + [int(v) for v in rng.integers(0, V, 12)]
    worst = sampled_residual_check(dims, U, x, kappa, csw, mus, 0, [(0, 0), (0, 0)], sites)
    announce(f"  oracle residual at {len(sites)} sampled sites: max {worst:.2e}")
    for k in range(2):
        log_solve(f"64^3x128 +-mu defect correction system {k} (library FP64 residual; oracle at sampled sites "
                  f"max {worst:.2e}; group {rep['group']}, {rep['t_total']:.1f} s)", prec, rep["true_rel_res"][k],
                  1e-10, rep["iters"])
    del Ud, b, x
    tm.tm_finalize()
    torch.cuda.empty_cache()


# ---------------------------------------------------------------- two-level method at 48^3x96
# With no setup iterations the aggregate basis on an aggregate depends only on the starting
# vectors there, and a row of the coarse stencil only on the basis of the aggregate and its eight
# neighbours and on the links and clover between them.  So the oracle builds the method on a 12^4
# window of 3^4 aggregates centred on a sampled aggregate (periodic boundaries: the window's own
# wrap only touches its outer aggregates) and its central coarse site is exact; restriction,
# prolongation and the coarse operator are checked there too.

MG_NV = 8


def mg_windows(cdims):
    rng = np.random.default_rng(48)
    picks = [np.zeros(4, int), np.array(cdims) - 1] + [rng.integers(0, cdims) for _ in range(2)]
    return [tuple(int(v) for v in p) for p in picks]


@pytest.fixture(scope="module")
def mg_48x96(lattice_48x96):
    import torch

    dims, U = lattice_48x96
    kappa, csw, mu = 0.1373, 1.5, 0.0009
    announce("full-size two-level method 48^3x96: 8 starting vectors, no setup iterations")
    v0 = synth.gaussian_spinor(dims, MG_NV, seed=480)
    Ud = torch.from_numpy(U).cuda()
    g = tm.MG(dims, Ud, kappa, mu, csw, torch.from_numpy(v0).cuda(), n_vec=MG_NV, setup_iters=0,
              block_dims=BLOCK)
    torch.cuda.empty_cache()
    yield dims, U, v0, g, kappa, csw, mu
    g.close()
    del Ud
    tm.tm_finalize()
    torch.cuda.empty_cache()


def window_mg(U, v0, dims, J, kappa, csw, mu):
    origin = [4 * (J[a] - 1) for a in range(4)]
    w = window_sites(dims, origin, (12, 12, 12, 12))
    op = oracle.Operator((12, 12, 12, 12), U[w], oracle.kappa_to_m(kappa), mu, csw)
    o = oracle.MG(op, BLOCK, MG_NV, delta=1.0)
    o.setup(v0[:, w])
    return o, w


def coarse_index(cdims, J):
    return ((J[0] * cdims[1] + J[1]) * cdims[2] + J[2]) * cdims[3] + J[3]


def test_two_level_48x96_stencil_restriction_prolongation(mg_48x96):
    import torch

    dims, U, v0, g, kappa, csw, mu = mg_48x96
    cdims = g.cdims
    _, Dc = g.export()
    Dc = host(Dc)
    r = synth.gaussian_spinor(dims, 1, seed=481)
    c = host(g.restrict(torch.from_numpy(r).cuda()))[0]
    rng = np.random.default_rng(482)
    cx = rng.normal(size=(1, g.nc, 2 * MG_NV)) + 1j * rng.normal(size=(1, g.nc, 2 * MG_NV))
    e = host(g.prolong(torch.from_numpy(cx).cuda()))[0]
    y = host(g.coarse_apply(torch.from_numpy(cx).cuda(), [2 * mu]))[0]
    centre = coarse_index((3, 3, 3, 3), (1, 1, 1, 1))
    for J in mg_windows(cdims):
        announce(f"two-level window around aggregate {J}")
        o, w = window_mg(U, v0, dims, J, kappa, csw, mu)
        j = coarse_index(cdims, J)
        assert np.abs(Dc[j] - o.Dc[centre]).max() < 1e-5 * np.abs(o.Dc[centre]).max()
        assert rel_err(c[j], o.restrict(r[0][w])[centre]) < 1e-5
        # the window's coarse vector: the full one at the window's aggregates
        wJ = np.array(np.unravel_index(np.arange(81), (3, 3, 3, 3))).T
        full_j = [coarse_index(cdims, [(J[a] - 1 + q[a]) % cdims[a] for a in range(4)]) for q in wJ]
        cw = cx[0][full_j]
        ew = o.prolong(cw).reshape(12, 12, 12, 12, 4, 3)[4:8, 4:8, 4:8, 4:8]
        eg = e[w].reshape(12, 12, 12, 12, 4, 3)[4:8, 4:8, 4:8, 4:8]
        assert rel_err(eg, ew) < 1e-6
        assert rel_err(y[j], o.coarse_apply(cw, 2 * mu)[centre]) < 1e-5


def test_two_level_48x96_galerkin_and_orthonormality(mg_48x96):
    # at every site: R P = 1 and D_c(mu, delta = 1) = P^+ D(mu) P (FP64 operator), both on the GPU
    import torch

    dims, U, v0, g, kappa, csw, mu = mg_48x96
    rng = np.random.default_rng(483)
    cx = rng.normal(size=(1, g.nc, 2 * MG_NV)) + 1j * rng.normal(size=(1, g.nc, 2 * MG_NV))
    cd = torch.from_numpy(cx).cuda()
    e = g.prolong(cd)
    assert rel_err(host(g.restrict(e)), cx) < 1e-5
    Ud = torch.from_numpy(U).cuda()
    De = tm.tm_dirac_apply(dims, Ud, e, kappa, [mu], csw, storage="f64")
    ref = host(g.restrict(De))
    assert rel_err(host(g.coarse_apply(cd, [mu])), ref) < 1e-5
    del Ud, De, e


def test_two_level_48x96_solve_sampled_residual(lattice_48x96):
    # the benchmark's configuration: 28 vectors, 5 setup iterations, 12 point sources
    import torch

    dims, U = lattice_48x96
    kappa, csw, mu = 0.1373, 1.5, 0.0009
    V = U.shape[0]
    announce("full-size two-level solve 48^3x96: 28 vectors, 5 setup iterations, 12 point sources")
    Ud = torch.from_numpy(U).cuda()
    gen = torch.Generator(device="cuda")
    gen.manual_seed(2024)
    v0 = torch.randn((28, V, 4, 3), dtype=torch.complex128, device="cuda", generator=gen)
    g = tm.MG(dims, Ud, kappa, mu, csw, v0)
    del v0
    torch.cuda.empty_cache()
    b = torch.zeros((12, V, 4, 3), dtype=torch.complex128, device="cuda")
    for k in range(12):
        b[k, 0, k // 3, k % 3] = 1.0
    x = torch.zeros_like(b)
    rc, rep = tm.tm_fgmres_solve(dims, Ud, b, x, kappa, [mu] * 12, csw, 1e-10, storage="f32",
                                 form="defect_correction", restart=8, mg=g)
    assert rc == 0, rep
    assert max(rep["true_rel_res"][:12]) <= 1e-10
    g.close()
    rng = np.random.default_rng(97)
    sites = [0, lex(dims, [0, 0, 0, 1]), lex(dims, [95, 47, 47, 47])] + list(rng.integers(0, V, 6))
    for s in sites:
        c = np.array(np.unravel_index(s, dims))
        origin = c - 2
        w = window_sites(dims, origin, (4, 4, 4, 4))
        xw = host(x[:, torch.from_numpy(w).cuda()])
        op = window_op(U, dims, origin, (4, 4, 4, 4), kappa, csw).with_mu(mu)
        centre = lex((4, 4, 4, 4), [2, 2, 2, 2])
        for k in range(12):
            dx = op.apply(xw[k]).reshape(-1, 4, 3)[centre]
            bs = np.zeros((4, 3), complex)
            if s == 0:
                bs[k // 3, k % 3] = 1.0
            assert np.linalg.norm(bs - dx) <= 1.05e-10, (s, k)
    del Ud, b, x
    tm.tm_finalize()
    torch.cuda.empty_cache()
