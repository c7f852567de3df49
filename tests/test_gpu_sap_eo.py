"""GPU parity of SAP with even-odd preconditioned block solves (section 2.5).

Each block system is reduced to its odd sites (Schur complement
D_oo - D_oe D_ee^-1 D_eo, sites split by the parity of t+z+y+x), MR runs on
the reduced system and the even half is recovered.  The HIP path and the FP64
oracle run the same red-black sweeps on the same seeded inputs; each result is
checked norm-wise and per site against the smoother's error model of gpu_util
(f64 1e-13, f32 2e-6, f16 2e-3, bf16 1.5e-2).
"""
import numpy as np
import pytest

import oracle
import paper_1610_02370_amd as tm
from paper_1610_02370_amd import synth

from gpu_util import TOL as ERR_TOL
from gpu_util import announce, check_close, dev, host, rel_err

pytestmark = pytest.mark.gpu

TOL = ERR_TOL["sap"]

CASES = [
    # dims, block, eps, kappa, mus, csw, cycles, mr, antiperiodic
    ((4, 4, 4, 4), (2, 2, 2, 2), 0.3, 0.16, [0.01], 0.0, 3, 4, False),
    ((8, 8, 8, 8), (4, 4, 4, 4), 0.5, 0.1632, [0.003, -0.003], 1.5, 2, 4, True),
    ((4, 12, 4, 4), (2, 6, 2, 2), 0.6, 0.1394, [0.001], 1.5, 2, 3, False),
    ((8, 8, 4, 16), (4, 4, 2, 8), 0.6, 0.1373, [0.0009, -0.0009, 0.02], 1.5, 1, 2, False),
    ((8, 8, 8, 16), (4, 4, 4, 8), 0.5, 0.1373, [0.0009], 1.5, 1, 2, False),  # 512-site blocks
    ((6, 6, 4, 4), (3, 3, 2, 2), 0.6, 0.1373, [0.0009], 1.5, 2, 3, False),  # odd extents in t and z
]


@pytest.fixture(scope="module")
def fields():
    out = []
    for k, (dims, bd, eps, kappa, mus, csw, cyc, mr, ap) in enumerate(CASES):
        U = synth.gauge_field(dims, eps, seed=40 + k)
        b = synth.gaussian_spinor(dims, len(mus), seed=140 + k)
        x0 = 0.1 * synth.gaussian_spinor(dims, len(mus), seed=240 + k)
        op = oracle.Operator(dims, U, oracle.kappa_to_m(kappa), 0.0, csw, antiperiodic_t=ap)
        ref = np.stack([op.with_mu(m).sap(b[i], bd, cyc, mr, x0=x0[i], eo=True).reshape(-1, 4, 3)
                        for i, m in enumerate(mus)])
        out.append((U, b, x0, ref))
    return out


@pytest.mark.parametrize("prec", ["f64", "f32", "f16", "bf16"])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_sap_eo_matches_oracle(fields, case, prec):
    dims, bd, eps, kappa, mus, csw, cyc, mr, ap = CASES[case]
    U, b, x0, ref = fields[case]
    announce(f"sap eo parity case={case} dims={dims} block={bd} prec={prec}")
    x = dev(x0)
    tm.tm_sap_smooth(dims, dev(U), dev(b), x, kappa, mus, csw, bd, cyc, mr, storage=prec, antiperiodic_t=ap,
                     eo=True)
    got = host(x)
    for i in range(len(mus)):
        check_close(got[i], ref[i], "sap", prec, f"eo case {case} {dims} block {bd} system {i}")


def test_sap_eo_zero_guess_and_repeat(fields):
    # zero initial guess (first-cycle shortcuts) and a second call reusing the cached inverses
    dims, bd, eps, kappa, mus, csw, cyc, mr, ap = CASES[1]
    U, b, _, _ = fields[1]
    announce("sap eo zero guess, cached inverses")
    op = oracle.Operator(dims, U, oracle.kappa_to_m(kappa), 0.0, csw, antiperiodic_t=ap)
    for _ in range(2):
        x = dev(np.zeros_like(b))
        tm.tm_sap_smooth(dims, dev(U), dev(b), x, kappa, mus, csw, bd, cyc, mr, storage="f32", antiperiodic_t=ap,
                         eo=True, gauge_tag=7)
        got = host(x)
        for i, m in enumerate(mus):
            ref = op.with_mu(m).sap(b[i], bd, cyc, mr, eo=True).reshape(-1, 4, 3)
            check_close(got[i], ref, "sap", "f32", f"eo zero guess system {i}")
    tm.tm_gauge_release(dev(U))


def test_sap_eo_error_paths(fields):
    dims, bd, eps, kappa, mus, csw, cyc, mr, ap = CASES[1]
    U, b, x0, _ = fields[1]
    announce("sap eo error paths")
    x = dev(x0)
    dims6 = (4, 4, 4, 6)
    U6 = synth.gauge_field(dims6, 0.3, seed=3)
    b6 = synth.gaussian_spinor(dims6, 1, seed=3)
    with pytest.raises(tm.TMError) as e:
        tm.tm_sap_smooth(dims6, dev(U6), dev(b6), dev(np.zeros_like(b6)), kappa, [0.01], csw, (2, 2, 2, 3), 1, 2,
                         storage="f32", eo=True)
    assert e.value.code == -3  # odd block extent in x
    b9 = synth.gaussian_spinor(dims, 9, seed=9)
    with pytest.raises(tm.TMError) as e:
        tm.tm_sap_smooth(dims, dev(U), dev(b9), dev(np.zeros_like(b9)), kappa, [0.001 * (k + 1) for k in range(9)],
                         csw, bd, 1, 2, storage="f32", eo=True)
    assert e.value.code == -1  # more than 8 distinct |mu|


@pytest.mark.parametrize("form,storage", [("flexible", "f64"), ("defect_correction", "f32")])
def test_solve_with_eo_smoother(form, storage):
    dims, kappa, csw = (8, 8, 8, 8), 0.1373, 1.5
    U = synth.gauge_field(dims, 0.6, seed=8)
    mus = [0.0009, -0.0009]
    b = synth.point_sources(dims, [(0, 0), (0, 0)])
    announce(f"solve 8^4 with eo SAP form={form} storage={storage}")
    x = dev(np.zeros_like(b))
    rc, rep = tm.tm_fgmres_solve(dims, dev(U), dev(b), x, kappa, mus, csw, 1e-10, storage=storage, form=form,
                                 restart=16, n_cycles=4, mr_iters=4, block_dims=(4, 4, 4, 4), eo=True)
    assert rc == 0, rep
    xg = host(x)
    op = oracle.Operator(dims, U, oracle.kappa_to_m(kappa), 0.0, csw)
    for i, m in enumerate(mus):
        r = b[i].reshape(-1, 4, 3) - op.with_mu(m).apply(xg[i])
        assert np.linalg.norm(r) / np.linalg.norm(b[i]) <= 1e-10 * 1.05
