"""GPU parity with twisted boundary conditions and parity-dependent twisted-mass
shifts (operator variants of the library beyond the paper's runs).

theta_mu: psi(x + L e_mu) = exp(i theta_mu) psi(x); mu_shift: the twist on
even / odd sites is mu + mu_shift[parity].  Every kernel that applies a hop
across the lattice boundary or the twist is compared with the FP64 oracle:
the operator, the smoother's three FP32 kernels (4^4 blocks, other shapes up
to 256 sites, larger blocks), the FP64 smoother, the even-odd block solves,
and the solvers (true residual from the oracle's operator).
Tolerances as in the parity tests without twists.
"""
import numpy as np
import pytest

import oracle
import paper_1610_02370_amd as tm
from paper_1610_02370_amd import synth

from gpu_util import announce, check_close, dev, host, rel_err

pytestmark = pytest.mark.gpu

THETA = (0.7, -1.3, 0.4, 2.1)
SHIFT = (0.004, -0.011)
KAPPA, CSW = 0.1373, 1.5


@pytest.fixture(scope="module")
def field():
    dims = (8, 8, 8, 16)
    return dims, synth.gauge_field(dims, 0.6, seed=71)


def op_for(dims, U, mu, ap=False):
    return oracle.Operator(dims, U, oracle.kappa_to_m(KAPPA), mu, CSW, antiperiodic_t=ap, theta=THETA,
                           mu_shift=SHIFT)


@pytest.mark.parametrize("prec", ["f64", "f32", "f16", "bf16"])
def test_dirac_twisted(field, prec):
    dims, U = field
    mus = [0.0009, -0.0009]
    psi = synth.gaussian_spinor(dims, 2, seed=171)
    announce(f"dirac twisted prec={prec}")
    out = host(tm.tm_dirac_apply(dims, dev(U), dev(psi), KAPPA, mus, CSW, storage=prec, antiperiodic_t=True,
                                 theta=THETA, mu_shift=SHIFT))
    for k, m in enumerate(mus):
        ref = op_for(dims, U, m, ap=True).apply(psi[k]).reshape(-1, 4, 3)
        check_close(out[k], ref, "dirac", prec, f"twisted system {k}")


@pytest.mark.parametrize("prec,block,eo", [
    ("f32", (4, 4, 4, 4), False),   # 4^4 kernel
    ("f32", (4, 4, 2, 4), False),   # general shapes up to 256 sites
    ("f32", (4, 4, 4, 8), False),   # larger blocks
    ("f64", (4, 4, 4, 4), False),
    ("f16", (4, 4, 4, 4), False),
    ("bf16", (4, 4, 4, 4), False),
    ("f32", (4, 4, 4, 4), True),    # even-odd block solves
    ("f64", (4, 4, 4, 4), True),
])
def test_sap_twisted(field, prec, block, eo):
    dims, U = field
    mus = [0.0009, -0.0009]
    b = synth.gaussian_spinor(dims, 2, seed=172)
    x0 = 0.1 * synth.gaussian_spinor(dims, 2, seed=272)
    announce(f"sap twisted prec={prec} block={block} eo={eo}")
    x = dev(x0)
    tm.tm_sap_smooth(dims, dev(U), dev(b), x, KAPPA, mus, CSW, block, 2, 3, storage=prec, theta=THETA,
                     mu_shift=SHIFT, eo=eo)
    got = host(x)
    for k, m in enumerate(mus):
        ref = op_for(dims, U, m).sap(b[k], block, 2, 3, x0=x0[k], eo=eo).reshape(-1, 4, 3)
        check_close(got[k], ref, "sap", prec, f"twisted block {block} eo {eo} system {k}")


@pytest.mark.parametrize("solver", ["fgmres_dc", "fgmres_eo", "cg"])
def test_solvers_twisted(field, solver):
    dims, U = field
    mus = [0.0009, -0.0009]
    b = synth.point_sources(dims, [(0, 0), (3, 2)])
    announce(f"solve twisted {solver}")
    x = dev(np.zeros_like(b))
    if solver == "cg":
        rc, rep = tm.tm_cg_solve(dims, dev(U), dev(b), x, KAPPA, mus, CSW, 1e-10, theta=THETA, mu_shift=SHIFT,
                                 antiperiodic_t=True)
    else:
        rc, rep = tm.tm_fgmres_solve(dims, dev(U), dev(b), x, KAPPA, mus, CSW, 1e-10, storage="f32",
                                     form="defect_correction", restart=8, block_dims=(4, 4, 4, 4), theta=THETA,
                                     mu_shift=SHIFT, antiperiodic_t=True, eo=(solver == "fgmres_eo"))
    assert rc == 0, rep
    xg = host(x)
    for k, m in enumerate(mus):
        r = b[k].reshape(-1, 4, 3) - op_for(dims, U, m, ap=True).apply(xg[k])
        assert np.linalg.norm(r) / np.linalg.norm(b[k]) <= 1.05e-10
