"""GPU CG on the squared even-odd reduced system (the FP64 CG baseline of the
paper's solver comparison) against the oracle.

The solution of D x = b is unique: the GPU x must give a true residual
||b - D x|| / ||b|| <= tol with the ORACLE's operator, and on 4^4 it is
compared with dense LU.  The reduced operator itself is checked through one
CG step on tiny lattices indirectly: the iteration counts of the GPU and the
oracle CG (same algorithm, same start) agree within one step.
"""
import numpy as np
import pytest

import oracle
import paper_1610_02370_amd as tm
from paper_1610_02370_amd import synth

from gpu_util import announce, dev, host

pytestmark = pytest.mark.gpu


def test_cg_4x4x4x4_against_dense_lu():
    dims, kappa, mu, csw = (4, 4, 4, 4), 0.16, 0.01, 1.5
    U = synth.gauge_field(dims, 0.3, seed=1)
    b = synth.gaussian_spinor(dims, 1, seed=101)
    announce("cg 4^4 vs dense LU")
    x = dev(np.zeros_like(b))
    rc, rep = tm.tm_cg_solve(dims, dev(U), dev(b), x, kappa, [mu], csw, 1e-11)
    assert rc == 0, rep
    op = oracle.Operator(dims, U, oracle.kappa_to_m(kappa), mu, csw)
    xs = np.linalg.solve(op.dense(), b[0].ravel())
    xg = host(x)[0].ravel()
    r = b[0].ravel() - op.apply(xg)
    assert np.linalg.norm(r) / np.linalg.norm(b) <= 1.05e-11
    assert abs(rep["true_rel_res"][0] - np.linalg.norm(r) / np.linalg.norm(b)) <= 1e-12
    assert np.linalg.norm(xg - xs) <= np.linalg.norm(r) / mu * 1.01
    _, rep_o = op.cg_eo(b[0].ravel(), 1e-11)
    assert abs(rep["iters"] - rep_o["iters"]) <= 1


@pytest.mark.parametrize("mus", [[0.003, -0.003], [0.0009] * 3 + [0.02]])
def test_cg_8x8x8x8_systems(mus):
    dims, kappa, csw = (8, 8, 8, 8), 0.1373, 1.5
    U = synth.gauge_field(dims, 0.6, seed=8)
    b = synth.gaussian_spinor(dims, len(mus), seed=108)
    x0 = 0.01 * synth.gaussian_spinor(dims, len(mus), seed=208)
    announce(f"cg 8^4 mus={mus}")
    x = dev(x0)
    rc, rep = tm.tm_cg_solve(dims, dev(U), dev(b), x, kappa, mus, csw, 1e-10)
    assert rc == 0, rep
    xg = host(x)
    op = oracle.Operator(dims, U, oracle.kappa_to_m(kappa), 0.0, csw)
    for k, m in enumerate(mus):
        r = b[k].reshape(-1, 4, 3) - op.with_mu(m).apply(xg[k])
        rel = np.linalg.norm(r) / np.linalg.norm(b[k])
        assert rel <= 1.05e-10, (k, rel)
        assert abs(rep["true_rel_res"][k] - rel) <= 0.05e-10


def test_cg_error_paths():
    U = synth.gauge_field((4, 4, 4, 6), 0.3, seed=2)
    b = synth.gaussian_spinor((4, 4, 4, 6), 1, seed=2)
    announce("cg error paths")
    with pytest.raises(tm.TMError) as e:
        tm.tm_cg_solve((4, 4, 4, 6), dev(U), dev(b), dev(np.zeros_like(b)), 0.16, [0.01], 1.5, 0.0)
    assert e.value.code == -1
    U3 = synth.gauge_field((4, 4, 4, 3), 0.3, seed=2)
    b3 = synth.gaussian_spinor((4, 4, 4, 3), 1, seed=2)
    with pytest.raises(tm.TMError) as e:
        tm.tm_cg_solve((4, 4, 4, 3), dev(U3), dev(b3), dev(np.zeros_like(b3)), 0.16, [0.01], 1.5, 1e-8)
    assert e.value.code == -2  # odd extent
