"""Seeded input generator: Philox known answers, SU(3) properties, site-local generation."""
import os

import numpy as np

from paper_1610_02370_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_philox_known_answers():
    n = 0
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            w = [int(t, 16) for t in line.split()]
            assert synth.philox4x32_10(w[0:4], w[4:6]) == tuple(w[6:10])
            n += 1
    assert n == 3


def test_links_are_su3():
    U = synth.gauge_field((2, 2, 2, 4), 0.6, seed=3).reshape(-1, 3, 3)
    eye = np.eye(3)
    uu = np.einsum("nij,nkj->nik", U, U.conj())
    assert np.abs(uu - eye).max() < 1e-14
    assert np.abs(np.linalg.det(U) - 1).max() < 1e-14


def test_mean_plaquette_scale():
    # <Re tr U>/3 = 1 - eps^2 <tr H^2>/6 + O(eps^4); <tr H^2> = 8 * (1/2) / ... = 4 for
    # H = sum h_a lambda_a/2 with tr(lambda_a lambda_b) = 2 delta_ab and h_a ~ N(0,1).
    eps = 0.05
    U = synth.gauge_field((8, 8, 8, 8), eps, seed=1).reshape(-1, 3, 3)
    tr = np.einsum("nii->n", U).real.mean() / 3
    expect = 1 - eps ** 2 * 4 / 6
    assert abs(tr - expect) < 5e-5


def test_site_local_generation_matches_full_field():
    dims = (4, 4, 4, 6)
    U = synth.gauge_field(dims, 0.5, seed=2)
    sites = np.array([0, 5, 17, 383], np.int64)
    assert np.array_equal(synth.gauge_links_at(sites, 0.5, seed=2), U[sites])


def test_seed_changes_field_and_gaussian_moments():
    a = synth.gauge_field((2, 2, 2, 2), 0.3, seed=1)
    b = synth.gauge_field((2, 2, 2, 2), 0.3, seed=2)
    assert np.abs(a - b).max() > 1e-3
    g = synth.gaussian_spinor((4, 4, 4, 4), 4, seed=101)
    assert abs(g.real.mean()) < 0.02 and abs(g.imag.mean()) < 0.02
    assert abs(g.real.var() - 1) < 0.03 and abs(g.imag.var() - 1) < 0.03


def test_point_sources():
    p = synth.all_point_sources((2, 2, 2, 2))
    assert p.shape == (12, 16, 4, 3)
    for k in range(12):
        assert p[k].sum() == 1 and p[k, 0, k // 3, k % 3] == 1
