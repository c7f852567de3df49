"""The oracle's pins must catch plausible mistakes.

Each case plants one mistake into a copy of the oracle source (on the CPU only),
builds it into a temporary library and runs the pin tests against it; at least one
pin must fail.  The shipped oracle itself is untouched.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "tm_oracle.c")

MUTATIONS = {
    # forward hop with (1 + gamma) instead of (1 - gamma)
    "projector_sign": ("add_hop(g[mu], -1.0, link(op->U, x, mu)", "add_hop(g[mu], +1.0, link(op->U, x, mu)"),
    # backward hop uses U_mu(x) instead of U_mu(x - mu)
    "backward_link_site": ("dag(link(op->U, xb, mu), Wd);\n                add_hop", "dag(link(op->U, x, mu), Wd);\n                add_hop"),
    # link transposed in the colour product
    "link_transposed": ("col += W[3 * c + cp] * psi_n[3 * sp + cp];", "col += W[3 * cp + c] * psi_n[3 * sp + cp];"),
    # twisted mass with the wrong sign
    "twist_sign": ("out[3 * s + c] += _Complex_I * mux", "out[3 * s + c] -= _Complex_I * mux"),
    # one clover leaf dropped
    "clover_leaf_dropped": ("mm4(d1, d2, link(U, xmm_mn, mu), link(U, xmn, nu), leaf);\n    for (int i = 0; i < 9; ++i) Q[i] += leaf[i];",
                            "mm4(d1, d2, link(U, xmm_mn, mu), link(U, xmn, nu), leaf);"),
    # clover normalisation 1/16 instead of 1/32
    "clover_norm": ("-(csw / 32.0)", "-(csw / 16.0)"),
    # MR step with conjugated alpha
    "mr_alpha_conj": ("or_cplx alpha = qr / qq;", "or_cplx alpha = conj(qr) / qq;"),
    # SAP sweeps colour 1 first
    "sap_colour_order": ("!= colour) continue;", "!= 1 - colour) continue;"),
    # Dirichlet cut missing: block operator keeps hops that leave the block
    "no_dirichlet_cut": ("if (lf >= 0) add_hop", "if (lf >= 0 || 1) add_hop"),
    # even-odd: Schur complement with + instead of -
    "eo_schur_sign": ("for (long i = 0; i < n; ++i) q[i] = u[i] - v[i];", "for (long i = 0; i < n; ++i) q[i] = u[i] + v[i];"),
    # even-odd: reduced right-hand side without the even-site correction
    "eo_rhs_uncorrected": ("for (long i = 0; i < n; ++i) rho[i] = r[i] - v[i];", "for (long i = 0; i < n; ++i) rho[i] = r[i];"),
    # even-odd: even sites taken as the reduced ones (parity flipped in the reconstruction)
    "eo_parity_flip": ("if (site_parity(op->dims, sites[l]) == 0)\n            for (int i = 0; i < 12; ++i) e[l * 12 + i] = t[l * 12 + i];",
                       "if (site_parity(op->dims, sites[l]) == 1)\n            for (int i = 0; i < 12; ++i) e[l * 12 + i] = t[l * 12 + i];"),
    # reduced operator with + instead of - before the Schur term
    "eo_dhat_sign": ("for (long i = 0; i < n; ++i) out[i] = u[i] - w[i];", "for (long i = 0; i < n; ++i) out[i] = u[i] + w[i];"),
    # reduced right-hand side without D_oo^-1 (b_o used directly)
    "eo_cg_rhs_no_inverse": ("diag_solve_parity(op, 1, b, t);\n    or_dirac(op, t, q);", "memcpy(t, b, sizeof(or_cplx) * n);\n    mask_parity(op->dims, 1, t);\n    or_dirac(op, t, q);"),
    # twisted boundary phase with the wrong sign on backward hops
    "bc_phase_sign": ("cexp(_Complex_I * (double)dir * op->theta[mu])", "cexp(_Complex_I * op->theta[mu])"),
    # parity shifts of mu swapped
    "mu_shift_parity": ("op->mu_shift[site_parity(op->dims, x)]", "op->mu_shift[1 - site_parity(op->dims, x)]"),
    # Givens rotation without the conjugate
    "givens_conj": ("g[j + 1] = -conj(sn[j]) * g[j];", "g[j + 1] = -sn[j] * g[j];"),
    # two-level method: aggregate inner product without the conjugate
    "mg_aggregate_dot_conj": ("t += conj(a[(size_t)sites[l] * 12 + k]) * b[(size_t)sites[l] * 12 + k];",
                              "t += a[(size_t)sites[l] * 12 + k] * b[(size_t)sites[l] * 12 + k];"),
    # coarse Gamma5 with the spin halves swapped
    "mg_gamma5c_sign": ("(a < nv ? 1.0 : -1.0)", "(a < nv ? -1.0 : 1.0)"),
    # coarse twist not scaled by delta
    "mg_delta_ignored": ("mg->delta * op->mu", "op->mu"),
    # forward and backward coarse couplings exchanged
    "mg_term_direction": ("dir = t <= 4 ? +1 : -1", "dir = t <= 4 ? -1 : +1"),
    # twist counted twice (Galerkin product taken at mu, then delta mu added)
    "mg_twist_twice": ("    op0.mu = 0.0;\n", "\n"),
    # post-smoothing skipped
    "mg_no_post_smoothing": ("if (mg->post_cycles > 0) or_sap_eo", "if (0) or_sap_eo"),
    # prolongation puts spin half 1 coefficients on spins 2 and 3 of half 0
    "mg_prolong_half": ("int sg = q / 6;", "int sg = q / 9;"),
    # setup without the global orthonormalisation
    "mg_setup_no_orthonormalization": ("        mg_orthonormalize(n, nv, v);\n", "\n"),
    # even-odd coarse reduction with + instead of - before the Schur term
    "mg_eo_schur_sign": ("    for (long i = 0; i < n; ++i) out[i] -= t[i];\n}", "    for (long i = 0; i < n; ++i) out[i] += t[i];\n}"),
    # even coarse sites recovered without the odd-site coupling
    "mg_eo_recovery": ("    for (long i = 0; i < n; ++i) t[i] = b[i] - t[i];", "    for (long i = 0; i < n; ++i) t[i] = b[i];"),
}


# The pin that must catch each planted mistake (one test of the pin files; every
# parametrisation of it runs).  Running one pin per mistake keeps the CPU suite short.
CATCHES = {
    "backward_link_site": "test_oracle_operator.py::test_gauge_covariance_of_D",
    "bc_phase_sign": "test_oracle_operator.py::test_twisted_boundary_plane_waves",
    "clover_leaf_dropped": "test_oracle_operator.py::test_clover_constant_abelian_field_closed_form",
    "clover_norm": "test_oracle_operator.py::test_clover_constant_abelian_field_closed_form",
    "eo_cg_rhs_no_inverse": "test_oracle_sap.py::test_cg_eo_against_dense_lu",
    "eo_dhat_sign": "test_oracle_sap.py::test_dhat_is_the_dense_schur_complement",
    "eo_parity_flip": "test_oracle_sap.py::test_mr_eo_dense_replica_and_exact_limit",
    "eo_rhs_uncorrected": "test_oracle_sap.py::test_mr_eo_dense_replica_and_exact_limit",
    "eo_schur_sign": "test_oracle_sap.py::test_mr_eo_dense_replica_and_exact_limit",
    "givens_conj": "test_oracle_sap.py::test_gmres_identity_preconditioner_terminates",
    "link_transposed": "test_oracle_operator.py::test_constant_nonabelian_links_plane_wave",
    "mg_aggregate_dot_conj": "test_oracle_mg.py::test_aggregate_basis_is_phase_fixed_qr",
    "mg_delta_ignored": "test_oracle_mg.py::test_unitary_prolongation_with_exact_coarse_solve_inverts_D",
    "mg_eo_recovery": "test_oracle_mg.py::test_coarse_gmres_eo_matches_dense_solve",
    "mg_eo_schur_sign": "test_oracle_mg.py::test_coarse_dhat_is_the_dense_schur_complement",
    "mg_gamma5c_sign": "test_oracle_mg.py::test_coarse_operator_galerkin_on_uneven_coarse_grid",
    "mg_no_post_smoothing": "test_oracle_mg.py::test_two_level_error_propagation",
    "mg_prolong_half": "test_oracle_mg.py::test_prolongation_commutes_with_gamma5",
    "mg_setup_no_orthonormalization": "test_oracle_mg.py::test_setup_iterations_follow_the_paper",
    "mg_term_direction": "test_oracle_mg.py::test_coarse_operator_galerkin_on_uneven_coarse_grid",
    "mg_twist_twice": "test_oracle_mg.py::test_coarse_operator_galerkin_on_uneven_coarse_grid",
    "mr_alpha_conj": "test_oracle_sap.py::test_mr_monotone_optimal_and_converges",
    "mu_shift_parity": "test_oracle_operator.py::test_mu_shifts_reduce_and_gamma5_hermiticity",
    "no_dirichlet_cut": "test_oracle_sap.py::test_sap_exact_blocks_closed_form",
    "projector_sign": "test_oracle_operator.py::test_free_field_eigenvalues_closed_form",
    "sap_colour_order": "test_oracle_sap.py::test_sap_exact_blocks_closed_form",
    "twist_sign": "test_oracle_operator.py::test_free_field_plane_waves",
}


def test_every_mistake_names_its_pin():
    assert sorted(CATCHES) == sorted(MUTATIONS)


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_catch_planted_mistake(name, tmp_path):
    old, new = MUTATIONS[name][:2]
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation anchor for {name} not found"
    mutated = tmp_path / "tm_oracle.c"
    mutated.write_text(src.replace(old, new))
    (tmp_path / "tm_oracle.h").write_text(open(os.path.join(ROOT, "oracle", "tm_oracle.h")).read())
    lib = tmp_path / "liboracle_mut.so"
    subprocess.check_call(["gcc", "-std=c11", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", str(lib), str(mutated), "-lm"])
    env = dict(os.environ, TM_ORACLE_LIB=str(lib), OMP_NUM_THREADS="2")
    r = subprocess.run(
        [sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", os.path.join(ROOT, "tests", CATCHES[name])],
        cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"planted mistake {name} was not caught by {CATCHES[name]}:\n{r.stdout[-2000:]}"
