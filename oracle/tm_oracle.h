/*
 * Plain FP64 CPU oracle for the twisted-mass Wilson-clover operator, the
 * red-black SAP smoother with minimal-residual block solves, and flexible
 * GMRES (arXiv:1610.02370).
 *
 * TEST INFRASTRUCTURE ONLY.  This code is the independent truth that the
 * GPU library is checked against.  It shares no code, header, table or
 * constant with the GPU library and must never be linked into it.  Only the
 * test suite, the smoke check and the benchmark's CPU-baseline leg load it.
 *
 * Conventions (the paper fixes gamma5 and the Clifford relation; the rest is
 * a reading, listed in the design notes):
 *   dims[4] = (T, Z, Y, X); site index lexicographic, t slowest, x fastest.
 *   Direction mu: 0 = t (x0), 1 = x (x1), 2 = y (x2), 3 = z (x3).
 *   Spinor at a site: psi[s][c], s = spin 0..3, c = colour 0..2 (12 complex).
 *   Links: U[site][mu][row][col], complex, SU(3).
 *   Clover: clov[site][12][12] complex, index 3*s + c.
 *   Chiral gamma basis with gamma5 = gamma0 gamma1 gamma2 gamma3 = diag(1,1,-1,-1).
 *   m = 1/(2 kappa) - 4 is applied by the caller; the oracle takes m.
 *
 * Parity status of each function is stated at its definition in tm_oracle.c.
 */
#ifndef TM_ORACLE_H
#define TM_ORACLE_H

#include <complex.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef double _Complex or_cplx;

typedef struct {
    int dims[4];            /* (T, Z, Y, X) */
    int antiperiodic_t;     /* 1: spinor hops across the t boundary pick up -1 */
    const or_cplx* U;       /* [V][4][3][3] */
    const or_cplx* clov;    /* [V][12][12], may be NULL when csw == 0 */
    double m;               /* bare mass: D contains (m + 4) */
    double mu;              /* twisted mass: D contains + i mu Gamma5 */
    double theta[4];        /* twisted boundary phases (radians), mu = t, x, y, z:
                               psi(x + L_mu e_mu) = exp(i theta_mu) psi(x); added to the
                               -1 of antiperiodic_t */
    double mu_shift[2];     /* added to mu on even / odd sites (parity of t+z+y+x) */
} or_op;

typedef struct {
    int iters;              /* total Arnoldi steps */
    int restarts;           /* completed restart cycles */
    int converged;          /* 1 when the true residual met tol */
    double true_rel_res;    /* ||b - D x|| / ||b|| at exit */
} or_report;

long or_volume(const int dims[4]);
/* gamma matrix mu (0..3), or gamma5 for mu == 4; g[4*row + col]. */
void or_gamma(int mu, or_cplx g[16]);

/* Clover term of the paper's Wilson operator: -(csw/32) sum_{mu,nu}
 * (gamma_mu gamma_nu) (x) (Q_munu - Q_numu), as a 12x12 matrix per site. */
void or_clover(const int dims[4], const or_cplx* U, double csw, or_cplx* clov);

/* out = D(mu) in over the whole lattice. */
void or_dirac(const or_op* op, const or_cplx* in, or_cplx* out);

/* out = block-diagonal part of D(mu) for Schwarz blocks bdims (hops that
 * leave a block dropped: Dirichlet cuts at block faces). */
void or_dirac_blockdiag(const or_op* op, const int bdims[4], const or_cplx* in, or_cplx* out);

/* Colour of the Schwarz block that holds site: (sum of block coords) mod 2. */
int or_block_colour(const int dims[4], const int bdims[4], long site);

/* Minimal-residual approximation of D_BB^{-1} r on one block, block given by
 * its block coordinates B[4]; r and e are full-lattice vectors, only the
 * block's sites are read / written (e is overwritten there). */
void or_mr_block(const or_op* op, const int bdims[4], const int B[4], const or_cplx* r,
                 or_cplx* e, int iters);

/* Block solve with even-odd preconditioning (section 2.5): sites split by the
 * parity of t+z+y+x (0 = even); MR runs `iters` steps on the odd-site Schur
 * complement Dhat = D_oo - D_oe D_ee^-1 D_eo of D_BB with right-hand side
 * r_o - D_oe D_ee^-1 r_e, then e_e = D_ee^-1 (r_e - D_eo e_o). */
void or_mr_block_eo(const or_op* op, const int bdims[4], const int B[4], const or_cplx* r,
                    or_cplx* e, int iters);

/* Red-black multiplicative SAP: n_cycles cycles, colour 0 then colour 1,
 * each block solved by mr_iters MR steps (mr_iters < 0: exact block solve by
 * dense Gaussian elimination, used only by the closed-form pins).
 * x is in/out. Returns 0, or -3 when a direction has an odd block count. */
int or_sap(const or_op* op, const int bdims[4], int n_cycles, int mr_iters, const or_cplx* b,
           or_cplx* x);
/* As or_sap; eo != 0 solves the blocks with or_mr_block_eo's method. */
int or_sap_eo(const or_op* op, const int bdims[4], int n_cycles, int mr_iters, int eo,
              const or_cplx* b, or_cplx* x);

/* Even-odd reduced operator of eq. (oereduced), even sites kept:
 * Dhat = D_ee - D_eo D_oo^-1 D_oe (parity of t+z+y+x, 0 = even).  in and out
 * are full-lattice vectors; only even sites are read, odd sites of out are 0. */
void or_dhat(const or_op* op, const or_cplx* in, or_cplx* out);
/* out = Dhat^+ in (even sites), as Gamma5 Dhat(-mu) Gamma5. */
void or_dhat_dag(const or_op* op, const or_cplx* in, or_cplx* out);
/* CG on the squared even-odd reduced system (section 3, the CG comparison):
 * Dhat^+ Dhat x_e = Dhat^+ bhat with bhat = b_e - D_eo D_oo^-1 b_o, run in the
 * least-squares form (the reduced residual r = bhat - Dhat x_e is updated
 * alongside), then x_o = D_oo^-1 (b_o - D_oe x_e).  The reduced residual is
 * the even part of the full residual and the odd part vanishes, so it stops
 * when ||r|| <= tol ||b||.  x is in/out (its even part is the initial guess).
 * Returns 0 when converged. */
int or_cg_eo(const or_op* op, const or_cplx* b, or_cplx* x, double tol, int max_iters, or_report* rep);

/* Flexible GMRES(restart) with right preconditioning (precond: 0 = none,
 * 1 = SAP with the given parameters), modified Gram-Schmidt, complex Givens
 * rotations.  x is in/out (initial guess).  Stops when the true relative
 * residual <= tol or after max_iters Arnoldi steps.  Returns 0 when
 * converged, 1 otherwise. */
int or_fgmres(const or_op* op, const or_cplx* b, or_cplx* x, double tol, int restart, int max_iters,
              int precond, const int bdims[4], int n_cycles, int mr_iters, or_report* rep);
/* As or_fgmres; eo != 0 uses SAP with even-odd preconditioned block solves. */
int or_fgmres_eo(const or_op* op, const or_cplx* b, or_cplx* x, double tol, int restart, int max_iters,
                 int precond, const int bdims[4], int n_cycles, int mr_iters, int eo, or_report* rep);

/* ------------------------------------------------ two-level method (2.3-2.6)
 *
 * Aggregates are blocks of adims sites split by spin half (spins {0,1} and
 * {2,3}, where gamma5 = +1 and -1).  Coarse vectors are [nc][2 nv] with the
 * coarse site index lexicographic in block coordinates (t slowest) and
 * component sg*nv + i for test vector i on spin half sg; Gamma5c = +1 on the
 * first nv components.  P is stored as nv lattice vectors [nv][V][12]; the
 * coarse stencil as Dc[nc][9][2nv][2nv], term t = 0 (the site itself), 1 + mu
 * (coupling to the aggregate one step forward along mu), 5 + mu (backward). */
typedef struct {
    int adims[4];           /* aggregate = Schwarz block of the smoother */
    int nv;                 /* test vectors */
    double delta;           /* coarse twist: mu_c = delta * mu (eq. (delta)) */
    double coarse_tol;      /* coarse GMRES: relative residual estimate target (<= 0: run every step) */
    int coarse_restart;     /* coarse GMRES restart length */
    int coarse_max_restarts;
    int post_cycles;        /* SAP post-smoothing cycles */
    int mr_iters;           /* MR steps per block solve */
    int setup_iters;        /* setup iterations (the first one is SAP only) */
    int setup_cycles;       /* SAP cycles per test vector in setup iteration 1 */
    int coarse_eo;          /* 1: coarse GMRES on the even-odd reduced coarse system */
    or_cplx* P;             /* [nv][V][12], caller-allocated */
    or_cplx* Dc;            /* [nc][9][2nv][2nv], caller-allocated */
} or_mg;

void or_mg_block_orthonormalize(const int dims[4], const int adims[4], int nv, const or_cplx* v, or_cplx* P);
void or_mg_restrict(const int dims[4], const int adims[4], int nv, const or_cplx* P, const or_cplx* r, or_cplx* c);
void or_mg_prolong(const int dims[4], const int adims[4], int nv, const or_cplx* P, const or_cplx* c, or_cplx* e);
void or_mg_coarse_build(const or_op* op, const int adims[4], int nv, const or_cplx* P, or_cplx* Dc);
void or_mg_coarse_apply(const int cdims[4], int nv, const or_cplx* Dc, double mu_c, const or_cplx* x, or_cplx* y);
int or_mg_coarse_gmres(const int cdims[4], int nv, const or_cplx* Dc, double mu_c, const or_cplx* b, or_cplx* x,
                       double tol, int restart, int max_restarts, or_report* rep);
/* Even-odd reduced coarse operator (coarse parity = sum of coarse coordinates mod 2,
 * odd sites kept): y_o = (D_oo - D_oe D_ee^-1 D_eo) x_o; even parts ignored / zero. */
void or_mg_coarse_dhat(const int cdims[4], int nv, const or_cplx* Dc, double mu_c, const or_cplx* x, or_cplx* y);
/* As or_mg_coarse_gmres on the reduced system, then the even sites recovered. */
int or_mg_coarse_gmres_eo(const int cdims[4], int nv, const or_cplx* Dc, double mu_c, const or_cplx* b, or_cplx* x,
                          double tol, int restart, int max_restarts, or_report* rep);
void or_mg_precond(const or_op* op, const or_mg* mg, const or_cplx* r, or_cplx* z);
int or_fgmres_mg(const or_op* op, const or_mg* mg, const or_cplx* b, or_cplx* x, double tol, int restart,
                 int max_iters, or_report* rep);
int or_mg_setup(const or_op* op, or_mg* mg, const or_cplx* v0, or_cplx* v_out);

/* Number of OpenMP threads the oracle uses (1 when built without OpenMP). */
int or_num_threads(void);
void or_set_num_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
