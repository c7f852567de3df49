/*
 * tm.h - C ABI of the MI355X library for the twisted-mass Wilson-clover
 * operator, its red-black Schwarz (SAP) smoother and the SAP-preconditioned
 * flexible GMRES solve (arXiv:1610.02370).
 *
 * Conventions shared by every call
 * --------------------------------
 * Lattice  dims = (T, Z, Y, X), V = T*Z*Y*X sites, lexicographic site index
 *          with t slowest and x fastest (section 2.1, lattice definition).
 * Direction mu: 0 = t (x0), 1 = x (x1), 2 = y (x2), 3 = z (x3).
 * Spinor   12 complex per site, index [spin][colour]; spin basis is the chiral
 *          basis with gamma5 = diag(1, 1, -1, -1) (section 2.1).
 * Links    U_mu(x) in SU(3), 3x3 complex, index [row][col].  The library
 *          stores two rows and rebuilds the third, so links must be special
 *          unitary to 1e-6 (TM_ERR_NOT_SU3 otherwise).
 * Mass     kappa gives the bare mass through m + 4 = 1 / (2 kappa).
 * Twist    system k carries the twist + i mu[k] Gamma5 (section 2.1:
 *          +mu for the u flavour, -mu for the d flavour).
 *
 * Canonical layout (io = TM_IO_CANONICAL): complex128 ("double _Complex")
 *   links  [V][4][3][3]
 *   spinor [nsys][V][4][3]
 * Internal layout (io = TM_IO_INTERNAL): opaque device buffers of
 *   tm_spinor_bytes() bytes, produced only by tm_spinor_import() with the same
 *   dims, nsys, storage precision and layout block; they let a caller keep
 *   many systems resident at storage precision (e.g. FP16 at 64^3 x 128).
 *
 * Memory ownership: every U / psi / out / b / x pointer is a caller-owned
 * DEVICE pointer on the current HIP device.  The library never frees caller
 * memory.  It converts U into its own link copy and clover term.  With
 * opts.gauge_tag == 0 it rebuilds them on every call (and synchronises once
 * to validate the links); with a nonzero tag it reuses the copy made for the
 * same (U pointer, tag, dims, kappa, c_sw, precision, tile), so the caller
 * must change the tag, or call tm_gauge_release(U), whenever the contents at
 * U change.  A new nonzero tag with the same U pointer rebuilds that
 * pointer's older copy of the same shape in place (no new allocation).
 * tm_finalize() frees everything the library allocated.
 *
 * Streams: all work is enqueued on opts->stream (NULL = the null stream).
 * tm_dirac_apply and tm_sap_smooth return after enqueueing (the caller
 * synchronises); tm_fgmres_solve synchronises once per Arnoldi step to read
 * the Hessenberg column and returns with the result complete.
 *
 * Errors: negative return values are errors and leave outputs unspecified;
 * tm_last_error() returns a thread-local message for the last failure.
 * Calls are not re-entrant on one stream: two calls that overlap on the same
 * device share the library's scratch buffers and race.
 */
#ifndef TM_H
#define TM_H

#include <stddef.h>

#if defined(__GNUC__) || defined(__clang__)
#define TM_API __attribute__((visibility("default")))
#else
#define TM_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ status codes */
#define TM_OK 0
#define TM_NOT_CONVERGED 1   /* solve stopped at max_iters; x holds the best iterate */
#define TM_ERR_ARG (-1)      /* null pointer or invalid argument value */
#define TM_ERR_DIMS (-2)     /* dims not positive, or not divisible by the block dims */
#define TM_ERR_BLOCKS (-3)   /* odd block count in a direction (breaks red-black) or block too large */
#define TM_ERR_PREC (-4)     /* unsupported precision combination */
#define TM_ERR_HIP (-5)      /* HIP runtime error */
#define TM_ERR_NOMEM (-6)    /* device allocation failed */
#define TM_ERR_NONFINITE (-7)/* NaN or Inf in an input field */
#define TM_ERR_NOT_SU3 (-8)  /* a link is not special unitary to 1e-6 */

/* ------------------------------------------------------------- precisions */
typedef enum { TM_F64 = 0, TM_F32 = 1, TM_F16 = 2, TM_BF16 = 3 } tm_prec;

#define TM_IO_CANONICAL 0
#define TM_IO_INTERNAL 1

#define TM_MAX_SYS 64

typedef struct {
    int dims[4];          /* (T, Z, Y, X) */
    int antiperiodic_t;   /* 1: spinor hops across the t boundary get a factor -1 */
    int nsys;             /* number of systems in psi / b / x (1 .. TM_MAX_SYS) */
    const double* mu;     /* HOST array [nsys]: twisted mass of each system */
    double theta[4];      /* twisted boundary conditions (radians) for mu = t, x, y, z:
                             psi(x + L_mu e_mu) = exp(i theta_mu) psi(x), so a hop across the
                             boundary along +mu takes exp(i theta_mu) and along -mu its conjugate;
                             combined with antiperiodic_t (which adds pi to theta_t); 0 = periodic */
    double mu_shift[2];   /* added to every system's mu on even / odd sites (parity of t+z+y+x):
                             the twist is i (mu_k + mu_shift[parity]) Gamma5; 0 = none */
} tm_geom;

typedef struct {
    int storage;          /* tm_prec of links and spinors inside the library */
    int compute;          /* TM_F64 (storage TM_F64 only) or TM_F32 */
    void* stream;         /* hipStream_t; NULL = null stream */
    int io;               /* TM_IO_CANONICAL or TM_IO_INTERNAL */
    int layout_block[4];  /* site tiling of internal buffers; zeros = default
                             (4^4 where it divides dims, else 2 or 1 per axis);
                             tm_sap_smooth always tiles by its block_dims */
    unsigned long long gauge_tag; /* 0: rebuild the gauge copy every call; else cache key (see above) */
    int sys_tile;         /* SAP: systems per workgroup (0 = all systems of the call in one workgroup,
                             so links and clover are read once per half-sweep) */
    int sap_eo;           /* SAP block solves (section 2.5): 0 = MR on D_BB; 1 = even-odd
                             preconditioned: MR on the odd-site Schur complement
                             D_oo - D_oe D_ee^-1 D_eo (parity of t+z+y+x), e_e recovered after.
                             Needs an even block extent in x (else TM_ERR_BLOCKS) and at most 8
                             distinct |mu| per call (else TM_ERR_ARG); the site inverses
                             (A + i mu gamma5)^-1 are built on first use per |mu| and kept with
                             the gauge copy (288 B per site at FP32, 576 B at FP64) */
} tm_opts;

/* Fills opts with: storage F64, compute F64, null stream, canonical io, tag 0. */
TM_API void tm_opts_default(tm_opts* opts);

/* --------------------------------------------------------------- library */
TM_API int tm_init(void);                 /* optional: creates per-device state */
TM_API int tm_finalize(void);             /* frees every library allocation */
TM_API const char* tm_last_error(void);   /* thread-local message of the last error */
TM_API int tm_gauge_release(const void* U);  /* drops every cached copy derived from U */

/* --------------------------------------------------------- the operator */
/*
 * out = D(mu_k) psi_k for every system k (section 2.1, the Wilson-clover
 * operator with twist):
 *   D = (m+4) - (c_sw/32) sum_{mu,nu} (gamma_mu gamma_nu) (x) (Q_munu - Q_numu)
 *       - 1/2 sum_mu [(1 - gamma_mu) U_mu(x) psi(x+mu) + (1 + gamma_mu) U_mu(x-mu)^+ psi(x-mu)]
 *       + i mu Gamma5,
 * with Q_munu the four-leaf clover of plaquettes.  Periodic in every
 * direction unless geom->antiperiodic_t / geom->theta twist the boundaries;
 * geom->mu_shift adds a parity-dependent shift to the twist (both are operator
 * variants of the library beyond the paper's runs).  psi and out must not alias.
 * Precision: opts->storage / opts->compute; the clover is built in FP64 and
 * rounded to storage (FP32 for FP16/BF16 storage).
 */
TM_API int tm_dirac_apply(const tm_geom* geom, const void* U, const void* psi, void* out, double kappa, double c_sw,
                   const tm_opts* opts);

/* ------------------------------------------------------------ the smoother */
/*
 * Red-black multiplicative SAP (section 2.4, eq. for E_SAP and the block
 * inverses B_rr, B_bb): the lattice is tiled by blocks block_dims (T,Z,Y,X)
 * coloured by the parity of the sum of block coordinates.  One cycle sweeps
 * colour 0 (the block holding the origin) then colour 1; each sweep sets
 * r = b - D x on the blocks of that colour and adds to x the result of
 * mr_iters minimal-residual steps on D restricted to the block (hops that
 * leave the block dropped), started from zero.  x is in/out (initial guess).
 * Every direction needs an even number (>= 2) of blocks (TM_ERR_BLOCKS), and
 * a block holds at most 1024 sites.  b and x must not alias.
 */
TM_API int tm_sap_smooth(const tm_geom* geom, const void* U, const void* b, void* x, double kappa, double c_sw,
                  const int block_dims[4], int n_cycles, int mr_iters, const tm_opts* opts);

/*
 * tm_sap_smooth for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, result and errors as tm_sap_smooth (sap_eo must be 0), and the
 * same kernels; it calls no hipMalloc, hipFree or other allocating routine.
 * The gauge copy, the clover term, the internal copies of canonical b and x
 * and the validation flags live in a fixed device array of
 * TM_NOALLOC_SCRATCH_BYTES that the library holds on every GPU it runs on
 * until the process ends; the gauge copy is rebuilt and validated on every
 * call (one stream synchronisation).  A call whose links + clover (+ b and x
 * for canonical io) need more than the array returns TM_ERR_ARG before any
 * device work: at FP32 storage that is V * (480 + 192 nsys) bytes with
 * canonical buffers, V * 480 with internal ones (FP64: twice that; FP16 /
 * BF16: V * (384 + 104 nsys)), so e.g. 16^4 sites with 2 systems at FP32.
 * Every call on a device shares that device's array and leaves its contents
 * there: calls that overlap on one device race.  tm_init sets the array up
 * for the current device; otherwise the first call on a device does.
 */
#define TM_NOALLOC_SCRATCH_BYTES (64ull * 1024ull * 1024ull)
TM_API int tm_sap_smooth_noalloc(const tm_geom* geom, const void* U, const void* b, void* x, double kappa,
                                 double c_sw, const int block_dims[4], int n_cycles, int mr_iters,
                                 const tm_opts* opts);

/* ---------------------------------------------------------------- solves */
#define TM_SOLVE_FLEXIBLE 0          /* FP64 FGMRES, SAP at opts->storage */
#define TM_SOLVE_DEFECT_CORRECTION 1 /* FP64 residual loop around an FP32 FGMRES+SAP solve */

typedef struct tm_mg tm_mg;  /* two-level method, see tm_mg_setup */

typedef struct {
    int form;             /* TM_SOLVE_FLEXIBLE or TM_SOLVE_DEFECT_CORRECTION */
    int restart;          /* FGMRES restart length (outer, or inner for defect correction) */
    int max_iters;        /* cap on Arnoldi steps (per system, summed over restarts) */
    int n_cycles;         /* SAP cycles per preconditioner application */
    int mr_iters;         /* MR steps per block solve */
    int block_dims[4];    /* SAP blocks; zeros = the shape tm_autotune_sap cached for this problem in the
                             file named by the TM_TUNE_CACHE environment variable, or 4^4 when that
                             variable is unset or holds no entry (report->block_dims has the shape used) */
    double inner_tol;     /* defect correction: relative tolerance of each system's inner solve,
                             raised to 0.5 tol ||b_k|| / ||r_k|| (at most 0.5) when that is larger, so
                             no system is solved further than its outer tolerance needs; a system
                             already at tol gets no correction */
    int max_outer;        /* defect correction: cap on outer corrections */
    int group;            /* systems solved together (0 = all nsys) */
    tm_mg* mg;            /* NULL: SAP preconditioner.  Else the two-level method of this handle
                             (tm_mg_setup) preconditions FGMRES: its blocks, post-smoothing and
                             coarse solve replace block_dims, n_cycles and mr_iters; needs
                             opts->storage TM_F32 and geom equal to the handle's but for nsys and mu.
                             The preconditioner uses the handle's own gauge copy and the operator
                             this call's U, kappa and c_sw: a handle set up for other ones still
                             gives solutions to tol (FGMRES admits any preconditioner), only in
                             more iterations */
    int x_in;             /* 1: x holds the starting vector; 0: the solve starts from zero and x is
                             output only (its contents are not read) */
} tm_solver_opts;

/* restart 20, max_iters 2000, 4 cycles, 4 MR steps, 4^4 blocks, flexible form,
 * inner_tol 1e-6, max_outer 50, group 0, no two-level method, x_in 1. */
TM_API void tm_solver_opts_default(tm_solver_opts* sopts);

typedef struct {
    int iters;                          /* Arnoldi steps, max over systems */
    int outer;                          /* defect-correction corrections (0 for flexible form) */
    int converged;                      /* systems whose true residual met tol */
    double true_rel_res[TM_MAX_SYS];    /* ||b - D x|| / ||b|| per system, in FP64 */
    double t_total;                     /* seconds inside the call */
    double t_sap;                       /* seconds in SAP kernels (event-timed) */
    long long sap_cycles;               /* SAP cycles launched (each over a whole group of systems) */
    long long sap_sys_cycles;           /* SAP cycles times the systems they carried */
    int group;                          /* systems solved together (after fitting device memory) */
    int block_dims[4];                  /* Schwarz block shape the smoother used */
    int sys_tile;                       /* SAP systems per workgroup used (0 = all of a group) */
} tm_solve_report;

/*
 * Solves D(mu_k) x_k = b_k for every system to ||b - D x|| <= tol ||b||
 * (true residual in FP64) with flexible GMRES right-preconditioned by SAP
 * (section 2.5: the outer method must be flexible because SAP with MR is not
 * a fixed linear map).  TM_SOLVE_FLEXIBLE keeps the Krylov basis in FP64 and
 * runs SAP at opts->storage; TM_SOLVE_DEFECT_CORRECTION repeats
 * r = b - D x (FP64), an FP32 FGMRES+SAP solve of D c = r to inner_tol, and
 * x += c (the mixed-precision solver of section 3.1).  x is in/out (output
 * only with sopts->x_in 0).  Returns
 * TM_OK when every system converged, TM_NOT_CONVERGED otherwise (report
 * filled; x holds the last iterate).  report may be NULL.
 */
TM_API int tm_fgmres_solve(const tm_geom* geom, const void* U, const void* b, void* x, double kappa, double c_sw,
                    double tol, const tm_solver_opts* sopts, const tm_opts* opts, tm_solve_report* report);

/*
 * CG on the squared even-odd reduced system, the plain FP64 baseline of the
 * paper's solver comparison (section 3): Dhat^+ Dhat x_e = Dhat^+ bhat with
 * Dhat = D_ee - D_eo D_oo^-1 D_oe (eq. (oereduced), even sites kept, parity
 * of t+z+y+x) and bhat = b_e - D_eo D_oo^-1 b_o, run in the least-squares form;
 * then x_o = D_oo^-1 (b_o - D_oe x_e).  The odd rows of b - D x vanish by
 * construction and the even rows are the reduced residual, so CG stops when
 * that (recursively updated) residual is <= tol ||b|| per system; then
 * ||b - D x|| / ||b|| is recomputed with the full operator into
 * report->true_rel_res, and a system counts as converged only when that true
 * residual is <= tol: otherwise CG restarts from it (at most 3 restarts, all
 * within max_iters steps).  FP64 throughout
 * (opts->storage TM_F64), canonical buffers, x in/out (the even-site part of x
 * is the initial guess).  Needs even dims (TM_ERR_DIMS) and at most 8 distinct
 * |mu| per call; systems are solved in groups that fit device memory
 * (report->group).  Returns TM_NOT_CONVERGED when some system's true residual
 * is still above tol (x then holds the last iterate).
 */
TM_API int tm_cg_solve(const tm_geom* geom, const void* U, const void* b, void* x, double kappa, double c_sw,
                       double tol, int max_iters, const tm_opts* opts, tm_solve_report* report);

/* ------------------------------------------------------ internal buffers */
/* Bytes of an internal spinor buffer for geom->nsys systems at opts->storage. */
TM_API size_t tm_spinor_bytes(const tm_geom* geom, const tm_opts* opts);
/* canonical complex128 -> internal (opts->storage, opts->layout_block) */
TM_API int tm_spinor_import(const tm_geom* geom, const void* canon, void* internal, const tm_opts* opts);
/* internal -> canonical complex128 */
TM_API int tm_spinor_export(const tm_geom* geom, const void* internal, void* canon, const tm_opts* opts);
/* As tm_spinor_import / tm_spinor_export for systems first .. first+count-1 of an internal buffer
 * that holds geom->nsys systems; canon holds `count` systems [count][V][4][3].  Lets a caller fill or
 * read a large resident batch one system at a time.  TM_ERR_ARG when the range leaves 0..nsys-1. */
TM_API int tm_spinor_import_range(const tm_geom* geom, const void* canon, void* internal, int first, int count,
                                  const tm_opts* opts);
TM_API int tm_spinor_export_range(const tm_geom* geom, const void* internal, void* canon, int first, int count,
                                  const tm_opts* opts);

/* ------------------------------------------ two-level method (2.3 - 2.6) */
/*
 * Aggregation-based coarse-grid correction with SAP post-smoothing, the
 * multigrid preconditioner of section 2.2 with two levels.  Aggregates are
 * the smoother's Schwarz blocks (section 2.4 fixes them equal) split by spin
 * half, spins {0,1} and {2,3} (section 2.3, "standard aggregation"), so the
 * prolongation commutes with Gamma5 (eq. (gamma5_symmetry)).  On each
 * aggregate the N_v test vectors are orthonormalised (modified Gram-Schmidt
 * in vector order); P is built from them, R = P^+, and the coarse operator is
 * D_c(mu) = P^+ D P + i delta mu Gamma5c (eq. (delta)) where the Galerkin
 * product is taken at mu = 0 with the parity shifts of mu (geom->mu_shift)
 * kept, so that with no shifts D_c(mu) equals P^+ D(mu) P at delta = 1.
 * The coarse lattice has one site per block, index lexicographic in block
 * coordinates (t slowest); a coarse vector is [nsys][nc][2 N_v] complex128
 * with component sg * N_v + i for test vector i on spin half sg (Gamma5c = +1
 * on sg = 0).  The stencil D_c is [nc][9][2 N_v][2 N_v] complex128, row-major
 * per matrix: term 0 couples a site to itself, 1 + mu to the aggregate one
 * step forward along mu (t, x, y, z), 5 + mu one step backward.
 *
 * Preconditioner application (eq. (error_propagation), no pre-smoothing):
 * z = P D_c(mu)^-1 P^+ r with D_c solved by GMRES(coarse_restart) from zero
 * to coarse_tol (relative residual estimate), at most coarse_max_restarts
 * cycles, then post_cycles SAP cycles on D z = r starting from that z.
 *
 * Setup (section 2.6): setup iteration 1 replaces each starting vector v_i by
 * setup_cycles SAP cycles applied to it (v_i as right-hand side, zero guess);
 * iterations 2 .. setup_iters apply the two-level method built from the
 * previous vectors instead.  After every iteration the vectors are
 * orthonormalised over the whole lattice (in order) and P and D_c rebuilt.
 * The twist of the setup is geom->mu[0].
 *
 * Everything runs at FP32 (opts->storage and opts->compute TM_F32); inner
 * products accumulate in FP64.  The handle holds P (N_v FP32 spinor fields),
 * D_c (nc * 9 * (2 N_v)^2 * 8 bytes) and its own FP32 copy of the links and
 * the clover term (480 bytes per site) made at setup, so U may be freed after
 * tm_mg_setup; all of it lives on the device that was current at setup, every
 * call must run with that device current, and calls that use one handle must
 * not overlap.
 */
typedef struct {
    int block_dims[4];       /* aggregates = Schwarz blocks; an even number (>= 2) per direction,
                                at most 1024 sites */
    int n_vec;               /* test vectors N_v, 1 .. 32 */
    int setup_iters;         /* n_setup (0: P from the starting vectors as given) */
    int setup_cycles;        /* SAP cycles per test vector in setup iteration 1 */
    double delta;            /* coarse twist factor */
    double coarse_tol;       /* coarse GMRES target of ||b - D_c x|| / ||b|| (0: run every step) */
    int coarse_restart;      /* 1 .. 128 */
    int coarse_max_restarts; /* >= 1 */
    int post_cycles;         /* SAP post-smoothing cycles (>= 0) */
    int mr_iters;            /* MR steps per block solve */
    int coarse_eo;           /* 1: the coarse GMRES runs on the even-odd reduced coarse system (coarse
                                parity = sum of the aggregate coordinates mod 2), the odd sites'
                                Schur complement, with the even sites recovered from the even-site
                                block inverses; 0: GMRES on the full coarse operator */
} tm_mg_params;

typedef struct {
    int cdims[4];              /* coarse lattice (T, Z, Y, X) */
    int n_vec;
    double t_setup;            /* seconds in tm_mg_setup */
    long long applications;    /* preconditioner applications since setup (systems counted once per call) */
    long long coarse_iters;    /* coarse GMRES steps over those applications (max over systems per call) */
    double t_coarse;           /* seconds in coarse solves (event-timed) */
} tm_mg_info;

/* Table 1 values where a two-level method has them: 4^4 blocks, N_v 28,
 * 5 setup iterations, delta 5.2, coarse GMRES(100) with at most 5 restarts to
 * 1e-1 on the even-odd reduced system, 4 post-smoothing cycles, 3 MR steps;
 * setup_cycles 4 (the paper gives no number for these SAP steps). */
TM_API void tm_mg_params_default(tm_mg_params* p);
/* Builds the two-level method for D(geom->mu[0]) (geom->nsys must be 1).  v0: the
 * N_v starting vectors (the setup's random draws), canonical complex128
 * [N_v][V][4][3] on the device.  *mg receives the handle. */
TM_API int tm_mg_setup(const tm_geom* geom, const void* U, double kappa, double c_sw, const tm_mg_params* params,
                       const void* v0, tm_mg** mg, const tm_opts* opts);
TM_API int tm_mg_destroy(tm_mg* mg);
TM_API int tm_mg_get_info(const tm_mg* mg, tm_mg_info* info);
/* Copies P (canonical complex128 [N_v][V][4][3]: test vector i orthonormalised on
 * every aggregate) and D_c (layout above) to device buffers; either may be NULL. */
TM_API int tm_mg_export(tm_mg* mg, void* P, void* Dc, const tm_opts* opts);
/* c = P^+ r for nsys fine vectors (canonical [nsys][V][4][3]) into coarse vectors. */
TM_API int tm_mg_restrict(tm_mg* mg, int nsys, const void* r, void* c, const tm_opts* opts);
/* e = P c. */
TM_API int tm_mg_prolong(tm_mg* mg, int nsys, const void* c, void* e, const tm_opts* opts);
/* y_k = (D_c + i mu_c[k] Gamma5c) x_k; mu_c a host array [nsys]. */
TM_API int tm_mg_coarse_apply(tm_mg* mg, int nsys, const double* mu_c, const void* x, void* y, const tm_opts* opts);
/* GMRES(restart) for (D_c + i mu_c[k] Gamma5c) x_k = b_k from x = 0, stopping per system
 * when the residual estimate is <= tol ||b_k|| (tol 0: never) or after max_restarts
 * cycles; *iters (may be NULL) gets the largest step count.  With the handle's
 * coarse_eo the GMRES runs on the even-odd reduced system (the estimate is then that
 * of the odd-site residual, which equals the full one) and the even sites follow from
 * the block inverses, which the handle keeps for up to 4 coarse twists until the next
 * setup; more distinct twists in one call are solved in runs of at most 4. */
TM_API int tm_mg_coarse_solve(tm_mg* mg, int nsys, const double* mu_c, const void* b, void* x, double tol,
                              int restart, int max_restarts, int* iters, const tm_opts* opts);
/* z = the two-level preconditioner applied to r, for geom->nsys systems with twists
 * geom->mu (coarse twists delta * mu); canonical fine vectors.  geom must equal the
 * handle's but for nsys and mu. */
TM_API int tm_mg_precond(const tm_geom* geom, tm_mg* mg, const void* r, void* z, const tm_opts* opts);

/* --------------------------------------------------------------- tuning */
/*
 * Times SAP applications (n_cycles cycles of mr_iters MR steps, geom->nsys
 * systems, opts->storage) for candidate Schwarz block shapes (divisors of
 * dims with an even block count per direction, 16..256 sites) and systems-
 * per-workgroup tiles, and returns the fastest in best_block[4] and
 * *best_sys_tile.  The choice is stored in a text cache (path from the
 * TM_TUNE_CACHE environment variable, default ./tm_tune.txt) keyed by
 * (dims, nsys, storage, n_cycles, mr_iters); tm_fgmres_solve with block_dims
 * all zero uses a cached shape only when TM_TUNE_CACHE names the cache (and
 * it holds an entry for the problem), else 4^4.  The objective is
 * smoother throughput only: the block shape also changes the preconditioner,
 * so a tuned shape can converge in a different number of iterations.
 * Allocates its own test vectors; U is read through the gauge cache.
 */
TM_API int tm_autotune_sap(const tm_geom* geom, const void* U, double kappa, double c_sw, int n_cycles, int mr_iters,
                           const tm_opts* opts, int best_block[4], int* best_sys_tile);

/* ----------------------------------------------------------- measurement */
/*
 * Measured FP32 vector arithmetic ceiling of the current device, for roofline
 * statements: a loop of independent FMA chains held in registers, 16
 * workgroups of 256 threads per compute unit, compiled like every kernel of
 * the library (without packed FP32 instructions).  Four launches on
 * opts->stream (the first warms up); *tflops gets the best of the other three
 * in TFLOP/s (an FMA counts 2).  Synchronises the stream; allocates nothing
 * beyond the library's reduction scratch.
 */
TM_API int tm_probe_fp32_fma(double* tflops, const tm_opts* opts);

#ifdef __cplusplus
}
#endif
#endif
