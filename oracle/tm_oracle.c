/*
 * Plain FP64 CPU oracle (see tm_oracle.h for conventions).
 *
 * TEST INFRASTRUCTURE ONLY: never linked into, called by or sharing code with
 * the GPU library.  Loops follow the paper's definitions term by term; there
 * is no blocking, fusion or reordering beyond what the definitions state.
 * OpenMP only splits independent sites / blocks across threads so that the
 * benchmark can time the oracle on the host cores.
 *
 * Pins (checked by the CPU test suite, independent of this code's formulas):
 *   or_gamma        Clifford relation, Hermiticity, gamma5 = diag(1,1,-1,-1).
 *   or_clover       zero on the free field; Hermitian; commutes with gamma5;
 *                   gauge covariant; closed form on a constant abelian
 *                   field strength.
 *   or_dirac        plane-wave closed form on the free field (with and
 *                   without constant abelian phases, with twisted boundary
 *                   phases); twisted boundaries equal periodic ones with the
 *                   phase on the boundary links; parity shifts of mu equal to
 *                   each other reduce to a shifted mu; Gamma5-hermiticity;
 *                   D(mu)^+ D(mu) = D(0)^+ D(0) + mu^2; smallest singular
 *                   value >= |mu|; conjugate spectra of +-mu; gauge
 *                   covariance.
 *   or_dirac_blockdiag  equals the full D with all inter-block link
 *                   products removed (dense check against projector algebra);
 *                   blocks of one colour do not couple.
 *   or_mr_block     residual norms non-increasing; converges to the dense LU
 *                   block solve; optimal step length (perturbing alpha never
 *                   lowers the residual).
 *   or_mr_block_eo  a dense replica (Schur complement of the dense block
 *                   matrix split by site parity, MR in NumPy); converges to
 *                   the dense LU block solve.
 *   or_sap          with exact block solves, the closed form
 *                   x_n = (I - E^n) D^-1 b + E^n x_0, E = (I-B1 D)(I-B0 D);
 *                   residual vanishes on the colour just swept;
 *                   1-homogeneity; block-order independence.
 *   or_dhat         equals the dense Schur complement D_ee - D_eo D_oo^-1 D_oe
 *                   of the dense D split by site parity (numpy); or_dhat_dag
 *                   its conjugate transpose.
 *   or_cg_eo        solution against dense LU; the odd rows of the full
 *                   residual vanish; the reduced residual equals the full one.
 *   or_fgmres       solution against dense LU (numpy); identity-
 *                   preconditioned GMRES(N) exact termination.
 */
#include "tm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NS 4
#define NC 3
#define NSC 12

/* ---------------------------------------------------------------- lattice */

long or_volume(const int dims[4]) {
    return (long)dims[0] * dims[1] * dims[2] * dims[3];
}

/* Array axis of direction mu: t is axis 0, x axis 3, y axis 2, z axis 1. */
static int axis_of(int mu) {
    static const int ax[4] = {0, 3, 2, 1};
    return ax[mu];
}

static void site_coords(const int dims[4], long s, int c[4]) {
    for (int a = 3; a >= 0; --a) {
        c[a] = (int)(s % dims[a]);
        s /= dims[a];
    }
}

static long coords_site(const int dims[4], const int c[4]) {
    long s = 0;
    for (int a = 0; a < 4; ++a) s = s * dims[a] + c[a];
    return s;
}

/* Neighbour of s one step along direction mu (dir = +1 or -1), periodic.
 * *wrapped is set to 1 when the step crosses the lattice boundary. */
static long neighbour(const int dims[4], long s, int mu, int dir, int* wrapped) {
    int c[4];
    site_coords(dims, s, c);
    int a = axis_of(mu);
    int v = c[a] + dir;
    *wrapped = 0;
    if (v < 0) { v += dims[a]; *wrapped = 1; }
    if (v >= dims[a]) { v -= dims[a]; *wrapped = 1; }
    c[a] = v;
    return coords_site(dims, c);
}

static const or_cplx* link(const or_cplx* U, long s, int mu) {
    return U + ((size_t)s * 4 + mu) * 9;
}

/* ------------------------------------------------------------- small algebra */

/* c = a b (3x3) */
static void mm(const or_cplx* a, const or_cplx* b, or_cplx* c) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            or_cplx t = 0;
            for (int k = 0; k < 3; ++k) t += a[3 * i + k] * b[3 * k + j];
            c[3 * i + j] = t;
        }
}

/* c = a^dagger (3x3) */
static void dag(const or_cplx* a, or_cplx* c) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) c[3 * i + j] = conj(a[3 * j + i]);
}

/* product of four 3x3 matrices */
static void mm4(const or_cplx* a, const or_cplx* b, const or_cplx* c, const or_cplx* d, or_cplx* out) {
    or_cplx t1[9], t2[9];
    mm(a, b, t1);
    mm(t1, c, t2);
    mm(t2, d, out);
}

/* -------------------------------------------------------------- gammas */

static void gamma_basic(int mu, or_cplx g[16]) {
    /* Chiral basis: gamma0 = [[0,-1],[-1,0]], gamma_k = [[0,-i sigma_k],[i sigma_k,0]]. */
    const or_cplx ii = _Complex_I;
    or_cplx sig[4][4]; /* sig[k] as 2x2 row-major, k = 1..3 */
    or_cplx s1[4] = {0, 1, 1, 0};
    or_cplx s2[4] = {0, -ii, ii, 0};
    or_cplx s3[4] = {1, 0, 0, -1};
    memcpy(sig[1], s1, sizeof s1);
    memcpy(sig[2], s2, sizeof s2);
    memcpy(sig[3], s3, sizeof s3);
    for (int i = 0; i < 16; ++i) g[i] = 0;
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 2; ++c) {
            or_cplx up, lo; /* upper-right block, lower-left block */
            if (mu == 0) {
                up = (r == c) ? -1.0 : 0.0;
                lo = (r == c) ? -1.0 : 0.0;
            } else {
                up = -ii * sig[mu][2 * r + c];
                lo = ii * sig[mu][2 * r + c];
            }
            g[4 * r + (c + 2)] = up;
            g[4 * (r + 2) + c] = lo;
        }
}

void or_gamma(int mu, or_cplx g[16]) {
    if (mu < 4) {
        gamma_basic(mu, g);
        return;
    }
    /* gamma5 = gamma0 gamma1 gamma2 gamma3, formed by multiplication. */
    or_cplx acc[16], gm[16], tmp[16];
    gamma_basic(0, acc);
    for (int nu = 1; nu < 4; ++nu) {
        gamma_basic(nu, gm);
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) {
                or_cplx t = 0;
                for (int k = 0; k < 4; ++k) t += acc[4 * i + k] * gm[4 * k + j];
                tmp[4 * i + j] = t;
            }
        memcpy(acc, tmp, sizeof acc);
    }
    memcpy(g, acc, sizeof acc);
}

/* -------------------------------------------------------------- clover */

/* Q_munu(x): sum of the four plaquette leaves exactly as the paper writes them. */
static void clover_leaf_sum(const int dims[4], const or_cplx* U, long x, int mu, int nu, or_cplx* Q) {
    int w;
    long xpm = neighbour(dims, x, mu, +1, &w);
    long xpn = neighbour(dims, x, nu, +1, &w);
    long xmm = neighbour(dims, x, mu, -1, &w);
    long xmn = neighbour(dims, x, nu, -1, &w);
    long xmm_pn = neighbour(dims, xmm, nu, +1, &w);
    long xmm_mn = neighbour(dims, xmm, nu, -1, &w);
    long xmn_pm = neighbour(dims, xmn, mu, +1, &w);

    or_cplx d1[9], d2[9], d3[9], leaf[9];
    for (int i = 0; i < 9; ++i) Q[i] = 0;

    /* U_mu(x) U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+ */
    dag(link(U, xpn, mu), d1);
    dag(link(U, x, nu), d2);
    mm4(link(U, x, mu), link(U, xpm, nu), d1, d2, leaf);
    for (int i = 0; i < 9; ++i) Q[i] += leaf[i];

    /* U_nu(x) U_mu(x-mu+nu)^+ U_nu(x-mu)^+ U_mu(x-mu) */
    dag(link(U, xmm_pn, mu), d1);
    dag(link(U, xmm, nu), d2);
    mm4(link(U, x, nu), d1, d2, link(U, xmm, mu), leaf);
    for (int i = 0; i < 9; ++i) Q[i] += leaf[i];

    /* U_mu(x-mu)^+ U_nu(x-mu-nu)^+ U_mu(x-mu-nu) U_nu(x-nu) */
    dag(link(U, xmm, mu), d1);
    dag(link(U, xmm_mn, nu), d2);
    mm4(d1, d2, link(U, xmm_mn, mu), link(U, xmn, nu), leaf);
    for (int i = 0; i < 9; ++i) Q[i] += leaf[i];

    /* U_nu(x-nu)^+ U_mu(x-nu) U_nu(x-nu+mu) U_mu(x)^+ */
    dag(link(U, xmn, nu), d1);
    dag(link(U, x, mu), d3);
    mm4(d1, link(U, xmn, mu), link(U, xmn_pm, nu), d3, leaf);
    for (int i = 0; i < 9; ++i) Q[i] += leaf[i];
}

void or_clover(const int dims[4], const or_cplx* U, double csw, or_cplx* clov) {
    long V = or_volume(dims);
    or_cplx g[4][16];
    for (int mu = 0; mu < 4; ++mu) or_gamma(mu, g[mu]);
#pragma omp parallel for schedule(static)
    for (long x = 0; x < V; ++x) {
        or_cplx* C = clov + (size_t)x * 144;
        for (int i = 0; i < 144; ++i) C[i] = 0;
        for (int mu = 0; mu < 4; ++mu)
            for (int nu = 0; nu < 4; ++nu) {
                or_cplx Qmn[9], Qnm[9], gg[16];
                clover_leaf_sum(dims, U, x, mu, nu, Qmn);
                clover_leaf_sum(dims, U, x, nu, mu, Qnm);
                for (int i = 0; i < 4; ++i)
                    for (int j = 0; j < 4; ++j) {
                        or_cplx t = 0;
                        for (int k = 0; k < 4; ++k) t += g[mu][4 * i + k] * g[nu][4 * k + j];
                        gg[4 * i + j] = t;
                    }
                for (int s = 0; s < 4; ++s)
                    for (int sp = 0; sp < 4; ++sp)
                        for (int c = 0; c < 3; ++c)
                            for (int cp = 0; cp < 3; ++cp)
                                C[(3 * s + c) * 12 + 3 * sp + cp] +=
                                    -(csw / 32.0) * gg[4 * s + sp] * (Qmn[3 * c + cp] - Qnm[3 * c + cp]);
            }
    }
}

/* -------------------------------------------------------------- operator */

/* Boundary phase of a hop along mu that crosses the lattice boundary in the
 * direction dir (+1 forward, -1 backward): exp(i dir theta_mu), times -1 for t
 * when antiperiodic; 1 when the hop does not cross. */
static or_cplx bc_phase(const or_op* op, int mu, int dir, int wrapped) {
    if (!wrapped) return 1.0;
    or_cplx ph = cexp(_Complex_I * (double)dir * op->theta[mu]);
    if (mu == 0 && op->antiperiodic_t) ph = -ph;
    return ph;
}

/* Contribution of one hop: out += -1/2 (I + sgn*gamma_mu) (x) W  psi_n, with
 * sgn = -1 for the forward hop (W = U_mu(x)) and +1 for the backward hop
 * (W = U_mu(x-mu)^+); phase is the boundary phase of the hop. */
static void add_hop(const or_cplx* gmu, double sgn, const or_cplx* W, const or_cplx* psi_n, or_cplx phase,
                    or_cplx* out) {
    for (int s = 0; s < 4; ++s)
        for (int c = 0; c < 3; ++c) {
            or_cplx acc = 0;
            for (int sp = 0; sp < 4; ++sp) {
                or_cplx proj = (s == sp ? 1.0 : 0.0) + sgn * gmu[4 * s + sp];
                if (proj == 0) continue;
                or_cplx col = 0;
                for (int cp = 0; cp < 3; ++cp) col += W[3 * c + cp] * psi_n[3 * sp + cp];
                acc += proj * col;
            }
            out[3 * s + c] += -0.5 * phase * acc;
        }
}

static int site_parity(const int dims[4], long s);

/* Diagonal part at one site: (m+4) psi + clov psi + i mu(x) gamma5 psi with
 * mu(x) = mu + mu_shift[parity of x]. */
static void add_diag(const or_op* op, const or_cplx* g5, long x, const or_cplx* psi, or_cplx* out) {
    const double mux = op->mu + op->mu_shift[site_parity(op->dims, x)];
    for (int i = 0; i < 12; ++i) out[i] += (op->m + 4.0) * psi[i];
    if (op->clov) {
        const or_cplx* C = op->clov + (size_t)x * 144;
        for (int i = 0; i < 12; ++i) {
            or_cplx t = 0;
            for (int j = 0; j < 12; ++j) t += C[12 * i + j] * psi[j];
            out[i] += t;
        }
    }
    for (int s = 0; s < 4; ++s)
        for (int sp = 0; sp < 4; ++sp) {
            if (g5[4 * s + sp] == 0) continue;
            for (int c = 0; c < 3; ++c) out[3 * s + c] += _Complex_I * mux * g5[4 * s + sp] * psi[3 * sp + c];
        }
}

/* Block coordinates of site s. */
static void block_of(const int dims[4], const int bdims[4], long s, int B[4]) {
    int c[4];
    site_coords(dims, s, c);
    for (int a = 0; a < 4; ++a) B[a] = c[a] / bdims[a];
}

static int same_block(const int dims[4], const int bdims[4], long s1, long s2) {
    int B1[4], B2[4];
    block_of(dims, bdims, s1, B1);
    block_of(dims, bdims, s2, B2);
    return B1[0] == B2[0] && B1[1] == B2[1] && B1[2] == B2[2] && B1[3] == B2[3];
}

/* out = D in, restricted to hops allowed by `keep` (NULL bdims: all hops). */
static void dirac_generic(const or_op* op, const int* bdims, const or_cplx* in, or_cplx* out) {
    long V = or_volume(op->dims);
    or_cplx g[4][16], g5[16];
    for (int mu = 0; mu < 4; ++mu) or_gamma(mu, g[mu]);
    or_gamma(4, g5);
#pragma omp parallel for schedule(static)
    for (long x = 0; x < V; ++x) {
        or_cplx acc[12];
        for (int i = 0; i < 12; ++i) acc[i] = 0;
        add_diag(op, g5, x, in + (size_t)x * 12, acc);
        for (int mu = 0; mu < 4; ++mu) {
            int wf, wb;
            long xf = neighbour(op->dims, x, mu, +1, &wf);
            long xb = neighbour(op->dims, x, mu, -1, &wb);
            or_cplx pf = bc_phase(op, mu, +1, wf);
            or_cplx pb = bc_phase(op, mu, -1, wb);
            if (!bdims || same_block(op->dims, bdims, x, xf))
                add_hop(g[mu], -1.0, link(op->U, x, mu), in + (size_t)xf * 12, pf, acc);
            if (!bdims || same_block(op->dims, bdims, x, xb)) {
                or_cplx Wd[9];
                dag(link(op->U, xb, mu), Wd);
                add_hop(g[mu], +1.0, Wd, in + (size_t)xb * 12, pb, acc);
            }
        }
        memcpy(out + (size_t)x * 12, acc, sizeof acc);
    }
}

void or_dirac(const or_op* op, const or_cplx* in, or_cplx* out) {
    dirac_generic(op, NULL, in, out);
}

void or_dirac_blockdiag(const or_op* op, const int bdims[4], const or_cplx* in, or_cplx* out) {
    dirac_generic(op, bdims, in, out);
}

int or_block_colour(const int dims[4], const int bdims[4], long site) {
    int B[4];
    block_of(dims, bdims, site, B);
    return (B[0] + B[1] + B[2] + B[3]) & 1;
}

/* ------------------------------------------------------------ block solves */

/* Sites of block B in local lexicographic order (t slowest). */
static void block_sites(const int dims[4], const int bdims[4], const int B[4], long* sites) {
    long n = 0;
    int c[4];
    for (int a0 = 0; a0 < bdims[0]; ++a0)
        for (int a1 = 0; a1 < bdims[1]; ++a1)
            for (int a2 = 0; a2 < bdims[2]; ++a2)
                for (int a3 = 0; a3 < bdims[3]; ++a3) {
                    c[0] = B[0] * bdims[0] + a0;
                    c[1] = B[1] * bdims[1] + a1;
                    c[2] = B[2] * bdims[2] + a2;
                    c[3] = B[3] * bdims[3] + a3;
                    sites[n++] = coords_site(dims, c);
                }
}

/* Local index of site s in block B, or -1 when s is outside B. */
static long local_index(const int dims[4], const int bdims[4], const int B[4], long s) {
    int c[4];
    site_coords(dims, s, c);
    long l = 0;
    for (int a = 0; a < 4; ++a) {
        int rel = c[a] - B[a] * bdims[a];
        if (rel < 0 || rel >= bdims[a]) return -1;
        l = l * bdims[a] + rel;
    }
    return l;
}

/* out = D_BB in for block-local vectors (Vb x 12): diagonal part plus the hops
 * whose both ends lie in the block. */
static void dirac_block_local(const or_op* op, const int bdims[4], const int B[4], const long* sites, long Vb,
                              const or_cplx* in, or_cplx* out) {
    or_cplx g[4][16], g5[16];
    for (int mu = 0; mu < 4; ++mu) or_gamma(mu, g[mu]);
    or_gamma(4, g5);
    for (long l = 0; l < Vb; ++l) {
        long x = sites[l];
        or_cplx acc[12];
        for (int i = 0; i < 12; ++i) acc[i] = 0;
        add_diag(op, g5, x, in + l * 12, acc);
        for (int mu = 0; mu < 4; ++mu) {
            int wf, wb;
            long xf = neighbour(op->dims, x, mu, +1, &wf);
            long xb = neighbour(op->dims, x, mu, -1, &wb);
            long lf = local_index(op->dims, bdims, B, xf);
            long lb = local_index(op->dims, bdims, B, xb);
            or_cplx pf = bc_phase(op, mu, +1, wf);
            or_cplx pb = bc_phase(op, mu, -1, wb);
            if (lf >= 0) add_hop(g[mu], -1.0, link(op->U, x, mu), in + lf * 12, pf, acc);
            if (lb >= 0) {
                or_cplx Wd[9];
                dag(link(op->U, xb, mu), Wd);
                add_hop(g[mu], +1.0, Wd, in + lb * 12, pb, acc);
            }
        }
        memcpy(out + l * 12, acc, sizeof acc);
    }
}

static or_cplx vdot(const or_cplx* a, const or_cplx* b, long n) {
    or_cplx t = 0;
    for (long i = 0; i < n; ++i) t += conj(a[i]) * b[i];
    return t;
}

/* Minimal residual on one block (Saad): e = 0, rho = r; repeat
 * q = D_BB rho, alpha = <q,rho>/<q,q>, e += alpha rho, rho -= alpha q. */
static void mr_local(const or_op* op, const int bdims[4], const int B[4], const long* sites, long Vb,
                     const or_cplx* r, or_cplx* e, int iters) {
    long n = Vb * 12;
    or_cplx* rho = malloc(sizeof(or_cplx) * n);
    or_cplx* q = malloc(sizeof(or_cplx) * n);
    memcpy(rho, r, sizeof(or_cplx) * n);
    for (long i = 0; i < n; ++i) e[i] = 0;
    for (int k = 0; k < iters; ++k) {
        dirac_block_local(op, bdims, B, sites, Vb, rho, q);
        or_cplx qr = vdot(q, rho, n);
        double qq = creal(vdot(q, q, n));
        if (qq == 0.0) break;
        or_cplx alpha = qr / qq;
        for (long i = 0; i < n; ++i) {
            e[i] += alpha * rho[i];
            rho[i] -= alpha * q[i];
        }
    }
    free(rho);
    free(q);
}

/* Exact solve D_BB e = r by dense Gaussian elimination with partial pivoting. */
static void exact_local(const or_op* op, const int bdims[4], const int B[4], const long* sites, long Vb,
                        const or_cplx* r, or_cplx* e) {
    long n = Vb * 12;
    or_cplx* A = malloc(sizeof(or_cplx) * n * n); /* column j = D_BB e_j, stored row-major A[i*n+j] */
    or_cplx* unit = calloc(n, sizeof(or_cplx));
    or_cplx* col = malloc(sizeof(or_cplx) * n);
    or_cplx* rhs = malloc(sizeof(or_cplx) * n);
    for (long j = 0; j < n; ++j) {
        unit[j] = 1.0;
        dirac_block_local(op, bdims, B, sites, Vb, unit, col);
        unit[j] = 0.0;
        for (long i = 0; i < n; ++i) A[i * n + j] = col[i];
    }
    memcpy(rhs, r, sizeof(or_cplx) * n);
    for (long k = 0; k < n; ++k) {
        long p = k;
        for (long i = k + 1; i < n; ++i)
            if (cabs(A[i * n + k]) > cabs(A[p * n + k])) p = i;
        if (p != k) {
            for (long j = 0; j < n; ++j) {
                or_cplx t = A[k * n + j];
                A[k * n + j] = A[p * n + j];
                A[p * n + j] = t;
            }
            or_cplx t = rhs[k];
            rhs[k] = rhs[p];
            rhs[p] = t;
        }
        for (long i = k + 1; i < n; ++i) {
            or_cplx f = A[i * n + k] / A[k * n + k];
            if (f == 0) continue;
            for (long j = k; j < n; ++j) A[i * n + j] -= f * A[k * n + j];
            rhs[i] -= f * rhs[k];
        }
    }
    for (long i = n - 1; i >= 0; --i) {
        or_cplx t = rhs[i];
        for (long j = i + 1; j < n; ++j) t -= A[i * n + j] * e[j];
        e[i] = t / A[i * n + i];
    }
    free(A);
    free(unit);
    free(col);
    free(rhs);
}

/* ------------------------------------------- even-odd reduced block solves */

/* Site parity (t + z + y + x) mod 2 of the global coordinates: 0 = even. */
static int site_parity(const int dims[4], long s) {
    int c[4];
    site_coords(dims, s, c);
    return (c[0] + c[1] + c[2] + c[3]) & 1;
}

/* out = D_xx^-1 in at one site, D_xx = (m+4) + C(x) + i mu gamma5 the
 * site-diagonal part of D, by Gaussian elimination on its 12x12 matrix. */
static void diag_solve(const or_op* op, const or_cplx* g5, long x, const or_cplx* in, or_cplx* out) {
    or_cplx A[12][12], rhs[12], unit[12], col[12];
    for (int j = 0; j < 12; ++j) {
        for (int i = 0; i < 12; ++i) unit[i] = (i == j) ? 1.0 : 0.0, col[i] = 0;
        add_diag(op, g5, x, unit, col);
        for (int i = 0; i < 12; ++i) A[i][j] = col[i];
    }
    for (int i = 0; i < 12; ++i) rhs[i] = in[i];
    for (int k = 0; k < 12; ++k) {
        int p = k;
        for (int i = k + 1; i < 12; ++i)
            if (cabs(A[i][k]) > cabs(A[p][k])) p = i;
        if (p != k) {
            for (int j = 0; j < 12; ++j) {
                or_cplx t = A[k][j];
                A[k][j] = A[p][j];
                A[p][j] = t;
            }
            or_cplx t = rhs[k];
            rhs[k] = rhs[p];
            rhs[p] = t;
        }
        for (int i = k + 1; i < 12; ++i) {
            or_cplx f = A[i][k] / A[k][k];
            for (int j = k; j < 12; ++j) A[i][j] -= f * A[k][j];
            rhs[i] -= f * rhs[k];
        }
    }
    for (int i = 11; i >= 0; --i) {
        or_cplx t = rhs[i];
        for (int j = i + 1; j < 12; ++j) t -= A[i][j] * out[j];
        out[i] = t / A[i][i];
    }
}

/* Keep the sites of parity `par` of a block-local vector, zero the others. */
static void keep_parity(const int dims[4], const long* sites, long Vb, int par, or_cplx* v) {
    for (long l = 0; l < Vb; ++l)
        if (site_parity(dims, sites[l]) != par)
            for (int i = 0; i < 12; ++i) v[l * 12 + i] = 0;
}

/* D_ee^-1 applied on the even sites of a block-local vector (odd sites zeroed). */
static void diag_solve_even(const or_op* op, const long* sites, long Vb, const or_cplx* in, or_cplx* out) {
    or_cplx g5[16];
    or_gamma(4, g5);
    for (long l = 0; l < Vb; ++l) {
        if (site_parity(op->dims, sites[l]) == 0)
            diag_solve(op, g5, sites[l], in + l * 12, out + l * 12);
        else
            for (int i = 0; i < 12; ++i) out[l * 12 + i] = 0;
    }
}

/* q_o = Dhat rho_o with Dhat = D_oo - D_oe D_ee^-1 D_eo, the block operator
 * reduced to its odd sites (section 2.5).  rho, q: block-local, odd sites
 * only; u, t, v: scratch. */
static void dhat_local(const or_op* op, const int bdims[4], const int B[4], const long* sites, long Vb,
                       const or_cplx* rho, or_cplx* q, or_cplx* u, or_cplx* t, or_cplx* v) {
    long n = Vb * 12;
    dirac_block_local(op, bdims, B, sites, Vb, rho, u); /* u_o = D_oo rho_o, u_e = D_eo rho_o */
    diag_solve_even(op, sites, Vb, u, t);                /* t_e = D_ee^-1 D_eo rho_o */
    dirac_block_local(op, bdims, B, sites, Vb, t, v);   /* v_o = D_oe t_e */
    for (long i = 0; i < n; ++i) q[i] = u[i] - v[i];
    keep_parity(op->dims, sites, Vb, 1, q);
}

/* Block solve with even-odd preconditioning (section 2.5): reduce r to the
 * odd sites, rhat_o = r_o - D_oe D_ee^-1 r_e; run `iters` MR steps on
 * Dhat e_o = rhat_o from e_o = 0; recover e_e = D_ee^-1 (r_e - D_eo e_o). */
static void mr_local_eo(const or_op* op, const int bdims[4], const int B[4], const long* sites, long Vb,
                        const or_cplx* r, or_cplx* e, int iters) {
    long n = Vb * 12;
    or_cplx* rho = malloc(sizeof(or_cplx) * n);
    or_cplx* q = malloc(sizeof(or_cplx) * n);
    or_cplx* u = malloc(sizeof(or_cplx) * n);
    or_cplx* t = malloc(sizeof(or_cplx) * n);
    or_cplx* v = malloc(sizeof(or_cplx) * n);
    /* rhat_o = r_o - D_oe D_ee^-1 r_e */
    diag_solve_even(op, sites, Vb, r, t);
    dirac_block_local(op, bdims, B, sites, Vb, t, v);
    for (long i = 0; i < n; ++i) rho[i] = r[i] - v[i];
    keep_parity(op->dims, sites, Vb, 1, rho);
    /* MR on Dhat over the odd sites */
    for (long i = 0; i < n; ++i) e[i] = 0;
    for (int k = 0; k < iters; ++k) {
        dhat_local(op, bdims, B, sites, Vb, rho, q, u, t, v);
        or_cplx qr = vdot(q, rho, n);
        double qq = creal(vdot(q, q, n));
        if (qq == 0.0) break;
        or_cplx alpha = qr / qq;
        for (long i = 0; i < n; ++i) {
            e[i] += alpha * rho[i];
            rho[i] -= alpha * q[i];
        }
    }
    /* e_e = D_ee^-1 (r_e - D_eo e_o) */
    dirac_block_local(op, bdims, B, sites, Vb, e, u);
    for (long i = 0; i < n; ++i) v[i] = r[i] - u[i];
    diag_solve_even(op, sites, Vb, v, t);
    for (long l = 0; l < Vb; ++l)
        if (site_parity(op->dims, sites[l]) == 0)
            for (int i = 0; i < 12; ++i) e[l * 12 + i] = t[l * 12 + i];
    free(rho);
    free(q);
    free(u);
    free(t);
    free(v);
}

void or_mr_block_eo(const or_op* op, const int bdims[4], const int B[4], const or_cplx* r, or_cplx* e, int iters) {
    long Vb = (long)bdims[0] * bdims[1] * bdims[2] * bdims[3];
    long* sites = malloc(sizeof(long) * Vb);
    or_cplx* rl = malloc(sizeof(or_cplx) * Vb * 12);
    or_cplx* el = malloc(sizeof(or_cplx) * Vb * 12);
    block_sites(op->dims, bdims, B, sites);
    for (long l = 0; l < Vb; ++l) memcpy(rl + l * 12, r + (size_t)sites[l] * 12, sizeof(or_cplx) * 12);
    mr_local_eo(op, bdims, B, sites, Vb, rl, el, iters);
    for (long l = 0; l < Vb; ++l) memcpy(e + (size_t)sites[l] * 12, el + l * 12, sizeof(or_cplx) * 12);
    free(sites);
    free(rl);
    free(el);
}

void or_mr_block(const or_op* op, const int bdims[4], const int B[4], const or_cplx* r, or_cplx* e, int iters) {
    long Vb = (long)bdims[0] * bdims[1] * bdims[2] * bdims[3];
    long* sites = malloc(sizeof(long) * Vb);
    or_cplx* rl = malloc(sizeof(or_cplx) * Vb * 12);
    or_cplx* el = malloc(sizeof(or_cplx) * Vb * 12);
    block_sites(op->dims, bdims, B, sites);
    for (long l = 0; l < Vb; ++l) memcpy(rl + l * 12, r + (size_t)sites[l] * 12, sizeof(or_cplx) * 12);
    mr_local(op, bdims, B, sites, Vb, rl, el, iters);
    for (long l = 0; l < Vb; ++l) memcpy(e + (size_t)sites[l] * 12, el + l * 12, sizeof(or_cplx) * 12);
    free(sites);
    free(rl);
    free(el);
}

/* ------------------------------------------------------------------- SAP */

int or_sap(const or_op* op, const int bdims[4], int n_cycles, int mr_iters, const or_cplx* b, or_cplx* x) {
    return or_sap_eo(op, bdims, n_cycles, mr_iters, 0, b, x);
}

int or_sap_eo(const or_op* op, const int bdims[4], int n_cycles, int mr_iters, int eo, const or_cplx* b,
              or_cplx* x) {
    int nb[4];
    for (int a = 0; a < 4; ++a) {
        if (bdims[a] <= 0 || op->dims[a] % bdims[a] != 0) return -2;
        nb[a] = op->dims[a] / bdims[a];
        if (nb[a] % 2 != 0) return -3;
    }
    long V = or_volume(op->dims);
    long Vb = (long)bdims[0] * bdims[1] * bdims[2] * bdims[3];
    long nblocks = (long)nb[0] * nb[1] * nb[2] * nb[3];
    or_cplx* r = malloc(sizeof(or_cplx) * V * 12);

    for (int cyc = 0; cyc < n_cycles; ++cyc) {
        for (int colour = 0; colour < 2; ++colour) {
            /* residual r = b - D x on the whole lattice */
            or_dirac(op, x, r);
            for (long i = 0; i < V * 12; ++i) r[i] = b[i] - r[i];
            /* every block of this colour: e_B ~ D_BB^-1 r_B, x_B += e_B */
#pragma omp parallel for schedule(dynamic)
            for (long bi = 0; bi < nblocks; ++bi) {
                int B[4];
                long t = bi;
                for (int a = 3; a >= 0; --a) {
                    B[a] = (int)(t % nb[a]);
                    t /= nb[a];
                }
                if (((B[0] + B[1] + B[2] + B[3]) & 1) != colour) continue;
                long* sites = malloc(sizeof(long) * Vb);
                or_cplx* rl = malloc(sizeof(or_cplx) * Vb * 12);
                or_cplx* el = malloc(sizeof(or_cplx) * Vb * 12);
                block_sites(op->dims, bdims, B, sites);
                for (long l = 0; l < Vb; ++l) memcpy(rl + l * 12, r + (size_t)sites[l] * 12, sizeof(or_cplx) * 12);
                if (mr_iters >= 0 && eo)
                    mr_local_eo(op, bdims, B, sites, Vb, rl, el, mr_iters);
                else if (mr_iters >= 0)
                    mr_local(op, bdims, B, sites, Vb, rl, el, mr_iters);
                else
                    exact_local(op, bdims, B, sites, Vb, rl, el);
                for (long l = 0; l < Vb; ++l)
                    for (int i = 0; i < 12; ++i) x[(size_t)sites[l] * 12 + i] += el[l * 12 + i];
                free(sites);
                free(rl);
                free(el);
            }
        }
    }
    free(r);
    return 0;
}

/* ------------------------------------------- even-odd reduced operator, CG */

static double vnorm(const or_cplx* a, long n);
static double true_residual(const or_op* op, const or_cplx* b, const or_cplx* x, or_cplx* r, long n);

/* Zero the sites whose parity differs from par. */
static void mask_parity(const int dims[4], int par, or_cplx* v) {
    long V = or_volume(dims);
    for (long x = 0; x < V; ++x)
        if (site_parity(dims, x) != par)
            for (int i = 0; i < 12; ++i) v[x * 12 + i] = 0;
}

/* out = D_pp^-1 in on the sites of parity par (site-diagonal part of D), zero elsewhere. */
static void diag_solve_parity(const or_op* op, int par, const or_cplx* in, or_cplx* out) {
    long V = or_volume(op->dims);
    or_cplx g5[16];
    or_gamma(4, g5);
#pragma omp parallel for schedule(static)
    for (long x = 0; x < V; ++x) {
        if (site_parity(op->dims, x) == par)
            diag_solve(op, g5, x, in + x * 12, out + x * 12);
        else
            for (int i = 0; i < 12; ++i) out[x * 12 + i] = 0;
    }
}

void or_dhat(const or_op* op, const or_cplx* in, or_cplx* out) {
    long n = or_volume(op->dims) * 12;
    or_cplx* v = malloc(sizeof(or_cplx) * n);
    or_cplx* u = malloc(sizeof(or_cplx) * n);
    or_cplx* t = malloc(sizeof(or_cplx) * n);
    or_cplx* w = malloc(sizeof(or_cplx) * n);
    memcpy(v, in, sizeof(or_cplx) * n);
    mask_parity(op->dims, 0, v);
    or_dirac(op, v, u);                    /* u_e = D_ee v_e, u_o = D_oe v_e */
    diag_solve_parity(op, 1, u, t);        /* t_o = D_oo^-1 D_oe v_e */
    or_dirac(op, t, w);                    /* w_e = D_eo t_o */
    for (long i = 0; i < n; ++i) out[i] = u[i] - w[i];
    mask_parity(op->dims, 0, out);
    free(v);
    free(u);
    free(t);
    free(w);
}

void or_dhat_dag(const or_op* op, const or_cplx* in, or_cplx* out) {
    /* Dhat(mu)^+ = Gamma5 Dhat(-mu) Gamma5, from D(mu)^+ = Gamma5 D(-mu) Gamma5 (section 2.1)
     * and Gamma5 being site-diagonal */
    long n = or_volume(op->dims) * 12;
    or_cplx* v = malloc(sizeof(or_cplx) * n);
    or_cplx g5[16];
    or_gamma(4, g5);
    for (long x = 0; x < n / 12; ++x)
        for (int s = 0; s < 4; ++s)
            for (int c = 0; c < 3; ++c) v[x * 12 + 3 * s + c] = g5[5 * s] * in[x * 12 + 3 * s + c];
    or_op neg = *op;
    neg.mu = -op->mu;
    neg.mu_shift[0] = -op->mu_shift[0];
    neg.mu_shift[1] = -op->mu_shift[1];
    or_dhat(&neg, v, out);
    for (long x = 0; x < n / 12; ++x)
        for (int s = 0; s < 4; ++s)
            for (int c = 0; c < 3; ++c) out[x * 12 + 3 * s + c] *= g5[5 * s];
    free(v);
}

int or_cg_eo(const or_op* op, const or_cplx* b, or_cplx* x, double tol, int max_iters, or_report* rep) {
    long n = or_volume(op->dims) * 12;
    or_cplx* bh = malloc(sizeof(or_cplx) * n);
    or_cplx* r = malloc(sizeof(or_cplx) * n);
    or_cplx* s = malloc(sizeof(or_cplx) * n);
    or_cplx* p = malloc(sizeof(or_cplx) * n);
    or_cplx* q = malloc(sizeof(or_cplx) * n);
    or_cplx* t = malloc(sizeof(or_cplx) * n);
    double bnorm = vnorm(b, n);
    int iters = 0;
    /* reduced right-hand side bhat_e = b_e - D_eo D_oo^-1 b_o */
    diag_solve_parity(op, 1, b, t);
    or_dirac(op, t, q);
    for (long i = 0; i < n; ++i) bh[i] = b[i] - q[i];
    mask_parity(op->dims, 0, bh);
    /* CG on Dhat^+ Dhat x_e = Dhat^+ bhat (in the least-squares form: r is the residual of the
     * reduced system, s = Dhat^+ r the residual of the normal equations) */
    mask_parity(op->dims, 0, x);
    or_dhat(op, x, q);
    for (long i = 0; i < n; ++i) r[i] = bh[i] - q[i];
    or_dhat_dag(op, r, s);
    memcpy(p, s, sizeof(or_cplx) * n);
    double gamma = vnorm(s, n);
    gamma *= gamma;
    while (vnorm(r, n) > tol * bnorm && iters < max_iters && gamma > 0) {
        or_dhat(op, p, q);
        double qq = vnorm(q, n);
        double alpha = gamma / (qq * qq);
        for (long i = 0; i < n; ++i) {
            x[i] += alpha * p[i];
            r[i] -= alpha * q[i];
        }
        or_dhat_dag(op, r, s);
        double gnew = vnorm(s, n);
        gnew *= gnew;
        double beta = gnew / gamma;
        for (long i = 0; i < n; ++i) p[i] = s[i] + beta * p[i];
        gamma = gnew;
        ++iters;
    }
    /* odd sites: x_o = D_oo^-1 (b_o - D_oe x_e) */
    or_dirac(op, x, q);
    for (long i = 0; i < n; ++i) t[i] = b[i] - q[i];
    diag_solve_parity(op, 1, t, q);
    for (long xs = 0; xs < n / 12; ++xs)
        if (site_parity(op->dims, xs) == 1)
            for (int i = 0; i < 12; ++i) x[xs * 12 + i] = q[xs * 12 + i];
    double rel = bnorm > 0 ? true_residual(op, b, x, t, n) / bnorm : 0.0;
    if (rep) {
        rep->iters = iters;
        rep->restarts = 0;
        rep->converged = rel <= tol;
        rep->true_rel_res = rel;
    }
    free(bh);
    free(r);
    free(s);
    free(p);
    free(q);
    free(t);
    return rel <= tol ? 0 : 1;
}

/* ---------------------------------------------------------------- FGMRES */

static double vnorm(const or_cplx* a, long n) {
    double t = 0;
    for (long i = 0; i < n; ++i) t += creal(a[i]) * creal(a[i]) + cimag(a[i]) * cimag(a[i]);
    return sqrt(t);
}

static double true_residual(const or_op* op, const or_cplx* b, const or_cplx* x, or_cplx* r, long n) {
    or_dirac(op, x, r);
    for (long i = 0; i < n; ++i) r[i] = b[i] - r[i];
    return vnorm(r, n);
}

int or_fgmres(const or_op* op, const or_cplx* b, or_cplx* x, double tol, int restart, int max_iters, int precond,
              const int bdims[4], int n_cycles, int mr_iters, or_report* rep) {
    return or_fgmres_eo(op, b, x, tol, restart, max_iters, precond, bdims, n_cycles, mr_iters, 0, rep);
}

/* Right preconditioner of FGMRES: z = M v (z is overwritten). */
typedef void (*or_precond_fn)(const void* ctx, const or_cplx* v, or_cplx* z);

typedef struct {
    const or_op* op;
    const int* bdims;
    int n_cycles, mr_iters, eo;
} sap_ctx;

/* SAP from a zero guess. */
static void sap_precond(const void* ctx, const or_cplx* v, or_cplx* z) {
    const sap_ctx* c = (const sap_ctx*)ctx;
    long n = or_volume(c->op->dims) * 12;
    for (long i = 0; i < n; ++i) z[i] = 0;
    or_sap_eo(c->op, c->bdims, c->n_cycles, c->mr_iters, c->eo, v, z);
}

static int fgmres_core(const or_op* op, const or_cplx* b, or_cplx* x, double tol, int restart, int max_iters,
                       or_precond_fn prec, const void* pctx, or_report* rep);

int or_fgmres_eo(const or_op* op, const or_cplx* b, or_cplx* x, double tol, int restart, int max_iters,
                 int precond, const int bdims[4], int n_cycles, int mr_iters, int eo, or_report* rep) {
    sap_ctx c = {op, bdims, n_cycles, mr_iters, eo};
    return fgmres_core(op, b, x, tol, restart, max_iters, precond ? sap_precond : NULL, &c, rep);
}

/* Flexible GMRES(restart): right preconditioning by prec (NULL: none), modified
 * Gram-Schmidt, complex Givens rotations; stops on the true residual. */
static int fgmres_core(const or_op* op, const or_cplx* b, or_cplx* x, double tol, int restart, int max_iters,
                       or_precond_fn prec, const void* pctx, or_report* rep) {
    long n = or_volume(op->dims) * 12;
    int m = restart;
    or_cplx* Vv = malloc(sizeof(or_cplx) * n * (m + 1));
    or_cplx* Z = malloc(sizeof(or_cplx) * n * m);
    or_cplx* w = malloc(sizeof(or_cplx) * n);
    or_cplx* r = malloc(sizeof(or_cplx) * n);
    or_cplx* H = calloc((size_t)(m + 1) * m, sizeof(or_cplx)); /* H[i*m + j] */
    double* cs = malloc(sizeof(double) * m);
    or_cplx* sn = malloc(sizeof(or_cplx) * m);
    or_cplx* g = malloc(sizeof(or_cplx) * (m + 1));
    or_cplx* y = malloc(sizeof(or_cplx) * m);

    double bnorm = vnorm(b, n);
    int iters = 0, restarts = 0, converged = 0;
    double rel = 0.0;
    if (bnorm == 0.0) {
        for (long i = 0; i < n; ++i) x[i] = 0;
        converged = 1;
        goto done;
    }
    rel = true_residual(op, b, x, r, n) / bnorm;
    while (rel > tol && iters < max_iters) {
        double beta = vnorm(r, n);
        for (long i = 0; i < n; ++i) Vv[i] = r[i] / beta;
        for (int i = 0; i <= m; ++i) g[i] = 0;
        g[0] = beta;
        int j_done = 0;
        for (int j = 0; j < m && iters < max_iters; ++j) {
            or_cplx* vj = Vv + (size_t)j * n;
            or_cplx* zj = Z + (size_t)j * n;
            /* z_j = M v_j */
            if (prec) {
                prec(pctx, vj, zj);
            } else {
                memcpy(zj, vj, sizeof(or_cplx) * n);
            }
            /* w = D z_j, then modified Gram-Schmidt */
            or_dirac(op, zj, w);
            for (int i = 0; i <= j; ++i) {
                or_cplx h = vdot(Vv + (size_t)i * n, w, n);
                H[i * m + j] = h;
                for (long k = 0; k < n; ++k) w[k] -= h * Vv[(size_t)i * n + k];
            }
            double hn = vnorm(w, n);
            H[(j + 1) * m + j] = hn;
            if (hn > 0)
                for (long k = 0; k < n; ++k) Vv[(size_t)(j + 1) * n + k] = w[k] / hn;
            /* apply earlier rotations to the new column */
            for (int i = 0; i < j; ++i) {
                or_cplx a = H[i * m + j], c2 = H[(i + 1) * m + j];
                H[i * m + j] = cs[i] * a + sn[i] * c2;
                H[(i + 1) * m + j] = -conj(sn[i]) * a + cs[i] * c2;
            }
            /* new rotation zeroing H[j+1][j] */
            or_cplx a = H[j * m + j], c2 = H[(j + 1) * m + j];
            double t = sqrt(creal(a) * creal(a) + cimag(a) * cimag(a) + creal(c2) * creal(c2) + cimag(c2) * cimag(c2));
            if (cabs(a) == 0.0) {
                cs[j] = 0.0;
                sn[j] = 1.0;
            } else {
                cs[j] = cabs(a) / t;
                sn[j] = (a / cabs(a)) * conj(c2) / t;
            }
            H[j * m + j] = cs[j] * a + sn[j] * c2;
            H[(j + 1) * m + j] = 0;
            g[j + 1] = -conj(sn[j]) * g[j];
            g[j] = cs[j] * g[j];
            ++iters;
            j_done = j + 1;
            if (cabs(g[j + 1]) / bnorm <= tol || hn == 0.0) break;
        }
        /* y = H^-1 g (upper triangular), x += Z y */
        for (int i = j_done - 1; i >= 0; --i) {
            or_cplx t2 = g[i];
            for (int k = i + 1; k < j_done; ++k) t2 -= H[i * m + k] * y[k];
            y[i] = t2 / H[i * m + i];
        }
        for (int k = 0; k < j_done; ++k)
            for (long i = 0; i < n; ++i) x[i] += y[k] * Z[(size_t)k * n + i];
        ++restarts;
        rel = true_residual(op, b, x, r, n) / bnorm;
    }
    converged = rel <= tol;
done:
    if (rep) {
        rep->iters = iters;
        rep->restarts = restarts;
        rep->converged = converged;
        rep->true_rel_res = rel;
    }
    free(Vv);
    free(Z);
    free(w);
    free(r);
    free(H);
    free(cs);
    free(sn);
    free(g);
    free(y);
    return converged ? 0 : 1;
}

/* ------------------------------------------------- two-level method (2.3, 2.4) */

/* Coarse lattice: one site per aggregate block; coarse index lexicographic in
 * the block coordinates (t slowest), like the fine sites. */
static void mg_cdims(const int dims[4], const int adims[4], int cd[4]) {
    for (int a = 0; a < 4; ++a) cd[a] = dims[a] / adims[a];
}

static long mg_coarse_of_site(const int dims[4], const int adims[4], long s) {
    int c[4], cd[4];
    site_coords(dims, s, c);
    mg_cdims(dims, adims, cd);
    long j = 0;
    for (int a = 0; a < 4; ++a) j = j * cd[a] + c[a] / adims[a];
    return j;
}

/* Coarse site coupled through stencil term t: 0 = j itself, 1 + mu = the
 * aggregate one step forward along mu, 5 + mu = one step backward. */
static long mg_coarse_nbr(const int cd[4], long j, int t) {
    int J[4];
    site_coords(cd, j, J);
    if (t >= 1) {
        int mu = (t - 1) % 4, dir = t <= 4 ? +1 : -1, a = axis_of(mu);
        J[a] = (J[a] + dir + cd[a]) % cd[a];
    }
    return coords_site(cd, J);
}

/* <a, b> over the sites of one aggregate, spin half sg (spins 2sg, 2sg+1). */
static or_cplx agg_dot(const or_cplx* a, const or_cplx* b, const long* sites, long Vb, int sg) {
    or_cplx t = 0;
    for (long l = 0; l < Vb; ++l)
        for (int k = 6 * sg; k < 6 * sg + 6; ++k) t += conj(a[(size_t)sites[l] * 12 + k]) * b[(size_t)sites[l] * 12 + k];
    return t;
}

/* Aggregate-wise orthonormalisation of the test vectors (section 2.3): on every
 * aggregate A_{j,+-} = block j x spins {0,1} or {2,3} x colour, modified
 * Gram-Schmidt over i = 0 .. nv-1.  Column (j, sg, i) of P is P_i restricted
 * to A_{j,sg}, so Gamma5 P = P Gamma5c holds by construction. */
void or_mg_block_orthonormalize(const int dims[4], const int adims[4], int nv, const or_cplx* v, or_cplx* P) {
    long V = or_volume(dims), Vb = or_volume(adims), nc = V / Vb;
    int cd[4];
    mg_cdims(dims, adims, cd);
    memcpy(P, v, sizeof(or_cplx) * (size_t)nv * V * 12);
#pragma omp parallel for schedule(dynamic)
    for (long j = 0; j < nc; ++j) {
        int J[4];
        site_coords(cd, j, J);
        long* sites = malloc(sizeof(long) * Vb);
        block_sites(dims, adims, J, sites);
        for (int sg = 0; sg < 2; ++sg)
            for (int i = 0; i < nv; ++i) {
                or_cplx* Pi = P + (size_t)i * V * 12;
                for (int k = 0; k < i; ++k) {
                    const or_cplx* Pk = P + (size_t)k * V * 12;
                    or_cplx h = agg_dot(Pk, Pi, sites, Vb, sg);
                    for (long l = 0; l < Vb; ++l)
                        for (int q = 6 * sg; q < 6 * sg + 6; ++q) Pi[(size_t)sites[l] * 12 + q] -= h * Pk[(size_t)sites[l] * 12 + q];
                }
                double nrm = sqrt(creal(agg_dot(Pi, Pi, sites, Vb, sg)));
                if (nrm > 0)
                    for (long l = 0; l < Vb; ++l)
                        for (int q = 6 * sg; q < 6 * sg + 6; ++q) Pi[(size_t)sites[l] * 12 + q] /= nrm;
            }
        free(sites);
    }
}

/* c = P^+ r: c[j][sg*nv + i] = <P_i on A_{j,sg}, r>. */
void or_mg_restrict(const int dims[4], const int adims[4], int nv, const or_cplx* P, const or_cplx* r, or_cplx* c) {
    long V = or_volume(dims), Vb = or_volume(adims), nc = V / Vb;
    int cd[4];
    mg_cdims(dims, adims, cd);
#pragma omp parallel for schedule(static)
    for (long j = 0; j < nc; ++j) {
        int J[4];
        site_coords(cd, j, J);
        long* sites = malloc(sizeof(long) * Vb);
        block_sites(dims, adims, J, sites);
        for (int sg = 0; sg < 2; ++sg)
            for (int i = 0; i < nv; ++i) c[(size_t)j * 2 * nv + sg * nv + i] = agg_dot(P + (size_t)i * V * 12, r, sites, Vb, sg);
        free(sites);
    }
}

/* e = P c: e(x, s, col) = sum_i P_i(x, s, col) c[j(x)][sg(s)*nv + i]. */
void or_mg_prolong(const int dims[4], const int adims[4], int nv, const or_cplx* P, const or_cplx* c, or_cplx* e) {
    long V = or_volume(dims);
#pragma omp parallel for schedule(static)
    for (long x = 0; x < V; ++x) {
        long j = mg_coarse_of_site(dims, adims, x);
        for (int q = 0; q < 12; ++q) {
            int sg = q / 6;
            or_cplx t = 0;
            for (int i = 0; i < nv; ++i) t += P[((size_t)i * V + x) * 12 + q] * c[(size_t)j * 2 * nv + sg * nv + i];
            e[(size_t)x * 12 + q] = t;
        }
    }
}

/* Coarse basis vector (src, b) at fine site y: P_i on A_{src,sg} (b = sg*nv + i), zero elsewhere. */
static void mg_basis_at(const int dims[4], const int adims[4], int nv, const or_cplx* P, long src, int b, long y,
                        or_cplx out[12]) {
    for (int q = 0; q < 12; ++q) out[q] = 0;
    if (mg_coarse_of_site(dims, adims, y) != src) return;
    long V = or_volume(dims);
    int sg = b / nv, i = b % nv;
    for (int q = 6 * sg; q < 6 * sg + 6; ++q) out[q] = P[((size_t)i * V + y) * 12 + q];
}

/* One term of D at fine site x applied to the basis vector (src, b):
 * t = 0: the block-diagonal part D_BB (diagonal and the hops inside x's aggregate);
 * t = 1 + mu: the forward hop along mu when it leaves the aggregate;
 * t = 5 + mu: the backward hop along mu when it leaves the aggregate. */
static void mg_term_at(const or_op* op, const int adims[4], int nv, const or_cplx* P, int t, long src, int b, long x,
                       or_cplx out[12]) {
    or_cplx g[4][16], g5[16], e[12];
    for (int mu = 0; mu < 4; ++mu) or_gamma(mu, g[mu]);
    or_gamma(4, g5);
    for (int q = 0; q < 12; ++q) out[q] = 0;
    if (t == 0) {
        mg_basis_at(op->dims, adims, nv, P, src, b, x, e);
        add_diag(op, g5, x, e, out);
    }
    for (int mu = 0; mu < 4; ++mu) {
        int wf, wb;
        long xf = neighbour(op->dims, x, mu, +1, &wf);
        long xb = neighbour(op->dims, x, mu, -1, &wb);
        int inf = same_block(op->dims, adims, x, xf), inb = same_block(op->dims, adims, x, xb);
        if ((t == 0 && inf) || (t == 1 + mu && !inf)) {
            mg_basis_at(op->dims, adims, nv, P, src, b, xf, e);
            add_hop(g[mu], -1.0, link(op->U, x, mu), e, bc_phase(op, mu, +1, wf), out);
        }
        if ((t == 0 && inb) || (t == 5 + mu && !inb)) {
            or_cplx Wd[9];
            dag(link(op->U, xb, mu), Wd);
            mg_basis_at(op->dims, adims, nv, P, src, b, xb, e);
            add_hop(g[mu], +1.0, Wd, e, bc_phase(op, mu, -1, wb), out);
        }
    }
}

/* Coarse stencil of the Galerkin operator P^+ D P (section 2.3) without the
 * twist: Dc[j][t][a][b] = < column (j, a), D_t column (nbr_t(j), b) > with D_t
 * the term of mg_term_at, computed at op with mu = 0 (its mu_shift stays: a
 * site-dependent twist enters through the Galerkin product).  The coarse
 * operator is then D_c(mu, delta) = Dc + i delta mu Gamma5c. */
void or_mg_coarse_build(const or_op* op, const int adims[4], int nv, const or_cplx* P, or_cplx* Dc) {
    or_op op0 = *op;
    op0.mu = 0.0;
    long V = or_volume(op->dims), Vb = or_volume(adims), nc = V / Vb;
    int cd[4], n2 = 2 * nv;
    mg_cdims(op->dims, adims, cd);
#pragma omp parallel for schedule(dynamic)
    for (long j = 0; j < nc; ++j) {
        int J[4];
        site_coords(cd, j, J);
        long* sites = malloc(sizeof(long) * Vb);
        or_cplx* w = malloc(sizeof(or_cplx) * Vb * 12);
        block_sites(op->dims, adims, J, sites);
        for (int t = 0; t < 9; ++t) {
            long src = mg_coarse_nbr(cd, j, t);
            for (int b = 0; b < n2; ++b) {
                for (long l = 0; l < Vb; ++l) mg_term_at(&op0, adims, nv, P, t, src, b, sites[l], w + l * 12);
                for (int a = 0; a < n2; ++a) {
                    int sg = a / nv, i = a % nv;
                    or_cplx acc = 0;
                    for (long l = 0; l < Vb; ++l)
                        for (int q = 6 * sg; q < 6 * sg + 6; ++q)
                            acc += conj(P[((size_t)i * V + sites[l]) * 12 + q]) * w[l * 12 + q];
                    Dc[(((size_t)j * 9 + t) * n2 + a) * n2 + b] = acc;
                }
            }
        }
        free(sites);
        free(w);
    }
}

/* y = (Dc + i mu_c Gamma5c) x on the coarse lattice, Gamma5c = +1 on the first
 * nv components of a coarse site and -1 on the other nv. */
void or_mg_coarse_apply(const int cdims[4], int nv, const or_cplx* Dc, double mu_c, const or_cplx* x, or_cplx* y) {
    long nc = or_volume(cdims);
    int n2 = 2 * nv;
#pragma omp parallel for schedule(static)
    for (long j = 0; j < nc; ++j) {
        for (int a = 0; a < n2; ++a) {
            or_cplx acc = _Complex_I * mu_c * (a < nv ? 1.0 : -1.0) * x[(size_t)j * n2 + a];
            for (int t = 0; t < 9; ++t) {
                long src = mg_coarse_nbr(cdims, j, t);
                const or_cplx* M = Dc + (((size_t)j * 9 + t) * n2 + a) * n2;
                for (int b = 0; b < n2; ++b) acc += M[b] * x[(size_t)src * n2 + b];
            }
            y[(size_t)j * n2 + a] = acc;
        }
    }
}

typedef void (*or_apply_fn)(const void* ctx, const or_cplx* in, or_cplx* out);

/* GMRES(restart) for A x = b from x = 0, modified Gram-Schmidt and Givens
 * rotations.  Stops when the residual estimate |g_{j+1}| <= tol * bref
 * (tol <= 0: never) or after max_restarts cycles; each cycle restarts from
 * the recomputed residual.  Returns 0 when the estimate met tol. */
static int gmres_op(long n, or_apply_fn A, const void* actx, const or_cplx* b, or_cplx* x, double tol, double bref,
                    int restart, int max_restarts, or_report* rep) {
    int m = restart;
    or_cplx* Vv = malloc(sizeof(or_cplx) * n * (m + 1));
    or_cplx* w = malloc(sizeof(or_cplx) * n);
    or_cplx* H = calloc((size_t)(m + 1) * m, sizeof(or_cplx));
    double* cs = malloc(sizeof(double) * m);
    or_cplx* sn = malloc(sizeof(or_cplx) * m);
    or_cplx* g = malloc(sizeof(or_cplx) * (m + 1));
    or_cplx* y = malloc(sizeof(or_cplx) * m);
    for (long i = 0; i < n; ++i) x[i] = 0;
    double bnorm = bref, est = vnorm(b, n);
    int iters = 0, cycles = 0, met = est == 0.0;
    while (!met && cycles < max_restarts) {
        /* r = b - A x */
        A(actx, x, w);
        for (long i = 0; i < n; ++i) w[i] = b[i] - w[i];
        double beta = vnorm(w, n);
        est = beta;
        if (beta == 0.0 || (tol > 0 && beta <= tol * bnorm)) {
            met = 1;
            break;
        }
        for (long i = 0; i < n; ++i) Vv[i] = w[i] / beta;
        for (int i = 0; i <= m; ++i) g[i] = 0;
        g[0] = beta;
        int jd = 0;
        for (int j = 0; j < m; ++j) {
            A(actx, Vv + (size_t)j * n, w);
            for (int i = 0; i <= j; ++i) {
                or_cplx h = vdot(Vv + (size_t)i * n, w, n);
                H[i * m + j] = h;
                for (long k = 0; k < n; ++k) w[k] -= h * Vv[(size_t)i * n + k];
            }
            double hn = vnorm(w, n);
            H[(j + 1) * m + j] = hn;
            if (hn > 0)
                for (long k = 0; k < n; ++k) Vv[(size_t)(j + 1) * n + k] = w[k] / hn;
            for (int i = 0; i < j; ++i) {
                or_cplx a = H[i * m + j], c2 = H[(i + 1) * m + j];
                H[i * m + j] = cs[i] * a + sn[i] * c2;
                H[(i + 1) * m + j] = -conj(sn[i]) * a + cs[i] * c2;
            }
            or_cplx a = H[j * m + j], c2 = H[(j + 1) * m + j];
            double tt = sqrt(creal(a) * creal(a) + cimag(a) * cimag(a) + creal(c2) * creal(c2) + cimag(c2) * cimag(c2));
            if (cabs(a) == 0.0) {
                cs[j] = 0.0;
                sn[j] = 1.0;
            } else {
                cs[j] = cabs(a) / tt;
                sn[j] = (a / cabs(a)) * conj(c2) / tt;
            }
            H[j * m + j] = cs[j] * a + sn[j] * c2;
            H[(j + 1) * m + j] = 0;
            g[j + 1] = -conj(sn[j]) * g[j];
            g[j] = cs[j] * g[j];
            ++iters;
            jd = j + 1;
            est = cabs(g[j + 1]);
            if ((tol > 0 && est <= tol * bnorm) || hn == 0.0) {
                met = tol > 0 && est <= tol * bnorm;
                if (hn == 0.0) met = 1;
                break;
            }
        }
        for (int i = jd - 1; i >= 0; --i) {
            or_cplx t2 = g[i];
            for (int k = i + 1; k < jd; ++k) t2 -= H[i * m + k] * y[k];
            y[i] = t2 / H[i * m + i];
        }
        for (int k = 0; k < jd; ++k)
            for (long i = 0; i < n; ++i) x[i] += y[k] * Vv[(size_t)k * n + i];
        ++cycles;
    }
    if (rep) {
        rep->iters = iters;
        rep->restarts = cycles;
        rep->converged = met;
        rep->true_rel_res = bnorm > 0 ? est / bnorm : 0.0;
    }
    free(Vv);
    free(w);
    free(H);
    free(cs);
    free(sn);
    free(g);
    free(y);
    return met ? 0 : 1;
}

typedef struct {
    const int* cdims;
    int nv;
    const or_cplx* Dc;
    double mu_c;
    const or_cplx* Minv;  /* even-odd: inverses of the even-site blocks */
    or_cplx* t;           /* even-odd: workspace, two coarse vectors */
} coarse_ctx;

static void coarse_apply_fn(const void* ctx, const or_cplx* in, or_cplx* out) {
    const coarse_ctx* c = (const coarse_ctx*)ctx;
    or_mg_coarse_apply(c->cdims, c->nv, c->Dc, c->mu_c, in, out);
}

/* GMRES(restart) for (Dc + i mu_c Gamma5c) x = b from x = 0; the stopping
 * estimate is relative to ||b||. */
int or_mg_coarse_gmres(const int cdims[4], int nv, const or_cplx* Dc, double mu_c, const or_cplx* b, or_cplx* x,
                       double tol, int restart, int max_restarts, or_report* rep) {
    long n = or_volume(cdims) * 2 * nv;
    coarse_ctx c = {cdims, nv, Dc, mu_c, NULL, NULL};
    return gmres_op(n, coarse_apply_fn, &c, b, x, tol, vnorm(b, n), restart, max_restarts, rep);
}

/* Parity of a coarse site: sum of its coordinates mod 2 (0 = even). */
static int coarse_parity(const int cdims[4], long j) {
    int J[4];
    site_coords(cdims, j, J);
    return (J[0] + J[1] + J[2] + J[3]) & 1;
}

/* out = [s_self (Dc[j][0] + i mu_c Gamma5c) x_self + sum_{t>=1} Dc[j][t] x_hop(nbr_t(j))] on the
 * coarse sites of parity p, 0 on the others; a NULL input is a zero vector. */
static void coarse_part(const int cdims[4], int nv, const or_cplx* Dc, double mu_c, int p, const or_cplx* x_self,
                        const or_cplx* x_hop, or_cplx* out) {
    long nc = or_volume(cdims);
    int n2 = 2 * nv;
#pragma omp parallel for schedule(static)
    for (long j = 0; j < nc; ++j) {
        for (int a = 0; a < n2; ++a) {
            or_cplx acc = 0;
            if (coarse_parity(cdims, j) == p) {
                if (x_self) {
                    acc = _Complex_I * mu_c * (a < nv ? 1.0 : -1.0) * x_self[(size_t)j * n2 + a];
                    const or_cplx* M = Dc + (((size_t)j * 9) * n2 + a) * n2;
                    for (int b = 0; b < n2; ++b) acc += M[b] * x_self[(size_t)j * n2 + b];
                }
                if (x_hop)
                    for (int t = 1; t < 9; ++t) {
                        long src = mg_coarse_nbr(cdims, j, t);
                        const or_cplx* M = Dc + (((size_t)j * 9 + t) * n2 + a) * n2;
                        for (int b = 0; b < n2; ++b) acc += M[b] * x_hop[(size_t)src * n2 + b];
                    }
            }
            out[(size_t)j * n2 + a] = acc;
        }
    }
}

/* Inverses of the site blocks Dc[j][0] + i mu_c Gamma5c at the sites of parity p
 * (Gauss-Jordan elimination with partial pivoting); Minv [nc][n2][n2]. */
static void coarse_block_inverses(const int cdims[4], int nv, const or_cplx* Dc, double mu_c, int p, or_cplx* Minv) {
    long nc = or_volume(cdims);
    int n2 = 2 * nv;
#pragma omp parallel for schedule(dynamic)
    for (long j = 0; j < nc; ++j) {
        if (coarse_parity(cdims, j) != p) continue;
        or_cplx* a = malloc(sizeof(or_cplx) * n2 * 2 * n2);  /* [A | I] */
        for (int r = 0; r < n2; ++r)
            for (int c = 0; c < 2 * n2; ++c) {
                or_cplx v = c < n2 ? Dc[(((size_t)j * 9) * n2 + r) * n2 + c] : (c - n2 == r ? 1.0 : 0.0);
                if (c == r) v += _Complex_I * mu_c * (r < nv ? 1.0 : -1.0);
                a[r * 2 * n2 + c] = v;
            }
        for (int k = 0; k < n2; ++k) {
            int piv = k;
            for (int r = k + 1; r < n2; ++r)
                if (cabs(a[r * 2 * n2 + k]) > cabs(a[piv * 2 * n2 + k])) piv = r;
            if (piv != k)
                for (int c = 0; c < 2 * n2; ++c) {
                    or_cplx t = a[k * 2 * n2 + c];
                    a[k * 2 * n2 + c] = a[piv * 2 * n2 + c];
                    a[piv * 2 * n2 + c] = t;
                }
            or_cplx d = a[k * 2 * n2 + k];
            for (int c = 0; c < 2 * n2; ++c) a[k * 2 * n2 + c] /= d;
            for (int r = 0; r < n2; ++r) {
                if (r == k) continue;
                or_cplx f = a[r * 2 * n2 + k];
                if (f == 0) continue;
                for (int c = 0; c < 2 * n2; ++c) a[r * 2 * n2 + c] -= f * a[k * 2 * n2 + c];
            }
        }
        for (int r = 0; r < n2; ++r)
            for (int c = 0; c < n2; ++c) Minv[((size_t)j * n2 + r) * n2 + c] = a[r * 2 * n2 + n2 + c];
        free(a);
    }
}

/* y = Minv x on the sites of parity p, 0 elsewhere. */
static void coarse_block_mul(const int cdims[4], int nv, const or_cplx* Minv, int p, const or_cplx* x, or_cplx* y) {
    long nc = or_volume(cdims);
    int n2 = 2 * nv;
    for (long j = 0; j < nc; ++j)
        for (int a = 0; a < n2; ++a) {
            or_cplx acc = 0;
            if (coarse_parity(cdims, j) == p)
                for (int b = 0; b < n2; ++b) acc += Minv[((size_t)j * n2 + a) * n2 + b] * x[(size_t)j * n2 + b];
            y[(size_t)j * n2 + a] = acc;
        }
}

/* Reduced operator on the odd coarse sites (section 2.5, applied to the coarse
 * grid): y_o = (D_oo - D_oe D_ee^-1 D_eo) x_o; x and y are full coarse vectors
 * whose even parts are ignored / zero. */
static void coarse_dhat_fn(const void* ctx, const or_cplx* in, or_cplx* out) {
    const coarse_ctx* c = (const coarse_ctx*)ctx;
    long n = or_volume(c->cdims) * 2 * c->nv;
    or_cplx* t = c->t;
    or_cplx* u = c->t + n;
    coarse_part(c->cdims, c->nv, c->Dc, c->mu_c, 0, NULL, in, t);        /* t_e = D_eo x_o */
    coarse_block_mul(c->cdims, c->nv, c->Minv, 0, t, u);                /* u_e = D_ee^-1 t_e */
    coarse_part(c->cdims, c->nv, c->Dc, c->mu_c, 1, in, NULL, out);      /* D_oo x_o */
    coarse_part(c->cdims, c->nv, c->Dc, c->mu_c, 1, NULL, u, t);         /* D_oe u_e */
    for (long i = 0; i < n; ++i) out[i] -= t[i];
}

void or_mg_coarse_dhat(const int cdims[4], int nv, const or_cplx* Dc, double mu_c, const or_cplx* x, or_cplx* y) {
    long n = or_volume(cdims) * 2 * nv;
    or_cplx* Minv = malloc(sizeof(or_cplx) * or_volume(cdims) * 4 * nv * nv);
    or_cplx* t = malloc(sizeof(or_cplx) * 2 * n);
    coarse_block_inverses(cdims, nv, Dc, mu_c, 0, Minv);
    coarse_ctx c = {cdims, nv, Dc, mu_c, Minv, t};
    coarse_dhat_fn(&c, x, y);
    free(Minv);
    free(t);
}

/* Even-odd preconditioned GMRES on the coarse grid (the paper's coarsest-grid
 * solver, section 2.5): GMRES(restart) for the odd-site system
 * Dhat x_o = b_o - D_oe D_ee^-1 b_e from x = 0, then x_e = D_ee^-1 (b_e - D_eo x_o).
 * The full residual's even part vanishes and its odd part is the reduced
 * residual, so the estimate is compared with tol ||b||. */
int or_mg_coarse_gmres_eo(const int cdims[4], int nv, const or_cplx* Dc, double mu_c, const or_cplx* b, or_cplx* x,
                          double tol, int restart, int max_restarts, or_report* rep) {
    long nc = or_volume(cdims), n = nc * 2 * nv;
    or_cplx* Minv = malloc(sizeof(or_cplx) * nc * 4 * nv * nv);
    or_cplx* t = malloc(sizeof(or_cplx) * 2 * n);
    or_cplx* bh = malloc(sizeof(or_cplx) * n);
    or_cplx* u = malloc(sizeof(or_cplx) * n);
    coarse_block_inverses(cdims, nv, Dc, mu_c, 0, Minv);
    coarse_ctx c = {cdims, nv, Dc, mu_c, Minv, t};
    /* bhat_o = b_o - D_oe D_ee^-1 b_e */
    coarse_block_mul(cdims, nv, Minv, 0, b, u);
    coarse_part(cdims, nv, Dc, mu_c, 1, NULL, u, bh);
    for (long j = 0; j < nc; ++j)
        for (int a = 0; a < 2 * nv; ++a) {
            size_t i = (size_t)j * 2 * nv + a;
            bh[i] = coarse_parity(cdims, j) == 1 ? b[i] - bh[i] : 0;
        }
    int rc = gmres_op(n, coarse_dhat_fn, &c, bh, x, tol, vnorm(b, n), restart, max_restarts, rep);
    /* x_e = D_ee^-1 (b_e - D_eo x_o) */
    coarse_part(cdims, nv, Dc, mu_c, 0, NULL, x, t);
    for (long i = 0; i < n; ++i) t[i] = b[i] - t[i];
    coarse_block_mul(cdims, nv, Minv, 0, t, u);
    for (long j = 0; j < nc; ++j)
        if (coarse_parity(cdims, j) == 0)
            for (int a = 0; a < 2 * nv; ++a) x[(size_t)j * 2 * nv + a] = u[(size_t)j * 2 * nv + a];
    free(Minv);
    free(t);
    free(bh);
    free(u);
    return rc;
}

/* Two-level preconditioner (eq. (multigrid_preconditioning) followed by
 * post-smoothing, no pre-smoothing): z = P D_c(mu, delta)^-1 P^+ r with the
 * coarse system solved by GMRES, then post_cycles SAP cycles on D z = r
 * starting from that z. */
void or_mg_precond(const or_op* op, const or_mg* mg, const or_cplx* r, or_cplx* z) {
    int cd[4];
    mg_cdims(op->dims, mg->adims, cd);
    long nc = or_volume(cd), n2 = 2 * mg->nv;
    or_cplx* c = malloc(sizeof(or_cplx) * nc * n2);
    or_cplx* ec = malloc(sizeof(or_cplx) * nc * n2);
    or_mg_restrict(op->dims, mg->adims, mg->nv, mg->P, r, c);
    if (mg->coarse_eo)
        or_mg_coarse_gmres_eo(cd, mg->nv, mg->Dc, mg->delta * op->mu, c, ec, mg->coarse_tol, mg->coarse_restart,
                              mg->coarse_max_restarts, NULL);
    else
        or_mg_coarse_gmres(cd, mg->nv, mg->Dc, mg->delta * op->mu, c, ec, mg->coarse_tol, mg->coarse_restart,
                           mg->coarse_max_restarts, NULL);
    or_mg_prolong(op->dims, mg->adims, mg->nv, mg->P, ec, z);
    if (mg->post_cycles > 0) or_sap_eo(op, mg->adims, mg->post_cycles, mg->mr_iters, 0, r, z);
    free(c);
    free(ec);
}

typedef struct {
    const or_op* op;
    const or_mg* mg;
} mg_ctx;

static void mg_precond_fn(const void* ctx, const or_cplx* v, or_cplx* z) {
    const mg_ctx* c = (const mg_ctx*)ctx;
    or_mg_precond(c->op, c->mg, v, z);
}

int or_fgmres_mg(const or_op* op, const or_mg* mg, const or_cplx* b, or_cplx* x, double tol, int restart,
                 int max_iters, or_report* rep) {
    mg_ctx c = {op, mg};
    return fgmres_core(op, b, x, tol, restart, max_iters, mg_precond_fn, &c, rep);
}

/* Global modified Gram-Schmidt of nv lattice vectors, in order. */
static void mg_orthonormalize(long n, int nv, or_cplx* v) {
    for (int i = 0; i < nv; ++i) {
        or_cplx* vi = v + (size_t)i * n;
        for (int k = 0; k < i; ++k) {
            const or_cplx* vk = v + (size_t)k * n;
            or_cplx h = vdot(vk, vi, n);
            for (long q = 0; q < n; ++q) vi[q] -= h * vk[q];
        }
        double nrm = vnorm(vi, n);
        if (nrm > 0)
            for (long q = 0; q < n; ++q) vi[q] /= nrm;
    }
}

/* Adaptive setup (section 2.6): iteration 1 replaces each test vector v_i by
 * setup_cycles SAP cycles applied to it (as a right-hand side, from a zero
 * guess); iterations 2 .. setup_iters replace it by the two-level method
 * applied to it.  After every iteration the vectors are orthonormalised and P
 * and the coarse stencil rebuilt from them.  v0 holds the nv starting vectors
 * ([nv][V][12], the random draws); v (optional) receives the final vectors. */
int or_mg_setup(const or_op* op, or_mg* mg, const or_cplx* v0, or_cplx* v_out) {
    long V = or_volume(op->dims), n = V * 12;
    int nv = mg->nv;
    or_cplx* v = malloc(sizeof(or_cplx) * (size_t)nv * n);
    or_cplx* t = malloc(sizeof(or_cplx) * n);
    memcpy(v, v0, sizeof(or_cplx) * (size_t)nv * n);
    int rc = 0;
    for (int k = 1; k <= mg->setup_iters; ++k) {
        for (int i = 0; i < nv; ++i) {
            or_cplx* vi = v + (size_t)i * n;
            if (k == 1) {
                for (long q = 0; q < n; ++q) t[q] = 0;
                rc = or_sap_eo(op, mg->adims, mg->setup_cycles, mg->mr_iters, 0, vi, t);
                if (rc) goto out;
            } else {
                or_mg_precond(op, mg, vi, t);
            }
            memcpy(vi, t, sizeof(or_cplx) * n);
        }
        mg_orthonormalize(n, nv, v);
        or_mg_block_orthonormalize(op->dims, mg->adims, nv, v, mg->P);
        or_mg_coarse_build(op, mg->adims, nv, mg->P, mg->Dc);
    }
    if (mg->setup_iters <= 0) {
        or_mg_block_orthonormalize(op->dims, mg->adims, nv, v, mg->P);
        or_mg_coarse_build(op, mg->adims, nv, mg->P, mg->Dc);
    }
    if (v_out) memcpy(v_out, v, sizeof(or_cplx) * (size_t)nv * n);
out:
    free(v);
    free(t);
    return rc;
}

int or_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void or_set_num_threads(int n) {
#ifdef _OPENMP
    omp_set_num_threads(n);
#else
    (void)n;
#endif
}
