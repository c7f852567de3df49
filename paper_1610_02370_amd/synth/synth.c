/*
 * Seeded synthetic inputs: SU(3) gauge links, Gaussian and point-source
 * spinors.  This module holds no arithmetic of the solver; it only produces
 * the inputs that the GPU library and the oracle both consume.
 *
 * Random numbers: Philox4x32-10 counter-based generator (Salmon, Moraes,
 * Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC 2011),
 * written from its published definition.  Uniforms are (x + 1/2) 2^-32;
 * normals come from the Box-Muller transform on consecutive uniform pairs.
 *
 * Links: U = exp(i eps H), H = sum_a h_a lambda_a / 2 with the eight
 * Gell-Mann matrices and h_a ~ N(0,1); exp by Taylor series with scaling
 * and squaring, then re-unitarised (Gram-Schmidt on rows 0 and 1,
 * row 2 = conj(row0 x row1)).  Counter = (site low, site high, mu, draw),
 * key = (seed, stream tag), so any site can be generated on its own.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

typedef double _Complex cplx;

#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void synth_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        uint64_t p0 = (uint64_t)PHILOX_M0 * c0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

static double u01(uint32_t x) { return ((double)x + 0.5) * (1.0 / 4294967296.0); }

/* 8 normals from counter (lo, hi, a, draw pair) */
static void normals8(uint32_t seed, uint32_t tag, uint64_t idx, uint32_t a, double out[8]) {
    uint32_t key[2] = {seed, tag};
    for (int d = 0; d < 2; ++d) {
        uint32_t ctr[4] = {(uint32_t)idx, (uint32_t)(idx >> 32), a, (uint32_t)d};
        uint32_t r[4];
        synth_philox4x32_10(ctr, key, r);
        for (int p = 0; p < 2; ++p) {
            double u1 = u01(r[2 * p]), u2 = u01(r[2 * p + 1]);
            double rad = sqrt(-2.0 * log(u1));
            double th = 6.283185307179586476925286766559 * u2;
            out[4 * d + 2 * p] = rad * cos(th);
            out[4 * d + 2 * p + 1] = rad * sin(th);
        }
    }
}

static void mat_mul3(const cplx* a, const cplx* b, cplx* c) {
    cplx t[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            cplx s = 0;
            for (int k = 0; k < 3; ++k) s += a[3 * i + k] * b[3 * k + j];
            t[3 * i + j] = s;
        }
    memcpy(c, t, sizeof t);
}

/* Hermitian traceless H = sum h_a lambda_a / 2 */
static void gellmann_H(const double h[8], cplx H[9]) {
    const cplx ii = _Complex_I;
    const double r3 = 1.0 / sqrt(3.0);
    memset(H, 0, 9 * sizeof(cplx));
    H[1] += h[0];  H[3] += h[0];                   /* lambda1 */
    H[1] += -ii * h[1]; H[3] += ii * h[1];           /* lambda2 */
    H[0] += h[2];  H[4] += -h[2];                  /* lambda3 */
    H[2] += h[3];  H[6] += h[3];                   /* lambda4 */
    H[2] += -ii * h[4]; H[6] += ii * h[4];           /* lambda5 */
    H[5] += h[5];  H[7] += h[5];                   /* lambda6 */
    H[5] += -ii * h[6]; H[7] += ii * h[6];           /* lambda7 */
    H[0] += h[7] * r3; H[4] += h[7] * r3; H[8] += -2.0 * h[7] * r3; /* lambda8 */
    for (int i = 0; i < 9; ++i) H[i] *= 0.5;
}

/* exp(A) by scaling and squaring with a Taylor series. */
static void expm3(const cplx A_in[9], cplx E[9]) {
    double nrm = 0;
    for (int i = 0; i < 9; ++i) nrm += creal(A_in[i]) * creal(A_in[i]) + cimag(A_in[i]) * cimag(A_in[i]);
    nrm = sqrt(nrm);
    int k = 0;
    while (nrm > 0.25) { nrm *= 0.5; ++k; }
    cplx A[9], term[9];
    double sc = ldexp(1.0, -k);
    for (int i = 0; i < 9; ++i) A[i] = A_in[i] * sc;
    for (int i = 0; i < 9; ++i) { E[i] = (i % 4 == 0) ? 1.0 : 0.0; term[i] = E[i]; }
    for (int n = 1; n <= 12; ++n) {  /* ||A|| <= 1/4: truncation below 1e-17 */
        mat_mul3(term, A, term);
        for (int i = 0; i < 9; ++i) { term[i] /= (double)n; E[i] += term[i]; }
    }
    for (int s = 0; s < k; ++s) mat_mul3(E, E, E);
}

/* Gram-Schmidt on rows 0, 1; row 2 = conj(row0 x row1): exact SU(3) up to rounding. */
static void reunitarise(cplx U[9]) {
    double n0 = 0;
    for (int j = 0; j < 3; ++j) n0 += creal(U[j] * conj(U[j]));
    n0 = 1.0 / sqrt(n0);
    for (int j = 0; j < 3; ++j) U[j] *= n0;
    cplx d = 0;
    for (int j = 0; j < 3; ++j) d += conj(U[j]) * U[3 + j];
    for (int j = 0; j < 3; ++j) U[3 + j] -= d * U[j];
    double n1 = 0;
    for (int j = 0; j < 3; ++j) n1 += creal(U[3 + j] * conj(U[3 + j]));
    n1 = 1.0 / sqrt(n1);
    for (int j = 0; j < 3; ++j) U[3 + j] *= n1;
    U[6] = conj(U[1] * U[5] - U[2] * U[4]);
    U[7] = conj(U[2] * U[3] - U[0] * U[5]);
    U[8] = conj(U[0] * U[4] - U[1] * U[3]);
}

static void one_link(uint32_t seed, uint32_t tag, double eps, uint64_t site, uint32_t mu, cplx* U) {
    double h[8];
    cplx H[9], A[9];
    normals8(seed, tag, site, mu, h);
    gellmann_H(h, H);
    for (int i = 0; i < 9; ++i) A[i] = _Complex_I * eps * H[i];
    expm3(A, U);
    reunitarise(U);
}

/* Links for sites [0, V): out[V][4][3][3]. */
void synth_gauge(uint32_t seed, uint32_t tag, double eps, int64_t V, cplx* out) {
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < V; ++s)
        for (uint32_t mu = 0; mu < 4; ++mu) one_link(seed, tag, eps, (uint64_t)s, mu, out + ((size_t)s * 4 + mu) * 9);
}

/* Links of selected sites only: out[n][4][3][3]. */
void synth_gauge_sites(uint32_t seed, uint32_t tag, double eps, int64_t n, const int64_t* sites, cplx* out) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        for (uint32_t mu = 0; mu < 4; ++mu)
            one_link(seed, tag, eps, (uint64_t)sites[i], mu, out + ((size_t)i * 4 + mu) * 9);
}

/* One SU(3) matrix per site (gauge transformations): out[V][3][3]. */
void synth_su3_field(uint32_t seed, uint32_t tag, double eps, int64_t V, cplx* out) {
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < V; ++s) one_link(seed, tag, eps, (uint64_t)s, 7u, out + (size_t)s * 9);
}

/* Gaussian spinor: re and im i.i.d. N(0,1); out[n_elems] complex, element i
 * uses counter (i/4, ..): 8 normals per counter = 4 complex numbers. */
void synth_gaussian(uint32_t seed, uint32_t tag, int64_t n, cplx* out) {
    int64_t groups = (n + 3) / 4;
#pragma omp parallel for schedule(static)
    for (int64_t g = 0; g < groups; ++g) {
        double z[8];
        normals8(seed, tag, (uint64_t)g, 0x5350u, z);
        for (int k = 0; k < 4; ++k) {
            int64_t i = 4 * g + k;
            if (i < n) out[i] = z[2 * k] + _Complex_I * z[2 * k + 1];
        }
    }
}
