// Device-side building blocks shared by the library's kernels: storage
// types, the internal site layout, complex arithmetic and the spin algebra
// of the chiral gamma basis (gamma5 = gamma0 gamma1 gamma2 gamma3 =
// diag(1,1,-1,-1), section 2.1).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tmsap {

// ------------------------------------------------------------ storage types

struct bf16 {
    uint16_t bits;
};
typedef _Float16 f16;

// Round-to-nearest-even FP32 -> BF16 (NaN kept quiet).
__host__ __device__ inline bf16 to_bf16(float f) {
    uint32_t u = __builtin_bit_cast(uint32_t, f);
    bf16 r;
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) {
        r.bits = (uint16_t)((u >> 16) | 0x40);
        return r;
    }
    u += 0x7fffu + ((u >> 16) & 1u);
    r.bits = (uint16_t)(u >> 16);
    return r;
}
__host__ __device__ inline float from_bf16(bf16 b) {
    return __builtin_bit_cast(float, (uint32_t)b.bits << 16);
}

// Four reals of storage type S, converted to / from the compute type R.
template <class S> struct Unit;

template <> struct Unit<double> {
    static constexpr int bytes = 32;
    template <class R> __device__ static inline void load(const void* base, size_t i, R out[4]) {
        const double2* p = reinterpret_cast<const double2*>(base) + 2 * i;
        double2 a = p[0], b = p[1];
        out[0] = (R)a.x; out[1] = (R)a.y; out[2] = (R)b.x; out[3] = (R)b.y;
    }
    template <class R> __device__ static inline void store(void* base, size_t i, const R v[4]) {
        double2* p = reinterpret_cast<double2*>(base) + 2 * i;
        p[0] = make_double2((double)v[0], (double)v[1]);
        p[1] = make_double2((double)v[2], (double)v[3]);
    }
};

template <> struct Unit<float> {
    static constexpr int bytes = 16;
    template <class R> __device__ static inline void load(const void* base, size_t i, R out[4]) {
        float4 a = reinterpret_cast<const float4*>(base)[i];
        out[0] = (R)a.x; out[1] = (R)a.y; out[2] = (R)a.z; out[3] = (R)a.w;
    }
    template <class R> __device__ static inline void store(void* base, size_t i, const R v[4]) {
        reinterpret_cast<float4*>(base)[i] = make_float4((float)v[0], (float)v[1], (float)v[2], (float)v[3]);
    }
};

struct alignas(8) h4 { f16 v[4]; };
template <> struct Unit<f16> {
    static constexpr int bytes = 8;
    template <class R> __device__ static inline void load(const void* base, size_t i, R out[4]) {
        h4 a = reinterpret_cast<const h4*>(base)[i];
        for (int k = 0; k < 4; ++k) out[k] = (R)(float)a.v[k];
    }
    template <class R> __device__ static inline void store(void* base, size_t i, const R v[4]) {
        h4 a;
        for (int k = 0; k < 4; ++k) a.v[k] = (f16)(float)v[k];
        reinterpret_cast<h4*>(base)[i] = a;
    }
};

struct alignas(8) b4 { bf16 v[4]; };
template <> struct Unit<bf16> {
    static constexpr int bytes = 8;
    template <class R> __device__ static inline void load(const void* base, size_t i, R out[4]) {
        b4 a = reinterpret_cast<const b4*>(base)[i];
        for (int k = 0; k < 4; ++k) out[k] = (R)from_bf16(a.v[k]);
    }
    template <class R> __device__ static inline void store(void* base, size_t i, const R v[4]) {
        b4 a;
        for (int k = 0; k < 4; ++k) a.v[k] = to_bf16((float)v[k]);
        reinterpret_cast<b4*>(base)[i] = a;
    }
};

// FP16 spinors carry one FP32 scale per site and system (the power of two
// just above the largest |component|, see store_spinor): without it a
// unit-norm field on a large lattice falls below FP16's normal range.  Other
// storage types carry no scale.
template <class S> struct HasScale { static constexpr bool value = false; };
template <> struct HasScale<f16> { static constexpr bool value = true; };

// ---------------------------------------------------------------- complex

template <class R> struct cplx {
    R re, im;
};
template <class R> __device__ __host__ inline cplx<R> cmk(R a, R b) { return cplx<R>{a, b}; }
template <class R> __device__ inline cplx<R> operator+(cplx<R> a, cplx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <class R> __device__ inline cplx<R> operator-(cplx<R> a, cplx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <class R> __device__ inline cplx<R> operator-(cplx<R> a) { return {-a.re, -a.im}; }
template <class R> __device__ inline cplx<R> operator*(cplx<R> a, cplx<R> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <class R> __device__ inline cplx<R> operator*(R s, cplx<R> a) { return {s * a.re, s * a.im}; }
template <class R> __device__ inline cplx<R> conj(cplx<R> a) { return {a.re, -a.im}; }
template <class R> __device__ inline cplx<R> times_i(cplx<R> a) { return {-a.im, a.re}; }
template <class R> __device__ inline cplx<R> times_mi(cplx<R> a) { return {a.im, -a.re}; }
// a * b + c
template <class R> __device__ inline cplx<R> cmad(cplx<R> a, cplx<R> b, cplx<R> c) {
    return {c.re + a.re * b.re - a.im * b.im, c.im + a.re * b.im + a.im * b.re};
}
// conj(a) * b + c
template <class R> __device__ inline cplx<R> cjmad(cplx<R> a, cplx<R> b, cplx<R> c) {
    return {c.re + a.re * b.re + a.im * b.im, c.im + a.re * b.im - a.im * b.re};
}

// ---------------------------------------------------------------- layout

// The internal layout tiles the lattice by `lb` (T,Z,Y,X): sites of a tile are
// contiguous (local index lexicographic, t slowest), tiles are lexicographic
// over the tile grid.  Every field is stored structure-of-arrays: element k
// of site s lives at [k][s], so a wavefront touches consecutive addresses.
struct Geo {
    int d[4];    // lattice dims (T, Z, Y, X)
    int lb[4];   // tile dims
    int nb[4];   // tiles per axis
    int Vb;      // sites per tile
    long long V; // sites
    double bcr[4], bci[4];  // boundary phase of a forward hop across the lattice boundary along mu
                            // (a backward one takes the conjugate): exp(i theta_mu), -1 for
                            // antiperiodic t
    float bcrf[4], bcif[4]; // the same phases rounded to FP32 on the host (FP32 kernels read these
                            // as scalar operands instead of converting per lane)
    double mu_shift[2];     // added to the twisted mass on even / odd sites
};


// Array axis of direction mu (t, x, y, z) -> (0, 3, 2, 1).
__host__ __device__ inline int axis_of(int mu) { return mu == 0 ? 0 : 4 - mu; }

__host__ __device__ inline void site_coords(const Geo& g, long long s, int c[4]) {
    long long blk = s / g.Vb;
    int l = (int)(s - blk * g.Vb);
    int B[4], L[4];
    for (int a = 3; a >= 0; --a) {
        B[a] = (int)(blk % g.nb[a]);
        blk /= g.nb[a];
        L[a] = l % g.lb[a];
        l /= g.lb[a];
    }
    for (int a = 0; a < 4; ++a) c[a] = B[a] * g.lb[a] + L[a];
}

__host__ __device__ inline long long coords_site(const Geo& g, const int c[4]) {
    long long blk = 0;
    int l = 0;
    for (int a = 0; a < 4; ++a) {
        int B = c[a] / g.lb[a];
        blk = blk * g.nb[a] + B;
        l = l * g.lb[a] + (c[a] - B * g.lb[a]);
    }
    return blk * g.Vb + l;
}

// Workgroups are dealt to the eight XCDs round-robin (workgroup j to XCD j mod 8),
// and each XCD has its own L2.  This bijection of [0, n) gives the workgroups of
// one XCD consecutive block numbers, so that neighbouring blocks, which read the
// same face spinors, run at the same time on the same L2.
__host__ __device__ inline long long xcd_swizzle(long long j, long long n) {
    const long long q = n / 8, r = n % 8, x = j % 8, p = j / 8;
    return x * q + (x < r ? x : r) + p;
}

// The 8 neighbours of site s in the tiled layout, s +- mu (periodic), the
// hops that cross the lattice boundary (bit mu forward, bit 4+mu backward) and
// the parity of s.  32-bit arithmetic: the library limits the volume to 2^29
// sites.  In-tile neighbours are s plus a fixed stride; across a tile face the
// local coordinate wraps and the tile index steps (with the lattice's
// periodic wrap).
__host__ __device__ inline void tiled_neighbours(const Geo& g, long long s, int nf[4], int nbk[4], unsigned* wrap,
                                        int* parity) {
    const unsigned su = (unsigned)s;
    const unsigned Vb = (unsigned)g.Vb;
    const unsigned blk = su / Vb;
    const unsigned l = su - blk * Vb;
    int L[4], B[4];
    unsigned t = l, tb = blk;
    int csum = 0;
#pragma unroll
    for (int a = 3; a >= 0; --a) {
        const unsigned lb = (unsigned)g.lb[a], nb = (unsigned)g.nb[a];
        const unsigned tq = t / lb, bq = tb / nb;
        L[a] = (int)(t - tq * lb);
        B[a] = (int)(tb - bq * nb);
        csum += B[a] * g.lb[a] + L[a];
        t = tq;
        tb = bq;
    }
    *parity = csum & 1;
    int ls[4], bs[4];
    ls[3] = 1;
    bs[3] = 1;
#pragma unroll
    for (int a = 2; a >= 0; --a) {
        ls[a] = ls[a + 1] * g.lb[a + 1];
        bs[a] = bs[a + 1] * g.nb[a + 1];
    }
    unsigned w = 0;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        const int a = axis_of(mu);
        if (L[a] + 1 < g.lb[a]) {
            nf[mu] = (int)su + ls[a];
        } else {
            int bn = (int)blk + bs[a];
            if (B[a] + 1 == g.nb[a]) {
                bn -= g.nb[a] * bs[a];
                w |= 1u << mu;
            }
            nf[mu] = bn * g.Vb + (int)l - (g.lb[a] - 1) * ls[a];
        }
        if (L[a] > 0) {
            nbk[mu] = (int)su - ls[a];
        } else {
            int bn = (int)blk - bs[a];
            if (B[a] == 0) {
                bn += g.nb[a] * bs[a];
                w |= 1u << (4 + mu);
            }
            nbk[mu] = bn * g.Vb + (int)l + (g.lb[a] - 1) * ls[a];
        }
    }
    *wrap = w;
}

// Lexicographic (canonical) index of coordinates.
__host__ __device__ inline long long lex_site(const Geo& g, const int c[4]) {
    return (((long long)c[0] * g.d[1] + c[1]) * g.d[2] + c[2]) * g.d[3] + c[3];
}

// ------------------------------------------------------------ spin algebra
// gamma_mu = [[0, B_mu], [B_mu^+, 0]] on (upper, lower) spin pairs with
// B_0 = -1, B_k = -i sigma_k.  A spinor is 4 spins x 3 colours, index 3s+c.

// B_mu applied to the lower pair (p2, p3) -> pair (o0, o1), one colour.
template <class R>
__device__ inline void apply_B(int mu, cplx<R> p2, cplx<R> p3, cplx<R>& o0, cplx<R>& o1) {
    switch (mu) {
        case 0: o0 = -p2; o1 = -p3; break;               // -1
        case 1: o0 = times_mi(p3); o1 = times_mi(p2); break;  // [[0,-i],[-i,0]]
        case 2: o0 = -p3; o1 = p2; break;                // [[0,-1],[1,0]]
        default: o0 = times_mi(p2); o1 = times_i(p3); break;  // [[-i,0],[0,i]]
    }
}

// B_mu^+ applied to an upper pair (p0, p1) -> pair (o0, o1), one colour.
template <class R>
__device__ inline void apply_Bdag(int mu, cplx<R> p0, cplx<R> p1, cplx<R>& o0, cplx<R>& o1) {
    switch (mu) {
        case 0: o0 = -p0; o1 = -p1; break;               // -1
        case 1: o0 = times_i(p1); o1 = times_i(p0); break;    // [[0,i],[i,0]]
        case 2: o0 = p1; o1 = -p0; break;                // [[0,1],[-1,0]]
        default: o0 = times_i(p0); o1 = times_mi(p1); break;  // [[i,0],[0,-i]]
    }
}

// ---------------------------------------------------------------- links
// Links are stored as their first two rows (12 reals); the third row of an
// SU(3) matrix is conj(row0 x row1).
template <class R> struct Link {
    cplx<R> u[3][3];
};

template <class R> __device__ inline void complete_su3(Link<R>& L) {
    L.u[2][0] = conj(L.u[0][1] * L.u[1][2] - L.u[0][2] * L.u[1][1]);
    L.u[2][1] = conj(L.u[0][2] * L.u[1][0] - L.u[0][0] * L.u[1][2]);
    L.u[2][2] = conj(L.u[0][0] * L.u[1][1] - L.u[0][1] * L.u[1][0]);
}

// Half spinor: 2 spins x 3 colours.
template <class R> struct Half {
    cplx<R> h[2][3];
};

// g = U h
template <class R> __device__ inline void su3_mul(const Link<R>& L, const Half<R>& h, Half<R>& g) {
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            cplx<R> t = L.u[i][0] * h.h[s][0];
            t = cmad(L.u[i][1], h.h[s][1], t);
            t = cmad(L.u[i][2], h.h[s][2], t);
            g.h[s][i] = t;
        }
}

// g = U^+ h
template <class R> __device__ inline void su3_dag_mul(const Link<R>& L, const Half<R>& h, Half<R>& g) {
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            cplx<R> t = cjmad(L.u[0][i], h.h[s][0], cmk<R>(0, 0));
            t = cjmad(L.u[1][i], h.h[s][1], t);
            t = cjmad(L.u[2][i], h.h[s][2], t);
            g.h[s][i] = t;
        }
}

template <class R> struct Spinor {
    cplx<R> v[12];
};

// p <- phase p for a hop along mu that crosses the lattice boundary
// (dir = +1 forward, -1 backward).
template <class R>
__device__ inline void apply_bc(const Geo& g, int mu, int dir, Spinor<R>& p) {
    R re, im;
    if constexpr (sizeof(R) == 4) {
        re = g.bcrf[mu];
        im = dir > 0 ? g.bcif[mu] : -g.bcif[mu];
    } else {
        re = (R)g.bcr[mu];
        im = dir > 0 ? (R)g.bci[mu] : -(R)g.bci[mu];
    }
#pragma unroll
    for (int i = 0; i < 12; ++i) p.v[i] = cmk(re * p.v[i].re - im * p.v[i].im, re * p.v[i].im + im * p.v[i].re);
}

// Hop accumulators: the operator adds -1/2 (hu; hd) at the end.
// Forward hop into x from x+mu: (1 - gamma_mu) U_mu(x) psi(x+mu):
//   h = upper - B d,  g = U h,  hu += g,  hd += -B^+ g.
template <class R>
__device__ inline void hop_forward(int mu, const Link<R>& L, const Spinor<R>& p, R sign, Spinor<R>& acc) {
    Half<R> h, g;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        cplx<R> b0, b1;
        apply_B(mu, p.v[6 + c], p.v[9 + c], b0, b1);
        h.h[0][c] = p.v[c] - b0;
        h.h[1][c] = p.v[3 + c] - b1;
    }
    su3_mul(L, h, g);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        cplx<R> d0, d1;
        apply_Bdag(mu, g.h[0][c], g.h[1][c], d0, d1);
        acc.v[c] = acc.v[c] + sign * g.h[0][c];
        acc.v[3 + c] = acc.v[3 + c] + sign * g.h[1][c];
        acc.v[6 + c] = acc.v[6 + c] - sign * d0;
        acc.v[9 + c] = acc.v[9 + c] - sign * d1;
    }
}

// Backward hop into x from x-mu: (1 + gamma_mu) U_mu(x-mu)^+ psi(x-mu):
//   h = upper + B d,  g = U^+ h,  hu += g,  hd += B^+ g.
template <class R>
__device__ inline void hop_backward(int mu, const Link<R>& L, const Spinor<R>& p, R sign, Spinor<R>& acc) {
    Half<R> h, g;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        cplx<R> b0, b1;
        apply_B(mu, p.v[6 + c], p.v[9 + c], b0, b1);
        h.h[0][c] = p.v[c] + b0;
        h.h[1][c] = p.v[3 + c] + b1;
    }
    su3_dag_mul(L, h, g);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        cplx<R> d0, d1;
        apply_Bdag(mu, g.h[0][c], g.h[1][c], d0, d1);
        acc.v[c] = acc.v[c] + sign * g.h[0][c];
        acc.v[3 + c] = acc.v[3 + c] + sign * g.h[1][c];
        acc.v[6 + c] = acc.v[6 + c] + sign * d0;
        acc.v[9 + c] = acc.v[9 + c] + sign * d1;
    }
}

// Split form of the backward hop used when the neighbour computes the product:
// the site x-mu forms g = U_mu(x-mu)^+ (upper + B lower) of its own spinor ...
template <class R>
__device__ inline void backward_product(int mu, const Link<R>& L, const Spinor<R>& p, Half<R>& g) {
    Half<R> h;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        cplx<R> b0, b1;
        apply_B(mu, p.v[6 + c], p.v[9 + c], b0, b1);
        h.h[0][c] = p.v[c] + b0;
        h.h[1][c] = p.v[3 + c] + b1;
    }
    su3_dag_mul(L, h, g);
}

// ... and the site x adds it: hu += g, hd += B^+ g.
template <class R>
__device__ inline void backward_accumulate(int mu, const Half<R>& g, Spinor<R>& acc) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        cplx<R> d0, d1;
        apply_Bdag(mu, g.h[0][c], g.h[1][c], d0, d1);
        acc.v[c] = acc.v[c] + g.h[0][c];
        acc.v[3 + c] = acc.v[3 + c] + g.h[1][c];
        acc.v[6 + c] = acc.v[6 + c] + d0;
        acc.v[9 + c] = acc.v[9 + c] + d1;
    }
}

// Forward hop without a boundary sign (hops inside a Schwarz block never wrap).
template <class R>
__device__ inline void hop_forward_in(int mu, const Link<R>& L, const Spinor<R>& p, Spinor<R>& acc) {
    Half<R> h, g;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        cplx<R> b0, b1;
        apply_B(mu, p.v[6 + c], p.v[9 + c], b0, b1);
        h.h[0][c] = p.v[c] - b0;
        h.h[1][c] = p.v[3 + c] - b1;
    }
    su3_mul(L, h, g);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        cplx<R> d0, d1;
        apply_Bdag(mu, g.h[0][c], g.h[1][c], d0, d1);
        acc.v[c] = acc.v[c] + g.h[0][c];
        acc.v[3 + c] = acc.v[3 + c] + g.h[1][c];
        acc.v[6 + c] = acc.v[6 + c] - d0;
        acc.v[9 + c] = acc.v[9 + c] - d1;
    }
}

// ---------------------------------------------------------------- clover
// Per site: two Hermitian 6x6 blocks (spins {0,1} and {2,3}; index
// 3*(s mod 2) + c), each packed as 6 real diagonals followed by the 15
// complex entries above the diagonal in row-major order: 36 reals, 72 per
// site, holding (m+4) + clover.  The twist i mu Gamma5 is added on the fly.
template <class R> struct Clover {
    R a[72];
};

// out = (A_blk + i tw) v for one 6x6 block (tw = +mu upper, -mu lower).
template <class R>
__device__ inline void clover_block_apply(const R* A, R tw, const cplx<R>* v, cplx<R>* out) {
    cplx<R> o[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) o[i] = cmk<R>(A[i] * v[i].re - tw * v[i].im, A[i] * v[i].im + tw * v[i].re);
    int k = 6;
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int j = i + 1; j < 6; ++j) {
            cplx<R> a = cmk<R>(A[k], A[k + 1]);
            k += 2;
            o[i] = cmad(a, v[j], o[i]);
            o[j] = cjmad(a, v[i], o[j]);
        }
#pragma unroll
    for (int i = 0; i < 6; ++i) out[i] = o[i];
}

// out += (A_blk + i tw) v for one 6x6 block.
template <class R>
__device__ inline void clover_block_acc(const R* A, R tw, const cplx<R>* v, cplx<R>* out) {
#pragma unroll
    for (int i = 0; i < 6; ++i)
        out[i] = cmk<R>(out[i].re + A[i] * v[i].re - tw * v[i].im, out[i].im + A[i] * v[i].im + tw * v[i].re);
    int k = 6;
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int j = i + 1; j < 6; ++j) {
            cplx<R> a = cmk<R>(A[k], A[k + 1]);
            k += 2;
            out[i] = cmad(a, v[j], out[i]);
            out[j] = cjmad(a, v[i], out[j]);
        }
}

template <class R>
__device__ inline void clover_acc(const Clover<R>& C, R mu, const Spinor<R>& in, Spinor<R>& out) {
    clover_block_acc(C.a, mu, in.v, out.v);
    clover_block_acc(C.a + 36, -mu, in.v + 6, out.v + 6);
}

template <class R>
__device__ inline void clover_apply(const Clover<R>& C, R mu, const Spinor<R>& in, Spinor<R>& out) {
    clover_block_apply(C.a, mu, in.v, out.v);
    clover_block_apply(C.a + 36, -mu, in.v + 6, out.v + 6);
}

// out = D_pp^-1 in at a site of the parity of an inverse set (entry h = s / 2):
// the two 6x6 chiral-block inverses; adj uses their adjoints (the inverses for
// -mu, the diagonal block being Hermitian up to the twist).
template <class C, class R>
__device__ inline void eo_inverse_apply(const void* inv, long long half, long long h, bool adj, const Spinor<R>& in,
                                        Spinor<R>& out) {
#pragma unroll
    for (int i = 0; i < 12; ++i) out.v[i] = cmk<R>(0, 0);
#pragma unroll
    for (int blk = 0; blk < 2; ++blk) {
        const cplx<R>* v = in.v + 6 * blk;
        cplx<R>* o = out.v + 6 * blk;
#pragma unroll
        for (int u = 0; u < 18; ++u) {
            R w[4];
            Unit<C>::load(inv, (size_t)(18 * blk + u) * half + h, w);
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const int e = 2 * u + k, i = e / 6, j = e % 6;
                const cplx<R> m = cmk(w[2 * k], w[2 * k + 1]);
                if (adj)
                    o[j] = cjmad(m, v[i], o[j]);
                else
                    o[i] = cmad(m, v[j], o[i]);
            }
        }
    }
}

// ------------------------------------------------------------- field access

template <class R, class S>
__device__ inline void load_spinor(const void* base, const float* scale, long long V, long long s, Spinor<R>& p) {
    R u[4];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        Unit<S>::load(base, (size_t)k * V + s, u);
        p.v[2 * k] = cmk(u[0], u[1]);
        p.v[2 * k + 1] = cmk(u[2], u[3]);
    }
    if constexpr (HasScale<S>::value) {
        R sc = (R)scale[s];
#pragma unroll
        for (int i = 0; i < 12; ++i) p.v[i] = sc * p.v[i];
    }
}

// FP16 scale of a site: the power of two 2^e with m = f 2^e, f in [0.5, 1),
// for the largest |component| m (0 for a zero site).  Scaling by 2^-e is an
// exponent shift (ldexp), exact and finite for every finite m, subnormal FP32
// included, where a reciprocal 1/m would overflow below about 2.9e-39; the
// scaled components lie in (-1, 1).
__device__ inline int fp16_site_exponent(float m, float* scale) {
    if (!(m > 0.f)) {
        *scale = 0.f;
        return 0;
    }
    int e;
    (void)frexpf(m, &e);
    *scale = ldexpf(1.0f, e);
    return e;
}

template <class R, class S>
__device__ inline void store_spinor(void* base, float* scale, long long V, long long s, const Spinor<R>& p) {
    if constexpr (HasScale<S>::value) {
        float m = 0.f;
#pragma unroll
        for (int i = 0; i < 12; ++i) {
            m = fmaxf(m, fabsf((float)p.v[i].re));
            m = fmaxf(m, fabsf((float)p.v[i].im));
        }
        float sc;
        const int e = fp16_site_exponent(m, &sc);
        scale[s] = sc;
        const bool zero = sc == 0.f;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            float u[4] = {(float)p.v[2 * k].re, (float)p.v[2 * k].im, (float)p.v[2 * k + 1].re,
                          (float)p.v[2 * k + 1].im};
#pragma unroll
            for (int q = 0; q < 4; ++q) u[q] = zero ? u[q] * 0.f : ldexpf(u[q], -e);  // NaN stays NaN
            Unit<S>::store(base, (size_t)k * V + s, u);
        }
    } else {
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            R u[4] = {p.v[2 * k].re, p.v[2 * k].im, p.v[2 * k + 1].re, p.v[2 * k + 1].im};
            Unit<S>::store(base, (size_t)k * V + s, u);
        }
    }
}

// Link (mu) of site s: [mu][3 units][V].
template <class R, class G>
__device__ inline void load_link(const void* base, long long V, long long s, int mu, Link<R>& L) {
    R u[4];
    size_t b = (size_t)mu * 3 * V;
    Unit<G>::load(base, b + s, u);
    L.u[0][0] = cmk(u[0], u[1]); L.u[0][1] = cmk(u[2], u[3]);
    Unit<G>::load(base, b + V + s, u);
    L.u[0][2] = cmk(u[0], u[1]); L.u[1][0] = cmk(u[2], u[3]);
    Unit<G>::load(base, b + 2 * V + s, u);
    L.u[1][1] = cmk(u[0], u[1]); L.u[1][2] = cmk(u[2], u[3]);
    complete_su3(L);
}

// Clover of site s: [18 units][V].
template <class R, class C>
__device__ inline void load_clover(const void* base, long long V, long long s, Clover<R>& A) {
#pragma unroll
    for (int k = 0; k < 18; ++k) Unit<C>::load(base, (size_t)k * V + s, A.a + 4 * k);
}

}  // namespace tmsap
