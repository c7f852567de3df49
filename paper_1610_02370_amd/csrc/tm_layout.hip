// Layout kernels: gauge-link ingest, clover construction, spinor import /
// export between the canonical complex128 layout and the internal tiled
// structure-of-arrays layout, and precision conversion between internal
// fields.
#include "tm_internal.h"

namespace tmsap {

namespace {

constexpr int kThreads = 256;

inline unsigned grid_for(long long n) { return (unsigned)((n + kThreads - 1) / kThreads); }

struct C64 {
    double re, im;
};
__device__ inline C64 cm(C64 a, C64 b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ inline C64 cadd(C64 a, C64 b) { return {a.re + b.re, a.im + b.im}; }
__device__ inline C64 csub(C64 a, C64 b) { return {a.re - b.re, a.im - b.im}; }
__device__ inline C64 cconj(C64 a) { return {a.re, -a.im}; }

struct M3 {
    C64 m[3][3];
};

__device__ inline M3 load_canon_link(const double* U, long long lex, int mu) {
    const double2* p = reinterpret_cast<const double2*>(U) + ((size_t)lex * 4 + mu) * 9;
    M3 r;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double2 v = p[3 * i + j];
            r.m[i][j] = {v.x, v.y};
        }
    return r;
}

__device__ inline M3 mmul(const M3& a, const M3& b) {
    M3 c;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            C64 t = {0, 0};
            for (int k = 0; k < 3; ++k) t = cadd(t, cm(a.m[i][k], b.m[k][j]));
            c.m[i][j] = t;
        }
    return c;
}

__device__ inline M3 mdag(const M3& a) {
    M3 c;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) c.m[i][j] = cconj(a.m[j][i]);
    return c;
}

__device__ inline void atomic_max_nonneg(unsigned* p, float v) { atomicMax(p, __float_as_uint(v)); }

// ------------------------------------------------------------ link ingest
// stats[0]: max deviation from SU(3) (float bits), stats[1]: nonfinite flag.
template <class G>
__global__ void __launch_bounds__(kThreads) k_link_ingest(Geo g, const double* __restrict__ U, void* links,
                                                          unsigned* stats) {
    long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= g.V) return;
    int c[4];
    site_coords(g, s, c);
    long long lex = lex_site(g, c);
    float dev = 0.f;
    bool bad = false;
    for (int mu = 0; mu < 4; ++mu) {
        M3 L = load_canon_link(U, lex, mu);
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
                if (!isfinite(L.m[i][j].re) || !isfinite(L.m[i][j].im)) bad = true;
        // |U U^+ - 1| and |det U - 1|
        M3 P = mmul(L, mdag(L));
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                double e = fabs(P.m[i][j].re - (i == j ? 1.0 : 0.0)) + fabs(P.m[i][j].im);
                dev = fmaxf(dev, (float)e);
            }
        C64 det = {0, 0};
        det = cadd(det, cm(L.m[0][0], csub(cm(L.m[1][1], L.m[2][2]), cm(L.m[1][2], L.m[2][1]))));
        det = csub(det, cm(L.m[0][1], csub(cm(L.m[1][0], L.m[2][2]), cm(L.m[1][2], L.m[2][0]))));
        det = cadd(det, cm(L.m[0][2], csub(cm(L.m[1][0], L.m[2][1]), cm(L.m[1][1], L.m[2][0]))));
        dev = fmaxf(dev, (float)(fabs(det.re - 1.0) + fabs(det.im)));
        double u[12] = {L.m[0][0].re, L.m[0][0].im, L.m[0][1].re, L.m[0][1].im, L.m[0][2].re, L.m[0][2].im,
                        L.m[1][0].re, L.m[1][0].im, L.m[1][1].re, L.m[1][1].im, L.m[1][2].re, L.m[1][2].im};
        size_t base = (size_t)mu * 3 * g.V;
        for (int k = 0; k < 3; ++k) Unit<G>::store(links, base + (size_t)k * g.V + s, u + 4 * k);
    }
    if (bad) atomicOr(&stats[1], 1u);
    if (!(dev == dev)) dev = 1e30f;
    atomic_max_nonneg(&stats[0], dev);
}

// ------------------------------------------------------------ clover build
// A = (m+4) - (c_sw/16) sum_{mu<nu} (gamma_mu gamma_nu) (x) (Q_munu - Q_numu),
// Q the four-leaf clover.  In the chiral basis gamma_mu gamma_nu =
// diag(B_mu B_nu^+, B_mu^+ B_nu), so A splits into two Hermitian 6x6 blocks.

__device__ inline void spin_B(int mu, C64 B[2][2]) {
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) B[i][j] = {0, 0};
    switch (mu) {
        case 0: B[0][0] = {-1, 0}; B[1][1] = {-1, 0}; break;
        case 1: B[0][1] = {0, -1}; B[1][0] = {0, -1}; break;
        case 2: B[0][1] = {-1, 0}; B[1][0] = {1, 0}; break;
        default: B[0][0] = {0, -1}; B[1][1] = {0, 1}; break;
    }
}

__device__ inline M3 link_at(const Geo& g, const double* U, const int c[4], int mu) {
    return load_canon_link(U, lex_site(g, c), mu);
}

__device__ inline void shift(const Geo& g, int c[4], int mu, int dir) {
    int a = axis_of(mu);
    c[a] += dir;
    if (c[a] < 0) c[a] += g.d[a];
    if (c[a] >= g.d[a]) c[a] -= g.d[a];
}

// Q_munu at coordinates c: four plaquettes in the (mu,nu) plane, each
// starting and ending at c, traversed in the same orientation.
__device__ M3 leaf_sum(const Geo& g, const double* U, const int c0[4], int mu, int nu) {
    int x[4], xpm[4], xpn[4], xmm[4], xmn[4], xmmpn[4], xmmmn[4], xmnpm[4];
    for (int a = 0; a < 4; ++a) x[a] = xpm[a] = xpn[a] = xmm[a] = xmn[a] = c0[a];
    shift(g, xpm, mu, +1);
    shift(g, xpn, nu, +1);
    shift(g, xmm, mu, -1);
    shift(g, xmn, nu, -1);
    for (int a = 0; a < 4; ++a) { xmmpn[a] = xmm[a]; xmmmn[a] = xmm[a]; xmnpm[a] = xmn[a]; }
    shift(g, xmmpn, nu, +1);
    shift(g, xmmmn, nu, -1);
    shift(g, xmnpm, mu, +1);

    M3 Q;
    // path x -> x+mu -> x+mu+nu -> x+nu -> x
    M3 t = mmul(mmul(link_at(g, U, x, mu), link_at(g, U, xpm, nu)),
                mmul(mdag(link_at(g, U, xpn, mu)), mdag(link_at(g, U, x, nu))));
    Q = t;
    // path x -> x+nu -> x-mu+nu -> x-mu -> x
    t = mmul(mmul(link_at(g, U, x, nu), mdag(link_at(g, U, xmmpn, mu))),
             mmul(mdag(link_at(g, U, xmm, nu)), link_at(g, U, xmm, mu)));
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Q.m[i][j] = cadd(Q.m[i][j], t.m[i][j]);
    // path x -> x-mu -> x-mu-nu -> x-nu -> x
    t = mmul(mmul(mdag(link_at(g, U, xmm, mu)), mdag(link_at(g, U, xmmmn, nu))),
             mmul(link_at(g, U, xmmmn, mu), link_at(g, U, xmn, nu)));
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Q.m[i][j] = cadd(Q.m[i][j], t.m[i][j]);
    // path x -> x-nu -> x-nu+mu -> x+mu -> x
    t = mmul(mmul(mdag(link_at(g, U, xmn, nu)), link_at(g, U, xmn, mu)),
             mmul(link_at(g, U, xmnpm, nu), mdag(link_at(g, U, x, mu))));
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Q.m[i][j] = cadd(Q.m[i][j], t.m[i][j]);
    return Q;
}

template <class C>
__global__ void __launch_bounds__(kThreads) k_clover_build(Geo g, const double* __restrict__ U, double m4,
                                                           double csw, void* clover) {
    long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= g.V) return;
    int c[4];
    site_coords(g, s, c);
    C64 A[2][6][6];
    for (int b = 0; b < 2; ++b)
        for (int i = 0; i < 6; ++i)
            for (int j = 0; j < 6; ++j) A[b][i][j] = {i == j ? m4 : 0.0, 0.0};
    if (csw != 0.0) {
        const double f = -csw / 16.0;
        for (int mu = 0; mu < 4; ++mu)
            for (int nu = mu + 1; nu < 4; ++nu) {
                M3 Q = leaf_sum(g, U, c, mu, nu);
                M3 F;
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j) F.m[i][j] = csub(Q.m[i][j], cconj(Q.m[j][i]));
                C64 Bm[2][2], Bn[2][2], Su[2][2], Sd[2][2];
                spin_B(mu, Bm);
                spin_B(nu, Bn);
                for (int i = 0; i < 2; ++i)
                    for (int j = 0; j < 2; ++j) {
                        C64 su = {0, 0}, sd = {0, 0};
                        for (int k = 0; k < 2; ++k) {
                            su = cadd(su, cm(Bm[i][k], cconj(Bn[j][k])));  // B_mu B_nu^+
                            sd = cadd(sd, cm(cconj(Bm[k][i]), Bn[k][j]));  // B_mu^+ B_nu
                        }
                        Su[i][j] = su;
                        Sd[i][j] = sd;
                    }
                for (int s1 = 0; s1 < 2; ++s1)
                    for (int s2 = 0; s2 < 2; ++s2)
                        for (int c1 = 0; c1 < 3; ++c1)
                            for (int c2 = 0; c2 < 3; ++c2) {
                                C64 fu = cm(Su[s1][s2], F.m[c1][c2]);
                                C64 fd = cm(Sd[s1][s2], F.m[c1][c2]);
                                A[0][3 * s1 + c1][3 * s2 + c2] =
                                    cadd(A[0][3 * s1 + c1][3 * s2 + c2], {f * fu.re, f * fu.im});
                                A[1][3 * s1 + c1][3 * s2 + c2] =
                                    cadd(A[1][3 * s1 + c1][3 * s2 + c2], {f * fd.re, f * fd.im});
                            }
            }
    }
    double packed[72];
    for (int b = 0; b < 2; ++b) {
        double* p = packed + 36 * b;
        for (int i = 0; i < 6; ++i) p[i] = A[b][i][i].re;
        int k = 6;
        for (int i = 0; i < 6; ++i)
            for (int j = i + 1; j < 6; ++j) {
                p[k++] = A[b][i][j].re;
                p[k++] = A[b][i][j].im;
            }
    }
    for (int k = 0; k < 18; ++k) Unit<C>::store(clover, (size_t)k * g.V + s, packed + 4 * k);
}

// FP32 clover from the FP64 one of the same field: the build rounds its FP64
// result once at the store, so this rounding gives the same values.
__global__ void __launch_bounds__(kThreads) k_clover_to_f32(long long n_units, const double* __restrict__ src,
                                                            float* dst) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_units) return;
    const double4 a = reinterpret_cast<const double4*>(src)[i];
    reinterpret_cast<float4*>(dst)[i] = make_float4((float)a.x, (float)a.y, (float)a.z, (float)a.w);
}

// ------------------------------------------------------------ spinors
// canonical [nsys][V][12] complex128 -> internal
template <class S>
__global__ void __launch_bounds__(kThreads) k_spinor_import(Geo g, int nsys, const double* __restrict__ canon,
                                                            void* data, float* scale, unsigned* flag) {
    long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int sys = blockIdx.y;
    if (s >= g.V || sys >= nsys) return;
    int c[4];
    site_coords(g, s, c);
    long long lex = lex_site(g, c);
    const double2* p = reinterpret_cast<const double2*>(canon) + ((size_t)sys * g.V + lex) * 12;
    Spinor<double> v;
    bool bad = false;
    for (int i = 0; i < 12; ++i) {
        double2 t = p[i];
        v.v[i] = cmk(t.x, t.y);
        if (!isfinite(t.x) || !isfinite(t.y)) bad = true;
    }
    if (bad) atomicOr(flag, 1u);
    store_spinor<double, S>(reinterpret_cast<char*>(data) + (size_t)sys * 6 * g.V * Unit<S>::bytes,
                            scale ? scale + (size_t)sys * g.V : nullptr, g.V, s, v);
}

template <class S>
__global__ void __launch_bounds__(kThreads) k_spinor_export(Geo g, int nsys, const void* __restrict__ data,
                                                            const float* __restrict__ scale, double* canon) {
    long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int sys = blockIdx.y;
    if (s >= g.V || sys >= nsys) return;
    int c[4];
    site_coords(g, s, c);
    long long lex = lex_site(g, c);
    Spinor<double> v;
    load_spinor<double, S>(reinterpret_cast<const char*>(data) + (size_t)sys * 6 * g.V * Unit<S>::bytes,
                           scale ? scale + (size_t)sys * g.V : nullptr, g.V, s, v);
    double2* p = reinterpret_cast<double2*>(canon) + ((size_t)sys * g.V + lex) * 12;
    for (int i = 0; i < 12; ++i) p[i] = make_double2(v.v[i].re, v.v[i].im);
}

template <class Si, class So>
__global__ void __launch_bounds__(kThreads) k_spinor_convert(Geo g, int nsys, const void* __restrict__ in,
                                                             const float* __restrict__ in_scale, void* out,
                                                             float* out_scale) {
    long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int sys = blockIdx.y;
    if (s >= g.V || sys >= nsys) return;
    Spinor<double> v;
    load_spinor<double, Si>(reinterpret_cast<const char*>(in) + (size_t)sys * 6 * g.V * Unit<Si>::bytes,
                            in_scale ? in_scale + (size_t)sys * g.V : nullptr, g.V, s, v);
    store_spinor<double, So>(reinterpret_cast<char*>(out) + (size_t)sys * 6 * g.V * Unit<So>::bytes,
                             out_scale ? out_scale + (size_t)sys * g.V : nullptr, g.V, s, v);
}

}  // namespace

// Even-odd site inverses: thread h takes the site of the requested parity in the pair (2h, 2h+1)
// (one even and one odd site, since the block x-extent is even), forms the
// two chiral blocks A_up + i absmu and A_dn - i absmu of the packed clover
// (A = (m+4) + clover, Hermitian) and inverts each by Gauss-Jordan with
// partial pivoting in FP64.
template <class C>
__global__ void __launch_bounds__(kThreads) k_eo_inverse(Geo g, const void* __restrict__ clover, double absmu,
                                                         int parity, void* inv) {
    const long long h = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long half = g.V / 2;
    if (h >= half) return;
    long long s = 2 * h;
    int c[4];
    site_coords(g, s, c);
    if (((c[0] + c[1] + c[2] + c[3]) & 1) != parity) ++s;
    Clover<double> A;
    load_clover<double, C>(clover, g.V, s, A);
    for (int blk = 0; blk < 2; ++blk) {
        const double* P = A.a + 36 * blk;
        const double tw = blk == 0 ? absmu : -absmu;
        cplx<double> M[6][6], X[6][6];
        for (int i = 0; i < 6; ++i)
            for (int j = 0; j < 6; ++j) {
                M[i][j] = cmk(0.0, 0.0);
                X[i][j] = cmk(i == j ? 1.0 : 0.0, 0.0);
            }
        for (int i = 0; i < 6; ++i) M[i][i] = cmk(P[i], tw);
        int k = 6;
        for (int i = 0; i < 6; ++i)
            for (int j = i + 1; j < 6; ++j) {
                M[i][j] = cmk(P[k], P[k + 1]);
                M[j][i] = cmk(P[k], -P[k + 1]);
                k += 2;
            }
        for (int col = 0; col < 6; ++col) {
            int p = col;
            double best = M[col][col].re * M[col][col].re + M[col][col].im * M[col][col].im;
            for (int i = col + 1; i < 6; ++i) {
                const double m2 = M[i][col].re * M[i][col].re + M[i][col].im * M[i][col].im;
                if (m2 > best) {
                    best = m2;
                    p = i;
                }
            }
            if (p != col)
                for (int j = 0; j < 6; ++j) {
                    cplx<double> t = M[col][j];
                    M[col][j] = M[p][j];
                    M[p][j] = t;
                    t = X[col][j];
                    X[col][j] = X[p][j];
                    X[p][j] = t;
                }
            const cplx<double> d = M[col][col];
            const double dn = 1.0 / (d.re * d.re + d.im * d.im);
            const cplx<double> di = cmk(d.re * dn, -d.im * dn);
            for (int j = 0; j < 6; ++j) {
                M[col][j] = di * M[col][j];
                X[col][j] = di * X[col][j];
            }
            for (int i = 0; i < 6; ++i) {
                if (i == col) continue;
                const cplx<double> f = M[i][col];
                for (int j = 0; j < 6; ++j) {
                    M[i][j] = M[i][j] - f * M[col][j];
                    X[i][j] = X[i][j] - f * X[col][j];
                }
            }
        }
        for (int u = 0; u < 18; ++u) {
            const int e0 = 2 * u, e1 = 2 * u + 1;
            const double w[4] = {X[e0 / 6][e0 % 6].re, X[e0 / 6][e0 % 6].im, X[e1 / 6][e1 % 6].re,
                                 X[e1 / 6][e1 % 6].im};
            Unit<C>::store(inv, (size_t)(18 * blk + u) * half + h, w);
        }
    }
}

#define TM_DISPATCH_PREC(P, T, ...)                  \
    switch (P) {                                     \
        case P_F64: { typedef double T; __VA_ARGS__; break; } \
        case P_F32: { typedef float T; __VA_ARGS__; break; }  \
        case P_F16: { typedef f16 T; __VA_ARGS__; break; }    \
        default: { typedef bf16 T; __VA_ARGS__; break; }      \
    }

hipError_t launch_link_ingest(const Geo& g, Prec G, const void* Ucanon, void* links, unsigned* stats,
                              hipStream_t st) {
    TM_DISPATCH_PREC(G, T, hipLaunchKernelGGL(k_link_ingest<T>, dim3(grid_for(g.V)), dim3(kThreads), 0, st, g,
                                              (const double*)Ucanon, links, stats));
    return hipGetLastError();
}

hipError_t launch_clover_build(const Geo& g, Prec C, const void* Ucanon, double m4, double csw, void* clover,
                               hipStream_t st) {
    if (C == P_F16 || C == P_BF16) return hipErrorInvalidValue;
    TM_DISPATCH_PREC(C, T, hipLaunchKernelGGL(k_clover_build<T>, dim3(grid_for(g.V)), dim3(kThreads), 0, st, g,
                                              (const double*)Ucanon, m4, csw, clover));
    return hipGetLastError();
}

hipError_t launch_clover_to_f32(const Geo& g, const void* clover64, void* clover32, hipStream_t st) {
    const long long n = 18 * g.V;
    hipLaunchKernelGGL(k_clover_to_f32, dim3(grid_for(n)), dim3(kThreads), 0, st, n,
                       static_cast<const double*>(clover64), static_cast<float*>(clover32));
    return hipGetLastError();
}

hipError_t launch_spinor_import(const Geo& g, const SpinorBuf& dst, const void* canon, unsigned* flag,
                                hipStream_t st) {
    dim3 grid(grid_for(g.V), dst.nsys);
    TM_DISPATCH_PREC(dst.prec, T, hipLaunchKernelGGL(k_spinor_import<T>, grid, dim3(kThreads), 0, st, g, dst.nsys,
                                                     (const double*)canon, dst.data, dst.scale, flag));
    return hipGetLastError();
}

hipError_t launch_spinor_export(const Geo& g, const SpinorBuf& src, void* canon, hipStream_t st) {
    dim3 grid(grid_for(g.V), src.nsys);
    TM_DISPATCH_PREC(src.prec, T, hipLaunchKernelGGL(k_spinor_export<T>, grid, dim3(kThreads), 0, st, g, src.nsys,
                                                     src.data, src.scale, (double*)canon));
    return hipGetLastError();
}

hipError_t launch_spinor_convert(const Geo& g, const SpinorBuf& src, const SpinorBuf& dst, hipStream_t st) {
    dim3 grid(grid_for(g.V), src.nsys);
    TM_DISPATCH_PREC(src.prec, Ti,
                     TM_DISPATCH_PREC(dst.prec, To,
                                      hipLaunchKernelGGL((k_spinor_convert<Ti, To>), grid, dim3(kThreads), 0, st, g,
                                                         src.nsys, src.data, src.scale, dst.data, dst.scale)));
    return hipGetLastError();
}

hipError_t launch_eo_inverse(const Geo& g, Prec C, const void* clover, double absmu, int parity, void* inv,
                             hipStream_t st) {
    if (C != P_F64 && C != P_F32) return hipErrorInvalidValue;
    const long long half = g.V / 2;
    const unsigned nb = (unsigned)((half + kThreads - 1) / kThreads);
    TM_DISPATCH_PREC(C, T, hipLaunchKernelGGL(k_eo_inverse<T>, dim3(nb > 0 ? nb : 1), dim3(kThreads), 0, st, g,
                                              clover, absmu, parity, inv));
    return hipGetLastError();
}

}  // namespace tmsap
