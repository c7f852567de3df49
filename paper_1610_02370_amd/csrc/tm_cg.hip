// Kernels of the even-odd reduced operator and of CG on its normal
// equations (the CG comparison of section 3, eq. (oereduced)).
//
// Vectors live on one parity: with the tile's x-extent even, the sites 2h and
// 2h+1 of the tiled layout are one even and one odd site, so a parity vector
// is a compact field [nsys][6 units][V/2] indexed by h = s / 2.  FP64 only:
// the CG is the plain FP64 baseline.
#include "tm_internal.h"

namespace tmsap {

namespace {

constexpr int kThreads = 256;

__device__ inline int site_parity_tiled(const Geo& g, unsigned s) {
    const unsigned Vb = (unsigned)g.Vb;
    const unsigned blk = s / Vb;
    unsigned l = s - blk * Vb, tb = blk;
    int sum = 0;
#pragma unroll
    for (int a = 3; a >= 0; --a) {
        const unsigned lb = (unsigned)g.lb[a], nb = (unsigned)g.nb[a];
        const unsigned lq = l / lb, bq = tb / nb;
        sum += (int)(tb - bq * nb) * g.lb[a] + (int)(l - lq * lb);
        l = lq;
        tb = bq;
    }
    return sum & 1;
}

__device__ inline void gamma5(Spinor<double>& v) {
#pragma unroll
    for (int i = 6; i < 12; ++i) v.v[i] = -v.v[i];
}

// out_p = (D_pp^-1)? [ hop_sign * H in_hop + D_pp in_diag + add_sign * in_add ], H = -1/2 sum of hops
// between the parities, D_pp = (m+4) + clover + i mu Gamma5 on parity p; the Gamma5 flags multiply
// the hop input, the diagonal input and the output.
template <bool HOP, bool DIAG, bool INV, bool G5HOP>
__global__ void __launch_bounds__(kThreads) k_parity_op(ParityArgs a) {
    const Geo& g = a.g;
    const long long half = g.V / 2;
    const long long h = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= half) return;
    unsigned s = 2u * (unsigned)h;
    if (site_parity_tiled(g, s) != a.p) ++s;
    int nf[4], nbk[4], par = a.p;
    unsigned wrap = 0;
    if (HOP) tiled_neighbours(g, s, nf, nbk, &wrap, &par);
    const size_t vs = (size_t)6 * half;  // units per system
    for (int sys = 0; sys < a.nsys; ++sys) {
        const double mu = a.mu_sign * (a.mu[sys] + g.mu_shift[a.p]);
        Spinor<double> v;
#pragma unroll
        for (int i = 0; i < 12; ++i) v.v[i] = cmk(0.0, 0.0);
        if (DIAG) {
            Spinor<double> d;
            load_spinor<double, double>(a.in_diag + sys * vs * 4, nullptr, half, h, d);
            if (a.g5_diag) gamma5(d);
            Clover<double> A;
            load_clover<double, double>(a.clover, g.V, s, A);
            clover_acc(A, mu, d, v);
        }
        if (HOP) {
            const double* in = a.in_hop + sys * vs * 4;
            Spinor<double> acc;
#pragma unroll
            for (int i = 0; i < 12; ++i) acc.v[i] = cmk(0.0, 0.0);
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                Link<double> L;
                Spinor<double> p;
                load_link<double, double>(a.links, g.V, s, m, L);
                load_spinor<double, double>(in, nullptr, half, nf[m] >> 1, p);
                if (G5HOP) gamma5(p);
                {  // boundary phase (1 inside the lattice), branch-free: fewer registers
                    const bool w = wrap & (1u << m);
                    const double re = w ? g.bcr[m] : 1.0, im = w ? g.bci[m] : 0.0;
#pragma unroll
                    for (int i = 0; i < 12; ++i)
                        p.v[i] = cmk(re * p.v[i].re - im * p.v[i].im, re * p.v[i].im + im * p.v[i].re);
                }
                hop_forward(m, L, p, 1.0, acc);
                load_link<double, double>(a.links, g.V, nbk[m], m, L);
                load_spinor<double, double>(in, nullptr, half, nbk[m] >> 1, p);
                if (G5HOP) gamma5(p);
                {
                    const bool w = wrap & (16u << m);
                    const double re = w ? g.bcr[m] : 1.0, im = w ? -g.bci[m] : 0.0;
#pragma unroll
                    for (int i = 0; i < 12; ++i)
                        p.v[i] = cmk(re * p.v[i].re - im * p.v[i].im, re * p.v[i].im + im * p.v[i].re);
                }
                hop_backward(m, L, p, 1.0, acc);
            }
#pragma unroll
            for (int i = 0; i < 12; ++i) v.v[i] = v.v[i] + (-0.5 * a.hop_sign) * acc.v[i];
        }
        if (a.in_add) {
            Spinor<double> d;
            load_spinor<double, double>(a.in_add + sys * vs * 4, nullptr, half, h, d);
#pragma unroll
            for (int i = 0; i < 12; ++i) v.v[i] = v.v[i] + a.add_sign * d.v[i];
        }
        if (INV) {
            Spinor<double> t;
            eo_inverse_apply<double, double>(a.inv[a.sel[sys]], half, h, mu < 0, v, t);
            v = t;
        }
        if (a.g5_out) gamma5(v);
        store_spinor<double, double>(a.out + sys * vs * 4, nullptr, half, h, v);
    }
}

// canonical complex128 [nsys][V][4][3] <-> the two compact parity fields
__global__ void __launch_bounds__(kThreads) k_parity_import(Geo g, int nsys, const double* __restrict__ canon,
                                                            double* even, double* odd, unsigned* flag) {
    const long long half = g.V / 2;
    const long long h = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int sys = blockIdx.y;
    if (h >= half || sys >= nsys) return;
    for (int k = 0; k < 2; ++k) {
        const unsigned s = 2u * (unsigned)h + k;
        int c[4];
        site_coords(g, s, c);
        const double2* p = reinterpret_cast<const double2*>(canon) + ((size_t)sys * g.V + lex_site(g, c)) * 12;
        Spinor<double> v;
        bool bad = false;
        for (int i = 0; i < 12; ++i) {
            const double2 t = p[i];
            v.v[i] = cmk(t.x, t.y);
            bad |= !isfinite(t.x) || !isfinite(t.y);
        }
        if (bad) atomicOr(flag, 1u);
        double* dst = ((c[0] + c[1] + c[2] + c[3]) & 1) ? odd : even;
        store_spinor<double, double>(dst + (size_t)sys * 6 * half * 4, nullptr, half, h, v);
    }
}

__global__ void __launch_bounds__(kThreads) k_parity_export(Geo g, int nsys, const double* __restrict__ even,
                                                            const double* __restrict__ odd, double* canon) {
    const long long half = g.V / 2;
    const long long h = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int sys = blockIdx.y;
    if (h >= half || sys >= nsys) return;
    for (int k = 0; k < 2; ++k) {
        const unsigned s = 2u * (unsigned)h + k;
        int c[4];
        site_coords(g, s, c);
        const double* src = ((c[0] + c[1] + c[2] + c[3]) & 1) ? odd : even;
        Spinor<double> v;
        load_spinor<double, double>(src + (size_t)sys * 6 * half * 4, nullptr, half, h, v);
        double2* p = reinterpret_cast<double2*>(canon) + ((size_t)sys * g.V + lex_site(g, c)) * 12;
        for (int i = 0; i < 12; ++i) p[i] = make_double2(v.v[i].re, v.v[i].im);
    }
}

// y = a[sys] x + b[sys] y on compact fields (a, b real, per system)
__global__ void __launch_bounds__(kThreads) k_axpby(const double* __restrict__ x, const double* a, double* y,
                                                    const double* b, long long n_per_sys) {
    const int sys = blockIdx.y;
    const double fa = a[sys], fb = b[sys];
    const double* xs = x + (size_t)sys * n_per_sys;
    double* ys = y + (size_t)sys * n_per_sys;
    for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < n_per_sys;
         i += (long long)gridDim.x * kThreads)
        ys[i] = fa * xs[i] + fb * ys[i];
}

// CG scalars per system (frozen systems take zero steps):
//   mode 0: alpha = gamma / qq,  neg = -alpha
//   mode 1: beta = gnew / gamma, gamma = gnew
__global__ void k_cg_scalars(int mode, int nsys, unsigned long long frozen, double* gamma, const double* v,
                             double* out, double* neg) {
    const int k = threadIdx.x;
    if (k >= nsys) return;
    const bool off = (frozen >> k) & 1ull;
    if (mode == 0) {
        const double a = (off || !(v[k] > 0)) ? 0.0 : gamma[k] / v[k];
        out[k] = a;
        neg[k] = -a;
    } else {
        const double b = (off || !(gamma[k] > 0)) ? 0.0 : v[k] / gamma[k];
        out[k] = b;
        if (!off) gamma[k] = v[k];
    }
}

}  // namespace

hipError_t launch_parity_op(const ParityArgs& a, hipStream_t st) {
    const long long half = a.g.V / 2;
    const dim3 grid((unsigned)((half + kThreads - 1) / kThreads)), blk(kThreads);
    const bool hop = a.in_hop != nullptr, diag = a.in_diag != nullptr, inv = a.do_inv != 0;
    if (hop && !diag && inv && a.g5_hop)
        hipLaunchKernelGGL((k_parity_op<true, false, true, true>), grid, blk, 0, st, a);
    else if (hop && !diag && inv)
        hipLaunchKernelGGL((k_parity_op<true, false, true, false>), grid, blk, 0, st, a);
    else if (hop && diag && !inv && !a.g5_hop)
        hipLaunchKernelGGL((k_parity_op<true, true, false, false>), grid, blk, 0, st, a);
    else if (hop && !diag && !inv && !a.g5_hop)
        hipLaunchKernelGGL((k_parity_op<true, false, false, false>), grid, blk, 0, st, a);
    else if (!hop && !diag && inv)
        hipLaunchKernelGGL((k_parity_op<false, false, true, false>), grid, blk, 0, st, a);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_parity_import(const Geo& g, int nsys, const void* canon, double* even, double* odd, unsigned* flag,
                                hipStream_t st) {
    const long long half = g.V / 2;
    hipLaunchKernelGGL(k_parity_import, dim3((unsigned)((half + kThreads - 1) / kThreads), nsys), dim3(kThreads), 0,
                       st, g, nsys, (const double*)canon, even, odd, flag);
    return hipGetLastError();
}

hipError_t launch_parity_export(const Geo& g, int nsys, const double* even, const double* odd, void* canon,
                                hipStream_t st) {
    const long long half = g.V / 2;
    hipLaunchKernelGGL(k_parity_export, dim3((unsigned)((half + kThreads - 1) / kThreads), nsys), dim3(kThreads), 0,
                       st, g, nsys, even, odd, (double*)canon);
    return hipGetLastError();
}

hipError_t launch_axpby(const double* x, const double* a, double* y, const double* b, int nsys, long long n_per_sys,
                        hipStream_t st) {
    const long long nb = (n_per_sys + kThreads - 1) / kThreads;
    hipLaunchKernelGGL(k_axpby, dim3((unsigned)(nb < 4096 ? nb : 4096), nsys), dim3(kThreads), 0, st, x, a, y, b,
                       n_per_sys);
    return hipGetLastError();
}

hipError_t launch_cg_scalars(int mode, int nsys, unsigned long long frozen, double* gamma, const double* v,
                             double* out, double* neg, hipStream_t st) {
    hipLaunchKernelGGL(k_cg_scalars, dim3(1), dim3(64), 0, st, mode, nsys, frozen, gamma, v, out, neg);
    return hipGetLastError();
}

}  // namespace tmsap
