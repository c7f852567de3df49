// The twisted-mass Wilson-clover operator on the whole lattice
// (section 2.1): out = [(m+4) + C + i mu Gamma5] psi
//   - 1/2 sum_mu [(1 - gamma_mu) U_mu(x) psi(x+mu) + (1 + gamma_mu) U_mu(x-mu)^+ psi(x-mu)].
// One thread per site; spin projection to half spinors before the SU(3)
// products; every field is read structure-of-arrays so a wavefront's loads
// are contiguous.
#include <type_traits>

#include "tm_internal.h"

namespace tmsap {

namespace {

constexpr int kThreads = 256;

// Link from its first two rows, stored as 12 reals (row-major, re/im pairs); third row rebuilt.
template <class R>
__device__ inline void link_from_rows(const R* u, Link<R>& L) {
    L.u[0][0] = cmk(u[0], u[1]);
    L.u[0][1] = cmk(u[2], u[3]);
    L.u[0][2] = cmk(u[4], u[5]);
    L.u[1][0] = cmk(u[6], u[7]);
    L.u[1][1] = cmk(u[8], u[9]);
    L.u[1][2] = cmk(u[10], u[11]);
    complete_su3(L);
}

template <class Si, class So, class G, class C, class R>
__global__ void __launch_bounds__(kThreads) k_dirac(DiracArgs a) {
    const Geo& g = a.g;
    // workgroups of one XCD on consecutive tiles (their neighbours' spinors and links share an L2)
    long long s = xcd_swizzle(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (s >= g.V) return;
    int nf[4], nbk[4], par;
    unsigned wrap;
    tiled_neighbours(g, s, nf, nbk, &wrap, &par);
    Clover<R> A;
    load_clover<R, C>(a.clover, g.V, s, A);
    // FP32 spinors and links: the 8 links of the site's hops (two rows each) are loaded once
    // for all systems.  The other forms reload them per system: holding them takes the FP64
    // and the FP16 / BF16 kernels to one wavefront per SIMD, which costs more than the loads.
    constexpr bool kHold = std::is_same<Si, float>::value && std::is_same<G, float>::value &&
                           std::is_same<R, float>::value;
    R lr[kHold ? 8 : 1][12];
    if constexpr (kHold) {
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) {
            const size_t b = (size_t)mu * 3 * g.V;
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                Unit<G>::load(a.links, b + (size_t)q * g.V + s, &lr[2 * mu][4 * q]);
                Unit<G>::load(a.links, b + (size_t)q * g.V + nbk[mu], &lr[2 * mu + 1][4 * q]);
            }
        }
    }
    const size_t in_stride = (size_t)6 * g.V * Unit<Si>::bytes;
    const size_t out_stride = (size_t)6 * g.V * Unit<So>::bytes;
    for (int sys = 0; sys < a.nsys; ++sys) {
        const void* in = reinterpret_cast<const char*>(a.in) + sys * in_stride;
        const float* isc = a.in_scale ? a.in_scale + (size_t)sys * g.V : nullptr;
        Spinor<R> acc;
#pragma unroll
        for (int i = 0; i < 12; ++i) acc.v[i] = cmk<R>(0, 0);
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) {
            Link<R> L;
            Spinor<R> p;
            if constexpr (kHold)
                link_from_rows(lr[2 * mu], L);
            else
                load_link<R, G>(a.links, g.V, s, mu, L);
            load_spinor<R, Si>(in, isc, g.V, nf[mu], p);
            {  // boundary phase (1 for hops inside the lattice), branch-free: fewer registers
                const bool w = wrap & (1u << mu);
                const R re = w ? (R)g.bcr[mu] : (R)1, im = w ? (R)g.bci[mu] : (R)0;
#pragma unroll
                for (int i = 0; i < 12; ++i) p.v[i] = cmk(re * p.v[i].re - im * p.v[i].im, re * p.v[i].im + im * p.v[i].re);
            }
            hop_forward(mu, L, p, (R)1, acc);
            if constexpr (kHold)
                link_from_rows(lr[2 * mu + 1], L);
            else
                load_link<R, G>(a.links, g.V, nbk[mu], mu, L);
            load_spinor<R, Si>(in, isc, g.V, nbk[mu], p);
            {
                const bool w = wrap & (16u << mu);
                const R re = w ? (R)g.bcr[mu] : (R)1, im = w ? -(R)g.bci[mu] : (R)0;
#pragma unroll
                for (int i = 0; i < 12; ++i) p.v[i] = cmk(re * p.v[i].re - im * p.v[i].im, re * p.v[i].im + im * p.v[i].re);
            }
            hop_backward(mu, L, p, (R)1, acc);
        }
        Spinor<R> self, out;
        load_spinor<R, Si>(in, isc, g.V, s, self);
        clover_apply(A, (R)(a.mu[sys] + g.mu_shift[par]), self, out);
#pragma unroll
        for (int i = 0; i < 12; ++i) out.v[i] = out.v[i] - (R)0.5 * acc.v[i];
        store_spinor<R, So>(reinterpret_cast<char*>(a.out) + sys * out_stride,
                            a.out_scale ? a.out_scale + (size_t)sys * g.V : nullptr, g.V, s, out);
    }
}

// FP64 links on 4^4 tiles (one tile per workgroup): the kernel above reloads the eight links of
// a site for every system, since at FP64 holding them leaves no registers, and those reloads are
// most of its HBM traffic (80 GB per 6-system application at 48^3x96 against 22 GB of fields).
// Here the workgroup stages its tile's own links (two rows each, 96 KiB) in LDS once, and every
// system takes its forward links there.  The backward links U_mu(x - mu) stay loads from memory:
// inside the tile they are the links just staged, still in L2, and read from LDS as well they
// made the compiler spill a kilobyte per lane.
template <class Si, class So, class C>
__global__ void __launch_bounds__(kThreads) k_dirac_lk(DiracArgs a) {
    __shared__ double2 lk[4][6][kThreads];  // [mu][row-major pair][site in tile]
    const Geo& g = a.g;
    const long long tile = xcd_swizzle(blockIdx.x, gridDim.x);
    const int l = threadIdx.x;
    const long long s = tile * kThreads + l;  // V is a multiple of the tile size
    const double2* src = reinterpret_cast<const double2*>(a.links);
#pragma unroll
    for (int mu = 0; mu < 4; ++mu)
#pragma unroll
        for (int q = 0; q < 3; ++q) {  // unit q of a link holds 4 reals: pairs 2q and 2q+1
            const size_t u = ((size_t)mu * 3 + q) * g.V + s;
            lk[mu][2 * q][l] = src[2 * u];
            lk[mu][2 * q + 1][l] = src[2 * u + 1];
        }
    int nf[4], nbk[4], par;
    unsigned wrap;
    tiled_neighbours(g, s, nf, nbk, &wrap, &par);
    Clover<double> A;
    load_clover<double, C>(a.clover, g.V, s, A);
    __syncthreads();
    const size_t in_stride = (size_t)6 * g.V * Unit<Si>::bytes;
    const size_t out_stride = (size_t)6 * g.V * Unit<So>::bytes;
    for (int sys = 0; sys < a.nsys; ++sys) {
        const void* in = reinterpret_cast<const char*>(a.in) + sys * in_stride;
        const float* isc = a.in_scale ? a.in_scale + (size_t)sys * g.V : nullptr;
        // the thread index again through a barrier the compiler cannot see through: the LDS reads
        // of the links do not depend on the system, and hoisted out of this loop they would be
        // held in registers
        int lx = l;
        asm volatile("" : "+v"(lx));
        Spinor<double> acc;
#pragma unroll
        for (int i = 0; i < 12; ++i) acc.v[i] = cmk(0.0, 0.0);
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) {
            Link<double> L;
            Spinor<double> p;
            {
                double u[12];
#pragma unroll
                for (int k = 0; k < 6; ++k) {
                    const double2 t = lk[mu][k][lx];
                    u[2 * k] = t.x;
                    u[2 * k + 1] = t.y;
                }
                link_from_rows(u, L);
            }
            load_spinor<double, Si>(in, isc, g.V, nf[mu], p);
            {  // boundary phase (1 for hops inside the lattice)
                const bool w = wrap & (1u << mu);
                const double re = w ? g.bcr[mu] : 1.0, im = w ? g.bci[mu] : 0.0;
#pragma unroll
                for (int i = 0; i < 12; ++i) p.v[i] = cmk(re * p.v[i].re - im * p.v[i].im, re * p.v[i].im + im * p.v[i].re);
            }
            hop_forward(mu, L, p, 1.0, acc);
            load_link<double, double>(a.links, g.V, nbk[mu], mu, L);
            load_spinor<double, Si>(in, isc, g.V, nbk[mu], p);
            {
                const bool w = wrap & (16u << mu);
                const double re = w ? g.bcr[mu] : 1.0, im = w ? -g.bci[mu] : 0.0;
#pragma unroll
                for (int i = 0; i < 12; ++i) p.v[i] = cmk(re * p.v[i].re - im * p.v[i].im, re * p.v[i].im + im * p.v[i].re);
            }
            hop_backward(mu, L, p, 1.0, acc);
        }
        Spinor<double> self, out;
        load_spinor<double, Si>(in, isc, g.V, s, self);
        clover_apply(A, a.mu[sys] + g.mu_shift[par], self, out);
#pragma unroll
        for (int i = 0; i < 12; ++i) out.v[i] = out.v[i] - 0.5 * acc.v[i];
        store_spinor<double, So>(reinterpret_cast<char*>(a.out) + sys * out_stride,
                                 a.out_scale ? a.out_scale + (size_t)sys * g.V : nullptr, g.V, s, out);
    }
}

template <class Si, class So, class G, class C, class R>
hipError_t run(const DiracArgs& a, hipStream_t st) {
    unsigned grid = (unsigned)((a.g.V + kThreads - 1) / kThreads);
    if constexpr (std::is_same<R, double>::value && std::is_same<G, double>::value) {
        const int* lb = a.g.lb;
        if (lb[0] == 4 && lb[1] == 4 && lb[2] == 4 && lb[3] == 4 && a.g.V % kThreads == 0) {
            hipLaunchKernelGGL((k_dirac_lk<Si, So, C>), dim3(grid), dim3(kThreads), 0, st, a);
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL((k_dirac<Si, So, G, C, R>), dim3(grid), dim3(kThreads), 0, st, a);
    return hipGetLastError();
}

}  // namespace

// Supported combinations (spinor in, spinor out, links, clover, compute):
//   all FP64; all FP32; FP16/BF16 spinors and links with FP32 clover and
//   compute; FP32/FP16/BF16 input with FP64 output, links, clover and compute
//   (the FP64 operator applied to a low-precision preconditioned vector);
//   FP16/BF16 input with FP32 output, links, clover and compute.
hipError_t launch_dirac(const DiracArgs& a, Prec in_p, Prec out_p, Prec link_p, Prec clover_p, Prec compute,
                        hipStream_t st) {
    if (compute == P_F32) {  // 4^4 tiles: the tiled kernel of tm_sap.hip
        const hipError_t e = launch_dirac_44(a, in_p, out_p, link_p, clover_p, st);
        if (e != hipErrorNotSupported) return e;
    }
#define TM_CASE(PI, PO, PL, PC, PR, TI, TO, TL, TC, TR)                                      \
    if (in_p == PI && out_p == PO && link_p == PL && clover_p == PC && compute == PR) \
        return run<TI, TO, TL, TC, TR>(a, st);
    TM_CASE(P_F64, P_F64, P_F64, P_F64, P_F64, double, double, double, double, double)
    TM_CASE(P_F32, P_F32, P_F32, P_F32, P_F32, float, float, float, float, float)
    TM_CASE(P_F16, P_F16, P_F16, P_F32, P_F32, f16, f16, f16, float, float)
    TM_CASE(P_BF16, P_BF16, P_BF16, P_F32, P_F32, bf16, bf16, bf16, float, float)
    TM_CASE(P_F32, P_F64, P_F64, P_F64, P_F64, float, double, double, double, double)
    TM_CASE(P_F16, P_F64, P_F64, P_F64, P_F64, f16, double, double, double, double)
    TM_CASE(P_BF16, P_F64, P_F64, P_F64, P_F64, bf16, double, double, double, double)
    TM_CASE(P_F16, P_F32, P_F32, P_F32, P_F32, f16, float, float, float, float)
    TM_CASE(P_BF16, P_F32, P_F32, P_F32, P_F32, bf16, float, float, float, float)
#undef TM_CASE
    return hipErrorInvalidValue;
}

}  // namespace tmsap
