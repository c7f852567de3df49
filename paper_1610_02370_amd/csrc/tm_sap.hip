// One half-sweep of the red-black multiplicative Schwarz smoother
// (section 2.4): for every Schwarz block of one colour,
//   r_B = b_B - (D x)_B                      (hops from the other colour read from HBM)
//   e_B = MR(D_BB, r_B), mr_iters steps from e = 0
//   x_B += e_B
// D_BB is D restricted to the block (Dirichlet cuts at the faces).  One
// workgroup owns one block, one thread one site; the vector being multiplied
// is exchanged through LDS, and the MR inner products are reduced across the
// wavefront with cross-lane shuffles and across the workgroup through LDS.
// Blocks of one colour do not couple, so all workgroups of a launch are
// independent; the colour-to-colour dependency is the launch boundary.
#include "tm_internal.h"

namespace tmsap {

namespace {

template <class R>
__device__ inline R wave_sum(R v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum of three values over the workgroup; every thread gets the result.
template <class R>
__device__ inline void block_sum3(R* red, R& a, R& b, R& c) {
    a = wave_sum(a);
    b = wave_sum(b);
    c = wave_sum(c);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    if (lane == 0) {
        red[4 * w] = a;
        red[4 * w + 1] = b;
        red[4 * w + 2] = c;
    }
    __syncthreads();
    a = b = c = (R)0;
    for (int i = 0; i < nw; ++i) {
        a += red[4 * i];
        b += red[4 * i + 1];
        c += red[4 * i + 2];
    }
}

template <class R>
__device__ inline void lds_put(R* sh, int stride, int l, const Spinor<R>& p) {
#pragma unroll
    for (int i = 0; i < 12; ++i) {
        sh[(2 * i) * stride + l] = p.v[i].re;
        sh[(2 * i + 1) * stride + l] = p.v[i].im;
    }
}

template <class R>
__device__ inline void lds_get(const R* sh, int stride, int l, Spinor<R>& p) {
#pragma unroll
    for (int i = 0; i < 12; ++i) p.v[i] = cmk(sh[(2 * i) * stride + l], sh[(2 * i + 1) * stride + l]);
}

template <class S, class G, class C, class R, int MAXT>
__global__ void __launch_bounds__(MAXT) k_sap_half(SapArgs a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const Geo& g = a.g;
    const int Vb = g.Vb;
    const int l = threadIdx.x;
    const int nt = blockDim.x;
    const bool active = l < Vb;
    R* sh = reinterpret_cast<R*>(smem_raw);
    R* red = sh + 24 * nt;

    // ---- which block: the blockIdx.x-th block of this colour
    const int half3 = g.nb[3] >> 1;
    int j = blockIdx.x;
    const int k3 = j % half3;
    j /= half3;
    const int B2 = j % g.nb[2];
    j /= g.nb[2];
    const int B1 = j % g.nb[1];
    const int B0 = j / g.nb[1];
    const int B3 = 2 * k3 + ((a.colour + B0 + B1 + B2) & 1);
    const int Bc[4] = {B0, B1, B2, B3};
    const long long blk = (((long long)B0 * g.nb[1] + B1) * g.nb[2] + B2) * g.nb[3] + B3;
    const long long s = blk * Vb + (active ? l : 0);

    // ---- neighbours: local index inside the block, or the global site outside it
    int Lc[4];
    {
        int t = active ? l : 0;
        for (int ax = 3; ax >= 0; --ax) {
            Lc[ax] = t % g.lb[ax];
            t /= g.lb[ax];
        }
    }
    int lstride[4];
    lstride[3] = 1;
    lstride[2] = g.lb[3];
    lstride[1] = g.lb[3] * g.lb[2];
    lstride[0] = g.lb[3] * g.lb[2] * g.lb[1];
    int nlf[4], nlb[4];
    long long ngf[4], ngb[4];
    R sgf[4], sgb[4];
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        const int ax = axis_of(mu);
        int c[4];
        for (int q = 0; q < 4; ++q) c[q] = Bc[q] * g.lb[q] + Lc[q];
        sgf[mu] = sgb[mu] = (R)1;
        if (Lc[ax] + 1 < g.lb[ax]) {
            nlf[mu] = l + lstride[ax];
            ngf[mu] = 0;
        } else {
            nlf[mu] = -1;
            int n[4] = {c[0], c[1], c[2], c[3]};
            if (++n[ax] == g.d[ax]) {
                n[ax] = 0;
                if (mu == 0 && g.antiperiodic_t) sgf[mu] = (R)-1;
            }
            ngf[mu] = coords_site(g, n);
        }
        if (Lc[ax] > 0) {
            nlb[mu] = l - lstride[ax];
            ngb[mu] = 0;
        } else {
            nlb[mu] = -1;
            int n[4] = {c[0], c[1], c[2], c[3]};
            if (--n[ax] < 0) {
                n[ax] = g.d[ax] - 1;
                if (mu == 0 && g.antiperiodic_t) sgb[mu] = (R)-1;
            }
            ngb[mu] = coords_site(g, n);
        }
    }
    const long long s0 = blk * Vb;

    Clover<R> A;
    if (active) load_clover<R, C>(a.clover, g.V, s, A);

    const size_t stride = (size_t)6 * g.V * Unit<S>::bytes;
    const int sys_begin = blockIdx.y * a.sys_tile;
    const int sys_end = min(a.nsys, sys_begin + a.sys_tile);

    for (int sys = sys_begin; sys < sys_end; ++sys) {
        const R mu_tw = (R)a.mu[sys];
        const void* bb = reinterpret_cast<const char*>(a.b) + sys * stride;
        void* xx = reinterpret_cast<char*>(a.x) + sys * stride;
        const float* bsc = a.b_scale ? a.b_scale + (size_t)sys * g.V : nullptr;
        float* xsc = a.x_scale ? a.x_scale + (size_t)sys * g.V : nullptr;

        Spinor<R> r, xv;
#pragma unroll
        for (int i = 0; i < 12; ++i) xv.v[i] = cmk<R>(0, 0);
        if (active) load_spinor<R, S>(bb, bsc, g.V, s, r);
        if (!(a.own_zero && a.halo_zero)) {
            // r = b - D x on the block: diagonal and in-block hops from LDS,
            // hops from the neighbouring blocks straight from memory.  When x
            // is still zero on this colour only the halo hops remain.
            const bool own = !a.own_zero;
            if (own) {
                if (active) {
                    load_spinor<R, S>(xx, xsc, g.V, s, xv);
                    lds_put(sh, nt, l, xv);
                }
                __syncthreads();
            }
            if (active) {
                Spinor<R> acc, dx;
#pragma unroll
                for (int i = 0; i < 12; ++i) acc.v[i] = cmk<R>(0, 0);
#pragma unroll
                for (int mu = 0; mu < 4; ++mu) {
                    Link<R> Lk;
                    Spinor<R> p;
                    if (nlf[mu] < 0 || own) {
                        load_link<R, G>(a.links, g.V, s, mu, Lk);
                        if (nlf[mu] >= 0)
                            lds_get(sh, nt, nlf[mu], p);
                        else
                            load_spinor<R, S>(xx, xsc, g.V, ngf[mu], p);
                        hop_forward(mu, Lk, p, sgf[mu], acc);
                    }
                    if (nlb[mu] >= 0) {
                        if (own) {
                            lds_get(sh, nt, nlb[mu], p);
                            load_link<R, G>(a.links, g.V, s0 + nlb[mu], mu, Lk);
                            hop_backward(mu, Lk, p, sgb[mu], acc);
                        }
                    } else {
                        load_spinor<R, S>(xx, xsc, g.V, ngb[mu], p);
                        load_link<R, G>(a.links, g.V, ngb[mu], mu, Lk);
                        hop_backward(mu, Lk, p, sgb[mu], acc);
                    }
                }
                if (own) {
                    clover_apply(A, mu_tw, xv, dx);
                } else {
#pragma unroll
                    for (int i = 0; i < 12; ++i) dx.v[i] = cmk<R>(0, 0);
                }
#pragma unroll
                for (int i = 0; i < 12; ++i) r.v[i] = r.v[i] - (dx.v[i] - (R)0.5 * acc.v[i]);
            }
            if (own) __syncthreads();
        }

        // ---- minimal residual on D_BB from e = 0
        Spinor<R> e, rho = r;
#pragma unroll
        for (int i = 0; i < 12; ++i) e.v[i] = cmk<R>(0, 0);
        for (int it = 0; it < a.mr_iters; ++it) {
            if (active) lds_put(sh, nt, l, rho);
            __syncthreads();
            Spinor<R> q;
            R qr_re = 0, qr_im = 0, qq = 0;
            if (active) {
                Spinor<R> acc;
#pragma unroll
                for (int i = 0; i < 12; ++i) acc.v[i] = cmk<R>(0, 0);
#pragma unroll
                for (int mu = 0; mu < 4; ++mu) {
                    Link<R> Lk;
                    Spinor<R> p;
                    if (nlf[mu] >= 0) {
                        load_link<R, G>(a.links, g.V, s, mu, Lk);
                        lds_get(sh, nt, nlf[mu], p);
                        hop_forward(mu, Lk, p, sgf[mu], acc);
                    }
                    if (nlb[mu] >= 0) {
                        load_link<R, G>(a.links, g.V, s0 + nlb[mu], mu, Lk);
                        lds_get(sh, nt, nlb[mu], p);
                        hop_backward(mu, Lk, p, sgb[mu], acc);
                    }
                }
                clover_apply(A, mu_tw, rho, q);
#pragma unroll
                for (int i = 0; i < 12; ++i) {
                    q.v[i] = q.v[i] - (R)0.5 * acc.v[i];
                    qr_re += q.v[i].re * rho.v[i].re + q.v[i].im * rho.v[i].im;
                    qr_im += q.v[i].re * rho.v[i].im - q.v[i].im * rho.v[i].re;
                    qq += q.v[i].re * q.v[i].re + q.v[i].im * q.v[i].im;
                }
            }
            block_sum3(red, qr_re, qr_im, qq);
            if (active && qq > (R)0) {
                const cplx<R> alpha = cmk(qr_re / qq, qr_im / qq);
#pragma unroll
                for (int i = 0; i < 12; ++i) {
                    e.v[i] = cmad(alpha, rho.v[i], e.v[i]);
                    rho.v[i] = rho.v[i] - alpha * q.v[i];
                }
            }
        }

        if (active) {
#pragma unroll
            for (int i = 0; i < 12; ++i) e.v[i] = e.v[i] + xv.v[i];
            store_spinor<R, S>(xx, xsc, g.V, s, e);
        }
    }
}

template <class S, class G, class C, class R>
hipError_t run(const SapArgs& a, hipStream_t st) {
    const int nt = (a.g.Vb + 63) & ~63;
    const long long nblocks = (long long)a.g.nb[0] * a.g.nb[1] * a.g.nb[2] * a.g.nb[3];
    dim3 grid((unsigned)(nblocks / 2), (unsigned)((a.nsys + a.sys_tile - 1) / a.sys_tile));
    const size_t lds = sap_lds_bytes(a.g.Vb, sizeof(R) == 8 ? P_F64 : P_F32);
    int dev = 0, max_lds = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (e != hipSuccess) return e;
    if (lds > (size_t)max_lds) return hipErrorInvalidConfiguration;
    const void* fn = nt <= 256 ? reinterpret_cast<const void*>(&k_sap_half<S, G, C, R, 256>)
                               : reinterpret_cast<const void*>(&k_sap_half<S, G, C, R, 1024>);
    if (lds > 65536) {
        e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    if (nt <= 256)
        hipLaunchKernelGGL((k_sap_half<S, G, C, R, 256>), grid, dim3(nt), lds, st, a);
    else
        hipLaunchKernelGGL((k_sap_half<S, G, C, R, 1024>), grid, dim3(nt), lds, st, a);
    return hipGetLastError();
}

}  // namespace

size_t sap_lds_bytes(int Vb, Prec compute) {
    const int nt = (Vb + 63) & ~63;
    const size_t rb = compute == P_F64 ? 8 : 4;
    return (24 * (size_t)nt + 4 * 16) * rb;
}

bool sap_supported(Prec sp, Prec lp, Prec cp, Prec r) {
    return (sp == P_F64 && lp == P_F64 && cp == P_F64 && r == P_F64) ||
           (sp == P_F32 && lp == P_F32 && cp == P_F32 && r == P_F32) ||
           (sp == P_F16 && lp == P_F16 && cp == P_F32 && r == P_F32) ||
           (sp == P_BF16 && lp == P_BF16 && cp == P_F32 && r == P_F32);
}

hipError_t launch_sap_half(const SapArgs& a, Prec sp, Prec lp, Prec cp, Prec r, hipStream_t st) {
    if (sp == P_F64 && lp == P_F64 && cp == P_F64 && r == P_F64) return run<double, double, double, double>(a, st);
    if (sp == P_F32 && lp == P_F32 && cp == P_F32 && r == P_F32) return run<float, float, float, float>(a, st);
    if (sp == P_F16 && lp == P_F16 && cp == P_F32 && r == P_F32) return run<f16, f16, float, float>(a, st);
    if (sp == P_BF16 && lp == P_BF16 && cp == P_F32 && r == P_F32) return run<bf16, bf16, float, float>(a, st);
    return hipErrorInvalidValue;
}

}  // namespace tmsap
