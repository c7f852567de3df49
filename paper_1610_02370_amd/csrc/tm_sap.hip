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
#include <cstddef>
#include <cstdlib>
#include <type_traits>

#include "tm_internal.h"
#include "tm_sap_index.h"

namespace tmsap {

namespace {

// TM_SAP_KERNEL=v1 / v2 select the generic kernel or the general-shape FP32
// kernel instead of the 4^4 one (A/B tests).
bool sap_v1_forced() {
    static int forced = -1;
    if (forced < 0) {
        const char* e = getenv("TM_SAP_KERNEL");
        forced = (e && e[0] == 'v' && e[1] == '1') ? 1 : 0;
    }
    return forced == 1;
}

bool sap_v2_forced() {
    static int forced = -1;
    if (forced < 0) {
        const char* e = getenv("TM_SAP_KERNEL");
        forced = (e && e[0] == 'v' && e[1] == '2') ? 1 : 0;
    }
    return forced == 1;
}

template <class R>
__device__ inline R wave_sum(R v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Wavefront sum with DPP row operations (no LDS crossbar): quad and row
// reductions, then row broadcasts; the total ends in lane 63.
template <int CTRL, int ROW_MASK>
__device__ inline float dpp_f(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, ROW_MASK, 0xf,
                                                                   true));
}

template <>
__device__ inline float wave_sum<float>(float v) {
    v += dpp_f<0xb1, 0xf>(v);   // quad_perm [1,0,3,2]
    v += dpp_f<0x4e, 0xf>(v);   // quad_perm [2,3,0,1]
    v += dpp_f<0x114, 0xf>(v);  // row_shr:4
    v += dpp_f<0x118, 0xf>(v);  // row_shr:8
    v += dpp_f<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
    v += dpp_f<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
}

// Smallest normal number.  An MR step is taken only when <q,q> is at least
// this: a block whose residual has (nearly) vanished keeps e, and neither the
// hardware reciprocal nor a flushed division meets a subnormal divisor
// (which would turn the step length into inf or NaN).
template <class R>
__device__ constexpr R min_normal() {
    return sizeof(R) == 8 ? (R)2.2250738585072014e-308 : (R)1.17549435e-38f;
}

// The minimal-residual step's local sums <q, rho> and <q, q> (section 2.4's block
// solver), added one product at a time so that each product is one fused
// multiply-add (a sum of two products added in one step costs a third instruction).
template <class R>
__device__ inline void mr_dots(const Spinor<R>& q, const Spinor<R>& rho, R& qr_re, R& qr_im, R& qq) {
#pragma unroll
    for (int i = 0; i < 12; ++i) {
        qr_re = qr_re + q.v[i].re * rho.v[i].re;
        qr_re = qr_re + q.v[i].im * rho.v[i].im;
        qr_im = qr_im + q.v[i].re * rho.v[i].im;
        qr_im = qr_im - q.v[i].im * rho.v[i].re;
        qq = qq + q.v[i].re * q.v[i].re;
        qq = qq + q.v[i].im * q.v[i].im;
    }
}

// rho -= alpha q as two fused multiply-adds per real component.
template <class R>
__device__ inline void mr_residual_update(cplx<R> alpha, const Spinor<R>& q, Spinor<R>& rho) {
    const cplx<R> na = cmk(-alpha.re, -alpha.im);
#pragma unroll
    for (int i = 0; i < 12; ++i) rho.v[i] = cmad(na, q.v[i], rho.v[i]);
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

// Per-thread geometry of the generic kernel: the thread's site, its
// neighbours as local indices inside the block (-1 when outside) or global
// sites outside it, the hops that cross the lattice boundary (bit mu forward,
// bit 4+mu backward), and the site parity.
template <class R>
struct GenSite {
    long long s, s0;  // site, first site of the block
    int nlf[4], nlb[4];
    long long ngf[4], ngb[4];
    unsigned wrap;
    int parity;  // (t + z + y + x) mod 2 of the global coordinates
};

// The blockIdx.x-th block of colour `colour`, thread l.
template <class R>
__device__ inline void gen_site_setup(const Geo& g, int colour, int l, bool active, GenSite<R>& t) {
    const int Vb = g.Vb;
    const int half3 = g.nb[3] >> 1;
    int j = blockIdx.x;
    const int k3 = j % half3;
    j /= half3;
    const int B2 = j % g.nb[2];
    j /= g.nb[2];
    const int B1 = j % g.nb[1];
    const int B0 = j / g.nb[1];
    const int B3 = 2 * k3 + ((colour + B0 + B1 + B2) & 1);
    const int Bc[4] = {B0, B1, B2, B3};
    const long long blk = (((long long)B0 * g.nb[1] + B1) * g.nb[2] + B2) * g.nb[3] + B3;
    t.s0 = blk * Vb;
    t.s = t.s0 + (active ? l : 0);

    int Lc[4];
    {
        int u = active ? l : 0;
        for (int ax = 3; ax >= 0; --ax) {
            Lc[ax] = u % g.lb[ax];
            u /= g.lb[ax];
        }
    }
    int lstride[4];
    lstride[3] = 1;
    lstride[2] = g.lb[3];
    lstride[1] = g.lb[3] * g.lb[2];
    lstride[0] = g.lb[3] * g.lb[2] * g.lb[1];
    int c[4];
    for (int q = 0; q < 4; ++q) c[q] = Bc[q] * g.lb[q] + Lc[q];
    t.parity = (c[0] + c[1] + c[2] + c[3]) & 1;
    t.wrap = 0;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        const int ax = axis_of(mu);
        if (Lc[ax] + 1 < g.lb[ax]) {
            t.nlf[mu] = l + lstride[ax];
            t.ngf[mu] = 0;
        } else {
            t.nlf[mu] = -1;
            int n[4] = {c[0], c[1], c[2], c[3]};
            if (++n[ax] == g.d[ax]) {
                n[ax] = 0;
                t.wrap |= 1u << mu;
            }
            t.ngf[mu] = coords_site(g, n);
        }
        if (Lc[ax] > 0) {
            t.nlb[mu] = l - lstride[ax];
            t.ngb[mu] = 0;
        } else {
            t.nlb[mu] = -1;
            int n[4] = {c[0], c[1], c[2], c[3]};
            if (--n[ax] < 0) {
                n[ax] = g.d[ax] - 1;
                t.wrap |= 16u << mu;
            }
            t.ngb[mu] = coords_site(g, n);
        }
    }
}

// Links of the block's sites staged in LDS (the FP64 kernel: a workgroup per
// block, one per CU): the two stored rows of each link as 3 units of 4 reals,
// [mu][unit][site]; the third row is rebuilt on use, as from memory.
template <class R, class G>
__device__ inline void lk_stage(const void* links, long long V, long long s, R* lk, int nt, int l) {
#pragma unroll
    for (int u = 0; u < 12; ++u) {
        R v[4];
        Unit<G>::load(links, (size_t)(u / 3) * 3 * V + (size_t)(u % 3) * V + s, v);
        R* d = lk + ((size_t)u * nt + l) * 4;
        d[0] = v[0];
        d[1] = v[1];
        d[2] = v[2];
        d[3] = v[3];
    }
}

template <class R>
__device__ inline void lk_get(const R* lk, int nt, int mu, int n, Link<R>& L) {
    const R* p0 = lk + ((size_t)(3 * mu) * nt + n) * 4;
    const R* p1 = p0 + (size_t)nt * 4;
    const R* p2 = p1 + (size_t)nt * 4;
    L.u[0][0] = cmk(p0[0], p0[1]);
    L.u[0][1] = cmk(p0[2], p0[3]);
    L.u[0][2] = cmk(p1[0], p1[1]);
    L.u[1][0] = cmk(p1[2], p1[3]);
    L.u[1][1] = cmk(p2[0], p2[1]);
    L.u[1][2] = cmk(p2[2], p2[3]);
    complete_su3(L);
}

// Own link (mu) of local site l, from LDS when the links are staged there.
template <bool LC, class R, class G>
__device__ inline void own_link(const SapArgs& a, const R* lk, int nt, long long s, int l, int mu, Link<R>& L) {
    if constexpr (LC)
        lk_get(lk, nt, mu, l, L);
    else
        load_link<R, G>(a.links, a.g.V, s, mu, L);
}

// r = b - D x on the block for one system: diagonal and in-block hops from
// LDS, hops from the neighbouring blocks straight from memory.  When x is
// still zero on this colour only the halo hops remain; xv returns the old x
// (zero when it was not read).  Contains barriers: every thread calls it.
template <class S, class G, class R, bool LC = false>
__device__ inline void gen_residual(const SapArgs& a, const GenSite<R>& t, const Clover<R>& A, R mu_tw, bool active,
                                    R* sh, int nt, int l, const void* bb, const float* bsc, const void* xx,
                                    const float* xsc, Spinor<R>& r, Spinor<R>& xv, const R* lk = nullptr) {
    const Geo& g = a.g;
#pragma unroll
    for (int i = 0; i < 12; ++i) xv.v[i] = cmk<R>(0, 0);
    if (active) load_spinor<R, S>(bb, bsc, g.V, t.s, r);
    if (a.own_zero && a.halo_zero) return;
    const bool own = !a.own_zero;
    if (own) {
        if (active) {
            load_spinor<R, S>(xx, xsc, g.V, t.s, xv);
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
            if (t.nlf[mu] < 0 || own) {
                own_link<LC, R, G>(a, lk, nt, t.s, l, mu, Lk);
                if (t.nlf[mu] >= 0) {
                    lds_get(sh, nt, t.nlf[mu], p);
                } else {
                    load_spinor<R, S>(xx, xsc, g.V, t.ngf[mu], p);
                    if (t.wrap & (1u << mu)) apply_bc(g, mu, +1, p);
                }
                hop_forward(mu, Lk, p, (R)1, acc);
            }
            if (t.nlb[mu] >= 0) {
                if (own) {
                    lds_get(sh, nt, t.nlb[mu], p);
                    own_link<LC, R, G>(a, lk, nt, t.s0 + t.nlb[mu], t.nlb[mu], mu, Lk);
                    hop_backward(mu, Lk, p, (R)1, acc);
                }
            } else {
                load_spinor<R, S>(xx, xsc, g.V, t.ngb[mu], p);
                if (t.wrap & (16u << mu)) apply_bc(g, mu, -1, p);
                load_link<R, G>(a.links, g.V, t.ngb[mu], mu, Lk);
                hop_backward(mu, Lk, p, (R)1, acc);
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

// acc += f * (sum over in-block neighbours of the hop terms) of the block
// vector held in LDS.
template <class G, class R, bool LC = false>
__device__ inline void gen_block_hops_add(const SapArgs& a, const GenSite<R>& t, const R* sh, int nt, int l, R f,
                                          Spinor<R>& acc, const R* lk = nullptr) {
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        Link<R> Lk;
        Spinor<R> p;
        if (t.nlf[mu] >= 0) {  // in-block hops never cross the lattice boundary
            own_link<LC, R, G>(a, lk, nt, t.s, l, mu, Lk);
            lds_get(sh, nt, t.nlf[mu], p);
            hop_forward(mu, Lk, p, f, acc);
        }
        if (t.nlb[mu] >= 0) {
            own_link<LC, R, G>(a, lk, nt, t.s0 + t.nlb[mu], t.nlb[mu], mu, Lk);
            lds_get(sh, nt, t.nlb[mu], p);
            hop_backward(mu, Lk, p, f, acc);
        }
    }
}

// acc = sum over in-block neighbours of the hop terms (before the factor
// -1/2) of the block vector held in LDS.
template <class G, class R, bool LC = false>
__device__ inline void gen_block_hops(const SapArgs& a, const GenSite<R>& t, const R* sh, int nt, int l,
                                      Spinor<R>& acc, const R* lk = nullptr) {
#pragma unroll
    for (int i = 0; i < 12; ++i) acc.v[i] = cmk<R>(0, 0);
    gen_block_hops_add<G, R, LC>(a, t, sh, nt, l, (R)1, acc, lk);
}

// LC: the block's links are staged in LDS once per workgroup (48 nt reals after
// the exchange and reduction space) and every own or in-block link is read from
// there; only the backward links of the halo hops come from memory.
template <class S, class G, class C, class R, int MAXT, bool LC = false>
__global__ void __launch_bounds__(MAXT) k_sap_half(SapArgs a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const Geo& g = a.g;
    const int l = threadIdx.x;
    const int nt = blockDim.x;
    const bool active = l < g.Vb;
    R* sh = reinterpret_cast<R*>(smem_raw);
    R* red = sh + 24 * nt;
    R* lk = LC ? red + 64 : nullptr;
    GenSite<R> t;
    gen_site_setup(g, a.colour, l, active, t);

    Clover<R> A;
    if (active) load_clover<R, C>(a.clover, g.V, t.s, A);
    if constexpr (LC) {
        if (active) lk_stage<R, G>(a.links, g.V, t.s, lk, nt, l);
        __syncthreads();
    }

    const size_t stride = (size_t)6 * g.V * Unit<S>::bytes;
    const int sys_begin = blockIdx.y * a.sys_tile;
    const int sys_end = min(a.nsys, sys_begin + a.sys_tile);

    for (int sys = sys_begin; sys < sys_end; ++sys) {
        const R mu_tw = (R)(a.mu[sys] + g.mu_shift[t.parity]);
        const void* bb = reinterpret_cast<const char*>(a.b) + sys * stride;
        void* xx = reinterpret_cast<char*>(a.x) + sys * stride;
        const float* bsc = a.b_scale ? a.b_scale + (size_t)sys * g.V : nullptr;
        float* xsc = a.x_scale ? a.x_scale + (size_t)sys * g.V : nullptr;

        Spinor<R> xv, rho;
        gen_residual<S, G, R, LC>(a, t, A, mu_tw, active, sh, nt, l, bb, bsc, xx, xsc, rho, xv, lk);

        // ---- minimal residual on D_BB from a zero correction, added to x as it goes
        // (x_new = x + sum_k alpha_k rho_k; no separate correction vector)
        for (int it = 0; it < a.mr_iters; ++it) {
            if (active) lds_put(sh, nt, l, rho);
            __syncthreads();
            Spinor<R> q;
            R qr_re = 0, qr_im = 0, qq = 0;
            if (active) {
                // q = (A + twist) rho - 1/2 (in-block hops of rho)
                clover_apply(A, mu_tw, rho, q);
                gen_block_hops_add<G, R, LC>(a, t, sh, nt, l, (R)-0.5, q, lk);
                mr_dots(q, rho, qr_re, qr_im, qq);
            }
            block_sum3(red, qr_re, qr_im, qq);
            if (active && qq >= min_normal<R>()) {
                const cplx<R> alpha = cmk(qr_re / qq, qr_im / qq);
#pragma unroll
                for (int i = 0; i < 12; ++i) xv.v[i] = cmad(alpha, rho.v[i], xv.v[i]);
                mr_residual_update(alpha, q, rho);
            }
        }

        if (active) store_spinor<R, S>(xx, xsc, g.V, t.s, xv);
    }
}

// Half-sweep with even-odd preconditioned block solves (section 2.5): the
// block system D_BB e = r is reduced to its odd sites,
//   rhat_o = r_o - D_oe D_ee^-1 r_e,  Dhat = D_oo - D_oe D_ee^-1 D_eo,
// MR runs on Dhat e_o = rhat_o from e_o = 0, and e_e = D_ee^-1 (r_e - D_eo e_o).
// D_oe and D_eo are the in-block hops (factor -1/2 included), D_ee and D_oo
// the site-diagonal parts; parity from the global coordinates.
template <class S, class G, class C, class R, int MAXT>
__global__ void __launch_bounds__(MAXT) k_sap_half_eo(SapArgs a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const Geo& g = a.g;
    const int l = threadIdx.x;
    const int nt = blockDim.x;
    const bool active = l < g.Vb;
    R* sh = reinterpret_cast<R*>(smem_raw);
    R* red = sh + 24 * nt;
    GenSite<R> t;
    gen_site_setup(g, a.colour, l, active, t);
    const bool odd = active && t.parity == 1;
    const bool even = active && t.parity == 0;
    const long long half = g.V / 2, h = t.s >> 1;

    Clover<R> A;  // every site for the residual; odd sites also for D_oo
    if (active) load_clover<R, C>(a.clover, g.V, t.s, A);

    const size_t stride = (size_t)6 * g.V * Unit<S>::bytes;
    const int sys_begin = blockIdx.y * a.sys_tile;
    const int sys_end = min(a.nsys, sys_begin + a.sys_tile);

    for (int sys = sys_begin; sys < sys_end; ++sys) {
        const R mu_tw = (R)(a.mu[sys] + g.mu_shift[t.parity]);
        const void* inv = a.eo_inv[a.eo_sel[sys]];
        const bool adj = (a.eo_adj >> sys) & 1ull;
        const void* bb = reinterpret_cast<const char*>(a.b) + sys * stride;
        void* xx = reinterpret_cast<char*>(a.x) + sys * stride;
        const float* bsc = a.b_scale ? a.b_scale + (size_t)sys * g.V : nullptr;
        float* xsc = a.x_scale ? a.x_scale + (size_t)sys * g.V : nullptr;

        Spinor<R> r, xv, tv, acc;
        gen_residual<S, G, R>(a, t, A, mu_tw, active, sh, nt, l, bb, bsc, xx, xsc, r, xv);

        // rhat_o = r_o - D_oe (D_ee^-1 r_e)
#pragma unroll
        for (int i = 0; i < 12; ++i) tv.v[i] = cmk<R>(0, 0);
        if (even) eo_inverse_apply<C, R>(inv, half, h, adj, r, tv);
        if (active) lds_put(sh, nt, l, tv);
        __syncthreads();
        Spinor<R> rho, e;
#pragma unroll
        for (int i = 0; i < 12; ++i) {
            rho.v[i] = cmk<R>(0, 0);
            e.v[i] = cmk<R>(0, 0);
        }
        if (odd) {
            gen_block_hops<G, R>(a, t, sh, nt, l, acc);
#pragma unroll
            for (int i = 0; i < 12; ++i) rho.v[i] = r.v[i] + (R)0.5 * acc.v[i];
        }

        // MR on Dhat over the odd sites
        for (int it = 0; it < a.mr_iters; ++it) {
            __syncthreads();
            if (active) lds_put(sh, nt, l, rho);
            __syncthreads();
            // even: t_e = D_ee^-1 D_eo rho_o
#pragma unroll
            for (int i = 0; i < 12; ++i) tv.v[i] = cmk<R>(0, 0);
            if (even) {
                gen_block_hops<G, R>(a, t, sh, nt, l, acc);
                Spinor<R> u;
#pragma unroll
                for (int i = 0; i < 12; ++i) u.v[i] = (R)-0.5 * acc.v[i];
                eo_inverse_apply<C, R>(inv, half, h, adj, u, tv);
            }
            __syncthreads();
            if (active) lds_put(sh, nt, l, tv);
            __syncthreads();
            // odd: q_o = D_oo rho_o - D_oe t_e
            Spinor<R> q;
            R qr_re = 0, qr_im = 0, qq = 0;
            if (odd) {
                gen_block_hops<G, R>(a, t, sh, nt, l, acc);
                clover_apply(A, mu_tw, rho, q);
#pragma unroll
                for (int i = 0; i < 12; ++i) q.v[i] = q.v[i] + (R)0.5 * acc.v[i];
                mr_dots(q, rho, qr_re, qr_im, qq);
            }
            block_sum3(red, qr_re, qr_im, qq);
            if (odd && qq >= min_normal<R>()) {
                const cplx<R> alpha = cmk(qr_re / qq, qr_im / qq);
#pragma unroll
                for (int i = 0; i < 12; ++i) e.v[i] = cmad(alpha, rho.v[i], e.v[i]);
                mr_residual_update(alpha, q, rho);
            }
        }

        // e_e = D_ee^-1 (r_e - D_eo e_o)
        __syncthreads();
        if (active) lds_put(sh, nt, l, e);
        __syncthreads();
        if (even) {
            gen_block_hops<G, R>(a, t, sh, nt, l, acc);
            Spinor<R> v;
#pragma unroll
            for (int i = 0; i < 12; ++i) v.v[i] = r.v[i] + (R)0.5 * acc.v[i];
            eo_inverse_apply<C, R>(inv, half, h, adj, v, e);
        }
        if (active) {
#pragma unroll
            for (int i = 0; i < 12; ++i) e.v[i] = e.v[i] + xv.v[i];
            store_spinor<R, S>(xx, xsc, g.V, t.s, e);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// FP32-compute half-sweep for blocks of at most 256 sites.  Everything the MR
// steps touch stays on chip: each thread keeps its own four links (third row
// rebuilt once) and its clover block in registers.  The block operator is
// applied by a push exchange through LDS: every site publishes its spinor
// (for the forward hops of its -mu neighbours) and, for each +mu neighbour
// inside the block, the finished backward product U_mu(x)^+ (1 + gamma_mu)
// psi(x) as a half spinor, so no link is read in the MR loop.
constexpr int kV2 = 256;

struct V2Shared {
    float xs[24 * kV2];      // spinor components [24][site]
    float gb[4 * 12 * kV2];  // backward products [mu][12][site]
    float red[64];
};
// xs and gb together hold the staged halo: [24][kHaloMax] spinor components.
constexpr int kHaloMax = 3 * kV2;

// LDS layout in 16-byte units: spinor [6][site] float4, backward products
// [mu][3][site] float4; consecutive lanes touch consecutive 16-byte words.
__device__ inline void v2_put_spinor(float* xs, int l, const Spinor<float>& p) {
    float4* x4 = reinterpret_cast<float4*>(xs);
#pragma unroll
    for (int k = 0; k < 6; ++k)
        x4[k * kV2 + l] = make_float4(p.v[2 * k].re, p.v[2 * k].im, p.v[2 * k + 1].re, p.v[2 * k + 1].im);
}

__device__ inline void v2_get_spinor(const float* xs, int l, Spinor<float>& p) {
    const float4* x4 = reinterpret_cast<const float4*>(xs);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const float4 t = x4[k * kV2 + l];
        p.v[2 * k] = cmk(t.x, t.y);
        p.v[2 * k + 1] = cmk(t.z, t.w);
    }
}

__device__ inline void v2_put_half(float* gb, int mu, int l, const Half<float>& g) {
    float4* g4 = reinterpret_cast<float4*>(gb);
    const cplx<float>* v = &g.h[0][0];
#pragma unroll
    for (int k = 0; k < 3; ++k) g4[(mu * 3 + k) * kV2 + l] = make_float4(v[2 * k].re, v[2 * k].im, v[2 * k + 1].re, v[2 * k + 1].im);
}

__device__ inline void v2_get_half(const float* gb, int mu, int l, Half<float>& g) {
    const float4* g4 = reinterpret_cast<const float4*>(gb);
    cplx<float>* v = &g.h[0][0];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float4 t = g4[(mu * 3 + k) * kV2 + l];
        v[2 * k] = cmk(t.x, t.y);
        v[2 * k + 1] = cmk(t.z, t.w);
    }
}

// A link kept as its first two rows; the third is rebuilt where it is used.
struct Link2 {
    cplx<float> u[2][3];
};

template <class G>
__device__ inline void load_link2(const void* base, long long V, long long s, int mu, Link2& L) {
    float u[4];
    const size_t b = (size_t)mu * 3 * V;
    Unit<G>::load(base, b + s, u);
    L.u[0][0] = cmk(u[0], u[1]);
    L.u[0][1] = cmk(u[2], u[3]);
    Unit<G>::load(base, b + V + s, u);
    L.u[0][2] = cmk(u[0], u[1]);
    L.u[1][0] = cmk(u[2], u[3]);
    Unit<G>::load(base, b + 2 * V + s, u);
    L.u[1][1] = cmk(u[0], u[1]);
    L.u[1][2] = cmk(u[2], u[3]);
}

__device__ inline void expand_link(const Link2& c, Link<float>& L) {
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int k = 0; k < 3; ++k) L.u[r][k] = c.u[r][k];
    complete_su3(L);
}

// Third row of an SU(3) link, element k: conj(row0 x row1)_k.
__device__ inline cplx<float> row2(const Link2& c, int k) {
    const int a = (k + 1) % 3, b = (k + 2) % 3;
    return conj(c.u[0][a] * c.u[1][b] - c.u[0][b] * c.u[1][a]);
}

// g = U h with the third row rebuilt element by element.
__device__ inline void su3_mul2(const Link2& c, const Half<float>& h, Half<float>& g) {
#pragma unroll
    for (int s = 0; s < 2; ++s) {
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            cplx<float> t = c.u[i][0] * h.h[s][0];
            t = cmad(c.u[i][1], h.h[s][1], t);
            g.h[s][i] = cmad(c.u[i][2], h.h[s][2], t);
        }
    }
    const cplx<float> r0 = row2(c, 0), r1 = row2(c, 1), r2 = row2(c, 2);
#pragma unroll
    for (int s = 0; s < 2; ++s) g.h[s][2] = cmad(r2, h.h[s][2], cmad(r1, h.h[s][1], r0 * h.h[s][0]));
}

// g = U^+ h with the third row rebuilt.
__device__ inline void su3_dag_mul2(const Link2& c, const Half<float>& h, Half<float>& g) {
    const cplx<float> r0 = row2(c, 0), r1 = row2(c, 1), r2 = row2(c, 2);
    const cplx<float> r[3] = {r0, r1, r2};
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            cplx<float> t = cjmad(c.u[0][i], h.h[s][0], cmk(0.f, 0.f));
            t = cjmad(c.u[1][i], h.h[s][1], t);
            g.h[s][i] = cjmad(r[i], h.h[s][2], t);
        }
}

// h = upper - B_mu lower of the spinor of local site n (from LDS).
__device__ inline void project_forward_lds(const float* xs, int mu, int n, Half<float>& h) {
    Spinor<float> p;
    v2_get_spinor(xs, n, p);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        cplx<float> b0, b1;
        apply_B(mu, p.v[6 + c], p.v[9 + c], b0, b1);
        h.h[0][c] = p.v[c] - b0;
        h.h[1][c] = p.v[3 + c] - b1;
    }
}

// acc += (1 - gamma_mu) lift of g: upper += g, lower -= B^+ g.
__device__ inline void forward_accumulate(int mu, const Half<float>& g, Spinor<float>& acc) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        cplx<float> d0, d1;
        apply_Bdag(mu, g.h[0][c], g.h[1][c], d0, d1);
        acc.v[c] = acc.v[c] + g.h[0][c];
        acc.v[3 + c] = acc.v[3 + c] + g.h[1][c];
        acc.v[6 + c] = acc.v[6 + c] - d0;
        acc.v[9 + c] = acc.v[9 + c] - d1;
    }
}

// Publish v: spinor plus backward products for the in-block +mu neighbours.
__device__ inline void v2_push(V2Shared& sm, int l, bool active, const bool fin[4], const Link<float> Uo[4],
                               const Spinor<float>& v) {
    if (!active) return;
    v2_put_spinor(sm.xs, l, v);
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        // keep one direction's operands live at a time
        __builtin_amdgcn_sched_barrier(0);
        if (fin[mu]) {
            Half<float> h, g;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                cplx<float> b0, b1;
                apply_B(mu, v.v[6 + c], v.v[9 + c], b0, b1);
                h.h[0][c] = v.v[c] + b0;
                h.h[1][c] = v.v[3 + c] + b1;
            }
            su3_dag_mul(Uo[mu], h, g);
            v2_put_half(sm.gb, mu, l, g);
        }
    }
    __builtin_amdgcn_sched_barrier(0);
}

// acc += in-block hop terms (unscaled; the operator adds -1/2 acc).
__device__ inline void v2_pull(const V2Shared& sm, int l, const bool fin[4], const bool bin[4], const int str[4],
                               const Link<float> Uo[4], Spinor<float>& acc) {
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        __builtin_amdgcn_sched_barrier(0);
        if (fin[mu]) {
            Half<float> h, g;
            project_forward_lds(sm.xs, mu, l + str[mu], h);
            su3_mul(Uo[mu], h, g);
            forward_accumulate(mu, g, acc);
        }
        __builtin_amdgcn_sched_barrier(0);
        if (bin[mu]) {
            Half<float> g;
            v2_get_half(sm.gb, mu, l - str[mu], g);
            backward_accumulate(mu, g, acc);
        }
    }
    __builtin_amdgcn_sched_barrier(0);
}

template <class S, class G, class C>
__global__ void __launch_bounds__(kV2) k_sap_half_v2(SapArgs a) {
    __shared__ V2Shared sm;
    const Geo& g = a.g;
    const int Vb = g.Vb;
    const int l = threadIdx.x;
    const bool active = l < Vb;

    const int half3 = g.nb[3] >> 1;
    int j = blockIdx.x;
    const int k3 = j % half3;
    j /= half3;
    const int B2 = j % g.nb[2];
    j /= g.nb[2];
    const int B1 = j % g.nb[1];
    const int B0 = j / g.nb[1];
    const int B3 = 2 * k3 + ((a.colour + B0 + B1 + B2) & 1);
    const long long blk = (((long long)B0 * g.nb[1] + B1) * g.nb[2] + B2) * g.nb[3] + B3;
    const long long s = blk * Vb + (active ? l : 0);

    int Lc[4];
    {
        int t = active ? l : 0;
        for (int ax = 3; ax >= 0; --ax) {
            Lc[ax] = t % g.lb[ax];
            t /= g.lb[ax];
        }
    }
    bool fin[4], bin[4];
    int str[4];
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        const int ax = axis_of(mu);
        int st = 1;
        for (int q = ax + 1; q < 4; ++q) st *= g.lb[q];
        str[mu] = st;
        fin[mu] = active && Lc[ax] + 1 < g.lb[ax];
        bin[mu] = active && Lc[ax] > 0;
    }

    // Halo faces: f = 2*axis + side (side 0: the layer below the block, 1: above);
    // entry of a face site = lexicographic index over the other three axes.
    const int Bc[4] = {B0, B1, B2, B3};
    int hoff[9];
    hoff[0] = 0;
    for (int f = 0; f < 8; ++f) hoff[f + 1] = hoff[f] + Vb / g.lb[f >> 1];
    const int nhalo = hoff[8];
    const bool stage_halo = nhalo <= kHaloMax;
    int hent_f[4], hent_b[4];
    long long nbk[4];
    unsigned wrap = 0;  // hops that cross the lattice boundary: bit mu forward, bit 4+mu backward
    int parity = 0;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        const int ax = axis_of(mu);
        int p = 0;
        for (int q = 0; q < 4; ++q)
            if (q != ax) p = p * g.lb[q] + Lc[q];
        hent_f[mu] = hoff[2 * ax + 1] + p;
        hent_b[mu] = hoff[2 * ax] + p;
        int c[4];
        for (int q = 0; q < 4; ++q) c[q] = Bc[q] * g.lb[q] + Lc[q];
        if (mu == 0) parity = (c[0] + c[1] + c[2] + c[3]) & 1;
        if (c[ax] == g.d[ax] - 1) wrap |= 1u << mu;
        if (c[ax] == 0) wrap |= 16u << mu;
        c[ax] = c[ax] == 0 ? g.d[ax] - 1 : c[ax] - 1;
        nbk[mu] = coords_site(g, c);
    }

    // own links with the third row rebuilt once; the clover kept as -2A so that
    // the MR direction q' = (hops) - 2 A rho = -2 D_BB rho needs no rescaling
    Link<float> Uo[4];
    Clover<float> A;
    if (active) {
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) load_link<float, G>(a.links, g.V, s, mu, Uo[mu]);
        load_clover<float, C>(a.clover, g.V, s, A);
#pragma unroll
        for (int i = 0; i < 72; ++i) A.a[i] *= -2.f;
    }

    const size_t stride = (size_t)6 * g.V * Unit<S>::bytes;
    const int sys_begin = blockIdx.y * a.sys_tile;
    const int sys_end = min(a.nsys, sys_begin + a.sys_tile);
    const bool own = !a.own_zero;
    const bool halo = !(a.own_zero && a.halo_zero);

    for (int sys = sys_begin; sys < sys_end; ++sys) {
        const float mu_tw = (float)(a.mu[sys] + g.mu_shift[parity]);
        const void* bb = reinterpret_cast<const char*>(a.b) + sys * stride;
        void* xx = reinterpret_cast<char*>(a.x) + sys * stride;
        const float* bsc = a.b_scale ? a.b_scale + (size_t)sys * g.V : nullptr;
        float* xsc = a.x_scale ? a.x_scale + (size_t)sys * g.V : nullptr;

        // ---- r = b - D x on the block; e starts at x so that x_new = e
        Spinor<float> r, e, acc;
#pragma unroll
        for (int i = 0; i < 12; ++i) {
            e.v[i] = cmk(0.f, 0.f);
            acc.v[i] = cmk(0.f, 0.f);
        }
        if (active) {
            load_spinor<float, S>(bb, bsc, g.V, s, r);
            if (own) load_spinor<float, S>(xx, xsc, g.V, s, e);
        }
        if (own) {
            v2_push(sm, l, active, fin, Uo, e);
            __syncthreads();
            if (active) v2_pull(sm, l, fin, bin, str, Uo, acc);
        }
        if (halo && stage_halo) {
            // The other colour's face spinors, staged once per system by the whole
            // workgroup (one memory latency instead of one per direction); face
            // lanes fetch the links of their backward halo hops meanwhile.
            float* hb = sm.xs;  // xs and gb are contiguous: room for kHaloMax entries
            for (int e2 = l; e2 < nhalo; e2 += blockDim.x) {
                int f = 0;
                while (f < 7 && e2 >= hoff[f + 1]) ++f;
                const int ax = f >> 1;
                int p = e2 - hoff[f];
                int c[4];
                for (int q = 3; q >= 0; --q) {
                    if (q == ax) continue;
                    c[q] = p % g.lb[q];
                    p /= g.lb[q];
                }
                c[ax] = (f & 1) ? g.lb[ax] : -1;
                for (int q = 0; q < 4; ++q) {
                    c[q] += Bc[q] * g.lb[q];
                    if (c[q] < 0) c[q] += g.d[q];
                    if (c[q] >= g.d[q]) c[q] -= g.d[q];
                }
                Spinor<float> hv;
                load_spinor<float, S>(xx, xsc, g.V, coords_site(g, c), hv);
#pragma unroll
                for (int i = 0; i < 12; ++i) {
                    hb[(2 * i) * kHaloMax + e2] = hv.v[i].re;
                    hb[(2 * i + 1) * kHaloMax + e2] = hv.v[i].im;
                }
            }
            Link2 Lb[4];
#pragma unroll
            for (int mu = 0; mu < 4; ++mu)
                if (active && !bin[mu]) load_link2<G>(a.links, g.V, nbk[mu], mu, Lb[mu]);
            __syncthreads();
            if (active) {
#pragma unroll
                for (int mu = 0; mu < 4; ++mu) {
                    if (!fin[mu]) {
                        Spinor<float> p;
#pragma unroll
                        for (int i = 0; i < 12; ++i)
                            p.v[i] = cmk(hb[(2 * i) * kHaloMax + hent_f[mu]], hb[(2 * i + 1) * kHaloMax + hent_f[mu]]);
                        if (wrap & (1u << mu)) apply_bc(g, mu, +1, p);
                        hop_forward(mu, Uo[mu], p, 1.f, acc);
                    }
                    if (!bin[mu]) {
                        Spinor<float> p;
#pragma unroll
                        for (int i = 0; i < 12; ++i)
                            p.v[i] = cmk(hb[(2 * i) * kHaloMax + hent_b[mu]], hb[(2 * i + 1) * kHaloMax + hent_b[mu]]);
                        Link<float> L;
                        expand_link(Lb[mu], L);
                        if (wrap & (16u << mu)) apply_bc(g, mu, -1, p);
                        hop_backward(mu, L, p, 1.f, acc);
                    }
                }
            }
            __syncthreads();
        } else if (halo && active) {
            const int Bcc[4] = {B0, B1, B2, B3};
#pragma unroll
            for (int mu = 0; mu < 4; ++mu) {
                const int ax = axis_of(mu);
                int n[4];
                for (int q = 0; q < 4; ++q) n[q] = Bcc[q] * g.lb[q] + Lc[q];
                if (!fin[mu]) {
                    if (++n[ax] == g.d[ax]) n[ax] = 0;
                    Spinor<float> p;
                    load_spinor<float, S>(xx, xsc, g.V, coords_site(g, n), p);
                    if (wrap & (1u << mu)) apply_bc(g, mu, +1, p);
                    hop_forward(mu, Uo[mu], p, 1.f, acc);
                    n[ax] = Bcc[ax] * g.lb[ax] + Lc[ax];
                }
                if (!bin[mu]) {
                    if (--n[ax] < 0) n[ax] = g.d[ax] - 1;
                    const long long nb = coords_site(g, n);
                    Spinor<float> p;
                    Link<float> Lk;
                    load_spinor<float, S>(xx, xsc, g.V, nb, p);
                    load_link<float, G>(a.links, g.V, nb, mu, Lk);
                    if (wrap & (16u << mu)) apply_bc(g, mu, -1, p);
                    hop_backward(mu, Lk, p, 1.f, acc);
                }
            }
        }
        if (active) {
            // r = b - (A x - acc/2) = b + (acc - 2 A x) / 2
            if (own) clover_acc(A, -2.f * mu_tw, e, acc);
#pragma unroll
            for (int i = 0; i < 12; ++i) r.v[i] = r.v[i] + 0.5f * acc.v[i];
        }
        if (own) __syncthreads();

        // ---- minimal residual on D_BB: e += alpha rho, rho -= alpha D_BB rho
        Spinor<float>& rho = r;
        for (int it = 0; it < a.mr_iters; ++it) {
            v2_push(sm, l, active, fin, Uo, rho);
            __syncthreads();
            Spinor<float> q;
            float qr_re = 0.f, qr_im = 0.f, qq = 0.f;
            if (active) {
#pragma unroll
                for (int i = 0; i < 12; ++i) q.v[i] = cmk(0.f, 0.f);
                v2_pull(sm, l, fin, bin, str, Uo, q);
                clover_acc(A, -2.f * mu_tw, rho, q);  // q = -2 D_BB rho
                mr_dots(q, rho, qr_re, qr_im, qq);
            }
            block_sum3(sm.red, qr_re, qr_im, qq);
            if (active && qq >= min_normal<float>()) {
                // with q = -2 D_BB rho: rho -= a q and e += -2 a rho, a = <q,rho>/<q,q>
                const float inv = __builtin_amdgcn_rcpf(qq);
                const cplx<float> alpha = cmk(qr_re * inv, qr_im * inv);
                const cplx<float> beta = cmk(-2.f * alpha.re, -2.f * alpha.im);
#pragma unroll
                for (int i = 0; i < 12; ++i) e.v[i] = cmad(beta, rho.v[i], e.v[i]);
                mr_residual_update(alpha, q, rho);
            }
        }
        if (active) store_spinor<float, S>(xx, xsc, g.V, s, e);
    }
}

// Lower-face halo product of direction MU: U_MU(y)^+ (1 + gamma_MU) psi(y) of the
// site y just below the face, stored in the layout [3][site] float4 at entry j.
template <int MU>
__device__ inline void s44_stage_backward(const Link<float>& L, const Spinor<float>& p, float sg, float* hb, int j) {
    Half<float> g;
    backward_product(MU, L, p, g);
    float4* h4 = reinterpret_cast<float4*>(hb);
    const cplx<float>* v = &g.h[0][0];
#pragma unroll
    for (int k = 0; k < 3; ++k)
        h4[k * kV2 + j] = make_float4(sg * v[2 * k].re, sg * v[2 * k].im, sg * v[2 * k + 1].re, sg * v[2 * k + 1].im);
}

// Sum of three values over the four waves of a 256-thread workgroup; the
// wave totals are written as one float4 each and read back together.
__device__ inline void block_sum3_w4(float* red, float& a, float& b, float& c) {
    a = wave_sum(a);
    b = wave_sum(b);
    c = wave_sum(c);
    float4* r4 = reinterpret_cast<float4*>(red);
    if ((threadIdx.x & 63) == 0) r4[threadIdx.x >> 6] = make_float4(a, b, c, 0.f);
    __syncthreads();
    const float4 p0 = r4[0], p1 = r4[1], p2 = r4[2], p3 = r4[3];
    a = (p0.x + p1.x) + (p2.x + p3.x);
    b = (p0.y + p1.y) + (p2.y + p3.y);
    c = (p0.z + p1.z) + (p2.z + p3.z);
}

// Upper-face halo of direction MU: h = upper - B_MU lower of the spinor just
// above the face, times the boundary phase when that hop crosses the lattice
// edge, stored in the layout [3][axis*64 + pos] float4 at entry j.
template <int MU>
__device__ inline void s44_stage_forward(const Geo& g, const Spinor<float>& p, bool wrap, float* dst, int j) {
    Half<float> h;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        cplx<float> b0, b1;
        apply_B(MU, p.v[6 + c], p.v[9 + c], b0, b1);
        h.h[0][c] = p.v[c] - b0;
        h.h[1][c] = p.v[3 + c] - b1;
    }
    if (wrap) {
        const cplx<float> ph = cmk(g.bcrf[MU], g.bcif[MU]);
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int c = 0; c < 3; ++c) h.h[s][c] = ph * h.h[s][c];
    }
    v2_put_half(dst, 0, j, h);
}

// The hop part of D on one 4^4 block for one system: acc = the sum over the eight
// hops of the spinor field x (unscaled; D adds -1/2 acc), e holding x at this
// thread's own site and xx the whole field (FP32 arithmetic, storage S).  Wave
// w stages axis w's halo: the backward product of the site below the lower face
// into the slot of its column's upper-face site, and, once the in-block hops
// have read xs, the projected half spinor of the site above the upper face into
// xs.  Starts by writing LDS (the caller must have passed a barrier since the
// last reads of xs and gb) and ends after the last reads, without a barrier.
// k_sap_half_44 takes the same steps written out in its residual: called there,
// the compiler allocates that kernel's registers differently and spills one
// more address per system, which cost 3 % of its time.
template <class S, class G>
__device__ __attribute__((always_inline)) inline void s44_stencil(V2Shared& sm, const Geo& g, const void* links, const void* xx, const float* xsc,
                                   int l, const Link<float> Uo[4], const bool fin[4], const int str[4],
                                   const S44Site& hx, int wax, int wmu, const Spinor<float>& e,
                                   Spinor<float>& acc) {
    const int up_site = (int)hx.up_site, dn_site = (int)hx.dn_site, top = hx.top;
    const bool up_wrap = hx.up_wrap, dn_wrap = hx.dn_wrap;
    float* hb = sm.gb + wmu * 3 * kV2 * 4;  // this wave's lower-face products, direction wmu
    // pass 1: in-block hops and the lower-face halo
    {
        Spinor<float> hd;
        Link<float> Ldn;  // U_mu(site below the lower face), mu = wmu
        load_spinor<float, S>(xx, xsc, g.V, dn_site, hd);
        load_link<float, G>(links, g.V, dn_site, wmu, Ldn);
        v2_push(sm, l, true, fin, Uo, e);
        if (dn_wrap) apply_bc(g, wmu, -1, hd);
        switch (wax) {
            case 0: s44_stage_backward<0>(Ldn, hd, 1.f, hb, top); break;
            case 1: s44_stage_backward<3>(Ldn, hd, 1.f, hb, top); break;
            case 2: s44_stage_backward<2>(Ldn, hd, 1.f, hb, top); break;
            default: s44_stage_backward<1>(Ldn, hd, 1.f, hb, top); break;
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 12; ++i) acc.v[i] = cmk(-0.f, -0.f);  // -0 + t = t: the first hop is stored
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        __builtin_amdgcn_sched_barrier(0);
        if (fin[mu]) {
            Half<float> h, gg;
            project_forward_lds(sm.xs, mu, l + str[mu], h);
            su3_mul(Uo[mu], h, gg);
            forward_accumulate(mu, gg, acc);
        }
        __builtin_amdgcn_sched_barrier(0);
        Half<float> gg;
        v2_get_half(sm.gb, mu, hx.bcol[mu], gg);
        backward_accumulate(mu, gg, acc);
    }
    __syncthreads();
    // pass 2: the upper-face halo, staged in xs
    {
        Spinor<float> hu;
        load_spinor<float, S>(xx, xsc, g.V, up_site, hu);
        switch (wax) {
            case 0: s44_stage_forward<0>(g, hu, up_wrap, sm.xs, l); break;
            case 1: s44_stage_forward<3>(g, hu, up_wrap, sm.xs, l); break;
            case 2: s44_stage_forward<2>(g, hu, up_wrap, sm.xs, l); break;
            default: s44_stage_forward<1>(g, hu, up_wrap, sm.xs, l); break;
        }
    }
    __syncthreads();
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        if (!fin[mu]) {
            Half<float> h, gg;
            v2_get_half(sm.xs, 0, hx.fsrc[mu], h);
            su3_mul(Uo[mu], h, gg);
            forward_accumulate(mu, gg, acc);
        }
    }
}

// ---------------------------------------------------------------------------
// FP32 half-sweep specialised to 4^4 blocks (the paper's level-1 Schwarz
// block): one site per thread, links and clover held in registers for all
// systems of the launch, two workgroups per compute unit (two waves per SIMD,
// so that one workgroup's LDS waits, barriers and loads overlap the other's
// arithmetic).  LDS holds only the exchange buffers xs and gb (72 KiB).  Wave w
// also owns array axis w of the halo: its lane p forms, at face position p, the
// backward hop product U_mu(y)^+ (1 + gamma_mu) psi(y) of the site y below the
// block's lower face and the projected half spinor (1 - gamma_mu) psi of the
// site above its upper face.
//   * The lower-face products go into gb slots that no site fills: on
//     direction mu the 64 upper-face sites have no in-block +mu neighbour, and
//     the product for the site below a column's lower face is kept in the slot
//     of that column's upper-face site.
//   * The upper-face halo is taken in a second pass of the residual: once every
//     in-block hop has read xs, the waves stage the projected halves there and
//     the face sites finish their forward hops from them.
// Every site takes each of its eight hops once, so the residual b - D x costs
// one stencil plus the halo staging; the MR steps exchange rho through xs and
// gb with two barriers per step.
template <class S, class G, class C>
__global__ void __launch_bounds__(kV2) __attribute__((amdgpu_waves_per_eu(2, 2))) k_sap_half_44(SapArgs a) {
    __shared__ V2Shared sm;
    const Geo& g = a.g;
    const int l = threadIdx.x;  // 256 threads, all sites active

    // block (the same for the whole workgroup), then the thread's site, in-block
    // neighbours and halo duty (tm_sap_index.h, checked on the host)
    int B[4];
    s44_block(g, a.colour, xcd_swizzle(blockIdx.x, gridDim.x), B);
#pragma unroll
    for (int q = 0; q < 4; ++q) B[q] = __builtin_amdgcn_readfirstlane(B[q]);
    const long long blk = s44_block_index(g, B);
    S44Site ix;
    s44_lane(g, B, blk, l, ix);
    int str[4];
    bool fin[4], bin[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        str[q] = ix.str[q];
        fin[q] = ix.fin[q];
        bin[q] = ix.bin[q];
    }
    const int wax = __builtin_amdgcn_readfirstlane(ix.wax);
    const int wmu = wax == 0 ? 0 : 4 - wax;
    const size_t stride = (size_t)6 * g.V * Unit<S>::bytes;
    const int sys_begin = blockIdx.y * a.sys_tile;
    const int sys_end = min(a.nsys, sys_begin + a.sys_tile);
    const bool own = !a.own_zero;
    const bool halo = !(a.own_zero && a.halo_zero);
    float* hb = sm.gb + wmu * 3 * kV2 * 4;  // this wave's lower-face products, direction wmu

    Link<float> Uo[4];
    Clover<float> A;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) load_link<float, G>(a.links, g.V, ix.s, mu, Uo[mu]);
    load_clover<float, C>(a.clover, g.V, ix.s, A);
#pragma unroll
    for (int i = 0; i < 72; ++i) A.a[i] *= -2.f;

    for (int sys = sys_begin; sys < sys_end; ++sys) {
        // The per-thread indices used outside the MR steps are recomputed for every system from
        // an index the compiler cannot see through: held across the MR steps they would be
        // spilled to scratch memory (the MR steps need every register at two waves per SIMD).
        int lx = l;
        asm volatile("" : "+v"(lx));
        S44Site hx;
        s44_lane(g, B, blk, lx, hx);
        const long long s = hx.s;
        const int up_site = (int)hx.up_site, dn_site = (int)hx.dn_site, top = hx.top;
        const bool up_wrap = hx.up_wrap, dn_wrap = hx.dn_wrap;
        int fsrc[4], bcol[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            fsrc[q] = hx.fsrc[q];
            bcol[q] = hx.bcol[q];
        }
        const float mu_tw = (float)(a.mu[sys] + g.mu_shift[hx.parity]);
        const void* bb = reinterpret_cast<const char*>(a.b) + sys * stride;
        void* xx = reinterpret_cast<char*>(a.x) + sys * stride;
        const float* bsc = a.b_scale ? a.b_scale + (size_t)sys * g.V : nullptr;
        float* xsc = a.x_scale ? a.x_scale + (size_t)sys * g.V : nullptr;

        Spinor<float> r, e;
#pragma unroll
        for (int i = 0; i < 12; ++i) e.v[i] = cmk(0.f, 0.f);
        if (!halo) load_spinor<float, S>(bb, bsc, g.V, s, r);
        if (halo) {
            // ---- r = b - D x.  Pass 1: in-block hops and the lower-face halo.
            if (own) load_spinor<float, S>(xx, xsc, g.V, s, e);
            {
                Spinor<float> hd;
                Link<float> Ldn;  // U_mu(site below the lower face), mu = wmu
                load_spinor<float, S>(xx, xsc, g.V, dn_site, hd);
                load_link<float, G>(a.links, g.V, dn_site, wmu, Ldn);
                if (own) v2_push(sm, l, true, fin, Uo, e);
                if (dn_wrap) apply_bc(g, wmu, -1, hd);
                switch (wax) {
                    case 0: s44_stage_backward<0>(Ldn, hd, 1.f, hb, top); break;
                    case 1: s44_stage_backward<3>(Ldn, hd, 1.f, hb, top); break;
                    case 2: s44_stage_backward<2>(Ldn, hd, 1.f, hb, top); break;
                    default: s44_stage_backward<1>(Ldn, hd, 1.f, hb, top); break;
                }
            }
            __syncthreads();
            Spinor<float> acc;
#pragma unroll
            for (int i = 0; i < 12; ++i) acc.v[i] = cmk(-0.f, -0.f);  // -0 + t = t: the first hop is stored
            if (own) {
#pragma unroll
                for (int mu = 0; mu < 4; ++mu) {
                    __builtin_amdgcn_sched_barrier(0);
                    if (fin[mu]) {
                        Half<float> h, gg;
                        project_forward_lds(sm.xs, mu, l + str[mu], h);
                        su3_mul(Uo[mu], h, gg);
                        forward_accumulate(mu, gg, acc);
                    }
                    __builtin_amdgcn_sched_barrier(0);
                    Half<float> gg;
                    v2_get_half(sm.gb, mu, bcol[mu], gg);
                    backward_accumulate(mu, gg, acc);
                }
            } else {
                // x zero on the block (own_zero): only the lower-face halo products, no in-block hops
#pragma unroll
                for (int mu = 0; mu < 4; ++mu) {
                    if (bcol[mu] > l) {  // bcol above l: a lower-face site, whose slot holds the halo
                        Half<float> gg;
                        v2_get_half(sm.gb, mu, bcol[mu], gg);
                        backward_accumulate(mu, gg, acc);
                    }
                }
            }
            __syncthreads();
            // ---- pass 2: the upper-face halo, staged in xs
            {
                Spinor<float> hu;
                load_spinor<float, S>(xx, xsc, g.V, up_site, hu);
                switch (wax) {
                    case 0: s44_stage_forward<0>(g, hu, up_wrap, sm.xs, l); break;
                    case 1: s44_stage_forward<3>(g, hu, up_wrap, sm.xs, l); break;
                    case 2: s44_stage_forward<2>(g, hu, up_wrap, sm.xs, l); break;
                    default: s44_stage_forward<1>(g, hu, up_wrap, sm.xs, l); break;
                }
            }
            __syncthreads();
#pragma unroll
            for (int mu = 0; mu < 4; ++mu) {
                if (!fin[mu]) {
                    Half<float> h, gg;
                    v2_get_half(sm.xs, 0, fsrc[mu], h);
                    su3_mul(Uo[mu], h, gg);
                    forward_accumulate(mu, gg, acc);
                }
            }
            // r = b + (acc - 2 A x) / 2
            if (own) clover_acc(A, -2.f * mu_tw, e, acc);
            // b only now: loaded earlier it would stay live through both passes and push
            // other values out of registers (this kernel has no room to spare at 2 waves/SIMD)
            load_spinor<float, S>(bb, bsc, g.V, s, r);
#pragma unroll
            for (int i = 0; i < 12; ++i) r.v[i] = r.v[i] + 0.5f * acc.v[i];
            __syncthreads();
        }

        // ---- minimal residual on D_BB with q = -2 D_BB rho
        Spinor<float>& rho = r;
        for (int it = 0; it < a.mr_iters; ++it) {
            v2_push(sm, l, true, fin, Uo, rho);
            __syncthreads();
            Spinor<float> q;
            float qr_re = 0.f, qr_im = 0.f, qq = 0.f;
            // -0 start: adding a term to -0 returns the term, so the first hop is stored, not added
#pragma unroll
            for (int i = 0; i < 12; ++i) q.v[i] = cmk(-0.f, -0.f);
            v2_pull(sm, l, fin, bin, str, Uo, q);
            clover_acc(A, -2.f * mu_tw, rho, q);
            mr_dots(q, rho, qr_re, qr_im, qq);
            block_sum3_w4(sm.red, qr_re, qr_im, qq);
            if (qq >= min_normal<float>()) {
                const float inv = __builtin_amdgcn_rcpf(qq);
                const cplx<float> alpha = cmk(qr_re * inv, qr_im * inv);
                const cplx<float> beta = cmk(-2.f * alpha.re, -2.f * alpha.im);
#pragma unroll
                for (int i = 0; i < 12; ++i) e.v[i] = cmad(beta, rho.v[i], e.v[i]);
                mr_residual_update(alpha, q, rho);
            }
        }
        // the site index again from an index the compiler cannot see through: held across the
        // MR steps it would be spilled and reloaded once per system
        int lo = l;
        asm volatile("" : "+v"(lo));
        const long long so = blk * 256 + lo;
        store_spinor<float, S>(xx, xsc, g.V, so, e);
        if constexpr (std::is_same<S, float>::value) {
            if (a.w_out) {
                // D x on the block, with x as just stored: the block's residual after the MR steps
                // is b - D x there (the other colour's x is unchanged), so D x = b - rho
                Spinor<float> t;
                load_spinor<float, S>(bb, bsc, g.V, so, t);
#pragma unroll
                for (int i = 0; i < 12; ++i) t.v[i] = t.v[i] - rho.v[i];
                store_spinor<float, S>(reinterpret_cast<char*>(a.w_out) + sys * stride, nullptr, g.V, so, t);
            }
        }
    }
}


// ---------------------------------------------------------------------------
// The operator out = D x on a lattice tiled in 4^4 blocks, FP32 arithmetic:
// one workgroup per block (every block, both colours), the block's stencil
// formed as in the residual of the half-sweep above (s44_stencil: links and
// clover in registers for all systems, the exchange and the halo in LDS), two
// workgroups per compute unit.  The generic k_dirac gathers its eight
// neighbours per thread from memory and holds its links at one wavefront per
// SIMD.
template <class Si, class So, class G, class C>
__global__ void __launch_bounds__(kV2) __attribute__((amdgpu_waves_per_eu(2, 2))) k_dirac_44(DiracArgs a) {
    __shared__ V2Shared sm;
    const Geo& g = a.g;
    const int l = threadIdx.x;

    int B[4];
    if (a.colour >= 0) {
        // the blocks of one colour, ordered as the half-sweep orders them
        s44_block(g, a.colour, xcd_swizzle(blockIdx.x, gridDim.x), B);
    } else {
        long long t = xcd_swizzle(blockIdx.x, gridDim.x);  // block index, lexicographic over the block grid
        B[3] = (int)(t % g.nb[3]);
        t /= g.nb[3];
        B[2] = (int)(t % g.nb[2]);
        t /= g.nb[2];
        B[1] = (int)(t % g.nb[1]);
        B[0] = (int)(t / g.nb[1]);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) B[q] = __builtin_amdgcn_readfirstlane(B[q]);
    const long long blk = s44_block_index(g, B);
    S44Site ix;
    s44_lane(g, B, blk, l, ix);
    int str[4];
    bool fin[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        str[q] = ix.str[q];
        fin[q] = ix.fin[q];
    }
    const int wax = __builtin_amdgcn_readfirstlane(ix.wax);
    const int wmu = wax == 0 ? 0 : 4 - wax;
    const size_t in_stride = (size_t)6 * g.V * Unit<Si>::bytes;
    const size_t out_stride = (size_t)6 * g.V * Unit<So>::bytes;

    Link<float> Uo[4];
    Clover<float> A;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) load_link<float, G>(a.links, g.V, ix.s, mu, Uo[mu]);
    load_clover<float, C>(a.clover, g.V, ix.s, A);
#pragma unroll
    for (int i = 0; i < 72; ++i) A.a[i] *= -2.f;

    for (int sys = 0; sys < a.nsys; ++sys) {
        // indices used outside the stencil's own loops recomputed per system (see k_sap_half_44)
        int lx = l;
        asm volatile("" : "+v"(lx));
        S44Site hx;
        s44_lane(g, B, blk, lx, hx);
        const long long s = hx.s;
        const float mu_tw = (float)(a.mu[sys] + g.mu_shift[hx.parity]);
        const void* in = reinterpret_cast<const char*>(a.in) + sys * in_stride;
        const float* isc = a.in_scale ? a.in_scale + (size_t)sys * g.V : nullptr;

        Spinor<float> e, acc;
        load_spinor<float, Si>(in, isc, g.V, s, e);
        s44_stencil<Si, G>(sm, g, a.links, in, isc, l, Uo, fin, str, hx, wax, wmu, e, acc);
        // out = (A + twist) x - acc / 2, from acc - 2 (A + twist) x
        clover_acc(A, -2.f * mu_tw, e, acc);
#pragma unroll
        for (int i = 0; i < 12; ++i) acc.v[i] = -0.5f * acc.v[i];
        store_spinor<float, So>(reinterpret_cast<char*>(a.out) + sys * out_stride,
                                a.out_scale ? a.out_scale + (size_t)sys * g.V : nullptr, g.V, s, acc);
        __syncthreads();  // every read of xs and gb done before the next system's push
    }
}

template <class Si, class So, class G, class C>
hipError_t run_dirac_44(const DiracArgs& a, hipStream_t st) {
    const long long nblocks = (long long)a.g.nb[0] * a.g.nb[1] * a.g.nb[2] * a.g.nb[3];
    const long long n = a.colour >= 0 ? nblocks / 2 : nblocks;
    hipLaunchKernelGGL((k_dirac_44<Si, So, G, C>), dim3((unsigned)n), dim3(kV2), 0, st, a);
    return hipGetLastError();
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
    if (a.eo) {
        const void* fe = nt <= 256 ? reinterpret_cast<const void*>(&k_sap_half_eo<S, G, C, R, 256>)
                                   : reinterpret_cast<const void*>(&k_sap_half_eo<S, G, C, R, 1024>);
        if (lds > 65536) {
            e = hipFuncSetAttribute(fe, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
        }
        if (nt <= 256)
            hipLaunchKernelGGL((k_sap_half_eo<S, G, C, R, 256>), grid, dim3(nt), lds, st, a);
        else
            hipLaunchKernelGGL((k_sap_half_eo<S, G, C, R, 1024>), grid, dim3(nt), lds, st, a);
        return hipGetLastError();
    }
    if constexpr (sizeof(R) == 4) {
        if (nt <= kV2 && !sap_v1_forced()) {
            const bool is44 = a.g.lb[0] == 4 && a.g.lb[1] == 4 && a.g.lb[2] == 4 && a.g.lb[3] == 4;
            if (is44 && !sap_v2_forced())
                hipLaunchKernelGGL((k_sap_half_44<S, G, C>), grid, dim3(nt), 0, st, a);
            else
                hipLaunchKernelGGL((k_sap_half_v2<S, G, C>), grid, dim3(nt), 0, st, a);
            return hipGetLastError();
        }
    }
    if constexpr (sizeof(R) == 8) {
        // FP64: one workgroup per CU either way (registers), so the block's links fit in LDS
        // beside the exchange buffer for blocks of up to 256 sites
        const size_t lds_lc = lds + (size_t)48 * nt * sizeof(R);
        if (nt <= 256 && lds_lc <= (size_t)max_lds) {
            const void* fl = reinterpret_cast<const void*>(&k_sap_half<S, G, C, R, 256, true>);
            if (lds_lc > 65536) {
                e = hipFuncSetAttribute(fl, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_lc);
                if (e != hipSuccess) return e;
            }
            hipLaunchKernelGGL((k_sap_half<S, G, C, R, 256, true>), grid, dim3(nt), lds_lc, st, a);
            return hipGetLastError();
        }
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

bool sap_fills_w(const Geo& g, Prec sp, Prec lp, Prec cp, bool eo) {
    const bool is44 = g.lb[0] == 4 && g.lb[1] == 4 && g.lb[2] == 4 && g.lb[3] == 4;
    return is44 && !eo && sp == P_F32 && lp == P_F32 && cp == P_F32 && !sap_v1_forced() && !sap_v2_forced();
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

hipError_t launch_dirac_44(const DiracArgs& a, Prec in_p, Prec out_p, Prec link_p, Prec clover_p,
                           hipStream_t st) {
    const bool is44 = a.g.lb[0] == 4 && a.g.lb[1] == 4 && a.g.lb[2] == 4 && a.g.lb[3] == 4;
    if (!is44 || sap_v1_forced() || sap_v2_forced()) return hipErrorNotSupported;
    if (in_p == P_F32 && out_p == P_F32 && link_p == P_F32 && clover_p == P_F32)
        return run_dirac_44<float, float, float, float>(a, st);
    if (in_p == P_F16 && out_p == P_F16 && link_p == P_F16 && clover_p == P_F32)
        return run_dirac_44<f16, f16, f16, float>(a, st);
    if (in_p == P_BF16 && out_p == P_BF16 && link_p == P_BF16 && clover_p == P_F32)
        return run_dirac_44<bf16, bf16, bf16, float>(a, st);
    if (in_p == P_F16 && out_p == P_F32 && link_p == P_F32 && clover_p == P_F32)
        return run_dirac_44<f16, float, float, float>(a, st);
    if (in_p == P_BF16 && out_p == P_F32 && link_p == P_F32 && clover_p == P_F32)
        return run_dirac_44<bf16, float, float, float>(a, st);
    return hipErrorNotSupported;
}

}  // namespace tmsap
