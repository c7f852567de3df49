// Two-level method (sections 2.3 and 2.4): the aggregation basis P, the
// restriction P^+ and prolongation P, the Galerkin coarse stencil P^+ D P and
// the coarse operator D_c + i delta mu Gamma5c, plus the vector kernels of the
// coarse GMRES.  Layouts are described in tm_mg.h.
//
// Per-aggregate kernels run one workgroup per aggregate (tile) with one site
// per thread; their reductions go through wavefront shuffles and LDS in a
// fixed order, so results do not depend on scheduling.
#include "tm_mg.h"

namespace tmsap {

namespace {

constexpr int kThreads = 256;
constexpr int kCoarseSys = 16;  // systems per coarse-operator workgroup
constexpr int kDots = 16;       // basis vectors per dot / axpy pass

__device__ inline float wave_sum(float v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ inline double wave_sum_d(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ inline const void* field(const void* base, size_t stride, int i) {
    return static_cast<const char*>(base) + (size_t)i * stride;
}

// Column b of P at site y: field b % nv with the other spin half zeroed.
__device__ inline void load_column(const MgArgs& m, int b, long long y, Spinor<float>& p) {
    const int i = b % m.nv, sg = b / m.nv;
    load_spinor<float, float>(field(m.P, m.P_stride, i), nullptr, m.g.V, y, p);
#pragma unroll
    for (int q = 0; q < 6; ++q) p.v[sg == 0 ? 6 + q : q] = cmk(0.f, 0.f);
}

template <int T>
__global__ void __launch_bounds__(kThreads) k_mg_term(MgArgs m, const void* __restrict__ links,
                                                      const void* __restrict__ clover, int b0, int nb, void* out,
                                                      size_t out_stride) {
    constexpr int t = T;
    const Geo& g = m.g;
    const long long s = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (s >= g.V) return;
    int nf[4], nbk[4], par;
    unsigned wrap;
    tiled_neighbours(g, s, nf, nbk, &wrap, &par);
    const unsigned blk = (unsigned)s / (unsigned)g.Vb;
    constexpr int mu = t == 0 ? 0 : (t - 1) % 4;
    constexpr bool fwd = t >= 1 && t <= 4;
    // neighbours along mu picked with static indices (no private-array indexing)
    int nfm = nf[0], nbm = nbk[0];
#pragma unroll
    for (int d = 1; d < 4; ++d)
        if (d == mu) {
            nfm = nf[d];
            nbm = nbk[d];
        }
    // the face hop of term t exists at this site only when it leaves the aggregate
    const bool face = t == 0 ? false : ((unsigned)(fwd ? nfm : nbm) / (unsigned)g.Vb != blk);
    Clover<float> A;
    if (t == 0) load_clover<float, float>(clover, g.V, s, A);
    for (int b = b0; b < b0 + nb; ++b) {
        Spinor<float> o, h, p;
#pragma unroll
        for (int q = 0; q < 12; ++q) o.v[q] = h.v[q] = cmk(0.f, 0.f);
        if (t == 0) {
            load_column(m, b, s, p);
            clover_apply(A, (float)g.mu_shift[par], p, o);
#pragma unroll
            for (int d = 0; d < 4; ++d) {
                if ((unsigned)nf[d] / (unsigned)g.Vb == blk) {
                    Link<float> L;
                    load_link<float, float>(links, g.V, s, d, L);
                    load_column(m, b, nf[d], p);
                    if (wrap & (1u << d)) apply_bc(g, d, +1, p);
                    hop_forward(d, L, p, 1.f, h);
                }
                if ((unsigned)nbk[d] / (unsigned)g.Vb == blk) {
                    Link<float> L;
                    load_link<float, float>(links, g.V, nbk[d], d, L);
                    load_column(m, b, nbk[d], p);
                    if (wrap & (16u << d)) apply_bc(g, d, -1, p);
                    hop_backward(d, L, p, 1.f, h);
                }
            }
        } else if (face) {
            Link<float> L;
            if (fwd) {
                load_link<float, float>(links, g.V, s, mu, L);
                load_column(m, b, nfm, p);
                if (wrap & (1u << mu)) apply_bc(g, mu, +1, p);
                hop_forward(mu, L, p, 1.f, h);
            } else {
                load_link<float, float>(links, g.V, nbm, mu, L);
                load_column(m, b, nbm, p);
                if (wrap & (16u << mu)) apply_bc(g, mu, -1, p);
                hop_backward(mu, L, p, 1.f, h);
            }
        }
#pragma unroll
        for (int q = 0; q < 12; ++q) o.v[q] = o.v[q] - 0.5f * h.v[q];
        store_spinor<float, float>(static_cast<char*>(out) + (size_t)(b - b0) * out_stride, nullptr, g.V, s, o);
    }
}

// Sum over the 64 lanes of a wave of 64 values per lane: after the exchange lane l
// holds the sum of value l.  Each step halves the values a lane keeps (it keeps the
// half selected by its lane bit and adds its partner's copy of that half), so the
// reduction costs 63 exchanges instead of 6 per value.
template <int H>
__device__ inline void transpose_step(float (&v)[64], int lane) {
    const bool up = lane & H;
#pragma unroll
    for (int i = 0; i < H; ++i) {
        const float send = up ? v[i] : v[i + H];
        const float keep = up ? v[i + H] : v[i];
        v[i] = keep + __shfl_xor(send, H, 64);
    }
    if constexpr (H > 1) transpose_step<H / 2>(v, lane);
}

__device__ inline float transpose_sum64(float (&v)[64]) {
    transpose_step<32>(v, threadIdx.x & 63);
    return v[0];
}

// Aggregate and system group of workgroup b when each aggregate has G system groups:
// runs of 8 aggregates take 8 G consecutive workgroups, group-major, so the G
// workgroups of one aggregate are 8 apart.  Workgroups are dealt to the 8 XCDs in
// turn, so all of an aggregate's groups run at about the same time on one XCD and
// the later ones find its part of P in that XCD's L2.
__device__ inline void agg_group(int b, int G, long long nc, int& j, int& grp) {
    constexpr int X = 8;
    const int run = b / (X * G);
    const int base = run * X;
    const int width = (int)min((long long)X, nc - base);
    const int within = b - run * X * G;
    grp = within / width;
    j = base + (within - grp * width);
}

// Restriction of S systems per workgroup (one aggregate of at most NT sites).
// Per site and test vector the 4 S partial sums (two spin halves, re / im, per
// system) of 16 / S test vectors at a time go through one wave-level transpose
// sum; the wave sums meet in LDS.
template <int S, int NT>
__global__ void __launch_bounds__(NT) k_mg_restrict(MgArgs m, const void* __restrict__ x, size_t x_stride,
                                                      int nsys, float2* out, size_t base, size_t s_stride,
                                                      size_t j_stride) {
    constexpr int PER = 16 / S;  // test vectors per 64-value chunk
    extern __shared__ float red[];  // [waves][chunks][64]
    const Geo& g = m.g;
    int j, grp;
    agg_group(blockIdx.x, (nsys + S - 1) / S, g.V / g.Vb, j, grp);
    const int l = threadIdx.x;
    const bool on = l < g.Vb;
    const long long s = (long long)j * g.Vb + l;
    const int s0 = grp * S;
    const int ns = min(S, nsys - s0);
    const int lane = l & 63, w = l >> 6, nw = blockDim.x >> 6, nv = m.nv;
    const int nch = (nv + PER - 1) / PER;
    Spinor<float> xv[S];
#pragma unroll
    for (int k = 0; k < S; ++k) {
        if (on && k < ns)
            load_spinor<float, float>(field(x, x_stride, s0 + k), nullptr, g.V, s, xv[k]);
        else
#pragma unroll
            for (int q = 0; q < 12; ++q) xv[k].v[q] = cmk(0.f, 0.f);
    }
    for (int c = 0; c < nch; ++c) {
        float v[64];
#pragma unroll
        for (int ii = 0; ii < PER; ++ii) {
            const int i = c * PER + ii;
            Spinor<float> p;
            if (on && i < nv)
                load_spinor<float, float>(field(m.P, m.P_stride, i), nullptr, g.V, s, p);
            else
#pragma unroll
                for (int q = 0; q < 12; ++q) p.v[q] = cmk(0.f, 0.f);
#pragma unroll
            for (int k = 0; k < S; ++k) {
                float d[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int q = 0; q < 12; ++q) {
                    const int h = q < 6 ? 0 : 2;
                    // one product per statement: each becomes one fused multiply-add
                    d[h] = d[h] + p.v[q].re * xv[k].v[q].re;
                    d[h] = d[h] + p.v[q].im * xv[k].v[q].im;
                    d[h + 1] = d[h + 1] + p.v[q].re * xv[k].v[q].im;
                    d[h + 1] = d[h + 1] - p.v[q].im * xv[k].v[q].re;
                }
#pragma unroll
                for (int e = 0; e < 4; ++e) v[(ii * S + k) * 4 + e] = d[e];
            }
        }
        red[(w * nch + c) * 64 + lane] = transpose_sum64(v);
    }
    __syncthreads();
    const int n2 = 2 * nv;
    for (int idx = l; idx < ns * n2; idx += blockDim.x) {
        const int k = idx / n2, a = idx - k * n2, sg = a / nv, i = a - sg * nv;
        const int c = i / PER, vi = ((i - c * PER) * S + k) * 4 + 2 * sg;
        float re = 0.f, im = 0.f;
        for (int q = 0; q < nw; ++q) {
            re += red[(q * nch + c) * 64 + vi];
            im += red[(q * nch + c) * 64 + vi + 1];
        }
        out[base + (size_t)(s0 + k) * s_stride + (size_t)j * j_stride + a] = make_float2(re, im);
    }
}

template <int S, int NT>
__global__ void __launch_bounds__(NT) k_mg_prolong(MgArgs m, const float2* __restrict__ c, int nsys, void* e,
                                                     size_t e_stride) {
    extern __shared__ float2 cs[];  // [S][2 nv]
    const Geo& g = m.g;
    const long long nc = g.V / g.Vb;
    int j, grp;
    agg_group(blockIdx.x, (nsys + S - 1) / S, nc, j, grp);
    const int l = threadIdx.x, nv = m.nv, n2 = 2 * nv;
    const int s0 = grp * S;
    const int ns = min(S, nsys - s0);
    for (int idx = l; idx < ns * n2; idx += blockDim.x) {
        const int k = idx / n2, a = idx - k * n2;
        cs[idx] = c[((size_t)(s0 + k) * nc + j) * n2 + a];
    }
    __syncthreads();
    if (l >= g.Vb) return;
    const long long s = (long long)j * g.Vb + l;
    Spinor<float> acc[S];
#pragma unroll
    for (int k = 0; k < S; ++k)
#pragma unroll
        for (int q = 0; q < 12; ++q) acc[k].v[q] = cmk(0.f, 0.f);
    for (int i = 0; i < nv; ++i) {
        Spinor<float> p;
        load_spinor<float, float>(field(m.P, m.P_stride, i), nullptr, g.V, s, p);
#pragma unroll
        for (int k = 0; k < S; ++k) {
            if (k < ns) {
                const float2 c0 = cs[k * n2 + i], c1 = cs[k * n2 + nv + i];
                const cplx<float> u = cmk(c0.x, c0.y), d = cmk(c1.x, c1.y);
#pragma unroll
                for (int q = 0; q < 12; ++q) acc[k].v[q] = cmad(p.v[q], q < 6 ? u : d, acc[k].v[q]);
            }
        }
    }
#pragma unroll
    for (int k = 0; k < S; ++k)
        if (k < ns) store_spinor<float, float>(static_cast<char*>(e) + (size_t)(s0 + k) * e_stride, nullptr, g.V, s,
                                               acc[k]);
}

// Sum of (a, b) over the workgroup, returned to every thread (FP64).
__device__ inline void block_sum2(double* lds, double& a, double& b) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    a = wave_sum_d(a);
    b = wave_sum_d(b);
    if (lane == 0) {
        lds[2 * w] = a;
        lds[2 * w + 1] = b;
    }
    __syncthreads();
    a = 0;
    b = 0;
    for (int q = 0; q < nw; ++q) {
        a += lds[2 * q];
        b += lds[2 * q + 1];
    }
    __syncthreads();
}

__global__ void __launch_bounds__(1024) k_mg_block_orthonormalize(MgArgs m, void* P) {
    __shared__ double lds[32];
    const Geo& g = m.g;
    const int j = blockIdx.x, sg = blockIdx.y, l = threadIdx.x;
    const bool on = l < g.Vb;
    const long long s = (long long)j * g.Vb + l;
    const int u0 = 3 * sg;
    for (int i = 0; i < m.nv; ++i) {
        float4* Pi = reinterpret_cast<float4*>(static_cast<char*>(P) + (size_t)i * m.P_stride);
        float4 v[3];
#pragma unroll
        for (int u = 0; u < 3; ++u) v[u] = on ? Pi[(size_t)(u0 + u) * g.V + s] : make_float4(0.f, 0.f, 0.f, 0.f);
        for (int k = 0; k < i; ++k) {
            const float4* Pk = reinterpret_cast<const float4*>(static_cast<const char*>(P) + (size_t)k * m.P_stride);
            float4 q[3];
            double re = 0, im = 0;
#pragma unroll
            for (int u = 0; u < 3; ++u) {
                q[u] = on ? Pk[(size_t)(u0 + u) * g.V + s] : make_float4(0.f, 0.f, 0.f, 0.f);
                re += (double)q[u].x * v[u].x + (double)q[u].y * v[u].y + (double)q[u].z * v[u].z +
                      (double)q[u].w * v[u].w;
                im += (double)q[u].x * v[u].y - (double)q[u].y * v[u].x + (double)q[u].z * v[u].w -
                      (double)q[u].w * v[u].z;
            }
            block_sum2(lds, re, im);
            const float hr = (float)re, hi = (float)im;
#pragma unroll
            for (int u = 0; u < 3; ++u) {
                v[u].x -= hr * q[u].x - hi * q[u].y;
                v[u].y -= hr * q[u].y + hi * q[u].x;
                v[u].z -= hr * q[u].z - hi * q[u].w;
                v[u].w -= hr * q[u].w + hi * q[u].z;
            }
        }
        double n2 = 0, dummy = 0;
#pragma unroll
        for (int u = 0; u < 3; ++u)
            n2 += (double)v[u].x * v[u].x + (double)v[u].y * v[u].y + (double)v[u].z * v[u].z +
                  (double)v[u].w * v[u].w;
        block_sum2(lds, n2, dummy);
        const float f = n2 > 0 ? (float)(1.0 / sqrt(n2)) : 0.f;
        if (on)
#pragma unroll
            for (int u = 0; u < 3; ++u)
                Pi[(size_t)(u0 + u) * g.V + s] = make_float4(f * v[u].x, f * v[u].y, f * v[u].z, f * v[u].w);
    }
}

__device__ inline int coarse_parity(const Geo& g, long long j) {
    int sum = 0;
    for (int a = 3; a >= 0; --a) {
        sum += (int)(j % g.nb[a]);
        j /= g.nb[a];
    }
    return sum & 1;
}

// One workgroup per coarse site and group of kCoarseSys systems.  The 9 stencil
// matrices of the site are 9 * n2 columns of n2 complex numbers, stored one after
// the other; thread t takes the row pair (2p, 2p + 1) with p = t % nv of the columns
// c = t / nv, t / nv + G, ... (G = 256 / nv column groups), so a wavefront reads
// consecutive 16-byte pieces and every thread has its own stream of loads.  The
// neighbours' x are staged in LDS; the column groups' partial sums meet there too.
// General form: y = add + (self term + i mu_c Gamma5c) x_self + hop_sign * (8 neighbour terms) x_hop
// on the coarse sites of `parity` (all sites when parity < 0); a null input drops its terms, a
// null mu_c the twist.  The other parity's sites get 0 when zero_other is set, else stay as they are.
// With a parity the grid covers site pairs (2b, 2b + 1), one of each parity since the innermost
// coarse extent is even: the workgroup computes its pair's site of `parity` (and zeroes the other).
__global__ void __launch_bounds__(kThreads) k_mg_coarse_apply(Geo g, int nv, const float2* __restrict__ Dc,
                                                              const double* __restrict__ mu_c,
                                                              const float2* __restrict__ x_self,
                                                              const float2* __restrict__ x_hop, float hop_sign,
                                                              const float2* add, int parity, int zero_other,
                                                              float2* y, int nsys) {
    // xs [9][ks][n2]; then [G][ks][n2] partial sums, ks = systems per workgroup (LDS sized by it)
    extern __shared__ float2 sh[];
    const int n2 = 2 * nv;
    const int ks = min(kCoarseSys, nsys);
    const long long nc = g.V / g.Vb;
    const int s0 = blockIdx.y * kCoarseSys;
    const int ns = min(kCoarseSys, nsys - s0);
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // one (term, system) row per wavefront
    constexpr int kWaves = kThreads / 64;
    long long j = blockIdx.x;
    if (parity >= 0) {
        const long long j0 = 2 * (long long)blockIdx.x;
        j = coarse_parity(g, j0) == parity ? j0 : j0 + 1;
        if (zero_other && lane < n2) {
            const long long jo = 2 * j0 + 1 - j;
            for (int k = wave; k < ns; k += kWaves) y[((size_t)(s0 + k) * nc + jo) * n2 + lane] = make_float2(0.f, 0.f);
        }
    }
    // coordinates of j once; the 8 neighbours by one coordinate step each
    int Bj[4];
    {
        int rem = (int)j;
#pragma unroll
        for (int a = 3; a >= 0; --a) {
            Bj[a] = rem % g.nb[a];
            rem /= g.nb[a];
        }
    }
    for (int tk = wave; tk < 9 * ns; tk += kWaves) {
        const int t = tk / ns, k = tk - t * ns;
        const float2* src = t == 0 ? x_self : x_hop;
        if (lane < n2) {
            float2 v = make_float2(0.f, 0.f);
            if (src) {
                int site = (int)j;
                if (t > 0) {
                    const int a = axis_of((t - 1) & 3), step = t <= 4 ? 1 : -1;
                    site = 0;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        int c = Bj[q];
                        if (q == a) {
                            c += step;
                            if (c == g.nb[q]) c = 0;
                            if (c < 0) c = g.nb[q] - 1;
                        }
                        site = site * g.nb[q] + c;
                    }
                }
                v = src[((size_t)(s0 + k) * nc + site) * n2 + lane];
                if (t > 0) v = make_float2(hop_sign * v.x, hop_sign * v.y);
            }
            sh[(t * ks + k) * n2 + lane] = v;
        }
    }
    __syncthreads();
    const int G = kThreads / nv;
    const int p = tid % nv, grp = tid / nv;
    float2 acc0[kCoarseSys], acc1[kCoarseSys];
#pragma unroll
    for (int k = 0; k < kCoarseSys; ++k) acc0[k] = acc1[k] = make_float2(0.f, 0.f);
    if (grp < G) {
        const float4* A = reinterpret_cast<const float4*>(Dc + (size_t)j * 9 * n2 * n2);
        const int c_lo = x_self ? 0 : n2, c_hi = x_hop ? 9 * n2 : n2;
        // column c = t n2 + r: term t, component r, stepped without a division per column
        const int dt = G / n2, dr = G - dt * n2;
        int t = (c_lo + grp) / n2, r = c_lo + grp - t * n2;
#pragma unroll 8
        for (int c = c_lo + grp; c < c_hi; c += G) {
            const float4 mv = A[(size_t)c * nv + p];  // rows 2p, 2p + 1 of column c
            const float2* xs = sh + (t * ks) * n2 + r;
            t += dt;
            r += dr;
            if (r >= n2) {
                r -= n2;
                ++t;
            }
#pragma unroll
            for (int k = 0; k < kCoarseSys; ++k) {
                if (k < ns) {
                    const float2 xv = xs[k * n2];
                    // one product per statement: each becomes one fused multiply-add
                    acc0[k].x = acc0[k].x + mv.x * xv.x;
                    acc0[k].x = acc0[k].x - mv.y * xv.y;
                    acc0[k].y = acc0[k].y + mv.x * xv.y;
                    acc0[k].y = acc0[k].y + mv.y * xv.x;
                    acc1[k].x = acc1[k].x + mv.z * xv.x;
                    acc1[k].x = acc1[k].x - mv.w * xv.y;
                    acc1[k].y = acc1[k].y + mv.z * xv.y;
                    acc1[k].y = acc1[k].y + mv.w * xv.x;
                }
            }
        }
    }
    __syncthreads();
    if (grp < G)
#pragma unroll
        for (int k = 0; k < kCoarseSys; ++k)
            if (k < ns) {
                sh[(grp * ks + k) * n2 + 2 * p] = acc0[k];
                sh[(grp * ks + k) * n2 + 2 * p + 1] = acc1[k];
            }
    __syncthreads();
    for (int k = wave; k < ns && lane < n2; k += kWaves) {
        const int r = lane;
        float2 sum = make_float2(0.f, 0.f);
        for (int q = 0; q < G; ++q) {
            const float2 v = sh[(q * ks + k) * n2 + r];
            sum.x += v.x;
            sum.y += v.y;
        }
        const size_t at = ((size_t)(s0 + k) * nc + j) * n2 + r;
        if (x_self && mu_c) {
            const float2 xv = x_self[at];
            const float tw = (float)mu_c[s0 + k] * (r < nv ? 1.f : -1.f);
            sum.x -= tw * xv.y;
            sum.y += tw * xv.x;
        }
        if (add) {
            const float2 av = add[at];
            sum.x += av.x;
            sum.y += av.y;
        }
        y[at] = sum;
    }
}

// (Dc[j][0] + i mu_c Gamma5c)^-1 at the coarse sites of `parity`, by Gauss-Jordan
// elimination with partial pivoting in FP64 (augmented matrix in LDS).  One workgroup
// per site pair (2b, 2b + 1), for its site j of `parity`; the result goes to Minv[b]
// (= Minv[j >> 1]) as FP32, column-major like the stencil (the innermost coarse extent
// is even, so the pair holds one site of each parity).
__global__ void __launch_bounds__(kThreads) k_mg_block_inverse(Geo g, int nv, const float2* __restrict__ Dc,
                                                               double mu_c, int parity, float2* Minv) {
    extern __shared__ double2 aug[];  // [n2][2 n2] row-major
    __shared__ double2 fac[64];
    __shared__ int piv_s;
    const long long j0 = 2 * (long long)blockIdx.x;
    const long long j = coarse_parity(g, j0) == parity ? j0 : j0 + 1;
    const int n2 = 2 * nv, W = 2 * n2, tid = threadIdx.x;
    const float2* A = Dc + (size_t)j * 9 * n2 * n2;
    for (int idx = tid; idx < n2 * W; idx += kThreads) {
        const int r = idx / W, c = idx - r * W;
        double2 v = make_double2(0.0, 0.0);
        if (c < n2) {
            const float2 a = A[(size_t)c * n2 + r];
            v = make_double2(a.x, a.y);
            if (c == r) v.y += mu_c * (r < nv ? 1.0 : -1.0);
        } else if (c - n2 == r) {
            v.x = 1.0;
        }
        aug[idx] = v;
    }
    __syncthreads();
    for (int k = 0; k < n2; ++k) {
        if (tid < 64) {  // pivot: largest |a_rk| for r >= k, the first on ties
            const int r = k + tid;
            double val = -1.0;
            int at = r;
            if (r < n2) {
                const double2 a = aug[r * W + k];
                val = a.x * a.x + a.y * a.y;
            }
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) {
                const double ov = __shfl_xor(val, off, 64);
                const int oa = __shfl_xor(at, off, 64);
                if (ov > val || (ov == val && oa < at)) {
                    val = ov;
                    at = oa;
                }
            }
            if (tid == 0) piv_s = at;
        }
        __syncthreads();
        const int piv = piv_s;
        if (piv != k)
            for (int c = tid; c < W; c += kThreads) {
                const double2 t = aug[k * W + c];
                aug[k * W + c] = aug[piv * W + c];
                aug[piv * W + c] = t;
            }
        __syncthreads();
        const double2 d = aug[k * W + k];
        const double dn = d.x * d.x + d.y * d.y;
        const double2 inv = make_double2(d.x / dn, -d.y / dn);
        __syncthreads();
        for (int c = tid; c < W; c += kThreads) {
            const double2 a = aug[k * W + c];
            aug[k * W + c] = make_double2(a.x * inv.x - a.y * inv.y, a.x * inv.y + a.y * inv.x);
        }
        for (int r = tid; r < n2; r += kThreads) fac[r] = r == k ? make_double2(0.0, 0.0) : aug[r * W + k];
        __syncthreads();
        for (int idx = tid; idx < n2 * W; idx += kThreads) {
            const int r = idx / W, c = idx - r * W;
            if (r == k) continue;
            const double2 f = fac[r], p = aug[k * W + c];
            const double2 a = aug[idx];
            aug[idx] = make_double2(a.x - (f.x * p.x - f.y * p.y), a.y - (f.x * p.y + f.y * p.x));
        }
        __syncthreads();
    }
    float2* out = Minv + (size_t)blockIdx.x * n2 * n2;
    for (int idx = tid; idx < n2 * n2; idx += kThreads) {
        const int c = idx / n2, r = idx - c * n2;  // column-major
        const double2 v = aug[r * W + n2 + c];
        out[idx] = make_float2((float)v.x, (float)v.y);
    }
}

// y_s = Minv_{sel[s]} x_s at the coarse sites of `parity` (the others get 0 when zero_other
// is set, else stay as they are).  One 64-lane workgroup per site pair (2b, 2b + 1), whose
// site of `parity` has inverse b; one lane per row; the systems of one inverse set go in
// chunks of kBlockMulSys, so each inverse is read from memory once per call.
constexpr int kBlockMulSys = 8;
__global__ void __launch_bounds__(64) k_mg_block_mul(BlockMulArgs a) {
    __shared__ float2 xs[kBlockMulSys][64];
    const Geo& g = a.g;
    const long long j0 = 2 * (long long)blockIdx.x;
    const long long j = coarse_parity(g, j0) == a.parity ? j0 : j0 + 1;
    const int lane = threadIdx.x, n2 = 2 * a.nv;
    const long long nc = g.V / g.Vb;
    if (a.zero_other && lane < n2) {
        const long long jo = 2 * j0 + 1 - j;
        for (int s = 0; s < a.nsys; ++s) a.y[((size_t)s * nc + jo) * n2 + lane] = make_float2(0.f, 0.f);
    }
    for (int q = 0; q < kMgMaxInv; ++q) {
        if (a.start[q] == a.start[q + 1]) continue;
        const float2* M = a.sets[q] + (size_t)blockIdx.x * n2 * n2 + lane;
        for (int c0 = a.start[q]; c0 < a.start[q + 1]; c0 += kBlockMulSys) {
            const int cn = min(kBlockMulSys, a.start[q + 1] - c0);
            __syncthreads();
            if (lane < n2)
                for (int k = 0; k < cn; ++k) xs[k][lane] = a.x[((size_t)a.order[c0 + k] * nc + j) * n2 + lane];
            __syncthreads();
            if (lane < n2) {
                float2 acc[kBlockMulSys];
#pragma unroll
                for (int k = 0; k < kBlockMulSys; ++k) acc[k] = make_float2(0.f, 0.f);
                for (int b = 0; b < n2; ++b) {
                    const float2 m = M[(size_t)b * n2];
#pragma unroll
                    for (int k = 0; k < kBlockMulSys; ++k) {
                        const float2 v = xs[k][b];
                        acc[k].x = acc[k].x + m.x * v.x;  // one fused multiply-add per product
                        acc[k].x = acc[k].x - m.y * v.y;
                        acc[k].y = acc[k].y + m.x * v.y;
                        acc[k].y = acc[k].y + m.y * v.x;
                    }
                }
#pragma unroll
                for (int k = 0; k < kBlockMulSys; ++k)
                    if (k < cn) a.y[((size_t)a.order[c0 + k] * nc + j) * n2 + lane] = acc[k];
            }
        }
    }
}

__global__ void k_mg_stencil_export(long long nc, int nv, const float2* __restrict__ Dc, double2* out) {
    const int n2 = 2 * nv;
    const long long total = nc * 9 * n2 * n2;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        // e indexes the row-major output [j][t][a][b]
        const long long mt = e / (n2 * n2);
        const int r = (int)(e - mt * n2 * n2), a = r / n2, b = r - a * n2;
        const float2 v = Dc[(size_t)mt * n2 * n2 + (size_t)b * n2 + a];
        out[e] = make_double2(v.x, v.y);
    }
}

__global__ void k_mg_coarse_import(const double2* __restrict__ in, float2* v, long long n, unsigned* flag) {
    bool bad = false;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
        const double2 t = in[e];
        bad |= !isfinite(t.x) || !isfinite(t.y);
        v[e] = make_float2((float)t.x, (float)t.y);
    }
    if (bad) atomicOr(flag, 1u);
}

__global__ void k_mg_coarse_export(const float2* __restrict__ v, double2* out, long long n) {
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x)
        out[e] = make_double2(v[e].x, v[e].y);
}

// ---- coarse vector kernels (float2 pairs read as float4; n is even)

__global__ void __launch_bounds__(kThreads) k_cdots(const float2* __restrict__ basis, size_t vec_stride, int cnt,
                                                    const float2* __restrict__ w, size_t sys_stride, long long n,
                                                    double* partials) {
    __shared__ double lds[(kThreads / 64) * 2 * kDots];
    const int sys = blockIdx.y, nblk = gridDim.x;
    const float4* w4 = reinterpret_cast<const float4*>(w + (size_t)sys * sys_stride);
    double acc[2 * kDots];
#pragma unroll
    for (int i = 0; i < 2 * kDots; ++i) acc[i] = 0;
    const long long n4 = n / 2;
    for (long long e = (long long)blockIdx.x * kThreads + threadIdx.x; e < n4; e += (long long)nblk * kThreads) {
        const float4 wv = w4[e];
#pragma unroll
        for (int i = 0; i < kDots; ++i) {
            if (i < cnt) {
                const float4 v = reinterpret_cast<const float4*>(basis + (size_t)i * vec_stride + (size_t)sys * sys_stride)[e];
                acc[2 * i] += (double)(v.x * wv.x + v.y * wv.y + v.z * wv.z + v.w * wv.w);
                acc[2 * i + 1] += (double)(v.x * wv.y - v.y * wv.x + v.z * wv.w - v.w * wv.z);
            }
        }
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < 2 * kDots; ++i) {
        if (i < 2 * cnt) {
            const double v = wave_sum_d(acc[i]);
            if (lane == 0) lds[wv * 2 * kDots + i] = v;
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < 2 * cnt) {
        double t = 0;
        for (int q = 0; q < kThreads / 64; ++q) t += lds[q * 2 * kDots + threadIdx.x];
        partials[((size_t)sys * 2 * cnt + threadIdx.x) * nblk + blockIdx.x] = t;
    }
}

// out values (per system, nval consecutive doubles) from the per-workgroup partials, summed in order
// Panel products for Gram-Schmidt of fields that share one basis: out (s, i) = <v_i, w_s> for
// i < cnt <= kPanelDots and s < nw <= kPanel, every basis and panel vector read once.
constexpr int kPanel = 4;
constexpr int kPanelDots = 4;
constexpr int kPanelAxpy = 8;
__global__ void __launch_bounds__(kThreads) k_pdots(const float2* __restrict__ basis, size_t vec_stride, int cnt,
                                                    const float2* __restrict__ w, size_t w_stride, int nw,
                                                    long long n, double* partials) {
    constexpr int NA = 2 * kPanelDots * kPanel;
    __shared__ double lds[(kThreads / 64) * NA];
    const int nblk = gridDim.x;
    double acc[NA];
#pragma unroll
    for (int i = 0; i < NA; ++i) acc[i] = 0;
    const long long n4 = n / 2;
    for (long long e = (long long)blockIdx.x * kThreads + threadIdx.x; e < n4; e += (long long)nblk * kThreads) {
        float4 wv[kPanel];
#pragma unroll
        for (int s = 0; s < kPanel; ++s)
            wv[s] = s < nw ? reinterpret_cast<const float4*>(w + (size_t)s * w_stride)[e] : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
        for (int i = 0; i < kPanelDots; ++i) {
            if (i < cnt) {
                const float4 v = reinterpret_cast<const float4*>(basis + (size_t)i * vec_stride)[e];
#pragma unroll
                for (int s = 0; s < kPanel; ++s) {
                    acc[2 * (s * kPanelDots + i)] += (double)(v.x * wv[s].x + v.y * wv[s].y + v.z * wv[s].z + v.w * wv[s].w);
                    acc[2 * (s * kPanelDots + i) + 1] +=
                        (double)(v.x * wv[s].y - v.y * wv[s].x + v.z * wv[s].w - v.w * wv[s].z);
                }
            }
        }
    }
    const int lane = threadIdx.x & 63, wvi = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < NA; ++i) {
        const double v = wave_sum_d(acc[i]);
        if (lane == 0) lds[wvi * NA + i] = v;
    }
    __syncthreads();
    // partials laid out for k_reduce: value k = 2 i + re/im of panel vector s at ((s * 2 cnt + k) * nblk + block)
    const int t = threadIdx.x;
    if (t < 2 * cnt * nw) {
        const int sv = t / (2 * cnt), k = t - sv * 2 * cnt;
        double sum = 0;
        for (int q = 0; q < kThreads / 64; ++q) sum += lds[q * NA + 2 * sv * kPanelDots + k];
        partials[((size_t)sv * 2 * cnt + k) * nblk + blockIdx.x] = sum;
    }
}

// w_s -= sum_i coef[s][i] v_i for s < nw <= kPanel, i < cnt <= kPanelAxpy (coef double2 at
// coef + s * coef_stride + i); every basis vector read once for the whole panel.
__global__ void __launch_bounds__(kThreads) k_paxpy(const float2* __restrict__ basis, size_t vec_stride, int cnt,
                                                    const double2* __restrict__ coef, int coef_stride, float2* w,
                                                    size_t w_stride, int nw, long long n) {
    float cr[kPanel][kPanelAxpy], ci[kPanel][kPanelAxpy];
#pragma unroll
    for (int s = 0; s < kPanel; ++s)
#pragma unroll
        for (int i = 0; i < kPanelAxpy; ++i) {
            const double2 c = (s < nw && i < cnt) ? coef[(size_t)s * coef_stride + i] : make_double2(0.0, 0.0);
            cr[s][i] = -(float)c.x;
            ci[s][i] = -(float)c.y;
        }
    const long long n4 = n / 2;
    for (long long e = (long long)blockIdx.x * kThreads + threadIdx.x; e < n4; e += (long long)gridDim.x * kThreads) {
        float4 t[kPanel];
#pragma unroll
        for (int s = 0; s < kPanel; ++s)
            t[s] = s < nw ? reinterpret_cast<const float4*>(w + (size_t)s * w_stride)[e] : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
        for (int i = 0; i < kPanelAxpy; ++i) {
            if (i < cnt) {
                const float4 v = reinterpret_cast<const float4*>(basis + (size_t)i * vec_stride)[e];
#pragma unroll
                for (int s = 0; s < kPanel; ++s) {
                    t[s].x += cr[s][i] * v.x - ci[s][i] * v.y;
                    t[s].y += cr[s][i] * v.y + ci[s][i] * v.x;
                    t[s].z += cr[s][i] * v.z - ci[s][i] * v.w;
                    t[s].w += cr[s][i] * v.w + ci[s][i] * v.z;
                }
            }
        }
#pragma unroll
        for (int s = 0; s < kPanel; ++s)
            if (s < nw) reinterpret_cast<float4*>(w + (size_t)s * w_stride)[e] = t[s];
    }
}

__global__ void k_reduce(const double* __restrict__ partials, int nval, int nblk, int nsys, double* out,
                         int out_stride) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nval * nsys) return;
    const int sys = k / nval, v = k - sys * nval;
    double t = 0;
    for (int b = 0; b < nblk; ++b) t += partials[(size_t)k * nblk + b];
    out[(size_t)sys * out_stride + v] = t;
}

__global__ void __launch_bounds__(kThreads) k_caxpy(const float2* __restrict__ basis, size_t vec_stride, int cnt,
                                                    const double2* __restrict__ coef, int coef_stride, float sign,
                                                    float2* w, size_t sys_stride, long long n) {
    const int sys = blockIdx.y;
    float cr[kDots], ci[kDots];
#pragma unroll
    for (int i = 0; i < kDots; ++i) {
        const double2 c = i < cnt ? coef[(size_t)sys * coef_stride + i] : make_double2(0.0, 0.0);
        cr[i] = sign * (float)c.x;
        ci[i] = sign * (float)c.y;
    }
    float4* w4 = reinterpret_cast<float4*>(w + (size_t)sys * sys_stride);
    const long long n4 = n / 2;
    for (long long e = (long long)blockIdx.x * kThreads + threadIdx.x; e < n4; e += (long long)gridDim.x * kThreads) {
        float4 t = w4[e];
#pragma unroll
        for (int i = 0; i < kDots; ++i) {
            if (i < cnt) {
                const float4 v = reinterpret_cast<const float4*>(basis + (size_t)i * vec_stride + (size_t)sys * sys_stride)[e];
                t.x += cr[i] * v.x - ci[i] * v.y;
                t.y += cr[i] * v.y + ci[i] * v.x;
                t.z += cr[i] * v.z - ci[i] * v.w;
                t.w += cr[i] * v.w + ci[i] * v.z;
            }
        }
        w4[e] = t;
    }
}

__global__ void __launch_bounds__(kThreads) k_cnorm2(const float2* __restrict__ w, size_t sys_stride, long long n,
                                                     double* partials) {
    __shared__ double lds[kThreads / 64];
    const int sys = blockIdx.y, nblk = gridDim.x;
    const float4* w4 = reinterpret_cast<const float4*>(w + (size_t)sys * sys_stride);
    double acc = 0;
    for (long long e = (long long)blockIdx.x * kThreads + threadIdx.x; e < n / 2; e += (long long)nblk * kThreads) {
        const float4 v = w4[e];
        acc += (double)(v.x * v.x + v.y * v.y + v.z * v.z + v.w * v.w);
    }
    acc = wave_sum_d(acc);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0;
        for (int q = 0; q < kThreads / 64; ++q) t += lds[q];
        partials[(size_t)sys * nblk + blockIdx.x] = t;
    }
}

__global__ void __launch_bounds__(kThreads) k_cscale(const float2* __restrict__ x, const double* __restrict__ f,
                                                     float2* y, size_t sys_stride, long long n) {
    const int sys = blockIdx.y;
    const float a = (float)f[sys];
    const float4* x4 = reinterpret_cast<const float4*>(x + (size_t)sys * sys_stride);
    float4* y4 = reinterpret_cast<float4*>(y + (size_t)sys * sys_stride);
    for (long long e = (long long)blockIdx.x * kThreads + threadIdx.x; e < n / 2; e += (long long)gridDim.x * kThreads) {
        const float4 v = x4[e];
        y4[e] = make_float4(a * v.x, a * v.y, a * v.z, a * v.w);
    }
}

__global__ void __launch_bounds__(kThreads) k_csub_from(const float2* __restrict__ x, float2* y, size_t sys_stride,
                                                        long long n) {
    const int sys = blockIdx.y;
    const float4* x4 = reinterpret_cast<const float4*>(x + (size_t)sys * sys_stride);
    float4* y4 = reinterpret_cast<float4*>(y + (size_t)sys * sys_stride);
    for (long long e = (long long)blockIdx.x * kThreads + threadIdx.x; e < n / 2; e += (long long)gridDim.x * kThreads) {
        const float4 a = x4[e], b = y4[e];
        y4[e] = make_float4(a.x - b.x, a.y - b.y, a.z - b.z, a.w - b.w);
    }
}

int agg_threads(const Geo& g) { return (g.Vb + 63) & ~63; }

}  // namespace

hipError_t launch_mg_term(const MgArgs& m, const void* links, const void* clover, int t, int b0, int nb, void* out,
                          size_t out_stride, hipStream_t st) {
    if (t < 0 || t > 8 || nb <= 0) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((m.g.V + kThreads - 1) / kThreads)), blk(kThreads);
    switch (t) {
        case 0: hipLaunchKernelGGL(k_mg_term<0>, grid, blk, 0, st, m, links, clover, b0, nb, out, out_stride); break;
        case 1: hipLaunchKernelGGL(k_mg_term<1>, grid, blk, 0, st, m, links, clover, b0, nb, out, out_stride); break;
        case 2: hipLaunchKernelGGL(k_mg_term<2>, grid, blk, 0, st, m, links, clover, b0, nb, out, out_stride); break;
        case 3: hipLaunchKernelGGL(k_mg_term<3>, grid, blk, 0, st, m, links, clover, b0, nb, out, out_stride); break;
        case 4: hipLaunchKernelGGL(k_mg_term<4>, grid, blk, 0, st, m, links, clover, b0, nb, out, out_stride); break;
        case 5: hipLaunchKernelGGL(k_mg_term<5>, grid, blk, 0, st, m, links, clover, b0, nb, out, out_stride); break;
        case 6: hipLaunchKernelGGL(k_mg_term<6>, grid, blk, 0, st, m, links, clover, b0, nb, out, out_stride); break;
        case 7: hipLaunchKernelGGL(k_mg_term<7>, grid, blk, 0, st, m, links, clover, b0, nb, out, out_stride); break;
        default: hipLaunchKernelGGL(k_mg_term<8>, grid, blk, 0, st, m, links, clover, b0, nb, out, out_stride); break;
    }
    return hipGetLastError();
}

// Aggregates of up to 256 sites take 4 systems per workgroup, larger ones 1 (register budget).
hipError_t launch_mg_restrict(const MgArgs& m, const void* x, size_t x_stride, int nsys, float2* out, size_t base,
                              size_t s_stride, size_t j_stride, hipStream_t st) {
    const int nt = agg_threads(m.g);
    if (nt > 1024 || m.nv < 1 || m.nv > kMgMaxVec || nsys < 1) return hipErrorInvalidValue;
    const int S = nt <= 256 ? 4 : 1;
    const int nch = (m.nv + 16 / S - 1) / (16 / S);
    const size_t lds = (size_t)(nt / 64) * nch * 64 * sizeof(float);
    const dim3 grid((unsigned)(m.g.V / m.g.Vb * ((nsys + S - 1) / S)));
    if (nt <= 256)
        hipLaunchKernelGGL((k_mg_restrict<4, 256>), grid, dim3(nt), lds, st, m, x, x_stride, nsys, out, base,
                           s_stride, j_stride);
    else
        hipLaunchKernelGGL((k_mg_restrict<1, 1024>), grid, dim3(nt), lds, st, m, x, x_stride, nsys, out, base,
                           s_stride, j_stride);
    return hipGetLastError();
}

hipError_t launch_mg_prolong(const MgArgs& m, const float2* c, int nsys, void* e, size_t e_stride, hipStream_t st) {
    const int nt = agg_threads(m.g);
    if (nt > 1024 || m.nv < 1 || m.nv > kMgMaxVec || nsys < 1) return hipErrorInvalidValue;
    const int S = nt <= 256 ? 4 : 2;
    const size_t lds = (size_t)S * 2 * m.nv * sizeof(float2);
    const dim3 grid((unsigned)(m.g.V / m.g.Vb * ((nsys + S - 1) / S)));
    if (nt <= 256)
        hipLaunchKernelGGL((k_mg_prolong<4, 256>), grid, dim3(nt), lds, st, m, c, nsys, e, e_stride);
    else
        hipLaunchKernelGGL((k_mg_prolong<2, 1024>), grid, dim3(nt), lds, st, m, c, nsys, e, e_stride);
    return hipGetLastError();
}

hipError_t launch_mg_block_orthonormalize(const MgArgs& m, void* P, hipStream_t st) {
    const int nt = agg_threads(m.g);
    if (nt > 1024) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_mg_block_orthonormalize, dim3((unsigned)(m.g.V / m.g.Vb), 2), dim3(nt), 0, st, m, P);
    return hipGetLastError();
}

hipError_t launch_mg_coarse_part(const Geo& g, int nv, const float2* Dc, const double* mu_c, const float2* x_self,
                                 const float2* x_hop, double hop_sign, const float2* add, int parity, bool zero_other,
                                 float2* y, int nsys, hipStream_t st) {
    if (nv < 1 || nv > kMgMaxVec || nsys < 1 || nsys > kMaxSys) return hipErrorInvalidValue;
    const int n2 = 2 * nv, ks = nsys < kCoarseSys ? nsys : kCoarseSys;
    const size_t xs = (size_t)9 * ks * n2, red = (size_t)(kThreads / nv) * ks * n2;
    const size_t lds = (xs > red ? xs : red) * sizeof(float2);  // at most 9 * 16 * 64 * 8 = 72 KiB
    if (lds > 65536) {
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_mg_coarse_apply),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    if (parity >= 0 && g.nb[3] % 2 != 0) return hipErrorInvalidValue;
    const long long nc = g.V / g.Vb;
    const dim3 grid((unsigned)(parity >= 0 ? nc / 2 : nc), (unsigned)((nsys + kCoarseSys - 1) / kCoarseSys));
    hipLaunchKernelGGL(k_mg_coarse_apply, grid, dim3(kThreads), lds, st, g, nv, Dc, mu_c, x_self, x_hop,
                       (float)hop_sign, add, parity, (int)zero_other, y, nsys);
    return hipGetLastError();
}

hipError_t launch_mg_coarse_apply(const Geo& g, int nv, const float2* Dc, const double* mu_c, const float2* x,
                                  float2* y, int nsys, hipStream_t st) {
    return launch_mg_coarse_part(g, nv, Dc, mu_c, x, x, 1.0, nullptr, -1, true, y, nsys, st);
}

hipError_t launch_mg_block_inverse(const Geo& g, int nv, const float2* Dc, double mu_c, int parity, float2* Minv,
                                   hipStream_t st) {
    if (nv < 1 || nv > kMgMaxVec || g.nb[3] % 2 != 0) return hipErrorInvalidValue;
    const size_t lds = (size_t)(2 * nv) * (4 * nv) * sizeof(double2);  // at most 128 KiB
    if (lds > 65536) {
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_mg_block_inverse),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_mg_block_inverse, dim3((unsigned)(g.V / g.Vb / 2)), dim3(kThreads), lds, st, g, nv, Dc,
                       mu_c, parity, Minv);
    return hipGetLastError();
}

hipError_t launch_mg_block_mul(const BlockMulArgs& a, hipStream_t st) {
    if (a.nv < 1 || a.nv > kMgMaxVec || a.nsys < 1 || a.nsys > kMaxSys || a.g.nb[3] % 2 != 0)
        return hipErrorInvalidValue;
    BlockMulArgs k = a;  // systems grouped by inverse set
    int pos = 0;
    for (int q = 0; q < kMgMaxInv; ++q) {
        k.start[q] = pos;
        for (int s = 0; s < a.nsys; ++s)
            if (a.sel[s] == q) {
                if (!a.sets[q]) return hipErrorInvalidValue;
                k.order[pos++] = (unsigned char)s;
            }
    }
    k.start[kMgMaxInv] = pos;
    if (pos != a.nsys) return hipErrorInvalidValue;  // a selector outside 0 .. kMgMaxInv - 1
    hipLaunchKernelGGL(k_mg_block_mul, dim3((unsigned)(a.g.V / a.g.Vb / 2)), dim3(64), 0, st, k);
    return hipGetLastError();
}

hipError_t launch_mg_stencil_export(long long nc, int nv, const float2* Dc, void* out, hipStream_t st) {
    hipLaunchKernelGGL(k_mg_stencil_export, dim3(1024), dim3(kThreads), 0, st, nc, nv, Dc, (double2*)out);
    return hipGetLastError();
}

hipError_t launch_mg_coarse_import(const void* canon, float2* v, long long n, unsigned* flag, hipStream_t st) {
    hipLaunchKernelGGL(k_mg_coarse_import, dim3(1024), dim3(kThreads), 0, st, (const double2*)canon, v, n, flag);
    return hipGetLastError();
}

hipError_t launch_mg_coarse_export(const float2* v, void* canon, long long n, hipStream_t st) {
    hipLaunchKernelGGL(k_mg_coarse_export, dim3(1024), dim3(kThreads), 0, st, v, (double2*)canon, n);
    return hipGetLastError();
}

int mg_blas_blocks(long long n) {
    const long long b = (n / 2 + kThreads - 1) / kThreads;
    return (int)(b < 1 ? 1 : (b > 512 ? 512 : b));
}

hipError_t mg_blas_dots(const float2* basis, size_t vec_stride, int cnt, const float2* w, size_t sys_stride, int nsys,
                        long long n, double* partials, double2* out, int out_stride, hipStream_t st) {
    if (cnt < 1 || cnt > kDots || (n & 1)) return hipErrorInvalidValue;
    const int nblk = mg_blas_blocks(n);
    hipLaunchKernelGGL(k_cdots, dim3(nblk, nsys), dim3(kThreads), 0, st, basis, vec_stride, cnt, w, sys_stride, n,
                       partials);
    const int tot = 2 * cnt * nsys;
    hipLaunchKernelGGL(k_reduce, dim3((tot + 63) / 64), dim3(64), 0, st, partials, 2 * cnt, nblk, nsys,
                       reinterpret_cast<double*>(out), 2 * out_stride);
    return hipGetLastError();
}

hipError_t mg_blas_axpy(const float2* basis, size_t vec_stride, int cnt, const double2* coef, int coef_stride,
                        double sign, float2* w, size_t sys_stride, int nsys, long long n, hipStream_t st) {
    if (cnt < 1 || cnt > kDots || (n & 1)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_caxpy, dim3(mg_blas_blocks(n), nsys), dim3(kThreads), 0, st, basis, vec_stride, cnt, coef,
                       coef_stride, (float)sign, w, sys_stride, n);
    return hipGetLastError();
}

hipError_t mg_blas_norm2(const float2* w, size_t sys_stride, int nsys, long long n, double* partials, double* out,
                         hipStream_t st) {
    if (n & 1) return hipErrorInvalidValue;
    const int nblk = mg_blas_blocks(n);
    hipLaunchKernelGGL(k_cnorm2, dim3(nblk, nsys), dim3(kThreads), 0, st, w, sys_stride, n, partials);
    hipLaunchKernelGGL(k_reduce, dim3((nsys + 63) / 64), dim3(64), 0, st, partials, 1, nblk, nsys, out, 1);
    return hipGetLastError();
}

hipError_t mg_blas_scale(const float2* x, const double* f, float2* y, size_t sys_stride, int nsys, long long n,
                         hipStream_t st) {
    if (n & 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_cscale, dim3(mg_blas_blocks(n), nsys), dim3(kThreads), 0, st, x, f, y, sys_stride, n);
    return hipGetLastError();
}

hipError_t mg_blas_panel_dots(const float2* basis, size_t vec_stride, int cnt, const float2* w, size_t w_stride, int nw,
                              long long n, double* partials, double2* out, int out_stride, hipStream_t st) {
    if (cnt < 1 || cnt > kPanelDots || nw < 1 || nw > kPanel || (n & 1)) return hipErrorInvalidValue;
    const int nblk = mg_blas_blocks(n);
    hipLaunchKernelGGL(k_pdots, dim3(nblk), dim3(kThreads), 0, st, basis, vec_stride, cnt, w, w_stride, nw, n, partials);
    const int tot = 2 * cnt * nw;
    hipLaunchKernelGGL(k_reduce, dim3((tot + 63) / 64), dim3(64), 0, st, partials, 2 * cnt, nblk, nw,
                       reinterpret_cast<double*>(out), 2 * out_stride);
    return hipGetLastError();
}

hipError_t mg_blas_panel_axpy(const float2* basis, size_t vec_stride, int cnt, const double2* coef, int coef_stride,
                              float2* w, size_t w_stride, int nw, long long n, hipStream_t st) {
    if (cnt < 1 || cnt > kPanelAxpy || nw < 1 || nw > kPanel || (n & 1)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_paxpy, dim3(mg_blas_blocks(n)), dim3(kThreads), 0, st, basis, vec_stride, cnt, coef,
                       coef_stride, w, w_stride, nw, n);
    return hipGetLastError();
}

hipError_t mg_blas_sub_from(const float2* x, float2* y, size_t sys_stride, int nsys, long long n, hipStream_t st) {
    if (n & 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_csub_from, dim3(mg_blas_blocks(n), nsys), dim3(kThreads), 0, st, x, y, sys_stride, n);
    return hipGetLastError();
}

}  // namespace tmsap
