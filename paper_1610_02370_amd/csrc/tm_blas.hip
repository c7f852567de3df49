// Vector kernels of the Krylov solvers on internal spinor fields: classical
// Gram-Schmidt with delayed reorthogonalisation (a dots sweep and an update
// sweep per Arnoldi step), norms, scaling, the solution update x += Z y,
// residual b - Dx and precision-changing accumulations.  Every
// inner product accumulates in FP64; per-workgroup partials are summed by a
// second kernel in a fixed order, so results do not depend on scheduling.
#include "tm_blas.h"

#include <type_traits>

namespace tmsap {

namespace {

constexpr int kThreads = 256;
constexpr int kMaxVec = 24;  // basis vectors handled by one pass

__device__ inline double wave_sum_d(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <class P>
__device__ inline void ld(const VecRef& r, int sys, long long V, long long s, Spinor<double>& out) {
    load_spinor<double, P>(static_cast<const char*>(r.data) + (size_t)sys * r.sys_stride,
                           r.scale ? r.scale + (size_t)sys * V : nullptr, V, s, out);
}

template <class P>
__device__ inline void st(const VecRef& r, int sys, long long V, long long s, const Spinor<double>& v) {
    store_spinor<double, P>(static_cast<char*>(r.data) + (size_t)sys * r.sys_stride,
                            r.scale ? r.scale + (size_t)sys * V : nullptr, V, s, v);
}

// Workgroup reduction of the first n of N values per thread into
// partials[(sys*n + i)*nblk + blockIdx.x] (compile-time N keeps vals in registers).
template <int N>
__device__ inline void reduce_out(double* vals, int n, double* lds, double* partials, int sys, int nblk) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const double v = wave_sum_d(i < n ? vals[i] : 0.0);
        if (lane == 0 && i < n) lds[w * 2 * kMaxVec + i] = v;
    }
    __syncthreads();
    if ((int)threadIdx.x < n) {
        double t = 0;
        for (int k = 0; k < kThreads / 64; ++k) t += lds[k * 2 * kMaxVec + threadIdx.x];
        partials[((size_t)sys * n + threadIdx.x) * nblk + blockIdx.x] = t;
    }
}

// out = ||x||^2 per system: values at the vectors' precision R (FP64 or FP32) per site, the sum
// over sites in FP64.
template <class P>
__global__ void __launch_bounds__(kThreads) k_norm2(VecRef x, double* partials, long long V) {
    typedef typename std::conditional<std::is_same<P, double>::value, double, float>::type R;
    __shared__ double lds[(kThreads / 64) * 2 * kMaxVec];
    const int sys = blockIdx.y;
    const char* x0 = static_cast<const char*>(x.data) + (size_t)sys * x.sys_stride;
    double acc[1] = {0};
    for (long long s = (long long)blockIdx.x * kThreads + threadIdx.x; s < V; s += (long long)gridDim.x * kThreads) {
        Spinor<R> v;
        load_spinor<R, P>(x0, nullptr, V, s, v);
        R n2 = 0;
#pragma unroll
        for (int k = 0; k < 12; ++k) n2 += v.v[k].re * v.v[k].re + v.v[k].im * v.v[k].im;
        acc[0] += (double)n2;
    }
    reduce_out<1>(acc, 1, lds, partials, sys, gridDim.x);
}

// Classical Gram-Schmidt with delayed reorthogonalisation: two sweeps over the
// stored vectors per Arnoldi step.  The slots hold u_0..u_j: u_0 = v_0, and each
// later u_i the direction of step i - 1 projected once against v_0..v_{i-1} and
// scaled to about unit norm.  The orthonormal basis is never stored: u_i =
// sum_{k<i} T_ki v_k + T_ii v_i with T upper triangular (T_ii = beta_i), so
// V = U T^-1, and T (per system, a few hundred numbers) carries every product
// with V.  w = D z_j.
//
// Dots sweep over stored vectors [i0, i0 + n): per system 4 n values
// (<u_i, u>, <u_i, w>) as complex pairs, and with `head` 4 more: <u, u>,
// <u, w> (complex), <w, w>, for u = u_j.
template <class P, int NV>
__global__ void __launch_bounds__(kThreads) k_dgs_dots(VecRef basis, size_t vec_stride, int i0, int n, VecRef u,
                                                       VecRef w, int head, double* partials, long long V) {
    typedef typename std::conditional<std::is_same<P, double>::value, double, float>::type R;
    __shared__ double lds[(kThreads / 64) * 2 * kMaxVec];
    const int sys = blockIdx.y;
    const int nblk = gridDim.x;
    double acc[4 * NV + 4];
#pragma unroll
    for (int i = 0; i < 4 * NV + 4; ++i) acc[i] = 0;
    const char* b0 = static_cast<const char*>(basis.data) + (size_t)sys * basis.sys_stride + (size_t)i0 * vec_stride;
    const char* u0 = static_cast<const char*>(u.data) + (size_t)sys * u.sys_stride;
    const char* w0 = static_cast<const char*>(w.data) + (size_t)sys * w.sys_stride;
    for (long long s = (long long)blockIdx.x * kThreads + threadIdx.x; s < V; s += (long long)nblk * kThreads) {
        Spinor<R> uv, wv;
        load_spinor<R, P>(u0, nullptr, V, s, uv);
        load_spinor<R, P>(w0, nullptr, V, s, wv);
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            if (i < n) {
                Spinor<R> v;
                load_spinor<R, P>(b0 + i * vec_stride, nullptr, V, s, v);
                R cr = 0, ci = 0, ar = 0, ai = 0;
#pragma unroll
                for (int k = 0; k < 12; ++k) {
                    cr += v.v[k].re * uv.v[k].re + v.v[k].im * uv.v[k].im;
                    ci += v.v[k].re * uv.v[k].im - v.v[k].im * uv.v[k].re;
                    ar += v.v[k].re * wv.v[k].re + v.v[k].im * wv.v[k].im;
                    ai += v.v[k].re * wv.v[k].im - v.v[k].im * wv.v[k].re;
                }
                acc[4 * i] += (double)cr;
                acc[4 * i + 1] += (double)ci;
                acc[4 * i + 2] += (double)ar;
                acc[4 * i + 3] += (double)ai;
            }
        }
        if (head) {
            R uu = 0, uwr = 0, uwi = 0, ww = 0;
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                uu += uv.v[k].re * uv.v[k].re + uv.v[k].im * uv.v[k].im;
                uwr += uv.v[k].re * wv.v[k].re + uv.v[k].im * wv.v[k].im;
                uwi += uv.v[k].re * wv.v[k].im - uv.v[k].im * wv.v[k].re;
                ww += wv.v[k].re * wv.v[k].re + wv.v[k].im * wv.v[k].im;
            }
            acc[4 * NV] += (double)uu;
            acc[4 * NV + 1] += (double)uwr;
            acc[4 * NV + 2] += (double)uwi;
            acc[4 * NV + 3] += (double)ww;
        }
    }
    // the head values follow the n dot pairs
#pragma unroll
    for (int i = 0; i < 4 * NV; ++i)
#pragma unroll
        for (int t = 0; t < 4; ++t)
            if (head && i == 4 * n + t) acc[i] = acc[4 * NV + t];
    reduce_out<4 * NV + 4>(acc, 4 * n + (head ? 4 : 0), lds, partials, sys, nblk);
}

// Coefficients of the update sweep, one thread per system, from the dots d (4 nb + 4 values
// per system) and the triangular factor t of the system (column-major from the earlier
// steps, kTri x kTri complex; column nb is written here).  In the basis V:
//   c = V^H u_j = T^-H (U^H u_j),  a = V^H w = T^-H (U^H w)      (forward substitution)
//   beta = sqrt(<u, u> - |c|^2)   (u_j is already orthogonal to V up to rounding, so this
//                                   has no cancellation); v_j = (u_j - V c) / beta
//   h = <v_j, w> = (<u, w> - c^H a) / beta,  e = h / beta
//   w' = w - V a - h v_j = w - e u_j - V (a - c e) = w - e u_j - U g,  T g = a - c e
//                                                                     (back substitution)
//   s = 1 / sqrt(<w, w> - |a|^2 - |h|^2), the norm of w' by Pythagoras, floored at
//       1e-6 <w, w> (only the scale of the next direction s w'; its exact norm is returned by
//       the update sweep)
// At the first step of a cycle (nb == 0) u_0 is v_0 itself: beta = 1.
// coef per system (4 + 2 nb): [s, s e (complex), 0, (s g_i) complex]; rep per system
// (4 + 4 kTri): [beta, h (complex), s, then (c_i, a_i) complex pairs].  Frozen systems (bit set
// in `off`) and a vanishing beta (u_j in the span of the basis: the previous column ends the
// Krylov space) get zero coefficients and beta 0.
constexpr int kTri = kMaxVec;

__global__ void k_dgs_coef(const double* d, int nb, int nsys, unsigned long long off, double* coef, double* rep,
                           double* tri) {
    const int k = threadIdx.x;
    if (k >= nsys) return;
    const int ds = 4 * nb + 4, cstride = 4 + 2 * nb, rstride = 4 + 4 * kTri;
    const double* dk = d + (size_t)k * ds;
    double* ck = coef + (size_t)k * cstride;
    double* rk = rep + (size_t)k * rstride;
    double* tk = tri + (size_t)k * kTri * kTri * 2;  // T[i][j] at tk[(j * kTri + i) * 2]
    for (int i = 0; i < cstride; ++i) ck[i] = 0.0;
    for (int i = 0; i < 4 + 4 * nb; ++i) rk[i] = 0.0;
    if ((off >> k) & 1ull) return;
    double cr[kTri], ci[kTri], ar[kTri], ai[kTri];
    // forward substitution with T^H (lower triangular, real diagonal)
    for (int i = 0; i < nb; ++i) {
        double xr = dk[4 * i], xi = dk[4 * i + 1], yr = dk[4 * i + 2], yi = dk[4 * i + 3];
        for (int q = 0; q < i; ++q) {
            const double tr = tk[(i * kTri + q) * 2], ti = tk[(i * kTri + q) * 2 + 1];  // T[q][i]
            // conj(T[q][i]) * c_q
            xr -= tr * cr[q] + ti * ci[q];
            xi -= tr * ci[q] - ti * cr[q];
            yr -= tr * ar[q] + ti * ai[q];
            yi -= tr * ai[q] - ti * ar[q];
        }
        const double tii = tk[(i * kTri + i) * 2];
        cr[i] = xr / tii;
        ci[i] = xi / tii;
        ar[i] = yr / tii;
        ai[i] = yi / tii;
    }
    const double uu = dk[4 * nb], uwr = dk[4 * nb + 1], uwi = dk[4 * nb + 2], ww = dk[4 * nb + 3];
    double beta = 1.0, hr = uwr, hi = uwi;
    if (nb > 0) {
        double t = uu;
        for (int i = 0; i < nb; ++i) t -= cr[i] * cr[i] + ci[i] * ci[i];
        if (!(uu > 0) || !(t > 1e-28 * uu)) return;
        beta = sqrt(t);
        for (int i = 0; i < nb; ++i) {
            hr -= cr[i] * ar[i] + ci[i] * ai[i];
            hi -= cr[i] * ai[i] - ci[i] * ar[i];
        }
        hr /= beta;
        hi /= beta;
    }
    // column nb of T
    for (int i = 0; i < nb; ++i) {
        tk[(nb * kTri + i) * 2] = cr[i];
        tk[(nb * kTri + i) * 2 + 1] = ci[i];
    }
    tk[(nb * kTri + nb) * 2] = beta;
    tk[(nb * kTri + nb) * 2 + 1] = 0.0;
    const double er = hr / beta, ei = hi / beta;
    double est = ww - hr * hr - hi * hi;
    for (int i = 0; i < nb; ++i) est -= ar[i] * ar[i] + ai[i] * ai[i];
    const double s = ww > 0 ? 1.0 / sqrt(fmax(est, 1e-6 * ww)) : 0.0;
    // back substitution T g = a - c e, in place over (ar, ai)
    for (int i = nb - 1; i >= 0; --i) {
        double gr = ar[i] - (cr[i] * er - ci[i] * ei), gi = ai[i] - (cr[i] * ei + ci[i] * er);
        for (int q = i + 1; q < nb; ++q) {
            const double tr = tk[(q * kTri + i) * 2], ti = tk[(q * kTri + i) * 2 + 1];  // T[i][q]
            gr -= tr * ar[q] - ti * ai[q];
            gi -= tr * ai[q] + ti * ar[q];
        }
        const double tii = tk[(i * kTri + i) * 2];
        // keep a_i for the report before it is overwritten by g_i
        rk[4 + 4 * i + 2] = ar[i];
        rk[4 + 4 * i + 3] = ai[i];
        ar[i] = gr / tii;
        ai[i] = gi / tii;
    }
    ck[0] = s;
    ck[1] = s * er;
    ck[2] = s * ei;
    for (int i = 0; i < nb; ++i) {
        ck[4 + 2 * i] = s * ar[i];
        ck[4 + 2 * i + 1] = s * ai[i];
        rk[4 + 4 * i] = cr[i];
        rk[4 + 4 * i + 1] = ci[i];
    }
    rk[0] = beta;
    rk[1] = hr;
    rk[2] = hi;
    rk[3] = s;
}

// Update sweep with the coefficients of k_dgs_coef (per system at coef + sys * (4 + 2 nb)):
//   y = s w - (s e) u_j - sum_i (s g_i) u_i   written to y; out = ||y||^2 of the stored values
template <class P, int NV>
__global__ void __launch_bounds__(kThreads) k_dgs_update(VecRef basis, size_t vec_stride, int nb, VecRef u,
                                                         VecRef w, VecRef y, const double* __restrict__ coef,
                                                         double* partials, long long V) {
    typedef typename std::conditional<std::is_same<P, double>::value, double, float>::type R;
    __shared__ double lds[(kThreads / 64) * 2 * kMaxVec];
    const int sys = blockIdx.y;
    const int nblk = gridDim.x;
    const double* cf = coef + (size_t)sys * (4 + 2 * nb);
    const R sw = (R)cf[0];
    const cplx<R> ew = cmk((R)cf[1], (R)cf[2]);
    const char* b0 = static_cast<const char*>(basis.data) + (size_t)sys * basis.sys_stride;
    const char* u0 = static_cast<const char*>(u.data) + (size_t)sys * u.sys_stride;
    const char* w0 = static_cast<const char*>(w.data) + (size_t)sys * w.sys_stride;
    char* y0 = static_cast<char*>(y.data) + (size_t)sys * y.sys_stride;
    double acc[1] = {0};
    for (long long s = (long long)blockIdx.x * kThreads + threadIdx.x; s < V; s += (long long)nblk * kThreads) {
        Spinor<R> uv, yv;
        load_spinor<R, P>(u0, nullptr, V, s, uv);
        load_spinor<R, P>(w0, nullptr, V, s, yv);
#pragma unroll
        for (int k = 0; k < 12; ++k) yv.v[k] = sw * yv.v[k] - ew * uv.v[k];
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            if (i < nb) {
                Spinor<R> v;
                load_spinor<R, P>(b0 + i * vec_stride, nullptr, V, s, v);
                const cplx<R> qw = cmk((R)cf[4 + 2 * i], (R)cf[4 + 2 * i + 1]);
#pragma unroll
                for (int k = 0; k < 12; ++k) yv.v[k] = yv.v[k] - qw * v.v[k];
            }
        }
        store_spinor<R, P>(y0, nullptr, V, s, yv);
        R n2 = 0;
#pragma unroll
        for (int k = 0; k < 12; ++k) n2 += yv.v[k].re * yv.v[k].re + yv.v[k].im * yv.v[k].im;
        acc[0] += (double)n2;
    }
    reduce_out<1>(acc, 1, lds, partials, sys, nblk);
}

// out[sys*stride + off + i] = sum over blocks of value sys*n + i (fixed order).
__global__ void k_reduce_strided(const double* partials, int nblk, int n, int stride, int off, double* out) {
    __shared__ double lds[kThreads];
    const int v = blockIdx.x;
    double t = 0;
    for (int b = threadIdx.x; b < nblk; b += kThreads) t += partials[(size_t)v * nblk + b];
    lds[threadIdx.x] = t;
    __syncthreads();
    for (int o = kThreads / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) lds[threadIdx.x] += lds[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[(size_t)(v / n) * stride + off + v % n] = lds[0];
}

// out[sys*n + i] = sum over blocks (fixed order), optionally added to out.
__global__ void k_reduce(const double* partials, int nblk, int nval_total, double* out, int accumulate) {
    __shared__ double lds[kThreads];
    const int v = blockIdx.x;
    if (v >= nval_total) return;
    double t = 0;
    for (int b = threadIdx.x; b < nblk; b += kThreads) t += partials[(size_t)v * nblk + b];
    lds[threadIdx.x] = t;
    __syncthreads();
    for (int off = kThreads / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) lds[threadIdx.x] += lds[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[v] = accumulate ? out[v] + lds[0] : lds[0];
}

// y = a[sys] * x  (a real, per system, read from device memory)
template <class Pi, class Po>
__global__ void __launch_bounds__(kThreads) k_scale(VecRef x, const double* a, VecRef y, long long V) {
    const int sys = blockIdx.y;
    const double f = a[sys];
    for (long long s = (long long)blockIdx.x * kThreads + threadIdx.x; s < V; s += (long long)gridDim.x * kThreads) {
        Spinor<double> v;
        ld<Pi>(x, sys, V, s, v);
#pragma unroll
        for (int k = 0; k < 12; ++k) v.v[k] = f * v.v[k];
        st<Po>(y, sys, V, s, v);
    }
}

// x += sum_i y_i z_i (x = sum_i y_i z_i with `overwrite`: x is not read), y complex per
// (sys, i) from device memory
template <class Px, class Pz>
__global__ void __launch_bounds__(kThreads) k_xupdate(VecRef x, VecRef z, size_t zvec_stride, size_t zscale_stride,
                                                      int nvec, const double* y, int overwrite, long long V) {
    const int sys = blockIdx.y;
    for (long long s = (long long)blockIdx.x * kThreads + threadIdx.x; s < V; s += (long long)gridDim.x * kThreads) {
        Spinor<double> xv;
        if (overwrite) {
#pragma unroll
            for (int k = 0; k < 12; ++k) xv.v[k] = cmk(0.0, 0.0);
        } else {
            ld<Px>(x, sys, V, s, xv);
        }
        for (int i = 0; i < nvec; ++i) {
            VecRef zi = z;
            zi.data = static_cast<char*>(z.data) + i * zvec_stride;
            zi.scale = z.scale ? z.scale + i * zscale_stride : nullptr;
            Spinor<double> zv;
            ld<Pz>(zi, sys, V, s, zv);
            const cplx<double> c = cmk(y[((size_t)sys * nvec + i) * 2], y[((size_t)sys * nvec + i) * 2 + 1]);
#pragma unroll
            for (int k = 0; k < 12; ++k) xv.v[k] = cmad(c, zv.v[k], xv.v[k]);
        }
        st<Px>(x, sys, V, s, xv);
    }
}

// r = b - ax (r may alias ax when Pr is P), computed in FP64 and stored at Pr; partial ||r||^2
// and ||b||^2 of the FP64 values (2 values per system)
template <class P, class Pr = P>
__global__ void __launch_bounds__(kThreads) k_residual(VecRef b, VecRef ax, VecRef r, double* partials, long long V) {
    __shared__ double lds[(kThreads / 64) * 2 * kMaxVec];
    const int sys = blockIdx.y;
    double acc[2] = {0, 0};
    for (long long s = (long long)blockIdx.x * kThreads + threadIdx.x; s < V; s += (long long)gridDim.x * kThreads) {
        Spinor<double> bv, av;
        ld<P>(b, sys, V, s, bv);
        ld<P>(ax, sys, V, s, av);
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            av.v[k] = bv.v[k] - av.v[k];
            acc[0] += av.v[k].re * av.v[k].re + av.v[k].im * av.v[k].im;
            acc[1] += bv.v[k].re * bv.v[k].re + bv.v[k].im * bv.v[k].im;
        }
        st<Pr>(r, sys, V, s, av);
    }
    reduce_out<2>(acc, 2, lds, partials, sys, gridDim.x);
}

// x (Px) += c (Pc)
template <class Px, class Pc>
__global__ void __launch_bounds__(kThreads) k_accumulate(VecRef x, VecRef c, long long V) {
    const int sys = blockIdx.y;
    for (long long s = (long long)blockIdx.x * kThreads + threadIdx.x; s < V; s += (long long)gridDim.x * kThreads) {
        Spinor<double> xv, cv;
        ld<Px>(x, sys, V, s, xv);
        ld<Pc>(c, sys, V, s, cv);
#pragma unroll
        for (int k = 0; k < 12; ++k) xv.v[k] = xv.v[k] + cv.v[k];
        st<Px>(x, sys, V, s, xv);
    }
}

__global__ void k_zero(void* p, size_t n16) {
    for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < n16; i += (size_t)gridDim.x * kThreads)
        reinterpret_cast<float4*>(p)[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

// Test pattern in [-1, 1) from a 32-bit integer hash of the index (timing
// inputs only: values need be finite and of unit size, not random).
__device__ inline float pattern_value(size_t i, unsigned seed) {
    unsigned h = (unsigned)i * 0x9E3779B1u ^ (unsigned)(i >> 32) ^ seed;
    h ^= h >> 16;
    h *= 0x85EBCA6Bu;
    h ^= h >> 13;
    h *= 0xC2B2AE35u;
    h ^= h >> 16;
    return (float)(h >> 8) * (2.0f / 16777216.0f) - 1.0f;
}

template <class T>
__global__ void k_fill_pattern(T* data, size_t n, float* scale, size_t nscale, unsigned seed) {
    const size_t stride = (size_t)gridDim.x * kThreads;
    for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += stride) {
        const float v = pattern_value(i, seed);
        if constexpr (std::is_same<T, bf16>::value)
            data[i] = to_bf16(v);
        else
            data[i] = (T)v;
    }
    for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < nscale; i += stride) scale[i] = 1.0f;
}

}  // namespace

int blas_blocks(long long V) {
    long long n = (V + kThreads - 1) / kThreads;
    return (int)(n < 1024 ? n : 1024);
}

int blas_max_vec() { return kMaxVec; }

#define TM_DISPATCH_VEC(P, T, ...)                           \
    switch (P) {                                             \
        case P_F64: { typedef double T; __VA_ARGS__; break; } \
        case P_F32: { typedef float T; __VA_ARGS__; break; }  \
        case P_F16: { typedef f16 T; __VA_ARGS__; break; }    \
        default: { typedef bf16 T; __VA_ARGS__; break; }      \
    }

hipError_t blas_norm2(Prec p, const VecRef& x, double* partials, double* out, int nsys, long long V,
                      hipStream_t st) {
    if (p != P_F64 && p != P_F32) return hipErrorInvalidValue;
    const int nblk = blas_blocks(V);
    dim3 grid(nblk, nsys);
    if (p == P_F32)
        hipLaunchKernelGGL(k_norm2<float>, grid, dim3(kThreads), 0, st, x, partials, V);
    else
        hipLaunchKernelGGL(k_norm2<double>, grid, dim3(kThreads), 0, st, x, partials, V);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_reduce, dim3(nsys), dim3(kThreads), 0, st, partials, nblk, nsys, out, 0);
    return hipGetLastError();
}

hipError_t blas_dgs_dots(Prec p, const VecRef& basis, size_t vec_stride, int nb, const VecRef& u, const VecRef& w,
                        double* partials, double* out, int nsys, long long V, hipStream_t st) {
    if (nb < 0 || nb > kMaxVec - 1 || (p != P_F64 && p != P_F32)) return hipErrorInvalidValue;
    const int nblk = blas_blocks(V);
    const int chunk = p == P_F32 ? 8 : 4;  // FP64 spinors take twice the registers
    const int ds = 4 * nb + 4;
    dim3 grid(nblk, nsys);
    for (int i0 = 0;; i0 += chunk) {
        const int n = nb - i0 < chunk ? nb - i0 : chunk;
        const int head = i0 + n == nb;
        if (p == P_F32)
            hipLaunchKernelGGL((k_dgs_dots<float, 8>), grid, dim3(kThreads), 0, st, basis, vec_stride, i0, n, u, w,
                               head, partials, V);
        else
            hipLaunchKernelGGL((k_dgs_dots<double, 4>), grid, dim3(kThreads), 0, st, basis, vec_stride, i0, n, u, w,
                               head, partials, V);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        const int nv = 4 * n + (head ? 4 : 0);
        hipLaunchKernelGGL(k_reduce_strided, dim3(nsys * nv), dim3(kThreads), 0, st, partials, nblk, nv, ds, 4 * i0,
                           out);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if (head) break;
    }
    return hipSuccess;
}

hipError_t blas_dgs_coef(const double* d, int nb, int nsys, unsigned long long off, double* coef, double* rep,
                         double* tri, hipStream_t st) {
    if (nb < 0 || nb > kTri - 1 || nsys > 64) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_dgs_coef, dim3(1), dim3(64), 0, st, d, nb, nsys, off, coef, rep, tri);
    return hipGetLastError();
}

int blas_dgs_tri_stride() { return kTri; }

hipError_t blas_dgs_update(Prec p, const VecRef& basis, size_t vec_stride, int nb, const VecRef& u, const VecRef& w,
                           const VecRef& y, const double* coef, double* partials, double* out, int nsys, long long V,
                           hipStream_t st) {
    if (nb < 0 || nb > kMaxVec - 1 || (p != P_F64 && p != P_F32)) return hipErrorInvalidValue;
    const int nblk = blas_blocks(V);
    dim3 grid(nblk, nsys);
#define TM_DGS_LAUNCH(NVT)                                                                                     \
    if (p == P_F32)                                                                                            \
        hipLaunchKernelGGL((k_dgs_update<float, NVT>), grid, dim3(kThreads), 0, st, basis, vec_stride, nb, u, \
                           w, y, coef, partials, V);                                                           \
    else                                                                                                       \
        hipLaunchKernelGGL((k_dgs_update<double, NVT>), grid, dim3(kThreads), 0, st, basis, vec_stride, nb, u, \
                           w, y, coef, partials, V)
    if (nb <= 4) {
        TM_DGS_LAUNCH(4);
    } else if (nb <= 8) {
        TM_DGS_LAUNCH(8);
    } else if (nb <= 16) {
        TM_DGS_LAUNCH(16);
    } else {
        TM_DGS_LAUNCH(kMaxVec - 1);
    }
#undef TM_DGS_LAUNCH
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_reduce, dim3(nsys), dim3(kThreads), 0, st, partials, nblk, nsys, out, 0);
    return hipGetLastError();
}

hipError_t blas_scale(Prec pi, Prec po, const VecRef& x, const double* a, const VecRef& y, int nsys, long long V,
                      hipStream_t st) {
    dim3 grid(blas_blocks(V), nsys);
    TM_DISPATCH_VEC(pi, Ti, TM_DISPATCH_VEC(po, To, hipLaunchKernelGGL((k_scale<Ti, To>), grid, dim3(kThreads), 0, st,
                                                                        x, a, y, V)));
    return hipGetLastError();
}

hipError_t blas_xupdate(Prec px, Prec pz, const VecRef& x, const VecRef& z, size_t zvec_stride, size_t zscale_stride,
                        int nvec, const double* y, int overwrite, int nsys, long long V, hipStream_t st) {
    dim3 grid(blas_blocks(V), nsys);
    TM_DISPATCH_VEC(px, Tx, TM_DISPATCH_VEC(pz, Tz, hipLaunchKernelGGL((k_xupdate<Tx, Tz>), grid, dim3(kThreads), 0,
                                                                        st, x, z, zvec_stride, zscale_stride, nvec, y,
                                                                        overwrite, V)));
    return hipGetLastError();
}

hipError_t blas_residual(Prec p, const VecRef& b, const VecRef& ax, const VecRef& r, double* partials, double* out,
                         int nsys, long long V, hipStream_t st, Prec pr) {
    const int nblk = blas_blocks(V);
    dim3 grid(nblk, nsys);
    if (pr == p) {
        TM_DISPATCH_VEC(p, T, hipLaunchKernelGGL(k_residual<T>, grid, dim3(kThreads), 0, st, b, ax, r, partials, V));
    } else if (p == P_F64 && pr == P_F32) {
        hipLaunchKernelGGL((k_residual<double, float>), grid, dim3(kThreads), 0, st, b, ax, r, partials, V);
    } else {
        return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_reduce, dim3(2 * nsys), dim3(kThreads), 0, st, partials, nblk, 2 * nsys, out, 0);
    return hipGetLastError();
}

hipError_t blas_accumulate(Prec px, Prec pc, const VecRef& x, const VecRef& c, int nsys, long long V, hipStream_t st) {
    dim3 grid(blas_blocks(V), nsys);
    TM_DISPATCH_VEC(px, Tx, TM_DISPATCH_VEC(pc, Tc, hipLaunchKernelGGL((k_accumulate<Tx, Tc>), grid, dim3(kThreads),
                                                                        0, st, x, c, V)));
    return hipGetLastError();
}

hipError_t blas_zero(void* p, size_t bytes, hipStream_t st) {
    const size_t n16 = bytes / 16;
    const unsigned nb = (unsigned)((n16 + kThreads - 1) / kThreads < 4096 ? (n16 + kThreads - 1) / kThreads : 4096);
    hipLaunchKernelGGL(k_zero, dim3(nb > 0 ? nb : 1), dim3(kThreads), 0, st, p, n16);
    return hipGetLastError();
}

hipError_t blas_fill_pattern(const SpinorBuf& b, long long V, unsigned seed, hipStream_t st) {
    const size_t nreal = spinor_data_bytes(V, b.nsys, b.prec) / (unit_bytes(b.prec) / 4);
    const size_t nscale = b.scale ? (size_t)b.nsys * V : 0;
    const unsigned nb = 4096;
    TM_DISPATCH_VEC(b.prec, T,
                    hipLaunchKernelGGL(k_fill_pattern<T>, dim3(nb), dim3(kThreads), 0, st, static_cast<T*>(b.data),
                                       nreal, b.scale, nscale, seed));
    return hipGetLastError();
}

}  // namespace tmsap
