// Vector kernels used by the Krylov solvers (tm_blas.hip).
#pragma once

#include "tm_internal.h"

namespace tmsap {

// One internal field of nsys systems: data [nsys][6 units][V], FP16 scales [nsys][V].
struct VecRef {
    void* data = nullptr;
    float* scale = nullptr;
    size_t sys_stride = 0;  // bytes between systems
};

inline VecRef vec_ref(const SpinorBuf& b, long long V) {
    VecRef r;
    r.data = b.data;
    r.scale = b.scale;
    r.sys_stride = (size_t)6 * V * unit_bytes(b.prec);
    return r;
}

int blas_blocks(long long V);
int blas_max_vec();

// out[sys] = ||x_sys||^2 (FP64 or FP32 fields, no scales; the sum over sites in FP64)
hipError_t blas_norm2(Prec p, const VecRef& x, double* partials, double* out, int nsys, long long V,
                      hipStream_t st);
// Classical Gram-Schmidt with delayed reorthogonalisation, two sweeps over the stored vectors per
// Arnoldi step.  The stored vectors u_0..u_{nb-1} (at basis.data + i*vec_stride, FP64 or FP32, no
// scales) are the once-projected directions; the orthonormal basis is V = U T^-1 with T upper
// triangular, kept per system in `tri` by the coefficient kernel.  u is the newest direction
// u_nb, w the new operator output.
// Dots: out[sys*(4 nb + 4) + ...] = (<u_i, u>, <u_i, w>)_i as complex pairs, then <u, u>, <u, w>
// (complex), <w, w>.
hipError_t blas_dgs_dots(Prec p, const VecRef& basis, size_t vec_stride, int nb, const VecRef& u, const VecRef& w,
                         double* partials, double* out, int nsys, long long V, hipStream_t st);
// Coefficients of the update from those dots: coef (4 + 2 nb values per system), rep per system
// (stride 4 + 4 blas_dgs_tri_stride()): beta = ||u - V V^H u||, h = <v_nb, w> for v_nb = (u - V
// V^H u) / beta, s the scale of the next direction, then c = V^H u and a = V^H w as complex
// pairs; writes column nb of T (tri: per system blas_dgs_tri_stride()^2 complex, column-major).
// nb = 0 means u is v_0 itself (T_00 = 1).  Systems with bit k of `off` set get zero
// coefficients; beta = 0 flags u in the span of the basis.  nsys <= 64.
hipError_t blas_dgs_coef(const double* d, int nb, int nsys, unsigned long long off, double* coef, double* rep,
                         double* tri, hipStream_t st);
int blas_dgs_tri_stride();
// Update: y <- s (w - V a - h v_nb), formed from u, w and the stored vectors; out[sys] = ||y||^2 of
// the stored values.
hipError_t blas_dgs_update(Prec p, const VecRef& basis, size_t vec_stride, int nb, const VecRef& u, const VecRef& w,
                           const VecRef& y, const double* coef, double* partials, double* out, int nsys, long long V,
                           hipStream_t st);
// y = a[sys] x
hipError_t blas_scale(Prec pi, Prec po, const VecRef& x, const double* a, const VecRef& y, int nsys, long long V,
                      hipStream_t st);
// x += sum_i y[sys][i] z_i  (z_i at z.data + i*zvec_stride, scales at z.scale + i*zscale_stride);
// with overwrite != 0, x = sum_i y[sys][i] z_i and x is not read
hipError_t blas_xupdate(Prec px, Prec pz, const VecRef& x, const VecRef& z, size_t zvec_stride, size_t zscale_stride,
                        int nvec, const double* y, int overwrite, int nsys, long long V, hipStream_t st);
// r = b - ax (b, ax at p; r at pr, which is p or, from FP64, FP32: the FP64 difference rounded
// once), out[sys] = (||r||^2, ||b||^2) of the FP64 values
hipError_t blas_residual(Prec p, const VecRef& b, const VecRef& ax, const VecRef& r, double* partials, double* out,
                         int nsys, long long V, hipStream_t st, Prec pr);
// x += c
hipError_t blas_accumulate(Prec px, Prec pc, const VecRef& x, const VecRef& c, int nsys, long long V, hipStream_t st);
// zero a buffer with a kernel (bytes a multiple of 16)
hipError_t blas_zero(void* p, size_t bytes, hipStream_t st);
// fill an internal field with a fixed bounded pattern (FP16 scales set to 1); tuning inputs
hipError_t blas_fill_pattern(const SpinorBuf& b, long long V, unsigned seed, hipStream_t st);

}  // namespace tmsap
