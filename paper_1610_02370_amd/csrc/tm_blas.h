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

// Gram-Schmidt passes over basis vectors 0..nvec-1 (vector i at basis.data + i*vec_stride, FP64 or FP32, no
// scales; nvec < kMaxVec); coefficients per system at coef + sys*coef_stride as (re, im) pairs:
//   mode 0: out[sys] = (<v_i, w>)_i                                   (2 nvec values)
//   mode 1: w -= sum_i coef_i v_i, then out[sys] = (<v_i, w>)_i, ||w||^2  (2 nvec + 1 values)
//   mode 2: w -= sum_i coef_i v_i, then out[sys] = ||w||^2
//   mode 3: t = w - sum_i coef_i v_i; y = fac[sys] t (w unchanged); out[sys] = ||t||^2
// Values per system are contiguous in out; accumulate != 0 adds to out.
hipError_t blas_gs(Prec p, const VecRef& basis, size_t vec_stride, int nvec, const VecRef& w, const double* coef,
                   int coef_stride, int mode, const VecRef& y, const double* fac, double* partials, double* out,
                   int accumulate, int nsys, long long V, hipStream_t st);
// s[k] = 1/sqrt(hn_k[2 nvec] - sum_i hn_k[i]^2) for the mode-1 output hn (2 nvec + 1 values per system):
// the norm after the second projection by Pythagoras; 0 for bit k of `off` set or a vanishing norm.
hipError_t blas_pythagoras(const double* hn, int nvec, int nsys, unsigned long long off, double* s, hipStream_t st);
// y = a[sys] x
hipError_t blas_scale(Prec pi, Prec po, const VecRef& x, const double* a, const VecRef& y, int nsys, long long V,
                      hipStream_t st);
// x += sum_i y[sys][i] z_i  (z_i at z.data + i*zvec_stride, scales at z.scale + i*zscale_stride)
hipError_t blas_xupdate(Prec px, Prec pz, const VecRef& x, const VecRef& z, size_t zvec_stride, size_t zscale_stride,
                        int nvec, const double* y, int nsys, long long V, hipStream_t st);
// r = b - ax, out[sys] = (||r||^2, ||b||^2)
hipError_t blas_residual(Prec p, const VecRef& b, const VecRef& ax, const VecRef& r, double* partials, double* out,
                         int nsys, long long V, hipStream_t st);
// x += c
hipError_t blas_accumulate(Prec px, Prec pc, const VecRef& x, const VecRef& c, int nsys, long long V, hipStream_t st);
// zero a buffer with a kernel (bytes a multiple of 16)
hipError_t blas_zero(void* p, size_t bytes, hipStream_t st);
// fill an internal field with a fixed bounded pattern (FP16 scales set to 1); tuning inputs
hipError_t blas_fill_pattern(const SpinorBuf& b, long long V, unsigned seed, hipStream_t st);

}  // namespace tmsap
