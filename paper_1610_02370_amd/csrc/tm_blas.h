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

// Gram-Schmidt pass over basis vectors 0..nvec-1 (vector i at basis.data + i*vec_stride, FP64 or FP32, no scales):
//   mode 0: out[sys][i] = <v_i, w>
//   mode 1: w -= sum_i coef[sys][i] v_i, then out[sys][i] = <v_i, w>
//   mode 2: w -= sum_i coef[sys][i] v_i, then out[sys] = ||w||^2
// complex values as (re, im) pairs; accumulate != 0 adds to out.
hipError_t blas_gs(Prec p, const VecRef& basis, size_t vec_stride, int nvec, const VecRef& w, const double* coef,
                   int mode, double* partials, double* out, int accumulate, int nsys, long long V, hipStream_t st);
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
