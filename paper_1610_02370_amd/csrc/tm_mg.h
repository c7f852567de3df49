// Kernels of the two-level method (tm_mg.hip): aggregation, restriction and
// prolongation, the Galerkin coarse stencil, the coarse operator and the
// vector kernels of the coarse GMRES.
//
// Aggregates are the tiles of the internal layout (a tile = one Schwarz block)
// split by spin half: spins {0,1} (units 0..2 of a site) and {2,3} (units
// 3..5).  The basis P is nv FP32 internal fields; column (j, sg, i) of P is
// field i on tile j, spin half sg.  A coarse vector of one system is
// [nc][2 nv] complex FP32 (float2), component sg*nv + i, with the coarse site
// index j equal to the tile index (lexicographic in tile coordinates).  The
// coarse stencil is [nc][9][2nv][2nv] float2 stored column-major per matrix:
// element (a, b) of term t at site j sits at ((j*9 + t)*2nv + b)*2nv + a;
// term 0 is the site itself, 1 + mu the coupling to the aggregate one step
// forward along mu, 5 + mu one step backward.
#pragma once

#include "tm_internal.h"

namespace tmsap {

constexpr int kMgMaxVec = 32;  // test vectors (2 nv <= 64: one lane per coarse component)

struct MgArgs {
    Geo g;                // tile = aggregate
    int nv;               // test vectors
    const void* P;        // nv FP32 internal fields
    size_t P_stride;      // bytes between fields
};

// out_b = term t of D applied to column b of P on every aggregate at once, for b in
// [b0, b0 + nb): t = 0 the block-diagonal part (the diagonal at mu = 0 plus the
// parity shift, and the hops inside the aggregate); t = 1 + mu the forward hop along
// mu where it leaves the aggregate; t = 5 + mu the backward hop likewise.  out holds
// nb FP32 internal fields.
hipError_t launch_mg_term(const MgArgs& m, const void* links, const void* clover, int t, int b0, int nb, void* out,
                          size_t out_stride, hipStream_t st);
// c[s] = P^+ x_s for nsys FP32 internal fields x: c element (s, j, a) at
// out[base + s*s_stride + j*j_stride + a] (float2 units).
hipError_t launch_mg_restrict(const MgArgs& m, const void* x, size_t x_stride, int nsys, float2* out, size_t base,
                              size_t s_stride, size_t j_stride, hipStream_t st);
// e_s = P c_s (coarse vectors [nsys][nc][2nv]) into nsys FP32 internal fields.
hipError_t launch_mg_prolong(const MgArgs& m, const float2* c, int nsys, void* e, size_t e_stride, hipStream_t st);
// Aggregate-wise modified Gram-Schmidt of the nv fields (in place).
hipError_t launch_mg_block_orthonormalize(const MgArgs& m, void* P, hipStream_t st);
// y_s = (Dc + i mu_c[s] Gamma5c) x_s, nsys <= kMaxSys; mu_c in device memory.
hipError_t launch_mg_coarse_apply(const Geo& g, int nv, const float2* Dc, const double* mu_c, const float2* x,
                                  float2* y, int nsys, hipStream_t st);
// General form: y_s = add_s + (Dc[j][0] + i mu_c[s] Gamma5c) x_self + hop_sign * sum_{t>=1} Dc[j][t] x_hop(nbr_t(j))
// on the coarse sites of `parity` (coarse parity = sum of the tile coordinates mod 2; parity < 0: all
// sites); a null input drops its terms, a null mu_c the twist.  Sites of the other parity get 0 when
// zero_other is set and are left alone otherwise.  y may equal add, not x_self or x_hop.
hipError_t launch_mg_coarse_part(const Geo& g, int nv, const float2* Dc, const double* mu_c, const float2* x_self,
                                 const float2* x_hop, double hop_sign, const float2* add, int parity, bool zero_other,
                                 float2* y, int nsys, hipStream_t st);
// Minv[j >> 1] = (Dc[j][0] + i mu_c Gamma5c)^-1 (column-major, FP32; FP64 elimination) for the sites j of
// `parity`; Minv holds nc / 2 matrices.  Needs an even innermost coarse extent.
hipError_t launch_mg_block_inverse(const Geo& g, int nv, const float2* Dc, double mu_c, int parity, float2* Minv,
                                   hipStream_t st);
constexpr int kMgMaxInv = 4;  // inverse sets (distinct coarse twists) one call can use
struct BlockMulArgs {
    Geo g;
    int nv;
    const float2* sets[kMgMaxInv];
    unsigned char sel[kMaxSys];  // system -> inverse set
    unsigned char order[kMaxSys];  // filled by the launcher: systems grouped by set,
    int start[kMgMaxInv + 1];      // set q's at order[start[q] .. start[q + 1])
    int parity;
    bool zero_other;  // other-parity sites: 0, or left alone
    const float2* x;
    float2* y;
    int nsys;
};
// y_s = Minv_{sel[s]}[j >> 1] x_s at the coarse sites j of a.parity (y != x).
hipError_t launch_mg_block_mul(const BlockMulArgs& a, hipStream_t st);
// Transposes the stored stencil into complex128 [nc][9][2nv][2nv] row-major.
hipError_t launch_mg_stencil_export(long long nc, int nv, const float2* Dc, void* out, hipStream_t st);
// complex128 <-> FP32 coarse vectors (n complex per call)
hipError_t launch_mg_coarse_import(const void* canon, float2* v, long long n, unsigned* flag, hipStream_t st);
hipError_t launch_mg_coarse_export(const float2* v, void* canon, long long n, hipStream_t st);

// ---- coarse vector kernels: nsys vectors of n complex each, vector i of a basis at
// basis + i * vec_stride (float2 units), system s at + s * sys_stride.
int mg_blas_blocks(long long n);
// out[s][i0 + i] = <v_i, w_s> (double2) for i in [0, cnt), cnt <= 16
hipError_t mg_blas_dots(const float2* basis, size_t vec_stride, int cnt, const float2* w, size_t sys_stride, int nsys,
                        long long n, double* partials, double2* out, int out_stride, hipStream_t st);
// w_s += sign * sum_i coef[s][i] v_i for i in [0, cnt), cnt <= 16 (coef double2, per system at coef + s*coef_stride)
hipError_t mg_blas_axpy(const float2* basis, size_t vec_stride, int cnt, const double2* coef, int coef_stride,
                        double sign, float2* w, size_t sys_stride, int nsys, long long n, hipStream_t st);
// out[s] = ||w_s||^2
hipError_t mg_blas_norm2(const float2* w, size_t sys_stride, int nsys, long long n, double* partials, double* out,
                         hipStream_t st);
// y_s = f[s] x_s (f double in device memory)
hipError_t mg_blas_scale(const float2* x, const double* f, float2* y, size_t sys_stride, int nsys, long long n,
                         hipStream_t st);
// y_s = x_s - y_s
hipError_t mg_blas_sub_from(const float2* x, float2* y, size_t sys_stride, int nsys, long long n, hipStream_t st);
// Panels of vectors w_s = w + s * w_stride (s < nw <= 4) against one shared basis, each vector read once:
// out[s * out_stride + i] = <v_i, w_s> for i < cnt <= 4
hipError_t mg_blas_panel_dots(const float2* basis, size_t vec_stride, int cnt, const float2* w, size_t w_stride, int nw,
                              long long n, double* partials, double2* out, int out_stride, hipStream_t st);
// w_s -= sum_i coef[s * coef_stride + i] v_i for i < cnt <= 8
hipError_t mg_blas_panel_axpy(const float2* basis, size_t vec_stride, int cnt, const double2* coef, int coef_stride,
                              float2* w, size_t w_stride, int nw, long long n, hipStream_t st);

}  // namespace tmsap
