// Host-side declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "tm_device.h"

namespace tmsap {

enum Prec { P_F64 = 0, P_F32 = 1, P_F16 = 2, P_BF16 = 3 };

constexpr int kMaxSys = 64;

inline int unit_bytes(Prec p) { return p == P_F64 ? 32 : (p == P_F32 ? 16 : 8); }
inline bool prec_has_scale(Prec p) { return p == P_F16; }

// Internal spinor field: data [nsys][6 units][V], FP16 scales [nsys][V].
struct SpinorBuf {
    void* data = nullptr;
    float* scale = nullptr;
    Prec prec = P_F64;
    int nsys = 0;
};

// Bytes of the data part / scale part of an internal spinor field.
inline size_t spinor_data_bytes(long long V, int nsys, Prec p) { return (size_t)nsys * 6 * V * unit_bytes(p); }
inline size_t spinor_scale_bytes(long long V, int nsys, Prec p) {
    return prec_has_scale(p) ? (size_t)nsys * V * sizeof(float) : 0;
}
inline size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }

// Gauge data on the device at one precision: links [4][3 units][V] and the
// packed clover [18 units][V] holding (m+4) + clover.
// Site-diagonal inverses for even-odd solves, one set per (|mu|, parity):
// [36 units][V/2] at the clover precision, entry h for the site of that
// parity in the pair (2h, 2h+1) (tile x-extent even); units 0..17 hold
// (A_up + i|mu|)^-1, units 18..35 hold (A_dn - i|mu|)^-1, each 6x6 row-major
// as (re, im) pairs.
constexpr int kMaxEoMu = 8;
struct EoCache {
    int n = 0;
    double absmu[kMaxEoMu] = {};
    int parity[kMaxEoMu] = {};
    void* inv[kMaxEoMu] = {};
    void release();
    ~EoCache() { release(); }
};

struct GaugeDev {
    void* links = nullptr;
    void* clover = nullptr;
    Prec link_prec = P_F64;
    Prec clover_prec = P_F64;
    EoCache* eo = nullptr;  // owned by the cache entry that holds this
};

struct DiracArgs {
    Geo g;
    const void* links;
    const void* clover;
    const void* in;
    const float* in_scale;
    void* out;
    float* out_scale;
    int nsys;
    int colour = -1;     // -1: every 4^4 tile; 0 / 1: the blocks of that colour only (tiled operator)
    double mu[kMaxSys];
};

struct SapArgs {
    Geo g;               // tile = Schwarz block
    const void* links;
    const void* clover;
    const void* b;
    const float* b_scale;
    void* x;
    float* x_scale;
    int nsys;            // systems in the buffers
    int sys_tile;        // systems per workgroup (gridDim.y = ceil(nsys / sys_tile))
    int colour;
    int mr_iters;
    int own_zero;        // 1: x is zero on this colour's blocks (skip reading it)
    int halo_zero;       // 1: x is zero on the other colour's blocks too (then r = b)
    int eo;              // 1: even-odd preconditioned block solves
    void* w_out = nullptr;  // set (4^4 FP32 kernel, FP32 storage): D x on the swept blocks, written as
                            // b minus the final block residual, [nsys] fields like x
    unsigned long long eo_adj;            // bit k: system k uses the adjoint inverses (mu_k < 0)
    const void* eo_inv[kMaxEoMu];         // inverse sets by |mu|
    unsigned char eo_sel[kMaxSys];        // system -> inverse set
    double mu[kMaxSys];
};

// One step of the even-odd reduced operator on compact parity fields
// [nsys][6 units][V/2] (FP64): out_p = (D_pp^-1)? [hop_sign * H in_hop +
// D_pp in_diag + add_sign * in_add] with H = -1/2 sum of the hops between
// the parities; null inputs are skipped; the Gamma5 flags multiply the hop
// input, the diagonal input and the output (Dhat^+ = Gamma5 Dhat(-mu) Gamma5).
struct ParityArgs {
    Geo g;
    const void* links;   // FP64 [4][3 units][V]
    const void* clover;  // FP64 [18 units][V]
    const void* inv[kMaxEoMu];  // site inverse sets of parity p
    unsigned char sel[kMaxSys];
    int p;
    const double* in_hop;
    double hop_sign;
    const double* in_diag;
    const double* in_add;
    double add_sign;
    int do_inv;
    int g5_hop, g5_diag, g5_out;
    double mu_sign;
    double* out;
    int nsys;
    double mu[kMaxSys];
};

// ---- even-odd reduced operator and CG (tm_cg.hip)
hipError_t launch_parity_op(const ParityArgs& a, hipStream_t st);
hipError_t launch_parity_import(const Geo& g, int nsys, const void* canon, double* even, double* odd, unsigned* flag,
                                hipStream_t st);
hipError_t launch_parity_export(const Geo& g, int nsys, const double* even, const double* odd, void* canon,
                                hipStream_t st);
// y = a[sys] x + b[sys] y over n_per_sys doubles per system
hipError_t launch_axpby(const double* x, const double* a, double* y, const double* b, int nsys, long long n_per_sys,
                        hipStream_t st);
// mode 0: out = gamma / v (step length), neg = -out; mode 1: out = v / gamma, gamma = v; frozen systems get 0
hipError_t launch_cg_scalars(int mode, int nsys, unsigned long long frozen, double* gamma, const double* v,
                             double* out, double* neg, hipStream_t st);

// ---- layout kernels (tm_layout.hip)
hipError_t launch_link_ingest(const Geo& g, Prec G, const void* Ucanon, void* links, unsigned* stats, hipStream_t st);
// FP32 clover [18][V] units from the FP64 one (FP64 [18][V] double4 units) of the same geometry.
hipError_t launch_clover_to_f32(const Geo& g, const void* clover64, void* clover32, hipStream_t st);
hipError_t launch_clover_build(const Geo& g, Prec C, const void* Ucanon, double m4, double csw, void* clover,
                               hipStream_t st);
hipError_t launch_spinor_import(const Geo& g, const SpinorBuf& dst, const void* canon, unsigned* flag,
                                hipStream_t st);
hipError_t launch_spinor_export(const Geo& g, const SpinorBuf& src, void* canon, hipStream_t st);
hipError_t launch_spinor_convert(const Geo& g, const SpinorBuf& src, const SpinorBuf& dst, hipStream_t st);
// (A_up + i absmu)^-1 and (A_dn - i absmu)^-1 at every site of one parity, from the packed clover (FP64
// arithmetic)
hipError_t launch_eo_inverse(const Geo& g, Prec C, const void* clover, double absmu, int parity, void* inv,
                             hipStream_t st);
inline size_t eo_inverse_bytes(const Geo& g, Prec C) { return (size_t)36 * (g.V / 2) * unit_bytes(C); }

// ---- operator (tm_dirac.hip)
hipError_t launch_dirac(const DiracArgs& a, Prec in_p, Prec out_p, Prec link_p, Prec clover_p, Prec compute,
                        hipStream_t st);

// ---- smoother (tm_sap.hip)
// The operator on 4^4 tiles with FP32 arithmetic (tm_sap.hip); hipErrorNotSupported for other
// tiles or precision combinations, which launch_dirac then runs in its generic kernel.
hipError_t launch_dirac_44(const DiracArgs& a, Prec in_p, Prec out_p, Prec link_p, Prec clover_p,
                           hipStream_t st);
hipError_t launch_sap_half(const SapArgs& a, Prec spinor_p, Prec link_p, Prec clover_p, Prec compute,
                           hipStream_t st);
bool sap_supported(Prec spinor_p, Prec link_p, Prec clover_p, Prec compute);
// True when a half-sweep with these storage/link/clover precisions runs the 4^4 FP32 kernel with
// FP32 storage, whose w_out output is then available.
bool sap_fills_w(const Geo& g, Prec sp, Prec lp, Prec cp, bool eo);
size_t sap_lds_bytes(int Vb, Prec compute);

}  // namespace tmsap
